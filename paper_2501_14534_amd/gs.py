"""ctypes binding of libgs (include/gs_api.h): argument marshalling only.

Every entry point keeps the C name without its `gs_` prefix and takes torch
CUDA tensors (or None) where the C function takes device pointers; the work
itself runs in the HIP kernels of libgs.so.  Loading fails loudly when the
library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libgs.so")

GS_OK, GS_E_INVALID, GS_E_CAPACITY, GS_E_HIP, GS_E_UNSUPPORTED, GS_E_TOO_LARGE = 0, -1, -2, -3, -4, -5
MAX_VIEWS = 16
SPLAT_FLOATS = 12
GRAD_FLOATS = 9
MAX_BATCH = 1024

EXPORTS = ("gs_view_sizes", "gs_workspace_size", "gs_project", "gs_bin_sort", "gs_render_fwd", "gs_render_bwd",
           "gs_render_fwd_bwd_l2", "gs_blend_bwd", "gs_project_bwd", "gs_loss_workspace_size", "gs_loss_l1_dssim", "gs_l2_grad",
           "gs_mask_loss_workspace_size", "gs_mask_loss", "gs_mask_loss_noalloc", "gs_count_hits", "gs_significance_workspace_size",
           "gs_significance", "gs_blur_views", "gs_resize_views", "gs_strerror")

vp = C.c_void_p


class GsGaussians(C.Structure):
    _fields_ = [("means", vp), ("log_scales", vp), ("quats", vp), ("opacity_logits", vp), ("sh_dc", vp),
                ("sh_rest", vp), ("mask_logits", vp), ("sh_mask_logits", vp), ("n", C.c_int64),
                ("sh_degree", C.c_int32), ("mask_eps", C.c_float), ("sh_mask_eps", C.c_float)]


class GsCamera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class GsOpts(C.Structure):
    _fields_ = [("near_plane", C.c_float), ("tan_clamp", C.c_float), ("lowpass", C.c_float),
                ("bg", C.c_float * 3), ("tile_w", C.c_int32), ("tile_h", C.c_int32),
                ("batch_depth", C.c_int32), ("pixels_per_thread", C.c_int32), ("subtile_cull", C.c_int32),
                ("bwd_chunk", C.c_int32), ("fwd_chunk", C.c_int32), ("lowpass_progressive", C.c_int32)]


class GsProjected(C.Structure):
    _fields_ = [("splats", vp), ("tiles_touched", vp)]


class GsBinning(C.Structure):
    _fields_ = [("keys", vp), ("ids", vp), ("pair_index", vp), ("offsets", vp), ("ranges", vp), ("order", vp),
                ("capacity", C.c_uint64), ("count", vp), ("status", vp)]


class GsGrads(C.Structure):
    _fields_ = [("means", vp), ("log_scales", vp), ("quats", vp), ("opacity_logits", vp), ("sh_dc", vp),
                ("sh_rest", vp), ("mask_logits", vp), ("sh_mask_logits", vp), ("mean2d", vp), ("assign", C.c_int32)]


_lib = None


class GsError(RuntimeError):
    pass


def load():
    """Load libgs.so from the package directory; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise GsError(f"{LIB} is not built: run `python -m paper_2501_14534_amd.build` (or __graft_entry__.build())")
    L = C.CDLL(LIB)
    P = C.POINTER
    L.gs_view_sizes.argtypes = [P(GsCamera), C.c_int32, P(GsOpts), P(C.c_int64), P(C.c_int64)]
    L.gs_view_sizes.restype = C.c_int
    L.gs_workspace_size.argtypes = [C.c_int64, C.c_int32, P(GsCamera), P(GsOpts), C.c_uint64]
    L.gs_workspace_size.restype = C.c_size_t
    L.gs_project.argtypes = [P(GsGaussians), P(GsCamera), C.c_int32, P(GsOpts), P(GsProjected), vp]
    L.gs_project.restype = C.c_int
    L.gs_bin_sort.argtypes = [P(GsProjected), P(GsCamera), C.c_int32, C.c_int64, P(GsOpts), P(GsBinning), vp,
                              C.c_size_t, vp]
    L.gs_bin_sort.restype = C.c_int
    L.gs_render_fwd.argtypes = [P(GsProjected), P(GsBinning), P(GsCamera), C.c_int32, C.c_int64, P(GsOpts), vp, vp,
                                vp, vp, C.c_size_t, vp]
    L.gs_render_fwd.restype = C.c_int
    L.gs_render_bwd.argtypes = [P(GsGaussians), P(GsCamera), C.c_int32, P(GsOpts), P(GsProjected), P(GsBinning),
                                vp, vp, vp, P(GsGrads), vp, C.c_size_t, vp]
    L.gs_render_bwd.restype = C.c_int
    L.gs_render_fwd_bwd_l2.argtypes = [P(GsGaussians), P(GsCamera), C.c_int32, P(GsOpts), P(GsProjected),
                                       P(GsBinning), vp, C.c_int32, vp, vp, vp, vp, P(GsGrads), vp, C.c_size_t, vp]
    L.gs_render_fwd_bwd_l2.restype = C.c_int
    L.gs_blend_bwd.argtypes = [P(GsCamera), C.c_int32, C.c_int64, P(GsOpts), P(GsProjected), P(GsBinning), vp, vp,
                               vp, vp, vp, C.c_size_t, vp]
    L.gs_blend_bwd.restype = C.c_int
    L.gs_project_bwd.argtypes = [P(GsGaussians), P(GsCamera), C.c_int32, P(GsOpts), P(GsProjected), P(GsBinning),
                                 vp, P(GsGrads), vp, C.c_size_t, vp]
    L.gs_project_bwd.restype = C.c_int
    L.gs_loss_workspace_size.argtypes = [P(GsCamera), C.c_int32]
    L.gs_loss_workspace_size.restype = C.c_size_t
    L.gs_loss_l1_dssim.argtypes = [vp, vp, P(GsCamera), C.c_int32, C.c_float, vp, vp, vp, C.c_size_t, vp]
    L.gs_loss_l1_dssim.restype = C.c_int
    L.gs_l2_grad.argtypes = [vp, vp, P(GsCamera), C.c_int32, C.c_int32, vp, vp]
    L.gs_l2_grad.restype = C.c_int
    L.gs_mask_loss_workspace_size.argtypes = [C.c_int64]
    L.gs_mask_loss_workspace_size.restype = C.c_size_t
    L.gs_mask_loss.argtypes = [P(GsGaussians), C.c_float, C.c_float, vp, P(GsGrads), vp, C.c_size_t, vp]
    L.gs_mask_loss.restype = C.c_int
    L.gs_mask_loss_noalloc.argtypes = [P(GsGaussians), C.c_float, C.c_float, vp, P(GsGrads), vp]
    L.gs_mask_loss_noalloc.restype = C.c_int
    L.gs_count_hits.argtypes = [P(GsProjected), P(GsBinning), P(GsCamera), C.c_int32, C.c_int64, P(GsOpts), vp, vp]
    L.gs_count_hits.restype = C.c_int
    L.gs_significance_workspace_size.argtypes = []
    L.gs_significance_workspace_size.restype = C.c_size_t
    L.gs_significance.argtypes = [P(GsGaussians), vp, C.c_float, vp, vp, C.c_size_t, vp]
    L.gs_significance.restype = C.c_int
    L.gs_blur_views.argtypes = [vp, vp, P(GsCamera), C.c_int32, C.c_int32, C.c_float, vp]
    L.gs_blur_views.restype = C.c_int
    L.gs_resize_views.argtypes = [vp, P(GsCamera), vp, P(GsCamera), C.c_int32, vp]
    L.gs_resize_views.restype = C.c_int
    L.gs_strerror.argtypes = [C.c_int]
    L.gs_strerror.restype = C.c_char_p
    _lib = L
    return L


def strerror(code: int) -> str:
    return load().gs_strerror(int(code)).decode()


def check(code: int, what: str) -> None:
    if code != GS_OK:
        raise GsError(f"{what}: {strerror(code)} ({code})")


def ptr(t) -> int | None:
    """Device address of a tensor (None stays NULL)."""
    return None if t is None else t.data_ptr()


def cameras(cams) -> "C.Array":
    arr = (GsCamera * len(cams))()
    for i, c in enumerate(cams):
        R = [float(x) for x in c.R.reshape(9)]
        t = [float(x) for x in c.t.reshape(3)]
        arr[i].R = (C.c_float * 9)(*R)
        arr[i].t = (C.c_float * 3)(*t)
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        arr[i].width, arr[i].height = int(c.width), int(c.height)
    return arr


def options(o) -> GsOpts:
    s = GsOpts()
    s.near_plane, s.tan_clamp, s.lowpass = float(o.near_plane), float(o.tan_clamp), float(o.lowpass)
    s.bg = (C.c_float * 3)(*[float(b) for b in o.bg])
    s.tile_w, s.tile_h = int(o.tile_w), int(o.tile_h)
    s.batch_depth, s.pixels_per_thread = int(o.batch_depth), int(o.pixels_per_thread)
    s.subtile_cull = int(getattr(o, "subtile_cull", 1))
    s.bwd_chunk = int(getattr(o, "bwd_chunk", 1024))
    s.fwd_chunk = int(getattr(o, "fwd_chunk", 0))
    s.lowpass_progressive = int(getattr(o, "lowpass_progressive", 0))
    return s


def gaussians(params: dict, n: int, sh_degree: int, mask_eps: float, sh_mask_eps: float) -> GsGaussians:
    g = GsGaussians()
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh_dc", "sh_rest", "mask_logits", "sh_mask_logits"):
        setattr(g, k, ptr(params.get(k)))
    g.n, g.sh_degree, g.mask_eps, g.sh_mask_eps = int(n), int(sh_degree), float(mask_eps), float(sh_mask_eps)
    return g


def view_sizes(cams_arr, V, opts_s):
    t, p = C.c_int64(), C.c_int64()
    check(load().gs_view_sizes(cams_arr, V, C.byref(opts_s), C.byref(t), C.byref(p)), "gs_view_sizes")
    return int(t.value), int(p.value)


def workspace_size(n, cams_arr, V, opts_s, capacity) -> int:
    return int(load().gs_workspace_size(int(n), V, cams_arr, C.byref(opts_s), int(capacity)))


def project(g, cams_arr, V, opts_s, proj, stream) -> int:
    return load().gs_project(C.byref(g), cams_arr, V, C.byref(opts_s), C.byref(proj), stream)


def bin_sort(proj, cams_arr, V, n, opts_s, bins, ws, ws_bytes, stream) -> int:
    return load().gs_bin_sort(C.byref(proj), cams_arr, V, int(n), C.byref(opts_s), C.byref(bins), ws, ws_bytes, stream)


def render_fwd(proj, bins, cams_arr, V, n, opts_s, image, T_final, last, ws, ws_bytes, stream) -> int:
    return load().gs_render_fwd(C.byref(proj), C.byref(bins), cams_arr, V, int(n), C.byref(opts_s), image, T_final,
                                last, ws, ws_bytes, stream)


def render_bwd(g, cams_arr, V, opts_s, proj, bins, T_final, last, dL_dimage, grads, ws, ws_bytes, stream) -> int:
    return load().gs_render_bwd(C.byref(g), cams_arr, V, C.byref(opts_s), C.byref(proj), C.byref(bins), T_final, last,
                                dL_dimage, C.byref(grads), ws, ws_bytes, stream)


def render_fwd_bwd_l2(g, cams_arr, V, opts_s, proj, bins, target, mean_views, image, T_final, last, dL_dimage,
                      grads, ws, ws_bytes, stream) -> int:
    return load().gs_render_fwd_bwd_l2(C.byref(g), cams_arr, V, C.byref(opts_s), C.byref(proj), C.byref(bins), target,
                                       int(mean_views), image, T_final, last, dL_dimage, C.byref(grads), ws,
                                       ws_bytes, stream)


def blend_bwd(cams_arr, V, n, opts_s, proj, bins, T_final, last, dL_dimage, grad_pair, ws, ws_bytes, stream) -> int:
    return load().gs_blend_bwd(cams_arr, V, int(n), C.byref(opts_s), C.byref(proj), C.byref(bins), T_final, last,
                               dL_dimage, grad_pair, ws, ws_bytes, stream)


def project_bwd(g, cams_arr, V, opts_s, proj, bins, grad_pair, grads, ws, ws_bytes, stream) -> int:
    return load().gs_project_bwd(C.byref(g), cams_arr, V, C.byref(opts_s), C.byref(proj), C.byref(bins), grad_pair,
                                 C.byref(grads), ws, ws_bytes, stream)


def loss_workspace_size(cams_arr, V) -> int:
    return int(load().gs_loss_workspace_size(cams_arr, V))


def l2_grad(image, target, cams_arr, V, mean_views, dL_dimage, stream) -> int:
    return load().gs_l2_grad(image, target, cams_arr, V, int(mean_views), dL_dimage, stream)


def loss_l1_dssim(image, target, cams_arr, V, lambda_ssim, loss, dL_dimage, ws, ws_bytes, stream) -> int:
    return load().gs_loss_l1_dssim(image, target, cams_arr, V, float(lambda_ssim), loss, dL_dimage, ws, ws_bytes,
                                   stream)


def count_hits(proj, bins, cams_arr, V, n, opts_s, hits, stream) -> int:
    return load().gs_count_hits(C.byref(proj), C.byref(bins), cams_arr, V, int(n), C.byref(opts_s), hits, stream)


def significance_workspace_size() -> int:
    return int(load().gs_significance_workspace_size())


def significance(g, hits, volume_quantile, score, ws, ws_bytes, stream) -> int:
    return load().gs_significance(C.byref(g), hits, float(volume_quantile), score, ws, ws_bytes, stream)


def blur_views(inp, out, cams_arr, V, ksize, sigma, stream) -> int:
    return load().gs_blur_views(inp, out, cams_arr, V, int(ksize), float(sigma), stream)


def resize_views(inp, in_cams_arr, out, out_cams_arr, V, stream) -> int:
    return load().gs_resize_views(inp, in_cams_arr, out, out_cams_arr, V, stream)


def mask_loss_workspace_size(n) -> int:
    return int(load().gs_mask_loss_workspace_size(int(n)))


def mask_loss(g, lambda_m, lambda_sh, loss, grads, ws, ws_bytes, stream) -> int:
    return load().gs_mask_loss(C.byref(g), float(lambda_m), float(lambda_sh), loss,
                               C.byref(grads) if grads is not None else None, ws, ws_bytes, stream)


def mask_loss_noalloc(g, lambda_m, lambda_sh, loss, grads, stream) -> int:
    return load().gs_mask_loss_noalloc(C.byref(g), float(lambda_m), float(lambda_sh), loss,
                                       C.byref(grads) if grads is not None else None, stream)
