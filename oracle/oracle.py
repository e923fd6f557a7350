"""Python front end of the FP64 oracle (oracle.cpp), loaded with ctypes.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never touches it.

Inputs are the float32 arrays drawn by the scene generator, widened exactly to
float64.  Every stage is exposed separately so that tests can feed one stage
with another stage's output (for example binning from single-precision screen
positions produced elsewhere) as well as run the whole chain.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

_lock = threading.Lock()
_lib = None

D = C.POINTER(C.c_double)
F = C.POINTER(C.c_float)
I32 = C.POINTER(C.c_int32)
U32 = C.POINTER(C.c_uint32)
U64 = C.POINTER(C.c_uint64)
U8 = C.POINTER(C.c_uint8)


class OrcGaussians(C.Structure):
    _fields_ = [("means", D), ("log_scales", D), ("quats", D), ("opacity_logits", D), ("sh_dc", D),
                ("sh_rest", D), ("mask_logits", D), ("sh_mask_logits", D), ("n", C.c_int64),
                ("sh_degree", C.c_int32), ("pad_", C.c_int32), ("mask_eps", C.c_double),
                ("sh_mask_eps", C.c_double)]


class OrcCamera(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class OrcOpts(C.Structure):
    _fields_ = [("near_plane", C.c_double), ("tan_clamp", C.c_double), ("lowpass", C.c_double),
                ("bg", C.c_double * 3), ("tile_w", C.c_int32), ("tile_h", C.c_int32),
                ("lowpass_progressive", C.c_int32)]


class OrcGrads(C.Structure):
    _fields_ = [("means", D), ("log_scales", D), ("quats", D), ("opacity_logits", D), ("sh_dc", D),
                ("sh_rest", D), ("mask_logits", D), ("sh_mask_logits", D)]


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (OpenMP, no FMA contraction)."""
    with _lock:
        if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            tmp = LIB + ".tmp%d" % os.getpid()
            cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                   "-shared", SRC, "-o", tmp]
            subprocess.check_call(cmd)
            os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_sh_basis.argtypes = [C.c_int64, D, D]
        L.orc_cov3d.argtypes = [C.POINTER(OrcGaussians), D]
        L.orc_project.argtypes = [C.POINTER(OrcGaussians), C.POINTER(OrcCamera), C.POINTER(OrcOpts), I32, D, D, D,
                                  I32, D, D, D]
        L.orc_bin.restype = C.c_int64
        L.orc_bin.argtypes = [C.c_int32, C.c_int64, C.POINTER(OrcCamera), C.POINTER(OrcOpts), F, F, F, I32, I32,
                              U32, U64, U32, C.c_int64, U32]
        L.orc_composite_fwd.argtypes = [C.c_int32, C.c_int64, C.POINTER(OrcCamera), C.POINTER(OrcOpts), D, D, D, D,
                                        I32, U32, U32, D, D, I32, D, U8, U64, U8, U8, D, D]
        L.orc_composite_bwd.argtypes = [C.c_int32, C.c_int64, C.POINTER(OrcCamera), C.POINTER(OrcOpts), D, D, D, D,
                                        I32, U32, U32, D, D, U8]
        L.orc_project_bwd.argtypes = [C.POINTER(OrcGaussians), C.POINTER(OrcCamera), C.POINTER(OrcOpts), D,
                                      C.POINTER(OrcGrads)]
        L.orc_hits.argtypes = [C.c_int32, C.c_int64, C.POINTER(OrcCamera), C.POINTER(OrcOpts), D, D, D, D, I32, U32,
                               U32, D, U32, U32]
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _p(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class _Gauss:
    """Keeps the float64 copies alive while the C struct points at them."""

    def __init__(self, scene):
        self.arr = {k: _f64(v) for k, v in scene.arrays().items()}
        a = self.arr
        self.s = OrcGaussians(
            _p(a["means"], D), _p(a["log_scales"], D), _p(a["quats"], D), _p(a["opacity_logits"], D),
            _p(a["sh_dc"], D), _p(a.get("sh_rest"), D), _p(a.get("mask_logits"), D),
            _p(a.get("sh_mask_logits"), D), scene.n, scene.sh_degree, 0, float(scene.mask_eps),
            float(scene.sh_mask_eps))


def camera_struct(cam) -> OrcCamera:
    c = OrcCamera()
    R = np.asarray(cam.R, np.float64).reshape(9)
    t = np.asarray(cam.t, np.float64).reshape(3)
    for i in range(9):
        c.R[i] = R[i]
    for i in range(3):
        c.t[i] = t[i]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def opts_struct(o) -> OrcOpts:
    s = OrcOpts()
    s.near_plane, s.tan_clamp, s.lowpass = float(o.near_plane), float(o.tan_clamp), float(o.lowpass)
    for i in range(3):
        s.bg[i] = float(o.bg[i])
    s.tile_w, s.tile_h = int(o.tile_w), int(o.tile_h)
    s.lowpass_progressive = int(getattr(o, "lowpass_progressive", 0))
    return s


def _cams(cams):
    arr = (OrcCamera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = camera_struct(c)
    return arr


def tile_grid(cams, opts):
    """Per view (TX, TY, tile offset) and the total tile count."""
    out, off = [], 0
    for c in cams:
        tx = -(-c.width // opts.tile_w)
        ty = -(-c.height // opts.tile_h)
        out.append((tx, ty, off))
        off += tx * ty
    return out, off


def sh_basis(dirs: np.ndarray) -> np.ndarray:
    dirs = _f64(dirs).reshape(-1, 3)
    out = np.zeros((dirs.shape[0], 16))
    lib().orc_sh_basis(dirs.shape[0], _p(dirs, D), _p(out, D))
    return out


def cov3d(scene) -> np.ndarray:
    g = _Gauss(scene)
    out = np.zeros((scene.n, 6))
    lib().orc_cov3d(C.byref(g.s), _p(out, D))
    return out


def project(scene, cam, opts) -> dict:
    """FP64 projection of all Gaussians into one view."""
    n = scene.n
    g = _Gauss(scene)
    out = dict(valid=np.zeros(n, np.int32), uv=np.zeros((n, 2)), conic=np.zeros((n, 3)), depth=np.zeros(n),
               radius=np.zeros(n, np.int32), opacity=np.zeros(n), rgb=np.zeros((n, 3)), cov2d=np.zeros((n, 3)))
    c, o = camera_struct(cam), opts_struct(opts)
    lib().orc_project(C.byref(g.s), C.byref(c), C.byref(o), _p(out["valid"], I32), _p(out["uv"], D),
                      _p(out["conic"], D), _p(out["depth"], D), _p(out["radius"], I32), _p(out["opacity"], D),
                      _p(out["rgb"], D), _p(out["cov2d"], D))
    return out


def project_views(scene, cams, opts) -> dict:
    """Projection into every view, concatenated per record (view * n + gaussian)."""
    parts = [project(scene, c, opts) for c in cams]
    return {k: np.concatenate([p[k] for p in parts], 0) for k in parts[0]}


def bin(cams, opts, n, u, v, depth, radius, valid, want_lists=True):
    """Tile binning and ordering from single-precision (u, v, depth) and integer radius.

    Returns dict(tiles_touched, K, keys, ids, ranges)."""
    V = len(cams)
    u = np.ascontiguousarray(u, np.float32)
    v = np.ascontiguousarray(v, np.float32)
    depth = np.ascontiguousarray(depth, np.float32)
    radius = np.ascontiguousarray(radius, np.int32)
    valid = np.ascontiguousarray(valid, np.int32)
    cs, o = _cams(cams), opts_struct(opts)
    tt = np.zeros(V * n, np.uint32)
    L = lib()
    K = L.orc_bin(V, n, cs, C.byref(o), _p(u, F), _p(v, F), _p(depth, F), _p(radius, I32), _p(valid, I32),
                  _p(tt, U32), None, None, 0, None)
    out = dict(tiles_touched=tt, K=int(K))
    if want_lists:
        _, T = tile_grid(cams, opts)
        keys = np.zeros(max(K, 1), np.uint64)
        ids = np.zeros(max(K, 1), np.uint32)
        ranges = np.zeros((T, 2), np.uint32)
        L.orc_bin(V, n, cs, C.byref(o), _p(u, F), _p(v, F), _p(depth, F), _p(radius, I32), _p(valid, I32),
                  _p(tt, U32), _p(keys, U64), _p(ids, U32), max(K, 1), _p(ranges, U32))
        out.update(keys=keys[:K], ids=ids[:K], ranges=ranges)
    return out


def _splat_args(sp):
    uv = _f64(sp["uv"]).reshape(-1, 2)
    conic = _f64(sp["conic"]).reshape(-1, 3)
    op = _f64(sp["opacity"]).reshape(-1)
    rgb = _f64(sp["rgb"]).reshape(-1, 3)
    rad = np.ascontiguousarray(sp["radius"], np.int32).reshape(-1)
    return uv, conic, op, rgb, rad


def _mask(tile_mask):
    return None if tile_mask is None else np.ascontiguousarray(tile_mask, np.uint8)


def _eps(eps):
    """The seven near-threshold windows of the walk (missing trailing entries are 0):
    alpha relative (fixed part), T relative (fixed part), square edge in pixels
    (fixed part), alpha relative per unit of the exponent's terms, T relative per
    composited Gaussian, square edge relative to |dx|, depth relative (order of
    consecutive records reaching a pixel)."""
    if eps is None:
        return None
    e = np.zeros(7, np.float64)
    a = np.asarray(eps, np.float64).reshape(-1)
    e[:a.size] = a
    return e


def composite_fwd(cams, opts, n, splats, ids, ranges, eps=None, tile_mask=None, rec_flags=None, rec_win=None,
                  depth=None) -> dict:
    """Eq. 2 per pixel.  Returns flat image (views concatenated, each [3,H,W]),
    T_final, last_contrib, and (if eps given) near-threshold flags + decision hashes.
    tile_mask (uint8 per global tile) restricts the work to the marked tiles;
    rec_flags (uint8 per record, bit 1: radius near an integer) adds flag 16;
    rec_win ([records, 2]: screen-position error in pixels, conic relative error)
    widens the windows; depth (per record) with eps[6] adds flag 32."""
    V = len(cams)
    P = sum(c.width * c.height for c in cams)
    uv, conic, op, rgb, rad = _splat_args(splats)
    ids = np.ascontiguousarray(ids, np.uint32)
    if ids.size == 0:
        ids = np.zeros(1, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    img = np.zeros(3 * P)
    T = np.zeros(P)
    last = np.zeros(P, np.int32)
    flags = np.zeros(P, np.uint8)
    hsh = np.zeros(P, np.uint64)
    e = _eps(eps)
    tm = _mask(tile_mask)
    rf = None if rec_flags is None else np.ascontiguousarray(rec_flags, np.uint8)
    rw = None if rec_win is None else np.ascontiguousarray(rec_win, np.float64).reshape(-1)
    dp = None if depth is None else np.ascontiguousarray(depth, np.float64).reshape(-1)
    cs, o = _cams(cams), opts_struct(opts)
    lib().orc_composite_fwd(V, n, cs, C.byref(o), _p(uv, D), _p(conic, D), _p(op, D), _p(rgb, D), _p(rad, I32),
                            _p(ids, U32), _p(ranges, U32), _p(img, D), _p(T, D), _p(last, I32), _p(e, D),
                            _p(flags, U8) if e is not None else None,
                            _p(hsh, U64) if e is not None else None, _p(tm, U8), _p(rf, U8), _p(rw, D), _p(dp, D))
    return dict(image=img, T_final=T, last_contrib=last, flags=flags, hash=hsh)


def hits(cams, opts, n, splats, ids, ranges, eps=None) -> dict:
    """Per record, the number of pixels where it is composited (Eq. 4's ray hits) -> [V*n] uint32,
    and, if eps is given, per record the number of near-threshold pixels whose tile lists it."""
    V = len(cams)
    uv, conic, op, rgb, rad = _splat_args(splats)
    ids = np.ascontiguousarray(ids, np.uint32)
    if ids.size == 0:
        ids = np.zeros(1, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    h = np.zeros(V * n, np.uint32)
    u = np.zeros(V * n, np.uint32)
    e = _eps(eps)
    cs, o = _cams(cams), opts_struct(opts)
    lib().orc_hits(V, n, cs, C.byref(o), _p(uv, D), _p(conic, D), _p(op, D), _p(rgb, D), _p(rad, I32), _p(ids, U32),
                   _p(ranges, U32), _p(e, D), _p(h, U32), _p(u, U32) if e is not None else None)
    return dict(hits=h, uncertain=u)


def count_hits(scene, cams, opts, eps=None, splats=None, lists=None) -> dict:
    """Whole chain for Eq. 4's ray hits: project, bin, walk; per record and per Gaussian."""
    n = scene.n
    if splats is None:
        splats = project_views(scene, cams, opts)
    if lists is None:
        lists = bin(cams, opts, n, splats["uv"][:, 0].astype(np.float32), splats["uv"][:, 1].astype(np.float32),
                    splats["depth"].astype(np.float32), splats["radius"], splats["valid"])
    h = hits(cams, opts, n, splats, lists["ids"], lists["ranges"], eps=eps)
    h["per_gaussian"] = hits_per_gaussian(h["hits"], len(cams), n)
    h.update(splats=splats, lists=lists)
    return h


def hits_per_gaussian(hits_rec, V: int, n: int) -> np.ndarray:
    """Sum over the V views of the per-record hit counts -> [n] (records are view-major)."""
    return np.asarray(hits_rec, np.int64).reshape(V, n).sum(0)


def volume_rank(q: float, n: int) -> int:
    """Ascending rank (1-based) of the reference volume: ceil(q n) in double, clamped to [1, n]."""
    return min(max(int(math.ceil(float(q) * float(n))), 1), n)


def significance(scene, hits, q: float = 0.9) -> np.ndarray:
    """Significance score of Eq. 4 per Gaussian j: hits_j x o'_j x gamma_j, in FP64.
    hits_j = the number of (view, pixel) rays where Gaussian j is composited (summed over views);
    o'_j = sigmoid(opacity logit) x the hard volume mask of Eq. 3; gamma_j = min(vol_j / v_q, 1),
    vol_j = the product of its three scales, v_q the volume at ascending rank ceil(q n) (the
    normalisation by the volume of the largest Gaussians that Sec. 3.2.2 describes)."""
    n = scene.n
    h = np.asarray(hits, np.float64)
    op = 1.0 / (1.0 + np.exp(-scene.opacity_logits.astype(np.float64)))
    if scene.mask_logits is not None:
        op = op * (1.0 / (1.0 + np.exp(-scene.mask_logits.astype(np.float64))) > scene.mask_eps)
    vol = np.exp(scene.log_scales.astype(np.float64).sum(0))
    if n == 0:
        return np.zeros(0)
    vq = np.sort(vol)[volume_rank(q, n) - 1]
    return h * op * np.minimum(vol / vq, 1.0)


def composite_bwd(cams, opts, n, splats, ids, ranges, dL_dimage, tile_mask=None) -> np.ndarray:
    """Gradient of sum(dL_dimage * image) w.r.t. per-record (u, v, A, B, C, o', r, g, b) -> [V*n, 9]."""
    V = len(cams)
    uv, conic, op, rgb, rad = _splat_args(splats)
    ids = np.ascontiguousarray(ids, np.uint32)
    if ids.size == 0:
        ids = np.zeros(1, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    dl = _f64(dL_dimage).reshape(-1)
    out = np.zeros((V * n, 9))
    tm = _mask(tile_mask)
    cs, o = _cams(cams), opts_struct(opts)
    lib().orc_composite_bwd(V, n, cs, C.byref(o), _p(uv, D), _p(conic, D), _p(op, D), _p(rgb, D), _p(rad, I32),
                            _p(ids, U32), _p(ranges, U32), _p(dl, D), _p(out, D), _p(tm, U8))
    return out


GRAD_NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh_dc", "sh_rest", "mask_logits",
              "sh_mask_logits")


def zero_grads(scene) -> dict:
    return {k: np.zeros(v.shape, np.float64) for k, v in scene.arrays().items()}


def project_bwd(scene, cam, opts, grad_rec, grads: dict) -> dict:
    """Accumulate d/d(raw params) of sum(grad_rec * splat values) for one view into `grads`."""
    g = _Gauss(scene)
    gr = _f64(grad_rec).reshape(scene.n, 9)
    for k in grads:
        assert grads[k].dtype == np.float64 and grads[k].flags.c_contiguous
    s = OrcGrads(*[_p(grads.get(k), D) for k in GRAD_NAMES])
    c, o = camera_struct(cam), opts_struct(opts)
    lib().orc_project_bwd(C.byref(g.s), C.byref(c), C.byref(o), _p(gr, D), C.byref(s))
    return grads


def split_views(flat, cams, channels):
    out, off = [], 0
    for c in cams:
        k = channels * c.width * c.height
        shape = (channels, c.height, c.width) if channels > 1 else (c.height, c.width)
        out.append(flat[off:off + k].reshape(shape))
        off += k
    return out


def l2_grad(images, targets):
    """dL/dimage of L = mean over views of mean over 3HW of (image - target)^2."""
    V = len(images)
    return [2.0 * (np.asarray(im, np.float64) - np.asarray(t, np.float64)) / (im.size * V)
            for im, t in zip(images, targets)]


def render(scene, cams, opts, dL_dimages=None, eps=None, splats=None, lists=None) -> dict:
    """Whole chain: project (FP64) -> bin/order from the single-precision
    rounding of the projected values -> composite -> optional backward.

    `splats` (per-record dict) or `lists` (dict with ids, ranges) may be passed
    in to composite other projected values or other lists."""
    n = scene.n
    if splats is None:
        splats = project_views(scene, cams, opts)
    if lists is None:
        lists = bin(cams, opts, n, splats["uv"][:, 0].astype(np.float32), splats["uv"][:, 1].astype(np.float32),
                    splats["depth"].astype(np.float32), splats["radius"], splats["valid"])
    fw = composite_fwd(cams, opts, n, splats, lists["ids"], lists["ranges"], eps=eps)
    out = dict(splats=splats, lists=lists, fwd=fw,
               images=split_views(fw["image"], cams, 3),
               T_final=split_views(fw["T_final"], cams, 1),
               last_contrib=split_views(fw["last_contrib"], cams, 1))
    if dL_dimages is not None:
        dl = np.concatenate([np.asarray(d, np.float64).reshape(-1) for d in dL_dimages])
        grad_rec = composite_bwd(cams, opts, n, splats, lists["ids"], lists["ranges"], dl)
        grads = zero_grads(scene)
        for v, c in enumerate(cams):
            project_bwd(scene, c, opts, grad_rec[v * n:(v + 1) * n], grads)
        out.update(grad_rec=grad_rec, grads=grads)
    return out
