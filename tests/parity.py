"""GPU-path vs oracle comparison helpers (test infrastructure, used by the GPU
tests and by the smoke check).

Protocol.  Each stage of the HIP path is compared with the FP64 oracle fed
the same inputs:
  * projection: raw parameters -> records, against the oracle's FP64
    projection, with tolerances derived from single-precision rounding;
  * binning/order: the oracle's integer rule run on the GPU's single-precision
    (u, v, radius, depth) must reproduce tiles_touched, keys, ids and ranges
    bit for bit;
  * compositing: the oracle composites the GPU's records (widened to FP64)
    over the GPU's lists; image and T_final within 1e-5 absolute per pixel;
  * backward: the oracle's composite backward on the same records and lists,
    then its projection backward from the raw parameters; every gradient
    element within 1e-3 relative, floored at 1e-2 of the array's rms.
Pixels where a skip/stop/square-edge decision lies within single-precision
reach of its threshold (the oracle flags them) are excluded from the image
comparison and get zero loss weight in the backward comparison, so both sides
differentiate the same decisions.
"""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as O
from paper_2501_14534_amd import raster

# near-threshold windows: alpha (relative), transmittance (relative), square edge (pixels)
FLAG_EPS = (3e-5, 3e-5, 1e-3)
IMG_TOL = 1e-5
GRAD_RTOL = 1e-3
GRAD_FLOOR = 1e-2


def make_rasterizer(wl, opts=None, capacity=None, schedule=True):
    opts = opts or wl.opts
    sc = wl.scene
    return raster.Rasterizer(sc.n, sc.sh_degree, wl.cams, opts, mask_eps=sc.mask_eps, sh_mask_eps=sc.sh_mask_eps,
                             capacity=capacity, schedule=schedule, keep_keys=True)


def gpu_forward(wl, opts=None, capacity=None, params=None, schedule=True):
    r = make_rasterizer(wl, opts, capacity, schedule)
    params = params if params is not None else raster.to_device(wl.scene)
    r.forward(params)
    torch.cuda.synchronize()
    return r, params


def records(r) -> dict:
    rec = r.splat_records().cpu().numpy().astype(np.float64)
    return dict(uv=rec[:, 0:2], conic=rec[:, 2:5], opacity=rec[:, 5], radius=rec[:, 6].astype(np.int32),
                depth=rec[:, 7], rgb=rec[:, 8:11], valid=(rec[:, 11] == 1.0).astype(np.int32), raw=rec)


def gpu_lists(r) -> dict:
    K = r.pairs()
    return dict(K=K, keys=r.keys[:K].cpu().numpy().view(np.uint64), ids=r.ids[:K].cpu().numpy().view(np.uint32),
                ranges=r.ranges[: 2 * r.total_tiles].cpu().numpy().view(np.uint32).reshape(-1, 2),
                tiles_touched=r.tiles_touched[: r.V * r.n].cpu().numpy().view(np.uint32))


def check_binning(wl, opts, r) -> dict:
    """Oracle's integer rule on the GPU's single-precision records: bit-exact."""
    sp = records(r)
    rec32 = r.splat_records().cpu().numpy()
    ob = O.bin(wl.cams, opts, wl.scene.n, rec32[:, 0], rec32[:, 1], rec32[:, 7], sp["radius"], sp["valid"])
    gl = gpu_lists(r)
    assert not r.overflowed()
    np.testing.assert_array_equal(gl["tiles_touched"], ob["tiles_touched"])
    assert gl["K"] == ob["K"]
    np.testing.assert_array_equal(gl["keys"], ob["keys"])
    np.testing.assert_array_equal(gl["ids"], ob["ids"])
    np.testing.assert_array_equal(gl["ranges"], ob["ranges"])
    return gl


def oracle_forward_on_gpu_records(wl, opts, r):
    sp = records(r)
    gl = gpu_lists(r)
    fw = O.composite_fwd(wl.cams, opts, wl.scene.n, sp, gl["ids"], gl["ranges"], eps=FLAG_EPS)
    return fw, sp, gl


def check_forward(wl, opts, r) -> dict:
    fw, sp, gl = oracle_forward_on_gpu_records(wl, opts, r)
    img = r.image.cpu().numpy().astype(np.float64)
    T = r.T_final.cpu().numpy().astype(np.float64)
    last = r.last.cpu().numpy()
    flagged = fw["flags"] != 0
    ok_px = ~flagged
    ok3 = np.concatenate([np.tile(ok_px[o:o + c.width * c.height], 3) for o, c in
                          zip(np.cumsum([0] + [c.width * c.height for c in wl.cams[:-1]]), wl.cams)])
    err_img = np.abs(img - fw["image"])[ok3]
    err_T = np.abs(T - fw["T_final"])[ok_px]
    out = dict(max_img_err=float(err_img.max(initial=0.0)), max_T_err=float(err_T.max(initial=0.0)),
               flagged_frac=float(flagged.mean()), last_mismatch=int((last != fw["last_contrib"])[ok_px].sum()),
               fw=fw, flagged=flagged)
    assert out["max_img_err"] <= IMG_TOL, out["max_img_err"]
    assert out["max_T_err"] <= IMG_TOL, out["max_T_err"]
    assert out["last_mismatch"] == 0
    return out


def r24_violations(g, ref):
    """Elements outside |g - ref| <= 1e-3 max(|ref|, 1e-2 rms(ref)).

    The rms is taken over the reference's support (its non-zero elements):
    the floor stands for the gradient's typical magnitude, which elements
    that receive no gradient by construction (culled Gaussians, Gaussians
    outside a sampled subset of tiles) must not dilute."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    nz = ref[ref != 0.0]
    rms = float(np.sqrt(np.mean(nz ** 2))) if nz.size else 0.0
    tol = GRAD_RTOL * np.maximum(np.abs(ref), GRAD_FLOOR * rms)
    bad = np.abs(g - ref) > tol
    worst = float((np.abs(g - ref) / np.maximum(tol, 1e-300)).max(initial=0.0)) * GRAD_RTOL
    return int(bad.sum()), worst


def check_backward(wl, opts, r, params, flagged, seed=0) -> dict:
    """Random loss weights (zero on flagged pixels); GPU grads vs oracle grads."""
    P = r.total_pixels
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(3 * P).astype(np.float32) / np.float32(np.sqrt(3 * P))
    keep = np.concatenate([np.tile(~flagged[o:o + c.width * c.height], 3) for o, c in
                           zip(np.cumsum([0] + [c.width * c.height for c in wl.cams[:-1]]), wl.cams)])
    w[~keep] = 0.0
    dL = torch.from_numpy(w).cuda()
    grads = r.zero_grads(params)
    r.backward(params, dL, grads)
    torch.cuda.synchronize()
    sp = records(r)
    gl = gpu_lists(r)
    grad_rec = O.composite_bwd(wl.cams, opts, wl.scene.n, sp, gl["ids"], gl["ranges"], w.astype(np.float64))
    og = O.zero_grads(wl.scene)
    for v, c in enumerate(wl.cams):
        n = wl.scene.n
        O.project_bwd(wl.scene, c, opts, grad_rec[v * n:(v + 1) * n], og)
    res = {}
    gpu_rec = r.grad_records(dL).cpu().numpy()
    res["grad_rec"] = r24_violations(gpu_rec, grad_rec)
    for k, ref in og.items():
        res[k] = r24_violations(grads[k].cpu().numpy(), ref)
    return res


EPS32 = 2.0 ** -24


def check_projection(wl, opts, r) -> dict:
    """GPU records vs the oracle's FP64 projection.

    Tolerances follow single-precision rounding of each quantity: screen
    position and depth relative to the magnitudes summed in R mu + t; conic
    relative to its norm times the condition number of Sigma' (inversion);
    colour and opacity absolute.  Radius must match except where 3 sqrt(lambda)
    is within 1e-4 of an integer; validity must match except within 1e-5 of
    the near plane."""
    n = wl.scene.n
    o = O.project_views(wl.scene, wl.cams, opts)
    g = records(r)
    V = len(wl.cams)
    mu = np.tile(np.abs(wl.scene.means.astype(np.float64)).sum(0), V)
    tabs = np.concatenate([np.full(n, np.abs(c.t.astype(np.float64)).sum()) for c in wl.cams])
    fx = np.concatenate([np.full(n, float(c.fx)) for c in wl.cams])
    cx = np.concatenate([np.full(n, abs(float(c.cx)) + abs(float(c.cy))) for c in wl.cams])
    near = np.abs(o["depth"] - opts.near_plane) <= 1e-5 * np.maximum(1.0, np.abs(o["depth"]))
    vm = (g["valid"] != o["valid"]) & ~near
    assert not vm.any(), f"{int(vm.sum())} validity mismatches"
    both = (g["valid"] == 1) & (o["valid"] == 1)
    res = dict(valid=int(both.sum()))
    z = np.maximum(o["depth"][both], 1e-30)
    scale = mu[both] + tabs[both]
    tol_uv = 64 * EPS32 * (np.abs(o["uv"][both]).sum(1) + cx[both] + fx[both] * scale / z)
    err_uv = np.abs(g["uv"][both] - o["uv"][both]).max(1)
    res["uv"] = float((err_uv / tol_uv).max(initial=0))
    err_z = np.abs(g["depth"][both] - o["depth"][both])
    res["depth"] = float((err_z / (64 * EPS32 * scale)).max(initial=0))
    cov = o["cov2d"][both]
    mid = 0.5 * (cov[:, 0] + cov[:, 2])
    disc = np.sqrt(np.maximum(mid ** 2 - (cov[:, 0] * cov[:, 2] - cov[:, 1] ** 2), 0))
    kappa = (mid + disc) / np.maximum(mid - disc, 1e-30)
    qn = np.linalg.norm(o["conic"][both], axis=1)
    err_q = np.linalg.norm(g["conic"][both] - o["conic"][both], axis=1)
    res["conic"] = float((err_q / (256 * EPS32 * kappa * qn)).max(initial=0))
    res["opacity"] = float(np.abs(g["opacity"][both] - o["opacity"][both]).max(initial=0) / 1e-6)
    res["rgb"] = float(np.abs(g["rgb"][both] - o["rgb"][both]).max(initial=0) / 1e-5)
    s3 = 3 * np.sqrt(mid + disc)
    near_int = np.abs(s3 - np.round(s3)) <= 1e-4 * s3
    rad_bad = (g["radius"][both] != o["radius"][both]) & ~near_int
    res["radius_mismatch"] = int(rad_bad.sum())
    for k in ("uv", "depth", "conic", "opacity", "rgb"):
        assert res[k] <= 1.0, (k, res[k])
    assert res["radius_mismatch"] == 0
    return res
