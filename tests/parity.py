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
    over the GPU's lists; image and T_final within 1e-5 absolute per pixel,
    last_contrib equal;
  * backward: the oracle's composite backward on the same records and lists,
    then its projection backward from the raw parameters; every gradient
    element within 1e-3 relative, floored at 1e-2 of the reference's rms.

Near-threshold decisions (the decision-consistency protocol).  A pixel is
flagged when one of its skip/stop/cap/square-edge decisions lies within the
rounding that a single-precision evaluation can carry of its threshold.  Two
runs flag pixels:
  * the stage run: the oracle's walk over the GPU's records, with windows
    equal to the rounding bounds of the GPU's own float walk (FLAG_EPS);
  * the independent run: the oracle's whole FP64 chain (its own projection,
    binning and walk), with the same windows widened per record by the
    measured difference between the GPU's record and the FP64 one, and with
    near-equal depths and near-integer radii flagged.
A pixel that fails the image comparison must be flagged by the stage run (whose
windows bound the GPU walk's rounding on the same records); such pixels are the
excluded ones, and their fraction is bounded.  The independent run reports its
own flagged fraction and how far the GPU image is from the FP64 chain's image on
the pixels neither run flags.  The backward comparison gives every flagged pixel
zero loss weight on both sides, so both differentiate the same decisions.
"""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as O
from paper_2501_14534_amd import raster

EPS32 = 2.0 ** -24  # unit roundoff of single precision

# Rounding windows of the GPU's single-precision walk, per near-threshold
# decision, in units of the unit roundoff u (see the oracle's flag inputs):
#   alpha, fixed part: 4u (v_exp_f32 within 1 ulp = 2u, o' G rounded once, margin);
#   alpha, per unit of S = |A| dx^2/2 + |B dx dy| + |C| dy^2/2: 8u (the scaled
#     conic, dx, dy and the two fused multiply-adds put at most 7u S on the base-2
#     exponent, times ln 2 log2 e = 1 on alpha);
#   T, fixed part: u; T per composited Gaussian: 3u (1 - alpha and the product
#     rounded once each, margin), plus the propagated alpha window;
#   square edge: 2u |dx| (px - u rounded once; exact differences are not flagged);
#   depth order: not needed when the oracle walks the GPU's own lists.
FLAG_EPS = (4 * EPS32, 1 * EPS32, 0.0, 8 * EPS32, 3 * EPS32, 2 * EPS32, 0.0)
IMG_TOL = 1e-5
GRAD_RTOL = 1e-3
GRAD_FLOOR = 1e-2
# excluded pixels (failing the image comparison, all of them flagged): at most this fraction
MAX_EXCLUDED = 1e-4
# flagged pixels (zero loss weight in the backward comparison): at most this fraction
MAX_FLAGGED = 1e-3
# GPU image vs the independent FP64 chain on pixels no run flags (projection rounding included)
INDEP_TOL = 1e-3


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


def oracle_forward_on_gpu_records(wl, opts, r, tile_mask=None):
    sp = records(r)
    gl = gpu_lists(r)
    fw = O.composite_fwd(wl.cams, opts, wl.scene.n, sp, gl["ids"], gl["ranges"], eps=FLAG_EPS, tile_mask=tile_mask)
    return fw, sp, gl


def independent_flags(wl, opts, r, tile_mask=None, proj=None) -> dict:
    """Near-threshold pixels found by the oracle's own FP64 chain (projection, binning from
    the single-precision rounding of its values, walk), not by the GPU's records.

    The windows are FLAG_EPS widened, per record, by the measured difference between the
    GPU's record and the FP64 one: the screen-position difference (pixels) and the conic's
    relative difference (max over A and C of |dA|/|A|, plus |dB|/sqrt(|A C|), which bounds
    the change of the exponent by that multiple of S); opacity differences widen the fixed
    alpha window; records whose radius differs or whose 3 sqrt(lambda_max) lies within
    1e-4 of an integer flag the ring of pixels around their square.  Every measured
    difference is doubled.  Records that swap places in the depth order between the two
    runs are not flagged here: the stage run walks the GPU's own order and flags what
    such a swap can change there."""
    n = wl.scene.n
    o = proj if proj is not None else O.project_views(wl.scene, wl.cams, opts)
    g = records(r)
    both = (g["valid"] == 1) & (o["valid"] == 1)
    nrec = o["valid"].size
    rw = np.zeros((nrec, 2))
    rf = np.zeros(nrec, np.uint8)
    du = np.abs(g["uv"] - o["uv"]).max(1)
    A, B, Cc = (o["conic"][:, k] for k in range(3))
    dA, dB, dC = (np.abs(g["conic"][:, k] - o["conic"][:, k]) for k in range(3))
    with np.errstate(divide="ignore", invalid="ignore"):
        ec = np.maximum(dA / np.abs(A), dC / np.abs(Cc)) + dB / np.sqrt(np.abs(A * Cc))
        dop = np.abs(g["opacity"] - o["opacity"]) / o["opacity"]
    rw[both, 0] = 2.0 * du[both] + 1e-12
    rw[both, 1] = 2.0 * ec[both]
    cov = o["cov2d"]
    mid = 0.5 * (cov[:, 0] + cov[:, 2])
    disc = np.sqrt(np.maximum(mid ** 2 - (cov[:, 0] * cov[:, 2] - cov[:, 1] ** 2), 0))
    s3 = 3 * np.sqrt(np.maximum(mid + disc, 0))
    near_int = np.abs(s3 - np.round(s3)) <= 1e-4 * s3
    rf[(both & ((g["radius"] != o["radius"]) | near_int))] = 1
    eps = np.array(FLAG_EPS, np.float64)
    eps[0] += 2.0 * float(dop[both].max(initial=0.0))
    V = len(wl.cams)
    assert o["valid"].size == V * n
    lists = O.bin(wl.cams, opts, n, o["uv"][:, 0].astype(np.float32), o["uv"][:, 1].astype(np.float32),
                  o["depth"].astype(np.float32), o["radius"], o["valid"])
    fw = O.composite_fwd(wl.cams, opts, n, o, lists["ids"], lists["ranges"], eps=eps, tile_mask=tile_mask,
                         rec_flags=rf, rec_win=rw)
    return dict(flags=fw["flags"], image=fw["image"], eps=eps, max_pos_diff=float(du[both].max(initial=0.0)),
                max_conic_rel=float(ec[both].max(initial=0.0)))


def _per_channel(mask_px, cams):
    """Pixel mask [sum_v H W] -> image-element mask [sum_v 3 H W] (planar per view)."""
    out, off = [], 0
    for c in cams:
        k = c.width * c.height
        out.append(np.tile(mask_px[off:off + k], 3))
        off += k
    return np.concatenate(out) if out else np.zeros(0, bool)


def check_forward(wl, opts, r, tile_mask=None, pix_mask=None, max_excluded=MAX_EXCLUDED, independent=True) -> dict:
    """GPU image, T_final and last_contrib vs the oracle's walk over the GPU's records and lists.

    Every compared pixel (all, or pix_mask's) either matches (image and T_final within
    IMG_TOL, last_contrib equal) or is flagged near-threshold by the stage run; the
    fraction of such excluded pixels is at most max_excluded, and the flagged fraction at
    most MAX_FLAGGED.  The independent run (the oracle's own FP64 chain) reports its own
    flagged fraction and the largest difference between the GPU image and its image on the
    pixels neither run flags, which carries the single-precision projection's rounding
    (bounded by the projection comparison) and must stay under INDEP_TOL.
    Returns the fractions and the stage flags (zero loss weight for the backward)."""
    fw, sp, gl = oracle_forward_on_gpu_records(wl, opts, r, tile_mask)
    img = r.image.cpu().numpy().astype(np.float64)
    T = r.T_final.cpu().numpy().astype(np.float64)
    last = r.last.cpu().numpy()
    P = T.size
    cmp = np.ones(P, bool) if pix_mask is None else np.asarray(pix_mask, bool)
    stage = (fw["flags"] != 0) & cmp
    ind = independent_flags(wl, opts, r, tile_mask) if independent else None
    err_px = _max_per_pixel(np.abs(img - fw["image"]), wl.cams)
    err_T = np.abs(T - fw["T_final"])
    bad = cmp & ((err_px > IMG_TOL) | (err_T > IMG_TOL) | (last != fw["last_contrib"]))
    ncmp = max(int(cmp.sum()), 1)
    ok = cmp & ~bad
    out = dict(compared=int(cmp.sum()),
               max_img_err=float(err_px[ok].max(initial=0.0)), max_T_err=float(err_T[ok].max(initial=0.0)),
               unexplained=int((bad & ~stage).sum()), excluded=int(bad.sum()),
               excluded_frac=float(bad.sum()) / ncmp, flagged_frac=float(stage.sum()) / ncmp,
               flagged_ind_frac=None, indep_max_err=None, fw=fw, flagged=stage)
    if ind is not None:
        iflag = (ind["flags"] != 0) & cmp
        clean = cmp & ~iflag & ~stage
        out["flagged_ind_frac"] = float(iflag.sum()) / ncmp
        out["indep_max_err"] = float(_max_per_pixel(np.abs(img - ind["image"]), wl.cams)[clean].max(initial=0.0))
    print("  forward parity: " + ", ".join(f"{k} {out[k]:.3g}" if isinstance(out[k], float) else f"{k} {out[k]}"
                                            for k in ("compared", "max_img_err", "max_T_err", "excluded",
                                                      "excluded_frac", "flagged_frac", "flagged_ind_frac",
                                                      "indep_max_err") if out[k] is not None), flush=True)
    assert out["unexplained"] == 0, f"{out['unexplained']} pixels differ and are not near a threshold"
    assert out["excluded_frac"] <= max_excluded, out["excluded_frac"]
    assert out["flagged_frac"] <= MAX_FLAGGED, out["flagged_frac"]
    if ind is not None:
        assert out["indep_max_err"] <= INDEP_TOL, out["indep_max_err"]
    return out


def _max_per_pixel(err3, cams):
    """Image-element values [sum_v 3 H W] -> max over the three channels per pixel [sum_v H W]."""
    out, off = [], 0
    for c in cams:
        k = c.width * c.height
        out.append(err3[3 * off:3 * off + 3 * k].reshape(3, k).max(0))
        off += k
    return np.concatenate(out) if out else np.zeros(0)


def r24_violations(g, ref, support_rms=False, absparts=None, stats=None):
    """Elements outside |g - ref| <= 1e-3 max(|ref|, floor) (the gradient tolerance).

    floor = 1e-2 rms(ref), the rms over every element of the reference (with support_rms,
    over its non-zero elements, for comparisons on a sample of tiles where most Gaussians
    get no gradient by construction); with absparts (per element, the sum of the absolute
    contributions that cancel into it, oracle_param_grads) the floor is also at least
    1e-2 of that sum: an element that cancels more than a hundredfold is held to the
    typical size of what it sums, as a near-zero element is held to the array's.
    stats (dict), if given, receives the number of elements whose bound is the floor."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    base = ref[ref != 0.0] if support_rms else ref
    rms = float(np.sqrt(np.mean(base ** 2))) if base.size else 0.0
    floor = np.full(ref.shape, GRAD_FLOOR * rms)
    if absparts is not None:
        floor = np.maximum(floor, GRAD_FLOOR * np.asarray(absparts, np.float64))
    tol = GRAD_RTOL * np.maximum(np.abs(ref), floor)
    bad = np.abs(g - ref) > tol
    worst = float((np.abs(g - ref) / np.maximum(tol, 1e-300)).max(initial=0.0)) * GRAD_RTOL
    if stats is not None:
        stats["on_floor"] = int((floor > np.abs(ref)).sum())
        stats["on_cancel_floor"] = int(((floor > np.abs(ref)) & (floor > GRAD_FLOOR * rms)).sum())
    return int(bad.sum()), worst


def oracle_param_grads(wl, opts, grad_rec):
    """The oracle's projection backward (FP64) of per-record gradients [V*n, 9] into the raw
    parameters, and per parameter element the sum of the absolute values of its
    contributions from each (view, record-gradient component): how much cancels into it.
    Each Gaussian's chain reads only its own parameters, so the work runs over the
    Gaussians with a non-zero record gradient (all of them under the progressive
    low-pass, whose s depends on the Gaussian count)."""
    n = wl.scene.n
    V = len(wl.cams)
    gr = np.asarray(grad_rec, np.float64).reshape(V, n, -1)
    if getattr(opts, "lowpass_progressive", 0):
        idx = np.arange(n)
    else:
        idx = np.flatnonzero(np.any(gr != 0.0, axis=(0, 2)))
    sub = wl.scene.subset(idx)
    og_s = O.zero_grads(sub)
    absparts_s = {k: np.zeros_like(v) for k, v in og_s.items()}
    for v, c in enumerate(wl.cams):
        gv = np.ascontiguousarray(gr[v][idx])
        O.project_bwd(sub, c, opts, gv, og_s)
        for comp in range(gv.shape[1]):
            if not np.any(gv[:, comp]):
                continue
            x = np.zeros_like(gv)
            x[:, comp] = gv[:, comp]
            part = O.project_bwd(sub, c, opts, x, O.zero_grads(sub))
            for k in absparts_s:
                absparts_s[k] += np.abs(part[k])
    og = O.zero_grads(wl.scene)
    absparts = {k: np.zeros_like(v) for k, v in og.items()}
    for k in og:
        og[k][..., idx] = og_s[k]
        absparts[k][..., idx] = absparts_s[k]
    return og, absparts


def check_backward(wl, opts, r, params, flagged, seed=0) -> dict:
    """Random loss weights (zero on flagged pixels); GPU grads vs oracle grads."""
    P = r.total_pixels
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(3 * P).astype(np.float32) / np.float32(np.sqrt(3 * P))
    w[_per_channel(np.asarray(flagged, bool), wl.cams)] = 0.0
    dL = torch.from_numpy(w).cuda()
    grads = r.zero_grads(params)
    n = wl.scene.n
    V = len(wl.cams)
    # dL/d(u, v) per record, [V][2][n] (the densification statistics output), accumulated
    mean2d = torch.zeros(V * 2 * n, dtype=torch.float32, device=dL.device)
    r.backward(params, dL, grads, mean2d)
    torch.cuda.synchronize()
    sp = records(r)
    gl = gpu_lists(r)
    grad_rec = O.composite_bwd(wl.cams, opts, n, sp, gl["ids"], gl["ranges"], w.astype(np.float64))
    og, absparts = oracle_param_grads(wl, opts, grad_rec)
    res = {}
    gpu_rec = r.grad_records(dL).cpu().numpy()
    res["grad_rec"] = r24_violations(gpu_rec, grad_rec)
    ref_m2d = grad_rec[:, 0:2].reshape(V, n, 2).transpose(0, 2, 1).reshape(-1)
    res["mean2d"] = r24_violations(mean2d.cpu().numpy(), ref_m2d)
    floors = {}
    for k, ref in og.items():
        st = {}
        res[k] = r24_violations(grads[k].cpu().numpy(), ref, absparts=absparts[k], stats=st)
        floors[k] = (st["on_floor"], st["on_cancel_floor"])
    print("  backward parity (bad, worst): " + str(res) + "; elements on the floor (all, cancellation): " + str(floors), flush=True)
    return res




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
