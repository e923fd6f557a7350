"""Throughput of the rasterizer's fwd+bwd hot path on one MI355X.

Workload (default): 1,000,000 Gaussians (unit-sphere shell, SH degree 3,
volume and SH-band masks) rendered into 8 views of mixed progressive-training
resolutions (3x316x208, 3x632x416, 2x1264x832; 3.09 Mpix per step) in one
batched, HIP-graph-captured step.  A step = projection, binning/sort,
forward compositing, L2 loss gradient, backward (composite + projection).

Prints ONE JSON line: batched Mpix/s (the value), the per-view path's Mpix/s
and the batched-over-per-view speedup (with the agreement of the two paths),
per-stage times, the roofline of the dominant kernel and the FP64 oracle's
throughput on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_FP32_TFLOPS = 157.3   # MI355X published fp32 vector peak (packed FP32: 256 CU x 4 SIMD x 16 lanes x 2 x 2 x 2.4 GHz)
PEAK_FP32_ISSUE_TFLOPS = 78.6  # the same without packed FP32, which this build does not emit
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E
# Algorithmic work per composited (pixel, splat) pair: the forward blend costs
# about 20 vector operations and one exponential, the backward about 50 vector
# operations, one exponential and one reciprocal.  Counted per composited pair
# (sum of last_contrib over the pixels), each operation as one FLOP.
FWD_FLOP_PER_PAIR = 21.0
BWD_FLOP_PER_PAIR = 52.0
COUNT_FLOP_PER_PAIR = 14.0  # the forward walk without the colour update (7 of its 20 operations)
STAGE_REPS = 50             # stage timings: median over this many repetitions


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=4, help="workload 1..5")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--tile", type=str, default=None, help="WxH tile override, e.g. 16x16")
    ap.add_argument("--batch-depth", type=int, default=None)
    ap.add_argument("--ppt", type=int, default=None)
    ap.add_argument("--cull", type=int, default=None, choices=[0, 1], help="sub-tile culling override")
    ap.add_argument("--bwd-chunk", type=int, default=None, help="backward chunk length override (0: one per tile)")
    ap.add_argument("--fwd-chunk", type=int, default=None, help="forward chunk length override (0: one per tile)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target CPU work of the oracle sample")
    ap.add_argument("--calibration-copy-bytes", type=int, default=0,
                    help="also launch a plain copy kernel (elementwise x1) of this many bytes, for counter scaling")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2501_14534_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_counters(kernel: str, workload: str, src_hash: str):
    """VALU and LDS utilisation of a kernel from committed rocprofv3 --pmc summaries, if taken on this
    kernel source."""
    p = os.path.join(ROOT, "profiles", "pmc_valu_lds.json")
    if not os.path.exists(p):
        return None
    try:
        e = json.load(open(p)).get(f"{kernel}@{workload}")
        if e and e.get("source_hash") == src_hash:
            return {k: e[k] for k in ("valu_insts_per_simd_cycle", "valu_issue_frac_fp32", "valu_insts_per_wave",
                                      "lds_util", "lds_bank_conflict_per_access", "lds_bytes_per_launch") if k in e}
    except (ValueError, KeyError, TypeError):
        return None
    return None


def load_traffic(kernel: str, workload: str, src_hash: str):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, if taken on this kernel source."""
    p = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(f"{kernel}@{workload}")
        if e and e.get("source_hash") == src_hash:
            return float(e["hbm_bytes_per_launch"])
    except (ValueError, KeyError, TypeError):
        return None
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    import dataclasses

    import torch

    from paper_2501_14534_amd import autotune, gs, raster, scenes

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    gs.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibration_copy_bytes > 0:
        src = torch.ones(args.calibration_copy_bytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    wl = scenes.config(args.config)
    opts = autotune.best_opts(wl)
    if args.tile:
        tw, th = (int(x) for x in args.tile.lower().split("x"))
        opts = dataclasses.replace(opts, tile_w=tw, tile_h=th)
    if args.batch_depth:
        opts = dataclasses.replace(opts, batch_depth=args.batch_depth)
    if args.ppt:
        opts = dataclasses.replace(opts, pixels_per_thread=args.ppt)
    if args.cull is not None:
        opts = dataclasses.replace(opts, subtile_cull=args.cull)
    if args.bwd_chunk is not None:
        opts = dataclasses.replace(opts, bwd_chunk=args.bwd_chunk)
    if args.fwd_chunk is not None:
        opts = dataclasses.replace(opts, fwd_chunk=args.fwd_chunk)
    sc = wl.scene
    V = len(wl.cams)
    pixels = wl.pixels
    params = raster.to_device(sc)
    target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).to(dev)

    def make(cams, tgt):
        r = raster.Rasterizer(sc.n, sc.sh_degree, cams, opts, mask_eps=sc.mask_eps, sh_mask_eps=sc.sh_mask_eps)
        return raster.Step(r, params, tgt, graph=not args.no_graph, loss_views=V)

    # ---------------- batched path (all views in one call per stage) ----------------
    step = make(wl.cams, target)
    step.run()  # sizes the binning capacity (host check), captures the graph
    for _ in range(args.warmup):
        step.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step.launch()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert not step.rast.overflowed()
    ms = (t1 - t0) * 1e3 / args.steps
    value = pixels * args.steps / (t1 - t0) / 1e6

    # ---------------- per-view path (one call per stage per view) ----------------
    per_view = None
    if not args.no_per_view and V > 1:
        offs = np.cumsum([0] + [3 * c.pixels for c in wl.cams])
        pv = [make([c], target[offs[i]:offs[i + 1]]) for i, c in enumerate(wl.cams)]
        for s in pv:
            s.run()
        for _ in range(args.warmup):
            for s in pv:
                s.launch()
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.steps):
            for s in pv:
                s.launch()
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        # agreement: batched image == per-view images; gradients summed over views
        step.launch()
        torch.cuda.synchronize()
        img_b = step.rast.image
        img_p = torch.cat([s.rast.image for s in pv])
        img_err = float((img_b - img_p).abs().max())
        g_err = 0.0
        for k, gb in step.grads.items():
            gp = sum(s.grads[k] for s in pv)
            rms = float(gp.pow(2).mean().sqrt())
            tol = torch.clamp(gp.abs(), min=1e-2 * rms)
            g_err = max(g_err, float(((gb - gp).abs() / tol).max()) if gb.numel() else 0.0)
        per_view = dict(mpix_s=pixels * args.steps / (p1 - p0) / 1e6, ms_per_step=(p1 - p0) * 1e3 / args.steps,
                        speedup=(p1 - p0) / (t1 - t0), image_max_abs_diff=img_err, grad_max_rel_diff=g_err,
                        agree_1e5=bool(img_err <= 1e-5 and g_err <= 1e-5))
        del pv
        torch.cuda.empty_cache()

    # ---------------- stage timing with HIP events on the launch stream ----------------
    r = step.rast
    stream = torch.cuda.current_stream()  # every call below launches on it
    names = ["project", "bin_sort", "render_fwd", "blend_bwd", "project_bwd"]
    samples = {k: [] for k in names}
    grad_pair = torch.zeros(r.capacity * gs.GRAD_FLOATS, dtype=torch.float32, device=dev)
    dL = step.dL
    for _ in range(STAGE_REPS):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        ev[0].record(stream)
        r.project(params)
        ev[1].record(stream)
        r.bin_sort()
        ev[2].record(stream)
        r.render_fwd()
        ev[3].record(stream)
        r.blend_bwd(dL, grad_pair)
        ev[4].record(stream)
        r.project_bwd(params, grad_pair, step.grads, assign=True)
        ev[5].record(stream)
        torch.cuda.synchronize()
        for i, k in enumerate(names):
            samples[k].append(ev[i].elapsed_time(ev[i + 1]))
    stage_ms = {k: float(np.median(v)) for k, v in samples.items()}
    # the compositing walks and the loss gradient as one launch (gs_render_fwd_bwd_l2, which the
    # step uses) against the separate calls it stands for
    fsamples, ssamples = [], []
    for _ in range(STAGE_REPS):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        r.render_fwd_bwd_l2(params, step.target, step.loss_views, step.grads, dL_out=dL, assign=True)
        ev[1].record(stream)
        r.render_fwd()
        raster.l2_loss_grad(r, r.image, step.target, step.loss_views, dL)
        r.render_bwd(params, dL, step.grads, assign=True)
        ev[2].record(stream)
        torch.cuda.synchronize()
        fsamples.append(ev[0].elapsed_time(ev[1]))
        ssamples.append(ev[1].elapsed_time(ev[2]))
    fused_walks = dict(ms=round(float(np.median(fsamples)), 4), separate_ms=round(float(np.median(ssamples)), 4),
                       what="render_fwd + loss gradient + render_bwd (walk and projection backward) in one call; "
                            "separate_ms: the three calls")
    K = r.pairs()
    useful_pairs = int(r.last.to(torch.int64).sum())
    # list entries walked: per tile, the largest last_contrib of its pixels
    walked = 0
    off = 0
    for c in wl.cams:
        tw, th = opts.tile_w, opts.tile_h
        TX, TY = -(-c.width // tw), -(-c.height // th)
        lc = r.last[off:off + c.pixels].view(c.height, c.width)
        pad = torch.zeros(TY * th, TX * tw, dtype=lc.dtype, device=lc.device)
        pad[:c.height, :c.width] = lc
        walked += int(pad.view(TY, th, TX, tw).amax(dim=(1, 3)).to(torch.int64).sum())
        off += c.pixels

    # dominant single-kernel stage (project_bwd runs two kernels: colour, then geometry;
    # render_fwd's stage also holds a fill of the chunk-slot owners, ~5 us)
    single = {"render_fwd": "render_fwd_kernel", "blend_bwd": "render_bwd_kernel", "project": "project_kernel"}
    dom = max(single, key=lambda k: stage_ms[k])
    src_hash = kernel_source_hash()
    workload = f"config{args.config}"
    t_s = stage_ms[dom] * 1e-3
    if dom in ("render_fwd", "blend_bwd"):
        flop = useful_pairs * (FWD_FLOP_PER_PAIR if dom == "render_fwd" else BWD_FLOP_PER_PAIR)
        achieved = flop / t_s / 1e12
        roof = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_FP32_TFLOPS, 5),
                    frac_of_unpacked_peak=round(achieved / PEAK_FP32_ISSUE_TFLOPS, 5),
                    work=f"{FWD_FLOP_PER_PAIR if dom == 'render_fwd' else BWD_FLOP_PER_PAIR:g} FLOP per composited "
                         f"pair x {useful_pairs} composited pairs")
    else:
        nrec = V * sc.n
        byts = 252.0 * sc.n + 52.0 * nrec  # project: parameters read once, 48 + 4 B per record
        achieved = byts / t_s / 1e9
        roof = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(achieved / PEAK_HBM_GBS, 5))
    roof["kernel"] = single[dom]
    roof["ms_per_launch"] = round(stage_ms[dom], 4)
    roof["traffic"] = load_traffic(single[dom], workload, src_hash)
    roof["traffic_source"] = "profiles/pmc_traffic.json (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE of this kernel source)"
    # VALU and LDS utilisation of the two blend walks (rocprofv3 --pmc, committed summaries)
    walks = {k: load_counters(k, workload, src_hash) for k in ("render_fwd_kernel", "render_bwd_kernel")}
    roof["valu_lds"] = {k: v for k, v in walks.items() if v is not None} or None

    # ---------------- L1 + D-SSIM loss (Eq. 7) on the rendered views ----------------
    from paper_2501_14534_amd.photometric import PhotometricLoss
    pl = PhotometricLoss(wl.cams)
    dl_buf = torch.empty_like(r.image)
    for _ in range(3):
        pl(r.image, target, out=dl_buf)
    lev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    nl = max(5, args.steps)
    lev[0].record(stream)
    for _ in range(nl):
        pl(r.image, target, out=dl_buf)
    lev[1].record(stream)
    torch.cuda.synchronize()
    loss_ms = lev[0].elapsed_time(lev[1]) / nl
    elems = 3 * pixels
    loss_bytes = 44.0 * elems  # fwd: x, y in, 3 partial maps out; bwd: maps, x, y in, gradient out
    l1_dssim = dict(ms_per_call=round(loss_ms, 4), loss=round(float(pl.loss[-1]), 6),
                    roofline=dict(bound="hbm", achieved=round(loss_bytes / (loss_ms * 1e-3) / 1e9, 1),
                                  peak=PEAK_HBM_GBS, unit="GB/s",
                                  frac=round(loss_bytes / (loss_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 5)),
                    kernels="ssim_fwd_kernel + ssim_bwd_kernel + loss_reduce_kernel + loss_mean_kernel")

    # ---------------- significance score (Eq. 4) over the step's views ----------------
    hits = torch.zeros(sc.n, dtype=torch.int32, device=dev)
    score = torch.empty(sc.n, dtype=torch.float32, device=dev)
    for _ in range(2):
        r.count_hits(hits)
        raster.significance(params, hits, 0.9, sc.mask_eps, out=score)
    hits.zero_()
    sev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ns = max(5, args.steps)
    sev[0].record(stream)
    for _ in range(ns):
        r.count_hits(hits)
    sev[1].record(stream)
    for _ in range(ns):
        raster.significance(params, hits, 0.9, sc.mask_eps, out=score)
    sev[2].record(stream)
    torch.cuda.synchronize()
    count_ms = sev[0].elapsed_time(sev[1]) / ns
    score_ms = sev[1].elapsed_time(sev[2]) / ns
    hit_total = int(hits.to(torch.int64).sum()) // ns
    count_tflops = useful_pairs * COUNT_FLOP_PER_PAIR / (count_ms * 1e-3) / 1e12
    significance = dict(count_hits_ms=round(count_ms, 4), score_ms=round(score_ms, 4), hits_per_call=hit_total,
                        roofline=dict(bound="alu", achieved=round(count_tflops, 3), peak=PEAK_FP32_TFLOPS,
                                      unit="TFLOP/s", frac=round(count_tflops / PEAK_FP32_TFLOPS, 5)),
                        kernels="render_fwd_kernel<COUNT> + select_hist/pick (4 passes) + significance_kernel")

    # ---------------- FP64 oracle on the host cores (bounded sample) ----------------
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import baseline
        cpu = baseline.measure(wl, opts, target_seconds=args.cpu_seconds)
        cpu["cpu_model"] = baseline.cpu_model()
        cpu["host_threads"] = len(os.sched_getaffinity(0))
        cpu["one_thread"] = baseline.measure_one_thread(wl, opts, target_seconds=max(4.0, args.cpu_seconds / 3))

    out = {
        "metric": "fwd+bwd rasterized Mpix/s at 1M Gaussians; batched-vs-per-view speedup at 1e-5",
        "value": round(value, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Gaussians and cameras shaped like the paper's scenes; no dataset)",
        "config": {"workload": wl.name, "gaussians": sc.n, "views": V, "pixels_per_step": pixels,
                   "resolutions": [f"{c.width}x{c.height}" for c in wl.cams], "sh_degree": sc.sh_degree,
                   "tile": f"{opts.tile_w}x{opts.tile_h}", "batch_depth": opts.batch_depth,
                   "pixels_per_thread": opts.pixels_per_thread, "subtile_cull": opts.subtile_cull,
                   "bwd_chunk": opts.bwd_chunk, "fwd_chunk": opts.fwd_chunk,
                   "graph": not args.no_graph},
        "per_view": per_view,
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "fused_walks": fused_walks,
        "pairs": K,
        "walked_entries": walked,
        "evaluated_pairs": walked * opts.tile_w * opts.tile_h,
        "useful_pairs": useful_pairs,
        "stage_timing": f"HIP events on the launch stream, median of {STAGE_REPS} eager repetitions",
        "roofline": roof,
        "cpu_baseline": cpu,
        "l1_dssim": l1_dssim,
        "significance": significance,
        "kernel_source": src_hash,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
