"""Times the FP64 oracle on a bounded sample of a workload (benchmark CPU baseline).

TEST INFRASTRUCTURE ONLY (the benchmark's cpu_baseline leg).  The oracle is
run as it stands -- not tuned for speed -- on the host cores it was built for
(OpenMP threads as the environment sets them):
  * projection of every (view, Gaussian) record and binning/ordering of the
    whole workload are run in full;
  * forward and backward compositing run on every tile when a probe of 5% of
    the tiles says that fits 60% of the time budget, else on a random subset
    sized to the budget and scaled to all tiles by the tile fraction;
  * the projection backward runs on every record when that fits 30% of the
    budget, else on a random subset of one view's records, scaled by the
    record fraction and the view count.
The reported rate is total pixels / (sum of the scaled stage times).
A second, smaller run on one thread (measure_one_thread) times each stage on a
random sample -- projection and projection backward on a subset of the
Gaussians, compositing on a subset of the tiles, binning in full -- and scales
each by its sample fraction.
"""
from __future__ import annotations

import time

import numpy as np

from . import oracle as O


def _t(fn):
    t0 = time.perf_counter()
    out = fn()
    return out, time.perf_counter() - t0


def measure(wl, opts, target_seconds: float = 20.0, seed: int = 0) -> dict:
    sc = wl.scene
    n, V = sc.n, len(wl.cams)
    rng = np.random.default_rng(seed)
    sp, t_proj = _t(lambda: O.project_views(sc, wl.cams, opts))
    lists, t_bin = _t(lambda: O.bin(wl.cams, opts, n, sp["uv"][:, 0].astype(np.float32),
                                     sp["uv"][:, 1].astype(np.float32), sp["depth"].astype(np.float32),
                                     sp["radius"], sp["valid"]))
    T = lists["ranges"].shape[0]
    P = wl.pixels
    dl = rng.standard_normal(3 * P) / np.sqrt(3 * P)

    def composite(tiles):
        mask = np.zeros(T, np.uint8)
        mask[tiles] = 1
        _, tf = _t(lambda: O.composite_fwd(wl.cams, opts, n, sp, lists["ids"], lists["ranges"], tile_mask=mask))
        grec, tb = _t(lambda: O.composite_bwd(wl.cams, opts, n, sp, lists["ids"], lists["ranges"], dl,
                                              tile_mask=mask))
        return tf, tb

    order = rng.permutation(T)
    probe = order[: max(1, T // 20)]
    tf, tb = composite(probe)
    per_tile = (tf + tb) / len(probe)
    if per_tile * T <= 0.6 * target_seconds:
        sample = order  # every tile fits the budget
    else:
        budget = max(0.4 * target_seconds - (tf + tb), 0.0)
        extra = int(min(T - len(probe), budget / max(per_tile, 1e-9)))
        sample = order[: len(probe) + extra]
    tf, tb = composite(sample)
    ft = len(sample) / T

    # projection backward: a random subset of records with unit splat gradients
    rec_cost_probe = max(1, min(n, max(2000, n // 20)))
    idx = rng.choice(n, size=rec_cost_probe, replace=False)
    sub = sc.subset(np.sort(idx))
    grads = O.zero_grads(sub)
    gr = np.ones((sub.n, 9))
    _, tp = _t(lambda: O.project_bwd(sub, wl.cams[0], opts, gr, grads))
    per_rec = tp / sub.n
    if per_rec * n * V <= 0.3 * target_seconds:  # every view and Gaussian fits the budget
        grads = O.zero_grads(sc)
        gr = np.ones((n, 9))
        t0 = time.perf_counter()
        for c in wl.cams:
            O.project_bwd(sc, c, opts, gr, grads)
        tp = time.perf_counter() - t0
        sub, fr, t_pbwd_full, all_views = sc, 1.0, tp, True
    else:
        m = int(min(n, max(rec_cost_probe, 0.25 * target_seconds / max(per_rec, 1e-12))))
        idx = rng.choice(n, size=m, replace=False)
        sub = sc.subset(np.sort(idx))
        grads = O.zero_grads(sub)
        gr = np.ones((sub.n, 9))
        _, tp = _t(lambda: O.project_bwd(sub, wl.cams[0], opts, gr, grads))
        fr = sub.n / n
        t_pbwd_full = tp / fr * V
        all_views = False

    total = t_proj + t_bin + tf / ft + tb / ft + t_pbwd_full
    return {
        "value": round(P / total / 1e6, 5),
        "unit": "Mpix/s",
        "cores": O.num_threads(),
        "kind": "oracle",
        "sample": (f"FP64 oracle: projection of all {V * n} records and binning of all {lists['K']} pairs in full; "
                   f"forward+backward compositing on {len(sample)} of {T} tiles" +
                   (" (all)" if len(sample) == T else " (random), scaled by the tile fraction") +
                   f"; projection backward on {sub.n} of {n} Gaussians" +
                   (" in all views" if all_views else " in one view, scaled by the record fraction and view count")),
        "stage_s": {"project": round(t_proj, 3), "bin": round(t_bin, 3),
                    "composite_fwd_scaled": round(tf / ft, 3), "composite_bwd_scaled": round(tb / ft, 3),
                    "project_bwd_scaled": round(t_pbwd_full, 3)},
        "measured_s": round(t_proj + t_bin + tf + tb + tp, 3),
    }


def cpu_model() -> str:
    """The host CPU's model name (the "model name" line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measure_one_thread(wl, opts, target_seconds: float = 8.0, seed: int = 1) -> dict:
    """The oracle on one thread, each stage on a sample scaled by its fraction."""
    sc = wl.scene
    n, V = sc.n, len(wl.cams)
    rng = np.random.default_rng(seed)
    prev = O.num_threads()
    # lists of the whole workload (not timed, all threads)
    sp = O.project_views(sc, wl.cams, opts)
    O.set_threads(1)
    try:
        m = int(min(n, max(500, n // 200)))
        sub = sc.subset(np.sort(rng.choice(n, size=m, replace=False)))
        _, tp = _t(lambda: O.project_views(sub, wl.cams, opts))
        t_proj = tp * n / m
        lists, t_bin = _t(lambda: O.bin(wl.cams, opts, n, sp["uv"][:, 0].astype(np.float32),
                                         sp["uv"][:, 1].astype(np.float32), sp["depth"].astype(np.float32),
                                         sp["radius"], sp["valid"]))
        T = lists["ranges"].shape[0]
        P = wl.pixels
        dl = rng.standard_normal(3 * P) / np.sqrt(3 * P)
        order = rng.permutation(T)
        budget = 0.5 * target_seconds
        spent, k, tf, tb = 0.0, 0, 0.0, 0.0
        step = max(1, T // 200)
        while k < T and spent < budget:
            mask = np.zeros(T, np.uint8)
            mask[order[k:k + step]] = 1
            _, a = _t(lambda: O.composite_fwd(wl.cams, opts, n, sp, lists["ids"], lists["ranges"], tile_mask=mask))
            _, b = _t(lambda: O.composite_bwd(wl.cams, opts, n, sp, lists["ids"], lists["ranges"], dl,
                                              tile_mask=mask))
            tf, tb, spent, k = tf + a, tb + b, spent + a + b, k + step
        ft = min(k, T) / T
        grads = O.zero_grads(sub)
        gr = np.ones((sub.n, 9))
        _, tpb = _t(lambda: O.project_bwd(sub, wl.cams[0], opts, gr, grads))
        t_pbwd = tpb * (n / m) * V
    finally:
        O.set_threads(prev)
    total = t_proj + t_bin + (tf + tb) / ft + t_pbwd
    return {"value": round(wl.pixels / total / 1e6, 5), "unit": "Mpix/s", "cores": 1,
            "sample": f"one thread: projection and projection backward on {m} of {n} Gaussians, compositing on "
                      f"{min(k, T)} of {T} tiles (each scaled by its fraction), binning in full",
            "stage_s": {"project_scaled": round(t_proj, 3), "bin": round(t_bin, 3),
                        "composite_scaled": round((tf + tb) / ft, 3), "project_bwd_scaled": round(t_pbwd, 3)}}
