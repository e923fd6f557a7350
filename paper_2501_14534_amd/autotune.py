"""Tile-shape / batch-depth / pixels-per-thread / backward-chunk autotuner with a JSON cache.

The image does not depend on these choices (every pixel walks the same splats
in the same order whatever the tiling: each pixel applies the square test), so
the tuner may pick freely by time.  Candidates are timed as whole fwd+bwd
steps of the workload: first the tilings with the default backward chunk,
then the backward chunk lengths for the fastest tiling; the winner is stored
per (device arch, workload key).
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import Dict, Iterable, List, Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "autotune_cache.json")

# (tile_w, tile_h, batch_depth, pixels_per_thread, subtile_cull)
CANDIDATES: List[Tuple[int, int, int, int, int]] = [
    (16, 16, 256, 1, 0), (16, 16, 256, 1, 1), (16, 16, 512, 1, 1), (16, 16, 1024, 1, 1), (16, 16, 128, 1, 1), (16, 16, 64, 1, 1),
    (16, 16, 256, 2, 1), (16, 16, 128, 2, 1), (16, 16, 64, 2, 1),
    (16, 16, 256, 4, 1), (16, 16, 128, 4, 1), (16, 16, 64, 4, 1), (16, 16, 32, 4, 1),
    (8, 8, 64, 1, 1), (8, 8, 32, 1, 1), (16, 8, 128, 1, 1), (16, 8, 64, 2, 1), (32, 8, 256, 1, 1),
    (32, 8, 128, 2, 1), (32, 16, 256, 2, 1), (32, 16, 128, 4, 1),
]
# list entries per backward work item (0: one item per tile)
CHUNKS: List[int] = [256, 512, 1024, 2048, 4096, 0]


def workload_key(wl) -> str:
    res = ",".join(f"{c.width}x{c.height}" for c in wl.cams)
    sc = wl.scene
    nb = 1 << max(0, int(sc.n - 1).bit_length())  # power-of-two bucket of the Gaussian count
    return f"n<={nb}|deg{sc.sh_degree}|{res}"


def _arch() -> str:
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # noqa: BLE001 - no device: no cached entry applies
        return "none"


def load_cache() -> Dict[str, dict]:
    if not os.path.exists(CACHE):
        return {}
    try:
        return json.load(open(CACHE))
    except ValueError:
        return {}


def best_opts(wl, arch: Optional[str] = None):
    """Cached winner for this workload on this device, else the workload's default options."""
    arch = arch or _arch()
    e = load_cache().get(f"{arch}|{workload_key(wl)}")
    if not e:
        return wl.opts
    return dataclasses.replace(wl.opts, tile_w=e["tile_w"], tile_h=e["tile_h"], batch_depth=e["batch_depth"],
                               pixels_per_thread=e["pixels_per_thread"], subtile_cull=e.get("subtile_cull", 1),
                               bwd_chunk=e.get("bwd_chunk", wl.opts.bwd_chunk))


def tune(wl, candidates: Iterable[Tuple[int, int, int, int, int]] = CANDIDATES, chunks: Iterable[int] = CHUNKS,
         steps: int = 5, warmup: int = 2, write: bool = True, verbose: bool = True,
         cache_path: Optional[str] = None) -> dict:
    """Time each candidate's fwd+bwd step and store the fastest in the cache."""
    import numpy as np
    import torch

    from . import raster

    sc = wl.scene
    params = raster.to_device(sc)
    target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).cuda()
    results = []
    ref_img = None
    grid = [(tw, th, bd, ppt, cull, wl.opts.bwd_chunk) for tw, th, bd, ppt, cull in candidates]
    tried = set()

    def run(cands):
        nonlocal ref_img
        for cand in cands:
            if cand in tried:
                continue
            tried.add(cand)
            results.append(_time_one(wl, params, target, cand, steps, warmup, verbose))
            if ref_img is None:
                ref_img = results[-1].pop("_img")
            else:
                results[-1]["image_equal"] = bool(torch.equal(results[-1].pop("_img"), ref_img))

    run(grid)
    ok = [x for x in results if x["image_equal"]]
    b = min(ok, key=lambda x: x["ms"])
    run([(b["tile_w"], b["tile_h"], b["batch_depth"], b["pixels_per_thread"], b["subtile_cull"], ch) for ch in chunks])
    ok = [x for x in results if x["image_equal"]]
    best = min(ok, key=lambda x: x["ms"])
    if write:
        path = cache_path or CACHE
        cache = json.load(open(path)) if os.path.exists(path) else {}
        cache[f"{_arch()}|{workload_key(wl)}"] = best
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return dict(best=best, results=results)


def _time_one(wl, params, target, cand, steps, warmup, verbose) -> dict:
    """One candidate's fwd+bwd step time (graph replays) and its image."""
    import time

    import torch

    from . import raster

    sc = wl.scene
    tw, th, bd, ppt, cull, chunk = cand
    o = dataclasses.replace(wl.opts, tile_w=tw, tile_h=th, batch_depth=bd, pixels_per_thread=ppt,
                            subtile_cull=cull, bwd_chunk=chunk)
    r = raster.Rasterizer(sc.n, sc.sh_degree, wl.cams, o, mask_eps=sc.mask_eps, sh_mask_eps=sc.sh_mask_eps)
    st = raster.Step(r, params, target, graph=True)
    st.run()
    for _ in range(warmup):
        st.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st.launch()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    out = dict(tile_w=tw, tile_h=th, batch_depth=bd, pixels_per_thread=ppt, subtile_cull=cull, bwd_chunk=chunk,
               ms=ms, image_equal=True, _img=r.image.clone())
    if verbose:
        print(f"  tile {tw}x{th} batch {bd} ppt {ppt} cull {cull} chunk {chunk}: {ms:.3f} ms/step", flush=True)
    del st, r
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    import argparse

    from . import scenes

    ap = argparse.ArgumentParser(description="time the candidate launch shapes of a workload and cache the fastest")
    ap.add_argument("--config", type=int, nargs="+", default=[4])
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--cache", default=None, help="cache file to update (default: the package cache)")
    a = ap.parse_args()
    for k in a.config:
        wl = scenes.config(k)
        print(f"workload {k}: {wl.name}", flush=True)
        res = tune(wl, steps=a.steps, cache_path=a.cache)
        print(f"best: {res['best']}", flush=True)
