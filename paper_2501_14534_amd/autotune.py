"""Launch-shape autotuner with a JSON cache: tile shape, batch depth, pixels per
thread, sub-tile culling, backward chunk length and forward chunk length.

The image does not depend on the first five choices (every pixel walks the
same splats in the same order whatever the tiling: each pixel applies the
square test), so the tuner may pick among them freely by time; forward
chunking changes the image only by rounding, and a forward-chunk candidate is
accepted only within 1e-5 of the unchunked image.  Candidates are timed as
whole fwd+bwd steps of the workload (graph replays): first the tilings with
the default chunk lengths, then the backward chunk lengths for the fastest
tiling, then the forward chunk lengths.  The winner is stored per (device
arch, workload key) together with the hash of the kernel sources it was
timed on; an entry taken on other kernel sources is not used.
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import Dict, Iterable, List, Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "autotune_cache.json")

# (tile_w, tile_h, batch_depth, pixels_per_thread, subtile_cull).  The forward
# stages at most 64 records per wave and the backward at most 512 / waves per
# workgroup, so deeper batches than 128 change nothing.
CANDIDATES: List[Tuple[int, int, int, int, int]] = [
    (16, 16, 128, 1, 1), (16, 16, 128, 1, 0), (16, 16, 64, 1, 1), (16, 16, 32, 1, 1),
    (16, 16, 128, 2, 1), (16, 16, 64, 2, 1), (16, 16, 64, 4, 1),
    (8, 8, 64, 1, 1), (16, 8, 128, 1, 1), (16, 8, 64, 2, 1), (32, 8, 128, 1, 1), (32, 16, 128, 2, 1),
    (32, 16, 64, 2, 1), (32, 16, 128, 4, 1), (32, 32, 128, 4, 1), (64, 16, 128, 4, 1),
]
# list entries per backward work item (0: one item per tile)
CHUNKS: List[int] = [256, 512, 1024, 2048, 0]
# list entries per forward work item (0: one item per tile)
FWD_CHUNKS: List[int] = [0, 2048, 4096]
IMG_TOL = 1e-5  # a forward-chunk candidate's image against the unchunked one


def kernel_source_hash() -> str:
    """Hash of the HIP sources the timings depend on."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


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


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or CACHE
    if not os.path.exists(path):
        return {}
    try:
        return json.load(open(path))
    except ValueError:
        return {}


def best_opts(wl, arch: Optional[str] = None, cache_path: Optional[str] = None):
    """Cached winner for this workload on this device and these kernel sources, else the
    workload's default options."""
    arch = arch or _arch()
    e = load_cache(cache_path).get(f"{arch}|{workload_key(wl)}")
    if not e or e.get("source_hash") != kernel_source_hash():
        return wl.opts
    return dataclasses.replace(wl.opts, tile_w=e["tile_w"], tile_h=e["tile_h"], batch_depth=e["batch_depth"],
                               pixels_per_thread=e["pixels_per_thread"], subtile_cull=e.get("subtile_cull", 1),
                               bwd_chunk=e.get("bwd_chunk", wl.opts.bwd_chunk),
                               fwd_chunk=e.get("fwd_chunk", wl.opts.fwd_chunk))


def tune(wl, candidates: Iterable[Tuple[int, int, int, int, int]] = CANDIDATES, chunks: Iterable[int] = CHUNKS,
         fwd_chunks: Iterable[int] = FWD_CHUNKS, steps: int = 5, warmup: int = 2, write: bool = True,
         verbose: bool = True, cache_path: Optional[str] = None) -> dict:
    """Time each candidate's fwd+bwd step and store the fastest in the cache."""
    import numpy as np
    import torch

    from . import raster

    sc = wl.scene
    params = raster.to_device(sc)
    target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).cuda()
    results = []
    ref_img = None
    grid = [(tw, th, bd, ppt, cull, wl.opts.bwd_chunk, 0) for tw, th, bd, ppt, cull in candidates]
    tried = set()

    def run(cands):
        nonlocal ref_img
        for cand in cands:
            if cand in tried:
                continue
            tried.add(cand)
            results.append(_time_one(wl, params, target, cand, steps, warmup, verbose))
            img = results[-1].pop("_img")
            if ref_img is None:
                ref_img = img
            diff = float((img - ref_img).abs().max()) if img.numel() else 0.0
            results[-1]["image_max_abs_diff"] = diff
            # unchunked forwards must give the same bits; chunked ones the same up to rounding
            results[-1]["image_ok"] = bool(torch.equal(img, ref_img)) if cand[6] == 0 else diff <= IMG_TOL

    def fastest():
        return min((x for x in results if x["image_ok"]), key=lambda x: x["ms"])

    run(grid)
    b = fastest()
    shape = (b["tile_w"], b["tile_h"], b["batch_depth"], b["pixels_per_thread"], b["subtile_cull"])
    run([shape + (ch, 0) for ch in chunks])
    b = fastest()
    run([shape + (b["bwd_chunk"], fc) for fc in fwd_chunks])
    best = dict(fastest(), source_hash=kernel_source_hash(), workload=wl.name)
    if write:
        path = cache_path or CACHE
        cache = load_cache(path)
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
    tw, th, bd, ppt, cull, chunk, fchunk = cand
    o = dataclasses.replace(wl.opts, tile_w=tw, tile_h=th, batch_depth=bd, pixels_per_thread=ppt,
                            subtile_cull=cull, bwd_chunk=chunk, fwd_chunk=fchunk)
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
               fwd_chunk=fchunk, ms=ms, _img=r.image.clone())
    if verbose:
        print(f"  tile {tw}x{th} batch {bd} ppt {ppt} cull {cull} chunk {chunk} fwd chunk {fchunk}: {ms:.3f} ms/step",
              flush=True)
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
