"""The launch-shape autotuner on the GPU: tune() writes a winner, keyed by the kernel sources,
whose image equals the default options' image (GPU only)."""
import json

import numpy as np
import pytest
import torch

from paper_2501_14534_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_14534_amd import gs
    gs.load()


def test_tune_writes_a_winner_with_the_same_image(tmp_path):
    from paper_2501_14534_amd import autotune
    from tests import parity as P
    wl = scenes.scaled(2, n=20000, shrink=4)
    cache = str(tmp_path / "autotune.json")
    print("[autotune] scaled workload 2", flush=True)
    res = autotune.tune(wl, candidates=[(16, 16, 128, 1, 1), (8, 8, 64, 1, 1), (16, 16, 64, 2, 1)],
                        chunks=[512, 0], fwd_chunks=[0, 2048], steps=2, warmup=1, cache_path=cache)
    best = res["best"]
    assert best["source_hash"] == autotune.kernel_source_hash()
    assert len(res["results"]) >= 5
    # every unchunked forward gives the same bits (forward chunks may round further off and be rejected)
    assert all(x["image_ok"] for x in res["results"] if x["fwd_chunk"] == 0), \
        [(x["tile_w"], x["tile_h"], x["bwd_chunk"], x["image_max_abs_diff"]) for x in res["results"]]
    opts = autotune.best_opts(wl, cache_path=cache)
    for k in ("tile_w", "tile_h", "batch_depth", "pixels_per_thread", "subtile_cull", "bwd_chunk", "fwd_chunk"):
        assert getattr(opts, k) == best[k], k
    r0, _ = P.gpu_forward(wl)
    r1, _ = P.gpu_forward(wl, opts)
    if opts.fwd_chunk == 0:
        assert torch.equal(r0.image, r1.image)
    else:
        assert float((r0.image - r1.image).abs().max()) <= autotune.IMG_TOL
    # an entry timed on other kernel sources is not used
    d = json.load(open(cache))
    for e in d.values():
        e["source_hash"] = "0" * 16
    json.dump(d, open(cache, "w"))
    assert autotune.best_opts(wl, cache_path=cache) == wl.opts
