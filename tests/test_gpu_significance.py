"""Ray hits (gs_count_hits) and the significance score (gs_significance) of Eq. 4 vs the
FP64 oracle, through the C ABI (GPU only).

Hits are integers decided by float comparisons: the oracle walks the GPU's own
records over the GPU's lists, and the two must agree exactly for every
Gaussian, except by at most the number of near-threshold pixels (flagged by
the oracle) whose tiles list it.  The score is compared with the oracle's
FP64 formula applied to the GPU's hits (relative 1e-5: float log-volumes)."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2501_14534_amd import scenes

pytestmark = pytest.mark.gpu

Q90 = float(np.float32(0.9))
SCORE_RTOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cases():
    return {
        "tiny_masked": lambda: scenes.tiny(n=300, seed=1, width=70, height=45, deg=3, masks=True, band_masks=True),
        "cfg1": lambda: scenes.config(1),
        "cfg4_small": lambda: scenes.scaled(4, n=20000, shrink=4),
        "cfg5_small": lambda: scenes.scaled(5, n=60000, views=[0, 4], shrink=8),
    }


CASES = _cases()


def _gpu_hits(r, n, bins=None):
    hits = torch.zeros(n, dtype=torch.int32, device="cuda")
    r.count_hits(hits, bins)
    torch.cuda.synchronize()
    return hits.cpu().numpy().view(np.uint32).astype(np.int64)


def _compare_hits(wl, opts, r, got, ranges=None):
    from oracle import oracle as O
    from tests import parity as P
    sp = P.records(r)
    gl = P.gpu_lists(r)
    rg = gl["ranges"] if ranges is None else ranges
    ref = O.hits(wl.cams, opts, wl.scene.n, sp, gl["ids"], rg, eps=P.FLAG_EPS)
    V, n = len(wl.cams), wl.scene.n
    want = O.hits_per_gaussian(ref["hits"], V, n)
    slack = O.hits_per_gaussian(ref["uncertain"], V, n)
    diff = np.abs(got - want)
    bad = diff > slack
    assert not bad.any(), (int(bad.sum()), np.flatnonzero(bad)[:10])
    exact = slack == 0
    assert np.array_equal(got[exact], want[exact])
    return dict(total=int(want.sum()), exact=int(exact.sum()), differ=int((diff > 0).sum()))


@pytest.mark.parametrize("case", list(CASES))
def test_hits_parity(case):
    from tests import parity as P
    wl = CASES[case]()
    print(f"[hits] {case}: n={wl.scene.n} views={len(wl.cams)}", flush=True)
    r, _ = P.gpu_forward(wl)
    got = _gpu_hits(r, wl.scene.n)
    res = _compare_hits(wl, wl.opts, r, got)
    print(res)
    assert res["total"] > 0


def test_hits_are_identical_across_launch_configurations():
    """Integers from the same per-pixel decisions: every launch shape counts the same hits."""
    from tests import parity as P
    wl = scenes.scaled(4, n=20000, shrink=4)
    base = None
    for tile, batch, ppt, cull, sched in [((16, 16), 256, 1, 1, True), ((16, 16), 1024, 1, 1, False),
                                          ((16, 16), 64, 4, 0, True), ((32, 8), 128, 2, 1, True),
                                          ((8, 8), 7, 1, 1, True)]:
        opts = dataclasses.replace(wl.opts, tile_w=tile[0], tile_h=tile[1], batch_depth=batch,
                                   pixels_per_thread=ppt, subtile_cull=cull)
        print(f"[hits config] tile {tile} batch {batch} ppt {ppt} cull {cull} schedule {sched}", flush=True)
        r, _ = P.gpu_forward(wl, opts, schedule=sched)
        got = _gpu_hits(r, wl.scene.n)
        if base is None:
            base = got
            _compare_hits(wl, opts, r, got)
        else:
            np.testing.assert_array_equal(got, base)


def test_hits_accumulate_over_view_batches():
    """Counting view by view into one array equals counting all views in one call."""
    from paper_2501_14534_amd import raster
    from tests import parity as P
    wl = scenes.scaled(5, n=60000, views=[0, 2, 4], shrink=8)
    print("[hits] batches of views", flush=True)
    r, params = P.gpu_forward(wl)
    together = _gpu_hits(r, wl.scene.n)
    hits = torch.zeros(wl.scene.n, dtype=torch.int32, device="cuda")
    for c in wl.cams:
        rv = raster.Rasterizer(wl.scene.n, wl.scene.sh_degree, [c], wl.opts, mask_eps=wl.scene.mask_eps,
                               sh_mask_eps=wl.scene.sh_mask_eps)
        rv.accumulate_hits(params, hits)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(hits.cpu().numpy().astype(np.int64), together)
    out = raster.significance_scores(params, wl.scene.sh_degree, wl.cams, wl.opts, views_per_call=2,
                                     mask_eps=wl.scene.mask_eps, sh_mask_eps=wl.scene.sh_mask_eps)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out["hits"].cpu().numpy().astype(np.int64), together)


def test_hits_full_size_sampled_tiles():
    """The 8-view 1M-Gaussian workload in the benchmark's launch configuration: both sides walk
    the same sample of tiles (the 24 longest lists and 40 random ones; the other ranges emptied)."""
    from paper_2501_14534_amd import autotune, gs
    from tests import parity as P
    wl = scenes.config(4)
    opts = autotune.best_opts(wl)
    print(f"[hits full] n={wl.scene.n} views={len(wl.cams)}", flush=True)
    r, _ = P.gpu_forward(wl, opts)
    gl = P.gpu_lists(r)
    T = r.total_tiles
    lens = np.diff(gl["ranges"].astype(np.int64), axis=1).reshape(-1)
    deep = np.argsort(-lens, kind="stable")[:24]
    sample = np.union1d(deep, np.random.default_rng(4).choice(T, size=40, replace=False))
    rg = gl["ranges"].copy()
    keep = np.zeros(T, bool)
    keep[sample] = True
    rg[~keep] = 0
    ranges = torch.from_numpy(rg.reshape(-1).view(np.int32).copy()).cuda()
    b = r.bins
    bins = gs.GsBinning(b.keys, b.ids, b.pair_index, b.offsets, gs.ptr(ranges), b.order, b.capacity, b.count,
                        b.status)
    got = _gpu_hits(r, wl.scene.n, bins)
    res = _compare_hits(wl, opts, r, got, ranges=rg)
    print(res)
    assert res["total"] > 0


def _score_check(sc, hits, q, params=None):
    from oracle import oracle as O
    from paper_2501_14534_amd import raster
    params = params if params is not None else raster.to_device(sc)
    th = torch.from_numpy(np.asarray(hits, np.int64).astype(np.uint32).view(np.int32)).cuda()
    got = raster.significance(params, th, q, sc.mask_eps).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    ref = O.significance(sc, np.asarray(hits, np.int64), q)
    np.testing.assert_allclose(got, ref, rtol=SCORE_RTOL, atol=0)
    return got


@pytest.mark.parametrize("n,q,masks", [(1, Q90, False), (2, Q90, True), (257, Q90, True), (70001, Q90, False),
                                       (70001, 1.0, True), (4099, float(np.float32(0.05)), False)])
def test_significance_parity(n, q, masks):
    sc = scenes.random_scene(np.random.default_rng(n), n, means=np.zeros((3, n)), log_scale=(-3.0, 1.2),
                             opacity=(0.0, 2.0), deg=0, masks=masks, band_masks=False, mask_eps=0.3,
                             sh_mask_eps=0.5, unit_quats=True)
    hits = np.random.default_rng(n + 1).integers(0, 5000, n)
    hits[::7] = 0
    print(f"[significance] n={n} q={q} masks={masks}", flush=True)
    _score_check(sc, hits, q)


def test_significance_with_tied_volumes():
    """Many equal log-scales: the quantile falls inside a run of equal keys."""
    n = 5000
    sc = scenes.random_scene(np.random.default_rng(5), n, means=np.zeros((3, n)), log_scale=(-2.0, 0.5),
                             opacity=(0.0, 1.0), deg=0, masks=False, band_masks=False, mask_eps=0.5,
                             sh_mask_eps=0.5, unit_quats=True)
    sc.log_scales[:, ::2] = np.float32(-1.5)
    sc.log_scales[:, 1::4] = np.float32(-3.0)
    hits = np.random.default_rng(6).integers(1, 100, n)
    print("[significance] tied volumes", flush=True)
    _score_check(sc, hits, Q90)


def test_significance_end_to_end_vs_oracle_chain():
    """Hits and scores of the GPU's whole chain (its own float projection) against the oracle's
    whole chain (FP64 projection): equal hits for all but a few Gaussians (those with a pixel near
    a threshold, or a footprint radius at an integer boundary), equal scores where hits agree."""
    from oracle import oracle as O
    from paper_2501_14534_amd import raster
    wl = scenes.tiny(n=300, seed=3, width=70, height=45, deg=1, masks=True)
    params = raster.to_device(wl.scene)
    print("[significance] end to end", flush=True)
    out = raster.significance_scores(params, wl.scene.sh_degree, wl.cams, wl.opts, mask_eps=wl.scene.mask_eps)
    torch.cuda.synchronize()
    hits = out["hits"].cpu().numpy().astype(np.int64)
    ref = O.count_hits(wl.scene, wl.cams, wl.opts)
    same = hits == ref["per_gaussian"]
    assert (~same).sum() <= 0.01 * wl.scene.n, int((~same).sum())
    assert hits.sum() > 0
    sref = O.significance(wl.scene, ref["per_gaussian"], Q90)
    got = out["score"].cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got[same], sref[same], rtol=SCORE_RTOL, atol=0)
