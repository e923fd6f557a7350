"""Edge cases, metamorphic properties and full-size sampled parity of the HIP path (GPU only)."""
import dataclasses

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


@pytest.fixture(scope="module")
def P():
    from tests import parity
    return parity


def _run(P, wl, opts=None, capacity=None, seed=5, schedule=True):
    r, params = P.gpu_forward(wl, opts, capacity, schedule=schedule)
    rng = np.random.default_rng(seed)
    dL = torch.from_numpy(rng.standard_normal(3 * r.total_pixels).astype(np.float32) * 1e-3).cuda()
    grads = r.zero_grads(params)
    r.backward(params, dL, grads)
    torch.cuda.synchronize()
    return r, params, grads


def _rel_close(a, b, tol):
    """Every element within tol * max(|b|, 1e-2 rms(b)), the rms over b's non-zero elements (R24)."""
    a = a.double().cpu()
    b = b.double().cpu()
    if a.numel() == 0:
        return True
    nz = b[b != 0]
    rms = float(nz.pow(2).mean().sqrt()) if nz.numel() else 0.0
    return bool(((a - b).abs() <= tol * torch.clamp(b.abs(), min=1e-2 * rms) + 1e-30).all())


def test_empty_scene_gives_background(P):
    wl = scenes.tiny(n=50, seed=1, deg=1)
    sc = wl.scene.subset(np.zeros(wl.scene.n, bool))
    wl0 = dataclasses.replace(wl, scene=sc, opts=dataclasses.replace(wl.opts, bg=(0.1, 0.2, 0.3)))
    print("[edge] empty scene", flush=True)
    r, params = P.gpu_forward(wl0)
    img = r.images()[0].cpu().numpy()
    for c, b in enumerate((0.1, 0.2, 0.3)):
        assert np.all(img[c] == np.float32(b))
    assert r.pairs() == 0
    assert torch.all(r.T_final == 1.0)


def test_all_culled_gives_background_and_zero_grads(P):
    wl = scenes.tiny(n=80, seed=2, deg=2, masks=True)
    sc = wl.scene.copy()
    sc.means[1] = -np.abs(sc.means[1]) - 1.0  # everything behind the camera
    wl1 = dataclasses.replace(wl, scene=sc)
    print("[edge] all culled", flush=True)
    r, params, grads = _run(P, wl1)
    assert r.pairs() == 0
    assert torch.all(r.image == 0.0)
    for k, g in grads.items():
        assert torch.all(g == 0.0), k


def test_tile_batch_and_ppt_do_not_change_the_image(P):
    """Image and T_final are bit-identical for every tiling; gradients are bitwise equal across batch
    depths (same per-pair sums) and within the gradient tolerance across tile shapes and
    pixels-per-thread (different summation partitions)."""
    wl = scenes.scaled(2, n=20000, shrink=4)
    print("[edge] tile/batch/ppt invariance", flush=True)
    ref, _, gref = _run(P, wl)
    img = ref.image.clone()
    T = ref.T_final.clone()
    for tw, th, bd, ppt, cull in [(8, 8, 64, 1, 1), (32, 8, 256, 1, 1), (16, 16, 17, 1, 1), (16, 16, 1, 1, 1),
                                  (16, 16, 256, 1, 0), (16, 16, 96, 1, 0), (16, 16, 256, 2, 1), (16, 16, 100, 4, 1),
                                  (16, 16, 64, 4, 0), (32, 16, 256, 2, 1), (16, 32, 128, 4, 1), (64, 4, 256, 1, 1),
                                  (16, 16, 1024, 1, 1), (16, 16, 600, 1, 0), (32, 16, 128, 4, 1), (32, 32, 128, 4, 1),
                                  (64, 16, 128, 4, 1)]:
        o = dataclasses.replace(wl.opts, tile_w=tw, tile_h=th, batch_depth=bd, pixels_per_thread=ppt,
                                subtile_cull=cull)
        r, _, g = _run(P, wl, o)
        assert torch.equal(r.image, img), (tw, th, bd, ppt, cull)
        assert torch.equal(r.T_final, T), (tw, th, bd, ppt, cull)
        same_partition = (tw, th, ppt) == (wl.opts.tile_w, wl.opts.tile_h, wl.opts.pixels_per_thread)
        for k in g:
            if same_partition:
                assert torch.equal(g[k], gref[k]), (k, tw, th, bd, ppt)
            else:
                assert _rel_close(g[k], gref[k], 1e-3), (k, tw, th, bd, ppt)


def test_tile_schedule_is_heaviest_first_and_changes_nothing(P):
    """The tile order is a permutation with list lengths grouped by bit length in non-increasing
    order; image, T_final, last_contrib and every gradient are bitwise the same without it."""
    wl = scenes.scaled(4, n=30000, shrink=4)
    print("[edge] heaviest-first tile schedule", flush=True)
    r, _, g = _run(P, wl)
    T = r.total_tiles
    order = r.order[:T].cpu().numpy().view(np.uint32).astype(np.int64)
    np.testing.assert_array_equal(np.sort(order), np.arange(T))
    rg = r.ranges[: 2 * T].cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    lens = rg[:, 1] - rg[:, 0]
    groups = np.where(lens > 0, np.floor(np.log2(np.maximum(lens, 1))).astype(np.int64) + 1, 0)[order]
    assert (np.diff(groups) <= 0).all()
    r0, _, g0 = _run(P, wl, schedule=False)
    assert r0.order is None
    assert torch.equal(r.image, r0.image) and torch.equal(r.T_final, r0.T_final) and torch.equal(r.last, r0.last)
    for k in g:
        assert torch.equal(g[k], g0[k]), k


def test_backward_chunking(P):
    """Chunked backward walks (chunks of 16..1024 list entries, each started from the state the
    forward recorded) give the image bit for bit and gradients within the gradient tolerance of
    the single walk per tile; chunked batched == chunked per-view, bit for bit."""
    wl = scenes.scaled(4, n=30000, shrink=4)
    print("[edge] backward chunking", flush=True)
    r0, _, g0 = _run(P, wl, dataclasses.replace(wl.opts, bwd_chunk=0))
    lens = np.diff(r0.ranges[: 2 * r0.total_tiles].cpu().numpy().view(np.uint32).reshape(-1, 2), axis=1)
    assert lens.max() > 1024  # the scene has lists that span several chunks
    for ch in (16, 64, 256, 1024):
        o = dataclasses.replace(wl.opts, bwd_chunk=ch)
        r, _, g = _run(P, wl, o)
        assert torch.equal(r.image, r0.image) and torch.equal(r.last, r0.last), ch
        for k in g:
            assert _rel_close(g[k], g0[k], 1e-3), (k, ch)
    wc = dataclasses.replace(wl, opts=dataclasses.replace(wl.opts, bwd_chunk=64))
    rb, params = P.gpu_forward(wc)
    dLb = np.random.default_rng(9).standard_normal(3 * rb.total_pixels).astype(np.float32) * 1e-3
    gb = rb.zero_grads(params)
    rb.backward(params, torch.from_numpy(dLb).cuda(), gb)
    gsum = rb.zero_grads(params)
    off = 0
    for c in wc.cams:
        rv, _ = P.gpu_forward(dataclasses.replace(wc, cams=[c], targets=[None]), params=params)
        rv.backward(params, torch.from_numpy(dLb[off:off + 3 * c.pixels]).cuda(), gsum)
        off += 3 * c.pixels
    torch.cuda.synchronize()
    for k in gb:
        assert torch.equal(gb[k], gsum[k]), k


def test_capacity_overflow_then_retry(P):
    wl = scenes.scaled(3, n=30000, shrink=8)
    print("[edge] capacity overflow", flush=True)
    big, params = P.gpu_forward(wl)
    K = big.pairs()
    small = P.make_rasterizer(wl, capacity=max(1, K // 3))
    small.project(params)
    small.bin_sort()
    small.render_fwd()
    torch.cuda.synchronize()
    assert small.overflowed() and small.pairs() == K
    assert torch.all(small.ranges == 0)
    assert torch.all(small.image == 0.0)  # bg = 0: every list empty
    small.forward(params, check=True)  # grows and re-bins
    torch.cuda.synchronize()
    assert not small.overflowed() and small.capacity >= K
    assert torch.equal(small.image, big.image)
    assert torch.equal(small.keys[:K], big.keys[:K]) and torch.equal(small.ids[:K], big.ids[:K])


def test_forward_and_backward_are_deterministic(P):
    wl = scenes.scaled(4, n=20000, shrink=4)
    print("[edge] determinism", flush=True)
    a, params, g1 = _run(P, wl)
    img, keys, ids, ranges = a.image.clone(), a.keys.clone(), a.ids.clone(), a.ranges.clone()
    g1 = {k: v.clone() for k, v in g1.items()}
    rng = np.random.default_rng(5)
    dL = torch.from_numpy(rng.standard_normal(3 * a.total_pixels).astype(np.float32) * 1e-3).cuda()
    a.forward(params)
    g2 = a.zero_grads(params)
    a.backward(params, dL, g2)
    torch.cuda.synchronize()
    assert torch.equal(a.image, img)
    assert torch.equal(a.keys, keys) and torch.equal(a.ids, ids) and torch.equal(a.ranges, ranges)
    for k in g1:
        assert torch.equal(g1[k], g2[k]), k


def test_batched_equals_per_view(P):
    wl = scenes.scaled(4, n=20000, shrink=2)
    print("[edge] batched == per-view", flush=True)
    rb, params = P.gpu_forward(wl)
    rng = np.random.default_rng(9)
    dLb = rng.standard_normal(3 * rb.total_pixels).astype(np.float32) * 1e-3
    gb = rb.zero_grads(params)
    rb.backward(params, torch.from_numpy(dLb).cuda(), gb)
    gsum = rb.zero_grads(params)
    off = 0
    imgs = []
    for c in wl.cams:
        wv = dataclasses.replace(wl, cams=[c], targets=[None])
        rv, _ = P.gpu_forward(wv, params=params)
        k = 3 * c.pixels
        rv.backward(params, torch.from_numpy(dLb[off:off + k]).cuda(), gsum)
        imgs.append(rv.image.clone())
        off += k
    torch.cuda.synchronize()
    assert torch.equal(torch.cat(imgs), rb.image)
    for k in gb:  # per-view calls in view order add in the same association as the batched call
        assert torch.equal(gb[k], gsum[k]), (k, float((gb[k] - gsum[k]).abs().max()))


def test_graph_replay_matches_eager(P):
    from paper_2501_14534_amd import raster
    wl = scenes.scaled(4, n=20000, shrink=4)
    print("[edge] graph replay == eager", flush=True)
    target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).cuda()
    params = raster.to_device(wl.scene)
    eager = raster.Step(P.make_rasterizer(wl), params, target, graph=False)
    eager.run()
    torch.cuda.synchronize()
    img0 = eager.rast.image.clone()
    g0 = {k: v.clone() for k, v in eager.grads.items()}
    st = raster.Step(P.make_rasterizer(wl), params, target, graph=True)
    st.run()
    for rep in range(3):
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work between replays
        st.launch()
        torch.cuda.synchronize()
        assert torch.equal(st.rast.image, img0), rep
        for k in g0:
            assert _rel_close(st.grads[k], g0[k], 1e-5), (rep, k)
        del junk


@pytest.mark.parametrize("case", ["tiny_masked", "cfg4_small"])
def test_autograd_function_matches_oracle(P, case):
    """rasterize() through torch.autograd: the leaves' gradients (the straight-through
    mask-logit gradients of Eq. 3 and Eq. 5 included) against the oracle's composite
    backward and FP64 projection backward on the same records and lists, every element
    within the gradient tolerance; near-threshold pixels get zero loss weight."""
    from oracle import oracle as O
    from paper_2501_14534_amd import raster
    if case == "tiny_masked":
        wl = scenes.tiny(n=150, seed=4, deg=3, masks=True, band_masks=True, width=48, height=40)
    else:
        wl = scenes.scaled(4, n=20000, shrink=4)
    print(f"[edge] autograd vs oracle: {case}", flush=True)
    r = P.make_rasterizer(wl)
    params = raster.to_device(wl.scene)
    leaves = {k: v.clone().requires_grad_(True) for k, v in params.items()}
    img = raster.rasterize(r, leaves)
    torch.cuda.synchronize()
    fwd = P.check_forward(wl, wl.opts, r)
    rng = np.random.default_rng(9)
    w = (rng.standard_normal(img.numel()) / np.sqrt(img.numel())).astype(np.float32)
    w[P._per_channel(fwd["flagged"], wl.cams)] = 0.0
    (img * torch.from_numpy(w).cuda()).sum().backward()
    torch.cuda.synchronize()
    sp = P.records(r)
    gl = P.gpu_lists(r)
    n = wl.scene.n
    grad_rec = O.composite_bwd(wl.cams, wl.opts, n, sp, gl["ids"], gl["ranges"], w.astype(np.float64))
    og, absparts = P.oracle_param_grads(wl, wl.opts, grad_rec)
    assert "mask_logits" in og and "sh_mask_logits" in og
    res = {k: P.r24_violations(leaves[k].grad.cpu().numpy(), ref, absparts=absparts[k]) for k, ref in og.items()}
    print(" ", res)
    for k, (nb, worst) in res.items():
        assert nb == 0, (k, nb, worst)
        assert np.any(og[k] != 0), k


def test_autograd_second_forward_before_backward_raises(P):
    """Two forwards through one Rasterizer, then the first image's backward: an error, not
    the second forward's gradients.  The second image's backward still works."""
    from paper_2501_14534_amd import raster
    wl = scenes.tiny(n=80, seed=5, deg=1, width=32, height=32)
    r = P.make_rasterizer(wl)
    params = raster.to_device(wl.scene)
    l1 = {k: v.clone().requires_grad_(True) for k, v in params.items()}
    l2 = {k: v.clone().requires_grad_(True) for k, v in params.items()}
    img1 = raster.rasterize(r, l1)
    img2 = raster.rasterize(r, l2)
    with pytest.raises(RuntimeError, match="another forward"):
        img1.sum().backward()
    img2.sum().backward()
    assert all(torch.isfinite(l2[k].grad).all() for k in l2)


def test_mask_metamorphic_identities(P):
    wl = scenes.tiny(n=200, seed=6, deg=3, masks=True, band_masks=True, width=64, height=48)
    print("[edge] mask identities", flush=True)
    sc = wl.scene.copy()
    sc.mask_logits[:] = 3.0
    sc.sh_mask_logits[:] = 3.0
    on, _ = P.gpu_forward(dataclasses.replace(wl, scene=sc))
    plain = sc.copy()
    plain.mask_logits, plain.sh_mask_logits = None, None
    pl, _ = P.gpu_forward(dataclasses.replace(wl, scene=plain))
    assert torch.equal(on.image, pl.image)  # all masks on == unmasked
    off = sc.copy()
    off.sh_mask_logits[:] = -3.0
    ro, _ = P.gpu_forward(dataclasses.replace(wl, scene=off))
    d0 = plain.copy()
    d0.sh_degree, d0.sh_rest = 0, None
    r0, _ = P.gpu_forward(dataclasses.replace(wl, scene=d0))
    assert torch.equal(ro.image, r0.image)  # all band masks off == degree 0
    dele = sc.copy()
    dele.mask_logits[::4] = -3.0
    rd, _ = P.gpu_forward(dataclasses.replace(wl, scene=dele))
    keep = np.ones(sc.n, bool)
    keep[::4] = False
    rk, _ = P.gpu_forward(dataclasses.replace(wl, scene=dele.subset(keep)))
    assert torch.equal(rd.image, rk.image)  # mask 0 == Gaussian deleted


def test_gaussian_order_does_not_matter(P):
    wl = scenes.tiny(n=300, seed=8, deg=2, width=64, height=48)
    print("[edge] permutation invariance", flush=True)
    a, _ = P.gpu_forward(wl)
    perm = np.random.default_rng(0).permutation(wl.scene.n)
    b, _ = P.gpu_forward(dataclasses.replace(wl, scene=wl.scene.subset(perm)))
    assert torch.equal(a.image, b.image)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("cfg", [2, 3, 4, 5])
def test_full_size_sampled_parity(P, cfg):
    """Full-size workload in the benchmark's launch configuration; binning bit-exact in full,
    compositing (with the excluded and flagged fractions of the sampled pixels bounded) and
    gradients on a sample of tiles: the 24 longest lists and 40 random tiles."""
    from oracle import oracle as O
    from paper_2501_14534_amd import autotune
    wl = scenes.config(cfg)
    opts = autotune.best_opts(wl)
    print(f"[full] config {cfg}: n={wl.scene.n} views={len(wl.cams)} tile {opts.tile_w}x{opts.tile_h} "
          f"batch {opts.batch_depth} ppt {opts.pixels_per_thread} bwd_chunk {opts.bwd_chunk}", flush=True)
    r, params = P.gpu_forward(wl, opts)
    gl = P.check_binning(wl, opts, r)
    print(f"  binning bit-exact: K={gl['K']}", flush=True)
    rng = np.random.default_rng(cfg)
    T = r.total_tiles
    lens = np.diff(gl["ranges"].astype(np.int64), axis=1).reshape(-1)
    deep = np.argsort(-lens, kind="stable")[:min(T, 24)]
    sample = np.union1d(deep, rng.choice(T, size=min(T, 40), replace=False))
    mask = np.zeros(T, np.uint8)
    mask[sample] = 1
    print(f"  sampled tiles {sample.size}, deepest list {int(lens.max())}", flush=True)
    # pixels of the sampled tiles
    pix_mask = np.zeros(r.total_pixels, bool)
    off = 0
    for v, c in enumerate(wl.cams):
        TX = -(-c.width // opts.tile_w)
        t0 = int(sum(-(-cc.width // opts.tile_w) * -(-cc.height // opts.tile_h) for cc in wl.cams[:v]))
        ys, xs = np.mgrid[0:c.height, 0:c.width]
        gt = t0 + (ys // opts.tile_h) * TX + xs // opts.tile_w
        pix_mask[off:off + c.pixels] = mask[gt.reshape(-1)] == 1
        off += c.pixels
    fwd = P.check_forward(wl, opts, r, tile_mask=mask, pix_mask=pix_mask)
    ok = pix_mask & ~fwd["flagged"]
    # gradients from the sampled, unflagged pixels only
    ok3 = P._per_channel(ok, wl.cams)
    w = np.zeros(3 * r.total_pixels, np.float32)
    w[ok3] = (rng.standard_normal(int(ok3.sum())) * 1e-3).astype(np.float32)
    grads = r.zero_grads(params)
    r.backward(params, torch.from_numpy(w).cuda(), grads)
    torch.cuda.synchronize()
    sp = P.records(r)
    grad_rec = O.composite_bwd(wl.cams, opts, wl.scene.n, sp, gl["ids"], gl["ranges"], w.astype(np.float64),
                               tile_mask=mask)
    og, absparts = P.oracle_param_grads(wl, opts, grad_rec)
    # most Gaussians lie outside the sampled tiles: the floor's rms is over the gradient's support
    bad = {k: P.r24_violations(grads[k].cpu().numpy(), ref, support_rms=True, absparts=absparts[k])
           for k, ref in og.items()}
    print(" ", bad)
    for k, (nb, worst) in bad.items():
        assert nb == 0, (k, nb, worst)


@pytest.mark.parametrize("deg,masks", [(3, True), (1, False)])
def test_assign_mode_writes_what_accumulate_adds(P, deg, masks):
    """Gradients written (assign) over arrays of garbage equal zeroed-then-accumulated ones, bit for
    bit, with culled and off-screen Gaussians among them; accumulate mode adds onto what is there."""
    wl = scenes.tiny(n=300, seed=7, deg=deg, masks=masks, band_masks=masks)
    print(f"[edge] assign mode deg={deg} masks={masks}", flush=True)
    r, params = P.gpu_forward(wl)
    rng = np.random.default_rng(11)
    dL = torch.from_numpy(rng.standard_normal(3 * r.total_pixels).astype(np.float32) * 1e-3).cuda()
    ref = r.zero_grads(params)
    r.backward(params, dL, ref)
    got = r.zero_grads(params)
    for g in got.values():
        g.copy_(torch.from_numpy(rng.standard_normal(g.numel()).astype(np.float32)).cuda().view(g.shape))
    base = {k: v.clone() for k, v in got.items()}
    r.render_bwd(params, dL, got, assign=True)
    torch.cuda.synchronize()
    for k in ref:
        if deg == 0 and k in ("sh_rest", "sh_mask_logits"):
            continue
        assert torch.equal(got[k], ref[k]), k
    acc = {k: v.clone() for k, v in base.items()}
    r.render_bwd(params, dL, acc)
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(acc[k], base[k] + ref[k]), k


def test_unreached_pair_rows_are_never_read(P):
    """The backward walk writes the rows of the pairs it reaches and marks them; rows of the
    others keep whatever they held (here NaN) and must not reach the parameter gradients."""
    wl = scenes.config(1, n=4000, seed=3)
    print("[edge] unreached rows (NaN-filled pair buffer)", flush=True)
    r, params = P.gpu_forward(wl)
    rng = np.random.default_rng(2)
    dL = torch.from_numpy(rng.standard_normal(3 * r.total_pixels).astype(np.float32) * 1e-3).cuda()
    out = []
    for fill in (0.0, float("nan")):
        gp = torch.full((max(r.capacity, 1) * 9,), fill, dtype=torch.float32, device="cuda")
        g = r.zero_grads(params)
        r.blend_bwd(dL, gp)
        r.project_bwd(params, gp, g, assign=True)
        torch.cuda.synchronize()
        out.append(g)
    for k in out[0]:
        assert torch.isfinite(out[1][k]).all(), k
        assert torch.equal(out[0][k], out[1][k]), k
    ref = r.zero_grads(params)
    r.backward(params, dL, ref)
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(out[0][k], ref[k]), k
