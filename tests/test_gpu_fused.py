"""The fused compositing launch (gs_render_fwd_bwd_l2) against the three calls it stands for
(gs_render_fwd, gs_l2_grad, gs_render_bwd), through the C ABI: the same bits for the image,
T_final, last_contrib, dL/dimage and every gradient (GPU only)."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2501_14534_amd import gs, raster, scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gs.load()


CASES = {
    "tiny_masked": lambda: scenes.tiny(n=300, seed=1, width=70, height=45, deg=3, masks=True, band_masks=True),
    "cfg1": lambda: scenes.config(1),
    "cfg2_small": lambda: scenes.scaled(2, n=20000, shrink=4),
    "cfg4_small": lambda: scenes.scaled(4, n=20000, shrink=4),
    "cfg5_small": lambda: scenes.scaled(5, n=60000, views=[0, 4], shrink=8),
}
# (tile_w, tile_h, batch_depth, pixels_per_thread, subtile_cull, bwd_chunk)
SHAPES = [(16, 16, 128, 1, 1, 512), (16, 16, 128, 1, 1, 16), (32, 16, 128, 2, 1, 256), (32, 32, 128, 4, 1, 0),
          (16, 16, 64, 1, 0, 64), (8, 8, 64, 1, 1, 32)]


def _rast(wl, opts, schedule):
    sc = wl.scene
    return raster.Rasterizer(sc.n, sc.sh_degree, wl.cams, opts, mask_eps=sc.mask_eps, sh_mask_eps=sc.sh_mask_eps,
                             schedule=schedule)


def _target(r, seed):
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.random(r.image.numel(), dtype=np.float32)).cuda()


def _outputs(r, dL, grads):
    out = {"image": r.image.clone(), "T_final": r.T_final.clone(), "last": r.last.clone(), "dL": dL.clone()}
    out.update({"g_" + k: v.clone() for k, v in grads.items()})
    return out


def _separate(wl, opts, params, target, views, schedule):
    r = _rast(wl, opts, schedule)
    r.forward(params)
    dL = torch.empty_like(r.image)
    raster.l2_loss_grad(r, r.image, target, views, dL)
    grads = r.zero_grads(params)
    r.render_bwd(params, dL, grads, assign=True)
    torch.cuda.synchronize()
    return _outputs(r, dL, grads)


def _fused(wl, opts, params, target, views, schedule):
    r = _rast(wl, opts, schedule)
    r.forward(params)  # sizes the lists
    r.image.fill_(float("nan"))
    r.T_final.fill_(float("nan"))
    r.last.fill_(-7)
    dL = torch.full_like(r.image, float("nan"))
    grads = r.zero_grads(params)
    r.project(params)
    r.bin_sort()
    r.render_fwd_bwd_l2(params, target, views, grads, dL_out=dL, assign=True)
    torch.cuda.synchronize()
    assert not r.overflowed()
    return _outputs(r, dL, grads)


def _check_equal(a, b, label):
    for k in a:
        assert torch.equal(a[k], b[k]), (label, k, float((a[k].double() - b[k].double()).abs().max()))


@pytest.mark.parametrize("case", list(CASES))
def test_fused_equals_separate_calls(case):
    wl = CASES[case]()
    params = raster.to_device(wl.scene)
    V = len(wl.cams)
    for i, (tw, th, bd, ppt, cull, ch) in enumerate(SHAPES):
        opts = dataclasses.replace(wl.opts, tile_w=tw, tile_h=th, batch_depth=bd, pixels_per_thread=ppt,
                                   subtile_cull=cull, bwd_chunk=ch)
        target = None
        for schedule in (True, False) if i == 0 else (True,):
            print(f"[fused] {case} tile {tw}x{th} batch {bd} ppt {ppt} cull {cull} chunk {ch} schedule {schedule}",
                  flush=True)
            r0 = _rast(wl, opts, schedule)
            target = _target(r0, seed=i) if target is None else target
            del r0
            views = V + 2 if i == 1 else V  # a per-view call of a larger batch averages over its views
            a = _separate(wl, opts, params, target, views, schedule)
            b = _fused(wl, opts, params, target, views, schedule)
            _check_equal(a, b, (case, tw, th, bd, ppt, cull, ch, schedule))


def test_fused_step_equals_unfused_step():
    """raster.Step with the fused walks (the benchmark's step) against the unfused step: same
    image and gradients, bit for bit, eager and replayed from a graph."""
    wl = CASES["cfg4_small"]()
    params = raster.to_device(wl.scene)
    sc = wl.scene
    outs = []
    for fused in (False, True):
        r = raster.Rasterizer(sc.n, sc.sh_degree, wl.cams, wl.opts, mask_eps=sc.mask_eps, sh_mask_eps=sc.sh_mask_eps)
        target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).cuda()
        st = raster.Step(r, params, target, graph=True, fused=fused)
        print(f"[fused] step fused={fused}", flush=True)
        st.run()
        for _ in range(3):
            st.launch()
        torch.cuda.synchronize()
        outs.append(_outputs(r, st.dL, st.grads))
    _check_equal(outs[0], outs[1], "step")


def test_fused_with_forward_chunks_runs_the_three_calls():
    wl = CASES["cfg2_small"]()
    params = raster.to_device(wl.scene)
    opts = dataclasses.replace(wl.opts, fwd_chunk=64)
    V = len(wl.cams)
    print("[fused] forward chunks", flush=True)
    r0 = _rast(wl, opts, True)
    target = _target(r0, seed=3)
    del r0
    _check_equal(_separate(wl, opts, params, target, V, True), _fused(wl, opts, params, target, V, True), "fchunk")
    # without a dL/dimage buffer the three calls cannot run: refused before anything is launched
    r = _rast(wl, opts, True)
    r.forward(params)
    grads = r.zero_grads(params)
    with pytest.raises(gs.GsError):
        r.render_fwd_bwd_l2(params, target, V, grads, dL_out=None, assign=True)
