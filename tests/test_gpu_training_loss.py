"""Mask terms of the loss (gs_mask_loss) and the training step with the paper's loss and sparse
SH-rest updates (GPU only)."""
import numpy as np
import pytest
import torch

from paper_2501_14534_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("deg", [3, 1, 0])
def test_mask_loss_parity_and_accumulation(deg):
    from oracle import mask_loss as OM
    from paper_2501_14534_amd import gs, raster
    from tests.parity import r24_violations
    n = 70001  # several workgroups and a ragged tail
    rng = np.random.default_rng(deg)
    m = (rng.standard_normal(n) * 3).astype(np.float32)
    msh = (rng.standard_normal((3, n)) * 3).astype(np.float32)
    print(f"[mask loss] n={n} deg={deg}", flush=True)
    params = {"mask_logits": torch.from_numpy(m).cuda(), "sh_mask_logits": torch.from_numpy(msh).cuda()}
    g = gs.gaussians(params, n, deg, 0.5, 0.5)
    # accumulation targets pre-filled at the increments' own magnitude (~1e-7), so that
    # subtracting them afterwards keeps the increments' precision
    p_m = (rng.uniform(-1, 1, n) * 1e-7).astype(np.float32)
    p_sh = (rng.uniform(-1, 1, (3, n)) * 1e-7).astype(np.float32)
    pre_m = torch.from_numpy(p_m).cuda()
    pre_sh = torch.from_numpy(p_sh).cuda()
    grads = gs.GsGrads(None, None, None, None, None, None, gs.ptr(pre_m), gs.ptr(pre_sh), None)
    loss = torch.zeros(1, device="cuda")
    ws = torch.zeros(gs.mask_loss_workspace_size(n), dtype=torch.uint8, device="cuda")
    gs.check(gs.mask_loss(g, 0.05, 0.07, gs.ptr(loss), grads, gs.ptr(ws), ws.numel(), raster._stream()), "mask")
    torch.cuda.synchronize()
    ref = OM.mask_loss(m, msh, deg, 0.05, 0.07)
    assert abs(float(loss) - ref["loss"]) <= 1e-6 * max(1.0, abs(ref["loss"]))
    gm, gsh = OM.mask_loss_grad(m, msh, deg, 0.05, 0.07)
    assert r24_violations(pre_m.cpu().numpy().astype(np.float64) - p_m, gm)[0] == 0
    assert r24_violations(pre_sh.cpu().numpy().astype(np.float64) - p_sh, gsh)[0] == 0
    if deg < 3:
        assert np.array_equal(pre_sh[deg:].cpu().numpy(), p_sh[deg:])  # bands above the degree untouched


def test_step_with_the_paper_loss_and_sparse_sh_updates():
    from tests import parity as P
    from paper_2501_14534_amd import raster
    wl = scenes.scaled(4, n=20000, shrink=4)
    print("[step] L1 + D-SSIM + mask terms, SH bands every 4th step", flush=True)
    r = P.make_rasterizer(wl)
    params = raster.to_device(wl.scene)
    target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).cuda()
    results = {}
    for graph in (False, True):
        st = raster.Step(r, params, target, graph=graph, loss="l1_dssim", mask_loss=(0.05, 0.05), sh_rest_every=4)
        seq = []
        for k in range(5):
            st.launch()
            torch.cuda.synchronize()
            seq.append({n: v.clone() for n, v in st.grads.items()})
        results[graph] = seq
        # every step sees the same parameters: equal gradients, sh_rest only on steps 0 and 4
        for k in range(5):
            assert bool(torch.any(seq[k]["sh_rest"] != 0)) == (k % 4 == 0), k
            for name in seq[0]:
                if name != "sh_rest":
                    assert torch.equal(seq[k][name], seq[0][name]), (k, name)
        assert torch.equal(seq[4]["sh_rest"], seq[0]["sh_rest"])
    for k in range(5):
        for name in results[False][k]:
            assert torch.equal(results[False][k][name], results[True][k][name]), (k, name)
