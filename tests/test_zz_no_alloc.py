"""gs_mask_loss_noalloc (the entry point for callers that cannot allocate) against
gs_mask_loss through the C ABI: the same loss and gradients, bit for bit, on two calls in a
row, the second with fewer Gaussians, and the size limit (GPU only)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_14534_amd import gs
    gs.load()


def _inputs(n, deg, seed):
    rng = np.random.default_rng(seed)
    m = torch.from_numpy((rng.standard_normal(n) * 3).astype(np.float32)).cuda()
    msh = torch.from_numpy((rng.standard_normal((3, n)) * 3).astype(np.float32)).cuda()
    pre_m = torch.from_numpy((rng.uniform(-1, 1, n) * 1e-7).astype(np.float32)).cuda()
    pre_sh = torch.from_numpy((rng.uniform(-1, 1, (3, n)) * 1e-7).astype(np.float32)).cuda()
    return m, msh, pre_m, pre_sh


def _call(fn, n, deg, seed):
    from paper_2501_14534_amd import gs, raster
    m, msh, gm, gsh = _inputs(n, deg, seed)
    g = gs.gaussians({"mask_logits": m, "sh_mask_logits": msh}, n, deg, 0.5, 0.5)
    grads = gs.GsGrads(None, None, None, None, None, None, gs.ptr(gm), gs.ptr(gsh), None)
    loss = torch.full((1,), float("nan"), device="cuda")
    if fn == "ws":
        ws = torch.full((gs.mask_loss_workspace_size(n),), 255, dtype=torch.uint8, device="cuda")
        gs.check(gs.mask_loss(g, 0.05, 0.07, gs.ptr(loss), grads, gs.ptr(ws), ws.numel(), raster._stream()),
                 "gs_mask_loss")
    else:
        gs.check(gs.mask_loss_noalloc(g, 0.05, 0.07, gs.ptr(loss), grads, raster._stream()), "gs_mask_loss_noalloc")
    torch.cuda.synchronize()
    return loss.cpu(), gm.cpu(), gsh.cpu()


def test_noalloc_matches_workspace_call_twice_shrinking():
    """Two calls in a row, the second with a smaller input: each equals gs_mask_loss bit for bit
    (the second call's partial sums overwrite the first's in the shared scratch)."""
    for n, deg, seed in ((3_000_001, 3, 1), (70_001, 2, 2)):
        print(f"[no-alloc] n={n} deg={deg}", flush=True)
        ref = _call("ws", n, deg, seed)
        got = _call("noalloc", n, deg, seed)
        assert torch.isfinite(got[0]).all()
        for a, b in zip(got, ref):
            assert torch.equal(a, b)


def test_noalloc_rejects_too_many_gaussians():
    from paper_2501_14534_amd import gs, raster
    n = (1 << 24) + 1
    m = torch.zeros(1, device="cuda")  # never read: the size check comes first
    g = gs.gaussians({"mask_logits": m}, n, 0, 0.5, 0.5)
    rc = gs.mask_loss_noalloc(g, 0.05, 0.07, None, None, raster._stream())
    assert rc == gs.GS_E_TOO_LARGE
    assert "2^24" in gs.strerror(rc)
