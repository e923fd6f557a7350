"""gs_l2_grad: the mean-squared-error gradient of the benchmark step (GPU only)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2501_14534_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_14534_amd import gs
    gs.load()


@pytest.mark.parametrize("mean_views", [None, 8])
def test_l2_grad_matches_the_oracle_and_the_elementwise_formula(mean_views):
    from paper_2501_14534_amd import gs
    cams = [scenes.make_camera([0, -4, 0], [0, 0, 0], w, h, 0.9 * w) for w, h in ((40, 32), (33, 17), (64, 48))]
    V = len(cams)
    mv = V if mean_views is None else mean_views
    sizes = [3 * c.width * c.height for c in cams]
    rng = np.random.default_rng(4)
    img = rng.random(sum(sizes)).astype(np.float32)
    tgt = rng.random(sum(sizes)).astype(np.float32)
    print(f"[l2] views {V} mean over {mv}", flush=True)
    a, b = torch.from_numpy(img).cuda(), torch.from_numpy(tgt).cuda()
    out = torch.full_like(a, float("nan"))
    gs.check(gs.l2_grad(gs.ptr(a), gs.ptr(b), gs.cameras(cams), V, mv, gs.ptr(out),
                        torch.cuda.current_stream().cuda_stream), "gs_l2_grad")
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    # elementwise, the same float operations: (image - target) * float(2 / (3 H W mean_views))
    off = 0
    for k in sizes:
        scale = np.float32(2.0 / (k * mv))
        assert np.array_equal(got[off:off + k], (img[off:off + k] - tgt[off:off + k]) * scale)
        off += k
    # the oracle's mean over all V views (FP64), rescaled when averaging over mean_views
    ims, tgs, off = [], [], 0
    for c, k in zip(cams, sizes):
        ims.append(img[off:off + k].reshape(3, c.height, c.width).astype(np.float64))
        tgs.append(tgt[off:off + k].reshape(3, c.height, c.width).astype(np.float64))
        off += k
    ref = np.concatenate([g.ravel() for g in O.l2_grad(ims, tgs)]) * (V / mv)
    assert np.allclose(got, ref, rtol=1e-6, atol=0)
