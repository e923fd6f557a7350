"""Progressive training on the GPU (Sec. 3.2.4): the per-view low-pass through the whole
path, and the target blur and resize kernels, vs the FP64 oracle (GPU only)."""
import dataclasses
import math

import numpy as np
import pytest
import torch

from paper_2501_14534_amd import scenes

pytestmark = pytest.mark.gpu

# blur: at most 2 r + 1 <= 31 products per pass of values in [0, 1] with weights summing to
# one, twice: |error| <= 2 * 31 * 2^-24 ~ 4e-6
BLUR_TOL = 1e-5
# resize: a float sum of <= ceil(W/W'+1) ceil(H/H'+1) products, relative 2^-24 each
RESIZE_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cams(sizes):
    return [scenes.make_camera((0.0, -4.0, 0.0), (0, 0, 0), w, h, float(w)) for w, h in sizes]


def _split(flat, cams):
    out, o = [], 0
    for c in cams:
        k = 3 * c.width * c.height
        out.append(flat[o:o + k].reshape(3, c.height, c.width))
        o += k
    return out


@pytest.mark.parametrize("case", ["cfg4_small", "tiny_masked"])
def test_progressive_lowpass_whole_path_parity(case):
    """Per-view s = max(0.3, HW / (9 pi N)) on mixed resolutions: projection, binning,
    compositing and gradients against the oracle under the same rule."""
    from tests import parity as P
    wl = {"cfg4_small": lambda: scenes.scaled(4, n=200, shrink=4),
          "tiny_masked": lambda: scenes.tiny(n=120, seed=2, width=70, height=45, masks=True, band_masks=True)}[case]()
    opts = dataclasses.replace(wl.opts, lowpass_progressive=1)
    s = [c.width * c.height / (9 * math.pi * wl.scene.n) for c in wl.cams]
    assert min(s) > 0.3  # the progressive value is in force in every view
    print(f"[progressive lowpass] {case}: s per view {[round(x, 3) for x in s]}", flush=True)
    r, params = P.gpu_forward(wl, opts)
    P.check_projection(wl, opts, r)
    P.check_binning(wl, opts, r)
    fw = P.check_forward(wl, opts, r)
    res = P.check_backward(wl, opts, r, params, fw["flagged"])
    for k, (bad, worst) in res.items():
        assert bad == 0, (k, bad, worst)
    # and it differs from the fixed s
    r0, _ = P.gpu_forward(wl, wl.opts)
    assert not torch.equal(r0.image, r.image)


@pytest.mark.parametrize("k,sigma", [(9, 2.4), (3, 0.7), (1, 1.0), (31, 6.0), (7, 40.0)])
def test_blur_parity(k, sigma):
    from oracle import targets as TG
    from paper_2501_14534_amd import progressive as PG
    cams = _cams([(40, 32), (7, 5), (37, 23), (1, 9), (2, 3), (64, 16), (316, 208)])
    rng = np.random.default_rng(k)
    n = sum(3 * c.width * c.height for c in cams)
    img = rng.random(n).astype(np.float32)
    print(f"[blur] k={k} sigma={sigma}", flush=True)
    got = PG.blur(torch.from_numpy(img).cuda(), cams, k, sigma).cpu().numpy()
    ref = TG.blur_views(_split(img.astype(np.float64), cams), k, sigma)
    err = np.abs(got - np.concatenate([r.reshape(-1) for r in ref])).max()
    assert err <= BLUR_TOL, err


@pytest.mark.parametrize("ratio", [8.0, 2.0, 3.3, 1.0, 0.5])
def test_resize_parity(ratio):
    from oracle import targets as TG
    from paper_2501_14534_amd import progressive as PG
    src = _cams([(1264 // 4, 832 // 4), (37, 23), (5, 3), (64, 16)])
    dst = PG.scaled_cameras(src, ratio)
    rng = np.random.default_rng(int(ratio * 10))
    n = sum(3 * c.width * c.height for c in src)
    img = rng.random(n).astype(np.float32)
    print(f"[resize] ratio {ratio}: {[(c.width, c.height) for c in dst]}", flush=True)
    got = PG.resize(torch.from_numpy(img).cuda(), src, dst).cpu().numpy()
    ref = TG.resize_views(_split(img.astype(np.float64), src), [(c.width, c.height) for c in dst])
    err = np.abs(got - np.concatenate([r.reshape(-1) for r in ref])).max()
    assert err <= RESIZE_TOL, err


@pytest.mark.parametrize("start,iters", [(8.0, (0, 5000, 20000)), (1.0, (0, 5000, 19000))])
def test_progressive_targets_follow_the_schedules(start, iters):
    """Targets of iteration i: resized by the downsampling factor, then blurred by the kernel
    of that iteration scaled by the factor (with 8x downsampling the kernel stays under 3 taps,
    so only the resize acts; without it, the blur shrinks from 9 x 9)."""
    from oracle import targets as TG
    from paper_2501_14534_amd import progressive as PG
    wl = scenes.config(4, n=16)
    tgt = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).cuda()
    pt = PG.ProgressiveTargets(tgt, wl.cams, start=start)
    print(f"[progressive targets] start {start}", flush=True)
    for i in iters:
        cams, img = pt.at(i)
        f = PG.downsample_factor(i, start)
        kb = PG.blur_kernel(i, downsample=f)
        ref = [t.astype(np.float64) for t in wl.targets]
        if f > 1.0:
            ref = TG.resize_views(ref, [(c.width, c.height) for c in cams])
        if kb is not None:
            ref = TG.blur_views(ref, kb[0], kb[1])
        ref = np.concatenate([r.reshape(-1) for r in ref])
        assert img.numel() == ref.size
        assert np.abs(img.cpu().numpy() - ref).max() <= BLUR_TOL + RESIZE_TOL, i
        if start == 1.0 and i < 19000:
            assert kb is not None and kb[0] >= 5
