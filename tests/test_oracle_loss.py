"""Pins of the FP64 loss oracle (oracle/loss.py) against definitions it does not share code
with: closed forms, scipy's correlation, a torch float64 implementation with autograd, and
central finite differences."""
import numpy as np
import pytest
import scipy.signal
import torch

from oracle import loss as L

# SSIM stabilisers of the standard definition, (0.01 * 1)^2 and (0.03 * 1)^2 for a dynamic range of 1,
# written here independently of the oracle's constants
C1, C2 = 1e-4, 9e-4


def test_constants():
    assert (L.C1, L.C2, L.WINDOW, L.SIGMA, L.LAMBDA) == pytest.approx((C1, C2, 11, 1.5, 0.2), rel=1e-15)


def test_window_is_a_normalised_separable_gaussian():
    g = L.gaussian_1d()
    assert g.shape == (11,) and abs(g.sum() - 1.0) < 1e-15
    assert np.allclose(g, g[::-1]) and g.argmax() == 5
    k = np.arange(11) - 5.0
    direct = np.exp(-(k[:, None] ** 2 + k[None, :] ** 2) / (2 * 1.5 ** 2))
    assert np.allclose(L.window_2d(), direct / direct.sum(), rtol=0, atol=1e-16)


def test_filter_is_zero_padded_same_correlation():
    rng = np.random.default_rng(0)
    img = rng.random((13, 17))
    w = rng.random((11, 11))  # not symmetric: fixes the orientation
    ref = scipy.signal.correlate2d(img, w, mode="same", boundary="fill", fillvalue=0.0)
    assert np.allclose(L.filter2d(img, w), ref, rtol=0, atol=1e-12)
    delta = np.zeros((21, 21))
    delta[10, 10] = 1.0
    assert np.allclose(L.filter2d(delta, w)[5:16, 5:16], w[::-1, ::-1])


def test_ssim_of_an_image_with_itself_is_one():
    x = np.random.default_rng(1).random((19, 23))
    assert np.allclose(L.ssim_map(x, x), 1.0, rtol=0, atol=1e-12)


def test_ssim_is_symmetric():
    rng = np.random.default_rng(2)
    x, y = rng.random((15, 12)), rng.random((15, 12))
    assert np.allclose(L.ssim_map(x, y), L.ssim_map(y, x), rtol=0, atol=1e-14)


def test_constant_images_closed_form_away_from_the_border():
    a, b = 0.3, 0.7
    s = L.ssim_map(np.full((24, 24), a), np.full((24, 24), b))
    inner = s[5:-5, 5:-5]  # the window lies inside the image: no variance, sigma terms C2/C2
    assert np.allclose(inner, (2 * a * b + C1) / (a * a + b * b + C1), rtol=1e-12, atol=0)
    assert not np.allclose(s[0, 0], inner[0, 0])  # zero padding lowers the corner means


def _torch_loss(img, tgt, lam):
    """Independent float64 implementation: direct 2-D convolution with the window."""
    w = torch.from_numpy(L.window_2d())[None, None].expand(3, 1, 11, 11).contiguous()
    x = img[None]
    y = tgt[None]
    conv = lambda t: torch.nn.functional.conv2d(t, w, padding=5, groups=3)  # noqa: E731
    mx, my = conv(x), conv(y)
    sxx, syy, sxy = conv(x * x) - mx * mx, conv(y * y) - my * my, conv(x * y) - mx * my
    s = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
    return (1 - lam) * (x - y).abs().mean() + lam * (1 - s.mean())


@pytest.mark.parametrize("shape", [(3, 9, 8), (3, 20, 31), (3, 4, 6)])
def test_loss_and_gradient_match_torch_autograd(shape):
    rng = np.random.default_rng(sum(shape))
    img, tgt = rng.random(shape), rng.random(shape)
    t_img = torch.from_numpy(img).requires_grad_(True)
    ref = _torch_loss(t_img, torch.from_numpy(tgt), 0.2)
    ref.backward()
    assert abs(L.view_loss(img, tgt)["loss"] - ref.item()) < 1e-13
    assert np.allclose(L.view_loss_grad(img, tgt), t_img.grad.numpy(), rtol=1e-10, atol=1e-15)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(7)
    img, tgt = rng.random((3, 10, 12)), rng.random((3, 10, 12))
    g = L.view_loss_grad(img, tgt, 0.5)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 5, 7), (2, 9, 11), (0, 3, 2), (2, 0, 6)]:
        p, m = img.copy(), img.copy()
        p[idx] += h
        m[idx] -= h
        fd = (L.view_loss(p, tgt, 0.5)["loss"] - L.view_loss(m, tgt, 0.5)["loss"]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7 * max(1.0, abs(g[idx]) * 1e3), (idx, fd, g[idx])


def test_l1_part_alone():
    rng = np.random.default_rng(3)
    img, tgt = rng.random((3, 6, 5)), rng.random((3, 6, 5))
    tgt[0, 0, 0] = img[0, 0, 0]  # |t|' = 0 at t = 0
    assert L.view_loss(img, tgt, 0.0)["loss"] == pytest.approx(np.abs(img - tgt).mean(), abs=1e-15)
    g = L.view_loss_grad(img, tgt, 0.0)
    assert np.array_equal(g, np.sign(img - tgt) / img.size) and g[0, 0, 0] == 0.0


def test_batch_is_the_mean_over_views():
    rng = np.random.default_rng(4)
    imgs = [rng.random((3, 7, 9)), rng.random((3, 12, 5))]
    tgts = [rng.random((3, 7, 9)), rng.random((3, 12, 5))]
    b = L.batch_loss(imgs, tgts)
    assert b["loss"] == pytest.approx(np.mean([L.view_loss(i, t)["loss"] for i, t in zip(imgs, tgts)]), abs=1e-15)
    gb = L.batch_loss_grad(imgs, tgts)
    for gi, i, t in zip(gb, imgs, tgts):
        assert np.allclose(gi, L.view_loss_grad(i, t) / 2, rtol=0, atol=1e-18)
