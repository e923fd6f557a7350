"""Pins of the FP64 oracle for progressive training (Sec. 3.2.4): the per-view
low-pass s = max(0.3, HW / (9 pi N)) in the projection, the target blur and the
area resize.  CPU only."""
import dataclasses
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import brute
from oracle import targets as TG
from paper_2501_14534_amd import scenes
from tests.test_oracle import _axis_cam, _logit, _single


def _prog(**kw):
    return dataclasses.replace(scenes.Opts(), lowpass_progressive=1, **kw)


def test_progressive_lowpass_single_gaussian_closed_form(orc):
    """One Gaussian, 33 x 33 view: s = 33 * 33 / (9 pi) = 38.5, so the screen variance is
    (f sigma / z)^2 + 38.5 and the footprint radius ceil(3 sqrt(var))."""
    W = H = 33
    f, z, sig, o, col = 40.0, 3.0, 0.04, 0.8, [0.9, 0.4, 0.2]
    cam = _axis_cam(W, H, f)
    sc = _single([0, z, 0], [math.log(sig)] * 3, [1, 0, 0, 0], _logit(o), col)
    img = orc.render(sc, [cam], _prog())["images"][0]
    s = W * H / (9 * math.pi)
    assert s > 0.3
    var = (np.float64(cam.fx) * sig / z) ** 2 + s
    r = math.ceil(3 * math.sqrt(var))
    ys, xs = np.mgrid[0:H, 0:W] + 0.5
    dx, dy = xs - np.float64(cam.cx), ys - np.float64(cam.cy)
    o32 = 1 / (1 + math.exp(-float(np.float32(_logit(o)))))
    a = np.minimum(float(np.float32(0.99)), o32 * np.exp(-(dx ** 2 + dy ** 2) / (2 * var)))
    use = (np.abs(dx) <= r) & (np.abs(dy) <= r) & (a >= float(np.float32(1 / 255)))
    a = np.where(use, a, 0.0)
    for ch in range(3):
        np.testing.assert_allclose(img[ch], np.float64(np.float32(col[ch])) * a, atol=1e-12)
    # and the projected conic is the inverse of that variance (with the scale the float
    # log-scale holds)
    s32 = math.exp(float(np.float32(math.log(sig))))
    var32 = (np.float64(cam.fx) * s32 / z) ** 2 + s
    pr = orc.project_views(sc, [cam], _prog())
    np.testing.assert_allclose(pr["conic"][0], [1 / var32, 0.0, 1 / var32], rtol=1e-13, atol=1e-15)


def test_progressive_lowpass_is_bounded_below_by_s0(orc):
    """With many Gaussians HW / (9 pi N) < 0.3: the same result as the fixed s = 0.3."""
    wl = scenes.tiny(n=200, seed=40, width=33, height=33)
    assert 33 * 33 / (9 * math.pi * 200) < 0.3
    a = orc.render(wl.scene, wl.cams, wl.opts)
    b = orc.render(wl.scene, wl.cams, dataclasses.replace(wl.opts, lowpass_progressive=1))
    np.testing.assert_array_equal(a["images"][0], b["images"][0])
    # and with a larger s0 the bound is what applies
    c = orc.render(wl.scene, wl.cams, dataclasses.replace(wl.opts, lowpass=0.9))
    d = orc.render(wl.scene, wl.cams, dataclasses.replace(wl.opts, lowpass=0.9, lowpass_progressive=1))
    np.testing.assert_array_equal(c["images"][0], d["images"][0])
    assert not np.array_equal(a["images"][0], c["images"][0])


def test_progressive_lowpass_is_per_view(orc):
    """Two views of different sizes: each uses its own HW / (9 pi N)."""
    wl = scenes.tiny(n=30, seed=41, width=37, height=29)
    big = scenes.make_camera((0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 74, 58, 74.0)
    cams = [wl.cams[0], big]
    both = orc.project_views(wl.scene, cams, _prog())
    for v, c in enumerate(cams):
        s = c.width * c.height / (9 * math.pi * 30)
        one = orc.project_views(wl.scene, [c], dataclasses.replace(scenes.Opts(), lowpass=s))
        n = wl.scene.n
        np.testing.assert_allclose(both["conic"][v * n:(v + 1) * n], one["conic"], rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("seed,deg,masks", [(42, 3, True), (43, 0, False)])
def test_progressive_lowpass_matches_brute_force(orc, seed, deg, masks):
    wl = scenes.tiny(n=40, seed=seed, deg=deg, masks=masks, band_masks=masks, width=31, height=27)
    assert 31 * 27 / (9 * math.pi * 40) > 0.3
    opts = _prog()
    rng = np.random.default_rng(seed)
    w = [rng.standard_normal((3, c.height, c.width)) for c in wl.cams]
    o = orc.render(wl.scene, wl.cams, opts, dL_dimages=w)
    bf = brute.render(wl.scene, wl.cams, opts, weights=w)
    np.testing.assert_allclose(o["images"][0], bf["images"][0], atol=1e-12)
    for k, g in o["grads"].items():
        ref = bf["grads"][k]
        scale = max(np.abs(ref).max(), 1e-30)
        np.testing.assert_allclose(g, ref, atol=1e-9 * scale, rtol=1e-7, err_msg=k)


# ----------------------------------------------------------------------------------------------
# Target blur

def test_gaussian_taps():
    g = TG.gaussian_taps(9, 2.4)
    assert g.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(g, g[::-1], rtol=0, atol=0)
    assert np.all(np.diff(g[:5]) > 0)
    assert g[5] / g[4] == pytest.approx(math.exp(-1 / (2 * 2.4 ** 2)), rel=1e-14)
    np.testing.assert_array_equal(TG.gaussian_taps(1, 2.4), [1.0])
    with pytest.raises(ValueError):
        TG.gaussian_taps(4, 1.0)


@pytest.mark.parametrize("k,sigma,shape", [(9, 2.4, (23, 31)), (5, 1.1, (7, 40)), (3, 0.6, (2, 3)),
                                           (9, 2.4, (4, 4)), (7, 3.0, (1, 9))])
def test_blur_matches_scipy_mirror_correlation(k, sigma, shape):
    rng = np.random.default_rng(k)
    img = rng.random(shape)
    g = TG.gaussian_taps(k, sigma)
    ref = ndi.correlate1d(ndi.correlate1d(img, g, axis=1, mode="mirror"), g, axis=0, mode="mirror")
    np.testing.assert_allclose(TG.blur_plane(img, k, sigma), ref, atol=1e-14)


def test_blur_identities():
    rng = np.random.default_rng(0)
    img = rng.random((12, 17))
    np.testing.assert_array_equal(TG.blur_plane(img, 1, 2.4), img)
    np.testing.assert_allclose(TG.blur_plane(np.full((9, 13), 0.37), 9, 2.4), 0.37, atol=1e-15)
    # a delta far from the borders spreads into the outer product of the taps
    d = np.zeros((21, 21))
    d[10, 10] = 1.0
    g = TG.gaussian_taps(9, 2.4)
    exp = np.zeros((21, 21))
    exp[6:15, 6:15] = np.outer(g, g)
    np.testing.assert_allclose(TG.blur_plane(d, 9, 2.4), exp, atol=1e-16)
    assert [TG.mirror(i, 5) for i in range(-6, 11)] == [2, 3, 4, 3, 2, 1, 0, 1, 2, 3, 4, 3, 2, 1, 0, 1, 2]


# ----------------------------------------------------------------------------------------------
# Area resize

def test_resize_integer_factor_is_the_box_mean():
    rng = np.random.default_rng(1)
    img = rng.random((24, 40))
    exp = img.reshape(3, 8, 5, 8).mean(axis=(1, 3))
    np.testing.assert_allclose(TG.resize_plane(img, 5, 3), exp, atol=1e-15)
    np.testing.assert_allclose(TG.resize_plane(img, 40, 24), img, atol=0)


@pytest.mark.parametrize("src,dst", [((13, 7), (5, 3)), ((10, 9), (4, 9)), ((3, 5), (7, 11))])
def test_resize_exact_rational_integration(src, dst):
    """Each output pixel against the exact integral of the piecewise-constant input over its
    box, in rational arithmetic."""
    (W, H), (Wo, Ho) = src, dst
    rng = np.random.default_rng(W * H)
    img = rng.integers(0, 100, (H, W))
    got = TG.resize_plane(img, Wo, Ho)
    for yo in range(Ho):
        for xo in range(Wo):
            x0, x1 = Fraction(xo * W, Wo), Fraction((xo + 1) * W, Wo)
            y0, y1 = Fraction(yo * H, Ho), Fraction((yo + 1) * H, Ho)
            acc = Fraction(0)
            for y in range(H):
                for x in range(W):
                    ox = max(Fraction(0), min(x1, x + 1) - max(x0, x))
                    oy = max(Fraction(0), min(y1, y + 1) - max(y0, y))
                    acc += ox * oy * int(img[y, x])
            assert got[yo, xo] == pytest.approx(float(acc / ((x1 - x0) * (y1 - y0))), rel=1e-14)


def test_resize_preserves_mass_and_constants():
    rng = np.random.default_rng(2)
    img = rng.random((29, 37))
    out = TG.resize_plane(img, 11, 6)
    assert out.sum() * (37 / 11) * (29 / 6) == pytest.approx(img.sum(), rel=1e-13)
    np.testing.assert_allclose(TG.resize_plane(np.full((29, 37), 0.25), 11, 6), 0.25, atol=1e-15)
