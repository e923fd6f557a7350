"""Pins of the FP64 oracle of the significance score (Eq. 4): its ray hits against
an independent brute-force walk and closed forms, its volume normalisation
against hand-computed quantiles.  CPU only."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import brute
from paper_2501_14534_amd import scenes
from tests.test_oracle import _axis_cam, _concat, _logit, _single

Q90 = float(np.float32(0.9))


@pytest.mark.parametrize("seed,deg,masks", [(31, 3, False), (32, 1, True), (33, 0, False)])
def test_hits_equal_brute_force(orc, seed, deg, masks):
    """Tiled walk over the sorted lists vs every pixel against every Gaussian in depth order."""
    wl = scenes.tiny(n=70, seed=seed, deg=deg, masks=masks, band_masks=masks, width=41, height=27)
    # a second view from a little to the side, of another size
    wl.cams.append(scenes.make_camera((0.4, -0.2, 0.1), (0.0, 4.0, 0.0), 35, 30, 36.0))
    h = orc.count_hits(wl.scene, wl.cams, wl.opts)
    bf = brute.render(wl.scene, wl.cams, wl.opts, grad=False)
    n = wl.scene.n
    for v in range(len(wl.cams)):
        np.testing.assert_array_equal(h["hits"][v * n:(v + 1) * n], bf["hits"][v])
        # every composited pair is one hit: the per-pixel counts add up to the same total
        assert int(h["hits"][v * n:(v + 1) * n].sum()) == int(bf["counts"][v].sum())
    np.testing.assert_array_equal(h["per_gaussian"], np.sum(bf["hits"], 0))
    assert h["per_gaussian"].sum() > 0


@pytest.mark.parametrize("tile", [(8, 8), (32, 8), (64, 16)])
def test_hits_independent_of_tile_size(orc, tile):
    wl = scenes.tiny(n=90, seed=34, width=50, height=37)
    ref = orc.count_hits(wl.scene, wl.cams, wl.opts)["hits"]
    got = orc.count_hits(wl.scene, wl.cams, dataclasses.replace(wl.opts, tile_w=tile[0], tile_h=tile[1]))["hits"]
    np.testing.assert_array_equal(got, ref)


def test_single_gaussian_hits_closed_form(orc):
    """One isotropic Gaussian on the axis: its hits are the pixels of its square where
    o' exp(-r^2 / 2 var) >= 1/255, var = (f s / z)^2 + 0.3."""
    W = H = 33
    f, z, sig, o = 40.0, 3.0, 0.05, 0.6
    cam = _axis_cam(W, H, f)
    sc = _single([0, z, 0], [math.log(sig)] * 3, [1, 0, 0, 0], _logit(o), [0.5, 0.5, 0.5])
    got = orc.count_hits(sc, [cam], scenes.Opts())["hits"]
    var = (np.float64(cam.fx) * sig / z) ** 2 + 0.3
    r = math.ceil(3 * math.sqrt(var))
    o32 = 1 / (1 + math.exp(-float(np.float32(_logit(o)))))
    ys, xs = np.mgrid[0:H, 0:W] + 0.5
    dx, dy = xs - np.float64(cam.cx), ys - np.float64(cam.cy)
    a = np.minimum(float(np.float32(0.99)), o32 * np.exp(-(dx ** 2 + dy ** 2) / (2 * var)))
    use = (np.abs(dx) <= r) & (np.abs(dy) <= r) & (a >= float(np.float32(1 / 255)))
    assert 0 < int(use.sum()) < W * H
    assert int(got[0]) == int(use.sum())


def test_hits_stop_at_termination(orc):
    """Five opaque isotropic Gaussians stacked on the axis: per pixel, the closed-form alphas
    composited front to back until the transmittance would fall below 1e-4.  At the axis pixel
    that happens at the third (0.03^2 = 9e-4 >= 1e-4 > 0.03^3), so the three behind it are
    never hit there."""
    W = H = 33
    f = 40.0
    cam = _axis_cam(W, H, f)
    a, sig = 0.97, 0.004
    zs = [2.0 + 0.25 * i for i in range(5)]
    sc = _concat([_single([0, z, 0], [math.log(sig)] * 3, [1, 0, 0, 0], _logit(a), [0.5, 0.5, 0.5]) for z in zs])
    got = orc.count_hits(sc, [cam], scenes.Opts())["hits"]
    a32 = 1 / (1 + math.exp(-float(np.float32(_logit(a)))))
    amin, amax, tmin = float(np.float32(1 / 255)), float(np.float32(0.99)), float(np.float32(1e-4))
    ys, xs = np.mgrid[0:H, 0:W] + 0.5
    d2 = (xs - np.float64(cam.cx)) ** 2 + (ys - np.float64(cam.cy)) ** 2
    dmax = np.maximum(np.abs(xs - np.float64(cam.cx)), np.abs(ys - np.float64(cam.cy)))
    T = np.ones((H, W))
    alive = np.ones((H, W), bool)
    exp = []
    for z in zs:  # depth order
        var = (np.float64(cam.fx) * sig / z) ** 2 + 0.3
        r = math.ceil(3 * math.sqrt(var))
        al = np.minimum(amax, a32 * np.exp(-d2 / (2 * var)))
        use = alive & (dmax <= r) & (al >= amin)
        stop = use & (T * (1 - al) < tmin)
        alive &= ~stop
        take = use & ~stop
        T = np.where(take, T * (1 - al), T)
        exp.append(int(take.sum()))
        if z == zs[0]:
            assert take[H // 2, W // 2]
    assert not alive[H // 2, W // 2]
    np.testing.assert_array_equal(got, exp)
    # the axis pixel: hit by the first two only
    one = orc.count_hits(sc, [_axis_cam(1, 1, f)], scenes.Opts())["hits"]
    np.testing.assert_array_equal(one, [1, 1, 0, 0, 0])


def test_masked_gaussian_has_no_hits_and_no_score(orc):
    wl = scenes.tiny(n=60, seed=35, masks=True)
    sc = wl.scene.copy()
    sc.mask_logits[:] = 2.0
    sc.mask_logits[::4] = -2.0
    h = orc.count_hits(sc, wl.cams, wl.opts)["per_gaussian"]
    assert np.all(h[::4] == 0) and h.sum() > 0
    s = orc.significance(sc, h, Q90)
    assert np.all(s[::4] == 0.0)


def _vol_scene(vols, op=0.5):
    """Gaussians whose scale products are the given volumes (split evenly over the three axes)."""
    n = len(vols)
    ls = np.repeat((np.log(np.asarray(vols, np.float64)) / 3.0)[None, :], 3, 0).astype(np.float32)
    return scenes.Scene(means=np.zeros((3, n), np.float32), log_scales=ls,
                        quats=np.tile(np.array([[1], [0], [0], [0]], np.float32), (1, n)),
                        opacity_logits=np.full(n, _logit(op), np.float32), sh_dc=np.zeros((3, n), np.float32),
                        sh_rest=None, mask_logits=None, sh_mask_logits=None, sh_degree=0)


def test_volume_rank_is_the_ceiling_of_q_n(orc):
    assert orc.volume_rank(Q90, 10) == 9
    assert orc.volume_rank(Q90, 11) == 10   # 9.9 -> 10
    assert orc.volume_rank(Q90, 1) == 1
    assert orc.volume_rank(1.0, 7) == 7
    assert orc.volume_rank(1e-9, 7) == 1
    assert orc.volume_rank(Q90, 1000) == 900


def test_significance_volume_normalisation_by_hand(orc):
    """Volumes 1..10 in shuffled order: the reference volume is the 9th smallest (9), so
    gamma = min(v / 9, 1) -- the 10 is clipped to 1."""
    rng = np.random.default_rng(0)
    vols = rng.permutation(np.arange(1, 11)).astype(np.float64)
    sc = _vol_scene(vols, op=0.25)
    hits = np.arange(10, 20)
    op32 = 1 / (1 + math.exp(-float(np.float32(_logit(0.25)))))
    got = orc.significance(sc, hits, Q90)
    v32 = np.exp(sc.log_scales.astype(np.float64).sum(0))  # the volumes the float log-scales hold
    vq = np.sort(v32)[8]
    assert vq == pytest.approx(9.0, rel=1e-6)
    exp = hits * op32 * np.minimum(vols / 9.0, 1.0)
    np.testing.assert_allclose(got, exp, rtol=1e-6)
    assert got[np.argmax(vols)] == pytest.approx(hits[np.argmax(vols)] * op32, rel=1e-12)


def test_significance_equal_volumes_and_single_gaussian(orc):
    sc = _vol_scene([0.5] * 8, op=0.7)
    hits = np.array([0, 1, 2, 3, 5, 8, 13, 21])
    op32 = 1 / (1 + math.exp(-float(np.float32(_logit(0.7)))))
    np.testing.assert_allclose(orc.significance(sc, hits, Q90), hits * op32, rtol=1e-12)
    one = _vol_scene([3.0], op=0.7)
    np.testing.assert_allclose(orc.significance(one, np.array([4]), Q90), [4 * op32], rtol=1e-12)


def test_significance_is_linear_in_hits_and_opacity(orc):
    wl = scenes.tiny(n=40, seed=36)
    h = orc.count_hits(wl.scene, wl.cams, wl.opts)["per_gaussian"]
    s1 = orc.significance(wl.scene, h, Q90)
    np.testing.assert_allclose(orc.significance(wl.scene, 3 * h, Q90), 3 * s1, rtol=1e-12)
    # scaling every volume by the same factor leaves gamma unchanged
    sc = wl.scene.copy()
    sc.log_scales = (sc.log_scales + np.float32(0.5)).astype(np.float32)
    np.testing.assert_allclose(orc.significance(sc, h, Q90), s1, rtol=1e-5)
