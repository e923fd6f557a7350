"""Pins of the mask-loss oracle (oracle/mask_loss.py): closed forms, weights, central differences."""
import numpy as np
import pytest

from oracle import mask_loss as M


def test_weights_count_coefficients():
    assert np.allclose(M.band_weights(3), [3 / 15, 5 / 15, 7 / 15], rtol=0, atol=1e-16)
    assert np.allclose(M.band_weights(1), [1.0])
    assert M.band_weights(0).size == 0


def test_closed_forms():
    # sigmoid(0) = 1/2 everywhere: L_m = 1/2, L_sh = 1/2 (weights sum to one)
    z = np.zeros(10)
    r = M.mask_loss(z, np.zeros((3, 10)), 3, lam_m=1.0, lam_sh=1.0)
    assert r["l_m"] == pytest.approx(0.5, abs=1e-16) and r["l_sh"] == pytest.approx(0.5, abs=1e-16)
    gm, gsh = M.mask_loss_grad(z, np.zeros((3, 10)), 3, lam_m=1.0, lam_sh=1.0)
    assert np.allclose(gm, 0.25 / 10) and np.allclose(gsh, np.array([3, 5, 7])[:, None] / 15 * 0.25 / 10)
    # a single large logit: sigmoid -> 1, its derivative -> 0
    r = M.mask_loss(np.array([40.0]), None, 0, lam_m=1.0)
    assert r["l_m"] == pytest.approx(1.0, abs=1e-15) and r["loss"] == pytest.approx(1.0, abs=1e-15)


def test_bands_above_the_degree_are_ignored():
    rng = np.random.default_rng(0)
    sh = rng.standard_normal((3, 7))
    r1 = M.mask_loss(None, sh, 1, lam_sh=1.0)
    assert r1["l_sh"] == pytest.approx(float((1 / (1 + np.exp(-sh[0]))).mean()), abs=1e-15)
    _, g = M.mask_loss_grad(None, sh, 1)
    assert np.all(g[1:] == 0.0)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    m, sh = rng.standard_normal(6) * 2, rng.standard_normal((3, 6)) * 2
    gm, gsh = M.mask_loss_grad(m, sh, 3, 0.3, 0.7)
    h = 1e-6
    f = lambda a, b: M.mask_loss(a, b, 3, 0.3, 0.7)["loss"]  # noqa: E731
    for i in range(6):
        p, q = m.copy(), m.copy()
        p[i] += h
        q[i] -= h
        assert (f(p, sh) - f(q, sh)) / (2 * h) == pytest.approx(gm[i], abs=1e-9)
        for l in range(3):
            p, q = sh.copy(), sh.copy()
            p[l, i] += h
            q[l, i] -= h
            assert (f(m, p) - f(m, q)) / (2 * h) == pytest.approx(gsh[l, i], abs=1e-9)
