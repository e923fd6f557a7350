"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against a closed form, an invariant, a library
routine (scipy), brute force, or finite differences -- chosen so that a
dropped term, a wrong sign or index, or a transposed operand anywhere in the
oracle fails at least one of them.  CPU only.
"""
import dataclasses
import json
import math
import os

import numpy as np
import pytest
import scipy.special as sps
from scipy.spatial.transform import Rotation

from oracle import brute
from paper_2501_14534_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _opts(**kw):
    return dataclasses.replace(scenes.Opts(), **kw)


def _single(mu, log_s, quat, op_logit, dc, deg=0, rest=None):
    n = 1
    sc = scenes.Scene(
        means=np.asarray(mu, np.float32).reshape(3, n),
        log_scales=np.asarray(log_s, np.float32).reshape(3, n),
        quats=np.asarray(quat, np.float32).reshape(4, n),
        opacity_logits=np.asarray([op_logit], np.float32),
        sh_dc=np.asarray(dc, np.float32).reshape(3, n),
        sh_rest=None if rest is None else np.asarray(rest, np.float32).reshape(-1, 3, n),
        mask_logits=None, sh_mask_logits=None, sh_degree=deg)
    return sc


def _concat(scs):
    out = {}
    for f in dataclasses.fields(scs[0]):
        v = getattr(scs[0], f.name)
        if isinstance(v, np.ndarray):
            out[f.name] = np.concatenate([getattr(s, f.name) for s in scs], -1)
        else:
            out[f.name] = v
    return scenes.Scene(**out)


def _logit(p):
    return math.log(p / (1.0 - p))


# ----------------------------------------------------------------------------------------------
# Paper constants (golden fixture, each cited)

def test_paper_constants_fixture():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    # 59 parameters: mean 3 + scale 3 + rotation 4 + opacity 1 + diffuse colour 3 + SH rest 45
    assert 3 + 3 + 4 + 1 + 3 + g["sh_rest_dims"]["value"] == g["params_per_gaussian"]["value"]
    assert ((g["sh_bands"]["value"] + 1) ** 2 - 1) * 3 == g["sh_rest_dims"]["value"]
    assert scenes.Opts().lowpass == pytest.approx(g["lowpass_s"]["value"])


# ----------------------------------------------------------------------------------------------
# SH basis

def _unit_dirs(n, seed=0):
    d = np.random.default_rng(seed).standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_sh_basis_matches_scipy(orc):
    d = _unit_dirs(200)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2 * np.pi)
    ref = np.zeros((len(d), 16))
    for l in range(4):
        for m in range(-l, l + 1):
            Yc = sps.sph_harm_y(l, abs(m), theta, phi)  # complex, Condon-Shortley phase included
            if m > 0:
                val = math.sqrt(2) * Yc.real
            elif m < 0:
                val = math.sqrt(2) * Yc.imag
            else:
                val = Yc.real
            ref[:, l * l + l + m] = val
    got = orc.sh_basis(d)
    np.testing.assert_allclose(got, ref, atol=1e-13, rtol=0)


def test_sh_orthonormal_quadrature(orc):
    # Gauss-Legendre in cos(theta) x uniform phi integrates products of degree <= 6 exactly
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 16
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    Y = orc.sh_basis(d)
    gram = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


def test_sh_addition_theorem(orc):
    Y = orc.sh_basis(_unit_dirs(100, 1))
    for l in range(4):
        s = (Y[:, l * l:(l + 1) ** 2] ** 2).sum(1)
        np.testing.assert_allclose(s, (2 * l + 1) / (4 * np.pi), rtol=1e-13)


def test_brute_sh_agrees_with_oracle_on_sphere(orc):
    import torch
    d = _unit_dirs(64, 2)
    a = brute.sh_real(torch.tensor(d)).numpy()
    np.testing.assert_allclose(a, orc.sh_basis(d), atol=1e-14)


# ----------------------------------------------------------------------------------------------
# Projection

def test_cov3d_matches_scipy_rotation(orc):
    wl = scenes.tiny(n=20, seed=3, unit_quats=False)
    sc = wl.scene
    got = orc.cov3d(sc)
    q = sc.quats.astype(np.float64)
    Rm = Rotation.from_quat(np.stack([q[1], q[2], q[3], q[0]], 1)).as_matrix()  # scipy wants x,y,z,w
    s2 = np.exp(2 * sc.log_scales.astype(np.float64)).T
    Sig = np.einsum("nik,nk,njk->nij", Rm, s2, Rm)
    iu = np.triu_indices(3)
    np.testing.assert_allclose(got, Sig[:, iu[0], iu[1]], rtol=1e-12, atol=1e-16)


def test_camera_pose_and_depth(orc):
    cam = scenes.make_camera((0.0, -4.0, 0.0), (0, 0, 0), 64, 48, 50.0)
    sc = _concat([_single(m, [-3, -3, -3], [1, 0, 0, 0], 0.0, [0.5] * 3)
                  for m in ([0, 0, 0], [1, 0, 0], [0, 0, 1], [0, 1, 0])])
    pr = orc.project(sc, cam, scenes.Opts())
    assert pr["valid"].all()
    np.testing.assert_allclose(pr["uv"][0], [32.0, 24.0], atol=1e-6)   # origin at the principal point
    assert pr["uv"][1, 0] > 32.0 + 5 and abs(pr["uv"][1, 1] - 24.0) < 1e-5  # +x world is right
    assert pr["uv"][2, 1] < 24.0 - 5 and abs(pr["uv"][2, 0] - 32.0) < 1e-5  # +z world (up) is up
    np.testing.assert_allclose(pr["depth"], [4.0, 4.0, 4.0, 5.0], rtol=1e-6)
    np.testing.assert_allclose(pr["uv"][1, 0], 32.0 + 50.0 * 1.0 / 4.0, rtol=1e-6)  # pinhole: f x / z


def test_projection_closed_form_on_axis(orc):
    # identity rotation on the optical axis: Sigma' = diag((f sx/z)^2, (f sz/z)^2) + s I
    W, H, f, z = 64, 48, 80.0, 3.0
    cam = scenes.make_camera((0.0, 0.0, 0.0), (0.0, 1.0, 0.0), W, H, f)
    sx, sy, sz = 0.02, 0.07, 0.05  # world axes; camera x = world x, camera y = -world z
    sc = _single([0, z, 0], np.log([sx, sy, sz]), [1, 0, 0, 0], 0.3, [0.5] * 3)
    for lp in (0.3, 0.0, 1.7):
        pr = orc.project(sc, cam, _opts(lowpass=lp))
        a, b, c = pr["cov2d"][0]
        np.testing.assert_allclose([a, b, c], [(f * sx / z) ** 2 + lp, 0.0, (f * sz / z) ** 2 + lp],
                                   rtol=1e-6, atol=1e-12)
        lam = max(a, c)
        assert pr["radius"][0] == math.ceil(3 * math.sqrt(lam))
        A, B, C = pr["conic"][0]
        M = np.array([[a, b], [b, c]]) @ np.array([[A, B], [B, C]])
        np.testing.assert_allclose(M, np.eye(2), atol=1e-12)
        np.testing.assert_allclose(pr["uv"][0], [W / 2, H / 2], atol=1e-6)
        assert pr["opacity"][0] == pytest.approx(1 / (1 + math.exp(-0.3)), rel=1e-7)


def test_projection_jacobian_is_derivative_of_perspective_map(orc):
    # Off-axis, rotated, anisotropic: Sigma' must be J Sigma J^T + sI with J the derivative
    # (here by central differences) of the world -> pixel map at the mean.
    cam = scenes.make_camera((0.3, -2.0, 0.4), (0.1, 0.5, -0.2), 96, 72, 70.0)
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)

    def pix(x):
        c = R @ x + t
        return np.array([cam.fx * c[0] / c[2] + cam.cx, cam.fy * c[1] / c[2] + cam.cy])

    rng = np.random.default_rng(5)
    for _ in range(5):
        mu = np.array([rng.uniform(-0.4, 0.6), rng.uniform(0.0, 1.0), rng.uniform(-0.5, 0.3)], np.float32)
        q = rng.standard_normal(4).astype(np.float32)
        ls = rng.uniform(-4, -2, 3).astype(np.float32)
        sc = _single(mu, ls, q, 0.0, [0.5] * 3)
        pr = orc.project(sc, cam, scenes.Opts())
        assert pr["valid"][0]
        h = 1e-6
        J = np.stack([(pix(mu.astype(np.float64) + h * e) - pix(mu.astype(np.float64) - h * e)) / (2 * h)
                      for e in np.eye(3)], 1)
        iu = orc.cov3d(sc)[0]
        Sig = np.array([[iu[0], iu[1], iu[2]], [iu[1], iu[3], iu[4]], [iu[2], iu[4], iu[5]]])
        S2 = J @ Sig @ J.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(pr["cov2d"][0], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-6)
        np.testing.assert_allclose(pr["uv"][0], pix(mu.astype(np.float64)), rtol=1e-12)


def test_rotation_about_optical_axis_rotates_screen_covariance(orc):
    W, H, f, z = 64, 64, 60.0, 2.5
    cam = scenes.make_camera((0.0, 0.0, 0.0), (0.0, 1.0, 0.0), W, H, f)
    ls = np.log([0.05, 0.01, 0.02])
    base = orc.project(_single([0, z, 0], ls, [1, 0, 0, 0], 0.0, [0.5] * 3), cam, _opts(lowpass=0.0))["cov2d"][0]
    S0 = np.array([[base[0], base[1]], [base[1], base[2]]])
    for th in (0.3, 1.1, 2.0):
        # rotation by th about world +y, the optical axis; seen on screen as a rotation by -th
        q = [math.cos(th / 2), 0.0, math.sin(th / 2), 0.0]
        c = orc.project(_single([0, z, 0], ls, q, 0.0, [0.5] * 3), cam, _opts(lowpass=0.0))["cov2d"][0]
        S = np.array([[c[0], c[1]], [c[1], c[2]]])
        Rs = np.array([[math.cos(th), math.sin(th)], [-math.sin(th), math.cos(th)]])
        Rs2 = Rs.T
        ok = np.allclose(S, Rs @ S0 @ Rs.T, rtol=1e-5, atol=1e-9) or np.allclose(S, Rs2 @ S0 @ Rs2.T, rtol=1e-5,
                                                                                    atol=1e-9)
        assert ok
        np.testing.assert_allclose(np.linalg.eigvalsh(S), np.linalg.eigvalsh(S0), rtol=1e-6)


def _clamp_cam():
    # camera at the origin looking along world +y: camera x = world x, camera y = -world z,
    # camera z = world y (the rotation's entries are exactly 0 and +-1)
    return scenes.make_camera((0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 40, 30, 50.0)


@pytest.mark.parametrize("rx,ry", [(0.3, -0.2), (1.5, 0.0), (-1.5, 0.0), (0.0, 0.9), (0.0, -0.9), (2.0, -1.2)])
def test_jacobian_guard_closed_form(orc, rx, ry):
    """EWA with the lateral-ratio guard (reading R4 of Eq. 1's Jacobian): an isotropic Gaussian of
    world std sigma at camera position (rx z, ry z, z) has J J^T sigma^2 = (f/z)^2 sigma^2
    [[1 + rx'^2, rx' ry'], [rx' ry', 1 + ry'^2]] with rx' = clamp(rx, +-tan_clamp W/(2 f)) and
    ry' = clamp(ry, +-tan_clamp H/(2 f)); the cases put the ratios inside and beyond the limits on
    both sides of both axes."""
    cam = _clamp_cam()
    f, z, sig, tc = float(cam.fx), 3.0, 0.2, 1.3
    limx, limy = tc * cam.width / (2 * f), tc * cam.height / (2 * f)   # 0.52, 0.39
    sc = _single([rx * z, z, -ry * z], [math.log(sig)] * 3, [1, 0, 0, 0], 0.0, [0.5] * 3)
    lp = 0.3
    pr = orc.project(sc, cam, _opts(lowpass=lp, tan_clamp=tc))
    assert pr["valid"][0] == 1
    sig64 = math.exp(float(np.float32(math.log(sig))))  # exp of the stored float log-scale
    mu = sc.means.astype(np.float64)[:, 0]
    x, y, zz = mu[0], -mu[2], mu[1]                # camera coordinates
    rxc, ryc = np.clip(x / zz, -limx, limx), np.clip(y / zz, -limy, limy)
    k = (f / zz) ** 2 * sig64 ** 2
    exp = [k * (1 + rxc ** 2) + lp, k * rxc * ryc, k * (1 + ryc ** 2) + lp]
    np.testing.assert_allclose(pr["cov2d"][0], exp, rtol=1e-10, atol=1e-14)
    # the screen position uses the unclamped ratios
    np.testing.assert_allclose(pr["uv"][0], [f * x / zz + cam.cx, f * y / zz + cam.cy], rtol=1e-12)
    if abs(rx) > limx or abs(ry) > limy:
        # an unguarded Jacobian would give a different, larger covariance
        unguarded = [k * (1 + (x / zz) ** 2) + lp, k * (x / zz) * (y / zz), k * (1 + (y / zz) ** 2) + lp]
        assert not np.allclose(pr["cov2d"][0], unguarded, rtol=1e-6)


def test_jacobian_guard_is_the_perspective_derivative_at_the_clamped_point(orc):
    """Off-axis, rotated, anisotropic Gaussians beyond the guard: Sigma' = J~ Sigma J~^T + sI where
    J~ is the derivative (central differences) of the world -> pixel map at the point whose camera
    coordinates are (z rx', z ry', z), the mean moved laterally onto the clamp limit."""
    cam = _clamp_cam()
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    limx = 1.3 * cam.width / (2 * float(cam.fx))
    limy = 1.3 * cam.height / (2 * float(cam.fy))

    def pix(xw):
        c = R @ xw + t
        return np.array([cam.fx * c[0] / c[2] + cam.cx, cam.fy * c[1] / c[2] + cam.cy])

    rng = np.random.default_rng(17)
    checked = 0
    for rx, ry in ((0.9, 0.1), (-1.1, 0.2), (0.2, 0.7), (-0.1, -1.4), (1.6, 0.8)):
        z = rng.uniform(2.0, 5.0)
        mu = np.array([rx * z, z, -ry * z], np.float32)
        q = rng.standard_normal(4).astype(np.float32)
        ls = rng.uniform(-3, -1.5, 3).astype(np.float32)
        sc = _single(mu, ls, q, 0.0, [0.5] * 3)
        pr = orc.project(sc, cam, scenes.Opts())
        assert pr["valid"][0]
        cc = R @ mu.astype(np.float64) + t
        moved_cam = np.array([cc[2] * np.clip(cc[0] / cc[2], -limx, limx),
                              cc[2] * np.clip(cc[1] / cc[2], -limy, limy), cc[2]])
        moved = R.T @ (moved_cam - t)
        h = 1e-6
        J = np.stack([(pix(moved + h * e) - pix(moved - h * e)) / (2 * h) for e in np.eye(3)], 1)
        iu = orc.cov3d(sc)[0]
        Sig = np.array([[iu[0], iu[1], iu[2]], [iu[1], iu[3], iu[4]], [iu[2], iu[4], iu[5]]])
        S2 = J @ Sig @ J.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(pr["cov2d"][0], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-6)
        checked += 1
    assert checked == 5


def test_jacobian_guard_derivatives(orc):
    """Beyond the guard the covariance no longer depends on the clamped lateral coordinate but
    still on depth (the derivative of the implemented function, R17): central differences of the
    oracle's projected covariance in camera x and z, against the closed form
    d/dz [(f/z)^2 sigma^2 (1 + rx'^2)] = -2 (f/z)^2 sigma^2 (1 + rx'^2) / z."""
    cam = _clamp_cam()
    f, z, sig = float(cam.fx), 3.0, 0.2
    limx = 1.3 * cam.width / (2 * f)

    def cov(xc, zc):
        sc = _single([xc, zc, 0.0], [math.log(sig)] * 3, [1, 0, 0, 0], 0.0, [0.5] * 3)
        sc.means = sc.means.astype(np.float64)
        sc.means[:, 0] = [xc, zc, 0.0]
        return orc.project(sc, cam, _opts(lowpass=0.0))["cov2d"][0]

    s2 = math.exp(2 * float(np.float32(math.log(sig))))
    h = 1e-5
    for x in (1.2 * z, -1.2 * z):     # beyond the guard on both sides
        dx = (cov(x + h, z) - cov(x - h, z)) / (2 * h)
        np.testing.assert_allclose(dx, 0.0, atol=1e-9)
        dz = (cov(x, z + h) - cov(x, z - h)) / (2 * h)
        np.testing.assert_allclose(dz[0], -2 * (f / z) ** 2 * s2 * (1 + limx ** 2) / z, rtol=1e-6)
    x = 0.3 * z                        # inside: the lateral coordinate enters through rx
    dx = (cov(x + h, z) - cov(x - h, z)) / (2 * h)
    np.testing.assert_allclose(dx[0], 2 * (f / z) ** 2 * s2 * x / z ** 2, rtol=1e-6)


def test_oracle_gradients_match_finite_differences_beyond_the_guard(orc):
    """Gradients of a scene whose Gaussians sit beyond the Jacobian guard but still reach the
    screen (large, near the edges): the oracle's analytic derivative of the composited image
    against central differences of its own forward, which the closed forms above pin."""
    cam = scenes.make_camera((0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 40, 30, 40.0)
    rng = np.random.default_rng(41)
    n = 12
    z = rng.uniform(2.0, 3.0, n)
    side = rng.choice([-1.0, 1.0], n)
    axis = rng.integers(0, 2, n)
    # ratio beyond the guard (0.65 in x, 0.49 in y) by up to 40 %
    r = rng.uniform(1.05, 1.4, n)
    rx = np.where(axis == 0, side * 0.65 * r, rng.uniform(-0.3, 0.3, n))
    ry = np.where(axis == 1, side * 0.49 * r, rng.uniform(-0.2, 0.2, n))
    means = np.stack([rx * z, z, -ry * z]).astype(np.float32)
    sc = scenes.Scene(means=means, log_scales=rng.uniform(-1.6, -1.2, (3, n)).astype(np.float32),
                      quats=rng.standard_normal((4, n)).astype(np.float32),
                      opacity_logits=rng.normal(0.0, 0.5, n).astype(np.float32),
                      sh_dc=rng.normal(0.5, 0.2, (3, n)).astype(np.float32), sh_rest=None, mask_logits=None,
                      sh_mask_logits=None, sh_degree=0)
    pr = orc.project(sc, cam, scenes.Opts())
    lim = np.where(axis == 0, 0.65, 0.49)
    assert pr["valid"].all() and np.all(np.abs(np.where(axis == 0, rx, ry)) > lim)
    wl = scenes.Workload("beyond_guard", sc, [cam], scenes.Opts(), [np.zeros((3, 30, 40), np.float32)])
    img = orc.render(sc, [cam], scenes.Opts())["images"][0]
    assert np.abs(img).sum() > 1.0  # the guarded Gaussians do reach the screen
    w = _loss_weights(wl, 9)
    n_ok = _fd_check(orc, wl, w, ["means", "log_scales", "quats"], 8, 1)
    assert n_ok >= 12


def test_equal_depth_ties_are_ordered_by_index(orc):
    """Reading R2: Gaussians at bit-equal depth composite in index order.  Three coincident
    Gaussians on the axis pixel, all at depth 2 (same float bits), with distinct primary colours,
    so every other order gives another colour; at the axis pixel G = 1, so the colour is the
    closed form c_0 a_0 + c_1 a_1 (1 - a_0) + c_2 a_2 (1 - a_0)(1 - a_1)."""
    cam = _axis_cam()
    ops = [0.6, 0.5, 0.7]
    cols = [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]
    sc = _concat([_single([0.0, 2.0, 0.0], [math.log(0.05)] * 3, [1, 0, 0, 0], _logit(ops[i]), cols[i])
                  for i in range(3)])
    o = orc.render(sc, [cam], scenes.Opts())
    a = [1 / (1 + math.exp(-float(np.float32(_logit(p))))) for p in ops]
    exp = (np.array(cols[0]) * a[0] + np.array(cols[1]) * a[1] * (1 - a[0])
           + np.array(cols[2]) * a[2] * (1 - a[0]) * (1 - a[1]))
    np.testing.assert_allclose(o["images"][0][:, 16, 16], exp, rtol=1e-12)
    # the binning holds the equal keys in index order
    pr = orc.project(sc, cam, scenes.Opts())
    b = orc.bin([cam], scenes.Opts(), sc.n, pr["uv"][:, 0].astype(np.float32), pr["uv"][:, 1].astype(np.float32),
                pr["depth"].astype(np.float32), pr["radius"], pr["valid"])
    keys = b["keys"]
    same = keys[1:] == keys[:-1]
    assert same.sum() >= 2
    assert np.all(b["ids"][1:][same] > b["ids"][:-1][same])


def test_equal_depth_ties_match_brute_force(orc):
    """Many Gaussians sharing a few exact depths (world y on a coarse grid, axis camera): the tiled
    oracle's image equals the per-pixel brute-force renderer's, whose order is (depth, index)."""
    rng = np.random.default_rng(43)
    n = 80
    means = np.stack([rng.uniform(-0.6, 0.6, n), rng.choice([2.0, 2.25, 2.5], n), rng.uniform(-0.6, 0.6, n)])
    sc = scenes.Scene(means=means.astype(np.float32), log_scales=rng.normal(-2.6, 0.3, (3, n)).astype(np.float32),
                      quats=rng.standard_normal((4, n)).astype(np.float32),
                      opacity_logits=rng.normal(1.0, 1.0, n).astype(np.float32),
                      sh_dc=rng.uniform(0.0, 1.0, (3, n)).astype(np.float32), sh_rest=None, mask_logits=None,
                      sh_mask_logits=None, sh_degree=0)
    cam = _axis_cam(37, 29, 30.0)
    opts = scenes.Opts()
    pr = orc.project(sc, cam, opts)
    b = orc.bin([cam], opts, sc.n, pr["uv"][:, 0].astype(np.float32), pr["uv"][:, 1].astype(np.float32),
                pr["depth"].astype(np.float32), pr["radius"], pr["valid"])
    same = b["keys"][1:] == b["keys"][:-1]
    assert same.sum() > 50  # ties are common, not incidental
    o = orc.render(sc, [cam], opts)
    bf = brute.render(sc, [cam], opts, grad=False)
    np.testing.assert_allclose(o["images"][0], bf["images"][0], atol=1e-12)
    # reversing the index order of the tied Gaussians changes the image: the pin is not vacuous
    rev = sc.subset(np.arange(n)[::-1].copy())
    o_rev = orc.render(rev, [cam], opts)["images"][0]
    assert np.abs(o_rev - o["images"][0]).max() > 1e-3


def test_near_plane_and_invalid_inputs_are_culled(orc):
    cam = scenes.make_camera((0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 32, 32, 32.0)
    good = _single([0, 2, 0], [-3] * 3, [1, 0, 0, 0], 0.0, [0.5] * 3)
    behind = _single([0, -1, 0], [-3] * 3, [1, 0, 0, 0], 0.0, [0.5] * 3)
    near = _single([0, 0.1, 0], [-3] * 3, [1, 0, 0, 0], 0.0, [0.5] * 3)
    zeroq = _single([0, 2, 0], [-3] * 3, [0, 0, 0, 0], 0.0, [0.5] * 3)
    nanm = _single([np.nan, 2, 0], [-3] * 3, [1, 0, 0, 0], 0.0, [0.5] * 3)
    pr = orc.project(_concat([good, behind, near, zeroq, nanm]), cam, scenes.Opts())
    assert pr["valid"].tolist() == [1, 0, 0, 0, 0]


def test_sh_degree0_colour_is_diffuse_and_clamped(orc):
    wl = scenes.tiny(n=30, seed=4, deg=0)
    pr = orc.project(wl.scene, wl.cams[0], wl.opts)
    v = pr["valid"] == 1
    np.testing.assert_array_equal(pr["rgb"][v], np.maximum(wl.scene.sh_dc.T[v].astype(np.float64), 0.0))


def test_band_masks_off_equals_degree0(orc):
    wl = scenes.tiny(n=30, seed=5, deg=3, band_masks=True)
    sc = wl.scene.copy()
    sc.sh_mask_logits[:] = -5.0  # sigmoid < eps: every band masked
    pr = orc.project(sc, wl.cams[0], wl.opts)
    sc0 = sc.copy()
    sc0.sh_degree, sc0.sh_rest, sc0.sh_mask_logits = 0, None, None
    pr0 = orc.project(sc0, wl.cams[0], wl.opts)
    for k in ("uv", "conic", "rgb", "opacity", "radius", "valid"):
        np.testing.assert_array_equal(pr[k], pr0[k])


# ----------------------------------------------------------------------------------------------
# Binning and ordering

def _bin_from(orc, wl, pr):
    return orc.bin(wl.cams, wl.opts, wl.scene.n, pr["uv"][:, 0].astype(np.float32),
                   pr["uv"][:, 1].astype(np.float32), pr["depth"].astype(np.float32), pr["radius"], pr["valid"])


def test_binning_invariants(orc):
    wl = scenes.tiny(n=200, seed=6, width=70, height=45)
    pr = orc.project_views(wl.scene, wl.cams, wl.opts)
    b = _bin_from(orc, wl, pr)
    K = b["K"]
    assert K == int(b["tiles_touched"].sum()) > 0
    r = b["ranges"].astype(np.int64)
    assert int((r[:, 1] - r[:, 0]).sum()) == K
    keys = b["keys"]
    assert np.all(keys[1:] >= keys[:-1])
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    for t in range(r.shape[0]):
        seg = b["ids"][r[t, 0]:r[t, 1]]
        assert len(np.unique(seg)) == len(seg)
        assert np.all(tiles[r[t, 0]:r[t, 1]] == t)
    # equal keys are ordered by id
    same = keys[1:] == keys[:-1]
    assert np.all(b["ids"][1:][same] > b["ids"][:-1][same])


def test_tiled_oracle_equals_brute_force_per_pixel(orc):
    for seed, deg, masks in ((7, 3, False), (8, 2, True), (9, 0, False)):
        wl = scenes.tiny(n=60, seed=seed, deg=deg, masks=masks, band_masks=masks, width=37, height=29)
        o = orc.render(wl.scene, wl.cams, wl.opts)
        bf = brute.render(wl.scene, wl.cams, wl.opts, grad=False)
        np.testing.assert_allclose(o["images"][0], bf["images"][0], atol=1e-12)
        np.testing.assert_allclose(o["T_final"][0], bf["T_final"][0], atol=1e-12)
        # last_contrib bounds the number of composited pairs
        assert np.all(o["last_contrib"][0] >= bf["counts"][0])


@pytest.mark.parametrize("tile", [(8, 8), (32, 8), (4, 16), (64, 64)])
def test_image_independent_of_tile_size(orc, tile):
    wl = scenes.tiny(n=80, seed=10, width=50, height=37)
    ref = orc.render(wl.scene, wl.cams, wl.opts)["images"][0]
    o2 = dataclasses.replace(wl.opts, tile_w=tile[0], tile_h=tile[1])
    got = orc.render(wl.scene, wl.cams, o2)["images"][0]
    np.testing.assert_array_equal(got, ref)


# ----------------------------------------------------------------------------------------------
# Compositing closed forms

def _axis_cam(W=33, H=33, f=40.0):
    # principal point at a pixel centre, so the on-axis Gaussian sits exactly on pixel (W//2, H//2)
    return scenes.make_camera((0.0, 0.0, 0.0), (0.0, 1.0, 0.0), W, H, f, cx=W // 2 + 0.5, cy=H // 2 + 0.5)


def test_single_isotropic_gaussian_image(orc):
    W = H = 33
    f, z, sig, o, col = 40.0, 3.0, 0.04, 0.8, [0.9, 0.4, 0.2]
    cam = _axis_cam(W, H, f)
    sc = _single([0, z, 0], [math.log(sig)] * 3, [1, 0, 0, 0], _logit(o), col)
    bg = (0.1, 0.2, 0.3)
    opts = _opts(bg=bg)
    img = orc.render(sc, [cam], opts)["images"][0]
    var = (np.float64(cam.fx) * sig / z) ** 2 + 0.3
    r = math.ceil(3 * math.sqrt(var))
    ys, xs = np.mgrid[0:H, 0:W] + 0.5
    dx, dy = xs - np.float64(cam.cx), ys - np.float64(cam.cy)
    a = np.minimum(float(np.float32(0.99)), o * np.exp(-(dx ** 2 + dy ** 2) / (2 * var)))
    use = (np.abs(dx) <= r) & (np.abs(dy) <= r) & (a >= float(np.float32(1 / 255)))
    a = np.where(use, a, 0.0)
    o32 = 1 / (1 + math.exp(-np.float32(_logit(o))))
    a = a * (o32 / o)
    for ch in range(3):
        exp = np.float64(np.float32(col[ch])) * a + (1 - a) * bg[ch]
        np.testing.assert_allclose(img[ch], exp, atol=1e-12)


def test_telescoping_transmittance(orc):
    wl = scenes.tiny(n=120, seed=11, deg=0, opacity=(1.5, 1.0))
    sc = wl.scene.copy()
    sc.sh_dc[:] = 1.0
    o = orc.render(sc, wl.cams, wl.opts)
    np.testing.assert_allclose(o["images"][0][0], 1.0 - o["T_final"][0], atol=1e-12)


def test_termination_stack(orc):
    cam = _axis_cam()
    # four Gaussians on the axis pixel with alpha 0.95 at its centre, distinct depths and colours
    cols = [[0.9, 0.1, 0.1], [0.1, 0.8, 0.1], [0.1, 0.1, 0.7], [0.5, 0.5, 0.5]]
    a = 0.95
    sc = _concat([_single([0, 2.0 + 0.25 * i, 0], [math.log(0.05)] * 3, [1, 0, 0, 0], _logit(a), cols[i])
                  for i in range(4)])
    o = orc.render(sc, [cam], scenes.Opts())
    a32 = 1 / (1 + math.exp(-float(np.float32(_logit(a)))))
    px = o["images"][0][:, 16, 16]
    c = np.array(cols, np.float32).astype(np.float64)
    exp = c[0] * a32 + c[1] * a32 * (1 - a32) + c[2] * a32 * (1 - a32) ** 2  # the 4th is not composited
    np.testing.assert_allclose(px, exp, rtol=1e-12)
    assert o["T_final"][0][16, 16] == pytest.approx((1 - a32) ** 3, rel=1e-12)
    assert o["last_contrib"][0][16, 16] == 3


def test_alpha_cap_and_skip(orc):
    cam = _axis_cam()
    # opacity ~1 at the centre: alpha capped at the single-precision 0.99
    sc = _single([0, 2.0, 0], [math.log(0.05)] * 3, [1, 0, 0, 0], 30.0, [1.0, 1.0, 1.0])
    o = orc.render(sc, [cam], scenes.Opts())
    assert o["images"][0][0, 16, 16] == float(np.float32(0.99))
    # opacity below 1/255 everywhere: the image is the background exactly
    sc2 = _single([0, 2.0, 0], [math.log(0.05)] * 3, [1, 0, 0, 0], _logit(0.003), [1.0, 1.0, 1.0])
    o2 = orc.render(sc2, [cam], _opts(bg=(0.25, 0.5, 0.75)))
    for ch, b in enumerate((0.25, 0.5, 0.75)):
        assert np.all(o2["images"][0][ch] == b)


def test_mask_zero_equals_deleted(orc):
    wl = scenes.tiny(n=50, seed=12, masks=True)
    sc = wl.scene.copy()
    sc.mask_logits[:] = 2.0
    sc.mask_logits[::3] = -2.0  # sigmoid(-2) = 0.12 < 0.5: masked out
    o = orc.render(sc, wl.cams, wl.opts)
    keep = np.ones(sc.n, bool)
    keep[::3] = False
    sub = sc.subset(keep)
    o2 = orc.render(sub, wl.cams, wl.opts)
    np.testing.assert_array_equal(o["images"][0], o2["images"][0])


# ----------------------------------------------------------------------------------------------
# Derivatives

def _loss_weights(wl, seed=0):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((3, c.height, c.width)) for c in wl.cams]


@pytest.mark.parametrize("seed,deg,masks", [(20, 3, True), (21, 1, False), (22, 0, True)])
def test_oracle_gradients_match_brute_force_autograd(orc, seed, deg, masks):
    wl = scenes.tiny(n=40, seed=seed, deg=deg, masks=masks, band_masks=masks, width=31, height=27)
    w = _loss_weights(wl, seed)
    o = orc.render(wl.scene, wl.cams, wl.opts, dL_dimages=w)
    bf = brute.render(wl.scene, wl.cams, wl.opts, weights=w)
    for k, g in o["grads"].items():
        ref = bf["grads"][k]
        scale = max(np.abs(ref).max(), 1e-30)
        np.testing.assert_allclose(g, ref, atol=1e-9 * scale, rtol=1e-7, err_msg=k)


def _fd_check(orc, wl, w, names, count, seed, h_rel=1e-6):
    """Central differences of L = sum(w * image) at decision-stable points."""
    rng = np.random.default_rng(seed)
    eps = (1e-9, 1e-9, 1e-9)
    base = orc.render(wl.scene, wl.cams, wl.opts, dL_dimages=w, eps=eps)
    checked = 0
    for name in names:
        arr = getattr(wl.scene, name)
        flat_idx = rng.choice(arr.size, size=min(count, arr.size), replace=False)
        for fi in flat_idx:
            idx = np.unravel_index(fi, arr.shape)
            x0 = float(arr[idx])
            h = h_rel * max(1.0, abs(x0))
            vals, hashes = [], []
            for sgn in (1, -1):
                sc = wl.scene.copy()
                a64 = {k: v.astype(np.float64) for k, v in sc.arrays().items()}
                a64[name][idx] = x0 + sgn * h
                # the oracle widens float32 -> float64; perturb in float64 directly
                for k, v in a64.items():
                    setattr(sc, k, v)
                r = orc.render(sc, wl.cams, wl.opts, eps=eps, lists=None)
                vals.append(sum((im * ww).sum() for im, ww in zip(r["images"], w)))
                hashes.append(r["fwd"]["hash"])
            if not (np.array_equal(hashes[0], base["fwd"]["hash"]) and np.array_equal(hashes[1], base["fwd"]["hash"])):
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            an = base["grads"][name][idx]
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-4 * np.abs(base["grads"][name]).max(), 1e-12), \
                (name, idx, fd, an)
            checked += 1
    return checked


def test_oracle_gradients_match_finite_differences(orc):
    wl = scenes.tiny(n=25, seed=30, deg=3, masks=True, band_masks=True, width=24, height=20)
    w = _loss_weights(wl, 3)
    # mask logits are excluded: the hard masks are piecewise constant, so central differences see 0
    # where the straight-through estimator defines sigma'(m); test_straight_through_mask_identities pins those
    n = _fd_check(orc, wl, w, ["means", "log_scales", "quats", "opacity_logits", "sh_dc", "sh_rest"], 6, 0)
    assert n >= 24


def test_straight_through_mask_identities(orc):
    # o' = M o and s' = M s with dM/dm = sigma'(m): dL/dm = sigma'(m) (o dL/do' + sum_k s_k dL/ds'_k)
    # = sigma'(m) (dL/dl / (1 - sigma(l)) + sum_k dL/dlog_s_k) for the opacity logit l.
    wl = scenes.tiny(n=30, seed=31, deg=3, masks=True, band_masks=True)
    sc = wl.scene.copy()
    sc.mask_logits[:] = np.abs(sc.mask_logits) + 0.1  # every Gaussian on
    sc.sh_mask_logits[:] = np.abs(sc.sh_mask_logits) + 0.1  # every band on
    w = _loss_weights(wl, 4)
    g = orc.render(sc, wl.cams, wl.opts, dL_dimages=w)["grads"]
    m = sc.mask_logits.astype(np.float64)
    lo = sc.opacity_logits.astype(np.float64)
    sm, so = 1 / (1 + np.exp(-m)), 1 / (1 + np.exp(-lo))
    exp = sm * (1 - sm) * (g["opacity_logits"] / (1 - so) + g["log_scales"].sum(0))
    np.testing.assert_allclose(g["mask_logits"], exp, rtol=1e-9, atol=1e-14)
    # band l: dL/dm_l = sigma'(m_l) sum_{k in band, ch} c_k,ch dL/dc_k,ch
    bm = sc.sh_mask_logits.astype(np.float64)
    rest = sc.sh_rest.astype(np.float64)
    for l in range(1, 4):
        s = 1 / (1 + np.exp(-bm[l - 1]))
        ks = slice(l * l - 1, (l + 1) ** 2 - 1)
        e = s * (1 - s) * (rest[ks] * g["sh_rest"][ks]).sum((0, 1))
        np.testing.assert_allclose(g["sh_mask_logits"][l - 1], e, rtol=1e-9, atol=1e-14)


def test_masked_out_gaussians_get_zero_render_gradient(orc):
    wl = scenes.tiny(n=40, seed=32, deg=2, masks=True)
    w = _loss_weights(wl, 5)
    g = orc.render(wl.scene, wl.cams, wl.opts, dL_dimages=w)["grads"]
    off = 1 / (1 + np.exp(-wl.scene.mask_logits.astype(np.float64))) <= wl.scene.mask_eps
    assert off.any() and (~off).any()
    for k, v in g.items():
        assert np.all(v[..., off] == 0.0), k


def test_single_gaussian_closed_form_derivatives(orc):
    # pixel value c a(rho) + (1 - a) bg on the axis pixel: d/dc = a, d/d(opacity logit) = (c - bg) G o (1 - o)
    cam = _axis_cam()
    o, col, bg = 0.6, [0.7, 0.3, 0.5], (0.2, 0.2, 0.2)
    sc = _single([0, 2.5, 0], [math.log(0.05)] * 3, [1, 0, 0, 0], _logit(o), col)
    w = [np.zeros((3, 33, 33))]
    w[0][:, 16, 16] = 1.0
    r = orc.render(sc, [cam], _opts(bg=bg), dL_dimages=w)
    o32 = 1 / (1 + math.exp(-float(np.float32(_logit(o)))))
    np.testing.assert_allclose(r["grads"]["sh_dc"][:, 0], [o32] * 3, rtol=1e-12)
    c32 = np.array(col, np.float32).astype(np.float64)
    exp = ((c32 - bg[0]).sum()) * o32 * (1 - o32)  # G = 1 at the centre
    assert r["grads"]["opacity_logits"][0] == pytest.approx(exp, rel=1e-12)
