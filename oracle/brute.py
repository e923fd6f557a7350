"""Brute-force per-pixel renderer in torch float64 with autograd.

TEST INFRASTRUCTURE ONLY.  A second, independent statement of the same
function as oracle.cpp, for tiny scenes: no tiles, no lists, no hand-derived
derivatives.  Every pixel considers every Gaussian, ordered by
(single-precision depth, Gaussian index) -- the order the tile lists induce
on any one pixel -- and composites front to back (Eq. 2).  Gradients come
from torch autograd, so they check the oracle's own derivative code.

Follows: Eq. 1 (2D Gaussian from the EWA projection), the low-pass
Sigma' + sI (Sec. 3.2.4), Eq. 3 and Eq. 5 (hard masks with straight-through
gradients), Sec. 3.2.5 (diffuse colour separate from SH bands 1..3), Eq. 2.
"""
from __future__ import annotations

import math

import numpy as np
import torch

ALPHA_MAX = float(np.float32(0.99))
ALPHA_MIN = float(np.float32(1.0) / np.float32(255.0))
T_MIN = float(np.float32(1e-4))


def _t(x, grad=False):
    t = torch.tensor(np.asarray(x, np.float64), dtype=torch.float64)
    if grad:
        t.requires_grad_(True)
    return t


def params_of(scene, grad=True):
    """Torch float64 leaves for every parameter array of a scene."""
    return {k: _t(v, grad) for k, v in scene.arrays().items()}


def _ste(soft, eps):
    hard = (soft > eps).to(soft.dtype)
    return (hard - soft).detach() + soft


def sh_real(d):
    """Real SH basis, degree <= 3, at unit directions d [...,3] -> [...,16].

    Written from the spherical-harmonic polynomials
    r^l Y_lm = (normalisation) x (Legendre-type polynomial in x, y, z),
    with the Condon-Shortley sign (-1)^m kept on m > 0 and m < 0 terms."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    pi = math.pi
    out = [torch.full_like(x, 0.5 / math.sqrt(pi))]
    k1 = math.sqrt(3 / (4 * pi))
    out += [-k1 * y, k1 * z, -k1 * x]
    out += [0.5 * math.sqrt(15 / pi) * x * y,
            -0.5 * math.sqrt(15 / pi) * y * z,
            0.25 * math.sqrt(5 / pi) * (3 * z * z - 1.0),  # = 2z^2 - x^2 - y^2 on the unit sphere
            -0.5 * math.sqrt(15 / pi) * x * z,
            0.25 * math.sqrt(15 / pi) * (x * x - y * y)]
    out += [-0.25 * math.sqrt(35 / (2 * pi)) * y * (3 * x * x - y * y),
            0.5 * math.sqrt(105 / pi) * x * y * z,
            -0.25 * math.sqrt(21 / (2 * pi)) * y * (5 * z * z - 1.0),  # 4z^2 - x^2 - y^2 = 5z^2 - 1
            0.25 * math.sqrt(7 / pi) * z * (5 * z * z - 3.0),          # 2z^2 - 3x^2 - 3y^2 = 5z^2 - 3
            -0.25 * math.sqrt(21 / (2 * pi)) * x * (5 * z * z - 1.0),
            0.25 * math.sqrt(105 / pi) * z * (x * x - y * y),
            -0.25 * math.sqrt(35 / (2 * pi)) * x * (x * x - 3 * y * y)]
    return torch.stack(out, -1)


def _quat_to_rot(q):
    w, x, y, z = q.unbind(0)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 0),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 0),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 0)], 0)  # [3,3,N]


def project(p, scene, cam, opts):
    """Per-Gaussian screen values for one view (all tensors over N)."""
    R = _t(cam.R).reshape(3, 3)
    tv = _t(cam.t).reshape(3)
    mu = p["means"]
    n = mu.shape[1]
    keep = torch.ones(n, dtype=torch.bool)
    M = torch.ones(n, dtype=torch.float64)
    if "mask_logits" in p:
        soft = torch.sigmoid(p["mask_logits"])
        keep &= soft > scene.mask_eps
        M = _ste(soft, scene.mask_eps)
    tc = R @ mu + tv[:, None]                      # camera-space mean [3,N]
    keep &= tc[2] > opts.near_plane
    s = M[None, :] * torch.exp(p["log_scales"])    # masked scales
    q = p["quats"] / torch.linalg.norm(p["quats"], dim=0, keepdim=True)
    Rq = _quat_to_rot(q)                            # [3,3,N]
    RS = Rq * s[None, :, :]                         # columns scaled
    Sig = torch.einsum("ikn,jkn->ijn", RS, RS)      # [3,3,N]
    tz = tc[2]
    limx = opts.tan_clamp * 0.5 * cam.width / cam.fx
    limy = opts.tan_clamp * 0.5 * cam.height / cam.fy
    rx = torch.clamp(tc[0] / tz, -limx, limx)
    ry = torch.clamp(tc[1] / tz, -limy, limy)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([cam.fx / tz, zero, -cam.fx * rx / tz], 0),
                     torch.stack([zero, cam.fy / tz, -cam.fy * ry / tz], 0)], 0)  # [2,3,N]
    Tm = torch.einsum("ijn,jk->ikn", J, R)
    S2 = torch.einsum("ian,abn,jbn->ijn", Tm, Sig, Tm)
    lp = float(opts.lowpass)
    if getattr(opts, "lowpass_progressive", 0):   # Sec. 3.2.4: s = max(s0, H W / (9 pi N))
        lp = max(lp, cam.height * cam.width / (9.0 * math.pi * n))
    a = S2[0, 0] + lp
    b = S2[0, 1]
    c = S2[1, 1] + lp
    det = a * c - b * b
    keep &= det > 0
    A, B, Cc = c / det, -b / det, a / det
    mid = 0.5 * (a + c)
    lam = mid + torch.sqrt(torch.clamp(mid * mid - det, min=0.0))
    radius = torch.ceil(3.0 * torch.sqrt(lam)).detach()
    u = cam.fx * tc[0] / tz + cam.cx
    v = cam.fy * tc[1] / tz + cam.cy
    op = M * torch.sigmoid(p["opacity_logits"])
    # colour
    campos = -(R.T @ tv)
    d = mu - campos[:, None]
    dn = d / torch.linalg.norm(d, dim=0, keepdim=True)
    Y = sh_real(dn.T)                               # [N,16]
    rgb = p["sh_dc"].clone()                        # [3,N]
    deg = scene.sh_degree
    for l in range(1, deg + 1):
        Ml = torch.ones(n, dtype=torch.float64)
        if "sh_mask_logits" in p:
            Ml = _ste(torch.sigmoid(p["sh_mask_logits"][l - 1]), scene.sh_mask_eps)
        band = 0.0
        for k in range(l * l, (l + 1) * (l + 1)):
            band = band + Y[:, k][None, :] * p["sh_rest"][k - 1]
        rgb = rgb + Ml[None, :] * band
    rgb = torch.where(rgb < 0, torch.zeros_like(rgb), rgb)
    depth32 = torch.tensor(tz.detach().numpy().astype(np.float32).astype(np.float64))
    return dict(u=u, v=v, A=A, B=B, C=Cc, op=op, rgb=rgb, radius=radius, keep=keep.detach(),
                depth32=depth32)


def render_view(p, scene, cam, opts):
    """Image [3,H,W], T_final [H,W], the number of composited Gaussians per pixel and the
    number of pixels each Gaussian is composited at (its ray hits, Eq. 4)."""
    pr = project(p, scene, cam, opts)
    H, W = cam.height, cam.width
    ys, xs = torch.meshgrid(torch.arange(H, dtype=torch.float64) + 0.5,
                            torch.arange(W, dtype=torch.float64) + 0.5, indexing="ij")
    px, py = xs.reshape(-1), ys.reshape(-1)
    n = pr["u"].shape[0]
    order = np.lexsort((np.arange(n), pr["depth32"].numpy()))  # depth first, index breaks ties
    P = px.shape[0]
    T = torch.ones(P, dtype=torch.float64)
    Cimg = torch.zeros(3, P, dtype=torch.float64)
    alive = torch.ones(P, dtype=torch.bool)
    count = torch.zeros(P, dtype=torch.int64)
    hits = np.zeros(n, np.int64)
    for j in order:
        if not bool(pr["keep"][j]):
            continue
        dx = px - pr["u"][j]
        dy = py - pr["v"][j]
        r = pr["radius"][j]
        inside = (dx.detach().abs() <= r) & (dy.detach().abs() <= r)
        q = pr["A"][j] * dx * dx + 2 * pr["B"][j] * dx * dy + pr["C"][j] * dy * dy
        alpha = torch.clamp(pr["op"][j] * torch.exp(-0.5 * q), max=ALPHA_MAX)
        use = inside & alive & (alpha.detach() >= ALPHA_MIN)
        stop = use & (T.detach() * (1 - alpha.detach()) < T_MIN)
        alive = alive & ~stop
        use = use & ~stop
        a = torch.where(use, alpha, torch.zeros_like(alpha))
        Cimg = Cimg + pr["rgb"][:, j:j + 1] * (a * T)[None, :]
        T = T * (1 - a)
        count = count + use.long()
        hits[j] = int(use.sum())
    bg = torch.tensor(opts.bg, dtype=torch.float64)[:, None]
    img = Cimg + T[None, :] * bg
    return img.reshape(3, H, W), T.reshape(H, W), count.reshape(H, W), hits


def render(scene, cams, opts, weights=None, grad=True):
    """Images for all views; with `weights` (list of [3,H,W]) also the gradient of
    sum_v sum(weights_v * image_v) w.r.t. every raw parameter (float64 numpy)."""
    p = params_of(scene, grad=grad and weights is not None)
    imgs, Ts, counts, hits = [], [], [], []
    for cam in cams:
        im, T, c, h = render_view(p, scene, cam, opts)
        imgs.append(im)
        Ts.append(T)
        counts.append(c)
        hits.append(h)
    out = dict(images=[i.detach().numpy() for i in imgs], T_final=[t.detach().numpy() for t in Ts],
               counts=[c.numpy() for c in counts], hits=hits)
    if weights is not None:
        loss = sum((im * _t(w)).sum() for im, w in zip(imgs, weights))
        loss.backward()
        out["grads"] = {k: (v.grad.numpy() if v.grad is not None else np.zeros(v.shape)) for k, v in p.items()}
    return out
