"""FP64 oracle of the photometric part of the training loss (Eq. 7): test
infrastructure only, never called by the product path.

    L = (1 - lambda) L1 + lambda (1 - SSIM)                      (Eq. 7, first two terms)

per view, the batched loss being the mean over the views of a call.  The
paper leaves L1 and SSIM to 3DGS; the readings taken here:
  * L1 = mean over the view's 3 H W values of |x - y|;
  * SSIM = mean over the same values of the SSIM map of each colour plane,
    computed from Gaussian-weighted local moments: an 11 x 11 window, the
    outer product of a normalised 11-tap Gaussian of standard deviation 1.5
    (Sec. 3.2.5 describes the 11 x 11 kernel and its two 1-D factors),
    zero padding outside the image, C1 = 0.01^2, C2 = 0.03^2;
  * lambda = 0.2 unless given; d|t|/dt = sign(t), 0 at t = 0.

The gradient is written out from the moment form of the SSIM map:
    mu_x = w*x, mu_y = w*y, E_xx = w*(x x), E_yy = w*(y y), E_xy = w*(x y)
    S = (2 mu_x mu_y + C1)(2 (E_xy - mu_x mu_y) + C2)
        / ((mu_x^2 + mu_y^2 + C1)(E_xx - mu_x^2 + E_yy - mu_y^2 + C2))
    dS/dx(p) = sum_q w(q - p) [dS/dmu_x(q) + 2 x(p) dS/dE_xx(q) + y(p) dS/dE_xy(q)]
where * is the zero-padded correlation with the window (symmetric, so it is
its own adjoint).  The tests pin it against central finite differences and
against torch float64 autograd of an independent convolution.
"""
from __future__ import annotations

import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
LAMBDA = 0.2


def gaussian_1d(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """Normalised 1-D Gaussian taps centred on the middle tap."""
    k = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return g / g.sum()


def window_2d(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    g = gaussian_1d(size, sigma)
    return np.outer(g, g)


def filter2d(img: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Zero-padded 'same' correlation of an [H, W] plane with an odd square window."""
    img = np.asarray(img, np.float64)
    H, W = img.shape
    r = w.shape[0] // 2
    pad = np.zeros((H + 2 * r, W + 2 * r))
    pad[r:r + H, r:r + W] = img
    out = np.zeros((H, W))
    for dy in range(w.shape[0]):
        for dx in range(w.shape[1]):
            out += w[dy, dx] * pad[dy:dy + H, dx:dx + W]
    return out


def _moments(x, y, w):
    return filter2d(x, w), filter2d(y, w), filter2d(x * x, w), filter2d(y * y, w), filter2d(x * y, w)


def ssim_map(x: np.ndarray, y: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    """SSIM map of two [H, W] planes."""
    w = window_2d() if w is None else w
    mx, my, exx, eyy, exy = _moments(np.asarray(x, np.float64), np.asarray(y, np.float64), w)
    sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def view_loss(img: np.ndarray, tgt: np.ndarray, lam: float = LAMBDA) -> dict:
    """img, tgt: [3, H, W].  Returns the loss of one view and its two parts."""
    img = np.asarray(img, np.float64)
    tgt = np.asarray(tgt, np.float64)
    l1 = float(np.abs(img - tgt).mean())
    ssim = float(np.mean([ssim_map(img[c], tgt[c]).mean() for c in range(img.shape[0])]))
    return dict(loss=(1.0 - lam) * l1 + lam * (1.0 - ssim), l1=l1, ssim=ssim)


def view_loss_grad(img: np.ndarray, tgt: np.ndarray, lam: float = LAMBDA) -> np.ndarray:
    """dL/dimg of view_loss, [3, H, W]."""
    img = np.asarray(img, np.float64)
    tgt = np.asarray(tgt, np.float64)
    w = window_2d()
    n = img.size
    g = (1.0 - lam) * np.sign(img - tgt) / n
    for c in range(img.shape[0]):
        x, y = img[c], tgt[c]
        mx, my, exx, eyy, exy = _moments(x, y, w)
        sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
        n1, n2 = 2 * mx * my + C1, 2 * sxy + C2
        d1, d2 = mx * mx + my * my + C1, sxx + syy + C2
        s = n1 * n2 / (d1 * d2)
        ds_dmx = 2 * my * (n2 - n1) / (d1 * d2) - 2 * mx * s * (1.0 / d1 - 1.0 / d2)
        ds_dexx = -s / d2
        ds_dexy = 2 * n1 / (d1 * d2)
        dsdx = filter2d(ds_dmx, w) + 2 * x * filter2d(ds_dexx, w) + y * filter2d(ds_dexy, w)
        g[c] -= lam * dsdx / n
    return g


def batch_loss(images, targets, lam: float = LAMBDA) -> dict:
    """images, targets: lists of [3, H_v, W_v]; mean over views and per-view values."""
    per = [view_loss(i, t, lam) for i, t in zip(images, targets)]
    return dict(loss=float(np.mean([p["loss"] for p in per])), views=per)


def batch_loss_grad(images, targets, lam: float = LAMBDA):
    V = len(images)
    return [view_loss_grad(i, t, lam) / V for i, t in zip(images, targets)]
