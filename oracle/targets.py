"""FP64 oracle of the target-image side of progressive training (Sec. 3.2.4):
test infrastructure only, never called by the product path.

  * blur: the training images are blurred with a square Gaussian kernel that
    starts at 9 x 9, sigma 2.4 (Sec. 4.2) and shrinks during training.  Here a
    k x k kernel is the outer product of two normalised k-tap Gaussians of
    standard deviation sigma (separable), applied as a correlation with the
    image mirrored about its edge pixels (index -1 reads 1, W reads W - 2).
  * resize: the training images start 8x smaller (Sec. 4.2, Eq. 6).  Here an
    image is resampled to W' x H' by area averaging: output pixel x' averages
    the piecewise-constant input over [x' W / W', (x' + 1) W / W'), and
    likewise in y.  The overlap of input pixel x with that interval has the
    length max(0, min((x+1) W', (x'+1) W) - max(x W', x' W)) / W' (an integer
    over W'); divided by the interval's length W / W', the weight is that
    integer over W.

Views are [3, H, W] planes; the batched layout concatenates views.
"""
from __future__ import annotations

import numpy as np


def gaussian_taps(k: int, sigma: float) -> np.ndarray:
    """k (odd) normalised taps of a Gaussian of standard deviation sigma, centred."""
    if k < 1 or k % 2 == 0:
        raise ValueError("k must be odd and >= 1")
    t = np.arange(k, dtype=np.float64) - (k - 1) / 2.0
    g = np.exp(-(t * t) / (2.0 * float(sigma) ** 2))
    return g / g.sum()


def mirror(i: int, n: int) -> int:
    """Index i reflected into [0, n) about the edge pixels (period 2 (n - 1))."""
    if n == 1:
        return 0
    p = 2 * (n - 1)
    i %= p
    return i if i < n else p - i


def blur_plane(img: np.ndarray, k: int, sigma: float) -> np.ndarray:
    """Separable k x k Gaussian blur of one [H, W] plane, mirrored borders."""
    img = np.asarray(img, np.float64)
    H, W = img.shape
    g = gaussian_taps(k, sigma)
    r = (k - 1) // 2
    cols = np.array([[mirror(x + d, W) for d in range(-r, r + 1)] for x in range(W)])
    rows = np.array([[mirror(y + d, H) for d in range(-r, r + 1)] for y in range(H)])
    tmp = (img[:, cols] * g).sum(-1)            # horizontal pass: [H, W]
    return (tmp[rows, :] * g[None, :, None]).sum(1)  # vertical pass


def blur_views(images, k: int, sigma: float):
    return [np.stack([blur_plane(im[c], k, sigma) for c in range(im.shape[0])]) for im in images]


def area_weights(n_in: int, n_out: int) -> np.ndarray:
    """[n_out, n_in] matrix of the area-averaging weights along one axis."""
    w = np.zeros((n_out, n_in))
    for xo in range(n_out):
        for x in range(n_in):
            ov = min((x + 1) * n_out, (xo + 1) * n_in) - max(x * n_out, xo * n_in)
            if ov > 0:
                w[xo, x] = ov / n_in
    return w


def resize_plane(img: np.ndarray, w_out: int, h_out: int) -> np.ndarray:
    img = np.asarray(img, np.float64)
    H, W = img.shape
    return area_weights(H, h_out) @ img @ area_weights(W, w_out).T


def resize_views(images, sizes):
    """images: list of [3, H, W]; sizes: list of (W', H')."""
    return [np.stack([resize_plane(im[c], w, h) for c in range(im.shape[0])]) for im, (w, h) in zip(images, sizes)]
