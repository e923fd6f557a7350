"""FP64 oracle of the mask terms of the training loss (Eq. 7): test infrastructure only,
never called by the product path.

    lambda_m L_m + lambda_sh L_sh                                (Eq. 7, last two terms)

The paper takes both terms from the works it cites.  The readings taken here:
  * L_m  = mean over the n Gaussians of sigmoid(m_i), the soft volume mask of Eq. 3
    (the loss acts on the soft mask, not on its hard straight-through value);
  * L_sh = mean over the Gaussians of sum_l w_l sigmoid(m_i^l), bands l = 1..deg, with each
    band weighted by its number of coefficients (Sec. 3.2.3): w_l = (2l + 1) / sum_l' (2l' + 1);
  * lambda_m = lambda_sh = 0.05 (Sec. 4.2) unless given.
"""
from __future__ import annotations

import numpy as np

LAMBDA_M = 0.05
LAMBDA_SH = 0.05


def sigmoid(x):
    x = np.asarray(x, np.float64)
    return 1.0 / (1.0 + np.exp(-x))


def band_weights(deg: int) -> np.ndarray:
    c = np.array([2 * l + 1 for l in range(1, deg + 1)], np.float64)
    return c / c.sum() if deg > 0 else c


def mask_loss(mask_logits, sh_mask_logits, deg: int, lam_m: float = LAMBDA_M, lam_sh: float = LAMBDA_SH) -> dict:
    """mask_logits [n] or None; sh_mask_logits [3, n] (bands 1..3) or None."""
    lm = 0.0 if mask_logits is None else float(sigmoid(mask_logits).mean())
    lsh = 0.0
    if sh_mask_logits is not None and deg > 0:
        s = sigmoid(np.asarray(sh_mask_logits, np.float64)[:deg])
        lsh = float((band_weights(deg)[:, None] * s).sum(0).mean())
    return dict(loss=lam_m * lm + lam_sh * lsh, l_m=lm, l_sh=lsh)


def mask_loss_grad(mask_logits, sh_mask_logits, deg: int, lam_m: float = LAMBDA_M, lam_sh: float = LAMBDA_SH):
    """(d/d mask_logits [n] or None, d/d sh_mask_logits [3, n] or None); bands above deg get 0."""
    gm = gsh = None
    if mask_logits is not None:
        s = sigmoid(mask_logits)
        gm = lam_m * s * (1.0 - s) / s.size
    if sh_mask_logits is not None:
        x = np.asarray(sh_mask_logits, np.float64)
        gsh = np.zeros_like(x)
        if deg > 0:
            s = sigmoid(x[:deg])
            gsh[:deg] = lam_sh * band_weights(deg)[:, None] * s * (1.0 - s) / x.shape[1]
    return gm, gsh
