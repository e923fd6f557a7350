"""Progressive training around the rasterizer (Sec. 3.2.4, Eq. 6, Sec. 4.2).

Three schedules coarsen the problem early in training:
  * scales: the low-pass s of Sigma' + sI follows the Gaussian count,
    s = max(0.3, HW / (9 pi N)) per view -- set `lowpass_progressive=1` in the
    rasterizer options and libgs evaluates it in every projection;
  * resolution: the targets start 8x smaller and grow back to full size;
  * blur: the targets are blurred with a Gaussian that starts at 9 x 9,
    sigma 2.4 and shrinks every 100 iterations, divided by the current
    downsampling factor when both are active.
The schedules are host arithmetic; blur and resize of the target images run
in libgs (gs_blur_views, gs_resize_views).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import torch

from . import gs


def lowpass_s(n: int, width: int, height: int, s0: float = 0.3) -> float:
    """The per-view low-pass of progressive scaling: max(s0, W H / (9 pi n))."""
    return max(float(s0), width * height / (9.0 * math.pi * n)) if n > 0 else float(s0)


def resolution(i: int, res_s: int, res_e: int, tau: int) -> int:
    """Eq. 6: the training resolution at iteration i, from res_s to res_e by iteration tau."""
    return min(int(math.floor(res_s + (res_e - res_s) * i / tau + 0.5)), res_e)


def downsample_factor(i: int, start: float = 8.0, until: int = 19500) -> float:
    """Downsampling factor at iteration i: from `start` to 1 with a logarithmic decay (its
    logarithm falls linearly) that ends at `until` (Sec. 4.2)."""
    if i >= until:
        return 1.0
    return float(start) ** (1.0 - max(i, 0) / until)


def blur_kernel(i: int, k0: int = 9, sigma0: float = 2.4, every: int = 100, until: int = 19500,
                downsample: float = 1.0) -> Optional[Tuple[int, float]]:
    """(ksize, sigma) of the target blur at iteration i, or None once it is off.  The kernel
    shrinks linearly with the training progress, updated every `every` iterations, and is
    divided by the current downsampling factor; ksize is the largest odd size not above
    k0 times the remaining fraction."""
    step = (max(i, 0) // every) * every
    left = 1.0 - step / until
    if left <= 0.0:
        return None
    sigma = sigma0 * left / downsample
    k = int(math.floor(k0 * left / downsample))
    k -= 1 - k % 2
    if k < 3 or sigma <= 0.0:
        return None
    return k, sigma


def scaled_cameras(cams: Sequence, factor: float) -> List:
    """Cameras of the same views at 1/factor of the resolution (focal lengths and principal
    points scaled with it, so the field of view is kept)."""
    out = []
    for c in cams:
        w = max(1, int(round(c.width / factor)))
        h = max(1, int(round(c.height / factor)))
        sx, sy = w / c.width, h / c.height
        out.append(dataclasses.replace(c, width=w, height=h, fx=c.fx * sx, fy=c.fy * sy, cx=c.cx * sx,
                                       cy=c.cy * sy))
    return out


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _numel(cams) -> int:
    return sum(3 * c.width * c.height for c in cams)


def blur(images: torch.Tensor, cams: Sequence, ksize: int, sigma: float,
         out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """ksize x ksize Gaussian blur of every view (views concatenated, [3][H][W] each)."""
    if images.dtype != torch.float32 or not images.is_contiguous() or images.numel() != _numel(cams):
        raise ValueError("images must be contiguous float32 holding the views' [3][H][W] planes")
    out = out if out is not None else torch.empty_like(images)
    ca = gs.cameras(cams)
    gs.check(gs.blur_views(gs.ptr(images), gs.ptr(out), ca, len(cams), ksize, sigma, _stream()), "gs_blur_views")
    return out


def resize(images: torch.Tensor, in_cams: Sequence, out_cams: Sequence,
           out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Area resampling of every view from in_cams' sizes to out_cams' sizes."""
    if images.dtype != torch.float32 or not images.is_contiguous() or images.numel() != _numel(in_cams):
        raise ValueError("images must be contiguous float32 holding the views' [3][H][W] planes")
    if len(in_cams) != len(out_cams):
        raise ValueError("one output size per view")
    out = out if out is not None else torch.empty(_numel(out_cams), dtype=torch.float32, device=images.device)
    gs.check(gs.resize_views(gs.ptr(images), gs.cameras(in_cams), gs.ptr(out), gs.cameras(out_cams), len(in_cams),
                             _stream()), "gs_resize_views")
    return out


class ProgressiveTargets:
    """Training targets of iteration i: the full-resolution views resized to the current
    downsampling factor, then blurred with the current kernel (both from the schedules above)."""

    def __init__(self, targets: torch.Tensor, cams: Sequence, start: float = 8.0, until: int = 19500,
                 k0: int = 9, sigma0: float = 2.4, every: int = 100):
        self.targets, self.cams = targets, list(cams)
        self.start, self.until, self.k0, self.sigma0, self.every = start, until, k0, sigma0, every

    def at(self, i: int):
        """(cameras, targets) for iteration i."""
        f = downsample_factor(i, self.start, self.until)
        cams = scaled_cameras(self.cams, f) if f > 1.0 else self.cams
        img = resize(self.targets, self.cams, cams) if f > 1.0 else self.targets
        kb = blur_kernel(i, self.k0, self.sigma0, self.every, self.until, downsample=f)
        if kb is not None:
            img = blur(img, cams, kb[0], kb[1])
        return cams, img
