"""L1 + D-SSIM photometric loss of Eq. 7 on rendered views (binding of gs_loss_l1_dssim).

The loss and its gradient run in the HIP kernels of libgs (loss.hip); this
module only owns the workspace and marshals arguments.
"""
from __future__ import annotations

from typing import Optional, Sequence, Tuple

import torch

from . import gs

LAMBDA_SSIM = 0.2


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class PhotometricLoss:
    """Loss over a fixed set of views (the image layout of the rasterizer: [3][H][W] per view, concatenated)."""

    def __init__(self, cams: Sequence, lambda_ssim: float = LAMBDA_SSIM, device: str = "cuda"):
        gs.load()
        self.cams = list(cams)
        self.V = len(self.cams)
        self.cams_arr = gs.cameras(self.cams)
        self.lambda_ssim = float(lambda_ssim)
        self.numel = sum(3 * int(c.width) * int(c.height) for c in self.cams)
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.ws_bytes = gs.loss_workspace_size(self.cams_arr, self.V)
        if self.ws_bytes == 0:
            raise gs.GsError("invalid views for gs_loss_workspace_size")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.loss = torch.zeros(self.V + 1, dtype=torch.float32, device=dev)

    def __call__(self, image: torch.Tensor, target: torch.Tensor, grad: bool = True,
                 out: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
        """Returns (loss [V + 1]: per-view losses then their mean, dL/dimage or None)."""
        for t in (image, target):
            if t.device != self.device or t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != self.numel:
                raise ValueError("image and target must be contiguous float32 tensors in the views' layout")
        dL = None
        if grad:
            dL = out if out is not None else torch.empty_like(image)
        gs.check(gs.loss_l1_dssim(gs.ptr(image), gs.ptr(target), self.cams_arr, self.V, self.lambda_ssim,
                                  gs.ptr(self.loss), gs.ptr(dL), gs.ptr(self.ws), self.ws_bytes, _stream()),
                 "gs_loss_l1_dssim")
        return self.loss, dL
