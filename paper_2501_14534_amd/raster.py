"""Device buffers and call sequences around libgs; torch.autograd wrapper; graph-captured step.

`Rasterizer` owns the buffers of one (Gaussian count, view set, options)
configuration and issues the four C-ABI calls on the current torch stream.
PyTorch provides device memory and streams only; every step of the path runs
in libgs kernels.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import gs

PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh_dc", "sh_rest", "mask_logits", "sh_mask_logits")


def to_device(scene, device="cuda") -> Dict[str, torch.Tensor]:
    """Parameter arrays of a scenes.Scene as contiguous float32 device tensors."""
    return {k: torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(device) for k, v in scene.arrays().items()}


class Grads(dict):
    """Gradient tensors by parameter name; `flat` is the buffer they are views of."""
    flat: Optional[torch.Tensor] = None

    def zero_(self) -> None:
        if self.flat is not None:
            self.flat.zero_()
        else:
            for g in self.values():
                g.zero_()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Rasterizer:
    """Forward/backward rasterization of n Gaussians into a fixed set of views.

    capacity: number of (record, tile) pairs the sort buffers hold.  When a
    forward finds more pairs (device status word), `forward(check=True)`
    grows the buffers and re-runs the binning; graph-captured callers pass
    check=False and call `overflowed()` after the step.
    """

    def __init__(self, n: int, sh_degree: int, cams: Sequence, opts, *, mask_eps: float = 0.5,
                 sh_mask_eps: float = 0.5, capacity: Optional[int] = None, device: str = "cuda",
                 schedule: bool = True, keep_keys: bool = False):
        gs.load()
        if len(cams) < 1 or len(cams) > gs.MAX_VIEWS:
            raise ValueError(f"1..{gs.MAX_VIEWS} views per call")
        self.n, self.deg, self.V = int(n), int(sh_degree), len(cams)
        self.cams = list(cams)
        self.opts = opts
        self.mask_eps, self.sh_mask_eps = mask_eps, sh_mask_eps
        self.keep_keys = keep_keys  # the 64-bit sort keys are written only when asked for (tests)
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.cams_arr = gs.cameras(self.cams)
        self.opts_s = gs.options(opts)
        self.total_tiles, self.total_pixels = gs.view_sizes(self.cams_arr, self.V, self.opts_s)
        dev = self.device
        nrec = self.V * self.n
        self.splats = torch.zeros(max(nrec, 1) * gs.SPLAT_FLOATS, dtype=torch.float32, device=dev)
        self.tiles_touched = torch.zeros(max(nrec, 1), dtype=torch.int32, device=dev)
        self.offsets = torch.zeros(max(nrec, 1), dtype=torch.int32, device=dev)
        self.ranges = torch.zeros(max(self.total_tiles, 1) * 2, dtype=torch.int32, device=dev)
        # heaviest-first tile schedule written by gs_bin_sort (None: tile-id order)
        self.order = torch.zeros(max(self.total_tiles, 1), dtype=torch.int32, device=dev) if schedule else None
        self.count = torch.zeros(1, dtype=torch.int32, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.image = torch.zeros(3 * self.total_pixels, dtype=torch.float32, device=dev)
        self.T_final = torch.zeros(self.total_pixels, dtype=torch.float32, device=dev)
        self.last = torch.zeros(self.total_pixels, dtype=torch.int32, device=dev)
        self.proj = gs.GsProjected(gs.ptr(self.splats), gs.ptr(self.tiles_touched))
        # bumped by every projection: the records, lists and pixel states a backward
        # reads belong to the forward of this generation only
        self.generation = 0
        self.capacity = 0
        self.set_capacity(capacity if capacity is not None else max(1 << 16, 8 * nrec))

    # -- buffers ---------------------------------------------------------------------------------
    def set_capacity(self, capacity: int) -> None:
        capacity = int(min(max(capacity, 1), (1 << 32) - 1))
        self.capacity = capacity
        self.keys = torch.zeros(capacity, dtype=torch.int64, device=self.device) if self.keep_keys else None
        self.ids = torch.zeros(capacity, dtype=torch.int32, device=self.device)
        self.pair_index = torch.zeros(capacity, dtype=torch.int32, device=self.device)
        self.ws_bytes = gs.workspace_size(self.n, self.cams_arr, self.V, self.opts_s, capacity)
        if self.ws_bytes == 0:
            raise gs.GsError("invalid configuration for gs_workspace_size")
        self.ws = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.bins = gs.GsBinning(gs.ptr(self.keys), gs.ptr(self.ids), gs.ptr(self.pair_index), gs.ptr(self.offsets),
                                 gs.ptr(self.ranges), gs.ptr(self.order), capacity, gs.ptr(self.count),
                                 gs.ptr(self.status))

    def gaussians(self, params: Dict[str, torch.Tensor]) -> gs.GsGaussians:
        for k, t in params.items():
            if t is None:
                continue
            if t.device != self.device or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError(f"{k}: expected a contiguous float32 tensor on {self.device}")
        return gs.gaussians(params, self.n, self.deg, self.mask_eps, self.sh_mask_eps)

    # -- calls -----------------------------------------------------------------------------------
    def project(self, params) -> None:
        g = self.gaussians(params)
        self.generation += 1
        gs.check(gs.project(g, self.cams_arr, self.V, self.opts_s, self.proj, _stream()), "gs_project")

    def bin_sort(self) -> None:
        gs.check(gs.bin_sort(self.proj, self.cams_arr, self.V, self.n, self.opts_s, self.bins, gs.ptr(self.ws),
                             self.ws_bytes, _stream()), "gs_bin_sort")

    def render_fwd(self) -> None:
        gs.check(gs.render_fwd(self.proj, self.bins, self.cams_arr, self.V, self.n, self.opts_s, gs.ptr(self.image),
                               gs.ptr(self.T_final), gs.ptr(self.last), gs.ptr(self.ws), self.ws_bytes, _stream()),
                 "gs_render_fwd")

    def render_bwd(self, params, dL_dimage: torch.Tensor, grads: Dict[str, torch.Tensor],
                   mean2d: Optional[torch.Tensor] = None, assign: bool = False) -> None:
        """Gradients into `grads`: added, or with assign=True written (no zeroing needed)."""
        g = self.gaussians(params)
        if dL_dimage.numel() != self.image.numel() or not dL_dimage.is_contiguous():
            raise ValueError("dL_dimage must be contiguous and shaped like the image")
        gr = gs.GsGrads(*[gs.ptr(grads.get(k)) for k in PARAM_NAMES], gs.ptr(mean2d), int(assign))
        gs.check(gs.render_bwd(g, self.cams_arr, self.V, self.opts_s, self.proj, self.bins, gs.ptr(self.T_final),
                               gs.ptr(self.last), gs.ptr(dL_dimage), gr, gs.ptr(self.ws), self.ws_bytes, _stream()),
                 "gs_render_bwd")

    def render_fwd_bwd_l2(self, params, target: torch.Tensor, views: int, grads: Dict[str, torch.Tensor],
                          dL_out: Optional[torch.Tensor] = None, assign: bool = False) -> None:
        """Compositing forward, mean-squared-error gradient and backward in one launch of the walks
        (gs_render_fwd_bwd_l2): the image and the gradients of render_fwd, l2_loss_grad and
        render_bwd, bit for bit; dL_out, if given, receives dL/dimage."""
        g = self.gaussians(params)
        if target.numel() != self.image.numel() or not target.is_contiguous():
            raise ValueError("target must be contiguous and shaped like the image")
        if dL_out is not None and (dL_out.numel() != self.image.numel() or not dL_out.is_contiguous()):
            raise ValueError("dL_out must be contiguous and shaped like the image")
        gr = gs.GsGrads(*[gs.ptr(grads.get(k)) for k in PARAM_NAMES], None, int(assign))
        gs.check(gs.render_fwd_bwd_l2(g, self.cams_arr, self.V, self.opts_s, self.proj, self.bins, gs.ptr(target),
                                      int(views), gs.ptr(self.image), gs.ptr(self.T_final), gs.ptr(self.last),
                                      gs.ptr(dL_out), gr, gs.ptr(self.ws), self.ws_bytes, _stream()),
                 "gs_render_fwd_bwd_l2")

    def blend_bwd(self, dL_dimage: torch.Tensor, grad_pair: torch.Tensor) -> None:
        """Back-to-front walk only: writes the per-pair splat gradients [capacity, 9] (emission order)."""
        if grad_pair.numel() < self.capacity * gs.GRAD_FLOATS:
            raise ValueError("grad_pair must hold capacity x 9 floats")
        gs.check(gs.blend_bwd(self.cams_arr, self.V, self.n, self.opts_s, self.proj, self.bins, gs.ptr(self.T_final),
                              gs.ptr(self.last), gs.ptr(dL_dimage), gs.ptr(grad_pair), gs.ptr(self.ws),
                              self.ws_bytes, _stream()), "gs_blend_bwd")

    def project_bwd(self, params, grad_pair: torch.Tensor, grads: Dict[str, torch.Tensor], mean2d=None,
                    assign: bool = False) -> None:
        g = self.gaussians(params)
        gr = gs.GsGrads(*[gs.ptr(grads.get(k)) for k in PARAM_NAMES], gs.ptr(mean2d), int(assign))
        gs.check(gs.project_bwd(g, self.cams_arr, self.V, self.opts_s, self.proj, self.bins, gs.ptr(grad_pair), gr,
                                gs.ptr(self.ws), self.ws_bytes, _stream()), "gs_project_bwd")

    def count_hits(self, hits: torch.Tensor, bins: Optional[gs.GsBinning] = None) -> None:
        """Adds the ray hits of Eq. 4 over the current lists (last bin_sort) into hits [n] (int32
        tensor holding uint32 counts).  `bins` may replace the lists (same buffers, other ranges)."""
        if hits.numel() < self.n or hits.dtype != torch.int32 or not hits.is_contiguous():
            raise ValueError("hits must be a contiguous int32 tensor of n counters")
        gs.check(gs.count_hits(self.proj, bins if bins is not None else self.bins, self.cams_arr, self.V, self.n,
                               self.opts_s, gs.ptr(hits), _stream()), "gs_count_hits")

    def accumulate_hits(self, params, hits: torch.Tensor) -> None:
        """project -> bin/sort (grown on overflow) -> count: this view set's hits added into `hits`."""
        self.project(params)
        self.bin_sort()
        if self.overflowed():
            self.set_capacity(int(self.pairs() * 1.25) + 1024)
            self.bin_sort()
            assert not self.overflowed()
        self.count_hits(hits)

    def overflowed(self) -> bool:
        return bool(self.status.item())

    def pairs(self) -> int:
        return int(self.count.item()) & 0xFFFFFFFF

    def forward(self, params, check: bool = True) -> torch.Tensor:
        """project -> bin/sort -> composite; returns the flat image buffer (views concatenated)."""
        self.project(params)
        self.bin_sort()
        if check and self.overflowed():
            self.set_capacity(int(self.pairs() * 1.25) + 1024)
            self.bin_sort()
            assert not self.overflowed()
        self.render_fwd()
        return self.image

    def backward(self, params, dL_dimage, grads, mean2d=None) -> None:
        self.render_bwd(params, dL_dimage, grads, mean2d)

    # -- views of the outputs --------------------------------------------------------------------
    def split(self, flat: torch.Tensor, channels: int) -> List[torch.Tensor]:
        out, off = [], 0
        for c in self.cams:
            k = channels * c.width * c.height
            shape = (channels, c.height, c.width) if channels > 1 else (c.height, c.width)
            out.append(flat[off:off + k].view(shape))
            off += k
        return out

    def images(self) -> List[torch.Tensor]:
        return self.split(self.image, 3)

    def splat_records(self) -> torch.Tensor:
        return self.splats[: self.V * self.n * gs.SPLAT_FLOATS].view(self.V * self.n, gs.SPLAT_FLOATS)

    def grad_pairs(self, dL_dimage: torch.Tensor) -> torch.Tensor:
        """Per-pair splat gradients [K, 9] (emission order) of the current lists for dL_dimage, zero
        for the pairs the walk does not reach (for inspection: a separate backward walk)."""
        gp = torch.zeros(max(self.capacity, 1) * gs.GRAD_FLOATS, dtype=torch.float32, device=self.device)
        self.blend_bwd(dL_dimage, gp)
        return gp[: self.pairs() * gs.GRAD_FLOATS].view(-1, gs.GRAD_FLOATS)

    def grad_records(self, dL_dimage: torch.Tensor) -> torch.Tensor:
        """Per-record sums of the pair gradients for dL_dimage [V*n, 9] (float64, for inspection)."""
        nrec = self.V * self.n
        gp = self.grad_pairs(dL_dimage).double()
        tt = self.tiles_touched[:nrec].long()
        owner = torch.repeat_interleave(torch.arange(nrec, device=gp.device), tt)
        out = torch.zeros(nrec, gs.GRAD_FLOATS, dtype=torch.float64, device=gp.device)
        out.index_add_(0, owner, gp[: owner.numel()])
        return out

    def zero_grads(self, params) -> Dict[str, torch.Tensor]:
        """Zeroed gradient tensors shaped like params, views of one flat float32 buffer
        (each starting on a 256-byte boundary), so that `.flat.zero_()` of the result
        clears them all in one launch."""
        items = [(k, v) for k, v in params.items() if v is not None]
        offs, total = [], 0
        for _, v in items:
            offs.append(total)
            total += (v.numel() + 63) // 64 * 64
        dev = items[0][1].device if items else self.device
        flat = torch.zeros(max(total, 1), dtype=torch.float32, device=dev)
        out = Grads({k: flat[o:o + v.numel()].view(v.shape) for (k, v), o in zip(items, offs)})
        out.flat = flat
        return out


def significance(params: Dict[str, torch.Tensor], hits: torch.Tensor, volume_quantile: float = 0.9,
                 mask_eps: float = 0.5, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Significance score of Eq. 4 from summed ray hits: hits x o' x min(volume / v_q, 1) [n]."""
    n = int(params["log_scales"].shape[-1])
    g = gs.gaussians(params, n, 0, mask_eps, 0.5)
    score = out if out is not None else torch.empty(n, dtype=torch.float32, device=hits.device)
    ws_bytes = gs.significance_workspace_size()
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=hits.device)
    gs.check(gs.significance(g, gs.ptr(hits), volume_quantile, gs.ptr(score), gs.ptr(ws), ws_bytes, _stream()),
             "gs_significance")
    return score


def significance_scores(params: Dict[str, torch.Tensor], sh_degree: int, cams: Sequence, opts,
                        views_per_call: int = 8, volume_quantile: float = 0.9, mask_eps: float = 0.5,
                        sh_mask_eps: float = 0.5) -> Dict[str, torch.Tensor]:
    """Eq. 4 over a set of (training) views: ray hits summed over batches of views, then the score."""
    n = int(params["means"].shape[-1])
    hits = torch.zeros(n, dtype=torch.int32, device=params["means"].device)
    for k in range(0, len(cams), views_per_call):
        r = Rasterizer(n, sh_degree, cams[k:k + views_per_call], opts, mask_eps=mask_eps, sh_mask_eps=sh_mask_eps)
        r.accumulate_hits(params, hits)
    return dict(hits=hits, score=significance(params, hits, volume_quantile, mask_eps))


class RasterizeFn(torch.autograd.Function):
    """image = rasterize(params); backward through gs_render_bwd.

    The Rasterizer keeps one forward's state (records, lists, T_final,
    last_contrib, pixel states) until its next projection.  The backward of an
    image whose Rasterizer has projected again since raises instead of
    returning another forward's gradients: use one Rasterizer per forward in
    flight.  Gradients are written (assign mode) into fresh tensors."""

    @staticmethod
    def forward(ctx, rast: Rasterizer, names, *tensors):
        params = dict(zip(names, tensors))
        img = rast.forward(params).clone()
        ctx.rast = rast
        ctx.generation = rast.generation
        ctx.names = names
        ctx.save_for_backward(*tensors)
        return img

    @staticmethod
    def backward(ctx, dL):
        rast = ctx.rast
        if rast.generation != ctx.generation:
            raise RuntimeError("rasterize: the Rasterizer has run another forward since this image was rendered, "
                               "so this image's backward state is gone; use one Rasterizer per forward in flight")
        tensors = ctx.saved_tensors
        params = dict(zip(ctx.names, tensors))
        # every gradient the call computes is written; at SH degree 0 the band masks get none
        grads = {k: (torch.zeros_like(v) if rast.deg == 0 and k == "sh_mask_logits" else torch.empty_like(v))
                 for k, v in params.items()}
        rast.render_bwd(params, dL.contiguous(), grads, assign=True)
        return (None, None, *[grads[k] for k in ctx.names])


def rasterize(rast: Rasterizer, params: Dict[str, torch.Tensor]) -> torch.Tensor:
    names = tuple(k for k in PARAM_NAMES if params.get(k) is not None)
    return RasterizeFn.apply(rast, names, *[params[k] for k in names])


def l2_loss_grad(rast: "Rasterizer", image: torch.Tensor, target: torch.Tensor, views: int,
                 out: torch.Tensor) -> None:
    """dL/dimage of L = mean over `views` views of mean over 3HW of (image - target)^2, written into
    `out` by gs_l2_grad (one elementwise pass)."""
    if target.numel() != image.numel() or out.numel() != image.numel():
        raise ValueError("image, target and out must have the same size")
    gs.check(gs.l2_grad(gs.ptr(image), gs.ptr(target), rast.cams_arr, rast.V, int(views), gs.ptr(out), _stream()),
             "gs_l2_grad")


class Step:
    """One fwd+bwd step of a Rasterizer (project, bin/sort, composite, loss
    gradient, backward), run eagerly or replayed from a captured HIP graph.

    loss: "l2" (mean over views of the mean squared error; the benchmark's
    loss) or "l1_dssim" (the photometric terms of Eq. 7, gs_loss_l1_dssim).
    mask_loss: (lambda_m, lambda_sh) adds the mask terms of Eq. 7
    (gs_mask_loss), or None.  sh_rest_every: k > 1 computes the SH bands 1..3
    gradients only on every k-th step (the others skip writing them), the
    sparse SH update the paper adopts (Sec. 3.2.5); two graphs are captured and
    replayed in turn.  fused (loss "l2" only): the forward walk, the loss
    gradient and the backward walk run as one launch (gs_render_fwd_bwd_l2),
    with the same results as the three separate calls (slower on the
    benchmark workloads, so off by default).

    The binning capacity is fixed while a graph exists; `run()` reads the
    device status after the step and, on overflow, grows the buffers,
    re-captures and runs again."""

    def __init__(self, rast: Rasterizer, params, target_flat: torch.Tensor, graph: bool = True,
                 loss_views: Optional[int] = None, loss: str = "l2", mask_loss=None, sh_rest_every: int = 1,
                 fused: bool = False):
        self.rast = rast
        self.params = params
        self.target = target_flat
        self.dL = torch.zeros_like(rast.image)
        self.grads = rast.zero_grads(params)
        self.graph_enabled = graph
        self.graphs = {}
        self.pix = [c.width * c.height for c in rast.cams]
        # number of views the loss averages over (a per-view step of a batch uses the batch's count)
        self.loss_views = rast.V if loss_views is None else int(loss_views)
        if loss not in ("l2", "l1_dssim"):
            raise ValueError(loss)
        self.loss_kind = loss
        # loss "l2": the compositing walks of the step in one launch (gs_render_fwd_bwd_l2)
        self.fused = bool(fused)
        self.ploss = None
        if loss == "l1_dssim":
            from .photometric import PhotometricLoss
            if self.loss_views != rast.V:
                raise ValueError("the L1 + D-SSIM step averages over the rasterizer's own views")
            self.ploss = PhotometricLoss(rast.cams)
        self.mask_loss = mask_loss
        self.mask_value = torch.zeros(1, dtype=torch.float32, device=rast.device)
        self.mask_ws = None
        if mask_loss is not None:
            b = gs.mask_loss_workspace_size(rast.n)
            self.mask_ws = torch.zeros(max(b, 1), dtype=torch.uint8, device=rast.device)
        self.sh_rest_every = max(1, int(sh_rest_every))
        self.step_index = 0
        self.carries_sh_rest = True

    @property
    def graph(self):
        return self.graphs.get(True)

    @graph.setter
    def graph(self, g):
        if g is None:
            self.graphs = {}
        else:
            self.graphs[True] = g

    def _body(self, with_sh_rest: bool = True):
        r = self.rast
        r.project(self.params)
        r.bin_sort()
        # the gradients are written, not added: only the ones this step does not write are
        # cleared (the SH-rest gradient on sparse steps; the SH gradients at degree 0)
        grads = self.grads
        if not with_sh_rest:
            grads = {k: v for k, v in self.grads.items() if k != "sh_rest"}
        for k in self.grads:
            if (k == "sh_rest" and not with_sh_rest) or (r.deg == 0 and k in ("sh_rest", "sh_mask_logits")):
                self.grads[k].zero_()
        if self.ploss is None and self.fused:
            # mean squared error: forward, loss gradient and backward walks in one launch
            r.render_fwd_bwd_l2(self.params, self.target, self.loss_views, grads, dL_out=self.dL, assign=True)
        else:
            r.render_fwd()
            if self.ploss is not None:
                self.ploss(r.image, self.target, out=self.dL)
            else:
                l2_loss_grad(r, r.image, self.target, self.loss_views, self.dL)
            r.render_bwd(self.params, self.dL, grads, assign=True)
        if self.mask_loss is not None:
            g = r.gaussians(self.params)
            gr = gs.GsGrads(*[gs.ptr(grads.get(k)) for k in PARAM_NAMES], None)
            gs.check(gs.mask_loss(g, self.mask_loss[0], self.mask_loss[1], gs.ptr(self.mask_value), gr,
                                  gs.ptr(self.mask_ws), self.mask_ws.numel(), _stream()), "gs_mask_loss")

    def capture(self, with_sh_rest: bool = True):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self._body(with_sh_rest)  # warm-up on the side stream before capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._body(with_sh_rest)
        self.graphs[with_sh_rest] = g

    def launch(self, with_sh_rest: Optional[bool] = None):
        """Enqueue one step (no host synchronisation).  with_sh_rest None: the schedule decides
        (every sh_rest_every-th step carries the SH-rest gradient) and the step counts;
        True/False repeats a step of that kind without counting it (a retry).  Afterwards
        `carries_sh_rest` says whether this step wrote the SH-rest gradient: on the other
        steps the caller leaves that parameter group out of its optimiser update (the
        gradient array then holds zeros, which would still move an Adam state)."""
        if with_sh_rest is None:
            with_sh_rest = self.step_index % self.sh_rest_every == 0
            self.step_index += 1
        self.carries_sh_rest = bool(with_sh_rest)
        if self.graph_enabled:
            if with_sh_rest not in self.graphs:
                self.capture(with_sh_rest)
            self.graphs[with_sh_rest].replay()
        else:
            self._body(with_sh_rest)

    def run(self, headroom: float = 1.25):
        """One step with the capacity check (synchronises): grows the binning
        buffers on overflow and shrinks them when they exceed twice the need,
        re-capturing the graph in both cases."""
        self.launch()
        need = self.rast.pairs()
        if self.rast.overflowed() or self.rast.capacity > 2 * headroom * need + (1 << 20):
            self.rast.set_capacity(int(need * headroom) + 1024)
            self.graph = None
            self.launch(self.carries_sh_rest)  # the same step again: the schedule does not advance
            assert not self.rast.overflowed()
