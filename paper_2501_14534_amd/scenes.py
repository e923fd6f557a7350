"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws numbers: Gaussian parameters, camera poses and target
images.  It holds none of the rasterizer's arithmetic, so both the HIP path and
the FP64 oracle can consume what it returns without sharing any of the method.

The paper trains on Mip-NeRF 360, Tanks&Temples and Deep Blending (Sec. 4.1),
which are not available here; the five workloads below stand in for them with
Gaussian counts spanning the paper's range (Tables 1-3: a few hundred thousand
to six million Gaussians) and the view resolutions of the benchmark configs,
including the mixed resolutions produced by progressive-resolution training
(Sec. 3.2.4, Eq. 6).

Conventions (all arrays float32, structure-of-arrays with the Gaussian index
last):
  means [3,N], log_scales [3,N], quats [4,N] (w,x,y,z), opacity_logits [N],
  sh_dc [3,N] (the diffuse colour, band 0), sh_rest [(K-1),3,N] with
  K=(deg+1)^2 (bands 1..deg), mask_logits [N] (per-Gaussian volume mask,
  Sec. 3.2.1), sh_mask_logits [3,N] (bands 1..3, Sec. 3.2.3).
Cameras: world->camera rotation R (rows: right, down, forward), translation t,
pinhole intrinsics fx, fy, cx, cy, and the image size.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

F32 = np.float32


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh_dc: np.ndarray
    sh_rest: Optional[np.ndarray]
    mask_logits: Optional[np.ndarray]
    sh_mask_logits: Optional[np.ndarray]
    sh_degree: int
    mask_eps: float = 0.5
    sh_mask_eps: float = 0.5

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def arrays(self):
        """Name -> array for every parameter tensor that is present."""
        out = {
            "means": self.means,
            "log_scales": self.log_scales,
            "quats": self.quats,
            "opacity_logits": self.opacity_logits,
            "sh_dc": self.sh_dc,
        }
        if self.sh_rest is not None:
            out["sh_rest"] = self.sh_rest
        if self.mask_logits is not None:
            out["mask_logits"] = self.mask_logits
        if self.sh_mask_logits is not None:
            out["sh_mask_logits"] = self.sh_mask_logits
        return out

    def copy(self) -> "Scene":
        kw = {}
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            kw[f.name] = v.copy() if isinstance(v, np.ndarray) else v
        return Scene(**kw)

    def subset(self, idx) -> "Scene":
        kw = {}
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            kw[f.name] = np.ascontiguousarray(v[..., idx]) if isinstance(v, np.ndarray) else v
        return Scene(**kw)


@dataclasses.dataclass
class Camera:
    R: np.ndarray  # float32 [3,3] world->camera
    t: np.ndarray  # float32 [3]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def pixels(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class Opts:
    near_plane: float = 0.2
    tan_clamp: float = 1.3
    lowpass: float = 0.3
    bg: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    tile_w: int = 16
    tile_h: int = 16
    batch_depth: int = 128
    pixels_per_thread: int = 1
    subtile_cull: int = 1
    bwd_chunk: int = 512  # list entries per backward work item (0: one per tile)
    fwd_chunk: int = 0     # list entries per forward work item (0: one per tile)
    lowpass_progressive: int = 0  # 1: per view s = max(lowpass, H W / (9 pi N)) (Sec. 3.2.4)


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    cams: List[Camera]
    opts: Opts
    targets: List[np.ndarray]  # float32 [3,H,W] per view

    @property
    def pixels(self) -> int:
        return sum(c.pixels for c in self.cams)


def _f(x) -> float:
    """Round to the nearest float32 and return it as a Python float."""
    return float(F32(x))


def look_at(pos, target, up=(0.0, 0.0, 1.0)) -> Tuple[np.ndarray, np.ndarray]:
    """World->camera (R, t) for a camera at `pos` looking at `target`.

    Camera axes: x right, y down, z forward.  Computed in float64 and rounded
    to float32 once; both consumers read the same rounded values.
    """
    pos = np.asarray(pos, np.float64)
    f = np.asarray(target, np.float64) - pos
    f /= np.linalg.norm(f)
    up = np.asarray(up, np.float64)
    if abs(float(np.dot(f, up))) > 0.999:
        up = np.array([0.0, 1.0, 0.0])
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f], 0)
    t = -R @ pos
    return R.astype(F32), t.astype(F32)


def make_camera(pos, target, width, height, f, up=(0.0, 0.0, 1.0), cx=None, cy=None) -> Camera:
    R, t = look_at(pos, target, up)
    return Camera(R=R, t=t, fx=_f(f), fy=_f(f),
                  cx=_f(width / 2.0 if cx is None else cx),
                  cy=_f(height / 2.0 if cy is None else cy),
                  width=int(width), height=int(height))


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q.astype(F32)


def _colour(rng, n, deg):
    dc = rng.normal(0.5, 0.2, (3, n)).astype(F32)
    rest = None
    if deg > 0:
        k = (deg + 1) ** 2 - 1
        rest = rng.normal(0.0, 0.05, (k, 3, n)).astype(F32)
    return dc, rest


def random_scene(rng, n, *, means, log_scale=(-3.5, 0.4), opacity=(0.0, 1.0), deg=0,
                 masks=False, band_masks=False, mask_eps=0.5, sh_mask_eps=0.5,
                 unit_quats=True) -> Scene:
    """Draw a scene of n Gaussians; `means` is a [3,n] array already drawn."""
    log_scales = rng.normal(log_scale[0], log_scale[1], (3, n)).astype(F32)
    quats = _unit_quats(rng, n) if unit_quats else rng.standard_normal((4, n)).astype(F32)
    opac = rng.normal(opacity[0], opacity[1], n).astype(F32)
    dc, rest = _colour(rng, n, deg)
    mask = rng.standard_normal(n).astype(F32) if masks else None
    bmask = rng.standard_normal((3, n)).astype(F32) if (band_masks and deg > 0) else None
    return Scene(np.ascontiguousarray(means, dtype=F32), log_scales, quats, opac, dc, rest,
                 mask, bmask, deg, mask_eps, sh_mask_eps)


def _targets(rng, cams):
    return [rng.random((3, c.height, c.width), dtype=np.float32) for c in cams]


def _shell(rng, n, r0=0.6, r1=1.0):
    d = rng.standard_normal((3, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    return d * rng.uniform(r0, r1, n)


def _box_normal(rng, n, sd, half):
    """N(0, diag(sd^2)) redrawn until every point lies in the box |x_i| <= half_i."""
    sd = np.asarray(sd, np.float64)[:, None]
    half = np.asarray(half, np.float64)[:, None]
    out = rng.standard_normal((3, n)) * sd
    bad = np.any(np.abs(out) > half, axis=0)
    while bad.any():
        k = int(bad.sum())
        out[:, bad] = rng.standard_normal((3, k)) * sd
        bad = np.any(np.abs(out) > half, axis=0)
    return out


def config(k: int, n: Optional[int] = None, seed: Optional[int] = None) -> Workload:
    """The five benchmark workloads (k = 1..5), seeded with k unless `seed` is given.

    `n` overrides the Gaussian count (same distributions) for scaled-down runs.
    """
    rng = np.random.default_rng(k if seed is None else seed)
    opts = Opts()
    if k == 1:
        n = 2000 if n is None else n
        means = rng.uniform(-1.0, 1.0, (3, n))
        scene = random_scene(rng, n, means=means, log_scale=(-3.5, 0.4), opacity=(0.0, 1.0), deg=0)
        cams = [make_camera((0.0, -4.0, 0.0), (0, 0, 0), 128, 128, 128.0)]
        name = "single-view 2K Gaussians, SH0, 128x128"
    elif k == 2:
        n = 200_000 if n is None else n
        means = _shell(rng, n)
        scene = random_scene(rng, n, means=means, log_scale=(-4.5, 0.5), opacity=(0.0, 1.5), deg=3)
        cams = [make_camera((0.0, -4.0, 0.0), (0, 0, 0), 800, 800, 1111.0)]
        name = "single-view 200K Gaussians, SH3, 800x800"
    elif k == 3:
        n = 1_000_000 if n is None else n
        means = _box_normal(rng, n, (5.0, 5.0, 2.5), (10.0, 10.0, 5.0))
        scene = random_scene(rng, n, means=means, log_scale=(-3.8, 0.7), opacity=(0.0, 1.0), deg=3,
                             masks=True, band_masks=True)
        cams = [make_camera((0.0, -8.0, 1.0), (0, 0, 0), 1600, 1064, 1200.0)]
        name = "masked single-view 1M Gaussians, SH3, 1600x1064"
    elif k == 4:
        n = 1_000_000 if n is None else n
        means = _shell(rng, n)
        scene = random_scene(rng, n, means=means, log_scale=(-4.5, 0.5), opacity=(0.0, 1.5), deg=3,
                             masks=True, band_masks=True)
        sizes = [(316, 208), (632, 416), (1264, 832)]
        cams = []
        for v in range(8):
            th = 2.0 * math.pi * v / 8.0
            w, h = sizes[v % 3]
            cams.append(make_camera((8.0 * math.cos(th), 8.0 * math.sin(th), 0.0), (0, 0, 0), w, h,
                                    w * 1111.0 / 800.0))
        name = "batched 8 progressive-resolution views, 1M Gaussians, SH3, masks"
    elif k == 5:
        n = 6_000_000 if n is None else n
        means = rng.uniform([[-30.0], [-30.0], [-10.0]], [[30.0], [30.0], [10.0]], (3, n))
        scene = random_scene(rng, n, means=means, log_scale=(-3.5, 0.8), opacity=(-0.5, 1.5), deg=3,
                             masks=False, band_masks=True)
        cams = []
        for v in range(8):
            w, h = (1920, 1080) if v < 4 else (960, 540)
            pos = rng.uniform([-24.0, -24.0, -8.0], [24.0, 24.0, 8.0])
            yaw = rng.uniform(0.0, 2.0 * math.pi)
            pitch = math.radians(rng.uniform(-10.0, 10.0))
            fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
            cams.append(make_camera(pos, pos + fwd, w, h, 1500.0))
        name = "batched 4x1080p + 4x540p views, 6M Gaussians, SH3, band masks"
    else:
        raise ValueError(f"unknown workload {k}")
    return Workload(name=name, scene=scene, cams=cams, opts=opts, targets=_targets(rng, cams))


def tiny(n=48, seed=0, deg=3, width=40, height=32, masks=False, band_masks=False, f=None,
         log_scale=(-2.6, 0.35), opacity=(0.5, 1.2), depth=(3.0, 5.0), spread=0.9,
         unit_quats=False, mask_eps=0.5, sh_mask_eps=0.5, depth_levels: Optional[int] = None) -> Workload:
    """A small scene in front of one camera, for brute-force and FD tests.

    The camera sits at the origin looking down +y (world up +z); Gaussians lie
    in a frustum-shaped slab at depths `depth`.  With `depth_levels` the depths
    are drawn from that many evenly spaced values instead (the camera's depth
    axis is world y exactly, so Gaussians of one level share the same float
    depth: ties in the (tile, depth) order are common).
    """
    rng = np.random.default_rng(seed)
    f = float(width) if f is None else f
    if depth_levels:
        z = rng.choice(np.linspace(depth[0], depth[1], depth_levels).astype(F32).astype(np.float64), n)
    else:
        z = rng.uniform(depth[0], depth[1], n)
    x = rng.uniform(-spread, spread, n) * z * (width / 2.0) / f
    y = rng.uniform(-spread, spread, n) * z * (height / 2.0) / f
    # camera looks along +y with up +z: camera x = world x, camera y = -world z
    means = np.stack([x, z, -y], 0)
    scene = random_scene(rng, n, means=means, log_scale=log_scale, opacity=opacity, deg=deg,
                         masks=masks, band_masks=band_masks, mask_eps=mask_eps,
                         sh_mask_eps=sh_mask_eps, unit_quats=unit_quats)
    cam = make_camera((0.0, 0.0, 0.0), (0.0, 1.0, 0.0), width, height, f)
    return Workload(name=f"tiny n={n}", scene=scene, cams=[cam], opts=Opts(),
                    targets=_targets(rng, [cam]))


def scaled(k: int, n: int, views: Optional[Sequence[int]] = None, shrink: int = 1,
           seed: Optional[int] = None) -> Workload:
    """Workload k with n Gaussians, a subset of its views and resolutions divided by `shrink`.

    Focal lengths and principal points scale with the resolution so the field
    of view is kept (as progressive-resolution training does).
    """
    wl = config(k, n=n, seed=seed)
    cams = wl.cams if views is None else [wl.cams[i] for i in views]
    if shrink != 1:
        cams = [Camera(c.R, c.t, _f(c.fx / shrink), _f(c.fy / shrink), _f(c.cx / shrink),
                       _f(c.cy / shrink), max(1, c.width // shrink), max(1, c.height // shrink))
                for c in cams]
    rng = np.random.default_rng(1000 + k)
    return Workload(name=f"{wl.name} [n={n}, views={len(cams)}, /{shrink}]", scene=wl.scene,
                    cams=cams, opts=wl.opts, targets=_targets(rng, cams))
