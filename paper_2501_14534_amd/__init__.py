"""MI355X-native differentiable Gaussian-splatting tile rasterizer (Trick-GS hot path).

The compute path is the HIP library `libgs.so` (csrc/), reached through the
ctypes binding in `gs.py`.  Importing this package does not load the library;
`gs.load()` does, and fails loudly if it has not been built.
"""
__all__ = ["scenes", "gs", "raster"]
