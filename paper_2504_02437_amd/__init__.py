"""gsmap: MI355X-native differentiable tile rasterizer for Gaussian-splatting
mapping (MonoGS++, arXiv 2504.02437).  The kernels live in libgsmap.so
(include/gsmap.h); this package marshals torch device buffers into it."""

__all__ = ["raster", "build"]
