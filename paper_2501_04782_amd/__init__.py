"""MI355X-native differentiable 3D Gaussian rasterizer (GaussianVideo's fitting
hot path): gfx950 HIP kernels behind the C ABI of include/gv.h, with a thin
torch binding.  Importing the package does not touch the GPU; the first call
loads libgv.so and raises if it has not been built."""
from . import _lib
from .raster import (BatchGraph, Camera, RasterizeClip, RasterizeDynamicClip, RasterizeFrame, Scene, Workspace,
                     autotune, estimate_capacity, gaussian_pyramid, get_tuning, grad_buffers, project_fwd,
                     render_batch, render_batch_timed, render_bwd, render_fwd, set_tuning, visibility_counts)

__all__ = ["BatchGraph", "Camera", "RasterizeClip", "RasterizeDynamicClip", "RasterizeFrame", "Scene", "Workspace",
           "autotune", "estimate_capacity", "gaussian_pyramid", "visibility_counts", "get_tuning", "grad_buffers", "project_fwd", "render_batch", "render_batch_timed",
           "render_bwd", "render_fwd", "set_tuning", "load_library"]


def load_library():
    return _lib.load()
