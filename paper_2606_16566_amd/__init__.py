"""MI355X (gfx950) tile-based Gaussian-splatting rasterizer with the Local-GS
render stages (tile-local hoisting, wavefront culling, uniform blending).

The compute path is liblocalgs.so (HIP, C ABI in include/localgs.h); the
torch-facing wrappers live in ``rasterizer``; ``scenes`` draws synthetic
inputs.  Importing the package does not load the library or touch the GPU.
"""
__version__ = "0.1.0"

__all__ = ["scenes", "rasterizer"]
