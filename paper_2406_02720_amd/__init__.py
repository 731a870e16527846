"""MI355X-native tile rasterizer for 3D half-Gaussian splatting.

The compute path is ``libhgs.so`` (hand-written HIP kernels for gfx950 behind
a C ABI); :mod:`.binding` marshals arguments to it and :mod:`.raster` wraps it
in a ``torch.autograd.Function``.  Submodules are imported lazily so that the
seeded scene generator can be used without the GPU library.
"""
__all__ = ["scenes", "binding", "raster"]
