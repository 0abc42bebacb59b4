"""MI355X-native rasterizer for editable 3D Gaussians (iVR-GS hot path).

Submodules:
    native   ctypes binding of libivrgs.so (include/ivrgs.h)
    raster   torch-facing API: Renderer, rasterize (autograd), compose
    inputs   seeded synthetic scenes and cameras
    build    hipcc build of libivrgs.so for gfx950
"""
import importlib

__all__ = ["native", "raster", "inputs", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
