"""MI355X-native hybrid 2D/3D Gaussian splatting rasterizer (EGGS, Sec. 3.1).

The compute path is ``libhgs.so`` (hand-written HIP for gfx950, C ABI in
include/hgs.h); this package only marshals arguments.
"""
from . import _hgs  # noqa: F401

__all__ = ["build", "rasterizer"]


def build(verbose: bool = False) -> str:
    from .build import build as _b
    return _b(verbose=verbose)
