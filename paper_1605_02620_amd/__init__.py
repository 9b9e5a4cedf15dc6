"""MI355X-native RSOS deposition sweep (Kelling, Odor & Gemming, arXiv:1605.02620).

The simulation runs in librsos.so (hand-written HIP for gfx950, C ABI in
include/rsos.h); this package only marshals arguments to it, with torch
providing device memory and streams.
"""
from .surface import Batch, MultiSurface, Surface, philox, w2  # noqa: F401

__all__ = ["Surface", "Batch", "MultiSurface", "philox", "w2"]
