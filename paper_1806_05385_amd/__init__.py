"""Perceptual rasterization on MI355X (gfx950): foveated + rolling ray-cast
in conservative space-time-fovea bounds, behind the C ABI of libpr.so
(include/pr.h).  ``binding`` wraps the ABI with ctypes; ``render`` drives it
with torch device memory and streams."""
from . import binding  # noqa: F401

__all__ = ['binding']
