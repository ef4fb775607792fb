"""MI355X (gfx950) implementation of the RBE2D hot path: random batch Ewald
k-space and erfc real space for charges in a dielectrically confined,
doubly periodic slab, behind the C ABI of librbe2d.so (include/rbe2d.h)."""
from . import inputs  # noqa: F401

__all__ = ["inputs", "rbe2d"]
