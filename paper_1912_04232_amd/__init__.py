"""MI355X-native short-range molecular dynamics (cell list, neighbor list, LJ / soft-sphere
forces, velocity Verlet, FIRE) behind the C ABI declared in include/md.h.

Importing this package loads nothing; the HIP library is loaded on first use by
``paper_1912_04232_amd.md`` and a missing library raises at that point.
"""
__all__ = ["inputs"]
