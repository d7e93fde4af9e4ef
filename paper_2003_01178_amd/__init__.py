"""Tile-based fused query execution for MI355X (gfx950).

The kernels live in ``csrc/`` and are exported through the C ABI declared in
``include/crystal.h``; ``crystal`` is the thin ctypes binding over it.  The
binding is imported lazily so that ``datagen`` can be used without a GPU.
"""
__all__ = ["crystal", "datagen"]
