"""Low-rank Poisson solver for MI355X (gfx950).

The solver is a C-ABI shared library (``liblrpoisson.so``, declared in
``include/lrpoisson.h``) built from the HIP sources in ``csrc/``; this package
holds the thin ctypes binding over it (``binding``), the build script
(``build``), the seeded input generators (``inputs``) and the serving loop
driver (``serving``).  Importing the package loads nothing; the library is
loaded on first use and its absence is an error (there is no CPU fallback).
"""
__all__ = ["inputs"]
