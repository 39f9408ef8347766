"""MI355X (gfx950) sketch-and-precondition solver for overdetermined least squares
(Cartis, Fiala and Shao, Algorithm 1 with the dense and sparse variants of Section 6).

The computation lives in the HIP library libski.so (C interface in include/ski.h);
this package is its Python binding.
"""

from .api import Solver, SkiError, SkiLstsq, lstsq, params, sketch_noalloc  # noqa: F401
