"""Plain FP64 CPU oracle for the sketch-and-precondition least-squares method
(Cartis, Fiala and Shao, "Hashing embeddings of optimal dimension, with
applications to linear least squares", Algorithm 1 and Section 6).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package; only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library: it is written from the paper's definitions with numpy/scipy, slowly
and obviously, so that a reader can check it against the paper by eye.

Modules
-------
philox  -- Philox4x64-10 counter-based generator (Salmon et al., SC'11),
           written from its published definition.
sketch  -- the s-hashing matrix (Definition of s-hashing, Section 2.2), the
           random sign diagonal D and the Walsh-Hadamard transform H
           (Definition of HRHT, Section 4.3), and the sketch S[A b].
lls     -- QR of the sketch, the sketched solution and early exit, LSQR on
           W = A R^-1 with the (TC-lsqr) stopping test, the recovered x
           (Algorithm 1, Steps 2-5), the direct dense reference solve and the
           adjoint (backward) used for differentiation.
sparse_qr -- the sparse form of Step 2 (Section 6): the pattern of the sketch,
           the minimum-degree column ordering, the structure of R and the
           solve on the column-permuted matrix.
"""

from . import philox, sketch, lls, sparse_qr  # noqa: F401
