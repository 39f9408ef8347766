"""Writes dense_50000x4000_xstar.txt: x* = argmin ||A x - b||_2 for the dense 50000 x 4000
workload (workloads.dense_coherent, case 2), by the oracle's direct Householder QR solve
(the plain definition of the least-squares solution that Algorithm 1 reaches, Section 5).
Calls only the oracle and the seeded input generator.  Run from the repository root:
    python tests/golden/make_dense_xstar.py"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import lls  # noqa: E402


def main():
    c = workloads.CASES["dense"]
    A, b = workloads.dense_coherent(n=c["n"], d=c["d"], case=c["case"])
    x = lls.lstsq_direct(A, b)
    r = b - A @ x
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dense_50000x4000_xstar.txt")
    with open(out, "w") as f:
        f.write("# x* = argmin ||A x - b||_2 of the dense 50000 x 4000 workload "
                "(workloads.dense_coherent, case 2)\n")
        f.write("# by the oracle's direct Householder QR solve; written by make_dense_xstar.py\n")
        f.write(f"# ||r*|| = {np.linalg.norm(r):.17g}\n")
        for v in x:
            f.write(f"{v:.17g}\n")
    print("wrote", out, "||r*||", np.linalg.norm(r))


if __name__ == "__main__":
    main()
