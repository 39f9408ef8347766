"""Writes dense_50000x4000_oracle_run.txt: the oracle's run of Algorithm 1 on the dense
50000 x 4000 workload (workloads.dense_coherent, case 2) with the benchmark's sketch
(Walsh-Hadamard transform, s = 3, m = 6800, seed 2002) and tau_r = 1e-10: the LSQR
iteration count at which (TC-lsqr) first holds and LSQR's final estimates.  A GPU test
compares the library's iteration count with this one (to within one step).  Calls only
the oracle and the seeded input generator.  Run from the repository root:
    python tests/golden/make_dense_iters.py"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import lls  # noqa: E402


def main():
    c = workloads.CASES["dense"]
    A, b = workloads.dense_coherent(n=c["n"], d=c["d"], case=c["case"])
    t0 = time.time()
    X, info = lls.solve(A, b, seed=2002, s=c["s"], m=c["m"], tau_r=1e-10)
    rec = info["records"][0]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                       "dense_50000x4000_oracle_run.txt")
    with open(out, "w") as f:
        f.write("# the oracle's Algorithm 1 on the dense 50000 x 4000 workload (case 2):\n")
        f.write("# Walsh-Hadamard + 3-hashing, m 6800, seed 2002, tau_r 1e-10; "
                "written by make_dense_iters.py\n")
        for key in ("iters", "rnorm", "arnorm", "anorm", "tc"):
            f.write(f"{key}: {rec[key]!r}\n")
    print("wrote", out, rec, f"{time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
