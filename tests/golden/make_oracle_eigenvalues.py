"""Write the oracle's eigenvalues of the n = 2048 workload to a text fixture.

Calls only the FP64 oracle (Alg. 3 with LAPACK potrf and gesvd); the GPU
parity test at full size compares every form against this file.

    python tests/golden/make_oracle_eigenvalues.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import bse as ob  # noqa: E402
from paper_2008_08825_amd import inputs  # noqa: E402


def main():
    A, B = inputs.workload("n2048")
    t0 = time.time()
    lam, X = ob.solve_chol_svd(A, B)
    dt = time.time() - t0
    out = os.path.join(HERE, "oracle_n2048_eigenvalues.txt")
    with open(out, "w") as f:
        f.write("# positive eigenvalues (ascending) of H1 for the n = 2048 workload (seed 0),\n")
        f.write("# computed by oracle.bse.solve_chol_svd (Alg. 3: potrf x2, gesvd) in FP64\n")
        f.write(f"# by tests/golden/make_oracle_eigenvalues.py in {dt:.0f} s\n")
        for v in lam:
            f.write(f"{v:.17g}\n")
    print(out, dt)


if __name__ == "__main__":
    main()
