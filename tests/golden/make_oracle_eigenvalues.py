"""Write the oracle's eigenvalues of a full-size workload to a text fixture.

Calls only the FP64 oracle (Alg. 3 with LAPACK potrf and gesvd); the GPU
parity tests at full size compare every form against these files.

    python tests/golden/make_oracle_eigenvalues.py              # n = 2048 workload
    python tests/golden/make_oracle_eigenvalues.py n8192_clustered

n2048: oracle.bse.solve_chol_svd (vectors and values); n8192_clustered:
oracle.bse.eigenvalues_chol_svd (Alg. 3 steps 1-3, values only; several
minutes on a few host cores).
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


def main(name="n2048"):
    A, B = inputs.workload(name)
    n = A.shape[0]
    t0 = time.time()
    if name == "n2048":
        lam, _ = ob.solve_chol_svd(A, B)
        how = "oracle.bse.solve_chol_svd (Alg. 3: potrf x2, gesvd)"
    else:
        lam = ob.eigenvalues_chol_svd(A, B)
        how = "oracle.bse.eigenvalues_chol_svd (Alg. 3 steps 1-3: potrf x2, gesvd without vectors)"
    dt = time.time() - t0
    out = os.path.join(HERE, f"oracle_{name}_eigenvalues.txt")
    with open(out, "w") as f:
        f.write(f"# positive eigenvalues (ascending) of H1 for the {name} workload (n = {n}, seed 0),\n")
        f.write(f"# computed by {how} in FP64\n")
        f.write(f"# by tests/golden/make_oracle_eigenvalues.py in {dt:.0f} s\n")
        for v in lam:
            f.write(f"{v:.17g}\n")
    print(out, dt)


if __name__ == "__main__":
    main(*sys.argv[1:2])
