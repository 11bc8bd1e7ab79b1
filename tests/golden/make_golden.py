"""Write the oracle regression fixture ``oracle_poisson8.json``.

Calls only the oracle and the seeded input generators.  Run from the repository
root: ``python tests/golden/make_golden.py``.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2111_09512_amd import workloads as W  # noqa: E402


def main():
    A = W.poisson7(8)
    Ls, U = O.ilu0(A)
    d, dinv, Us = O.scale_rows(U)
    b = W.rhs(A.n, 0)
    x = O.smooth(A, Ls, Us, dinv, b, np.zeros(A.n), 1, 3, 3)
    idx = [0, 1, 7, 63, 100, 255, 300, 511]
    out = {
        "what": "oracle smoother, 7-pt Poisson N=8, ILU(0), row-scaled, 1 outer x 3/3 Richardson, b=U(-1,1) seed 0, x0=0",
        "idx": idx,
        "x_at_idx": [float(v) for v in x[idx]],
        "nrm2": float(O.nrm2(x)),
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_poisson8.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
