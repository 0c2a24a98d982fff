"""Writes ratings_oracle.txt: the FP64 oracle's solve of the ratings workload
(100000 x 20000, r = 20; seeded input, test matrix seed 4) with the default
rotation (100 steps, tolerance 1e-10) and 100 iterations, checked every 10
iterations.  Calls only the oracle and the seeded input generators.  The
float64 copy of X takes 16 GB and the run about 40 GB of host memory at peak.

    python tests/golden/make_ratings_oracle.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

import fullsize_oracle as F                        # noqa: E402
import oracle as O                                 # noqa: E402
from paper_2605_19325_amd import inputs            # noqa: E402

ITERS = 100
RANK = 20


def main():
    X32 = inputs.ratings()
    n = X32.shape[1]
    X = X32.astype(np.float64)          # the oracle's own float64 copy (exact)
    del X32
    om = inputs.omega(n, RANK + 10, 4)
    (U, V, rep), dt = F.timed(lambda: O.enmf(X, RANK, om, rot_max_iter=100, rot_tol=1e-10,
                                             max_iter=ITERS, check_every=10))
    rows_u = F.sample_rows(32, X.shape[0], 41)
    rows_v = F.sample_rows(32, X.shape[1], 42)
    F.write("ratings_oracle.txt",
            ["FP64 oracle, ratings 100000x20000 r=20 (inputs.ratings, omega seed 4),",
             f"rotation 100 steps / tol 1e-10, {ITERS} iterations, checked every 10;",
             "sampled rows of U (seed 41) and V (seed 42) at the end"],
            rep, U, V, rows_u, rows_v, dt)
    print(rep["relerr"], rep["kkt"], rep["iters"], rep["ext_iters_done"], f"{dt:.0f} s")


if __name__ == "__main__":
    main()
