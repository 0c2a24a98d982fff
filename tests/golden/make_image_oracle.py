"""Writes image_oracle.txt: the FP64 oracle's solve of the image-patch
workload (4096 x 10000, r = 49; seeded input, test matrix seed 1) with the
default rotation (100 steps, tolerance 1e-10) and 500 iterations, checked
every 10 iterations.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_image_oracle.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

import fullsize_oracle as F                        # noqa: E402
import oracle as O                                 # noqa: E402
from paper_2605_19325_amd import inputs            # noqa: E402

ITERS = 500


def main():
    X, r = inputs.config_image()
    om = inputs.omega(X.shape[1], r + 10, 1)
    (U, V, rep), dt = F.timed(lambda: O.enmf(X, r, om, rot_max_iter=100, rot_tol=1e-10,
                                             max_iter=ITERS, check_every=10))
    rows_u = F.sample_rows(32, X.shape[0], 21)
    rows_v = F.sample_rows(32, X.shape[1], 22)
    F.write("image_oracle.txt",
            ["FP64 oracle, image-patch 4096x10000 r=49 (inputs.config_image, omega seed 1),",
             f"rotation 100 steps / tol 1e-10, {ITERS} iterations, checked every 10;",
             "sampled rows of U (seed 21) and V (seed 22) at the end"],
            rep, U, V, rows_u, rows_v, dt)
    print(rep["relerr"], rep["kkt"], rep["iters"], rep["ext_iters_done"], f"{dt:.0f} s")


if __name__ == "__main__":
    main()
