"""Writes spectrogram_oracle.txt: the FP64 oracle's solve of the spectrogram
workload (513 x 20000, r = 40; seeded input, test matrix seed 3) run to a KKT
residual <= 1e-5 (checked every 10 iterations) or 1500 iterations.  Calls only
the oracle and the seeded input generators.

    python tests/golden/make_spectrogram_oracle.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O                                 # noqa: E402
from paper_2605_19325_amd import inputs            # noqa: E402


def main():
    X, r = inputs.config_spectrogram()
    om = inputs.omega(X.shape[1], r + 10, 3)
    t0 = time.perf_counter()
    U, V, rep = O.enmf(X, r, om, rot_max_iter=100, rot_tol=1e-10, max_iter=1500, kkt_tol=1e-5,
                       check_every=10)
    dt = time.perf_counter() - t0
    with open(os.path.join(HERE, "spectrogram_oracle.txt"), "w") as f:
        f.write("# FP64 oracle, spectrogram 513x20000 r=40 (inputs.config_spectrogram, omega seed 3),\n")
        f.write("# rotation 100 steps / tol 1e-10, stop at kkt <= 1e-5 (checked every 10) or 1500 iterations.\n")
        f.write(f"# written by make_spectrogram_oracle.py in {dt:.0f} s\n")
        for key in ("relerr", "relerr_svd", "kkt", "iters", "converged", "ext_iters_done"):
            f.write(f"{key} {rep[key]!r}\n")
    print(rep["relerr"], rep["kkt"], rep["iters"])


if __name__ == "__main__":
    main()
