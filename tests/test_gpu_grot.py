"""GPU parity of the generalized rotation (the appendix section on exact NMF,
Algorithm alg:rsr) against the FP64 oracle, through the C ABI.

Both sides start from the same float32 factors (the oracle promotes them) and
run the same number of ADMM steps in float64.  They differ in the order of
the float64 sums and in the Procrustes step (Newton-Schulz polar factor on
the GPU, the SVD in the oracle): R1, Lambda and R2 agree to about 1e-14
after a few steps and 1e-12 after 40 (measured); the bars below leave two
orders of magnitude for the growth of those differences.

* 5 and 40 steps on random factors of several shapes (r = 1, 7, 20, 33: every
  padded width) within 1e-10 (R1, R2, lambda; relative);
* the appendix's exact instances (40 x 50, r = 10 and 80 x 100, r = 20, 10%
  zeros in the true factors): after 500 steps no negative entry on either
  side, U V^T kept to float32 rounding, lambda within 1e-8;
* the tolerance stop, and argument errors.
"""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2605_19325_amd import enmf, inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def host(t):
    return t.detach().cpu().double().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("m,n,r,steps", [(9, 7, 1, 5), (30, 25, 7, 40), (40, 50, 20, 40),
                                         (70, 60, 33, 5), (70, 60, 33, 40)])
def test_rotate_general_parity(lib, m, n, r, steps):
    say(f"generalized rotation {m}x{n} r={r}, {steps} steps")
    rng = np.random.default_rng(m + n + r)
    U = rng.standard_normal((m, r)).astype(np.float32)
    V = rng.standard_normal((n, r)).astype(np.float32)
    Uo, Vo, R1, lam, R2, st, g0, g1 = O.rotate_general(U, V, max_iter=steps, tol=0.0)
    Ud, Vd = to_dev(U), to_dev(V)
    out = lib.rotate_general(Ud, Vd, max_iter=steps, tol=0.0)
    say(f"  R1 {rel(out['R1'], R1):.2e} R2 {rel(out['R2'], R2):.2e} lam {rel(out['lam'], lam):.2e} "
        f"neg {out['neg_mass_after']:.6e} oracle {g1:.6e}")
    assert out["steps"] == st == steps
    assert rel(out["R1"], R1) <= 1e-10 and rel(out["R2"], R2) <= 1e-10 and rel(out["lam"], lam) <= 1e-10
    assert abs(out["neg_mass_before"] - g0) <= 1e-12 * g0
    assert abs(out["neg_mass_after"] - g1) <= 1e-7 * g0
    # outputs are the oracle's float64 result rounded to float32
    assert rel(host(Ud), Uo) <= 1e-7 and rel(host(Vd), Vo) <= 1e-7


@pytest.mark.parametrize("m,n,r,seed", [(40, 50, 10, 1), (80, 100, 20, 0)])
def test_exact_instances(lib, m, n, r, seed):
    say(f"generalized rotation on the exact instance {m}x{n} r={r}, 500 steps")
    X, _, _ = inputs.exact_nmf(m, n, r, seed, sparsity=0.1)
    Us, Vs, _, _ = O.svd_init_exact(X, r)
    Us, Vs = Us.astype(np.float32), Vs.astype(np.float32)
    Uo, Vo, R1, lam, R2, st, g0, g1 = O.rotate_general(Us, Vs, max_iter=500, tol=0.0)
    Ud, Vd = to_dev(Us), to_dev(Vs)
    out = lib.rotate_general(Ud, Vd, max_iter=500, tol=0.0)
    Ug, Vg = host(Ud), host(Vd)
    say(f"  neg {out['neg_mass_before']:.4e} -> {out['neg_mass_after']:.3e} (oracle {g1:.3e}) "
        f"lam {rel(out['lam'], lam):.2e} |UV - X|/|X| {rel(Ug @ Vg.T, X):.2e}")
    assert g1 == 0.0 and out["neg_mass_after"] == 0.0
    assert Ug.min() >= 0.0 and Vg.min() >= 0.0
    assert rel(Ug @ Vg.T, Us.astype(np.float64) @ Vs.astype(np.float64).T) <= 1e-6
    assert rel(out["lam"], lam) <= 1e-8


def test_rotate_general_tolerance_stop(lib):
    say("generalized rotation stops on the change tolerance")
    X, _, _ = inputs.exact_nmf(40, 50, 10, 2, sparsity=0.1)
    Us, Vs, _, _ = O.svd_init_exact(X, 10)
    Us, Vs = Us.astype(np.float32), Vs.astype(np.float32)
    *_, st, g0, g1 = O.rotate_general(Us, Vs, max_iter=3000, tol=1e-6)
    out = lib.rotate_general(to_dev(Us), to_dev(Vs), max_iter=3000, tol=1e-6)
    say(f"  steps gpu {out['steps']} oracle {st}")
    assert st < 3000 and abs(out["steps"] - st) <= 2


def test_rotate_general_bad_arguments(lib):
    say("generalized rotation argument errors")
    U, V = to_dev(np.ones((5, 3))), to_dev(np.ones((4, 3)))
    with pytest.raises(enmf.EnmfError):
        lib.rotate_general(U, V, max_iter=-1)
    with pytest.raises(enmf.EnmfError):
        lib.rotate_general(U, V, rho0=0.0)
    with pytest.raises(enmf.EnmfError):
        lib.rotate_general(to_dev(np.ones((5, 65))), to_dev(np.ones((4, 65))))
