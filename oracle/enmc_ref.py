"""Plain FP64 reference of exterior nonnegative matrix completion (eNMC),
the masked extension of eNMF in the paper's appendix "Exterior NMC
algorithm" (test infrastructure only).

X is m x n, M (same shape, 0/1) marks the observed entries, U is m x r and
V is n x r.  The objective is the masked least-squares error of the appendix,
fhat(U, V) = 1/2 ||M o (X - U V^T)||_F^2, with gradients
grad_U = (M o (U V^T - X)) V and grad_V = (M o (U V^T - X))^T U.

Readings where the appendix is silent (also listed with the design notes):
  * M_E marks the observed entries (the masked objective only makes sense on
    known entries).
  * softImpute-ALS is run with lambda = 0, since the stated objective has no
    regulariser.  From a start (U, V) each iteration is an EM step on the
    imputed matrix X* = M o X + (1 - M) o (U V^T): U <- X* V (V^T V)^-1,
    then V <- X*^T U (U^T U)^-1 with the new U.  At lambda = 0 this gives the
    same products U V^T as the softImpute-ALS iteration of Hastie et al.
    (2015), whose extra steps only re-parameterise the factors.  The start is
    the rank-r randomized SVD (Algorithm 3 step 2 of eNMF) of the zero-filled
    M o X.
  * The exterior loop of Algorithm eNMC: every iteration pushes the negative
    entries of U by the fixed step (eq. negup), masks, runs PBCD with the
    masked gradient and the masked optimal row step, then the same for V.
    There is no HALS stage.  The masked optimal step minimises the masked row
    objective exactly (the derivation of eq. d_i with the mask inside):
    d_i = ||g_i||^2 / sum over observed j of (g_i . v_j)^2.

Nothing here is tuned.  This module never imports the HIP path.
"""

import numpy as np

from . import enmf_ref as E


def _f64(a):
    return np.asarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Masked objective and gradients (appendix "Exterior NMC algorithm")
# ---------------------------------------------------------------------------

def masked_objective(X, M, U, V):
    """fhat = 1/2 ||M o (X - U V^T)||_F^2."""
    R = _f64(M) * (_f64(X) - _f64(U) @ _f64(V).T)
    return 0.5 * float(np.sum(R * R))


def masked_gradients(X, M, U, V):
    """(grad_U, grad_V) = ((M o (U V^T - X)) V, (M o (U V^T - X))^T U)."""
    U, V = _f64(U), _f64(V)
    D = _f64(M) * (U @ V.T - _f64(X))
    return D @ V, D.T @ U


def masked_relerr(X, M, U, V):
    """||M o (X - U V^T)|| / ||M o X|| (the error over the observed entries)."""
    nx = float(np.linalg.norm(_f64(M) * _f64(X)))
    return np.sqrt(2.0 * masked_objective(X, M, U, V)) / nx if nx > 0 else 0.0


# ---------------------------------------------------------------------------
# softImpute-ALS at lambda = 0 (the initial local minimiser of fhat)
# ---------------------------------------------------------------------------

def softimpute_als(X, M, U, V, iters):
    """EM / alternating least squares on the imputed matrix (see the module
    docstring).  Returns (U, V, list of fhat after each iteration)."""
    X, M = _f64(X), _f64(M)
    U, V = _f64(U).copy(), _f64(V).copy()
    hist = []
    for _ in range(iters):
        Xs = M * X + (1.0 - M) * (U @ V.T)
        U = Xs @ V @ np.linalg.inv(V.T @ V)
        Xs = M * X + (1.0 - M) * (U @ V.T)
        V = Xs.T @ U @ np.linalg.inv(U.T @ U)
        hist.append(masked_objective(X, M, U, V))
    return U, V, hist


def enmc_init(X, M, r, omega, power_iters=2, als_iters=50):
    """Line 2 of Algorithm eNMC: the randomized SVD of M o X, then softImpute-ALS."""
    Xz = _f64(M) * _f64(X)
    U0, V0, _, _ = E.svd_init_randomized(Xz, r, omega, power_iters)
    return softimpute_als(X, M, U0, V0, als_iters)


# ---------------------------------------------------------------------------
# Masked PBCD and the exterior loop (Algorithm eNMC)
# ---------------------------------------------------------------------------

def masked_pbcd(U, X, M, V, mask, max_iter=5, fixed_step=None):
    """PBCD (Algorithm 2) on fhat for the rows of U with V fixed.

    g = M_U+ o ((M o (U V^T - X)) V); row i takes
    d_i = ||g_i||^2 / sum_j M_ij (g_i . v_j)^2 (0 when that sum is not
    positive) and U_ij <- (U_ij - d_i g_ij)_+ on the masked entries;
    unmasked entries are left alone.  max_iter sweeps.
    """
    U = _f64(U).copy()
    X, M, V = _f64(X), _f64(M), _f64(V)
    P = mask.astype(np.float64)
    for _ in range(max_iter):
        g = P * ((M * (U @ V.T - X)) @ V)
        num = np.sum(g * g, axis=1)
        den = np.sum(M * (g @ V.T) ** 2, axis=1)
        if fixed_step is not None:
            d = np.full(U.shape[0], float(fixed_step))
        else:
            d = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
        U = np.where(mask, np.maximum(0.0, U - d[:, None] * g), U)
    return U


def masked_kkt(X, M, U, V):
    """Check of the masked problem: the eNMF readings with the masked
    gradients, and errors over the observed entries.
      kappa_feas = max(||min(U,0)||/||U||, ||min(V,0)||/||V||)
      kappa_pg_U = ||proj grad_U|| / (||M o X|| ||V||), kappa_pg_V likewise
      kappa = max of the three."""
    X, M, U, V = _f64(X), _f64(M), _f64(U), _f64(V)
    gU, gV = masked_gradients(X, M, U, V)
    nx = float(np.linalg.norm(M * X))

    def pg(W, g):
        return np.where(W > 0, g, np.minimum(g, 0.0))

    nU, nV = float(np.linalg.norm(U)), float(np.linalg.norm(V))
    feas = max(float(np.linalg.norm(np.minimum(U, 0.0))) / nU if nU > 0 else 0.0,
               float(np.linalg.norm(np.minimum(V, 0.0))) / nV if nV > 0 else 0.0)
    pgu = float(np.linalg.norm(pg(U, gU))) / (nx * nV) if nV > 0 and nx > 0 else 0.0
    pgv = float(np.linalg.norm(pg(V, gV))) / (nx * nU) if nU > 0 and nx > 0 else 0.0
    f = masked_objective(X, M, U, V)
    return dict(f=f, relerr=np.sqrt(2.0 * f) / nx if nx > 0 else 0.0,
                kkt=max(feas, pgu, pgv), kkt_feas=feas, kkt_pg_u=pgu, kkt_pg_v=pgv,
                min_w=float(min(U.min(), V.min())))


def enmc_iterate(X, M, U, V, max_iter, ext_iters=10, pbcd_max_iter=5, step_u=None,
                 step_v=None, kkt_tol=-1.0):
    """The loop of Algorithm eNMC: push (eq. negup), mask, masked PBCD on U,
    then the same on V with the new U.  Checked at the top of every
    iteration and at k = max_iter; stops there when U, V >= 0 and
    kappa <= kkt_tol (a negative tolerance disables the test).  Push sizes as
    in eNMF (resolved once from the starting factors)."""
    X, M = _f64(X), _f64(M)
    U, V = _f64(U).copy(), _f64(V).copy()
    su0, sv0 = E.resolve_steps(U, V, ext_iters)
    su = su0 if step_u is None or step_u <= 0 else float(step_u)
    sv = sv0 if step_v is None or step_v <= 0 else float(step_v)
    k = 0
    ext_done = 0
    converged = False
    checks = []
    while True:
        rep = masked_kkt(X, M, U, V)
        rep["k"] = k
        checks.append(rep)
        feasible = U.min() >= 0 and V.min() >= 0
        if feasible and kkt_tol >= 0 and rep["kkt"] <= kkt_tol:
            converged = True
            break
        if k == max_iter:
            break
        ext_done += (U < 0).any() or (V < 0).any()
        U = E.push_negatives(U, su)
        U = masked_pbcd(U, X, M, V, U >= 0, pbcd_max_iter)
        V = E.push_negatives(V, sv)
        V = masked_pbcd(V, X.T, M.T, U, V >= 0, pbcd_max_iter)
        k += 1
    report = dict(checks[-1])
    report.update(iters=k, ext_iters_done=ext_done, converged=converged, step_u=su, step_v=sv,
                  checks=checks)
    return U, V, report


def enmc(X, M, r, omega, power_iters=2, als_iters=50, rho0=1.0, rot_max_iter=100,
         rot_tol=1e-10, **iter_opts):
    """Algorithm eNMC end to end: softImpute-ALS start, ADMM rotation, loop."""
    U0, V0, hist = enmc_init(X, M, r, omega, power_iters, als_iters)
    U, V, R, steps, g0, g1 = E.rotate(U0, V0, rho0, rot_max_iter, rot_tol)
    U, V, rep = enmc_iterate(X, M, U, V, **iter_opts)
    rep.update(als_hist=hist, R=R, rot_steps=steps)
    return U, V, rep
