"""Plain FP64 reference of the eNMF hot path (test infrastructure only).

Written from the paper "An Exterior Method for Nonnegative Matrix
Factorization".  Conventions: X is m x n with X >= 0, U is m x r, V is
n x r and X ~ U V^T (the appendix on computational complexity uses this
orientation; section 3 uses the transposed one).  Everything is float64
NumPy.  Rows that the paper says are independent (the PBCD row updates of
section 3.2, the HALS column update) are evaluated for all rows at once
with NumPy; nothing is blocked, fused or reordered beyond that.

Nothing here is tuned.  This module never imports the HIP path.
"""

import numpy as np

EXT = 0    # exterior phase: negative push + PBCD (section 3.2, Algorithm 3)
HALS = 1   # descent phase (section 3.3)


def _f64(a):
    return np.asarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Objective, gradients, errors  (problem statement, eq. 1)
# ---------------------------------------------------------------------------

def objective(X, U, V, block=4096):
    """f(U,V) = 1/2 ||X - U V^T||_F^2 (eq. 1), summed directly over row blocks."""
    X, U, V = _f64(X), _f64(U), _f64(V)
    f = 0.0
    for i0 in range(0, X.shape[0], block):
        E = X[i0:i0 + block] - U[i0:i0 + block] @ V.T
        f += float(np.sum(E * E))
    return 0.5 * f


def objective_expanded(X, U, V):
    """The same f expanded: 1/2||X||^2 - <U, XV> + 1/2 <U^T U, V^T V>."""
    X, U, V = _f64(X), _f64(U), _f64(V)
    return 0.5 * float(np.sum(X * X)) - float(np.sum(U * (X @ V))) \
        + 0.5 * float(np.sum((U.T @ U) * (V.T @ V)))


def relerr(X, U, V):
    """Relative reconstruction error ||X - U V^T||_F / ||X||_F."""
    return float(np.sqrt(2.0 * objective(X, U, V)) / np.linalg.norm(_f64(X)))


def gradients(X, U, V):
    """grad_U f = (U V^T - X) V and grad_V f = (U V^T - X)^T U (section 3.2).

    Evaluated through the identities (U V^T - X) V = U (V^T V) - X V and
    likewise for V, which the appendix on complexity uses as the core kernel.
    """
    X, U, V = _f64(X), _f64(U), _f64(V)
    gU = U @ (V.T @ V) - X @ V
    gV = V @ (U.T @ U) - X.T @ U
    return gU, gV


# ---------------------------------------------------------------------------
# Block (i): unconstrained optimum, section 3 opening and Algorithm 3 step 2
# ---------------------------------------------------------------------------

def fix_signs(U, V):
    """Singular-vector sign convention (the paper is silent).

    Flip each pair (u_j, v_j) so that sum_i U_ij > 0; when that sum is
    exactly zero, make the first nonzero entry of u_j positive.  The product
    U V^T is unchanged.
    """
    U, V = _f64(U).copy(), _f64(V).copy()
    for j in range(U.shape[1]):
        s = float(np.sum(U[:, j]))
        if s == 0.0:
            nz = np.flatnonzero(U[:, j])
            s = U[nz[0], j] if nz.size else 1.0
        if s < 0:
            U[:, j] = -U[:, j]
            V[:, j] = -V[:, j]
    return U, V


def balance(U, sigma, V):
    """Balanced factors U* = U Sigma^(1/2), V* = V Sigma^(1/2) (section 3)."""
    s = np.sqrt(_f64(sigma))
    return _f64(U) * s, _f64(V) * s


def _relerr_svd(X, sigma):
    nx2 = float(np.sum(_f64(X) ** 2))
    return float(np.sqrt(max(0.0, nx2 - float(np.sum(_f64(sigma) ** 2)))) / np.sqrt(nx2))


def svd_init_exact(X, r):
    """Rank-r truncated SVD X ~ U Sigma V^T, balanced (section 3).

    Returns (U*, V*, sigma, relerr_svd) with relerr_svd the Eckart-Young
    floor sqrt(||X||^2 - sum sigma^2) / ||X||.
    """
    X = _f64(X)
    Uf, s, Vt = np.linalg.svd(X, full_matrices=False)
    U, V = fix_signs(Uf[:, :r], Vt[:r].T)
    Us, Vs = balance(U, s[:r], V)
    return Us, Vs, s[:r].copy(), _relerr_svd(X, s[:r])


def svd_init_randomized(X, r, omega, power_iters=2):
    """Randomized truncated SVD, the drop-in the paper reports for the exact one.

    The paper replaces the Krylov SVD by a randomized SVD (remark after
    Algorithm 3; appendix table comparing the two) without giving its
    parameters.  Reading taken: the Halko-Martinsson-Tropp range finder
    with a Gaussian test matrix omega (n x (r+p)) supplied by the caller and
    q power iterations, each re-orthonormalised:

        Y = X omega;  q times: Q = qr(Y), Q' = qr(X^T Q), Y = X Q'
        Q = qr(Y);  B = Q^T X = Ub S W^T;  U = Q Ub[:, :r], V = W[:, :r]

    then the sign convention and the balanced scaling.
    """
    X, omega = _f64(X), _f64(omega)
    Y = X @ omega
    for _ in range(power_iters):
        Q, _ = np.linalg.qr(Y)
        Qp, _ = np.linalg.qr(X.T @ Q)
        Y = X @ Qp
    Q, _ = np.linalg.qr(Y)
    B = Q.T @ X
    Ub, s, Wt = np.linalg.svd(B, full_matrices=False)
    U, V = fix_signs(Q @ Ub[:, :r], Wt[:r].T)
    Us, Vs = balance(U, s[:r], V)
    return Us, Vs, s[:r].copy(), _relerr_svd(X, s[:r])


# ---------------------------------------------------------------------------
# Block (ii): rotation by ADMM, Algorithm 1 and section 3.1
# ---------------------------------------------------------------------------

def prox_h(b, rho):
    """Z-update of Algorithm 1, eq. 7: the minimiser of h(z) + rho/2 (z - b)^2.

    h(q) = max(0, -q).  Three cases: b > 0 keeps b; -1/rho <= b <= 0 gives 0;
    b < -1/rho gives b + 1/rho.
    """
    b = _f64(b)
    t = 1.0 / rho
    return np.where(b > 0, b, np.where(b >= -t, 0.0, b + t))


def procrustes(M):
    """R-update of Algorithm 1 (section 3.1): with W^T B = C S D^T, R = C D^T.

    R is the orthogonal polar factor of M = W^T B; reflections are allowed
    because only R^T R = I is imposed.
    """
    C, _, Dt = np.linalg.svd(_f64(M))
    return C @ Dt


def negativity_mass(W):
    """sum_ij h(W_ij) with h(q) = max(0, -q): the rotation objective."""
    return float(np.sum(np.maximum(0.0, -_f64(W))))


def rotate(U, V, rho0=1.0, max_iter=100, tol=1e-10, R0=None):
    """ADMM for min_R sum h(W R) s.t. R^T R = I (Algorithm 1, eq. for W).

    Readings where the paper gives symbols only: W = [U; V];
    rho = rho0 * sqrt(N r) / ||W||_F with N = m + n (so the prox threshold
    1/rho is the RMS entry of W / rho0); R^0 = I (or R0), Y^0 = 0; stop when
    ||R^{k+1} - R^k||_F <= tol or after max_iter steps (tol = 0 runs exactly
    max_iter steps).  The output is (U R, V R) with the last R.

    Returns (U R, V R, R, steps, g_before, g_after) with g the negativity mass.
    """
    U, V = _f64(U), _f64(V)
    m, r = U.shape
    W = np.vstack([U, V])
    N = W.shape[0]
    rho = rho0 * np.sqrt(N * r) / np.linalg.norm(W)
    R = np.eye(r) if R0 is None else _f64(R0).copy()
    Y = np.zeros_like(W)
    steps = 0
    for _ in range(max_iter):
        b = W @ R - Y / rho
        Z = prox_h(b, rho)
        B = Z + Y / rho
        R_new = procrustes(W.T @ B)
        Y = Y + rho * (Z - W @ R_new)
        dR = float(np.linalg.norm(R_new - R))
        R = R_new
        steps += 1
        if tol > 0 and dR <= tol:
            break
    WR = W @ R
    return WR[:m], WR[m:], R, steps, negativity_mass(W), negativity_mass(WR)


# ---------------------------------------------------------------------------
# Block (iii): exterior penalty + PBCD, section 3.2, Algorithms 2 and 3,
# appendix on the optimal ascent step
# ---------------------------------------------------------------------------

def resolve_steps(U, V, ext_iters=10):
    """Fixed push sizes rho_u delta_u and rho_v delta_v (eq. negup, negup_v).

    The paper gives no value.  Reading taken: step = max(-min W, 0) /
    (ext_iters - 0.5), resolved once from the rotated factors, so the most
    negative entry turns nonnegative on exactly the ext_iters-th push, half
    a step clear of zero.
    """
    d = float(ext_iters) - 0.5
    su = max(-float(np.min(U)), 0.0) / d
    sv = max(-float(np.min(V)), 0.0) / d
    return su, sv


def push_negatives(W, step):
    """eq. negup / negup_v: every negative entry moves up by the fixed step."""
    W = _f64(W).copy()
    W[W < 0] += step
    return W


def pbcd(U, P, G, mask, eps=0.0, max_iter=5, fixed_step=None):
    """Algorithm 2 (PBCD) with the optimal row steps of eq. d_i.

    P = X V and G = V^T V are fixed while V is fixed.  Masked gradient
    g = M o (U G - P) = M o ((U V^T - X) V).  Each row i takes
    d_i = ||g_i||^2 / ||g_i V^T||^2 = ||g_i||^2 / (g_i G g_i^T) (0 when the
    denominator is not positive) and U_ij <- (U_ij - d_i g_ij)_+ on the
    masked entries; unmasked entries are left alone.  The loop stops when
    ||M o grad||_F < eps * ||M o grad_init||_F or after max_iter sweeps.
    Rows are independent (section 3.2), so each sweep updates all rows at once.

    fixed_step: the fixed-step ablation of the appendix tables (one step for
    every row in place of d_i; see iterate, mode 2).
    """
    U = _f64(U).copy()
    P, G = _f64(P), _f64(G)
    M = mask.astype(np.float64)
    g = M * (U @ G - P)
    thr = eps * float(np.linalg.norm(g))
    sweeps = 0
    for _ in range(max_iter):
        if fixed_step is not None:
            d = np.full(U.shape[0], float(fixed_step))
        else:
            num = np.sum(g * g, axis=1)
            den = np.einsum("ia,ab,ib->i", g, G, g)
            d = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
        U = np.where(mask, np.maximum(0.0, U - d[:, None] * g), U)
        g = M * (U @ G - P)
        sweeps += 1
        if float(np.linalg.norm(g)) < thr:
            break
    return U, sweeps


def fixed_row_step(G):
    """Step of the fixed-step ablation (the paper gives no value).

    Reading taken: 1 / ||G||_F for the half's Gram G.  Since ||G||_F bounds
    the largest eigenvalue of G, the Lipschitz constant of the gradient in
    each row, this projected-gradient step never increases f, and it is at
    most every row's optimal step d_i (g G g^T <= lambda_max ||g||^2).
    """
    nf = float(np.linalg.norm(_f64(G)))
    return 1.0 / nf if nf > 0 else 0.0


def ext_half(U, P, G, step, eps=0.0, max_iter=5, fixed=False):
    """One half of an exterior iteration of Algorithm 3: push, mask, PBCD.

    The mask M_{U+} marks nonnegative entries (zero included), computed after
    the push.  fixed = True takes the fixed row step of fixed_row_step.
    """
    U = push_negatives(U, step)
    mask = U >= 0
    U, _ = pbcd(U, P, G, mask, eps, max_iter, fixed_row_step(G) if fixed else None)
    return U


def hals_half(U, P, G):
    """HALS half-sweep (section 3.3; the paper cites HALS without printing it).

    Textbook block-coordinate minimiser of eq. 1 over one column at a time,
    Gauss-Seidel over j = 1..r with the columns already updated:
    U_:j <- max(0, U_:j + (P_:j - U G_:j) / G_jj), skipped when G_jj = 0.
    No floor and no normalisation.
    """
    U = _f64(U).copy()
    P, G = _f64(P), _f64(G)
    for j in range(U.shape[1]):
        if G[j, j] > 0:
            U[:, j] = np.maximum(0.0, U[:, j] + (P[:, j] - U @ G[:, j]) / G[j, j])
    return U


# ---------------------------------------------------------------------------
# KKT conditions (appendix eq. kkt-nmf and the (delta_W, sigma_W) tuple)
# ---------------------------------------------------------------------------

def kkt(X, U, V, svd_tail_sq=None):
    """Objective, errors and KKT residual at (U, V).

    The paper states the conditions U >= 0, grad_U >= 0, grad_U o U = 0 (and
    for V) and reports (delta_W, sigma_W) = (max(grad_W o W), sum(grad_W o W))
    without a normalisation.  Reading taken for one dimensionless residual:
      kappa_feas = max(||min(U,0)||/||U||, ||min(V,0)||/||V||)
      projected gradient: grad where W > 0, min(grad, 0) where W <= 0
      kappa_pg_U = ||proj grad_U|| / (||X|| ||V||), kappa_pg_V likewise with U
      kappa = max(kappa_feas, kappa_pg_U, kappa_pg_V)
    relerr = ||X - U V^T|| / ||X||; re_paper is the paper's ratio to the
    truncated-SVD error (figure 1), given svd_tail_sq = ||X - X_r||^2.
    """
    X, U, V = _f64(X), _f64(U), _f64(V)
    f = objective(X, U, V)
    nx = float(np.linalg.norm(X))
    gU, gV = gradients(X, U, V)

    def pg(W, g):
        return np.where(W > 0, g, np.minimum(g, 0.0))

    def nrm(a):
        return float(np.linalg.norm(a))

    nU, nV = nrm(U), nrm(V)
    feas = max(nrm(np.minimum(U, 0.0)) / nU if nU > 0 else 0.0,
               nrm(np.minimum(V, 0.0)) / nV if nV > 0 else 0.0)
    pgu = nrm(pg(U, gU)) / (nx * nV) if nV > 0 else 0.0
    pgv = nrm(pg(V, gV)) / (nx * nU) if nU > 0 else 0.0
    prodU, prodV = gU * U, gV * V
    out = dict(
        f=f,
        relerr=float(np.sqrt(2.0 * f) / nx),
        kkt_feas=feas, kkt_pg_u=pgu, kkt_pg_v=pgv,
        kkt=max(feas, pgu, pgv),
        delta_w=float(max(prodU.max(), prodV.max())),
        sigma_w=float(prodU.sum() + prodV.sum()),
        sigma_u=float(prodU.sum()), sigma_v=float(prodV.sum()),
        min_w=float(min(U.min(), V.min())),
    )
    out["re_paper"] = (float(np.sqrt(2.0 * f / svd_tail_sq))
                       if svd_tail_sq is not None and svd_tail_sq > 0 else float("nan"))
    return out


# ---------------------------------------------------------------------------
# Algorithm 3 driver (blocks iii and iv)
# ---------------------------------------------------------------------------

def iterate(X, U, V, max_iter, ext_iters=10, pbcd_max_iter=5, pbcd_eps=0.0,
            step_u=None, step_v=None, check_every=1, kkt_tol=-1.0,
            relerr_tol=-1.0, relerr_svd=0.0, mode=0, svd_tail_sq=None):
    """Exterior iterations then HALS, as Algorithm 3 from its step 5 on.

    One iteration is a U half then a V half (the V half uses the new U, as
    eq. t_i states).  At the top of each iteration the phase is EXT when U or
    V has a negative entry, else HALS (Algorithm 3 repeats the exterior block
    until U, V are nonnegative, then runs HALS).  The state after k
    iterations is checked when k is a multiple of check_every and at
    k = max_iter; the run stops there when U, V >= 0 and kappa <= kkt_tol or
    relerr - relerr_svd <= relerr_tol (a negative tolerance disables a test).

    mode 0 is the full method; mode 1 clips the rotated factors to the
    orthant and runs HALS only (the projection ablation); mode 2 takes the
    fixed row step of fixed_row_step in the exterior phase (the step-size
    ablation); mode 3 stops as soon as the factors are feasible (F-eNMF).

    Returns (U, V, report) where report holds the steps, counters, the last
    check and the list of all checks.
    """
    X = _f64(X)
    U, V = _f64(U).copy(), _f64(V).copy()
    if mode == 1:
        U, V = np.maximum(U, 0.0), np.maximum(V, 0.0)
    su0, sv0 = resolve_steps(U, V, ext_iters)
    su = su0 if step_u is None or step_u <= 0 else float(step_u)
    sv = sv0 if step_v is None or step_v <= 0 else float(step_v)
    checks = []
    k = 0
    ext_done = 0
    converged = False
    while True:
        if k % check_every == 0 or k == max_iter:
            rep = kkt(X, U, V, svd_tail_sq)
            rep["k"] = k
            checks.append(rep)
            feasible = U.min() >= 0 and V.min() >= 0
            if feasible and ((kkt_tol >= 0 and rep["kkt"] <= kkt_tol) or
                             (relerr_tol >= 0 and rep["relerr"] - relerr_svd <= relerr_tol) or
                             mode == 3):
                converged = True
                break
            if k == max_iter:
                break
        phase = EXT if (U < 0).any() or (V < 0).any() else HALS
        P, G = X @ V, V.T @ V
        fixed = mode == 2
        U = ext_half(U, P, G, su, pbcd_eps, pbcd_max_iter, fixed) if phase == EXT else hals_half(U, P, G)
        Q, H = X.T @ U, U.T @ U
        V = ext_half(V, Q, H, sv, pbcd_eps, pbcd_max_iter, fixed) if phase == EXT else hals_half(V, Q, H)
        ext_done += phase == EXT
        k += 1
    report = dict(checks[-1])
    report.update(iters=k, ext_iters_done=ext_done, converged=converged,
                  step_u=su, step_v=sv, checks=checks)
    return U, V, report


def enmf(X, r, omega=None, power_iters=2, rho0=1.0, rot_max_iter=100, rot_tol=1e-10,
         **iter_opts):
    """Algorithm 3 end to end: SVD init, ADMM rotation, exterior + HALS."""
    if omega is None:
        Us, Vs, sigma, rsvd = svd_init_exact(X, r)
    else:
        Us, Vs, sigma, rsvd = svd_init_randomized(X, r, omega, power_iters)
    U, V, R, steps, g0, g1 = rotate(Us, Vs, rho0, rot_max_iter, rot_tol)
    tail = float(np.sum(_f64(X) ** 2)) - float(np.sum(sigma ** 2))
    iter_opts.setdefault("relerr_svd", rsvd)
    U, V, rep = iterate(X, U, V, svd_tail_sq=tail, **iter_opts)
    rep.update(sigma=sigma, relerr_svd=rsvd, R=R, rot_steps=steps,
               neg_mass_before=g0, neg_mass_after=g1)
    return U, V, rep
