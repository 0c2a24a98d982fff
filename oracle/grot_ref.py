"""Plain FP64 reference of the generalized rotation ADMM (test infrastructure
only): the appendix section on exact NMF, problem eq5 in the split form
eq:admm_form_2, solved by Algorithm alg:rsr.

Given balanced SVD factors U* (m x r) and V* (n x r) of X, find orthogonal
R1, R2 and a positive diagonal Lambda that move (U* R1 Lambda R2,
V* R1 Lambda^-1 R2), whose product is still U* V*^T, toward the nonnegative
orthant: minimise the negativity mass sum h(.), h(q) = max(0, -q).  With
W_svd = [U*; V*] the split variables are W1 = W_svd R1,
W2 = [W11 Lambda; W12 Lambda^-1] and W3 = W2 R2, with scaled duals M, N, P.

Readings where the appendix gives symbols only (also listed with the design
notes):
  * Penalties rho = gamma = t = rho0 sqrt(N r) / ||W_svd||_F, N = m + n, the
    same scale as the plain rotation.
  * Start: R1 = R2 = I, Lambda = I, W1 = W2 = W3 = W_svd, M = N = P = 0.
  * Lambda update: each lambda_i minimises the two gamma terms of f3 over
    lambda > 0.  Its stationary points are the positive real roots of the
    quartic of the appendix; the one with the least value is taken.  A column
    whose W11 or W12 part is zero leaves lambda_i unchanged (the minimum is
    then at 0 or at infinity).
  * Stop after max_iter steps, or once ||R1' - R1||_F + ||R2' - R2||_F +
    ||lambda' - lambda||_2 <= tol (tol = 0 runs exactly max_iter steps).
  * Output (U* R1 Lambda R2, V* R1 Lambda^-1 R2) with the last R1, Lambda, R2.

Nothing here is tuned.  This module never imports the HIP path.
"""

import numpy as np

from . import enmf_ref as E


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def penalty(W, rho0=1.0):
    """rho = gamma = t = rho0 sqrt(N r) / ||W||_F (the reading above)."""
    N, r = W.shape
    return rho0 * np.sqrt(N * r) / np.linalg.norm(W)


def lambda_objective(lam, w11, w12, a21, a22):
    """||a21 - lam w11||^2 + ||a22 - w12 / lam||^2 for one column (the two
    gamma terms of f3 over 2/gamma; a21 = W21 + N1, a22 = W22 + N2)."""
    return float(np.sum((a21 - lam * w11) ** 2) + np.sum((a22 - w12 / lam) ** 2))


def lambda_update(w11, w12, a21, a22, lam_old):
    """lambda minimising lambda_objective over lambda > 0: the positive real
    roots of a l^4 - b l^3 + c l - d = 0 (the quartic of the appendix) with
    a = |w11|^2, b = a21.w11, c = a22.w12, d = |w12|^2, the one of least
    objective.  a = 0 or d = 0 keeps lam_old."""
    a = float(w11 @ w11)
    b = float(a21 @ w11)
    c = float(a22 @ w12)
    d = float(w12 @ w12)
    if a == 0.0 or d == 0.0:
        return lam_old
    roots = np.roots([a, -b, 0.0, c, -d])
    cand = [z.real for z in roots if abs(z.imag) <= 1e-9 * max(1.0, abs(z)) and z.real > 0.0]
    return min(cand, key=lambda l: lambda_objective(l, w11, w12, a21, a22))


def update_w1(W, R1, M, W2, Nd, lam, m, rho, gamma):
    """W1 step of f1 (elementwise closed form of the appendix): rows < m
    (W11) and rows >= m (W12), lambda per column."""
    A = W @ R1 - M
    C = W2 + Nd
    return np.vstack([(rho * A[:m] + gamma * lam * C[:m]) / (rho + gamma * lam ** 2),
                      (rho * A[m:] + (gamma / lam) * C[m:]) / (rho + gamma / lam ** 2)])


def update_w2(W1, Nd, W3, P, R2, lam, m, gamma, t):
    """W2 step of f2 (closed form of the appendix; R2 R2^T = I)."""
    T = (W3 + P) @ R2.T
    return np.vstack([(gamma * W1[:m] * lam - gamma * Nd[:m] + t * T[:m]) / (gamma + t),
                      (gamma * W1[m:] / lam - gamma * Nd[m:] + t * T[m:]) / (gamma + t)])


def rotate_general(U, V, rho0=1.0, max_iter=500, tol=1e-10):
    """Algorithm alg:rsr on W_svd = [U; V].

    Returns (U_out, V_out, R1, lam, R2, steps, g_before, g_after) with g the
    negativity mass of [U; V] and of [U_out; V_out].
    """
    U, V = _f64(U), _f64(V)
    m, r = U.shape
    W = np.vstack([U, V])
    rho = gamma = t = penalty(W, rho0)
    R1, R2, lam = np.eye(r), np.eye(r), np.ones(r)
    W1, W2, W3 = W.copy(), W.copy(), W.copy()
    M, Nd, P = np.zeros_like(W), np.zeros_like(W), np.zeros_like(W)
    steps = 0
    for _ in range(max_iter):
        # f1: W3 (prox of h) and W1 (elementwise), from the previous W2, R1, R2, lambda
        W3 = E.prox_h(W2 @ R2 - P, t)
        W1 = update_w1(W, R1, M, W2, Nd, lam, m, rho, gamma)
        # f2: R1 (Procrustes) and W2 (closed form), with the previous R2 and lambda
        R1n = E.procrustes(W.T @ (W1 + M))
        W2 = update_w2(W1, Nd, W3, P, R2, lam, m, gamma, t)
        # f3: R2 (Procrustes) and lambda (per column)
        R2n = E.procrustes(W2.T @ (W3 + P))
        A21, A22 = W2[:m] + Nd[:m], W2[m:] + Nd[m:]
        lamn = np.array([lambda_update(W1[:m, i], W1[m:, i], A21[:, i], A22[:, i], lam[i])
                         for i in range(r)])
        # duals
        M = M + W1 - W @ R1n
        Nd = Nd + W2 - np.vstack([W1[:m] * lamn, W1[m:] / lamn])
        P = P + W3 - W2 @ R2n
        change = (np.linalg.norm(R1n - R1) + np.linalg.norm(R2n - R2) + np.linalg.norm(lamn - lam))
        R1, R2, lam = R1n, R2n, lamn
        steps += 1
        if tol > 0 and change <= tol:
            break
    Uo = U @ R1 @ np.diag(lam) @ R2
    Vo = V @ R1 @ np.diag(1.0 / lam) @ R2
    return (Uo, Vo, R1, lam, R2, steps, E.negativity_mass(W),
            E.negativity_mass(np.vstack([Uo, Vo])))
