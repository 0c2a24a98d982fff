"""Pins of the eNMC oracle (appendix "Exterior NMC algorithm") against what
the mathematics fixes, independent of the oracle's own code:
  * with every entry observed the masked objective, gradients, check and PBCD
    are those of eNMF (a separate implementation);
  * the masked gradients match central finite differences of fhat;
  * the masked optimal row step is the exact minimiser of the masked row
    objective (golden-section search on the objective evaluated literally);
  * softImpute-ALS at lambda = 0 never raises fhat, completes an exactly
    low-rank matrix from a random 60% of its entries when started near its
    factors, and with the full mask reaches the Eckart-Young error of the
    rank-r SVD;
  * planted mistakes fail these pins.
"""

import numpy as np

import oracle as O


def golden_section(f, a, b, tol=1e-12):
    g = (np.sqrt(5.0) - 1.0) / 2.0
    c, d = b - g * (b - a), a + g * (b - a)
    while abs(b - a) > tol * max(1.0, abs(a) + abs(b)):
        if f(c) < f(d):
            b = d
        else:
            a = c
        c, d = b - g * (b - a), a + g * (b - a)
    return 0.5 * (a + b)


def _case(seed, m=24, n=18, r=3, density=0.6):
    rng = np.random.default_rng(seed)
    X = rng.random((m, n))
    M = (rng.random((m, n)) < density).astype(np.float64)
    U = rng.standard_normal((m, r))
    V = rng.random((n, r))
    return X, M, U, V


def test_full_mask_reduces_to_enmf():
    X, _, U, V = _case(1)
    M = np.ones_like(X)
    assert abs(O.masked_objective(X, M, U, V) - O.objective(X, U, V)) <= 1e-12 * O.objective(X, U, V)
    gU, gV = O.masked_gradients(X, M, U, V)
    hU, hV = O.gradients(X, U, V)
    assert np.allclose(gU, hU, rtol=1e-12, atol=1e-12) and np.allclose(gV, hV, rtol=1e-12, atol=1e-12)
    mask = U >= 0
    a = O.masked_pbcd(U, X, M, V, mask, 3)
    b, _ = O.pbcd(U, X @ V, V.T @ V, mask, 0.0, 3)
    assert np.allclose(a, b, rtol=1e-11, atol=1e-12)
    Up, Vp = np.abs(U), V
    k1, k2 = O.masked_kkt(X, M, Up, Vp), O.kkt(X, Up, Vp)
    for key in ("f", "relerr", "kkt", "kkt_pg_u", "kkt_pg_v"):
        assert abs(k1[key] - k2[key]) <= 1e-12 * max(1.0, abs(k2[key])), key


def check_masked_gradients(grad):
    X, M, U, V = _case(2, m=7, n=6, r=2)
    gU, gV = grad(X, M, U, V)
    h = 1e-6
    for (A, g) in ((U, gU), (V, gV)):
        for idx in [(0, 0), (3, 1), (5, 0)]:
            Ap, Am = A.copy(), A.copy()
            Ap[idx] += h
            Am[idx] -= h
            args_p = (Ap, V) if A is U else (U, Ap)
            args_m = (Am, V) if A is U else (U, Am)
            fd = (O.masked_objective(X, M, *args_p) - O.masked_objective(X, M, *args_m)) / (2 * h)
            if abs(fd - g[idx]) > 1e-6 * max(1.0, abs(fd)):
                return False
    return True


def test_masked_gradients_finite_differences():
    assert check_masked_gradients(O.masked_gradients)


def test_masked_gradients_catch_planted_mistake():
    def unmasked(X, M, U, V):     # the mask dropped from the residual
        D = U @ V.T - X
        return D @ V, D.T @ U
    assert not check_masked_gradients(unmasked)


def check_masked_step(pbcd):
    X, M, U, V = _case(3, m=10, n=14, r=3)
    U = np.where(U < -1.2, U, np.abs(U))       # a few negatives outside the mask
    mask = U >= 0
    U1 = pbcd(U, X, M, V, mask, 1)
    D = M * (U @ V.T - X)
    g = mask * (D @ V)
    for i in range(U.shape[0]):
        if not np.any(g[i]):
            continue
        row = lambda d: float(np.sum((M[i] * (X[i] - (U[i] - d * g[i]) @ V.T)) ** 2))
        d_star = golden_section(row, -50.0, 50.0)
        want = np.where(mask[i], np.maximum(0.0, U[i] - d_star * g[i]), U[i])
        if not np.allclose(U1[i], want, atol=1e-7):
            return False
    return True


def test_masked_optimal_step_is_exact_line_minimiser():
    assert check_masked_step(O.masked_pbcd)


def test_masked_step_catches_planted_mistake():
    def unmasked_den(U, X, M, V, mask, max_iter=5):   # the denominator of eNMF's d_i
        U = U.copy()
        for _ in range(max_iter):
            g = mask * ((M * (U @ V.T - X)) @ V)
            num = np.sum(g * g, 1)
            den = np.einsum("ia,ab,ib->i", g, V.T @ V, g)
            d = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
            U = np.where(mask, np.maximum(0.0, U - d[:, None] * g), U)
        return U
    assert not check_masked_step(unmasked_den)


def _lowrank(seed, m=60, n=50, r=4, density=0.6, factors=False):
    rng = np.random.default_rng(seed)
    U = np.abs(rng.standard_normal((m, r)))
    V = np.abs(rng.standard_normal((n, r)))
    M = (rng.random((m, n)) < density).astype(np.float64)
    if factors:
        return U @ V.T, M, rng.standard_normal((n, r + 6)), U, V, rng
    return U @ V.T, M, rng.standard_normal((n, r + 6))


def check_als(als):
    """fhat never rises from the randomized-SVD start (EM is monotone; from
    such a start it may stall at a non-global stationary point), and from a
    start near the true factors it completes the missing entries exactly."""
    X, M, om, Ut, Vt, rng = _lowrank(4, factors=True)
    U0, V0, _, _ = O.svd_init_randomized(M * X, 4, om)
    U, V, hist = als(X, M, U0, V0, 120)
    if any(hist[i + 1] > hist[i] * (1 + 1e-10) + 1e-18 for i in range(len(hist) - 1)):
        return False
    Un = Ut + 0.05 * rng.standard_normal(Ut.shape)
    Vn = Vt + 0.05 * rng.standard_normal(Vt.shape)
    U, V, hist = als(X, M, Un, Vn, 200)
    miss = 1.0 - M
    return np.linalg.norm(miss * (X - U @ V.T)) <= 1e-6 * np.linalg.norm(miss * X)


def test_softimpute_als_monotone_and_completes():
    assert check_als(O.softimpute_als)


def test_softimpute_als_catches_planted_mistake():
    def zero_fill(X, M, U, V, iters):     # no imputation: least squares on M o X
        U, V = U.copy(), V.copy()
        hist = []
        for _ in range(iters):
            Xs = M * X
            U = Xs @ V @ np.linalg.inv(V.T @ V)
            V = Xs.T @ U @ np.linalg.inv(U.T @ U)
            hist.append(O.masked_objective(X, M, U, V))
        return U, V, hist
    assert not check_als(zero_fill)


def test_softimpute_als_full_mask_reaches_eckart_young():
    rng = np.random.default_rng(5)
    X = rng.random((40, 30))
    M = np.ones_like(X)
    r = 3
    s = np.linalg.svd(X, compute_uv=False)
    tail = float(np.sum(s[r:] ** 2))
    om = rng.standard_normal((30, r + 6))
    U0, V0, _, _ = O.svd_init_randomized(X, r, om, 0)
    U, V, hist = O.softimpute_als(X, M, U0, V0, 200)
    assert abs(2.0 * hist[-1] - tail) <= 1e-8 * tail


def test_enmc_reaches_feasible_low_error():
    X, M, om = _lowrank(6)      # a seed whose randomized-SVD start completes X
    U, V, rep = O.enmc(X, M, 4, om, als_iters=100, rot_max_iter=50, rot_tol=0.0, max_iter=150)
    assert U.min() >= 0 and V.min() >= 0
    assert rep["ext_iters_done"] == 10
    assert rep["relerr"] <= 1e-2
