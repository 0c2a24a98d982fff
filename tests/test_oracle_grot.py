"""Pins of the generalized-rotation oracle (the appendix section on exact NMF,
Algorithm alg:rsr) against what the mathematics fixes, independent of the
oracle's closed forms:
  * the W1 and W2 steps are stationary points of the parts of f1 and f2 that
    depend on them, written out from the appendix's cost functions (finite
    differences), and these quadratics are convex, so they are the minima;
  * each lambda step is the minimiser of the gamma terms of f3 over
    lambda > 0 (golden-section search on the cost written out);
  * the output pair keeps the product U V^T;
  * on exact-NMF instances of the appendix's sizes (40 x 50, r = 10 and
    80 x 100, r = 20, factors with 10% zeros) the negativity mass reaches
    zero: an exact nonnegative factorisation, which the single-rotation ADMM
    of Algorithm 1 does not reach in as many steps;
  * planted mistakes (Lambda for Lambda^-1 in the V block, a sign of the
    quartic) fail these pins.
"""

import numpy as np

import oracle as O
from oracle import grot_ref as G
from paper_2605_19325_amd import inputs


def golden_section(f, a, b, tol=1e-13):
    g = (np.sqrt(5.0) - 1.0) / 2.0
    c, d = b - g * (b - a), a + g * (b - a)
    while abs(b - a) > tol * max(1.0, abs(a) + abs(b)):
        if f(c) < f(d):
            b = d
        else:
            a = c
        c, d = b - g * (b - a), a + g * (b - a)
    return 0.5 * (a + b)


def _state(seed, m=7, n=6, r=3):
    rng = np.random.default_rng(seed)
    W = rng.standard_normal((m + n, r))
    R1 = np.linalg.qr(rng.standard_normal((r, r)))[0]
    R2 = np.linalg.qr(rng.standard_normal((r, r)))[0]
    lam = rng.uniform(0.5, 2.0, r)
    M, Nd, P, W2, W3 = (rng.standard_normal((m + n, r)) for _ in range(5))
    return W, R1, R2, lam, M, Nd, P, W2, W3, m


def f1_w1_terms(W1, W, R1, M, W2, Nd, lam, m, rho, gamma):
    """The W1-dependent terms of f1 as the appendix writes them."""
    L = np.diag(lam)
    Li = np.diag(1.0 / lam)
    return (rho / 2 * np.sum((W1 - W @ R1 + M) ** 2)
            + gamma / 2 * np.sum((W2[:m] - W1[:m] @ L + Nd[:m]) ** 2)
            + gamma / 2 * np.sum((W2[m:] - W1[m:] @ Li + Nd[m:]) ** 2))


def f2_w2_terms(W2, W1, Nd, W3, P, R2, lam, m, gamma, t):
    """The W2-dependent terms of f2 as the appendix writes them."""
    L = np.diag(lam)
    Li = np.diag(1.0 / lam)
    return (gamma / 2 * np.sum((W2[:m] - W1[:m] @ L + Nd[:m]) ** 2)
            + gamma / 2 * np.sum((W2[m:] - W1[m:] @ Li + Nd[m:]) ** 2)
            + t / 2 * np.sum((W3 - W2 @ R2 + P) ** 2))


def stationary(f, X, h=1e-6):
    """Central-difference gradient of f at X is zero (relative to the scale of f)."""
    scale = max(1.0, abs(f(X)))
    for idx in np.ndindex(*X.shape):
        Xp, Xm = X.copy(), X.copy()
        Xp[idx] += h
        Xm[idx] -= h
        if abs(f(Xp) - f(Xm)) / (2 * h) > 1e-6 * scale:
            return False
    return True


def check_w_steps(upd1, upd2):
    ok = True
    for seed in range(3):
        W, R1, R2, lam, M, Nd, P, W2, W3, m = _state(seed)
        rho, gamma, t = 0.7, 1.3, 0.9
        W1 = upd1(W, R1, M, W2, Nd, lam, m, rho, gamma)
        ok &= stationary(lambda X: f1_w1_terms(X, W, R1, M, W2, Nd, lam, m, rho, gamma), W1)
        W2n = upd2(W1, Nd, W3, P, R2, lam, m, gamma, t)
        ok &= stationary(lambda X: f2_w2_terms(X, W1, Nd, W3, P, R2, lam, m, gamma, t), W2n)
    return bool(ok)


def test_w_steps_minimise_their_cost_terms():
    assert check_w_steps(G.update_w1, G.update_w2)


def test_w_steps_catch_planted_mistake():
    def lam_for_inverse(W, R1, M, W2, Nd, lam, m, rho, gamma):     # Lambda in the V block too
        A, C = W @ R1 - M, W2 + Nd
        return (rho * A + gamma * lam * C) / (rho + gamma * lam ** 2)
    assert not check_w_steps(lam_for_inverse, G.update_w2)


def check_lambda(update):
    rng = np.random.default_rng(7)
    for _ in range(40):
        k = 9
        w11, w12 = rng.standard_normal(k), rng.standard_normal(k)
        a21 = 1.3 * w11 + 0.4 * rng.standard_normal(k)
        a22 = w12 / 1.3 + 0.4 * rng.standard_normal(k)
        f = lambda l: G.lambda_objective(l, w11, w12, a21, a22)
        ls = np.geomspace(1e-3, 1e3, 4001)
        l0 = ls[np.argmin([f(l) for l in ls])]
        lg = golden_section(f, l0 / 1.01, l0 * 1.01)
        got = update(w11, w12, a21, a22, 1.0)
        if abs(got - lg) > 1e-6 * lg and f(got) > f(lg) + 1e-12 * abs(f(lg)):
            return False
    return True


def test_lambda_step_is_the_minimiser():
    assert check_lambda(G.lambda_update)
    # a zero U or V part keeps the previous value
    z = np.zeros(4)
    assert G.lambda_update(z, np.ones(4), np.ones(4), np.ones(4), 0.7) == 0.7
    assert G.lambda_update(np.ones(4), z, np.ones(4), np.ones(4), 0.7) == 0.7


def test_lambda_step_catches_planted_mistake():
    def flipped(w11, w12, a21, a22, lam_old):      # sign of the cubic term
        a, b, c, d = w11 @ w11, a21 @ w11, a22 @ w12, w12 @ w12
        roots = np.roots([a, b, 0.0, c, -d])
        cand = [z.real for z in roots if abs(z.imag) < 1e-9 and z.real > 0]
        return min(cand, key=lambda l: G.lambda_objective(l, w11, w12, a21, a22)) if cand else lam_old
    assert not check_lambda(flipped)


def test_output_keeps_the_product():
    rng = np.random.default_rng(3)
    U, V = rng.standard_normal((30, 4)), rng.standard_normal((25, 4))
    Uo, Vo, R1, lam, R2, steps, g0, g1 = G.rotate_general(U, V, max_iter=60, tol=0.0)
    assert steps == 60
    assert np.linalg.norm(Uo @ Vo.T - U @ V.T) <= 1e-12 * np.linalg.norm(U @ V.T)
    assert np.linalg.norm(R1.T @ R1 - np.eye(4)) <= 1e-12 and np.linalg.norm(R2 @ R2.T - np.eye(4)) <= 1e-12
    assert np.all(lam > 0) and g1 <= g0


def test_exact_instances_reach_the_orthant():
    """The appendix's sizes: the generalized ADMM ends with no negative entry."""
    for (m, n, r, seed) in ((40, 50, 10, 1), (80, 100, 20, 0)):
        X, _, _ = inputs.exact_nmf(m, n, r, seed, sparsity=0.1)
        Us, Vs, _, _ = O.svd_init_exact(X, r)
        Uo, Vo, R1, lam, R2, steps, g0, g1 = G.rotate_general(Us, Vs, max_iter=500, tol=0.0)
        assert g1 == 0.0 and g0 > 10.0
        assert Uo.min() >= 0.0 and Vo.min() >= 0.0
        assert np.linalg.norm(Uo @ Vo.T - X) <= 1e-12 * np.linalg.norm(X)
        _, _, _, _, h0, h1 = O.rotate(Us, Vs, 1.0, 500, 0.0)
        assert h1 > 1e-4 * h0            # the single rotation stays outside
