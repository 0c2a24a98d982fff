"""GPU parity of the sparse-X path (compressed sparse rows, the paper's sparse
text collections) against the FP64 oracle, through the C ABI.

* X B and X^T A element by element under the float32 accumulation bound
  (n_i + 4) 2^-24 (|X| |B|)_ic, n_i the nonzeros of the output's row, on
  ragged shapes, empty rows and columns, an all-zero X, every lane-group
  width (k <= 16, <= 32, <= 64, > 64), rows and columns longer than the
  1024-nonzero pieces and rows and columns cut at the 65,536-wide panels of
  the gathered factor; the result is the same on every run;
* svd_init, the iteration (1, 12 and 200 iterations from the oracle's
  rotated point), objective/KKT and a whole solve against the oracle on the
  dense matrix the compressed rows describe, to the bars of the dense
  float32 path;
* the Reuters-shaped matrix (804,414 x 47,236, about 0.16% nonzero) at
  r = 40: sampled rows of both products against the oracle's row-by-row
  definition;
* malformed matrices and calls that do not take a sparse X raise.
"""

import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from paper_2605_19325_amd import enmf, inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
EPS32 = 2.0 ** -24


def say(msg):
    print(msg, flush=True)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def host(t):
    return t.detach().cpu().double().numpy()


def random_csr(m, n, density, seed, long_rows=(), long_cols=(), empty_rows=(), empty_cols=()):
    """Uniform random pattern plus the listed full rows / columns, minus the
    listed empty ones; values U(0, 1].  Returns (rowptr, colind, vals)."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    for i in long_rows:
        mask[i, :] = True
    for j in long_cols:
        mask[:, j] = True
    for i in empty_rows:
        mask[i, :] = False
    for j in empty_cols:
        mask[:, j] = False
    vals = (1.0 - rng.random((m, n))).astype(np.float32)
    rows, cols = np.nonzero(mask)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rowptr[1:])
    return rowptr, cols.astype(np.int32), vals[rows, cols]


def dense_of(rp, ci, v, shape):
    return O.csr_to_dense(rp, ci, v, shape)


def product_bound(Xd, B, counts):
    return (counts[:, None] + 4.0) * EPS32 * (np.abs(Xd) @ np.abs(B)) + 1e-30


@pytest.mark.parametrize("m,n,k,density,extra", [
    (1, 1, 1, 1.0, {}),
    (7, 5, 3, 0.5, {"empty_rows": (2,), "empty_cols": (4,)}),
    (130, 515, 16, 0.05, {}),
    (300, 200, 20, 0.1, {"empty_rows": (0, 299)}),
    (257, 3000, 49, 0.02, {"long_rows": (5, 100, 256)}),
    (2500, 60, 40, 0.05, {"long_cols": (0, 33, 59)}),
    (400, 350, 80, 0.03, {}),
    (64, 64, 64, 0.9, {}),
    (70000, 300, 16, 0.01, {"long_cols": (5,)}),
    (300, 70000, 24, 0.01, {"long_rows": (3,)}),
])
def test_sparse_products_parity(lib, m, n, k, density, extra):
    say(f"sparse products {m}x{n} k={k} density {density} {extra}")
    rp, ci, v = random_csr(m, n, density, m + n + k, **extra)
    Xs = lib.sparse(rp, ci, v, (m, n))
    Xd = dense_of(rp, ci, v, (m, n))
    rng = np.random.default_rng(k)
    B = rng.standard_normal((n, k)).astype(np.float32)
    A = rng.standard_normal((m, k)).astype(np.float32)
    P = lib.xv(Xs, to_dev(B))
    Q = lib.xtu(Xs, to_dev(A))
    rows_n = np.diff(rp).astype(np.float64)
    cols_n = np.bincount(ci, minlength=n).astype(np.float64)
    Pd, Qd = Xd @ B.astype(np.float64), Xd.T @ A.astype(np.float64)
    assert np.all(np.abs(host(P) - Pd) <= product_bound(Xd, B.astype(np.float64), rows_n))
    assert np.all(np.abs(host(Q) - Qd) <= product_bound(Xd.T, A.astype(np.float64), cols_n))
    # empty rows and columns give exact zeros
    assert np.all(host(P)[rows_n == 0] == 0.0) and np.all(host(Q)[cols_n == 0] == 0.0)
    # the same bits on a second run
    assert torch.equal(P, lib.xv(Xs, to_dev(B))) and torch.equal(Q, lib.xtu(Xs, to_dev(A)))
    Xs.close()


def test_all_zero_sparse_x(lib):
    say("sparse X with no stored entries")
    rp = np.zeros(6, dtype=np.int64)
    Xs = lib.sparse(rp, np.zeros(0, np.int32), np.zeros(0, np.float32), (5, 4))
    P = lib.xv(Xs, to_dev(np.ones((4, 3))))
    Q = lib.xtu(Xs, to_dev(np.ones((5, 3))))
    assert float(P.abs().max()) == 0.0 and float(Q.abs().max()) == 0.0
    U = to_dev(np.ones((5, 2)))
    V = to_dev(np.ones((4, 2)))
    k = lib.objective_kkt(Xs, U, V)
    assert k["f"] == 0.5 * 5 * 4 * 4.0
    assert k["relerr"] == 0.0
    Xs.close()


@pytest.fixture(scope="module")
def sparse_small():
    """The 500 x 400 low-rank workload with every entry below the 60th
    percentile dropped (40% of the entries stored), r = 10."""
    X, r = inputs.config_small()
    Xt = np.where(X >= np.quantile(X, 0.6), X, 0.0).astype(np.float32)
    rows, cols = np.nonzero(Xt)
    rp = np.zeros(X.shape[0] + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=X.shape[0]), out=rp[1:])
    om = inputs.omega(X.shape[1], r + 10, 7)
    return Xt, (rp, cols.astype(np.int32), Xt[rows, cols]), r, om


def test_sparse_svd_init_parity(lib, sparse_small):
    Xt, csr, r, om = sparse_small
    say("sparse svd_init vs the oracle on the dense matrix, 500x400 r=10")
    Xs = lib.sparse(*csr, Xt.shape)
    Uo, Vo, so, rso = O.svd_init_randomized(Xt, r, om, 2)
    U, V, sg, rs = lib.svd_init(Xs, r, to_dev(om), 10, 2)
    say(f"  |dUV|/|UV| {rel(host(U) @ host(V).T, Uo @ Vo.T):.2e} relerr_svd {rs:.9e} oracle {rso:.9e}")
    assert rel(host(U) @ host(V).T, Uo @ Vo.T) <= 1e-5
    assert rel(sg, so) <= 1e-6
    assert abs(rs - rso) <= 1e-7
    Xs.close()


def _rotated_start(X, r, om):
    Uo, Vo, _, rso = O.svd_init_randomized(X, r, om, 2)
    Ur, Vr, *_ = O.rotate(Uo.astype(np.float32), Vo.astype(np.float32), 1.0, 20, 0.0)
    return Ur.astype(np.float32), Vr.astype(np.float32), rso


@pytest.mark.parametrize("iters", [1, 12, 200])
def test_sparse_iterate_parity(lib, sparse_small, iters):
    Xt, csr, r, om = sparse_small
    say(f"sparse iterate, {iters} iterations from the oracle's rotated point")
    Xs = lib.sparse(*csr, Xt.shape)
    U0, V0, rso = _rotated_start(Xt, r, om)
    Uo, Vo, ro = O.iterate(Xt, U0, V0, max_iter=iters, relerr_svd=rso)
    U, V = to_dev(U0), to_dev(V0)
    rep = lib.iterate(Xs, U, V, max_iter=iters, relerr_svd=rso)
    say(f"  |dU|/|U| {rel(host(U), Uo):.2e} |dV|/|V| {rel(host(V), Vo):.2e} "
        f"f {rep['f']:.9e} oracle {ro['f']:.9e} ext {rep['ext_iters_done']}")
    assert rep["iters"] == iters and rep["ext_iters_done"] == ro["ext_iters_done"]
    assert rel(host(U), Uo) <= 1e-4 and rel(host(V), Vo) <= 1e-4
    if iters == 200:
        assert abs(rep["f"] - ro["f"]) <= 1e-5 * ro["f"]
        assert rep["kkt"] <= 1e-5 and abs(rep["kkt"] - ro["kkt"]) <= 1e-6
    Xs.close()


def test_sparse_objective_kkt_parity(lib, sparse_small):
    Xt, csr, r, om = sparse_small
    say("sparse objective/kkt vs the oracle")
    Xs = lib.sparse(*csr, Xt.shape)
    rng = np.random.default_rng(0)
    U0 = np.abs(rng.standard_normal((Xt.shape[0], r))).astype(np.float32)
    V0 = rng.standard_normal((Xt.shape[1], r)).astype(np.float32)
    k = lib.objective_kkt(Xs, to_dev(U0), to_dev(V0), 0.5)
    ref = O.kkt(Xt, U0, V0)
    for key in ("f", "relerr", "kkt", "kkt_feas", "kkt_pg_u", "kkt_pg_v", "sigma_w", "delta_w", "min_w"):
        assert abs(k[key] - ref[key]) <= 1e-6 * max(1.0, abs(ref[key])), key
    Xs.close()


def test_sparse_text_solve(lib):
    """A whole solve (svd_init, 20 ADMM steps, 150 iterations) on a
    term-document matrix (3000 x 2000, about 1% nonzero, r = 10)."""
    say("sparse text-like solve 3000x2000 r=10 vs the oracle")
    m, n, r = 3000, 2000, 10
    rp, ci, v = inputs.text_counts(m, n, mean_row_nnz=20.0, seed=21)
    Xd = dense_of(rp, ci, v, (m, n))
    om = inputs.omega(n, r + 10, 22)
    Uo, Vo, ro = O.enmf(Xd, r, om, rot_max_iter=20, rot_tol=0.0, max_iter=150)
    Xs = lib.sparse(rp, ci, v, (m, n))
    U, V, rep = lib.solve(Xs, r, to_dev(om), rot_max_iter=20, rot_tol=0.0, max_iter=150)
    say(f"  relerr {rep['relerr']:.8e} oracle {ro['relerr']:.8e} ext {rep['ext_iters_done']} "
        f"(oracle {ro['ext_iters_done']}) |dUV|/|UV| {rel(host(U) @ host(V).T, Uo @ Vo.T):.2e}")
    assert float(U.min()) >= 0.0 and float(V.min()) >= 0.0
    assert abs(rep["relerr"] - ro["relerr"]) <= 1e-5 * ro["relerr"]
    assert rel(host(U) @ host(V).T, Uo @ Vo.T) <= 1e-4
    Xs.close()


def test_reuters_shaped_products(lib):
    """The Reuters-shaped matrix at r = 40: 24 sampled rows of X V (among
    them the longest) and 24 of X^T U (among them the most frequent term,
    split into 1024-nonzero pieces) against the oracle's definitions."""
    (rp, ci, v), (m, n), r = inputs.config_text()
    say(f"Reuters-shaped sparse X {m}x{n} nnz {ci.size} r={r}")
    Xs = lib.sparse(rp, ci, v, (m, n))
    rng = np.random.default_rng(3)
    V = rng.random((n, r)).astype(np.float32)
    U = rng.random((m, r)).astype(np.float32)
    P = lib.xv(Xs, to_dev(V))
    Q = lib.xtu(Xs, to_dev(U))
    torch.cuda.synchronize()
    lens = np.diff(rp)
    deg = np.bincount(ci, minlength=n)
    rows = np.concatenate([[int(np.argmax(lens)), 0, m - 1], rng.integers(0, m, 21)])
    cols = np.concatenate([[int(np.argmax(deg)), 0, n - 1], rng.integers(0, n, 21)])
    Pr = O.csr_rows_times(rp, ci, v, rows, V)
    Qr = O.csr_cols_times(rp, ci, v, cols, U)
    Pg = host(P[torch.as_tensor(rows, device=DEV)])
    Qg = host(Q[torch.as_tensor(cols, device=DEV)])
    # nonnegative operands: |X||B| is the product itself
    bP = (lens[rows, None] + 4.0) * EPS32 * Pr + 1e-30
    bQ = (deg[cols, None] + 4.0) * EPS32 * Qr + 1e-30
    say(f"  max rel err X V {np.max(np.abs(Pg - Pr) / (Pr + 1e-30)):.2e}  "
        f"X^T U {np.max(np.abs(Qg - Qr) / (Qr + 1e-30)):.2e}")
    assert np.all(np.abs(Pg - Pr) <= bP) and np.all(np.abs(Qg - Qr) <= bQ)
    U2, V2 = to_dev(U), to_dev(V)
    k = lib.objective_kkt(Xs, U2, V2)
    assert np.isfinite(k["f"]) and k["f"] > 0
    Xs.close()


def test_sparse_bad_input(lib):
    say("sparse X argument errors")
    rp = np.array([0, 2, 3], dtype=np.int64)
    ok_ci = np.array([0, 2, 1], dtype=np.int32)
    v = np.ones(3, dtype=np.float32)
    Xs = lib.sparse(rp, ok_ci, v, (2, 3))
    Xs.close()
    for ci, vals, shape in [(np.array([2, 0, 1], np.int32), v, (2, 3)),       # unsorted row
                            (np.array([0, 0, 1], np.int32), v, (2, 3)),       # repeated column
                            (np.array([0, 3, 1], np.int32), v, (2, 3)),       # column out of range
                            (ok_ci, np.array([1, np.nan, 1], np.float32), (2, 3))]:
        with pytest.raises(enmf.EnmfError) as e:
            lib.sparse(rp, ci, vals, shape)
        assert e.value.status == 1
    with pytest.raises(enmf.EnmfError):
        lib.sparse(np.array([0, 3, 2], np.int64), ok_ci, v, (2, 3))         # decreasing rowptr
    with pytest.raises(enmf.EnmfError):
        lib.sparse(np.array([0, 2, 4], np.int64), ok_ci, v, (2, 3))         # rowptr[m] != nnz
    Xs = lib.sparse(rp, ok_ci, v, (2, 3))
    # a descriptor whose shape differs from the handle's
    M = enmf.Matrix(Xs._h.value, 3, 3, 0, enmf.CSR, 0)
    P = torch.empty((3, 2), dtype=torch.float32, device=DEV)
    B = to_dev(np.ones((3, 2)))
    st = lib._lib.enmf_xv(lib._h, ctypes.byref(M), ctypes.c_void_p(B.data_ptr()), 2,
                          ctypes.c_void_p(P.data_ptr()))
    assert st == 1
    # eNMC and the server take dense X only
    with pytest.raises(enmf.EnmfError):
        lib.enmc_grad(Xs, torch.zeros((2, 1), dtype=torch.int32, device=DEV), to_dev(np.ones((2, 1))),
                      to_dev(np.ones((3, 1))))
    srv = enmf.Server(lib, hbm_budget_bytes=1 << 26, max_slots=4)
    with pytest.raises(enmf.EnmfError):
        srv.submit(Xs, 1, to_dev(np.ones((3, 2))), oversample=1, max_iter=2)
    srv.stop()
    Xs.close()
