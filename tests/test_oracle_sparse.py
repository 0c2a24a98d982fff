"""Pins of the sparse-X oracle (compressed sparse rows) against a library
routine, scipy.sparse, which is independent of the oracle's code:
  * the dense matrix, sampled rows of X B and of X^T A and ||X||_F^2 agree
    with scipy's conversion and sparse products;
  * planted mistakes (an off-by-one row range, a transposed index) fail;
and of the Reuters-shaped generator's structure (host logic): offsets,
strictly increasing columns, unit rows, the density and the heavy-tailed
column degrees of a term-document matrix.
"""

import numpy as np
import scipy.sparse as sps

import oracle as O
from paper_2605_19325_amd import inputs


def _case(seed, m=60, n=45, density=0.1):
    rng = np.random.default_rng(seed)
    A = sps.random(m, n, density=density, random_state=rng, format="csr", dtype=np.float64)
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float32), A


def check_products(to_dense, rows_times, cols_times):
    rp, ci, v, A = _case(1)
    A = sps.csr_matrix((v.astype(np.float64), ci, rp), shape=A.shape)
    if not np.array_equal(to_dense(rp, ci, v, A.shape), A.toarray()):
        return False
    rng = np.random.default_rng(2)
    B = rng.standard_normal((A.shape[1], 7))
    C = rng.standard_normal((A.shape[0], 5))
    rows = [0, 3, 17, A.shape[0] - 1]
    cols = [0, 9, A.shape[1] - 1]
    if not np.allclose(rows_times(rp, ci, v, rows, B), (A @ B)[rows], rtol=1e-13, atol=1e-13):
        return False
    return np.allclose(cols_times(rp, ci, v, cols, C), (A.T @ C)[cols], rtol=1e-13, atol=1e-13)


def test_sparse_oracle_matches_scipy():
    assert check_products(O.csr_to_dense, O.csr_rows_times, O.csr_cols_times)
    _, _, v, A = _case(3)
    assert abs(O.csr_sumsq(v) - sps.linalg.norm(sps.csr_matrix(
        (v.astype(np.float64), A.indices, A.indptr), shape=A.shape)) ** 2) <= 1e-12 * O.csr_sumsq(v)


def test_sparse_oracle_catches_planted_mistakes():
    def short_rows(rowptr, colind, vals, rows, B):       # drops the last entry of each row
        out = np.zeros((len(rows), B.shape[1]))
        for t, i in enumerate(rows):
            a, b = int(rowptr[i]), int(rowptr[i + 1]) - 1
            out[t] = np.asarray(vals[a:b], np.float64) @ B[colind[a:b]]
        return out

    def swapped_dense(rowptr, colind, vals, shape):      # transposed index
        return O.csr_to_dense(rowptr, colind, vals, shape).T.reshape(shape)

    assert not check_products(O.csr_to_dense, short_rows, O.csr_cols_times)
    assert not check_products(swapped_dense, O.csr_rows_times, O.csr_cols_times)


def test_text_generator_structure():
    m, n = 3000, 2000
    rp, ci, v = inputs.text_counts(m, n, mean_row_nnz=20.0, seed=5)
    assert rp.dtype == np.int64 and ci.dtype == np.int32 and v.dtype == np.float32
    assert rp[0] == 0 and rp[-1] == ci.size and np.all(np.diff(rp) >= 1)
    for i in range(0, m, 97):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0) and row.min() >= 0 and row.max() < n
    assert np.all(v > 0)
    norms = np.sqrt(np.add.reduceat(v.astype(np.float64) ** 2, rp[:-1]))
    assert np.allclose(norms, 1.0, atol=1e-6)
    density = ci.size / (m * n)
    assert 0.007 <= density <= 0.01
    deg = np.bincount(ci, minlength=n)
    # term degrees are heavy tailed: the top 10% of terms hold over 25% of the
    # entries and the most frequent term appears in over 5x the median's rows
    top = np.sort(deg)[::-1][: n // 10].sum()
    assert top > 0.25 * ci.size and deg.max() > 5 * np.median(deg)
    again = inputs.text_counts(m, n, mean_row_nnz=20.0, seed=5)
    assert all(np.array_equal(a, b) for a, b in zip((rp, ci, v), again))
