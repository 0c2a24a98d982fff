"""Plain FP64 reference of the quantities of a sparse X given in compressed
sparse rows (test infrastructure only).

The paper runs eNMF on sparse text collections (the Verb counts and the
large Reuters matrix of its experiments and appendix table).  The method
itself is unchanged: X enters only through X V, X^T U, ||X||_F^2 and the
objective of eq. 1, so the dense reference of enmf_ref applies to the dense
matrix these functions build.  At shapes too large to densify, the functions
below give single rows of the products from their definitions.

Compressed sparse rows: row i holds the entries vals[p] at columns
colind[p] for rowptr[i] <= p < rowptr[i + 1].  Nothing here is tuned.  This
module never imports the HIP path.
"""

import numpy as np


def csr_to_dense(rowptr, colind, vals, shape):
    """The dense m x n float64 matrix described by the compressed rows
    (entries not stored are zero; a repeated column would add up)."""
    m, n = shape
    X = np.zeros((m, n))
    for i in range(m):
        a, b = int(rowptr[i]), int(rowptr[i + 1])
        np.add.at(X[i], np.asarray(colind[a:b], dtype=np.int64), np.asarray(vals[a:b], np.float64))
    return X


def csr_rows_times(rowptr, colind, vals, rows, B):
    """Rows `rows` of X B (B: n x k): row i is sum over its stored entries of
    x_ij B[j], in float64."""
    B = np.asarray(B, dtype=np.float64)
    out = np.zeros((len(rows), B.shape[1]))
    for t, i in enumerate(rows):
        a, b = int(rowptr[i]), int(rowptr[i + 1])
        v = np.asarray(vals[a:b], dtype=np.float64)
        out[t] = v @ B[np.asarray(colind[a:b], dtype=np.int64)]
    return out


def csr_cols_times(rowptr, colind, vals, cols, A):
    """Rows `cols` of X^T A (A: m x k): row j is sum over the stored entries
    of column j of x_ij A[i], in float64."""
    A = np.asarray(A, dtype=np.float64)
    m = len(rowptr) - 1
    row_of = np.repeat(np.arange(m), np.diff(np.asarray(rowptr, dtype=np.int64)))
    out = np.zeros((len(cols), A.shape[1]))
    for t, j in enumerate(cols):
        sel = np.flatnonzero(np.asarray(colind) == j)
        out[t] = np.asarray(vals[sel], dtype=np.float64) @ A[row_of[sel]]
    return out


def csr_sumsq(vals):
    """||X||_F^2 in float64 (the squares of the stored entries)."""
    v = np.asarray(vals, dtype=np.float64)
    return float(v @ v)
