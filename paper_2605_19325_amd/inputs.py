"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and the oracle.

This module only draws random inputs; it holds none of the method's
arithmetic.  Every generator is driven by NumPy's PCG64 ``default_rng`` and
returns float32 arrays (the FP32 data matrix that both sides consume; the
oracle promotes the very same values to float64).  The random test matrix
of the randomized SVD is drawn here too and passed in to both sides.

The workloads stand in for the paper's datasets, which are not available:
an image-patch matrix for the face data, a harmonic spectrogram for the
audio data, a dense rating-like matrix for the recommendation data, and a
stream of small uneven problems for serving.  Shapes and value
distributions follow the configurations listed with the design notes.
"""

import numpy as np


def _sparse_abs_normal(rng, shape, p_zero):
    a = np.abs(rng.standard_normal(shape))
    a[rng.random(shape) < p_zero] = 0.0
    return a


def omega(n, k, seed):
    """Gaussian test matrix (n x k) for the randomized range finder, float32."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, k)).astype(np.float32)


def lowrank_plus_noise(m, n, r, seed, p_zero=0.5, noise=0.01):
    """X = U* V*^T + E with |N(0,1)| factors zeroed w.p. p_zero, E ~ U[0, noise].

    Small exact-structure workload (500 x 400, true rank 10 in the plain
    configuration; also the per-request generator of the served stream).
    Returns (X float32, U*, V*).
    """
    rng = np.random.default_rng(seed)
    Us = _sparse_abs_normal(rng, (m, r), p_zero)
    Vs = _sparse_abs_normal(rng, (n, r), p_zero)
    X = Us @ Vs.T + rng.uniform(0.0, noise, size=(m, n))
    return X.astype(np.float32), Us, Vs


def config_small(seed=1001):
    """m=500, n=400, true rank 10, fit rank 10; returns (X, r)."""
    X, _, _ = lowrank_plus_noise(500, 400, 10, seed)
    return X, 10


def image_patches(m_side=64, n=10000, seed=1002, chunk=500):
    """Image-patch-like dense X: (m_side^2 pixels) x n samples, float32.

    Each column is a sum of 3..8 nonnegative Gaussian blobs on an
    m_side x m_side grid (centre uniform on the grid, width uniform in
    [2, 6] px, weight Gamma(2, 1)), clipped to [0, 1], plus U[0, 0.02] noise.
    Fresh blobs are drawn for every column.
    """
    rng = np.random.default_rng(seed)
    yy, xx = np.meshgrid(np.arange(m_side, dtype=np.float64),
                         np.arange(m_side, dtype=np.float64), indexing="ij")
    yy, xx = yy.reshape(-1), xx.reshape(-1)
    X = np.empty((m_side * m_side, n), dtype=np.float32)
    counts = rng.integers(3, 9, size=n)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        block = np.zeros((m_side * m_side, c1 - c0))
        for c in range(c0, c1):
            k = int(counts[c])
            cy = rng.uniform(0, m_side, k)
            cx = rng.uniform(0, m_side, k)
            sg = rng.uniform(2.0, 6.0, k)
            w = rng.gamma(2.0, 1.0, k)
            d2 = (yy[:, None] - cy[None, :]) ** 2 + (xx[:, None] - cx[None, :]) ** 2
            block[:, c - c0] = (w[None, :] * np.exp(-d2 / (2.0 * sg[None, :] ** 2))).sum(1)
        np.clip(block, 0.0, 1.0, out=block)
        block += rng.uniform(0.0, 0.02, size=block.shape)
        X[:, c0:c1] = block
    return X


def config_image(seed=1002):
    """4096 x 10000 image-patch matrix, r = 49."""
    return image_patches(64, 10000, seed), 49


def spectrogram(m=513, n=20000, r=40, seed=1003, chunk=2000):
    """Spectrogram-like X = (W H) o exp(0.1 N(0,1)), float32.

    W (m x r): harmonic templates, f0 ~ U[5, 60] bins, peaks at k f0 with
    amplitude 1/k and a Gaussian bin profile of width 1.  H (r x n):
    Gamma(0.5, 1) activations, each zeroed w.p. 0.7.
    """
    rng = np.random.default_rng(seed)
    bins = np.arange(m, dtype=np.float64)
    W = np.zeros((m, r))
    for j in range(r):
        f0 = rng.uniform(5.0, 60.0)
        k = 1
        while k * f0 <= m - 1:
            W[:, j] += np.exp(-0.5 * (bins - k * f0) ** 2) / k
            k += 1
    H = rng.gamma(0.5, 1.0, size=(r, n))
    H[rng.random((r, n)) < 0.7] = 0.0
    X = np.empty((m, n), dtype=np.float32)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        X[:, c0:c1] = (W @ H[:, c0:c1]) * np.exp(0.1 * rng.standard_normal((m, c1 - c0)))
    return X


def config_spectrogram(seed=1003):
    return spectrogram(seed=seed), 40


def ratings(m=100000, n=20000, r=20, seed=1004, chunk=5000, rows=None, workers=None):
    """Recommendation-like dense X = clip(U* V*^T + N(0, 0.3^2), 0, 5), float32.

    U*, V* ~ U[0, 0.7].  Generated in row chunks from spawned seed sequences
    so that any row slice can be reproduced on its own (and the chunks can be
    drawn on several threads with identical results).  ``rows`` limits the
    output to the first rows (a row-subsampled slice of the same matrix).
    """
    from concurrent.futures import ThreadPoolExecutor
    import os

    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(2 + (m + chunk - 1) // chunk)
    Us = np.random.default_rng(kids[0]).uniform(0.0, 0.7, size=(m, r))
    Vs = np.random.default_rng(kids[1]).uniform(0.0, 0.7, size=(n, r))
    mm = m if rows is None else min(rows, m)
    X = np.empty((mm, n), dtype=np.float32)

    def fill(ci):
        i0 = ci * chunk
        i1 = min(mm, i0 + chunk)
        rng = np.random.default_rng(kids[2 + ci])
        blk = Us[i0:i1] @ Vs.T + 0.3 * rng.standard_normal((i1 - i0, n))
        X[i0:i1] = np.clip(blk, 0.0, 5.0)

    nchunks = (mm + chunk - 1) // chunk
    workers = workers or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max(1, min(workers, nchunks))) as ex:
        list(ex.map(fill, range(nchunks)))
    return X


def serve_stream(count=4096, seed=1005, m_range=(64, 2048), r_range=(4, 32)):
    """Served-stream request shapes: m, n log-uniform, r uniform; per-request seeds.

    Returns a list of dicts (m, n, r, seed).  Each request's X comes from
    ``lowrank_plus_noise(m, n, r, seed)``.
    """
    rng = np.random.default_rng(seed)
    lo, hi = np.log(m_range[0]), np.log(m_range[1])
    out = []
    for i in range(count):
        m = int(round(np.exp(rng.uniform(lo, hi))))
        n = int(round(np.exp(rng.uniform(lo, hi))))
        r = int(rng.integers(r_range[0], r_range[1] + 1))
        r = min(r, m, n)
        out.append(dict(m=m, n=n, r=r, seed=int(rng.integers(1 << 31))))
    return out


def poisson_arrivals(count, rate, seed):
    """Arrival times (s) of a Poisson process with the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def exact_nmf(m, n, r, seed, sparsity=0.5, dist="uniform"):
    """Exactly factorable X = U0 V0^T with nonnegative, Bernoulli-sparsified factors.

    The paper's exact-factorisation set draws U, V ~ U(0, 1) and zeroes
    entries with a binary mask of sparsity s.  dist='absnormal' uses |N(0,1)|.
    Returns (X float32 exactly representable products are not guaranteed, U0, V0).
    """
    rng = np.random.default_rng(seed)
    draw = (lambda s: rng.uniform(0.0, 1.0, s)) if dist == "uniform" else \
        (lambda s: np.abs(rng.standard_normal(s)))
    U0 = draw((m, r)) * (rng.random((m, r)) >= sparsity)
    V0 = draw((n, r)) * (rng.random((n, r)) >= sparsity)
    return (U0 @ V0.T), U0, V0


def disjoint_support(m, n, r, seed, equal_norms=False):
    """Nonnegative U0, V0 whose columns have disjoint supports, X = U0 V0^T.

    Column j of U0 lives on rows {i : i mod r == j} (likewise V0), entries
    U(0.5, 1.5).  With equal_norms=False each column pair is rescaled so that
    ||u_j|| = ||v_j|| with distinct values across j (a gapped spectrum whose
    singular vectors are the columns themselves); with equal_norms=True every
    column has the same norm (a fully degenerate spectrum).
    """
    rng = np.random.default_rng(seed)
    U0 = np.zeros((m, r))
    V0 = np.zeros((n, r))
    for j in range(r):
        U0[j::r, j] = rng.uniform(0.5, 1.5, size=len(range(j, m, r)))
        V0[j::r, j] = rng.uniform(0.5, 1.5, size=len(range(j, n, r)))
    for j in range(r):
        target = 1.0 if equal_norms else 1.0 + 0.5 * j
        U0[:, j] *= target / np.linalg.norm(U0[:, j])
        V0[:, j] *= target / np.linalg.norm(V0[:, j])
    return U0 @ V0.T, U0, V0


def haar_orthogonal(r, seed, reflect=False):
    """Haar-random orthogonal r x r matrix (QR of a Gaussian with sign fix).

    reflect=True returns one with determinant -1.
    """
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((r, r))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))
    if (np.linalg.det(Q) < 0) != reflect:
        Q[:, 0] = -Q[:, 0]
    return Q


def completion(m, n, r, density, seed, noise=0.01):
    """Matrix-completion workload (eNMC, the recommendation-shaped stand-in for
    rating data): X = U* V*^T + U[0, noise] with U*, V* ~ |N(0, 1)| (each
    entry zeroed with probability 0.5), observed entries drawn independently
    with probability `density`.  Returns (X float32 with NaN at the
    unobserved entries, observed mask bool)."""
    X, _, _ = lowrank_plus_noise(m, n, r, seed, noise=noise)
    rng = np.random.default_rng(seed + 7)
    obs = rng.random((m, n)) < density
    X = X.astype(np.float32)
    X[~obs] = np.nan
    return X, obs


def text_counts(m=804414, n=47236, mean_row_nnz=108.0, seed=1006, topics=40, doc_topics=2,
                background=0.15, zipf_shift=10.0, zipf_power=1.0, topic_shift=3.0, topic_power=1.3,
                row_sigma=0.9, count_rate=0.7):
    """Sparse term-document X in compressed-sparse-row form, the stand-in for
    the paper's sparse text collections (the Reuters matrix, 804,414 x 47,236
    with 99.84% zeros, at the defaults; the Verb counts at small shapes).

    Topic model: each of `topics` topics ranks the terms by its own random
    permutation, and a background distribution by another; term weights
    follow Zipf-Mandelbrot laws, p(rank) proportional to
    1 / (rank + topic_shift)^topic_power in a topic and
    1 / (rank + zipf_shift)^zipf_power in the background.
    Row i (a document) takes round(LogNormal) terms (mean mean_row_nnz,
    log-sd row_sigma, clipped to [1, n]) and `doc_topics` distinct topics with
    Dirichlet(1) weights; each term comes from the background with
    probability `background`, else from one of the row's topics by weight.
    Repeated terms are merged, so rows keep slightly fewer (the defaults give
    about 0.16% density).  Values are TF-IDF-like: (1 + ln c) ln(1 + m / d_j)
    with count c = 1 + Poisson(count_rate) and d_j the number of rows holding
    term j, and each row is scaled to unit Euclidean norm.
    Returns (rowptr int64 (m + 1), colind int32, vals float32), columns
    strictly increasing within each row.
    """
    rng = np.random.default_rng(seed)
    mu = np.log(mean_row_nnz) - 0.5 * row_sigma ** 2
    lens = np.clip(np.rint(rng.lognormal(mu, row_sigma, m)), 1, n).astype(np.int64)
    ranks = np.arange(n, dtype=np.float64)
    w = 1.0 / (ranks + zipf_shift) ** zipf_power
    cdf = np.cumsum(w / w.sum())
    wt = 1.0 / (ranks + topic_shift) ** topic_power
    cdf_t = np.cumsum(wt / wt.sum())
    perms = np.stack([rng.permutation(n) for _ in range(topics + 1)]).astype(np.int32)
    nt = min(doc_topics, topics)
    dtop = np.argsort(rng.random((m, topics)), axis=1)[:, :nt] + 1
    dw = np.cumsum(rng.dirichlet(np.ones(nt), size=m), axis=1)
    total = int(lens.sum())
    keys = np.empty(total, dtype=np.int64)
    rows = np.repeat(np.arange(m, dtype=np.int64), lens)
    step = 1 << 24
    for a in range(0, total, step):
        b = min(total, a + step)
        rw = rows[a:b]
        bg = rng.random(b - a) < background
        u = rng.random(b - a)
        rank = np.where(bg, np.searchsorted(cdf, u, side="right"),
                        np.searchsorted(cdf_t, u, side="right"))
        rank = np.minimum(rank, n - 1)
        pick = (rng.random(b - a)[:, None] > dw[rw, :-1]).sum(axis=1)
        topic = np.where(bg, 0, dtop[rw, pick])
        keys[a:b] = rw * n + perms[topic, rank]
    del rows
    keys = np.unique(keys)
    rows = keys // n
    cols = (keys - rows * n).astype(np.int32)
    del keys
    df = np.bincount(cols, minlength=n)
    idf = np.log1p(m / np.maximum(df, 1))
    vals = (1.0 + np.log1p(rng.poisson(count_rate, cols.size))) * idf[cols]
    norms = np.sqrt(np.bincount(rows, weights=vals * vals, minlength=m))
    vals /= norms[rows]
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rowptr[1:])
    return rowptr, cols, vals.astype(np.float32)


def config_text(seed=1006):
    """Reuters-shaped sparse X (804,414 x 47,236, about 0.16% nonzero), r = 40."""
    return text_counts(seed=seed), (804414, 47236), 40
