"""GPU parity of the building blocks against the FP64 oracle's definitions.

Streaming products X B and X^T A are compared element by element with the
float64 product under the float32 accumulation bound
|P - P64| <= c * eps32 * sqrt(n) * (|X| |B|) elementwise (c = 8); Grams are
float64 accumulations of exact float32 products (1e-12 relative);
the BF16 conversion is bit-exact against round-to-nearest-even.
"""

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


def to_dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def ref_bound(Xd, Bd, n, split=1):
    """float32 accumulation bound plus the representation error of the three-term
    bfloat16 splits the matrix-core forms use: split = 1 for the factor alone
    (bfloat16 X; |b - b1 - b2 - b3| <= 2^-24 |b|), 2 for X and the factor (float32
    X through the bfloat16 matrix cores, whose three dropped cross terms add at
    most 2^-23), 0 for none."""
    extra = {0: 0.0, 1: 2.0 ** -23, 2: 2.0 ** -21}[split]
    c = 8 * EPS32 * np.sqrt(n) + extra
    return c * (np.abs(Xd) @ np.abs(Bd)) + 1e-30


def mfma_split(dt, k, product):
    """Split class of the product's matrix-core form (k >= 16) for X stored as dt."""
    if k < 16:
        return 0
    if dt == "bf16":
        return 1
    return 2 if dt == "f32" else 0


SHAPES = [(1, 1), (7, 5), (65, 129), (300, 1000), (130, 515), (1000, 77)]


@pytest.mark.parametrize("m,n", SHAPES)
@pytest.mark.parametrize("k", [1, 3, 10, 16, 20, 49, 64, 80])
@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_xv_xtu(lib, m, n, k, dt):
    say(f"xv/xtu m={m} n={n} k={k} dt={dt}")
    rng = np.random.default_rng(m * 1000 + n + k)
    X = rng.random((m, n)).astype(np.float32)
    B = rng.standard_normal((n, k)).astype(np.float32)
    A = rng.standard_normal((m, k)).astype(np.float32)
    Xt = torch.from_numpy(X).to(DEV)
    if dt == "bf16":
        Xt = lib.convert(Xt, torch.bfloat16)
        Xd = Xt.float().cpu().double().numpy()
    else:
        Xd = X.astype(np.float64)
    P = lib.xv(Xt, torch.from_numpy(B).to(DEV)).cpu().double().numpy()
    Q = lib.xtu(Xt, torch.from_numpy(A).to(DEV)).cpu().double().numpy()
    Bd, Ad = B.astype(np.float64), A.astype(np.float64)
    assert np.all(np.abs(P - Xd @ Bd) <= ref_bound(Xd, Bd, n, mfma_split(dt, k, "xv")))
    assert np.all(np.abs(Q - Xd.T @ Ad) <= ref_bound(Xd.T, Ad, m, mfma_split(dt, k, "xtu")))


@pytest.fixture(scope="module")
def valu_lib():
    """A second context whose products always take the vector-ALU form."""
    import os
    os.environ["ENMF_FORCE_VALU"] = "1"
    try:
        ctx = enmf.Context(0)
    finally:
        del os.environ["ENMF_FORCE_VALU"]
    yield ctx
    ctx.close()


@pytest.mark.parametrize("m,n,k", [(300, 1000, 20), (130, 515, 49), (1000, 77, 80), (65, 129, 16)])
@pytest.mark.parametrize("dt", ["f32", "bf16", "f16"])
def test_valu_form_matches_fp64(valu_lib, lib, m, n, k, dt):
    say(f"vector-ALU form m={m} n={n} k={k} dt={dt}")
    rng = np.random.default_rng(m + n + k)
    X = rng.random((m, n)).astype(np.float32)
    B = rng.standard_normal((n, k)).astype(np.float32)
    A = rng.standard_normal((m, k)).astype(np.float32)
    Xt = torch.from_numpy(X).to(DEV)
    if dt != "f32":
        Xt = lib.convert(Xt, torch.bfloat16 if dt == "bf16" else torch.float16)
    Xd = Xt.float().cpu().double().numpy()
    for ctx, form in ((valu_lib, "valu"), (lib, "mfma")):
        P = ctx.xv(Xt, torch.from_numpy(B).to(DEV)).cpu().double().numpy()
        Q = ctx.xtu(Xt, torch.from_numpy(A).to(DEV)).cpu().double().numpy()
        sv = 0 if form == "valu" or dt == "f16" else mfma_split(dt, k, "xv")
        su = 0 if form == "valu" or dt == "f16" else mfma_split(dt, k, "xtu")
        assert np.all(np.abs(P - Xd @ B) <= ref_bound(Xd, B.astype(np.float64), n, sv))
        assert np.all(np.abs(Q - Xd.T @ A) <= ref_bound(Xd.T, A.astype(np.float64), m, su))


def test_time_products_runs(lib, valu_lib):
    say("kernel timing entry point")
    X = torch.rand((512, 700), device=DEV)
    for ctx in (lib, valu_lib):
        a, b = ctx.time_products(X, 32, reps=3)
        assert a > 0 and b > 0


def test_xv_padded_leading_dimension(lib):
    say("xv ld padding")
    rng = np.random.default_rng(5)
    full = rng.random((50, 136)).astype(np.float32)
    full[:, 130:] = np.nan                      # padding beyond n must never be read into results
    Xt = torch.from_numpy(full).to(DEV)[:, :130]
    B = rng.standard_normal((130, 7)).astype(np.float32)
    P = lib.xv(Xt, torch.from_numpy(B).to(DEV)).cpu().double().numpy()
    Xd = full[:, :130].astype(np.float64)
    assert np.all(np.abs(P - Xd @ B) <= ref_bound(Xd, B.astype(np.float64), 130, 0))
    A = rng.standard_normal((50, 7)).astype(np.float32)
    Q = lib.xtu(Xt, torch.from_numpy(A).to(DEV)).cpu().double().numpy()
    assert np.all(np.abs(Q - Xd.T @ A) <= ref_bound(Xd.T, A.astype(np.float64), 50, 0))


@pytest.mark.parametrize("rows,k", [(1, 1), (33, 5), (1000, 49), (4097, 64), (513, 80)])
def test_gram(lib, rows, k):
    say(f"gram rows={rows} k={k}")
    A = np.random.default_rng(rows + k).standard_normal((rows, k)).astype(np.float32)
    G = lib.gram(torch.from_numpy(A).to(DEV)).cpu().numpy()
    Ad = A.astype(np.float64)
    ref = Ad.T @ Ad
    assert np.allclose(G, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


TORCH_DT = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}


@pytest.mark.parametrize("dt", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("m,n,r,pad", [(1, 1, 1, 0), (37, 70, 3, 0), (300, 517, 20, 0), (129, 640, 49, 0),
                                       (260, 300, 64, 3), (8000, 1280, 20, 8), (20000, 320, 16, 0),
                                       (6600, 1112, 49, 0)])
def test_direct_objective(lib, m, n, r, pad, dt):
    """f = 1/2 ||X - U V^T||^2 of the stored X (the direct float64 residual that
    objective_kkt reports) against the oracle's objective of the same stored
    values widened to float64.  The shapes take the 16-row groups of whole
    64-column runs on aligned rows (vector loads), ragged row groups and column
    runs, padded and unaligned leading dimensions (element loads), and
    contraction widths from 1 to 64."""
    say(f"direct objective {dt} {m}x{n} r={r} ld=n+{pad}")
    rng = np.random.default_rng(m + n + r)
    full = torch.from_numpy(rng.random((m, n + pad)).astype(np.float32)).to(TORCH_DT[dt])
    if pad:
        full[:, n:] = float("nan")                  # padding must never be read into the result
    Xh = full[:, :n]
    U0 = (rng.random((m, r)) / np.sqrt(r)).astype(np.float32)
    V0 = rng.random((n, r)).astype(np.float32)
    Xd = full.to(DEV)[:, :n]
    k = lib.objective_kkt(Xd, to_dev32(U0), to_dev32(V0), 0.5)
    ref = O.objective(Xh.double().numpy(), U0, V0)
    assert abs(k["f"] - ref) <= 1e-10 * ref, (k["f"], ref)


def test_convert_bf16_rne_bitexact(lib):
    say("convert bf16/f16")
    rng = np.random.default_rng(3)
    X = (rng.standard_normal((37, 101)) * 10.0 ** rng.integers(-20, 20, (37, 101))).astype(np.float32)
    X[0, :5] = [0.0, -0.0, np.inf, -np.inf, 1.0 + 2.0 ** -8]   # includes a tie
    Xt = torch.from_numpy(X).to(DEV)
    b = lib.convert(Xt, torch.bfloat16).cpu()
    ref = torch.from_numpy(X).to(torch.bfloat16)
    assert torch.equal(b.view(torch.int16), ref.view(torch.int16))
    h = lib.convert(Xt, torch.float16).cpu()
    assert torch.equal(h.view(torch.int16), torch.from_numpy(X).to(torch.float16).view(torch.int16))
