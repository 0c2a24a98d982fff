"""enmf_xv_static, the allocation-free form of enmf_xv, through the C ABI.

It runs the kernels and launch plan of enmf_xv with its scratch in a fixed
device array, so its product must equal enmf_xv's bit for bit.  Two calls in
a row (the second smaller, so the first leaves stale scratch behind), on the
matrix-core path (k >= 16) and the vector-ALU path (k < 16), float32 and
bfloat16 X; a shape whose scratch exceeds the array is refused before any
launch; a call allocates no device memory.
"""

import numpy as np
import pytest
import torch

from paper_2605_19325_amd import enmf

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)


def data(m, n, k, seed, dtype, lib):
    rng = np.random.default_rng(seed)
    X = torch.from_numpy(rng.random((m, n), dtype=np.float32)).to(DEV)
    if dtype is not torch.float32:
        X = lib.convert(X, dtype)
    B = torch.from_numpy(rng.standard_normal((n, k)).astype(np.float32)).to(DEV)
    return X, B


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_static_matches_workspace_form(lib, dtype):
    for m, n, k, seed in ((1500, 3001, 49, 1), (333, 517, 20, 2), (257, 130, 7, 3)):
        say(f"xv_static {dtype} m={m} n={n} k={k}")
        X, B = data(m, n, k, seed, dtype, lib)
        P_ws = lib.xv(X, B)
        P_st = lib.xv_static(X, B)
        torch.cuda.synchronize()
        assert torch.equal(P_ws, P_st), (m, n, k)
        # and the product itself, against float64
        Xd = X.float().cpu().double().numpy()
        ref = Xd @ B.cpu().double().numpy()
        bound = (8 * 2.0 ** -24 * np.sqrt(n) + 2.0 ** -21) * (np.abs(Xd) @ np.abs(B.cpu().double().numpy()))
        assert np.all(np.abs(P_st.cpu().double().numpy() - ref) <= bound + 1e-30)


def test_static_refuses_oversized_scratch(lib):
    # m * k * 4 bytes of split partials alone exceed the 64 MiB array
    m, n, k = 300000, 64, 64
    say(f"xv_static oversized m={m} n={n} k={k}: refused before any launch")
    X = torch.zeros((m, n), dtype=torch.float32, device=DEV)
    B = torch.zeros((n, k), dtype=torch.float32, device=DEV)
    P = torch.full((m, k), 7.0, dtype=torch.float32, device=DEV)
    with pytest.raises(enmf.EnmfError) as ei:
        lib.xv_static(X, B, P)
    assert ei.value.status == 2 and "bytes of scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool(torch.all(P == 7.0))          # nothing was launched


def test_static_allocates_nothing(lib):
    X1, B1 = data(2048, 4096, 32, 5, torch.float32, lib)
    X2, B2 = data(700, 900, 40, 6, torch.float32, lib)
    P1 = torch.empty((2048, 32), dtype=torch.float32, device=DEV)
    P2 = torch.empty((700, 40), dtype=torch.float32, device=DEV)
    lib.xv_static(X1, B1, P1)            # first launch loads the kernels
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    lib.xv_static(X2, B2, P2)
    lib.xv_static(X1, B1, P1)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert torch.equal(P1, lib.xv(X1, B1)) and torch.equal(P2, lib.xv(X2, B2))
