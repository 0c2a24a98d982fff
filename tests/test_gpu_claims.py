"""GPU checks of behaviour the library's documentation promises.

* Repeatability: two runs of enmf_iterate on the same input give bitwise the
  same factors and report (every reduction runs in a fixed order, no atomics),
  on the matrix-core path (r >= 16) and the vector-ALU path.
* The loop body replayed from a captured HIP graph gives bitwise the result
  of direct launches.
* Resume: 200 iterations equal 100 + 100 when the second call is given the
  push sizes the first one reported (the state of the loop is U, V and the
  resolved steps only).
* A non-finite X: enmf_iterate returns ENMF_ENUMERIC and leaves U, V at the
  iterate whose check found it (here the input factors, finite).
* The rotation's tolerance stop (Algorithm 1 with the stopping rule
  ||R_{k+1} - R_k||_F <= tol looked at every check_every steps): on an
  instance whose ADMM converges, the step count is the first multiple of
  check_every at which the oracle's step change is within tol, and R is the
  oracle's R after that many steps.
"""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2605_19325_amd import enmf, inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def host(t):
    return t.detach().cpu().double().numpy()


def rotated_start(X, r, om):
    Uo, Vo, _, rso = O.svd_init_randomized(X, r, om, 2)
    Ur, Vr, *_ = O.rotate(Uo.astype(np.float32), Vo.astype(np.float32), 1.0, 20, 0.0)
    return Ur.astype(np.float32), Vr.astype(np.float32), rso


@pytest.fixture(scope="module", params=[(900, 700, 24), (500, 400, 10)], ids=["mfma_r24", "valu_r10"])
def problem(request):
    m, n, r = request.param
    X, _, _ = inputs.lowrank_plus_noise(m, n, r, seed=m + r)
    om = inputs.omega(n, r + 10, 5)
    U0, V0, rso = rotated_start(X, r, om)
    return X, r, U0, V0, rso


def test_iterate_is_bitwise_repeatable(lib, problem):
    X, r, U0, V0, rso = problem
    say(f"repeatability {X.shape} r={r}: two runs of 60 iterations")
    Xd = to_dev(X)
    outs = []
    for _ in range(2):
        U, V = to_dev(U0), to_dev(V0)
        rep = lib.iterate(Xd, U, V, max_iter=60, relerr_svd=rso)
        outs.append((U, V, rep))
    (U1, V1, r1), (U2, V2, r2) = outs
    assert torch.equal(U1, U2) and torch.equal(V1, V2)
    for key in ("f", "kkt", "relerr", "iters", "ext_iters_done", "step_u", "step_v"):
        assert r1[key] == r2[key], key


@pytest.mark.parametrize("dt", [torch.float32, torch.bfloat16], ids=["f32", "bf16"])
def test_iterate_independent_of_pitch(lib, problem, dt):
    """X with its rows on 128-byte lines (enmf.pitched) gives bitwise the
    factors and report of the same values at the tight pitch: the pitch
    changes which lines a product fetches, not what it adds up or in what
    order."""
    X, r, U0, V0, rso = problem
    Xd = to_dev(X)
    if dt == torch.bfloat16:
        Xd = lib.convert(Xd, dt).contiguous()
    Xp = enmf.pitched(Xd)
    say(f"pitch {X.shape} r={r} {dt}: ld {Xd.stride(0)} against {Xp.stride(0)}")
    assert Xp.stride(0) * Xp.element_size() % 128 == 0 and torch.equal(Xp, Xd)
    outs = []
    for Xa in (Xd, Xp):
        U, V = to_dev(U0), to_dev(V0)
        rep = lib.iterate(Xa, U, V, max_iter=40, relerr_svd=rso)
        outs.append((U, V, rep))
    (U1, V1, r1), (U2, V2, r2) = outs
    assert torch.equal(U1, U2) and torch.equal(V1, V2)
    for key in ("f", "kkt", "relerr", "iters", "ext_iters_done"):
        assert r1[key] == r2[key], key


def test_iterate_resume(lib, problem):
    X, r, U0, V0, rso = problem
    say(f"resume {X.shape} r={r}: 200 iterations against 100 + 100")
    Xd = to_dev(X)
    Ua, Va = to_dev(U0), to_dev(V0)
    ra = lib.iterate(Xd, Ua, Va, max_iter=200, relerr_svd=rso)
    Ub, Vb = to_dev(U0), to_dev(V0)
    r1 = lib.iterate(Xd, Ub, Vb, max_iter=100, relerr_svd=rso)
    r2 = lib.iterate(Xd, Ub, Vb, max_iter=100, relerr_svd=rso, step_u=r1["step_u"],
                     step_v=r1["step_v"])
    say(f"  ext {ra['ext_iters_done']} = {r1['ext_iters_done']} + {r2['ext_iters_done']}; "
        f"max |dU| {float((Ua - Ub).abs().max()):.3e}")
    assert r1["ext_iters_done"] + r2["ext_iters_done"] == ra["ext_iters_done"]
    assert r2["step_u"] == r1["step_u"] and r2["step_v"] == r1["step_v"]
    assert torch.equal(Ua, Ub) and torch.equal(Va, Vb)
    assert r2["f"] == ra["f"] and r2["kkt"] == ra["kkt"]


@pytest.mark.parametrize("opts", [dict(max_iter=61), dict(max_iter=60, check_every=3),
                                  dict(max_iter=300, kkt_tol=1e-5),
                                  dict(max_iter=40, pbcd_eps=0.3, pbcd_max_iter=4),
                                  dict(max_iter=64, mode=3)],
                         ids=["odd", "check3", "kkt_stop", "pbcd_eps", "mode3"])
def test_iterate_graph_replay_matches_direct(lib, problem, opts):
    """The loop body replayed from a captured graph against every kernel
    launched directly (the default): the same factors, report and trace bit
    for bit, with the trailing odd iteration, a check period, a stop inside a
    replayed pair, the PBCD tolerance sweeps and the stop at feasibility.
    The graph is replayed up to 149 times in one call, with the host's stop
    look (a copy and an event) between replays."""
    X, r, U0, V0, rso = problem
    say(f"graph replay vs direct launches {X.shape} r={r} {opts}")
    Xd = to_dev(X)
    outs = []
    for replay in (0, 1):
        U, V = to_dev(U0), to_dev(V0)
        rep = lib.iterate(Xd, U, V, relerr_svd=rso, trace_cap=opts["max_iter"] + 1,
                          graph_replay=replay, **opts)
        outs.append((U, V, rep))
    (U1, V1, r1), (U2, V2, r2) = outs
    say(f"  iters {r1['iters']} / {r2['iters']} converged {r1['converged']} kkt {r1['kkt']:.3e}")
    assert torch.equal(U1, U2) and torch.equal(V1, V2)
    for key in ("f", "kkt", "relerr", "iters", "ext_iters_done", "converged", "step_u", "step_v"):
        assert r1[key] == r2[key], key
    t1, t2 = r1["trace"].cpu().numpy(), r2["trace"].cpu().numpy()
    n1 = int(np.count_nonzero(t1[:, 6]))
    assert n1 == int(np.count_nonzero(t2[:, 6])) and n1 > 0
    cols = [0, 1, 2, 3, 4, 5, 7]            # every field but the device clock
    assert np.array_equal(t1[:n1][:, cols], t2[:n1][:, cols])


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_iterate_nonfinite_x(lib, bad):
    say(f"non-finite X ({bad}): ENMF_ENUMERIC, factors left finite")
    X, r = inputs.config_small()
    om = inputs.omega(X.shape[1], r + 10, 7)
    U0, V0, rso = rotated_start(X, r, om)
    Xb = X.copy()
    Xb[123, 45] = bad
    U, V = to_dev(U0), to_dev(V0)
    with pytest.raises(enmf.EnmfError) as ei:
        lib.iterate(to_dev(Xb), U, V, max_iter=20, relerr_svd=rso)
    assert ei.value.status == 4
    assert bool(torch.isfinite(U).all()) and bool(torch.isfinite(V).all())
    assert np.array_equal(host(U), U0.astype(np.float64)) and np.array_equal(host(V), V0.astype(np.float64))


def oracle_step_changes(U32, V32, steps):
    """||R_k - R_(k-1)||_F for k = 1..steps from oracle runs of k steps."""
    prev = np.eye(U32.shape[1])
    out = []
    for k in range(1, steps + 1):
        R = O.rotate(U32, V32, 1.0, k, 0.0)[2]
        out.append(float(np.linalg.norm(R - prev)))
        prev = R
    return np.array(out)


@pytest.mark.parametrize("check_every", [1, 10])
def test_rotation_tolerance_stop(lib, check_every):
    m, n, r, tol = 500, 400, 10, 1e-10
    say(f"rotation tolerance stop {m}x{n} r={r} tol={tol} check_every={check_every}")
    X, _, _ = inputs.disjoint_support(m, n, r, 3, equal_norms=True)
    om = inputs.omega(n, r + 10, 7)
    Uo, Vo, _, _ = O.svd_init_randomized(X, r, om, 2)
    U32, V32 = Uo.astype(np.float32), Vo.astype(np.float32)
    d = oracle_step_changes(U32, V32, 60)
    ks = np.arange(1, d.size + 1)
    looked = (ks % check_every == 0)
    hit = np.flatnonzero(looked & (d <= tol))
    assert hit.size, "the oracle's ADMM does not converge on this instance"
    want = int(ks[hit[0]])
    # no step the device looks at sits within 5% of the tolerance
    assert np.all(np.abs(d[looked] - tol) > 0.05 * tol)
    U, V = to_dev(U32), to_dev(V32)
    out = lib.rotate(U, V, 1.0, 300, tol, check_every=check_every)
    Ur, Vr, R, *_ = O.rotate(U32, V32, 1.0, want, 0.0)
    Rg = np.array(out["R"]).reshape(r, r)
    say(f"  steps {out['steps']} (oracle's first look within tol: {want}) |dR| {np.linalg.norm(Rg - R):.2e}")
    assert out["steps"] == want
    assert np.linalg.norm(Rg - R) <= 1e-6
    assert float(np.linalg.norm(host(U) - Ur) / np.linalg.norm(Ur)) <= 1e-6
