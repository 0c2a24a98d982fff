"""GPU tests of the serving loop (enmf_serve_*), through the C ABI.

Each served solve runs Algorithm 3 end to end in one workgroup.  It is
compared with the FP64 oracle run of the same algorithm, on the same X and
test matrix omega:
* float32 X: the oracle's trajectory, with U and V within 1e-4 and f within 1e-5;
* bfloat16 X: the oracle's relative error within 1e-3 and a KKT residual <= 1e-5.

A request gives bitwise the same factors when it runs alone, in a mix of
uneven requests of several dtypes, under a different tick time, and with
its ticks launched one by one instead of replayed from a captured graph.
Requests at the large end of the stream (about 2048 x 2048, r = 30-32) meet
the same bar as the small ones, on the tick path and on the device-wide path
that wide requests take by default; a wide request gives bitwise the result
of the library's own solve calls with the same options, alone or in a mix.
Errors: r beyond the served range, a workspace that can never fit, and an
unknown ticket.
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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def host(t):
    return t.detach().cpu().double().numpy()


@pytest.fixture(scope="module")
def server(lib):
    # every request on the tick path (one workgroup per solve), whatever its size
    srv = enmf.Server(lib, hbm_budget_bytes=1 << 30, max_slots=64, wide_min_elems=-1)
    yield srv
    srv.stop()


def test_served_fp32_tracks_oracle(server):
    X, r = inputs.config_small()
    om = inputs.omega(X.shape[1], r + 10, 7)
    say("served fp32 500x400 r=10, 20 rotation steps, 200 iterations vs oracle")
    t, U, V = server.submit(to_dev(X), r, to_dev(om), rot_max_iter=20, rot_tol=0.0, max_iter=200)
    res = server.wait(t)
    Uo, Vo, ro = O.enmf(X, r, om, rot_max_iter=20, rot_tol=0.0, max_iter=200)
    say(f"  iters {res['iters']} ext {res['ext_iters_done']} relerr {res['relerr']:.8e} "
        f"oracle {ro['relerr']:.8e} latency {res['latency_s']:.3f} s")
    assert res["status"] == 0
    assert res["iters"] == ro["iters"] == 200
    assert res["ext_iters_done"] == ro["ext_iters_done"]
    assert rel(host(U), Uo) <= 1e-4 and rel(host(V), Vo) <= 1e-4
    assert abs(res["f"] - ro["f"]) <= 1e-5 * ro["f"]
    assert abs(res["kkt"] - ro["kkt"]) <= 1e-5


@pytest.mark.parametrize("mode", [2, 3])
def test_served_ablation_modes(server, mode):
    X, r = inputs.config_small()
    om = inputs.omega(X.shape[1], r + 10, 7)
    say(f"served fp32 500x400 r=10, mode {mode}, 60 iterations vs oracle")
    t, U, V = server.submit(to_dev(X), r, to_dev(om), rot_max_iter=20, rot_tol=0.0, max_iter=60,
                            mode=mode)
    res = server.wait(t)
    Uo, Vo, ro = O.enmf(X, r, om, rot_max_iter=20, rot_tol=0.0, max_iter=60, mode=mode)
    say(f"  iters {res['iters']} (oracle {ro['iters']}) relerr {res['relerr']:.8e} "
        f"oracle {ro['relerr']:.8e}")
    assert res["status"] == 0
    assert res["iters"] == ro["iters"] and res["ext_iters_done"] == ro["ext_iters_done"]
    assert rel(host(U), Uo) <= 1e-4 and rel(host(V), Vo) <= 1e-4


def test_served_bf16_reaches_oracle_error(lib, server):
    X, r = inputs.config_small()
    om = inputs.omega(X.shape[1], r + 10, 7)
    say("served bf16: relerr within 1e-3 of the oracle, kkt <= 1e-5")
    Uo, Vo, ro = O.enmf(X, r, om, rot_max_iter=20, rot_tol=0.0, max_iter=400, kkt_tol=1e-6)
    Xb = lib.convert(to_dev(X), torch.bfloat16)
    t, U, V = server.submit(Xb, r, to_dev(om), rot_max_iter=20, rot_tol=0.0, max_iter=400,
                            kkt_tol=1e-6)
    res = server.wait(t)
    Ug, Vg = host(U), host(V)
    err = O.relerr(X, Ug, Vg)
    say(f"  relerr {err:.6e} oracle {ro['relerr']:.6e} kkt {res['kkt']:.2e}")
    assert abs(err - ro["relerr"]) <= 1e-3
    assert res["kkt"] <= 1e-5
    assert Ug.min() >= 0 and Vg.min() >= 0


def _request(i, seed):
    rng = np.random.default_rng(seed)
    m, n = (int(v) for v in rng.integers(64, 400, 2))
    r = int(rng.integers(4, 33))
    r = min(r, m, n)
    X, _, _ = inputs.lowrank_plus_noise(m, n, r, seed + 1)
    om = inputs.omega(n, min(r + 10, 48), seed + 2)
    return X, r, om


def test_same_result_alone_and_in_the_mix(lib):
    say("one request alone, in a mix of 16 uneven requests, and with one step per tick")
    Xa, ra, oma = _request(0, 500)
    Xa_b = lib.convert(to_dev(Xa), torch.bfloat16)
    opts = dict(oversample=oma.shape[1] - ra, max_iter=150, kkt_tol=1e-6)

    def run(srv, others):
        live = []
        for i, (X, r, om, dt) in enumerate(others):
            Xd = to_dev(X) if dt == "f32" else lib.convert(to_dev(X), dt)
            live.append(srv.submit(Xd, r, to_dev(om), oversample=om.shape[1] - r, max_iter=150))
            if i == len(others) // 2:
                ta, Ua, Va = srv.submit(Xa_b, ra, to_dev(oma), **opts)
        if not others:
            ta, Ua, Va = srv.submit(Xa_b, ra, to_dev(oma), **opts)
        res = srv.wait(ta)
        for t, _, _ in live:
            assert srv.wait(t)["status"] == 0
        return host(Ua), host(Va), res

    srv = enmf.Server(lib, max_slots=64)
    try:
        U1, V1, r1 = run(srv, [])
        dts = ["f32", torch.bfloat16, torch.float16]
        mix = [(*_request(i, 600 + 10 * i), dts[i % 3]) for i in range(16)]
        U2, V2, r2 = run(srv, mix)
    finally:
        srv.stop()
    srv = enmf.Server(lib, max_slots=8, tick_time_us=1)   # one step per tick
    try:
        U3, V3, r3 = run(srv, mix[:6])
    finally:
        srv.stop()
    # the same ticks launched one by one instead of replayed from a graph, one per replay
    srv = enmf.Server(lib, max_slots=8, tick_time_us=3, ticks_per_launch=1, direct_launch=1)
    try:
        U4, V4, r4 = run(srv, mix[6:10])
    finally:
        srv.stop()
    say(f"  iters {r1['iters']} {r2['iters']} {r3['iters']} {r4['iters']}  relerr {r1['relerr']:.6e}")
    for Ux, Vx, rx in ((U2, V2, r2), (U3, V3, r3), (U4, V4, r4)):
        assert np.array_equal(U1, Ux) and np.array_equal(V1, Vx)
        assert r1["iters"] == rx["iters"] and r1["relerr"] == rx["relerr"]


def test_served_stream_sample_matches_oracle(lib, server):
    say("served-stream sample (bf16, stop at relerr - relerr_svd <= 1e-3 or kkt <= 1e-5)")
    reqs = [q for q in inputs.serve_stream(count=64) if q["m"] * q["n"] <= 150_000][:8]
    live = []
    for q in reqs:
        X, _, _ = inputs.lowrank_plus_noise(q["m"], q["n"], q["r"], q["seed"])
        om = inputs.omega(q["n"], q["r"] + 10, q["seed"] + 1)
        Xb = lib.convert(to_dev(X), torch.bfloat16)
        t, U, V = server.submit(Xb, q["r"], to_dev(om), max_iter=300, relerr_tol=1e-3, kkt_tol=1e-5)
        live.append((q, X, om, t, U, V))
    for q, X, om, t, U, V in live:
        res = server.wait(t)
        Uo, Vo, ro = O.enmf(X, q["r"], om, max_iter=300, relerr_tol=1e-3, kkt_tol=1e-5)
        err = O.relerr(X, host(U), host(V))
        say(f"  {q['m']}x{q['n']} r={q['r']}: iters {res['iters']} relerr {err:.5e} "
            f"oracle {ro['relerr']:.5e} ({ro['iters']} iters) latency {res['latency_s']:.3f} s")
        assert res["status"] == 0
        assert abs(err - ro["relerr"]) <= 1e-3
        assert host(U).min() >= 0 and host(V).min() >= 0


def test_served_large_requests_match_oracle(lib, server):
    """Requests at the large end of the served stream (m, n near 2048, r near
    32, bfloat16 X), submitted together: each reaches the oracle's relative
    error within 1e-3 (against the float32 X), with nonnegative factors."""
    say("served large requests (bf16, ~2048 x 2048, r 30-32) vs the oracle")
    shapes = [(2048, 1900, 32, 3101), (1850, 2048, 30, 3102), (2000, 2000, 32, 3103)]
    live = []
    for m, n, r, seed in shapes:
        X, _, _ = inputs.lowrank_plus_noise(m, n, r, seed)
        om = inputs.omega(n, r + 10, seed + 1)
        Xb = lib.convert(to_dev(X), torch.bfloat16)
        t, U, V = server.submit(Xb, r, to_dev(om), max_iter=300, relerr_tol=1e-3, kkt_tol=1e-5)
        live.append((m, n, r, X, om, t, U, V))
    for m, n, r, X, om, t, U, V in live:
        res = server.wait(t, timeout=300.0)
        Uo, Vo, ro = O.enmf(X, r, om, max_iter=300, relerr_tol=1e-3, kkt_tol=1e-5)
        err = O.relerr(X, host(U), host(V))
        say(f"  {m}x{n} r={r}: iters {res['iters']} relerr {err:.6e} oracle {ro['relerr']:.6e} "
            f"({ro['iters']} iters) kkt {res['kkt']:.2e} latency {res['latency_s']:.3f} s")
        assert res["status"] == 0 and res["converged"] == 1
        assert abs(err - ro["relerr"]) <= 1e-3
        assert host(U).min() >= 0 and host(V).min() >= 0


@pytest.mark.parametrize("shape", [(300, 517, 20), (1000, 333, 32), (77, 1100, 7), (640, 640, 16)],
                         ids=["300x517r20", "1000x333r32", "77x1100r7", "640x640r16"])
def test_served_bf16_matrix_cores_match_float32_form(lib, server, shape):
    """The bfloat16 requests run their products on the matrix cores (factor
    split into three bfloat16 terms), the float32 ones on the vector ALU.  On
    the same values (X rounded to bfloat16, then widened exactly to float32),
    at widths 16, 32 and 48 of the range finder and ragged row and column
    counts, the two give
    * the same SVD factors within 1e-5 and relative error within 1e-6;
    * after a 20-step rotation and 30 iterations, the same push count, the
      same relative error within 1e-6, and factors within max(1e-4, 10 times
      the move of the oracle's own factors when X changes by 2^-24 relative):
      these low-rank instances leave a residual of about 0.2% of X, so their
      factors move far more than their objective."""
    m, n, r = shape
    say(f"served bf16 (matrix cores) vs float32 (vector ALU) on the same values, {m}x{n} r={r}")
    X, _, _ = inputs.lowrank_plus_noise(m, n, r, 4100 + r)
    om_h = inputs.omega(n, min(r + 10, 48), 4200 + r)
    om = to_dev(om_h)
    Xb = lib.convert(to_dev(X), torch.bfloat16)
    Xf = Xb.float().contiguous()
    run_opts = dict(max_iter=30, rot_max_iter=20, rot_tol=0.0)
    Xo = host(Xf)
    Uo1, Vo1, _ = O.enmf(Xo, r, om_h, **run_opts)
    sign = np.where(np.random.default_rng(4300 + r).random(Xo.shape) < 0.5, -1.0, 1.0)
    Uo2, Vo2, _ = O.enmf(Xo * (1.0 + 2.0 ** -24 * sign), r, om_h, **run_opts)
    move = max(rel(Uo2, Uo1), rel(Vo2, Vo1))
    for opts, bar in ((dict(max_iter=0, rot_max_iter=0), 1e-5), (run_opts, max(1e-4, 10.0 * move))):
        tb, Ub, Vb = server.submit(Xb, r, om, oversample=om.shape[1] - r, **opts)
        tf, Uf, Vf = server.submit(Xf, r, om, oversample=om.shape[1] - r, **opts)
        rb, rf = server.wait(tb), server.wait(tf)
        du, dv = rel(host(Ub), host(Uf)), rel(host(Vb), host(Vf))
        say(f"  {opts}: |dU| {du:.2e} |dV| {dv:.2e} (bar {bar:.1e}; oracle move {move:.1e}) "
            f"relerr {rb['relerr']:.8e} / {rf['relerr']:.8e}")
        assert rb["status"] == 0 and rf["status"] == 0
        assert du <= bar and dv <= bar
        assert rb["ext_iters_done"] == rf["ext_iters_done"] and rb["iters"] == rf["iters"]
        assert abs(rb["relerr"] - rf["relerr"]) <= 1e-6


def test_serve_rejects_bad_requests(lib):
    say("serve: bad rank, workspace beyond the budget, unknown ticket")
    srv = enmf.Server(lib, hbm_budget_bytes=1 << 20, max_slots=4, wide_min_elems=-1)
    try:
        X = to_dev(np.ones((100, 80), np.float32))
        with pytest.raises(enmf.EnmfError) as e:
            srv.submit(X, 33, to_dev(np.ones((80, 43), np.float32)))
        assert e.value.status == 1
        Xbig = to_dev(np.ones((2000, 2000), np.float32))
        with pytest.raises(enmf.EnmfError) as e:
            srv.submit(Xbig, 30, to_dev(np.ones((2000, 40), np.float32)))
        assert e.value.status == 2
        with pytest.raises(enmf.EnmfError) as e:
            srv.poll(12345)
        assert e.value.status == 1
    finally:
        srv.stop()


WIDE = [(1100, 1000, 20, "bf16", 3201), (2048, 1900, 32, "bf16", 3202), (1300, 900, 12, "f32", 3203)]


def _wide_inputs(lib, m, n, r, dt, seed):
    X, _, _ = inputs.lowrank_plus_noise(m, n, r, seed)
    om = inputs.omega(n, r + 10, seed + 1)
    Xd = to_dev(X) if dt == "f32" else lib.convert(to_dev(X), torch.bfloat16)
    return X, om, Xd


def test_wide_requests_run_the_device_wide_solve(lib):
    """Requests of at least wide_min_elems elements take the device-wide path:
    each one's factors and report are bitwise those of the library's own
    svd_init, rotate and iterate calls with the same options, when it runs
    alone and when it is submitted among narrow requests that take slots."""
    say("wide requests: served alone, in a mix, and the same solve called directly")
    opts = dict(max_iter=300, relerr_tol=1e-3, kkt_tol=1e-5)
    data = [(m, n, r, *_wide_inputs(lib, m, n, r, dt, seed)) for m, n, r, dt, seed in WIDE]
    direct = []
    for m, n, r, X, om, Xd in data:
        U, V, rep = lib.solve(Xd, r, to_dev(om), **opts)
        direct.append((host(U), host(V), rep))
    srv = enmf.Server(lib, max_slots=16, wide_min_elems=1 << 20, wide_lanes=2)
    try:
        alone = []
        for m, n, r, X, om, Xd in data:
            t, U, V = srv.submit(Xd, r, to_dev(om), **opts)
            res = srv.wait(t, timeout=300.0)
            alone.append((host(U), host(V), res))
        live, narrow = [], []
        for i, (m, n, r, X, om, Xd) in enumerate(data):
            for j in range(3):
                Xs, rs, oms = _request(j, 700 + 10 * (3 * i + j))
                narrow.append(srv.submit(lib.convert(to_dev(Xs), torch.bfloat16), rs, to_dev(oms),
                                         oversample=oms.shape[1] - rs, max_iter=150))
            live.append(srv.submit(Xd, r, to_dev(om), **opts))
        mixed = []
        for t, U, V in live:
            res = srv.wait(t, timeout=300.0)
            mixed.append((host(U), host(V), res))
        for t, _, _ in narrow:
            assert srv.wait(t)["status"] == 0
    finally:
        srv.stop()
    for (m, n, r, *_), d, a, x in zip(data, direct, alone, mixed):
        say(f"  {m}x{n} r={r}: iters {d[2]['iters']} relerr {d[2]['relerr']:.8e} "
            f"latency alone {a[2]['latency_s']:.4f} s, in the mix {x[2]['latency_s']:.4f} s")
        for got in (a, x):
            assert got[2]["status"] == 0
            assert np.array_equal(got[0], d[0]) and np.array_equal(got[1], d[1])
            for key in ("iters", "ext_iters_done", "converged", "relerr", "f", "kkt"):
                assert got[2][key] == d[2][key], key


def test_wide_large_requests_match_oracle(lib):
    """The large end of the served stream on the device-wide path meets the
    oracle bar of the tick path: relative error within 1e-3 of the oracle's
    (against the float32 X) and nonnegative factors."""
    say("wide requests (bf16, ~2048 x 2048, r 30-32) vs the oracle")
    shapes = [(2048, 1900, 32, 3101), (2000, 2000, 32, 3103)]
    srv = enmf.Server(lib, max_slots=4)
    try:
        live = []
        for m, n, r, seed in shapes:
            X, om, Xb = _wide_inputs(lib, m, n, r, "bf16", seed)
            t, U, V = srv.submit(Xb, r, to_dev(om), max_iter=300, relerr_tol=1e-3, kkt_tol=1e-5)
            live.append((m, n, r, X, om, t, U, V))
        for m, n, r, X, om, t, U, V in live:
            res = srv.wait(t, timeout=300.0)
            Uo, Vo, ro = O.enmf(X, r, om, max_iter=300, relerr_tol=1e-3, kkt_tol=1e-5)
            err = O.relerr(X, host(U), host(V))
            say(f"  {m}x{n} r={r}: iters {res['iters']} relerr {err:.6e} oracle {ro['relerr']:.6e} "
                f"latency {res['latency_s']:.4f} s")
            assert res["status"] == 0
            assert abs(err - ro["relerr"]) <= 1e-3
            assert host(U).min() >= 0 and host(V).min() >= 0
    finally:
        srv.stop()
