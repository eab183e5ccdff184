"""Continuous-batching server on the GPU (through the C ABI).

A request's result is bitwise the same alone and in a mix; results agree with
the single-request path and the oracle; admission respects the memory cap.
"""
import numpy as np
import pytest

import oracle
from gpu_util import announce, rel_max
from paper_1806_04801_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04801_amd import hsma
    hsma.load()
    return hsma


@pytest.fixture(scope="module")
def plans(hs):
    out = {}
    for bc in (0, 1):
        for p in (8, 12):
            out[(bc, p)] = hs.Plan(1.0, bc, p, 10 * p * p, 10 * p * p, 2.7)
    return out


def mix(n_req, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_req):
        n = int(2 * round(10 ** rng.uniform(2.5, 3.7) / 2))
        bc = int(rng.integers(0, 2))
        p = int(rng.choice([8, 12]))
        x, q = W.uniform_neutral(n, 1.0, seed=1000 + seed * 100 + i)
        reqs.append((bc, p, x, q))
    return reqs


def energy_scale(plan, x, q):
    """1/2 sum |q_i phi_i| from the single-request FP64 path: single-precision
    terms err by ~6e-8 relative each, so the energy error of the FP32 path
    scales with this sum, not with |E| (which can be a small difference)."""
    e, phi, F = plan.energy_forces(torch.tensor(x, device="cuda"), torch.tensor(q, device="cuda"))
    return e, 0.5 * float(np.sum(np.abs(q * phi.cpu().numpy())))


GATE = 1e-5   # |dE| / |E| of a single-precision result against double precision


def rel_err(e, ref):
    return abs(e - ref) / abs(ref)


def run_all(srv, plans, reqs):
    ids = [srv.submit(plans[(bc, p)], x, q) for bc, p, x, q in reqs]
    out = []
    for rid, (bc, p, x, q) in zip(ids, reqs):
        srv.wait(rid)
        done, e, phi, F, lat = srv.result(rid, len(q))
        assert done
        out.append((e, phi, F, lat))
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_same_alone_and_in_mix(hs, plans, precision):
    announce("server alone vs mix precision=%d" % precision)
    reqs = mix(14, 3)
    srv = hs.Server(memory_bytes=2 << 30, max_active=8, precision=precision)
    alone = [run_all(srv, plans, [r])[0] for r in reqs[:3]]
    both = run_all(srv, plans, reqs)
    for a, b in zip(alone, both[:3]):
        assert a[0] == b[0]
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    st = srv.stats()
    assert st["completed"] == 17 and st["active"] == 0 and st["pending"] == 0


def test_server_matches_single_request_path_and_oracle(hs, plans):
    announce("server vs single path")
    reqs = mix(10, 5)
    s64 = hs.Server(memory_bytes=2 << 30, max_active=4, precision=hs.FP64)
    s32 = hs.Server(memory_bytes=2 << 30, max_active=4, precision=hs.FP32_COMP)
    r64 = run_all(s64, plans, reqs)
    r32 = run_all(s32, plans, reqs)
    for (bc, p, x, q), a, b in zip(reqs, r64, r32):
        e, phi, F = plans[(bc, p)].energy_forces(torch.tensor(x, device="cuda"),
                                                 torch.tensor(q, device="cuda"))
        scale = 0.5 * float(np.sum(np.abs(q * phi.cpu().numpy())))
        assert abs(a[0] - e) <= 1e-12 * scale
        assert rel_max(a[1], phi.cpu().numpy()) <= 1e-11
        # the single-precision server (default refinement) meets the gate
        assert rel_err(b[0], e) <= GATE
    for (bc, p, x, q), a, b in list(zip(reqs, r64, r32))[:3]:
        ref = oracle.solve(oracle.make_plan(1.0, bc, p, 10 * p * p, 10 * p * p, 2.7), x, q)
        assert rel_err(a[0], ref["energy"]) <= 1e-10
        assert rel_err(b[0], ref["energy"]) <= GATE


def test_admission_by_memory(hs, plans):
    """A 30 MiB arena holds about two of these requests (~13 MiB each with
    their partial buffers): admission is limited by memory, not by slots, and
    the arena never exceeds its cap."""
    announce("server admission")
    reqs = [(0, 12, *W.uniform_neutral(4000, 1.0, seed=40 + i)) for i in range(6)]
    cap = 30 << 20
    srv = hs.Server(memory_bytes=cap, max_active=16, precision=hs.FP32_COMP)
    ids = [srv.submit(plans[(bc, p)], x, q) for bc, p, x, q in reqs]
    peak_active = 0
    for _ in range(100000):
        srv.tick()
        st = srv.stats()
        peak_active = max(peak_active, st["active"])
        assert st["arena_used"] <= cap and st["arena_peak"] <= cap
        if st["completed"] == len(ids):
            break
    assert srv.stats()["completed"] == len(ids)
    assert 1 <= peak_active < len(ids)
    ref = plans[(0, 12)].energy_forces(torch.tensor(reqs[0][2], device="cuda"),
                                       torch.tensor(reqs[0][3], device="cuda"))[0]
    ok, e, *_ = srv.result(ids[0], 4000)
    assert ok and abs(e - ref) <= 1e-5 * abs(ref)
    for rid in ids[1:]:
        assert srv.result(rid, 4000)[0]
    big = W.uniform_neutral(400000, 1.0, seed=1)
    with pytest.raises(hs.HsmaError) as ei:
        srv.submit(plans[(0, 12)], *big)
    assert ei.value.status == -5


def test_trace_replay_batched_vs_sequential(hs, plans):
    announce("trace replay")
    reqs = mix(24, 7)
    arrivals = np.cumsum(np.random.default_rng(1).exponential(0.002, len(reqs)))
    pl = [plans[(bc, p)] for bc, p, _, _ in reqs]
    xs = [r[2] for r in reqs]
    qs = [r[3] for r in reqs]
    srv = hs.Server(memory_bytes=2 << 30, max_active=16, precision=hs.FP32_COMP)
    e32, lat32, wall32 = srv.run_trace(arrivals, pl, xs, qs)
    e64, lat64, wall64 = hs.run_trace_sequential(arrivals, pl, xs, qs)
    scale = np.array([energy_scale(p_, x, q)[1] for p_, x, q in zip(pl, xs, qs)])
    err = np.abs(e32 - e64)
    print("trace: max |dE|/scale %.2e, median |dE|/|E| %.2e, max |dE|/|E| %.2e, refined %d"
          % ((err / scale).max(), np.median(err / np.abs(e64)), (err / np.abs(e64)).max(),
             srv.stats()["refined"]))
    assert np.all(err <= GATE * np.abs(e64))
    assert np.all(lat32 > 0) and np.all(lat64 > 0)
    assert srv.stats()["completed"] == len(reqs)


@pytest.mark.parametrize("precision", [0, 1])
def test_pair_once_requests_in_the_server(hs, plans, precision, monkeypatch):
    """With the pair-once threshold lowered to 1000 particles, part of the mix
    runs its near sum in pair-once rounds and the rest in grouped tiles:
    results stay bitwise the same alone and in the mix, and agree with the
    single-request path (which makes the same choice)."""
    announce("server pair-once precision=%d" % precision)
    monkeypatch.setenv("HSMA_SYM_MIN", "1000")
    reqs = mix(10, 9)
    sizes = [len(q) for _, _, _, q in reqs]
    assert min(sizes) < 1000 <= max(sizes)
    srv = hs.Server(memory_bytes=2 << 30, max_active=8, precision=precision)
    order = sorted(range(len(reqs)), key=lambda i: -sizes[i])[:2] + [sizes.index(min(sizes))]
    alone = [run_all(srv, plans, [reqs[i]])[0] for i in order]
    both = run_all(srv, plans, reqs)
    for i, a in zip(order, alone):
        b = both[i]
        assert a[0] == b[0]
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    for (bc, p, x, q), b in zip(reqs, both):
        e, phi, F = plans[(bc, p)].energy_forces(torch.tensor(x, device="cuda"),
                                                 torch.tensor(q, device="cuda"))
        scale = 0.5 * float(np.sum(np.abs(q * phi.cpu().numpy())))
        if precision == 0:
            assert abs(b[0] - e) <= 1e-12 * scale
        else:
            assert rel_err(b[0], e) <= GATE


def test_refinement_in_double_precision(hs, plans):
    """refine_below: a single-precision result whose energy is below that
    fraction of 1/2 sum |q phi| is recomputed in double precision before it
    completes.  A threshold above every request's ratio refines all of them,
    and each then equals the double-precision single-request path bitwise
    (the refinement is that path); with 0 nothing is refined; a realistic
    threshold refines some and keeps the rest within the single-precision
    bound."""
    announce("server refinement")
    reqs = mix(8, 11)
    singles = []
    for bc, p, x, q in reqs:
        e, phi, F = plans[(bc, p)].energy_forces(torch.tensor(x, device="cuda"),
                                                 torch.tensor(q, device="cuda"))
        singles.append((e, phi.cpu().numpy(), F.cpu().numpy()))
    srv = hs.Server(memory_bytes=2 << 30, max_active=8, precision=hs.FP32_COMP, refine_below=1e9)
    out = run_all(srv, plans, reqs)
    assert srv.stats()["refined"] == len(reqs) and srv.stats()["completed"] == len(reqs)
    for (e, phi, F), r in zip(singles, out):
        assert r[0] == e
        assert np.array_equal(r[1], phi) and np.array_equal(r[2], F)
    srv0 = hs.Server(memory_bytes=2 << 30, max_active=8, precision=hs.FP32_COMP, refine_below=0.0)
    out0 = run_all(srv0, plans, reqs)
    assert srv0.stats()["refined"] == 0
    srv1 = hs.Server(memory_bytes=2 << 30, max_active=8, precision=hs.FP32_COMP, refine_below=5e-3)
    out1 = run_all(srv1, plans, reqs)
    n_ref = 0
    for (bc, p, x, q), (e, phi, F), a0, a1 in zip(reqs, singles, out0, out1):
        scale = 0.5 * float(np.sum(np.abs(q * phi)))
        if abs(a0[0]) < 5e-3 * scale:          # ill-conditioned: refined
            n_ref += 1
            assert a1[0] == e
        else:
            assert a1[0] == a0[0]              # untouched single-precision result
        assert rel_err(a1[0], e) <= GATE       # every served energy meets the gate
    assert srv1.stats()["refined"] == n_ref
    with pytest.raises(hs.HsmaError):
        hs.Server(memory_bytes=2 << 30, max_active=8, precision=hs.FP32_COMP, refine_below=-1.0)


def test_server_rejects_coincident_request_alone(hs):
    """A request with two charges at the same position fails with
    HSMA_E_COINCIDENT (-4); the requests around it complete as usual."""
    announce("serving coincident request")
    plan = hs.Plan(1.0, 0, 12, 1440, 1440, 2.7, precision=hs.FP32_COMP)
    good = [W.uniform_neutral(2000, 1.0, seed=s) for s in (31, 32)]
    bad_x, bad_q = W.uniform_neutral(3000, 1.0, seed=33)
    bad_x = np.array(bad_x)
    bad_x[100] = bad_x[2500]
    srv = hs.Server(memory_bytes=2 << 30, max_active=8, precision=hs.FP32_COMP)
    ids = [srv.submit(plan, *good[0]), srv.submit(plan, bad_x, bad_q), srv.submit(plan, *good[1])]
    for rid in ids:
        srv.wait(rid)
    for rid, (x, q) in ((ids[0], good[0]), (ids[2], good[1])):
        ok, e, *_ = srv.result(rid, len(q))
        ref, phi, _ = plan.energy_forces(torch.tensor(x, device="cuda"),
                                         torch.tensor(q, device="cuda"))
        assert ok and rel_err(e, ref) <= GATE
    with pytest.raises(hs.HsmaError) as ei:
        srv.result(ids[1], len(bad_q))
    assert ei.value.status == -4
    srv.close()


def test_serving_stream_at_its_stated_parameters(hs):
    """The serving stream as configured: N log-uniform in [1e3, 1e5] (even),
    periodic or grounded cube with probability 1/2, p in {12, 16, 20},
    K = M = 10 p^2, R = 2.7 L, on a bounded trace of 48 requests with Poisson
    arrivals.  Every energy of the batched single-precision server (default
    double-precision refinement) is within 1e-5 of the double-precision
    per-request path; three requests give bitwise the same result alone and in
    the mix; the two smallest agree with the oracle."""
    announce("serving stream 48 requests, p in {12,16,20}, N in [1e3,1e5]")
    trace = W.serving_trace(48, seed=4)
    ns = np.array([r["n"] for r in trace])
    assert ns.min() >= 1000 and ns.max() <= 100000
    assert {r["p"] for r in trace} == {12, 16, 20} and {r["bc"] for r in trace} == {0, 1}
    plans = {(bc, p): hs.Plan(1.0, bc, p, 10 * p * p, 10 * p * p, 2.7)
             for bc in (0, 1) for p in (12, 16, 20)}
    pl = [plans[(r["bc"], r["p"])] for r in trace]
    xs, qs = [], []
    for r in trace:
        x, q = W.uniform_neutral(r["n"], 1.0, seed=r["seed"])
        xs.append(x)
        qs.append(q)
    arrivals = np.array([r["t"] for r in trace]) * 2e-3   # ~500 requests/s offered
    srv = hs.Server(memory_bytes=8 << 30, max_active=32, precision=hs.FP32_COMP)
    e32, lat32, _ = srv.run_trace(arrivals, pl, xs, qs)
    e64, lat64, _ = hs.run_trace_sequential(arrivals, pl, xs, qs)
    rel = np.abs(e32 - e64) / np.abs(e64)
    print("stream: refined %d of %d, max |dE|/|E| %.2e, median %.2e"
          % (srv.stats()["refined"], len(trace), rel.max(), np.median(rel)))
    assert np.all(rel <= GATE)
    assert np.all(lat32 > 0) and np.all(lat64 > 0)
    # alone vs in the mix: the largest, a middle and the smallest request
    order = np.argsort(ns)
    pick = [int(order[-1]), int(order[len(order) // 2]), int(order[0])]
    mixed = run_all(srv, plans, [(trace[i]["bc"], trace[i]["p"], xs[i], qs[i]) for i in range(len(trace))])
    for i in pick:
        alone = run_all(srv, plans, [(trace[i]["bc"], trace[i]["p"], xs[i], qs[i])])[0]
        assert alone[0] == mixed[i][0]
        assert np.array_equal(alone[1], mixed[i][1]) and np.array_equal(alone[2], mixed[i][2])
    for i in order[:2]:
        r = trace[int(i)]
        ref = oracle.solve(oracle.make_plan(1.0, r["bc"], r["p"], 10 * r["p"] ** 2, 10 * r["p"] ** 2, 2.7),
                           xs[int(i)], qs[int(i)])
        assert rel_err(e64[int(i)], ref["energy"]) <= 1e-10
        assert rel_err(e32[int(i)], ref["energy"]) <= GATE


@pytest.mark.parametrize("precision", [0, 1])
def test_pair_once_side_streams_match_single_requests(hs, precision):
    """Requests of 1024 particles and more run their pair-once near sums on
    the server's side streams, several at the same time (periodic,
    grounded-cube and slab requests with different round counts).  Each
    result equals the single-request path to rounding (1e-12 of
    1/2 sum |q phi|: same schedule and arithmetic), and is bitwise the same
    alone and in the mix."""
    announce("server pair-once side streams precision=%d" % precision)
    plans = {bc: hs.Plan(1.0, bc, 8, 640, 640, 2.7, precision=precision) for bc in (0, 1, 2)}
    sizes = [(0, 1030), (1, 2050), (2, 3000), (0, 4100), (1, 5000), (2, 6100), (0, 12000), (1, 1500),
             (2, 2500)]
    reqs = []
    for i, (bc, n) in enumerate(sizes):
        x, q = W.slab_charges(n, 1.0, 60 + i) if bc == 2 else W.uniform_neutral(n, 1.0, 60 + i)
        reqs.append((bc, x, q))
    rounds = {plans[bc].near_schedule(len(q))["blocks"] for bc, _, q in reqs}
    assert all(plans[bc].near_schedule(len(q))["kind"] == 1 for bc, _, q in reqs)
    assert len(rounds) >= 3
    srv = hs.Server(memory_bytes=4 << 30, max_active=16, precision=precision, refine_below=0.0)
    ids = [srv.submit(plans[bc], x, q) for bc, x, q in reqs]
    mixed = []
    for rid, (bc, x, q) in zip(ids, reqs):
        srv.wait(rid)
        done, e, phi, F, _ = srv.result(rid, len(q))
        assert done
        mixed.append((e, phi, F))
    for (bc, x, q), (e, phi, F) in zip(reqs, mixed):
        e1, phi1, F1 = plans[bc].energy_forces(torch.tensor(x, device="cuda"),
                                               torch.tensor(q, device="cuda"))
        phi1 = phi1.cpu().numpy()
        scale = 0.5 * float(np.sum(np.abs(q * phi1)))
        assert abs(e - e1) <= 1e-12 * scale
        assert rel_max(phi, phi1, np.abs(phi1).max()) <= 1e-12
        assert rel_max(F, F1.cpu().numpy()) <= 1e-11
    for i in (2, 6):
        bc, x, q = reqs[i]
        rid = srv.submit(plans[bc], x, q)
        srv.wait(rid)
        done, e, phi, F, _ = srv.result(rid, len(q))
        assert e == mixed[i][0] and np.array_equal(phi, mixed[i][1]) and np.array_equal(F, mixed[i][2])
    srv.close()
