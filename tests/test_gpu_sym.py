"""Near sum with each unordered pair once (GPU, through the C ABI).

The pair-once kernel must give what the per-target tile kernel gives, up to
rounding, and match the oracle under the gates of its precision: in single
precision |dE|/|E| <= 1e-5, potential error <= 1e-5 of the particle's own
magnitude (rms as floor), force error <= 1e-4 of its maximum; in double
precision 1e-10 for all three.  Cases cover several rounds, an odd block count (a bye in every
round), ragged last blocks and slices, one and two rows per lane, both image
kinds, both precisions, and the adjoint, which reads the same near
accumulators.
"""
import numpy as np
import pytest

import oracle
from gpu_util import announce, rel_max, rms
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


def run(hs, plan, x, q, monkeypatch, sym, T=2):
    monkeypatch.setenv("HSMA_SYM", "1" if sym else "0")
    monkeypatch.setenv("HSMA_SYM_T", str(T))
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    qd = torch.tensor(q, dtype=torch.float64, device="cuda")
    e, phi, F, inter = plan.energy_forces(xd, qd, intermediates=True)
    torch.cuda.synchronize()
    return e, phi.cpu().numpy(), F.cpu().numpy(), {k: v.cpu().numpy() for k, v in inter.items()}


def rel_own(a, ref):
    """max_i |a_i - ref_i| / max(|ref_i|, rms(ref)): each particle against its
    own magnitude, with the rms as the floor.  A particle next to a grounded
    wall carries its own reflected image at twice the wall distance; at
    N = 4e4 the closest one sits 5e-8 from a wall and has |phi| ~ 1e7 against
    an rms of 5e4, so one single-precision rounding of that term alone is
    1e-5 of the rms."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.abs(ref), rms(ref))
    return float((np.abs(a - ref) / scale).max())


def charges(bc, n, seed):
    """n uniform charges of +-1; for the periodic box the last one is adjusted
    so that the system stays neutral (odd n gives it charge 0 or +-2)."""
    x, q = W.uniform_neutral(n + (n % 2), 1.0, seed=seed)
    x, q = x[:n].copy(), q[:n].copy()
    if bc == 0:
        q[-1] -= q.sum()
    return x, q


@pytest.mark.parametrize("bc,n,T", [(0, 3000, 1), (0, 3000, 2), (1, 3001, 1), (1, 3001, 2)])
def test_sym_vs_oracle(hs, monkeypatch, bc, n, T):
    # n = 3000: 2 blocks of 1536 rows (24 slices of 64 at T = 1, 12 of 128 at
    # T = 2); the second holds 1464 rows, so its last live slice is ragged
    # (56 rows) and the rest of the block is empty
    announce("sym vs oracle bc=%d n=%d T=%d" % (bc, n, T))
    x, q = charges(bc, n, 41 + n)
    ref = oracle.solve(oracle.make_plan(1.0, bc, 12, 1000, 600, 2.7), x, q)
    plan = hs.Plan(1.0, bc, 12, 1000, 600, 2.7, precision=hs.FP32_COMP)
    e, phi, F, inter = run(hs, plan, x, q, monkeypatch, True, T)
    err_e = abs(e - ref["energy"]) / abs(ref["energy"])
    err_pn = rel_own(inter["phi_near"], ref["phi_near"])
    err_fn = rel_max(inter["field_near"], ref["field_near"])
    err_F = rel_max(F, ref["forces"])
    print("sym bc=%d n=%d T=%d: dE/E %.2e dphi_near %.2e dE_near %.2e dF %.2e"
          % (bc, n, T, err_e, err_pn, err_fn, err_F))
    assert err_e <= 1e-5
    assert err_pn <= 1e-5
    assert err_fn <= 1e-4
    assert err_F <= 1e-4


@pytest.mark.parametrize("bc,n,T", [(0, 40001, 1), (1, 40000, 2)])
def test_sym_vs_tiles(hs, monkeypatch, bc, n, T):
    # n = 40001, T = 1: 32 blocks of 20 slices x 64 rows (31 rounds); the last
    # block holds 321 rows, so its sixth slice has one live row and the other
    # 14 none
    announce("sym vs tiles bc=%d n=%d T=%d" % (bc, n, T))
    x, q = charges(bc, n, 7 + n)
    plan = hs.Plan(1.0, bc, 12, 1000, 600, 2.7, precision=hs.FP32_COMP)
    plan64 = hs.Plan(1.0, bc, 12, 1000, 600, 2.7, precision=hs.FP64)
    e_s, phi_s, F_s, in_s = run(hs, plan, x, q, monkeypatch, True, T)
    e_t, phi_t, F_t, in_t = run(hs, plan, x, q, monkeypatch, False)
    e_d, phi_d, F_d, in_d = run(hs, plan64, x, q, monkeypatch, False)
    for name, (e, pn, fn) in {"sym": (e_s, in_s["phi_near"], in_s["field_near"]),
                              "tiles": (e_t, in_t["phi_near"], in_t["field_near"])}.items():
        err_e = abs(e - e_d) / abs(e_d)
        err_pn = rel_own(pn, in_d["phi_near"])
        err_fn = rel_max(fn, in_d["field_near"])
        print("%s bc=%d n=%d: dE/E %.2e dphi_near %.2e dE_near %.2e" % (name, bc, n, err_e, err_pn, err_fn))
        assert err_e <= 1e-5
        assert err_pn <= 1e-5
        assert err_fn <= 1e-4
    # each kernel is within 1e-5 of the double-precision path, so they are
    # within 2e-5 of each other
    assert rel_own(in_s["phi_near"], in_t["phi_near"]) <= 2e-5


@pytest.mark.parametrize("bc,n", [(1, 1), (1, 2), (0, 2), (0, 64), (1, 65)])
def test_sym_small(hs, monkeypatch, bc, n):
    announce("sym small bc=%d n=%d" % (bc, n))
    if n == 1:
        x, q = np.array([[0.3, 0.6, 0.45]]), np.array([1.0])
    else:
        x, q = charges(bc, n, 100 + n)
    ref = oracle.solve(oracle.make_plan(1.0, bc, 8, 1000, 600, 2.7), x, q)
    plan = hs.Plan(1.0, bc, 8, 1000, 600, 2.7, precision=hs.FP32_COMP)
    e, phi, F, inter = run(hs, plan, x, q, monkeypatch, True, 1)
    err_pn = rel_max(inter["phi_near"], ref["phi_near"])
    err_fn = rel_max(inter["field_near"], ref["field_near"])
    print("sym small bc=%d n=%d: dphi_near %.2e dE_near %.2e" % (bc, n, err_pn, err_fn))
    assert err_pn <= 1e-5
    assert err_fn <= 1e-4
    assert abs(e - ref["energy"]) <= 1e-5 * abs(ref["energy"])


def test_sym_adjoint(hs, monkeypatch):
    announce("sym adjoint")
    x, q = charges(0, 3000, 77)
    plan = hs.Plan(1.0, 0, 12, 1000, 600, 2.7, precision=hs.FP32_COMP)
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    qd = torch.tensor(q, dtype=torch.float64, device="cuda")
    out = {}
    for sym in (True, False):
        monkeypatch.setenv("HSMA_SYM", "1" if sym else "0")
        e, gx, gq = plan.energy_grad(xd, qd)
        torch.cuda.synchronize()
        out[sym] = (e, gx.cpu().numpy(), gq.cpu().numpy())
    (e1, gx1, gq1), (e0, gx0, gq0) = out[True], out[False]
    print("sym adjoint: dE %.2e dgx %.2e dgq %.2e"
          % (abs(e1 - e0) / abs(e0), rel_max(gx1, gx0), rel_max(gq1, gq0, rms(gq0))))
    assert abs(e1 - e0) <= 1e-5 * abs(e0)
    assert rel_max(gx1, gx0) <= 1e-4
    assert rel_max(gq1, gq0, rms(gq0)) <= 1e-5


@pytest.mark.parametrize("bc,n", [(0, 3000), (1, 3001), (0, 2), (1, 1)])
def test_sym_f64_vs_oracle(hs, monkeypatch, bc, n):
    # double precision: the same gates as the double tile path (1e-10)
    announce("sym f64 vs oracle bc=%d n=%d" % (bc, n))
    if n == 1:
        x, q = np.array([[0.3, 0.6, 0.45]]), np.array([1.0])
    else:
        x, q = charges(bc, n, 211 + n)
    ref = oracle.solve(oracle.make_plan(1.0, bc, 12, 1000, 600, 2.7), x, q)
    plan = hs.Plan(1.0, bc, 12, 1000, 600, 2.7, precision=hs.FP64)
    e, phi, F, inter = run(hs, plan, x, q, monkeypatch, True)
    err_e = abs(e - ref["energy"]) / abs(ref["energy"])
    err_pn = rel_own(inter["phi_near"], ref["phi_near"])
    err_fn = rel_max(inter["field_near"], ref["field_near"])
    err_F = rel_max(F, ref["forces"])
    print("sym f64 bc=%d n=%d: dE/E %.2e dphi_near %.2e dE_near %.2e dF %.2e"
          % (bc, n, err_e, err_pn, err_fn, err_F))
    assert err_e <= 1e-10
    assert err_pn <= 1e-10
    assert err_fn <= 1e-10
    assert err_F <= 1e-10


_ODD_REF = {}


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("bc", [0, 1])
def test_sym_odd_block_count_vs_oracle(hs, monkeypatch, bc, prec):
    """An odd block count, where one block sits out every round.  Block sizes
    are chosen to make the count even unless the slices reach their limit of
    64, so the default schedule gives an odd count only above ~5e5 particles;
    two rounds forced at n = 12000 give 3 blocks of 64 slices x 64 rows.  The
    last block holds 3808 rows: 59 full slices, one of 32 rows, four empty."""
    n = 12000
    announce("sym odd blocks vs oracle bc=%d %s" % (bc, prec))
    monkeypatch.setenv("HSMA_SYM", "1")
    monkeypatch.setenv("HSMA_SYM_T", "1")
    monkeypatch.setenv("HSMA_SYM_ROUNDS", "2")
    x, q = charges(bc, n, 301 + bc)
    if bc not in _ODD_REF:
        _ODD_REF[bc] = oracle.solve(oracle.make_plan(1.0, bc, 12, 1000, 600, 2.7), x, q)
    ref = _ODD_REF[bc]
    plan = hs.Plan(1.0, bc, 12, 1000, 600, 2.7,
                   precision=hs.FP32_COMP if prec == "fp32" else hs.FP64)
    sc = plan.near_schedule(n)
    assert sc["kind"] == 1 and sc["slices"] == 64 and sc["block"] == 4096, sc
    assert sc["blocks"] == 3 and sc["launches"] == 4, sc
    e, phi, F, inter = run(hs, plan, x, q, monkeypatch, True, 1)
    err_e = abs(e - ref["energy"]) / abs(ref["energy"])
    err_pn = rel_own(inter["phi_near"], ref["phi_near"])
    err_fn = rel_max(inter["field_near"], ref["field_near"])
    err_F = rel_max(F, ref["forces"])
    print("sym odd blocks bc=%d %s: dE/E %.2e dphi_near %.2e dE_near %.2e dF %.2e"
          % (bc, prec, err_e, err_pn, err_fn, err_F))
    if prec == "fp32":
        assert err_e <= 1e-5
        assert err_pn <= 1e-5
        assert err_fn <= 1e-4
        assert err_F <= 1e-4
    else:
        assert max(err_e, err_pn, err_fn, err_F) <= 1e-10


@pytest.mark.parametrize("bc,n", [(0, 40001), (1, 40000)])
def test_sym_f64_vs_tiles(hs, monkeypatch, bc, n):
    announce("sym f64 vs tiles bc=%d n=%d" % (bc, n))
    x, q = charges(bc, n, 17 + n)
    plan = hs.Plan(1.0, bc, 12, 1000, 600, 2.7, precision=hs.FP64)
    e_s, phi_s, F_s, in_s = run(hs, plan, x, q, monkeypatch, True)
    e_t, phi_t, F_t, in_t = run(hs, plan, x, q, monkeypatch, False)
    d_e = abs(e_s - e_t) / abs(e_t)
    d_pn = rel_own(in_s["phi_near"], in_t["phi_near"])
    d_fn = rel_max(in_s["field_near"], in_t["field_near"])
    print("sym f64 vs tiles bc=%d n=%d: dE/E %.2e dphi_near %.2e dE_near %.2e" % (bc, n, d_e, d_pn, d_fn))
    assert d_e <= 1e-11
    assert d_pn <= 1e-11
    assert d_fn <= 1e-11


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_sym_slab_vs_oracle(hs, monkeypatch, prec):
    # the slab: real charges only, each pair with its periodic and mirror blocks;
    # n = 2000: 32 blocks of 64 (T = 1), last block 16 rows
    announce("sym slab vs oracle %s" % prec)
    x, q = W.slab_charges(2000, 1.0, seed=23)
    ref = oracle.solve(oracle.make_plan(1.0, 2, 12, 1000, 600, 2.7), x, q)
    plan = hs.Plan(1.0, 2, 12, 1000, 600, 2.7, precision=hs.FP32_COMP if prec == "fp32" else hs.FP64)
    e, phi, F, inter = run(hs, plan, x, q, monkeypatch, True, 1)
    err_e = abs(e - ref["energy"]) / abs(ref["energy"])
    err_pn = rel_own(inter["phi_near"], ref["phi_near"])
    err_fn = rel_max(inter["field_near"], ref["field_near"])
    err_F = rel_max(F, ref["forces"])
    print("sym slab %s: dE/E %.2e dphi_near %.2e dE_near %.2e dF %.2e" % (prec, err_e, err_pn, err_fn, err_F))
    tol = (1e-5, 1e-5, 1e-4) if prec == "fp32" else (1e-10, 1e-10, 1e-10)
    assert err_e <= tol[0]
    assert err_pn <= tol[1]
    assert err_fn <= tol[2]
    assert err_F <= tol[2]


def test_sym_slab_vs_tiles(hs, monkeypatch):
    announce("sym slab vs tiles")
    x, q = W.slab_charges(40000, 1.0, seed=29)
    plan = hs.Plan(1.0, 2, 12, 1000, 600, 2.7, precision=hs.FP32_COMP)
    plan64 = hs.Plan(1.0, 2, 12, 1000, 600, 2.7, precision=hs.FP64)
    e_s, _, _, in_s = run(hs, plan, x, q, monkeypatch, True)
    e_t, _, _, in_t = run(hs, plan, x, q, monkeypatch, False)
    e_d, _, _, in_d = run(hs, plan64, x, q, monkeypatch, False)
    e_d1, _, _, in_d1 = run(hs, plan64, x, q, monkeypatch, True)
    for name, (e, pn, fn) in {"sym": (e_s, in_s["phi_near"], in_s["field_near"]),
                              "tiles": (e_t, in_t["phi_near"], in_t["field_near"])}.items():
        err_e = abs(e - e_d) / abs(e_d)
        err_pn = rel_own(pn, in_d["phi_near"])
        err_fn = rel_max(fn, in_d["field_near"])
        print("slab %s: dE/E %.2e dphi_near %.2e dE_near %.2e" % (name, err_e, err_pn, err_fn))
        assert err_e <= 1e-5
        assert err_pn <= 1e-5
        assert err_fn <= 1e-4
    d_pn = rel_own(in_d1["phi_near"], in_d["phi_near"])
    d_fn = rel_max(in_d1["field_near"], in_d["field_near"])
    print("slab f64 sym vs tiles: dE/E %.2e dphi_near %.2e dE_near %.2e" % (abs(e_d1 - e_d) / abs(e_d), d_pn, d_fn))
    assert abs(e_d1 - e_d) <= 1e-11 * abs(e_d)
    assert d_pn <= 1e-11
    assert d_fn <= 1e-11


def test_sym_slab_adjoint(hs, monkeypatch):
    announce("sym slab adjoint")
    x, q = W.slab_charges(3000, 1.0, seed=31)
    plan = hs.Plan(1.0, 2, 12, 1000, 600, 2.7, precision=hs.FP32_COMP)
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    qd = torch.tensor(q, dtype=torch.float64, device="cuda")
    out = {}
    for sym in (True, False):
        monkeypatch.setenv("HSMA_SYM", "1" if sym else "0")
        e, gx, gq = plan.energy_grad(xd, qd)
        torch.cuda.synchronize()
        out[sym] = (e, gx.cpu().numpy(), gq.cpu().numpy())
    (e1, gx1, gq1), (e0, gx0, gq0) = out[True], out[False]
    print("sym slab adjoint: dE %.2e dgx %.2e dgq %.2e"
          % (abs(e1 - e0) / abs(e0), rel_max(gx1, gx0), rel_max(gq1, gq0, rms(gq0))))
    assert abs(e1 - e0) <= 1e-5 * abs(e0)
    assert rel_max(gx1, gx0) <= 1e-4
    assert rel_max(gq1, gq0, rms(gq0)) <= 1e-5


def test_near_schedule_query(hs, monkeypatch):
    announce("near schedule query")
    monkeypatch.delenv("HSMA_SYM", raising=False)
    monkeypatch.delenv("HSMA_SYM_T", raising=False)
    monkeypatch.delenv("HSMA_SYM_MIN", raising=False)
    plan = hs.Plan(1.0, 0, 12, 1000, 600, 2.7, precision=hs.FP32_COMP)
    small = plan.near_schedule(1000)
    assert small["kind"] == 0 and small["launches"] == 0
    # every boundary condition (their kernels differ in resident waves, which
    # sets the part count) and both precisions
    plans = [plan] + [hs.Plan(1.0, bc, 12, 1000, 600, 2.7, precision=pr)
                      for bc, pr in ((1, hs.FP32_COMP), (2, hs.FP32_COMP), (0, hs.FP64), (1, hs.FP64))]
    for pl in plans:
        for n in (1024, 3000, 5120, 10000, 40001, 200000, 10 ** 6):
            sc = pl.near_schedule(n)
            assert sc["kind"] == 1 and sc["rows_per_lane"] == 1
            assert sc["block"] == 64 * sc["slices"] and 1 <= sc["slices"] <= 64
            assert sc["blocks"] * sc["block"] >= n > (sc["blocks"] - 1) * sc["block"]
            assert sc["launches"] == sc["blocks"] + (sc["blocks"] & 1)
            # at most 64 column parts of at least 16 columns
            assert 1 <= sc["parts"] <= 64 and sc["block"] // sc["parts"] >= 16
            # an even block count (no idle block per round) unless slices are
            # at their limit
            assert sc["blocks"] % 2 == 0 or sc["slices"] == 64, (n, sc)
    monkeypatch.setenv("HSMA_SYM", "0")
    assert plan.near_schedule(10 ** 6)["kind"] == 0
    monkeypatch.setenv("HSMA_SYM", "1")
    assert plan.near_schedule(5)["kind"] == 1
    # the sphere near set always runs per target
    sph = hs.Plan(1.0, 0, 12, 1000, 600, 2.7, precision=hs.FP32_COMP, near_mode=hs.NEAR_SPHERE)
    assert sph.near_schedule(10 ** 6)["kind"] == 0
    with pytest.raises(Exception):
        plan.near_schedule(0)
