"""Parity of the HIP path with the oracle (GPU, called through the C ABI).

FP64 bar (per result): |dE|/|E| <= 1e-10, max|dphi|/rms(phi) <= 1e-10,
max|dF|/max|F| <= 1e-10; the stage outputs b, A and the surface strengths are
compared too so that a failure names its stage.
"""
import numpy as np
import pytest

import oracle
from gpu_util import announce, rel_max, rms
from paper_1806_04801_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-10


@pytest.fixture(scope="module")
def hs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04801_amd import hsma
    hsma.load()
    return hsma


def run_gpu(hs, plan, x, q, intermediates=True):
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    qd = torch.tensor(q, dtype=torch.float64, device="cuda")
    out = plan.energy_forces(xd, qd, intermediates=intermediates)
    torch.cuda.synchronize()
    if intermediates:
        e, phi, F, inter = out
        return e, phi.cpu().numpy(), F.cpu().numpy(), {k: v.cpu().numpy() for k, v in inter.items()}
    e, phi, F = out
    return e, phi.cpu().numpy(), F.cpu().numpy(), None


def compare_full(hs, bc, p, M, K, R, x, q, L=1.0, tol=TOL64, stages=True):
    oplan = oracle.make_plan(L, bc, p, M, K, R)
    ref = oracle.solve(oplan, x, q)
    gplan = hs.Plan(L, bc, p, M, K, R)
    assert gplan.info["M_eff"] == len(oplan["S"])
    e, phi, F, inter = run_gpu(hs, gplan, x, q)
    if stages:
        assert rel_max(inter["b"], ref["b"]) < tol, "right-hand side"
        assert rel_max(inter["A"], ref["A"]) < 1e2 * tol, "coefficients"
        assert rel_max(inter["surf"][:, 3], ref["surf"][:, 3]) < 1e2 * tol, "surface charges"
        assert rel_max(inter["surf"][:, 4:7], ref["surf"][:, 4:7]) < 1e2 * tol, "surface dipoles"
        assert rel_max(inter["phi_near"], ref["phi_near"], rms(ref["phi_near"])) < tol, "near phi"
        assert rel_max(inter["field_near"], ref["field_near"]) < tol, "near field"
        assert rel_max(inter["phi_out"], ref["phi_out"], rms(ref["phi"])) < tol, "far phi"
    assert abs(e - ref["energy"]) <= tol * abs(ref["energy"])
    assert rel_max(phi, ref["phi"], rms(ref["phi"])) < tol
    assert rel_max(F, ref["forces"]) < tol
    return e, ref


def test_plan_geometry_matches_oracle(hs):
    for bc, K in ((0, 600), (1, 2000)):
        announce("plan geometry bc=%d" % bc)
        gp = hs.Plan(1.0, bc, 8, 1000, K, 2.7)
        op = oracle.make_plan(1.0, bc, 8, 1000, K, 2.7, seed=hs.DEFAULT_SEED)
        assert np.allclose(gp.points(0), op["X"], rtol=0, atol=1e-14)
        if bc == 0:
            assert np.allclose(gp.points(1), op["Xt"], rtol=0, atol=1e-14)
        S, w = gp.points(2)
        assert np.allclose(S, op["S"], rtol=0, atol=1e-13)
        assert np.allclose(w, op["w"], rtol=1e-13, atol=0)


def test_nacl_madelung_c1(hs):
    """8 ions, periodic, p=8, K=600, M=1000, R=2.7L, FP64."""
    announce("nacl8 periodic p=8")
    x, q, a = W.nacl(2, 1.0)
    e, ref = compare_full(hs, 0, 8, 1000, 600, 2.7, x, q)
    M = -2.0 * a * e / len(q)
    assert abs(M - 1.74756459463318219) / 1.74756459463318219 < 1e-5


@pytest.mark.parametrize("bc,n,p,K,M", [
    (0, 1000, 12, 600, 1000),     # periodic, ragged (1000 = 3 tiles of 256 + 232)
    (1, 1537, 16, 2000, 2500),    # grounded cube, ragged
    (2, 700, 12, 600, 1000),      # slab (1400 sources with the mirrors)
    (1, 3, 8, 600, 1000),         # fewer particles than one wave
    (0, 2, 6, 300, 500),          # two charges
])
def test_small_systems_full_parity(hs, bc, n, p, K, M):
    announce("full parity bc=%d n=%d p=%d" % (bc, n, p))
    if bc == 2:
        x, q = W.slab_charges(n - n % 5 if n % 5 else n, 1.0, seed=11)
    else:
        x, q = W.uniform_neutral(n if n % 2 == 0 else n + 1, 1.0, seed=7 + n)
        if n % 2 and bc == 1:
            x, q = x[:n], q[:n]   # a non-neutral grounded cube is allowed
    compare_full(hs, bc, p, M, K, 2.7, x, q)


def test_metallic_c2_sampled(hs):
    """Grounded cube at full size: N=10,000, p=16, K=2000, M=2500, FP64; the
    oracle computes b, A and the surface images in full and phi, F at 300
    sampled particles."""
    announce("metallic10k sampled")
    c = W.CONFIGS["metallic10k"]
    x, q = W.make_inputs("metallic10k")
    oplan = oracle.make_plan(1.0, 1, c["p"], c["M"], c["K"], c["R"])
    idx = np.random.default_rng(0).choice(len(q), 300, replace=False)
    ref = oracle.solve(oplan, x, q, targets=idx)
    gplan = hs.Plan(1.0, 1, c["p"], c["M"], c["K"], c["R"])
    e, phi, F, inter = run_gpu(hs, gplan, x, q)
    assert rel_max(inter["b"], ref["b"]) < TOL64
    assert rel_max(inter["A"], ref["A"]) < 1e2 * TOL64
    assert rel_max(phi[idx], ref["phi"], rms(ref["phi"])) < TOL64
    assert rel_max(F[idx], ref["forces"]) < TOL64
    # partial energy over the sample
    e_s = 0.5 * np.sum(q[idx] * phi[idx])
    assert abs(e_s - ref["energy"]) <= TOL64 * np.sum(np.abs(q[idx] * phi[idx]))


def test_host_entry_point_matches_device(hs):
    """The host-array entry point equals the device path bitwise, over calls
    that grow, keep and reuse the plan's device buffer."""
    announce("host entry point")
    gplan = hs.Plan(1.0, 0, 10, 1000, 600, 2.7)
    for n, seed in ((500, 3), (3000, 4), (200, 5), (3000, 4)):
        x, q = W.uniform_neutral(n, 1.0, seed=seed)
        e1, phi1, F1 = gplan.energy_forces_host(x, q)
        e2, phi2, F2, _ = run_gpu(hs, gplan, x, q, intermediates=False)
        assert e1 == e2
        assert np.array_equal(phi1, phi2) and np.array_equal(F1, F2)


def test_bitwise_repeatable(hs):
    announce("repeatability")
    x, q = W.uniform_neutral(3000, 1.0, seed=5)
    gplan = hs.Plan(1.0, 0, 12, 1000, 600, 2.7)
    a = run_gpu(hs, gplan, x, q, intermediates=False)
    b = run_gpu(hs, gplan, x, q, intermediates=False)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_error_paths(hs):
    announce("error paths")
    gplan = hs.Plan(1.0, 0, 6, 500, 300, 2.7)
    x, q = W.uniform_neutral(10, 1.0, seed=1)
    with pytest.raises(hs.HsmaError) as ei:
        gplan.energy_forces_host(x, q + 0.1)
    assert ei.value.status == -2
    mplan = hs.Plan(1.0, 1, 6, 500, 300, 2.7)
    xb = x.copy()
    xb[0, 1] = 1.0
    with pytest.raises(hs.HsmaError) as ei:
        mplan.energy_forces_host(xb, q)
    assert ei.value.status == -3
    # same checks on the device entry point (flags raised by the kernels)
    xd = torch.tensor(xb, device="cuda")
    qd = torch.tensor(q, device="cuda")
    with pytest.raises(hs.HsmaError) as ei:
        mplan.energy_forces(xd, qd)
    assert ei.value.status == -3
    with pytest.raises(hs.HsmaError) as ei:
        gplan.energy_forces(torch.tensor(x, device="cuda"), qd + 0.1)
    assert ei.value.status == -2
    xn = x.copy()
    xn[3, 0] = np.nan
    with pytest.raises(hs.HsmaError) as ei:
        gplan.energy_forces(torch.tensor(xn, device="cuda"), qd)
    assert ei.value.status == -1
