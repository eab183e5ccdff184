"""The paper's literal near set (every image inside the auxiliary sphere) on
the GPU against the oracle's sphere mode."""
import math

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


@pytest.mark.parametrize("bc,n,p,alpha,precision", [
    (0, 1000, 12, 1.3, 0),
    (0, 777 + 1, 10, 2.0, 0),
    (1, 600, 12, 1.5, 0),
    (2, 500, 10, 2.0, 0),
    (0, 2000, 12, 1.3, 1),
    (1, 1000, 10, 2.0, 1),
])
def test_sphere_near_set_vs_oracle(hs, bc, n, p, alpha, precision):
    announce("sphere bc=%d n=%d alpha=%.1f prec=%d" % (bc, n, alpha, precision))
    x, q = W.slab_charges(n, 1.0, 9) if bc == 2 else W.uniform_neutral(n, 1.0, 9 + n)
    R = alpha * math.sqrt(3.0) / 2.0
    K = max(2 * p * p, (p + 1) ** 2 + 50)
    ref = oracle.solve(oracle.make_plan(1.0, bc, p, 1976, K, R), x, q, near="sphere")
    plan = hs.Plan(1.0, bc, p, 1976, K, R, precision=precision, near_mode=hs.NEAR_SPHERE)
    e, phi, F, inter = plan.energy_forces(torch.tensor(x, device="cuda"),
                                          torch.tensor(q, device="cuda"), intermediates=True)
    phi, F = phi.cpu().numpy(), F.cpu().numpy()
    b = inter["b"].cpu().numpy()
    if precision == 0:
        assert rel_max(b, ref["b"]) <= 1e-10
        assert abs(e - ref["energy"]) <= 1e-10 * abs(ref["energy"])
        assert rel_max(phi, ref["phi"], rms(ref["phi"])) <= 1e-10
        assert rel_max(F, ref["forces"]) <= 1e-10
    else:
        # the single-precision gate: relative energy error 1e-5
        print("sphere fp32: |dE|/|E| %.3e" % (abs(e - ref["energy"]) / abs(ref["energy"])))
        assert abs(e - ref["energy"]) <= 1e-5 * abs(ref["energy"])
        assert rel_max(phi, ref["phi"], rms(ref["phi"])) <= 1e-5
        assert rel_max(F, ref["forces"]) <= 1e-4


def test_sphere_mode_rejected_by_adjoint_and_server(hs):
    announce("sphere rejections")
    plan = hs.Plan(1.0, 0, 8, 1000, 600, 1.3 * math.sqrt(3) / 2, near_mode=hs.NEAR_SPHERE)
    x, q = W.uniform_neutral(20, 1.0, 1)
    with pytest.raises(hs.HsmaError):
        plan.energy_grad(torch.tensor(x, device="cuda"), torch.tensor(q, device="cuda"))
    srv = hs.Server(memory_bytes=64 << 20, max_active=2)
    with pytest.raises(hs.HsmaError):
        srv.submit(plan, x, q)


@pytest.mark.parametrize("bc,near,dr_rel", [(0, "sphere", 1e-5), (1, "block", 1e-4), (2, "sphere", 1e-5)])
def test_paper_charge_layers_vs_oracle(hs, bc, near, dr_rel):
    """The paper's dipole discretization (two charge layers at R_s -+ dr/2,
    dr = 1e-5 R_s, or 1e-4 R_s as for its grounded example) against the
    oracle's charge layers; the layers cancel by R_s/dr, so the bound is
    looser than for exact dipoles."""
    announce("layers bc=%d near=%s" % (bc, near))
    x, q = W.slab_charges(400, 1.0, 8) if bc == 2 else W.uniform_neutral(600, 1.0, 8)
    alpha = 1.3 if near == "sphere" else 3.118
    R = alpha * math.sqrt(3.0) / 2.0
    dr = dr_rel * R
    ref = oracle.solve(oracle.make_plan(1.0, bc, 12, 1976, 400, R), x, q, near=near,
                       dipole="layers", dr=dr)
    plan = hs.Plan(1.0, bc, 12, 1976, 400, R, near_mode=hs.NEAR_SPHERE if near == "sphere" else hs.NEAR_BLOCK,
                   dipole_mode=hs.DIPOLE_LAYERS, dr=dr)
    assert plan.info["dipole_mode"] == 1 and abs(plan.info["dr"] - dr) < 1e-18
    e, phi, F = plan.energy_forces(torch.tensor(x, device="cuda"), torch.tensor(q, device="cuda"))
    phi, F = phi.cpu().numpy(), F.cpu().numpy()
    tol = 1e-16 * R / dr * 1e3
    assert abs(e - ref["energy"]) <= tol * abs(ref["energy"])
    assert rel_max(phi, ref["phi"], rms(ref["phi"])) <= tol
    assert rel_max(F, ref["forces"]) <= 10 * tol
    # the layers approximate the exact dipole to O(dr^2)
    ex = oracle.solve(oracle.make_plan(1.0, bc, 12, 1976, 400, R), x, q, near=near)
    assert abs(e - ex["energy"]) <= 1e-6 * abs(ex["energy"])


@pytest.mark.parametrize("bc,p,precision", [(0, 20, 0), (1, 16, 0), (2, 12, 0), (0, 16, 1)])
def test_direct_far_field_vs_oracle(hs, bc, p, precision):
    """Far field evaluated straight from the fitted series at the particles
    (value and gradient of sum_k A_k B_k) against the oracle's direct form."""
    announce("direct far bc=%d p=%d prec=%d" % (bc, p, precision))
    x, q = W.slab_charges(600, 1.0, 12) if bc == 2 else W.uniform_neutral(1000, 1.0, 12)
    K = 2 * (p + 1) ** 2
    ref = oracle.solve(oracle.make_plan(1.0, bc, p, 2500, K, 2.7), x, q, far="direct")
    plan = hs.Plan(1.0, bc, p, 2500, K, 2.7, precision=precision, far_mode=hs.FAR_DIRECT)
    e, phi, F, inter = plan.energy_forces(torch.tensor(x, device="cuda"),
                                          torch.tensor(q, device="cuda"), intermediates=True)
    po = inter["phi_out"].cpu().numpy()
    fo = inter["field_out"].cpu().numpy()
    if precision == 0:
        assert rel_max(po, ref["phi_out"], rms(ref["phi"])) <= 1e-10
        assert rel_max(fo, ref["field_out"], np.abs(ref["field"]).max()) <= 1e-10
        assert abs(e - ref["energy"]) <= 1e-10 * abs(ref["energy"])
        assert rel_max(F.cpu().numpy(), ref["forces"]) <= 1e-10
    else:
        print("direct fp32: |dE|/|E| %.3e" % (abs(e - ref["energy"]) / abs(ref["energy"])))
        assert abs(e - ref["energy"]) <= 1e-5 * abs(ref["energy"])
    # and it agrees with the surface mapping to the quadrature error (in FP32
    # mode the coefficients carry the single-precision right-hand side)
    sref = oracle.solve(oracle.make_plan(1.0, bc, p, 2500, K, 2.7), x, q)
    assert rel_max(po, sref["phi_out"], rms(sref["phi"])) <= (1e-8 if precision == 0 else 1e-5)
