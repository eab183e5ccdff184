"""Adjoint (exact gradient of the computed energy) on the GPU.

Checked against the oracle's adjoint, against finite differences of the GPU
FP64 energy (exact for dE/dq: E is quadratic in q), the Euler identity
sum_j q_j dE/dq_j = 2E, and through torch.autograd.
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


def inputs(bc, n, seed):
    if bc == 2:
        return W.slab_charges(n, 1.0, seed)
    return W.uniform_neutral(n, 1.0, seed)


def dev(a):
    return torch.tensor(a, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("bc,n,p,K,M", [
    (0, 600, 10, 600, 1000),
    (1, 777 + 1, 12, 900, 1000),
    (2, 500, 10, 600, 1000),
])
def test_adjoint_fp64_vs_oracle(hs, bc, n, p, K, M):
    announce("adjoint fp64 bc=%d n=%d" % (bc, n))
    x, q = inputs(bc, n, 50 + bc)
    E0, dx0, dq0 = oracle.adjoint(oracle.make_plan(1.0, bc, p, M, K, 2.7), x, q)
    plan = hs.Plan(1.0, bc, p, M, K, 2.7)
    e, dx, dq = plan.energy_grad(dev(x), dev(q))
    dx, dq = dx.cpu().numpy(), dq.cpu().numpy()
    assert abs(e - E0) <= 1e-10 * abs(E0)
    assert rel_max(dq, dq0) <= 1e-9
    assert rel_max(dx, dx0) <= 1e-9
    # Euler identity for a quadratic form
    assert abs(np.sum(q * dq) - 2 * e) <= 1e-10 * abs(e)


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_adjoint_fp64_finite_differences(hs, bc):
    announce("adjoint fd bc=%d" % bc)
    x, q = inputs(bc, 200, 60 + bc)
    x = 0.05 + 0.9 * x if bc != 2 else np.column_stack([x[:, :2], 0.025 + 0.9 * x[:, 2]])
    plan = hs.Plan(1.0, bc, 10, 1000, 600, 2.7)
    e, dx, dq = plan.energy_grad(dev(x), dev(q))
    dx, dq = dx.cpu().numpy(), dq.cpu().numpy()

    def energy(xx, qq):
        return plan.energy_forces(dev(xx), dev(qq))[0]

    # dE/dq along neutral directions: exact up to rounding (E quadratic in q)
    for j, k in ((0, 1), (5, 17), (40, 99)):
        h = 1e-2
        d = np.zeros_like(q)
        d[j], d[k] = h, -h
        fd = (energy(x, q + d) - energy(x, q - d)) / (2 * h)
        assert fd == pytest.approx(dq[j] - dq[k], rel=1e-8, abs=1e-8 * np.abs(dq).max())
    # dE/dx: central differences h = 1e-4 with Richardson extrapolation
    for i, a in ((0, 0), (7, 1), (123, 2)):
        def fd(h):
            e1 = np.zeros_like(x)
            e1[i, a] = h
            return (energy(x + e1, q) - energy(x - e1, q)) / (2 * h)
        rich = (4 * fd(0.5e-4) - fd(1e-4)) / 3
        assert rich == pytest.approx(dx[i, a], rel=1e-6, abs=1e-6 * np.abs(dx).max())


def test_autograd_function(hs):
    announce("autograd")
    x, q = inputs(0, 300, 70)
    plan = hs.Plan(1.0, 0, 8, 1000, 600, 2.7)
    Fn = hs.make_energy_function()
    xt = dev(x).requires_grad_(True)
    qt = dev(q).requires_grad_(True)
    E = Fn.apply(xt, qt, plan)
    (3.0 * E).backward()
    e, dx, dq = plan.energy_grad(dev(x), dev(q))
    assert float(E) == e
    assert torch.equal(xt.grad, 3.0 * dx) and torch.equal(qt.grad, 3.0 * dq)


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_adjoint_fp32_vs_fp64(hs, bc):
    announce("adjoint fp32 bc=%d" % bc)
    x, q = inputs(bc, 2000, 80 + bc)
    p64 = hs.Plan(1.0, bc, 12, 1000, 900, 2.7)
    p32 = hs.Plan(1.0, bc, 12, 1000, 900, 2.7, precision=hs.FP32_COMP)
    e64, dx64, dq64 = p64.energy_grad(dev(x), dev(q))
    e32, dx32, dq32 = p32.energy_grad(dev(x), dev(q))
    assert abs(e32 - e64) <= 1e-5 * abs(e64)
    assert rel_max(dq32.cpu().numpy(), dq64.cpu().numpy()) <= 1e-5
    assert rel_max(dx32.cpu().numpy(), dx64.cpu().numpy()) <= 1e-4
