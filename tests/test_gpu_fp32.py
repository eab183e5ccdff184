"""FP32-compensated path against the oracle (GPU, through the C ABI).

Gate: |dE|/|E| <= 1e-5.  Potential and force errors are bounded too, at the
level single-precision terms with compensated sums give (stated per test).
"""
import numpy as np
import pytest

import oracle
from gpu_util import announce, rel_max, rms
from paper_1806_04801_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_E32 = 1e-5


@pytest.fixture(scope="module")
def hs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04801_amd import hsma
    hsma.load()
    return hsma


def gpu(hs, plan, x, q):
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    qd = torch.tensor(q, dtype=torch.float64, device="cuda")
    e, phi, F, inter = plan.energy_forces(xd, qd, intermediates=True)
    torch.cuda.synchronize()
    return e, phi.cpu().numpy(), F.cpu().numpy(), {k: v.cpu().numpy() for k, v in inter.items()}


@pytest.mark.parametrize("bc,n,p,K,M", [
    (0, 4000, 12, 600, 1000),
    (1, 3001, 16, 2000, 2500),
    (2, 2000, 12, 600, 1000),
    (0, 2, 6, 300, 500),
])
def test_fp32_comp_vs_oracle(hs, bc, n, p, K, M):
    announce("fp32 parity bc=%d n=%d" % (bc, n))
    if bc == 2:
        x, q = W.slab_charges(n, 1.0, seed=21)
    else:
        x, q = W.uniform_neutral(n + (n % 2), 1.0, seed=31 + n)
        x, q = x[:n], q[:n]
    ref = oracle.solve(oracle.make_plan(1.0, bc, p, M, K, 2.7), x, q)
    plan = hs.Plan(1.0, bc, p, M, K, 2.7, precision=hs.FP32_COMP)
    e, phi, F, inter = gpu(hs, plan, x, q)
    err_e = abs(e - ref["energy"]) / abs(ref["energy"])
    err_phi = rel_max(phi, ref["phi"], rms(ref["phi"]))
    err_F = rel_max(F, ref["forces"])
    print("fp32 bc=%d n=%d: dE/E %.2e dphi %.2e dF %.2e" % (bc, n, err_e, err_phi, err_F))
    assert err_e <= TOL_E32
    assert err_phi <= 1e-5
    assert err_F <= 1e-4
    # each single-precision term carries ~6e-8 relative error, so b errs by
    # about 6e-8 sqrt(sum 1/r^2) over its 27N image terms (a few 1e-5 here)
    assert rel_max(inter["b"], ref["b"]) <= 1e-4


def test_fp32_close_pairs_and_walls(hs):
    """Pairs 1e-5 apart and charges 1e-6 from a grounded wall: the split
    hi/lo coordinates keep the image distances accurate."""
    announce("fp32 close pairs")
    rng = np.random.default_rng(4)
    base = rng.random((50, 3)) * 0.8 + 0.1
    x = np.concatenate([base, base + 1e-5 * rng.standard_normal((50, 3))])
    x[0] = [1e-6, 0.5, 0.5]
    x[50] = [1e-6 + 2e-6, 0.5, 0.5]
    q = np.concatenate([np.ones(50), -np.ones(50)])
    ref = oracle.solve(oracle.make_plan(1.0, 1, 8, 1000, 600, 2.7), x, q)
    plan = hs.Plan(1.0, 1, 8, 1000, 600, 2.7, precision=hs.FP32_COMP)
    e, phi, F, _ = gpu(hs, plan, x, q)
    assert abs(e - ref["energy"]) / abs(ref["energy"]) <= TOL_E32
    assert rel_max(phi, ref["phi"], np.abs(ref["phi"]).max()) <= 1e-5
    assert rel_max(F, ref["forces"]) <= 1e-4
