"""The allocation-free entry point (static device scratch) against the
workspace entry point through the C ABI, on two calls in a row with the
second smaller, in both precisions."""
import numpy as np
import pytest

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


def both_paths(hs, plan, x, q):
    xd = torch.tensor(x, device="cuda")
    qd = torch.tensor(q, device="cuda")
    e0, phi0, F0 = plan.energy_forces(xd, qd)
    phi1 = torch.full_like(phi0, float("nan"))
    F1 = torch.full_like(F0, float("nan"))
    e1 = plan.energy_forces_noalloc(xd, qd, phi1, F1)
    torch.cuda.synchronize()
    return (e0, phi0.cpu().numpy(), F0.cpu().numpy()), (e1, phi1.cpu().numpy(), F1.cpu().numpy())


@pytest.mark.parametrize("bc,precision", [(0, 0), (1, 0), (0, 1), (2, 1)])
def test_noalloc_matches_workspace_entry_point(hs, bc, precision):
    plan = hs.Plan(1.0, bc, 8, 640, 640, 2.7, precision=precision)
    tol_e, tol_p, tol_f = (1e-10, 1e-10, 1e-10) if precision == 0 else (1e-5, 1e-5, 1e-4)
    for n in (6000, 1500):     # pair-once near sum, then a smaller call
        announce("noalloc bc=%d precision=%d n=%d" % (bc, precision, n))
        x, q = W.slab_charges(n, 1.0, 70 + n) if bc == 2 else W.uniform_neutral(n, 1.0, 70 + n)
        (e0, phi0, F0), (e1, phi1, F1) = both_paths(hs, plan, x, q)
        print("noalloc bc=%d prec=%d n=%d: dE/E %.2e dphi %.2e dF %.2e"
              % (bc, precision, n, abs(e1 - e0) / abs(e0), rel_max(phi1, phi0, rms(phi0)),
                 rel_max(F1, F0)))
        assert np.isfinite(e1) and np.all(np.isfinite(phi1)) and np.all(np.isfinite(F1))
        assert abs(e1 - e0) <= tol_e * abs(e0)
        assert rel_max(phi1, phi0, rms(phi0)) <= tol_p
        assert rel_max(F1, F0) <= tol_f


def test_noalloc_rejects_sizes_beyond_its_scratch(hs):
    announce("noalloc size limit")
    plan = hs.Plan(1.0, 0, 8, 640, 640, 2.7)
    n = 300000
    x, q = W.uniform_neutral(n, 1.0, 5)
    xd = torch.tensor(x, device="cuda")
    qd = torch.tensor(q, device="cuda")
    phi = torch.empty(n, dtype=torch.float64, device="cuda")
    F = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(hs.HsmaError) as ei:
        plan.energy_forces_noalloc(xd, qd, phi, F)
    assert ei.value.status == -5
    # the entry point still works afterwards
    x, q = W.uniform_neutral(800, 1.0, 6)
    (e0, phi0, _), (e1, phi1, _) = both_paths(hs, plan, x, q)
    assert abs(e1 - e0) <= 1e-10 * abs(e0)
