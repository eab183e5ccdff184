"""Single-precision arrays at the device entry point
(hsma_energy_forces_device_typed): inputs that are exactly representable in
float give, after widening, the same double arithmetic as the double entry
point, so the energy is bitwise equal and phi, F are the double results
rounded to float, for every boundary condition and both plan precisions."""
import ctypes

import numpy as np
import pytest

from gpu_util import announce
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


def system(bc, n, seed):
    if bc == 2:
        x, q = W.slab_charges(n, 1.0, seed)
    else:
        x, q = W.uniform_neutral(n, 1.0, seed)
    return x.astype(np.float32).astype(np.float64), q


@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("prec", [0, 1])
def test_float_arrays_match_double_arrays(hs, bc, prec):
    announce("dtype f32 bc=%d precision=%d" % (bc, prec))
    x, q = system(bc, 3000, 17 + bc)
    plan = hs.Plan(1.0, bc, 8, 1000, 300, 2.7, precision=prec)
    x64, q64 = torch.tensor(x, device="cuda"), torch.tensor(q, device="cuda")
    e64, phi64, F64 = plan.energy_forces(x64, q64)
    e32, phi32, F32 = plan.energy_forces(x64.float(), q64.float())
    torch.cuda.synchronize()
    assert phi32.dtype == torch.float32 and F32.dtype == torch.float32
    assert e32 == e64
    assert torch.equal(phi32, phi64.float())
    assert torch.equal(F32, F64.float())


def test_dtype_rejected(hs):
    announce("dtype rejection")
    plan = hs.Plan(1.0, 0, 8, 1000, 300, 2.7)
    x, q = system(0, 100, 3)
    xd, qd = torch.tensor(x, device="cuda"), torch.tensor(q, device="cuda")
    ws = plan.workspace(100, xd.device)
    phi = torch.empty(100, dtype=torch.float64, device="cuda")
    F = torch.empty((100, 3), dtype=torch.float64, device="cuda")
    e = ctypes.c_double(7.0)
    st = hs.load().hsma_energy_forces_device_typed(
        plan._h, xd.data_ptr(), qd.data_ptr(), 100, 2, None, ws.data_ptr(), ws.numel(), ctypes.byref(e),
        phi.data_ptr(), F.data_ptr())
    assert st == -1 and e.value == 7.0
