"""The dielectric box (Eq. (diel), image weights gamma^|k|, |gamma| < 1) on the
GPU against the oracle's dielectric mode, in double precision."""
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


def inside(n, seed):
    """n charges of +-1 (not necessarily neutral) strictly inside the box."""
    rng = np.random.default_rng(seed)
    x = 0.02 + 0.96 * rng.random((n, 3))
    q = rng.choice([-1.0, 1.0], n)
    return x, q


@pytest.mark.parametrize("gamma,n,p,shells,far", [
    (0.3, 300, 10, 8, "surface"),
    (-0.45, 1000, 10, 8, "surface"),     # ragged target tiles (1000 = 3 x 256 + 232)
    (0.3, 64, 8, 0, "surface"),          # the library's automatic shell count
    (0.6, 257, 12, 6, "direct"),
])
def test_dielectric_box_vs_oracle(hs, gamma, n, p, shells, far):
    announce("dielectric gamma=%.2f n=%d p=%d shells=%d far=%s" % (gamma, n, p, shells, far))
    x, q = inside(n, 100 + n)
    K = 2 * (p + 1) ** 2
    plan = hs.Plan(1.0, hs.BC_DIELECTRIC, p, 1000, K, 2.7, gamma=gamma, far_shells=shells,
                   far_mode=hs.FAR_DIRECT if far == "direct" else hs.FAR_SURFACE)
    S = plan.info["far_shells"]
    assert plan.info["bc"] == 3 and abs(plan.info["gamma"] - gamma) == 0.0
    if shells == 0:
        assert S == oracle.far_shell_count(gamma, 1e-13)
    else:
        assert S == shells
    ref = oracle.solve(oracle.make_plan(1.0, oracle.BC_DIELECTRIC, p, 1000, K, 2.7, gamma=gamma,
                                        shells=S), x, q, far=far)
    e, phi, F, inter = plan.energy_forces(torch.tensor(x, device="cuda"), torch.tensor(q, device="cuda"),
                                          intermediates=True)
    phi, F = phi.cpu().numpy(), F.cpu().numpy()
    b = inter["b"].cpu().numpy()
    A = inter["A"].cpu().numpy()
    errs = dict(b=rel_max(b, ref["b"]), A=rel_max(A, ref["A"]),
                E=abs(e - ref["energy"]) / abs(ref["energy"]), phi=rel_max(phi, ref["phi"], rms(ref["phi"])),
                F=rel_max(F, ref["forces"]))
    print("dielectric: " + " ".join("%s %.2e" % kv for kv in errs.items()))
    assert errs["b"] <= 1e-10 and errs["A"] <= 1e-8
    assert errs["E"] <= 1e-10 and errs["phi"] <= 1e-10 and errs["F"] <= 1e-10


def test_dielectric_gamma_zero_is_free_space(hs):
    """No image carries charge at gamma = 0: the energy is the bare Coulomb
    energy of the charges."""
    announce("dielectric gamma=0")
    x, q = inside(200, 7)
    plan = hs.Plan(1.0, hs.BC_DIELECTRIC, 8, 1000, 300, 2.7, gamma=0.0)
    e, phi, F = plan.energy_forces(torch.tensor(x, device="cuda"), torch.tensor(q, device="cuda"))
    d = np.linalg.norm(x[:, None, :] - x[None, :, :], axis=-1)
    np.fill_diagonal(d, np.inf)
    E = 0.5 * np.sum(q[:, None] * q[None, :] / d)
    assert abs(e - E) <= 1e-12 * abs(E)


def test_dielectric_rejections(hs):
    """Single precision, the sphere near set, |gamma| >= 1, positions outside
    the box, the adjoint and the server are refused for the dielectric box."""
    announce("dielectric rejections")
    for kw in (dict(precision=hs.FP32_COMP, gamma=0.3), dict(near_mode=hs.NEAR_SPHERE, gamma=0.3),
               dict(gamma=1.0), dict(gamma=-1.5)):
        with pytest.raises(hs.HsmaError) as ei:
            hs.Plan(1.0, hs.BC_DIELECTRIC, 8, 1000, 300, 2.7, **kw)
        assert ei.value.status == -1
    plan = hs.Plan(1.0, hs.BC_DIELECTRIC, 8, 1000, 300, 2.7, gamma=0.3, far_shells=4)
    x, q = inside(50, 3)
    xd, qd = torch.tensor(x, device="cuda"), torch.tensor(q, device="cuda")
    with pytest.raises(hs.HsmaError):
        plan.energy_grad(xd, qd)
    srv = hs.Server(memory_bytes=64 << 20, max_active=2, precision=hs.FP64)
    with pytest.raises(hs.HsmaError):
        srv.submit(plan, x, q)
    srv.close()
    bad = x.copy()
    bad[3, 1] = 1.2
    with pytest.raises(hs.HsmaError) as ei:
        plan.energy_forces(torch.tensor(bad, device="cuda"), qd)
    assert ei.value.status == -3
