"""HSMA oracle -- test infrastructure only.

A plain, slow, double-precision CPU implementation of the harmonic surface
mapping algorithm (Zhao, Liang & Xu, arXiv:1806.04801), written from the paper
to check the GPU library.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
GPU library (``paper_1806_04801_amd``) and imports nothing from it.

Pinning (see tests/test_oracle_*.py): Madelung constant of rock salt (Sec. III),
tin-foil Ewald sums (periodic, grounded cube via its 2L-periodic mirror cell,
grounded slab via its doubled cell), closed forms of the quadrature and of the
low-degree solid harmonics, Laplace residual of the basis, recovery of a planted
harmonic polynomial by the least-squares step, agreement of the exact dipole
with the paper's central-difference charge layers, and finite differences of
the adjoint.  Every oracle function is pinned by at least one of these.
"""
from .hsma import (  # noqa: F401
    BC_PERIODIC, BC_METALLIC, BC_SLAB, BC_DIELECTRIC,
    normalize, monitoring_points, fibonacci_pair, integration_points,
    basis, householder_qr, qr_solve_ls, qr_apply_q,
    make_plan, solve, adjoint, splitmix64_uniform,
    near_sum, potential_at, surface_sum, charges_sum, check_adjoint,
    surface_images_paper_literal, sphere_images, near_explicit,
    basis_gradient, far_field_direct, far_shells, image_series, far_shell_count,
)
