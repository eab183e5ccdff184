"""Tin-foil Ewald sums: an independent exact reference for the oracle pins.

Textbook Ewald splitting for a periodic cubic cell of side Lb (no surface
term, i.e. conducting boundary at infinity), written directly in numpy.  The
splitting parameter and cutoffs keep both truncation errors far below 1e-13
for the tiny systems used in the tests.
"""
import math

import numpy as np
from scipy.special import erfc


def ewald(pos, q, Lb, alpha=None, nreal=2, mmax=10):
    """Per-particle potential (bare self term removed), field E = -grad phi and
    energy 1/2 sum q phi for point charges in a periodic cube of side Lb."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    n = len(q)
    a = 4.0 / Lb if alpha is None else alpha
    phi = np.zeros(n)
    fld = np.zeros((n, 3))
    rng = range(-nreal, nreal + 1)
    shifts = np.array([(i, j, k) for i in rng for j in rng for k in rng], dtype=np.float64) * Lb
    d0 = pos[:, None, :] - pos[None, :, :]             # r_i - r_j
    for s in shifts:
        d = d0 + s
        r = np.sqrt(np.sum(d * d, axis=2))
        if not s.any():
            np.fill_diagonal(r, np.inf)
        er = erfc(a * r) / r
        phi += er @ q
        g = (er + 2.0 * a / math.sqrt(math.pi) * np.exp(-a * a * r * r)) / (r * r)
        fld += np.einsum("ij,ijc,j->ic", g, d, q)
    V = Lb ** 3
    m = np.arange(-mmax, mmax + 1)
    K = np.array([(i, j, k) for i in m for j in m for k in m if (i, j, k) != (0, 0, 0)],
                 dtype=np.float64) * (2.0 * math.pi / Lb)
    k2 = np.sum(K * K, axis=1)
    f = 4.0 * math.pi / V * np.exp(-k2 / (4.0 * a * a)) / k2
    kr = pos @ K.T                                      # n x nk
    S = (q[:, None] * np.exp(1j * kr)).sum(axis=0)      # structure factor
    z = S[None, :] * np.exp(-1j * kr)                   # sum_j q_j e^{-i k.(r_i - r_j)}
    phi += (z.real * f[None, :]).sum(axis=1)
    fld += (z.imag * f[None, :]) @ K * -1.0
    phi -= 2.0 * a / math.sqrt(math.pi) * q
    return phi, fld, 0.5 * float(np.sum(q * phi))


def grounded_cube(pos_api, q, L):
    """Charges in a grounded cube [0,L]^3: the 8 mirror copies form a neutral
    cell of side 2L whose periodic (absolutely convergent) sum is the
    grounded-cube potential.  Returns phi, field and energy of the real
    charges."""
    pos_api = np.asarray(pos_api, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    P, Q = [], []
    for sx in (0, 1):
        for sy in (0, 1):
            for sz in (0, 1):
                p = pos_api.copy()
                if sx:
                    p[:, 0] = -p[:, 0]
                if sy:
                    p[:, 1] = -p[:, 1]
                if sz:
                    p[:, 2] = -p[:, 2]
                P.append(p)
                Q.append(q * (-1.0) ** (sx + sy + sz))
    P = np.concatenate(P)
    Q = np.concatenate(Q)
    phi, fld, _ = ewald(P, Q, 2.0 * L)
    n = len(q)
    return phi[:n], fld[:n], 0.5 * float(np.sum(q * phi[:n]))


def grounded_slab(pos_api, q, L):
    """Charges between grounded walls z = 0 and z = L/2, periodic in x, y with
    period L: the mirror charges -q at z -> -z make a cube of side L whose
    tin-foil periodic sum vanishes on both walls."""
    pos_api = np.asarray(pos_api, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    m = pos_api.copy()
    m[:, 2] = -m[:, 2]
    P = np.concatenate([pos_api, m])
    Q = np.concatenate([q, -q])
    phi, fld, _ = ewald(P, Q, L)
    n = len(q)
    return phi[:n], fld[:n], 0.5 * float(np.sum(q * phi[:n]))
