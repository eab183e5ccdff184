"""HSMA oracle in double precision (test infrastructure only).

Each function cites the passage of Zhao, Liang & Xu, "Harmonic surface mapping
algorithm for fast electrostatic sums" (arXiv:1806.04801) that it follows.
The heavy pair sums are in ``hsma_oracle.c`` (plain double loops); the rest is
numpy.  Nothing here is blocked, fused or reordered beyond the definitions.

Conventions (readings where the paper is silent):
  * Gaussian units, Phi = sum q/r; energy E = 1/2 sum_i q_i phi_i where phi_i
    leaves out only the bare self term (self-images count).
  * Coordinates given in [0, L)^3 are centred on the box (the paper centres the
    box at the origin, Sec. II.A).
  * Near set = the 27 images of every source in the 3x3x3 block of boxes.
  * Basis B_{nm}(r) = (|r|/R0)^n Y_nm, with Y the orthonormal real spherical
    harmonics without the Condon-Shortley phase, index k = n^2 + n + m.
  * Periodic: A_00 is undetermined by the periodic residual and set to 0.
  * Surface dipole: exact point dipole (the dr -> 0 limit of Eq. (cd)); the
    paper's two charge layers are available for comparison.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

BC_PERIODIC = 0
BC_METALLIC = 1
BC_SLAB = 2  # grounded walls at z = 0 and z = L/2, periodic in x and y
BC_DIELECTRIC = 3  # dielectric box: the image series of Eq. (diel) with |gamma| < 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "hsma_oracle.c")
_lib = None


def build(force=False):
    """Compile the C pair sums (plain -O2, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", _SO, "-lm"])


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        d = ctypes.POINTER(ctypes.c_double)
        lg = ctypes.POINTER(ctypes.c_long)
        L_ = ctypes.c_long
        D = ctypes.c_double
        lib.orc_potential_at.argtypes = [ctypes.c_int, D, D, d, L_, d, L_, d]
        lib.orc_near.argtypes = [ctypes.c_int, D, D, d, L_, lg, L_, d, d]
        lib.orc_far_shells.argtypes = [D, D, d, L_, d, L_, ctypes.c_int, d]
        lib.orc_image_series.argtypes = [ctypes.c_int, D, D, d, L_, lg, L_, ctypes.c_int, d, d]
        lib.orc_surface.argtypes = [d, L_, d, L_, d, d]
        lib.orc_charges.argtypes = [d, L_, d, L_, d, d]
        lib.orc_check_adjoint.argtypes = [ctypes.c_int, D, D, d, L_, d, d, L_, d, d]
        lib.orc_near_explicit.argtypes = [d, lg, L_, d, lg, ctypes.POINTER(ctypes.c_int), L_, d, d]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------
# Pair sums (thin wrappers over the C loops)
# --------------------------------------------------------------------------
def potential_at(bc, L, src, pts, gamma=-1.0):
    """Phi_in at points: all 27 images of every source (Sec. II.A); gamma is
    the image weight of a dielectric box (Eq. (diel))."""
    src, pts = _c(src), _c(pts)
    out = np.zeros(len(pts))
    _load().orc_potential_at(bc, L, gamma, _p(src), len(src), _p(pts), len(pts), _p(out))
    return out


def near_sum(bc, L, src, tidx, gamma=-1.0):
    """phi and E = -grad phi at source targets from the near images (Sec. II.C)."""
    src = _c(src)
    tidx = np.ascontiguousarray(tidx, dtype=np.int64)
    phi = np.zeros(len(tidx))
    fld = np.zeros((len(tidx), 3))
    _load().orc_near(bc, L, gamma, _p(src), len(src),
                     tidx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), len(tidx), _p(phi), _p(fld))
    return phi, fld


def far_shells(L, gamma, src, pts, S):
    """The far part of the dielectric image series at points: images in the
    shells 2 <= max|k_a| <= S with weights gamma^|k| (Eq. (diel))."""
    src, pts = _c(src), _c(pts)
    out = np.zeros(len(pts))
    _load().orc_far_shells(L, gamma, _p(src), len(src), _p(pts), len(pts), int(S), _p(out))
    return out


def image_series(bc, L, src, tidx, S, gamma=-1.0):
    """The image series itself, truncated at shells max|k_a| <= S, at source
    targets (bare self term left out): a reference for the whole method.
    Returns (phi, E) with E = -grad phi, images held fixed."""
    src = _c(src)
    tidx = np.ascontiguousarray(tidx, dtype=np.int64)
    phi = np.zeros(len(tidx))
    fld = np.zeros((len(tidx), 3))
    _load().orc_image_series(bc, L, gamma, _p(src), len(src),
                             tidx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), len(tidx), int(S),
                             _p(phi), _p(fld))
    return phi, fld


def surface_sum(pts, surf):
    """phi and E of the surface charges and exact dipoles (Sec. II.B)."""
    pts, surf = _c(pts), _c(surf)
    phi = np.zeros(len(pts))
    fld = np.zeros((len(pts), 3))
    _load().orc_surface(_p(pts), len(pts), _p(surf), len(surf), _p(phi), _p(fld))
    return phi, fld


def charges_sum(pts, chg):
    """phi and E of plain point charges (no images)."""
    pts, chg = _c(pts), _c(chg)
    phi = np.zeros(len(pts))
    fld = np.zeros((len(pts), 3))
    _load().orc_charges(_p(pts), len(pts), _p(chg), len(chg), _p(phi), _p(fld))
    return phi, fld


def check_adjoint(bc, L, pos, pts, lam):
    """g_j = sum_i lam_i sum_k s_k/|p_i - I_k(r_j)| and its r_j-gradient."""
    pos, pts, lam = _c(pos), _c(pts), _c(lam)
    g = np.zeros(len(pos))
    dg = np.zeros((len(pos), 3))
    _load().orc_check_adjoint(bc, L, -1.0, _p(pos), len(pos), _p(pts), _p(lam), len(pts), _p(g),
                              _p(dg))
    return g, dg


def sphere_images(bc, L, src, Rs):
    """The paper's near set (Sec. II.A): every image of every source whose
    position lies inside the auxiliary sphere |r| < Rs (box centred at 0).
    Images: r + kL (periodic) or (-1)^k o r + kL with charge (-1)^|k| q
    (grounded cube), for all integer k with a box that reaches the sphere.
    Returns (img m x 4, owner m, center m) in the order source-major, then k
    lexicographic."""
    kr = int(math.ceil(Rs / L + 0.5))
    rng = range(-kr, kr + 1)
    ks = [(a, b, c) for a in rng for b in rng for c in rng]
    imgs, owner, center = [], [], []
    for j, (x, y, z, q) in enumerate(np.asarray(src, dtype=np.float64)):
        for k in ks:
            if bc == BC_PERIODIC:
                p = (x + k[0] * L, y + k[1] * L, z + k[2] * L)
                s = 1.0
            else:
                r = [x, y, z]
                p = tuple((r[a] if k[a] % 2 == 0 else -r[a]) + k[a] * L for a in range(3))
                s = (-1.0) ** (abs(k[0]) + abs(k[1]) + abs(k[2]))
            if p[0] * p[0] + p[1] * p[1] + p[2] * p[2] < Rs * Rs:
                imgs.append((p[0], p[1], p[2], s * q))
                owner.append(j)
                center.append(1 if k == (0, 0, 0) else 0)
    return (np.array(imgs).reshape(-1, 4), np.array(owner, dtype=np.int64),
            np.array(center, dtype=np.int32))


def near_explicit(src, tidx, img, owner, center):
    """phi and E at source targets from explicit images, bare self term left out."""
    src, img = _c(src), _c(img)
    tidx = np.ascontiguousarray(tidx, dtype=np.int64)
    owner = np.ascontiguousarray(owner, dtype=np.int64)
    center = np.ascontiguousarray(center, dtype=np.int32)
    phi = np.zeros(len(tidx))
    fld = np.zeros((len(tidx), 3))
    _load().orc_near_explicit(_p(src), tidx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), len(tidx),
                              _p(img), owner.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                              center.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(img),
                              _p(phi), _p(fld))
    return phi, fld


# --------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------
def normalize(x, L, bc):
    """Centre API coordinates [0,L)^3 on the box (Sec. II.A: box centred at 0).

    Periodic: wrap into [-L/2, L/2).  Metallic: must lie in the box.
    Slab (walls at z = 0 and z = L/2): centre x, y only; z stays in [0, L/2].
    """
    x = np.asarray(x, dtype=np.float64)
    if bc == BC_PERIODIC:
        c = x - 0.5 * L
        return c - L * np.floor(c / L + 0.5)
    if bc in (BC_METALLIC, BC_DIELECTRIC):
        c = x - 0.5 * L
        if np.any(np.abs(c) > 0.5 * L):
            raise ValueError("position outside the box")
        return c
    c = x.copy()
    c[:, 0:2] -= 0.5 * L
    c[:, 0:2] -= L * np.floor(c[:, 0:2] / L + 0.5)
    if np.any(c[:, 2] < 0) or np.any(c[:, 2] > 0.5 * L):
        raise ValueError("position outside the slab")
    return c


def double_slab(c, q):
    """Grounded slab -> periodic cube: mirror every charge through z = 0 with
    the opposite sign (mirror reflections plus periodic extension, Sec. I and
    Sec. II).  The doubled cell z in [-L/2, L/2] is a cube of side L."""
    m = c.copy()
    m[:, 2] = -m[:, 2]
    return np.concatenate([c, m]), np.concatenate([q, -q])


_MASK64 = (1 << 64) - 1


def splitmix64_uniform(seed, counter):
    """Uniform double in [0,1) from SplitMix64 (Steele, Lea & Flood, 2014):
    the (counter+1)-th output of the generator started at state `seed`,
    top 53 bits scaled by 2^-53."""
    z = (seed + (counter + 1) * 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    z = z ^ (z >> 31)
    return (z >> 11) * (1.0 / 9007199254740992.0)


def monitoring_points(bc, L, K, seed):
    """Monitoring points (Sec. II.A).

    Periodic: Fibonacci grid on the circumsphere of the box, latitude
    arcsin((2i-1)/K - 1), azimuth 2 pi i w with w = (sqrt5 - 1)/2, i = 1..K;
    twin points x~ = x - kL inside the box with k = floor(x/L + 1/2).
    Metallic: K points on the faces, point i on face i mod 6 (-x,+x,-y,+y,-z,+z),
    tangential coordinates uniform from SplitMix64(seed).
    Dielectric: the Fibonacci grid on the circumsphere without twins (the far
    field itself is fitted there).
    Returns (x, x_twin or None).
    """
    if bc in (BC_PERIODIC, BC_SLAB, BC_DIELECTRIC):
        R0 = math.sqrt(3.0) * L / 2.0
        w = (math.sqrt(5.0) - 1.0) / 2.0
        pts = np.zeros((K, 3))
        for i in range(1, K + 1):
            s = (2.0 * i - 1.0) / K - 1.0          # sin(latitude)
            lat = math.asin(s)
            az = 2.0 * math.pi * i * w
            pts[i - 1] = (R0 * math.cos(lat) * math.cos(az),
                          R0 * math.cos(lat) * math.sin(az),
                          R0 * math.sin(lat))
        if bc == BC_DIELECTRIC:
            return pts, None
        twin = pts - L * np.floor(pts / L + 0.5)
        return pts, twin
    pts = np.zeros((K, 3))
    for i in range(K):
        u = splitmix64_uniform(seed, 2 * i)
        v = splitmix64_uniform(seed, 2 * i + 1)
        f = i % 6
        axis, side = f // 2, (-1.0 if f % 2 == 0 else 1.0)
        t = [a for a in range(3) if a != axis]
        pts[i, axis] = side * 0.5 * L
        pts[i, t[0]] = L * (u - 0.5)
        pts[i, t[1]] = L * (v - 0.5)
    return pts, None


def fibonacci_pair(M):
    """Successive Fibonacci numbers F1 < F2 whose Hannay-Nye point count
    2(F2+1) is nearest to M (ties go to the larger F2)."""
    a, b = 1, 2
    best = None
    while True:
        cnt = 2 * (b + 1)
        d = abs(cnt - M)
        if best is None or d <= best[0]:
            best = (d, a, b)
        if cnt > M and d > best[0]:
            break
        a, b = b, a + b
        if b > 10 ** 7:
            break
    return best[1], best[2]


def integration_points(Rs, M):
    """Fibonacci (Hannay-Nye) quadrature on the sphere of radius Rs (Sec. II.B).

    For j = 0..F2: z_j = -1 + 2j/F2, cos(theta_j) = z_j + sin(pi z_j)/pi,
    phi_j = pi j F1/F2; points (Rs, theta_j, phi_j) and (Rs, theta_j, phi_j + pi)
    each with weight (2 pi Rs^2 / F2)(1 + cos(pi z_j)).
    Returns (points 2(F2+1) x 3, weights, unit normals, F1, F2).
    """
    F1, F2 = fibonacci_pair(M)
    pts, wts = [], []
    for j in range(F2 + 1):
        z = -1.0 + 2.0 * j / F2
        ct = z + math.sin(math.pi * z) / math.pi
        ct = max(-1.0, min(1.0, ct))
        st = math.sqrt(max(0.0, 1.0 - ct * ct))
        ph = math.pi * j * F1 / F2
        wt = 2.0 * math.pi * Rs * Rs / F2 * (1.0 + math.cos(math.pi * z))
        for extra in (0.0, math.pi):
            pts.append((Rs * st * math.cos(ph + extra), Rs * st * math.sin(ph + extra), Rs * ct))
            wts.append(wt)
    pts = np.array(pts)
    return pts, np.array(wts), pts / Rs, F1, F2


# --------------------------------------------------------------------------
# Basis: r^n Y_n^m in real form (Eq. (harmonic); real form per Sec. II.C)
# --------------------------------------------------------------------------
def _legendre_normalized(P, x, s):
    """Fully normalized associated Legendre functions (no Condon-Shortley phase)
    Pbar[n][m] = sqrt((2n+1)/(4 pi) (n-m)!/(n+m)!) P_n^m(x), via the standard
    three-term recurrence in n at fixed m.  x = cos(theta), s = sin(theta)."""
    Pb = {}
    Pb[(0, 0)] = np.full_like(x, 1.0 / math.sqrt(4.0 * math.pi))
    for m in range(1, P + 1):
        Pb[(m, m)] = math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * Pb[(m - 1, m - 1)]
    for m in range(0, P):
        Pb[(m + 1, m)] = math.sqrt(2.0 * m + 3.0) * x * Pb[(m, m)]
    for m in range(0, P + 1):
        for n in range(m + 2, P + 1):
            a = math.sqrt((4.0 * n * n - 1.0) / (n * n - m * m))
            b = math.sqrt(((n - 1.0) ** 2 - m * m) / (4.0 * (n - 1.0) ** 2 - 1.0))
            Pb[(n, m)] = a * (x * Pb[(n - 1, m)] - b * Pb[(n - 2, m)])
    return Pb


def basis(pts, P, R0):
    """B_k(r) = (|r|/R0)^n Y_nm(theta, phi), k = n^2 + n + m, for n <= P.

    Y_n0 = Pbar_n^0; Y_nm = sqrt2 Pbar_n^m cos(m phi) (m > 0);
    Y_n,-m = sqrt2 Pbar_n^m sin(m phi).  Computed from spherical angles.
    """
    pts = np.asarray(pts, dtype=np.float64)
    rho = np.sqrt(np.sum(pts * pts, axis=1))
    safe = np.where(rho > 0, rho, 1.0)
    x = np.where(rho > 0, pts[:, 2] / safe, 1.0)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    az = np.arctan2(pts[:, 1], pts[:, 0])
    Pb = _legendre_normalized(P, x, s)
    B = np.zeros((len(pts), (P + 1) ** 2))
    for n in range(P + 1):
        rn = (rho / R0) ** n
        for m in range(0, n + 1):
            if m == 0:
                B[:, n * n + n] = rn * Pb[(n, 0)]
            else:
                B[:, n * n + n + m] = rn * math.sqrt(2.0) * Pb[(n, m)] * np.cos(m * az)
                B[:, n * n + n - m] = rn * math.sqrt(2.0) * Pb[(n, m)] * np.sin(m * az)
    return B


def basis_gradient(pts, P, R0):
    """grad B_k(r) for the basis of basis(), from spherical angles:
    grad f = df/dr r^ + (1/r) df/dtheta theta^ + (1/(r sin theta)) df/dphi phi^,
    with dPbar_n^m/dtheta from the identity
    (1 - x^2) dPbar_n^m/dx = -n x Pbar_n^m + sqrt((2n+1)(n^2-m^2)/(2n-1)) Pbar_{n-1}^m
    (x = cos theta).
    Points must avoid the origin and the z axis.  Returns (npts, N_b, 3)."""
    pts = np.asarray(pts, dtype=np.float64)
    r = np.sqrt(np.sum(pts * pts, axis=1))
    x = pts[:, 2] / r
    st = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    az = np.arctan2(pts[:, 1], pts[:, 0])
    Pb = _legendre_normalized(P, x, st)
    rhat = np.stack([st * np.cos(az), st * np.sin(az), x], axis=1)
    that = np.stack([x * np.cos(az), x * np.sin(az), -st], axis=1)
    phat = np.stack([-np.sin(az), np.cos(az), np.zeros_like(az)], axis=1)
    G = np.zeros((len(pts), (P + 1) ** 2, 3))
    for n in range(P + 1):
        rn = (r / R0) ** n
        for m in range(0, n + 1):
            prev = Pb[(n - 1, m)] if n - 1 >= m else np.zeros_like(x)
            dPdth = (n * x * Pb[(n, m)] - math.sqrt((2.0 * n + 1.0) * (n * n - m * m) / (2.0 * n - 1.0)) * prev
                     ) / st if n > 0 else np.zeros_like(x)
            variants = [(n * n + n, 1.0, np.ones_like(az), np.zeros_like(az))] if m == 0 else [
                (n * n + n + m, math.sqrt(2.0), np.cos(m * az), -m * np.sin(m * az)),
                (n * n + n - m, math.sqrt(2.0), np.sin(m * az), m * np.cos(m * az))]
            for k, c, T, dT in variants:
                f = rn * c * Pb[(n, m)] * T
                dr_ = n * f / r
                dth = rn * c * dPdth * T / r
                dph = rn * c * Pb[(n, m)] * dT / (r * st)
                G[:, k, :] = dr_[:, None] * rhat + dth[:, None] * that + dph[:, None] * phat
    return G


def far_field_direct(plan, A, pts):
    """Phi_out and E_out = -grad Phi_out at points straight from the fitted
    series sum_k A_k B_k (Eq. (harmonic)), without the surface mapping."""
    phi = basis(pts, plan["p"], plan["R0"]) @ A
    grad = np.einsum("ikc,k->ic", basis_gradient(pts, plan["p"], plan["R0"]), A)
    return phi, -grad


def degree_of(P):
    """n for each basis index k = n^2 + n + m."""
    return np.array([n for n in range(P + 1) for _ in range(2 * n + 1)], dtype=np.float64)


# --------------------------------------------------------------------------
# Least squares by Householder QR (Sec. II.A; factorization in the
# preparation step, Sec. II.C)
# --------------------------------------------------------------------------
def householder_qr(F):
    """Householder QR of a tall matrix.  Returns (V, R): V holds the unit
    reflector vectors (column j acts on rows j..m-1), R is n x n upper."""
    A = np.array(F, dtype=np.float64, copy=True)
    m, n = A.shape
    V = np.zeros((m, n))
    for j in range(n):
        x = A[j:, j].copy()
        nx = np.linalg.norm(x)
        alpha = -nx if x[0] >= 0 else nx
        v = x
        v[0] -= alpha
        nv = np.linalg.norm(v)
        if nv > 0:
            v /= nv
        V[j:, j] = v
        A[j:, j:] -= 2.0 * np.outer(v, v @ A[j:, j:])
    return V, np.triu(A[:n, :])


def qr_apply_qt(V, b):
    """Q^T b by the reflectors in order."""
    b = np.array(b, dtype=np.float64, copy=True)
    for j in range(V.shape[1]):
        v = V[j:, j]
        b[j:] -= 2.0 * v * (v @ b[j:])
    return b


def qr_apply_q(V, y):
    """Q y by the reflectors in reverse order (y has length m)."""
    y = np.array(y, dtype=np.float64, copy=True)
    for j in range(V.shape[1] - 1, -1, -1):
        v = V[j:, j]
        y[j:] -= 2.0 * v * (v @ y[j:])
    return y


def _back_substitute(R, c):
    n = R.shape[0]
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = (c[i] - R[i, i + 1:] @ x[i + 1:]) / R[i, i]
    return x


def _forward_substitute_transposed(R, c):
    """Solve R^T y = c (R upper triangular)."""
    n = R.shape[0]
    y = np.zeros(n)
    for i in range(n):
        y[i] = (c[i] - R[:i, i] @ y[:i]) / R[i, i]
    return y


def qr_solve_ls(V, R, b):
    """argmin_x ||F x - b||_2 from the QR factors."""
    c = qr_apply_qt(V, b)[: R.shape[0]]
    return _back_substitute(R, c)


# --------------------------------------------------------------------------
# Plan (preparation step, Sec. II.C) and update step
# --------------------------------------------------------------------------
def far_shell_count(gamma, tol=1e-13):
    """Shells S of the far dielectric images whose omitted tail is below
    tol * sum|q| / L at every point of the circumsphere: a shell s >= 2 holds
    images with |k| >= s at distance >= (s - 1/2 - sqrt(3)/2) L, and the
    weights of a shell sum to at most 6 |gamma|^s c^2 with
    c = 1 + 2|gamma|/(1 - |gamma|), so the tail beyond S is at most
    6 c^2 |gamma|^(S+1) / ((1 - |gamma|) (S + 1/2 - sqrt(3)/2))."""
    g = abs(gamma)
    if g == 0.0:
        return 1
    c = 1.0 + 2.0 * g / (1.0 - g)
    S = 2
    while 6.0 * c * c * g ** (S + 1) / ((1.0 - g) * (S + 0.5 - math.sqrt(3.0) / 2.0)) > tol:
        S += 1
    return S


def make_plan(L, bc, p, M, K, R, seed=12345, gamma=None, shells=None):
    """Preparation step: monitoring points, fitting matrix and its QR,
    integration points and mapping matrix (Sec. II.C, Table I).  A dielectric
    box (bc = BC_DIELECTRIC) takes the image weight gamma, |gamma| < 1, and
    the number of far image shells (default far_shell_count(gamma))."""
    if bc == BC_DIELECTRIC:
        if gamma is None or not abs(gamma) < 1.0:
            raise ValueError("a dielectric box needs |gamma| < 1")
        if shells is None:
            shells = far_shell_count(gamma)
    R0 = math.sqrt(3.0) * L / 2.0
    X, Xt = monitoring_points(bc, L, K, seed)
    B = basis(X, p, R0)
    if bc in (BC_PERIODIC, BC_SLAB):
        # periodic residual Phi(x) - Phi(x~); the constant column vanishes
        F = (B - basis(Xt, p, R0))[:, 1:]
    else:
        F = B
    V, Rf = householder_qr(F)
    S, w, nrm, F1, F2 = integration_points(R, M)
    Bs = basis(S, p, R0)
    return dict(L=L, bc=bc, p=p, M=M, K=K, Rs=R, R0=R0, seed=seed,
                X=X, Xt=Xt, F=F, V=V, R=Rf, S=S, w=w, nrm=nrm, F1=F1, F2=F2, Bs=Bs,
                deg=degree_of(p), gamma=gamma, shells=shells)


def _rhs(plan, src, images=None):
    """Right-hand side: Phi_in at the monitoring points, differenced with the
    twins for the periodic residual (Sec. II.A).  images: explicit near set
    (sphere mode) instead of the 27-image block."""
    if images is not None:
        b = charges_sum(plan["X"], images[0])[0]
        if plan["Xt"] is not None:
            b = b - charges_sum(plan["Xt"], images[0])[0]
        return b
    if plan["bc"] == BC_DIELECTRIC:
        # the far images themselves: the fit reproduces Phi_far at the points
        # (A = argmin ||F A + b|| with b = -Phi_far)
        return -far_shells(plan["L"], plan["gamma"], src, plan["X"], plan["shells"])
    bc = BC_PERIODIC if plan["bc"] in (BC_PERIODIC, BC_SLAB) else BC_METALLIC
    b = potential_at(bc, plan["L"], src, plan["X"])
    if plan["Xt"] is not None:
        b = b - potential_at(bc, plan["L"], src, plan["Xt"])
    return b


def coefficients_from_rhs(plan, b):
    """A = argmin ||F A + b||  (the residual v = b + F A is minimized)."""
    a = qr_solve_ls(plan["V"], plan["R"], -b)
    if plan["bc"] in (BC_PERIODIC, BC_SLAB):
        return np.concatenate([[0.0], a])
    return a


def surface_images(plan, A):
    """Harmonic surface mapping (Sec. II.B, Eq. (green)): on the sphere R_s,
    surface charge sigma = dPhi_out/dn = (1/R_s) sum n A_nm B_nm and surface
    dipole Phi_out; with the Fibonacci weights w_j:
    Q_j = w_j sigma_j / (4 pi),  p_j = -w_j Phi_out(R_j) n_j / (4 pi)."""
    Phi = plan["Bs"] @ A
    sigma = plan["Bs"] @ (plan["deg"] * A) / plan["Rs"]
    Q = plan["w"] * sigma / (4.0 * math.pi)
    pd = -(plan["w"] * Phi / (4.0 * math.pi))[:, None] * plan["nrm"]
    return np.concatenate([plan["S"], Q[:, None], pd], axis=1)


def surface_images_paper_literal(plan, A, dr):
    """The paper's form (Eq. (cd), Eq. (integrals)): the surface charge on R_s
    plus the dipole replaced by two charge layers on R_s -+ dr/2 with charges
    +- w_j Phi_out(R_j) / (4 pi dr).  Returns 3 M x 4 (X, Y, Z, Q)."""
    Phi = plan["Bs"] @ A
    sigma = plan["Bs"] @ (plan["deg"] * A) / plan["Rs"]
    w = plan["w"]
    n = plan["nrm"]
    Rs = plan["Rs"]
    q0 = w * sigma / (4.0 * math.pi)
    ql = w * Phi / (4.0 * math.pi * dr)
    c0 = np.concatenate([plan["S"], q0[:, None]], axis=1)
    cm = np.concatenate([(Rs - dr / 2) * n, ql[:, None]], axis=1)
    cp = np.concatenate([(Rs + dr / 2) * n, -ql[:, None]], axis=1)
    return np.concatenate([c0, cm, cp])


def _prepare_sources(plan, x, q):
    c = normalize(x, plan["L"], plan["bc"])
    q = np.asarray(q, dtype=np.float64)
    if plan["bc"] == BC_SLAB:
        c, q = double_slab(c, q)
    return np.concatenate([c, q[:, None]], axis=1)


def solve(plan, x, q, targets=None, dipole="exact", dr=None, near="block", far="surface"):
    """Update step (Sec. II.C): images, least squares, surface images, then
    potential, field, energy and forces at the targets (indices of real
    sources; default all).  E = 1/2 sum_targets q_i phi_i, F_i = q_i E_i.
    near: "block" (27 images per source) or "sphere" (every image inside the
    auxiliary sphere, the paper's literal near set).  far: "surface" (the
    harmonic surface mapping) or "direct" (the fitted series evaluated at the
    targets)."""
    x = np.asarray(x, dtype=np.float64)
    n_real = len(x)
    src = _prepare_sources(plan, x, q)
    if targets is None:
        targets = np.arange(n_real)
    targets = np.asarray(targets, dtype=np.int64)
    bc_img = BC_PERIODIC if plan["bc"] in (BC_PERIODIC, BC_SLAB) else BC_METALLIC
    gamma = -1.0
    if plan["bc"] == BC_DIELECTRIC:
        if near != "block":
            raise ValueError("a dielectric box uses the block near set")
        bc_img, gamma = BC_DIELECTRIC, plan["gamma"]
    images = sphere_images(bc_img, plan["L"], src, plan["Rs"]) if near == "sphere" else None
    b = _rhs(plan, src, images)
    A = coefficients_from_rhs(plan, b)
    if images is not None:
        pn, en = near_explicit(src, targets, *images)
    else:
        pn, en = near_sum(bc_img, plan["L"], src, targets, gamma)
    tpos = src[targets, :3]
    if far == "direct":
        surf = None
        po, eo = far_field_direct(plan, A, tpos)
    elif dipole == "exact":
        surf = surface_images(plan, A)
        po, eo = surface_sum(tpos, surf)
    else:
        surf = surface_images_paper_literal(plan, A, dr)
        po, eo = charges_sum(tpos, surf)
    phi = pn + po
    fld = en + eo
    qt = src[targets, 3]
    return dict(b=b, A=A, surf=surf, phi_near=pn, field_near=en, phi_out=po, field_out=eo,
                phi=phi, field=fld, forces=qt[:, None] * fld, energy=0.5 * np.sum(qt * phi))


def _mapping_transpose(plan, wpot, wvec):
    """T^T applied to the surface responses, T being the linear map from the
    coefficients A to (Q_j, p_j) of surface_images()."""
    Bs, w, n, deg, Rs = plan["Bs"], plan["w"], plan["nrm"], plan["deg"], plan["Rs"]
    yq = w * wpot / (4.0 * math.pi)                          # dQ_j coefficients
    yp = -(w / (4.0 * math.pi)) * np.sum(n * wvec, axis=1)   # dp_j . wvec_j
    return deg / Rs * (Bs.T @ yq) + Bs.T @ yp


def adjoint(plan, x, q, targets=None):
    """Exact gradient of the computed energy E(x, q) of solve().

    E = 1/2 sum_{i in T} q_i (phi_near_i + phi_out_i), T = the real charges.
    E_out = 1/2 u_T^T T A with u_T = sum_{i in T} q_i [1/|d|, d/|d|^3] at the
    surface points (d = r_i - R_j), T the linear map A -> (Q_j, p_j) and
    A = -R^{-1} Q^T b.  With lam = Q R^{-T} T^T u_T (so E_out = -1/2 lam^T b),
    and G(r) = sum_k lam_k g_k(r), g_k(r) the contribution of a unit charge at
    r to b_k:
      dE/dq_j = phi_near_j + 1/2 phi_out_j - 1/2 G(r_j)
      dE/dr_j = q_j grad phi_near_j + 1/2 q_j grad phi_out_j - 1/2 q_j grad G(r_j)
    For the slab every real charge also moves its mirror (x, y, -z) of charge
    -q, so G and grad G enter through that map as well.
    Returns (E, dE/dx, dE/dq); with `targets` (indices of real charges) the
    derivatives are evaluated at those charges only and E is the partial
    energy 1/2 sum over the targets of q_i phi_i.
    """
    if plan["bc"] == BC_DIELECTRIC:
        raise ValueError("no adjoint for the dielectric box")
    x = np.asarray(x, dtype=np.float64)
    n_real = len(x)
    src = _prepare_sources(plan, x, q)
    T = np.arange(n_real)
    sel = T if targets is None else np.asarray(targets, dtype=np.int64)
    bc_img = BC_PERIODIC if plan["bc"] in (BC_PERIODIC, BC_SLAB) else BC_METALLIC
    b = _rhs(plan, src)
    A = coefficients_from_rhs(plan, b)
    surf = surface_images(plan, A)
    if targets is None:
        pn, en = near_sum(bc_img, plan["L"], src, T)
        po, eo = surface_sum(src[T, :3], surf)
        energy = 0.5 * np.sum(src[T, 3] * (pn + po))
    else:
        pn, en = near_sum(bc_img, plan["L"], src, sel)
        po, eo = surface_sum(src[sel, :3], surf)
        energy = 0.5 * np.sum(src[sel, 3] * (pn + po))
    # response of the real charges at the surface points
    upot, ufld = charges_sum(plan["S"], src[T])    # ufld = sum q (R_j - r_i)/|.|^3
    uvec = -ufld                                   # sum q (r_i - R_j)/|.|^3
    tw = _mapping_transpose(plan, upot, uvec)
    periodic = plan["bc"] in (BC_PERIODIC, BC_SLAB)
    if periodic:
        tw = tw[1:]
    y = _forward_substitute_transposed(plan["R"], tw)
    ypad = np.zeros(plan["V"].shape[0])
    ypad[: len(y)] = y
    lam = qr_apply_q(plan["V"], ypad)
    if periodic:
        pts = np.concatenate([plan["X"], plan["Xt"]])
        lw = np.concatenate([lam, -lam])
    else:
        pts, lw = plan["X"], lam
    if plan["bc"] == BC_SLAB:
        gpos = np.concatenate([src[sel, :3], src[sel + n_real, :3]])
    else:
        gpos = src[sel, :3]
    g, dg = check_adjoint(bc_img, plan["L"], gpos, pts, lw)
    qT = src[sel, 3]
    ns = len(sel)
    if plan["bc"] == BC_SLAB:
        mir = np.array([1.0, 1.0, -1.0])
        G = g[:ns] - g[ns:]
        dG = dg[:ns] - dg[ns:] * mir
    else:
        G, dG = g, dg
    dq = pn + 0.5 * po - 0.5 * G
    # grad phi = -E (field)
    dx = -qT[:, None] * en - 0.5 * qT[:, None] * eo - 0.5 * qT[:, None] * dG
    return energy, dx, dq
