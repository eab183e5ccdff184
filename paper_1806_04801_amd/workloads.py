"""Seeded synthetic inputs (positions and charges only; no HSMA arithmetic).

These stand in for the paper's synthetic systems (Sec. III): rock-salt
lattices, charges in a grounded cavity, random-sign charges on a lattice and
uniform random neutral systems.  numpy's PCG64 with an explicit seed makes
every input reproducible on any host.  Coordinates are API coordinates in
[0, L)^3 (slab: z in [0, L/2]).
"""
import math

import numpy as np


def nacl(n_side=2, L=1.0):
    """Rock-salt sub-lattice: n_side^3 ions at the cell centres of an
    n_side^3 grid, q = (-1)^(i+j+k).  Returns (x, q, nearest-neighbour a)."""
    a = L / n_side
    idx = np.array([(i, j, k) for i in range(n_side) for j in range(n_side) for k in range(n_side)],
                   dtype=np.float64)
    x = (idx + 0.5) * a
    q = (-1.0) ** idx.sum(axis=1)
    return x, q, a


def uniform_neutral(n, L=1.0, seed=0):
    """n uniform random positions in (0, L)^3 with n/2 charges +1 and n/2
    charges -1 in random order (n even)."""
    if n % 2:
        raise ValueError("n must be even for a neutral +-1 system")
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3)) * L
    q = np.concatenate([np.ones(n // 2), -np.ones(n - n // 2)])
    rng.shuffle(q)
    return x, q


def random_sign_lattice(n_side, L=1.0, seed=0):
    """Charges on a uniform lattice, unit charge of random sign, neutral."""
    n = n_side ** 3
    rng = np.random.default_rng(seed)
    g = (np.arange(n_side) + 0.5) * (L / n_side)
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    q = np.concatenate([np.ones(n // 2), -np.ones(n - n // 2)])
    if n % 2:
        q[-1] = 0.0
    rng.shuffle(q)
    return x, q


def slab_charges(n, L=1.0, seed=5):
    """Slab L x L x L/2, x, y uniform in (0, L), z uniform in (0, L/2);
    charges fixed at n/5 of +2, n/5 of +1 and 3n/5 of -1 (neutral), randomly
    permuted (n divisible by 5)."""
    if n % 5:
        raise ValueError("n must be divisible by 5")
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3)) * L
    x[:, 2] *= 0.5
    q = np.concatenate([np.full(n // 5, 2.0), np.full(n // 5, 1.0), np.full(3 * n // 5, -1.0)])
    rng.shuffle(q)
    return x, q


def serving_trace(n_requests=4096, seed=4, rate=1.0, n_min=1e3, n_max=1e5,
                  degrees=(12, 16, 20)):
    """Request stream: arrival times of a Poisson process of the given rate,
    N = even(round(10^U[log10 n_min, log10 n_max])), boundary condition
    periodic or metallic with probability 1/2, degree uniform over `degrees`.
    Returns a list of dicts with keys t, n, bc (0 periodic, 1 metallic), p, seed."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    logn = rng.uniform(math.log10(n_min), math.log10(n_max), n_requests)
    n = 2 * np.round(10.0 ** logn / 2.0).astype(np.int64)
    bc = rng.integers(0, 2, n_requests)
    p = rng.choice(np.array(degrees), n_requests)
    seeds = rng.integers(0, 2 ** 31 - 1, n_requests)
    return [dict(t=float(t[i]), n=int(n[i]), bc=int(bc[i]), p=int(p[i]), seed=int(seeds[i]))
            for i in range(n_requests)]


# Configurations of the hot path (name -> parameters).  The inputs are drawn by
# the functions above; 'seed' selects the draw.
CONFIGS = {
    "nacl8": dict(L=1.0, bc=0, p=8, M=1000, K=600, R=2.7, n=8, seed=None,
                  desc="NaCl 2x2x2 sub-lattice, periodic, p=8, K=600, M=1000, FP64"),
    "metallic10k": dict(L=1.0, bc=1, p=16, M=2500, K=2000, R=2.7, n=10_000, seed=2,
                        desc="grounded cube, 10k uniform +-1 charges, p=16, K=2000, M=2500, FP64"),
    "periodic1m": dict(L=1.0, bc=0, p=20, M=4000, K=4000, R=2.7, n=1_000_000, seed=3,
                       desc="periodic cube, 1e6 uniform +-1 charges, p=20, K=4000, M=4000, FP32-comp"),
    # The paper's timing system (Sec. III): unit charges of random sign on a
    # uniform lattice, periodic, alpha = 1.3 (R_s = 1.3 sqrt(3)/2 L), P = 25,
    # N_m = 2 P^2 monitoring points, N_o = 5928 surface images over three
    # spheres = 2 x 988 points per sphere.  46^3 = 97,336 sites.
    "paper100k": dict(L=1.0, bc=0, p=25, M=1976, K=1250, R=1.3 * math.sqrt(3.0) / 2.0, n=46 ** 3,
                      seed=7, desc="paper timing system: 46^3 random-sign lattice, periodic, alpha=1.3, "
                                   "P=25, N_m=2P^2=1250, N_o=5928 (1976 per sphere)"),
    "slab200k": dict(L=1.0, bc=2, p=16, M=2500, K=3000, R=2.7, n=200_000, seed=5,
                     desc="grounded slab 1x1x0.5, 2e5 charges {+2,+1,-1}, p=16, K=3000, M=2500, FP32"),
}


def make_inputs(name, n=None, seed=None):
    """Inputs (x, q) of a named configuration, optionally at another size."""
    c = CONFIGS[name]
    n = c["n"] if n is None else n
    seed = c["seed"] if seed is None else seed
    if name == "nacl8":
        side = round(n ** (1.0 / 3.0))
        x, q, _ = nacl(side, c["L"])
        return x, q
    if name == "slab200k":
        return slab_charges(n, c["L"], seed)
    if name == "paper100k":
        side = round(n ** (1.0 / 3.0))
        return random_sign_lattice(side, c["L"], seed)
    return uniform_neutral(n, c["L"], seed)
