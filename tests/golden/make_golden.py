"""Write oracle reference values at full workload sizes (sampled outputs).

Calls only the oracle (double precision CPU) on the seeded synthetic inputs of
paper_1806_04801_amd.workloads.  For each workload: the right-hand side b and
the coefficients A in full (they need every source), and potential, forces
(and for the slab the adjoint) at a seeded sample of particles.  The GPU tests
regenerate the same inputs and compare.  Run from the repository root:
    python tests/golden/make_golden.py periodic1m slab200k
Takes minutes (periodic1m: 2.2e11 pair evaluations in the right-hand side).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1806_04801_amd import workloads as W  # noqa: E402

N_SAMPLE = 256


def sample_indices(n, seed=2024):
    return np.sort(np.random.default_rng(seed).choice(n, N_SAMPLE, replace=False))


def make(name):
    c = W.CONFIGS[name]
    x, q = W.make_inputs(name)
    t0 = time.time()
    plan = oracle.make_plan(c["L"], c["bc"], c["p"], c["M"], c["K"], c["R"])
    idx = sample_indices(len(q))
    r = oracle.solve(plan, x, q, targets=idx)
    out = {
        "workload": name, "desc": c["desc"], "n": int(len(q)), "sample_seed": 2024,
        "idx": idx.tolist(), "b": r["b"].tolist(), "A": r["A"].tolist(),
        "phi": r["phi"].tolist(), "forces": r["forces"].tolist(),
        "phi_near": r["phi_near"].tolist(), "phi_out": r["phi_out"].tolist(),
        "partial_energy": float(r["energy"]),
    }
    if name == "slab200k":
        E, dx, dq = oracle.adjoint(plan, x, q, targets=idx)
        out["dEdx"] = dx.tolist()
        out["dEdq"] = dq.tolist()
    out["oracle_seconds"] = time.time() - t0
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), name + ".json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, "%.0f s" % out["oracle_seconds"])


if __name__ == "__main__":
    for n in sys.argv[1:]:
        make(n)
