"""Benchmark of the HSMA hot path on one MI355X.

One step = one full update step (Sec. II.C of the paper): right-hand side at
the monitoring points, least squares, surface mapping, near-field pair sum and
surface sum at every particle, energy and forces.  Default workload: periodic
cube, 1e6 uniform random +-1 charges, p=20, K=4000, M=4000 (M_eff=3196),
R=2.7L, near and right-hand-side pair sums in FP32 with two-sum compensated
accumulation (double precision elsewhere).  Inputs are synthetic and resident
in HBM before the timed region.

Prints one JSON line.  `value` = pair interactions per second of the whole
step (near + right-hand side + surface).  `roofline` is for the near-field
pair kernel, timed with HIP events on its own stream inside the library.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak
FP64_PEAK_TFLOPS = 78.6      # MI355X published FP64 vector peak
NEAR_FLOPS_PER_PAIR = 20     # potential + field, rsqrt counted as one flop


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="periodic1m")
    ap.add_argument("--precision", default=None, help="fp64 or fp32 (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-targets", type=int, default=256)
    return ap.parse_args()


def cpu_baseline(x, q, cfg, n_targets):
    """The oracle's near-field sum (plain FP64 C, OpenMP) on a bounded sample
    of the same workload: n_targets particles against all 27N images."""
    import numpy as np

    import oracle
    from oracle import hsma as oh
    oh.build()
    c = oh.normalize(x, cfg["L"], cfg["bc"])
    src = np.concatenate([c, q[:, None]], axis=1)
    idx = np.random.default_rng(0).choice(len(q), n_targets, replace=False)
    img = oracle.BC_METALLIC if cfg["bc"] == 1 else oracle.BC_PERIODIC
    t0 = time.perf_counter()
    oracle.near_sum(img, cfg["L"], src, idx)
    dt = time.perf_counter() - t0
    pairs = n_targets * 27.0 * len(q)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": pairs / dt, "unit": "pair interactions/s", "cores": cores, "kind": "oracle",
            "sample": "near-field sum at %d of %d particles against all 27N images (%.3g pairs, %.1f s)"
                      % (n_targets, len(q), pairs, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1806_04801_amd import hsma, workloads

    cfg = dict(workloads.CONFIGS[args.workload])
    prec_name = args.precision or ("fp32" if args.workload in ("periodic1m", "slab200k") else "fp64")
    prec = hsma.FP32_COMP if prec_name == "fp32" else hsma.FP64
    x, q = workloads.make_inputs(args.workload)
    n = len(q)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    plan = hsma.Plan(cfg["L"], cfg["bc"], cfg["p"], cfg["M"], cfg["K"], cfg["R"], precision=prec)
    info = plan.info
    xd = torch.tensor(x, dtype=torch.float64, device=dev)
    qd = torch.tensor(q, dtype=torch.float64, device=dev)
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    F = torch.empty((n, 3), dtype=torch.float64, device=dev)
    plan.workspace(n, dev)
    for _ in range(args.warmup):
        plan.energy_forces(xd, qd, phi, F)
    torch.cuda.synchronize()
    hsma.timing_read()
    hsma.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    energies = []
    for i in range(args.steps):
        e, _, _ = plan.energy_forces(xd, qd, phi, F)
        energies.append(e)
        print("step %d done: energy %.10e" % (i, e), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    hsma.timing_enable(False)
    kt = hsma.timing_read()

    ns = 2 * n if cfg["bc"] == 2 else n
    near_pairs = n * 27.0 * ns - n
    rhs_pairs = info["n_check"] * 27.0 * ns
    surf_pairs = float(n) * info["M_eff"]
    pairs_step = near_pairs + rhs_pairs + surf_pairs
    ms_step = 1e3 * dt / args.steps
    near_ms, near_launches = kt["near"]
    near_avg_s = near_ms / max(near_launches, 1) / 1e3
    achieved = NEAR_FLOPS_PER_PAIR * near_pairs / near_avg_s / 1e12
    peak = FP32_PEAK_TFLOPS if prec == hsma.FP32_COMP else FP64_PEAK_TFLOPS
    rec = {
        "metric": "pair interactions/s",
        "value": pairs_step / (dt / args.steps),
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == hsma.FP32_COMP else "f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "desc": cfg["desc"],
            "N": n, "bc": cfg["bc"], "p": cfg["p"], "K": cfg["K"], "M_eff": info["M_eff"],
            "R": cfg["R"], "precision": "fp32 pair sums + two-sum accumulation" if prec else "fp64",
            "pairs_per_step": {"near": near_pairs, "rhs": rhs_pairs, "surface": surf_pairs},
            "near_pairs_per_s": near_pairs / near_avg_s,
            "kernel_ms_avg": {k: (v[0] / max(v[1], 1)) for k, v in kt.items()},
            "energy": energies[-1],
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": None,
        },
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(x, q, cfg, args.cpu_targets)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
