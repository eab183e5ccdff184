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
# Pair-once near kernel: one evaluation (20 flops) serves both directions and
# adds 8 (4 products and 4 sums for the reverse terms), 28 per unordered pair,
# i.e. 14 per ordered pair.  Its diagonal blocks are evaluated per ordered pair
# (20 flops each) and are under 1% of the pairs; they are counted at 14 too,
# which understates the work.
NEAR_FLOPS_PER_PAIR_ONCE = 14


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="periodic1m")
    ap.add_argument("--precision", default=None, help="fp64 or fp32 (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--host-entry", type=int, default=0,
                    help="also time this many calls of the host-array entry point (PCIe copies and "
                         "its own device allocation included); reported in config, never as value")
    ap.add_argument("--cpu-targets", type=int, default=2048,
                    help="particles in the oracle sample (about 17 s on 16 host threads at 1e6)")
    ap.add_argument("--requests", type=int, default=1024, help="serving: trace length")
    ap.add_argument("--refine", type=float, default=3e-3,
                    help="serving: recompute in double precision the requests whose FP32 energy "
                         "is below this fraction of 1/2 sum |q phi| (0: never)")
    ap.add_argument("--grad", action="store_true", help="time energy + exact gradient (adjoint)")
    ap.add_argument("--near", default="block", choices=["block", "sphere"],
                    help="near set: 27-image block or every image inside the auxiliary sphere")
    ap.add_argument("--dipole", default="exact", choices=["exact", "layers"],
                    help="surface dipoles exact, or the paper's two charge layers (dr = 1e-5 R_s)")
    ap.add_argument("--far", default="surface", choices=["surface", "direct"],
                    help="far field through the surface mapping, or the series evaluated directly")
    ap.add_argument("--paper-time", action="store_true",
                    help="report seconds per update step against the paper's GPU timing")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy a 1 GiB device buffer (reference kernel for HBM counters)")
    return ap.parse_args()


def sphere_image_count(x, cfg):
    """Number of images inside the auxiliary sphere (the sources of the
    sphere near set), counted from the same geometry the library uses."""
    import math

    import numpy as np
    L, R, bc = cfg["L"], cfg["R"], cfg["bc"]
    c = x - 0.5 * L
    if bc == 0:
        c -= L * np.floor(c / L + 0.5)
    elif bc == 2:
        c[:, :2] -= L * np.floor(c[:, :2] / L + 0.5)
        c[:, 2] = x[:, 2]
        c = np.concatenate([c, c * np.array([1.0, 1.0, -1.0])])
    kr = int(math.ceil(R / L + 0.5))
    n_img = 0
    for a in range(-kr, kr + 1):
        for b in range(-kr, kr + 1):
            for k in range(-kr, kr + 1):
                kk = np.array([a, b, k])
                if bc == 1:
                    p = np.where(kk % 2 == 0, c, -c) + kk * L
                else:
                    p = c + kk * L
                n_img += int(np.sum(np.sum(p * p, axis=1) < R * R))
    return n_img


NEAR_SOURCES = {"tiles": ("pairs.hip", "pair_math.h"), "pair-once": ("sym.hip", "pair_math.h")}


def kernel_source_hash(kind="tiles"):
    """Hash of the code (line comments and blank lines removed) of the sources
    that define the near kernel of that kind."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in NEAR_SOURCES[kind]:
        text = open(os.path.join(ROOT, "paper_1806_04801_amd", "csrc", name)).read()
        for line in text.splitlines():
            code = re.sub(r"//.*", "", line).rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def profile_name(workload, precision_tag, kind="tiles"):
    stem = "near_pair_once" if kind == "pair-once" else "near"
    return "%s_%s_%s" % (stem, precision_tag, workload)


def profiled_traffic(workload, precision_tag, kind="tiles"):
    """HBM bytes of one near-field sum (all launches of its kernel) from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    source."""
    path = os.path.join(ROOT, "profiles", profile_name(workload, precision_tag, kind) + "_pmc.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().split()[0]
    if fields.get("kernel_source_sha256_16") != kernel_source_hash(kind):
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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


def serving(args):
    """Serving stream: requests with N log-uniform in [1e3, 1e5] (even), periodic or
    grounded cube with probability 1/2, p in {12, 16, 20}, K = M = 10 p^2,
    R = 2.7L.  Closed loop (all arrivals at t = 0) gives solves/s; open loop
    (Poisson arrivals at 0.8 of each path's closed-loop rate) gives p50/p99
    latency.  Batched FP32-compensated server vs one FP64 solve per request."""
    import numpy as np
    import torch

    from paper_1806_04801_amd import hsma, workloads

    torch.cuda.set_device(0)
    trace = workloads.serving_trace(args.requests, seed=4)
    plans = {}
    for bc in (0, 1):
        for p in (12, 16, 20):
            plans[(bc, p)] = hsma.Plan(1.0, bc, p, 10 * p * p, 10 * p * p, 2.7)
    pl, xs, qs = [], [], []
    for r in trace:
        x, q = workloads.uniform_neutral(r["n"], 1.0, seed=r["seed"])
        pl.append(plans[(r["bc"], r["p"])])
        xs.append(x)
        qs.append(q)
    n = len(trace)
    pairs = 0.0
    for r in trace:
        nchk = (2 if r["bc"] == 0 else 1) * 10 * r["p"] ** 2
        pairs += 27.0 * r["n"] * r["n"] + 27.0 * nchk * r["n"]
    srv = hsma.Server(memory_bytes=16 << 30, max_active=64, precision=hsma.FP32_COMP,
                      refine_below=args.refine)
    zero = np.zeros(n)
    # warm-up of both paths on a few requests
    srv.run_trace(zero[:8], pl[:8], xs[:8], qs[:8])
    hsma.run_trace_sequential(zero[:8], pl[:8], xs[:8], qs[:8])
    print("serving: closed loop, batched fp32", file=sys.stderr, flush=True)
    refined0 = srv.stats()["refined"]
    e32, lat32c, wall32 = srv.run_trace(zero, pl, xs, qs)
    refined = srv.stats()["refined"] - refined0
    print("serving: closed loop, sequential fp64 (%.1f s batched)" % wall32, file=sys.stderr, flush=True)
    e64, lat64c, wall64 = hsma.run_trace_sequential(zero, pl, xs, qs)
    mu32, mu64 = n / wall32, n / wall64
    rng = np.random.default_rng(44)
    gaps = rng.exponential(1.0, n)
    print("serving: open loop (%.1f s sequential)" % wall64, file=sys.stderr, flush=True)
    arr32 = np.cumsum(gaps) / (0.8 * mu32)
    _, lat32, _ = srv.run_trace(arr32, pl, xs, qs)
    print("serving: open loop, batched at 0.8 of its capacity done", file=sys.stderr, flush=True)
    arr64 = np.cumsum(gaps) / (0.8 * mu64)
    _, lat64, _ = hsma.run_trace_sequential(arr64, pl, xs, qs)
    print("serving: open loop, sequential at 0.8 of its capacity done", file=sys.stderr, flush=True)
    _, lat32s, _ = srv.run_trace(arr64, pl, xs, qs)      # batched at the sequential path's load
    print("serving: open loop, batched at the sequential load done", file=sys.stderr, flush=True)
    rel = np.abs(e32 - e64) / np.abs(e64)
    pct = lambda a, q_: float(np.percentile(a, q_)) * 1e3
    rec = {
        "metric": "solves/s", "value": mu32, "unit": "solves/s", "n_gpus": 1,
        "steps": n, "warmup": 8, "ms_per_step": 1e3 / mu32, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": "serving", "requests": n,
            "desc": "N log-uniform [1e3,1e5] even, bc periodic/grounded 1/2, p in {12,16,20}, "
                    "K=M=10p^2, R=2.7L; FP32-comp batched server (ill-conditioned energies "
                    "refined in FP64) vs FP64 per-request",
            "pair_interactions": pairs,
            "batched_fp32": {"solves_per_s": mu32, "pairs_per_s": pairs / wall32,
                             "p50_ms_at_0.8mu": pct(lat32, 50), "p99_ms_at_0.8mu": pct(lat32, 99),
                             "p50_ms_at_0.8mu64": pct(lat32s, 50), "p99_ms_at_0.8mu64": pct(lat32s, 99)},
            "sequential_fp64": {"solves_per_s": mu64, "pairs_per_s": pairs / wall64,
                                "p50_ms_at_0.8mu": pct(lat64, 50), "p99_ms_at_0.8mu": pct(lat64, 99)},
            "speedup_solves_per_s": mu32 / mu64,
            "refine_below": args.refine,
            "refined_in_fp64": {"requests": int(refined), "fraction": refined / n},
            "rel_energy_err_fp32_vs_fp64": {"p50": float(np.median(rel)),
                                            "p99": float(np.percentile(rel, 99)),
                                            "max": float(rel.max()),
                                            "frac_le_1e-5": float(np.mean(rel <= 1e-5))},
        },
    }
    print(json.dumps(rec))


def adjoint_bench(args, cfg, x, q, prec):
    """Energy plus exact gradient (forward + adjoint kernels) per step."""
    import torch

    from paper_1806_04801_amd import hsma
    dev = torch.device("cuda:0")
    plan = hsma.Plan(cfg["L"], cfg["bc"], cfg["p"], cfg["M"], cfg["K"], cfg["R"], precision=prec)
    xd = torch.tensor(x, device=dev)
    qd = torch.tensor(q, device=dev)
    for _ in range(args.warmup):
        plan.energy_grad(xd, qd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        e, dx, dq = plan.energy_grad(xd, qd)
        print("grad step %d done: energy %.10e" % (i, e), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    n = len(q)
    ns = 2 * n if cfg["bc"] == 2 else n
    info = plan.info
    pairs = n * 27.0 * ns + info["n_check"] * 27.0 * ns * 2 + 2.0 * n * info["M_eff"]
    rec = {
        "metric": "pair interactions/s", "value": pairs / dt, "unit": "pair interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == hsma.FP32_COMP else "f64", "data": "synthetic",
        "config": {"workload": args.workload + "+grad", "desc": cfg["desc"] + "; energy + dE/dx + dE/dq",
                   "N": n, "pairs_per_step": pairs, "energy": e},
    }
    print(json.dumps(rec))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("copied %d bytes device to device" % (src.numel() * 8), file=sys.stderr, flush=True)
        del src, dst
    if args.workload == "serving":
        return serving(args)
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
    if args.grad:
        return adjoint_bench(args, cfg, x, q, prec)
    near_mode = hsma.NEAR_SPHERE if args.near == "sphere" else hsma.NEAR_BLOCK
    plan = hsma.Plan(cfg["L"], cfg["bc"], cfg["p"], cfg["M"], cfg["K"], cfg["R"], precision=prec,
                     near_mode=near_mode,
                     dipole_mode=hsma.DIPOLE_LAYERS if args.dipole == "layers" else hsma.DIPOLE_EXACT,
                     far_mode=hsma.FAR_DIRECT if args.far == "direct" else hsma.FAR_SURFACE)
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

    host_entry = None
    if args.host_entry > 0:
        import numpy as np
        xh = np.ascontiguousarray(x, dtype=np.float64)
        qh = np.ascontiguousarray(q, dtype=np.float64)
        plan.energy_forces_host(xh, qh)
        t1 = time.perf_counter()
        for i in range(args.host_entry):
            plan.energy_forces_host(xh, qh)
            print("host-entry call %d done" % i, file=sys.stderr, flush=True)
        host_entry = {"calls": args.host_entry,
                      "ms_per_call": 1e3 * (time.perf_counter() - t1) / args.host_entry}

    ns = 2 * n if cfg["bc"] == 2 else n
    if near_mode == hsma.NEAR_SPHERE:
        n_img = sphere_image_count(x, cfg)
        near_pairs = float(n) * n_img - n
        rhs_pairs = info["n_check"] * float(n_img)
    else:
        near_pairs = n * 27.0 * ns - n
        rhs_pairs = info["n_check"] * 27.0 * ns
    surf_pairs = float(n) * info["M_eff"] * (3 if args.dipole == "layers" else 1)
    if args.far == "direct":
        surf_pairs = 0.0   # no surface images: the series is evaluated per particle
    pairs_step = near_pairs + rhs_pairs + surf_pairs
    ms_step = 1e3 * dt / args.steps
    near_ms, near_launches = kt["near"]
    near_avg_s = near_ms / max(near_launches, 1) / 1e3
    sched = plan.near_schedule(n)
    flops_pair = NEAR_FLOPS_PER_PAIR_ONCE if sched["kind"] == 1 else NEAR_FLOPS_PER_PAIR
    achieved = flops_pair * near_pairs / near_avg_s / 1e12
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
            "near_set": args.near,
            "surface_dipole": args.dipole,
            "far_field": args.far,
            "desc": cfg["desc"],
            "N": n, "bc": cfg["bc"], "p": cfg["p"], "K": cfg["K"], "M_eff": info["M_eff"],
            "R": cfg["R"], "precision": "fp32 pair sums + two-sum accumulation" if prec else "fp64",
            "pairs_per_step": {"near": near_pairs, "rhs": rhs_pairs, "surface": surf_pairs},
            "near_pairs_per_s": near_pairs / near_avg_s,
            "near_kernel": ("pair-once" if sched["kind"] == 1 else "tiles"),
            "near_schedule": sched,
            "near_flops_per_pair": flops_pair,
            "kernel_ms_avg": {k: (v[0] / max(v[1], 1)) for k, v in kt.items()},
            "energy": energies[-1],
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": profiled_traffic(args.workload, "f32" if prec == hsma.FP32_COMP else "f64",
                                        "pair-once" if sched["kind"] == 1 else "tiles"),
        },
    }
    if host_entry is not None:
        host_entry["pairs_per_s"] = pairs_step / (host_entry["ms_per_call"] / 1e3)
        rec["config"]["host_entry"] = host_entry
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(x, q, cfg, args.cpu_targets)
    if args.paper_time:
        # The paper reports an HSMA step under 1 s at N = 100k on two Tesla P100
        # (Sec. III, Fig. 5); vs_baseline = this step's time / 1 s (an upper bound).
        rec = {"metric": "seconds per HSMA update step", "value": dt / args.steps, "unit": "s",
               "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": ms_step, "higher_is_better": False, "scaling": "strong",
               "vs_baseline": (dt / args.steps) / 1.0, "dtype": rec["dtype"], "data": "synthetic",
               "config": rec["config"], "roofline": rec["roofline"]}
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
