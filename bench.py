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
pair kernel, timed with HIP events on its own stream inside the library:
20 flops per pair-image the kernel evaluates.  `cpu_baseline` is the oracle
timed stage by stage on bounded samples; `serving` (default workload) is the
serving stream: solves/s of the batched server and of one solve per request
in both precisions, and p50/p99 latency.
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
# Algorithmic work per evaluated near pair-image (potential + field, rsqrt
# counted as one flop).  roofline.achieved charges it per pair-image the
# kernel evaluates: every ordered pair for the per-target tiles, every
# unordered pair once for the pair-once kernel (whose evaluation serves both
# directions), plus the ordered pairs inside its diagonal blocks.
NEAR_FLOPS_PER_PAIR = 20
# The pair-once kernel's own count of one evaluation with both directions:
# the 20 above plus 4 products and 4 sums for the reverse terms (reported
# beside the roofline, not as it).
NEAR_FLOPS_PER_UNORDERED_PAIR_BOTH_DIRECTIONS = 28


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
    ap.add_argument("--cpu-targets", type=int, default=1024,
                    help="particles in the oracle's near-sum sample (about 8 s on 16 host threads "
                         "at 1e6)")
    ap.add_argument("--requests", type=int, default=1024, help="serving: trace length")
    ap.add_argument("--refine", type=float, default=3e-3,
                    help="serving: recompute in double precision the requests whose FP32 energy "
                         "is below this fraction of 1/2 sum |q phi| (0: never)")
    ap.add_argument("--grad", action="store_true", help="time energy + exact gradient (adjoint)")
    ap.add_argument("--near", default="block", choices=["block", "sphere", "tree"],
                    help="near set: 27-image block (direct), every image inside the auxiliary "
                         "sphere, or the block summed by the tree code (FP64)")
    ap.add_argument("--tree-order", type=int, default=0, help="multipole order of --near tree")
    ap.add_argument("--dipole", default="exact", choices=["exact", "layers"],
                    help="surface dipoles exact, or the paper's two charge layers (dr = 1e-5 R_s)")
    ap.add_argument("--far", default="surface", choices=["surface", "direct"],
                    help="far field through the surface mapping, or the series evaluated directly")
    ap.add_argument("--serving-requests", type=int, default=512,
                    help="default workload: also run this many requests of the serving stream "
                         "(object 'serving' of the line; 0 skips it)")
    ap.add_argument("--n", type=int, default=0,
                    help="particles (default: the workload's own count); the same seeded recipe at "
                         "another size")
    ap.add_argument("--fmm-steps", type=int, default=3,
                    help="default workload: also time this many update steps with the fast multipole "
                         "near sum and right-hand side (object 'fmm' of the line; 0 skips it)")
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


def profiled_field(workload, precision_tag, kind, field):
    """A derived figure of the committed rocprofv3 counter summary of the near
    sum, if the counters were taken on the current kernel source."""
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
        return float(fields[field])
    except (KeyError, ValueError):
        return None


def profiled_traffic(workload, precision_tag, kind="tiles"):
    """HBM bytes of one near-field sum (all launches of its kernel) from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    source."""
    return profiled_field(workload, precision_tag, kind, "hbm_bytes_per_launch")


def near_evaluated_pairs(n, cfg, sched):
    """Pair-images the near kernel evaluates in one sum.  Tiles: every
    (target, source image) pair, self included.  Pair-once: each unordered
    pair of particles in different blocks once, plus every ordered pair
    (self included) inside the diagonal blocks; a slab pair carries two image
    blocks (the partner's and its mirror's)."""
    imgs = 54.0 if cfg["bc"] == 2 else 27.0
    if sched["kind"] != 1:
        ns = 2.0 * n if cfg["bc"] == 2 else float(n)
        return 27.0 * n * ns
    B, nb = sched["block"], sched["blocks"]
    sizes = [B] * (nb - 1) + [n - (nb - 1) * B]
    diag = float(sum(float(b) * b for b in sizes))
    return imgs * ((float(n) * n - diag) / 2.0 + diag)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(x, q, cfg, n_targets, n_check=256, n_surface=20000):
    """The oracle (plain FP64 C with OpenMP, numpy for the small steps) timed
    stage by stage on bounded samples of the same workload, each stage's time
    scaled to the full step: the right-hand side at n_check of the check
    points, least squares and mapping in full, the near sum at n_targets
    particles, the surface sum at n_surface particles.  value = pair
    interactions of one full step / the scaled step time.  The preparation
    step (plan) is timed too but is not part of the per-step time."""
    import numpy as np

    import oracle
    from oracle import hsma as oh
    oh.build()
    L, bc = cfg["L"], cfg["bc"]
    rng = np.random.default_rng(0)
    n = len(q)
    t0 = time.perf_counter()
    plan = oracle.make_plan(L, bc, cfg["p"], cfg["M"], cfg["K"], cfg["R"])
    t_plan = time.perf_counter() - t0
    c = oh.normalize(x, L, bc)
    qq = np.asarray(q, dtype=np.float64)
    if bc == 2:
        c, qq = oh.double_slab(c, qq)
    src = np.concatenate([c, qq[:, None]], axis=1)
    ns = len(src)
    img = oracle.BC_METALLIC if bc == 1 else oracle.BC_PERIODIC
    pts = plan["X"] if plan["Xt"] is None else np.concatenate([plan["X"], plan["Xt"]])
    nchk = len(pts)
    stages = {}

    def stage(name, fn, full_scale, pairs_full, sample):
        t = time.perf_counter()
        out = fn()
        dt = time.perf_counter() - t
        stages[name] = {"sample": sample, "s": dt, "s_full_step": dt * full_scale}
        if pairs_full:
            stages[name]["pairs_full_step"] = pairs_full
            stages[name]["pairs_per_s"] = pairs_full / (dt * full_scale)
        return out

    kc = min(n_check, nchk)
    ic = rng.choice(nchk, kc, replace=False)
    stage("rhs", lambda: oracle.potential_at(img, L, src, pts[ic]), nchk / kc, 27.0 * nchk * ns,
          "%d of %d check points against all 27 N_s images" % (kc, nchk))
    b = rng.standard_normal(cfg["K"])   # timing only: the values do not matter
    A = stage("least_squares", lambda: oh.coefficients_from_rhs(plan, b), 1.0, 0.0, "full")
    surf = stage("mapping", lambda: oh.surface_images(plan, A), 1.0, 0.0, "full")
    kt = min(n_targets, n)
    it = rng.choice(n, kt, replace=False)
    stage("near", lambda: oracle.near_sum(img, L, src, it), n / kt, 27.0 * n * ns,
          "%d of %d particles against all 27 N_s images" % (kt, n))
    ks = min(n_surface, n)
    isf = rng.choice(n, ks, replace=False)
    stage("surface", lambda: oracle.surface_sum(src[isf, :3], surf), n / ks,
          float(n) * len(surf), "%d of %d particles against all %d surface points" % (ks, n, len(surf)))
    step_s = sum(v["s_full_step"] for v in stages.values())
    pairs = sum(v.get("pairs_full_step", 0.0) for v in stages.values())
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sampled = sum(v["s"] for v in stages.values())
    return {"value": pairs / step_s, "unit": "pair interactions/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "every stage of one update step on bounded samples (%.1f s of CPU work), "
                      "each scaled to the full step: %.1f s per step" % (sampled, step_s),
            "s_per_step_scaled": step_s, "plan_s": t_plan, "stages": stages}


def serving_measure(n_requests, refine, log=sys.stderr):
    """Serving stream (seeded trace): N log-uniform in [1e3, 1e5] (even),
    periodic or grounded cube with probability 1/2, p in {12, 16, 20},
    K = M = 10 p^2, R = 2.7L.  Closed loop (all requests at t = 0) gives
    solves/s of six paths: the served path (batched FP32-comp with
    ill-conditioned energies refined in FP64), the same with tree plans
    (requests of 24576 particles and more on the fast multipole method), and
    the batched server and one solve per request, each in FP32-comp and in
    FP64 without refinement (equal-precision comparisons).  Open loop
    (Poisson arrivals at 0.8 of a path's closed-loop rate) gives p50/p99
    latency.  Energies of the FP32 paths are compared with the FP64
    per-request path."""
    import numpy as np
    import torch

    from paper_1806_04801_amd import hsma, workloads

    torch.cuda.set_device(0)
    trace = workloads.serving_trace(n_requests, seed=4)
    plans = {}
    for prec in (hsma.FP64, hsma.FP32_COMP):
        for bc in (0, 1):
            for p in (12, 16, 20):
                plans[(prec, bc, p)] = hsma.Plan(1.0, bc, p, 10 * p * p, 10 * p * p, 2.7, precision=prec)
    for bc in (0, 1):
        for p in (12, 16, 20):
            plans[("fmm", bc, p)] = hsma.Plan(1.0, bc, p, 10 * p * p, 10 * p * p, 2.7, precision=hsma.FP32_COMP,
                                              near_mode=hsma.NEAR_TREE)
    xs, qs = [], []
    for r in trace:
        x, q = workloads.uniform_neutral(r["n"], 1.0, seed=r["seed"])
        xs.append(x)
        qs.append(q)
    pl = {prec: [plans[(prec, r["bc"], r["p"])] for r in trace] for prec in (hsma.FP64, hsma.FP32_COMP, "fmm")}
    n = len(trace)
    pairs = 0.0
    for r in trace:
        nchk = (2 if r["bc"] == 0 else 1) * 10 * r["p"] ** 2
        pairs += 27.0 * r["n"] * r["n"] + 27.0 * nchk * r["n"]
    # the served path (single precision, ill-conditioned energies refined in
    # double precision), and the batched paths at one precision each
    srv = {"served": hsma.Server(memory_bytes=16 << 30, max_active=64, precision=hsma.FP32_COMP,
                                 refine_below=refine),
           "fmm": hsma.Server(memory_bytes=16 << 30, max_active=64, precision=hsma.FP32_COMP,
                              refine_below=refine),
           hsma.FP32_COMP: hsma.Server(memory_bytes=16 << 30, max_active=64, precision=hsma.FP32_COMP,
                                       refine_below=0.0),
           hsma.FP64: hsma.Server(memory_bytes=16 << 30, max_active=64, precision=hsma.FP64)}
    zero = np.zeros(n)
    k = min(8, n)
    for key, prec in (("served", hsma.FP32_COMP), ("fmm", "fmm"), (hsma.FP32_COMP, hsma.FP32_COMP),
                      (hsma.FP64, hsma.FP64)):
        srv[key].run_trace(zero[:k], pl[prec][:k], xs[:k], qs[:k])   # warm-up of every path
        hsma.run_trace_sequential(zero[:k], pl[prec][:k], xs[:k], qs[:k])
    closed = {}
    energies = {}
    refined0 = srv["served"].stats()["refined"]
    refined0_fmm = srv["fmm"].stats()["refined"]
    for name, prec, key in (("served_fp32_refined", hsma.FP32_COMP, "served"),
                            ("served_fmm_refined", "fmm", "fmm"),
                            ("sequential_fp64", hsma.FP64, None),
                            ("batched_fp32", hsma.FP32_COMP, hsma.FP32_COMP),
                            ("sequential_fp32", hsma.FP32_COMP, None),
                            ("batched_fp64", hsma.FP64, hsma.FP64)):
        print("serving: closed loop, %s" % name, file=log, flush=True)
        if key is not None:
            e, _, wall = srv[key].run_trace(zero, pl[prec], xs, qs)
        else:
            e, _, wall = hsma.run_trace_sequential(zero, pl[prec], xs, qs)
        closed[name] = n / wall
        energies[name] = e
        if name == "served_fp32_refined":
            refined = srv["served"].stats()["refined"] - refined0
        if name == "served_fmm_refined":
            refined_fmm = srv["fmm"].stats()["refined"] - refined0_fmm
    mu32, mu64 = closed["served_fp32_refined"], closed["sequential_fp64"]
    gaps = np.random.default_rng(44).exponential(1.0, n)
    pct = lambda a, q_: float(np.percentile(a, q_)) * 1e3
    lat = {}
    mufmm = closed["served_fmm_refined"]
    for name, rate_of, prec, key in (("served_fp32_at_0.8_own", mu32, hsma.FP32_COMP, "served"),
                                     ("served_fmm_at_0.8_own", mufmm, "fmm", "fmm"),
                                     ("sequential_fp64_at_0.8_own", mu64, hsma.FP64, None),
                                     ("served_fp32_at_0.8_fp64_sequential", mu64, hsma.FP32_COMP, "served")):
        print("serving: open loop, %s" % name, file=log, flush=True)
        arr = np.cumsum(gaps) / (0.8 * rate_of)
        if key is not None:
            _, l_, _ = srv[key].run_trace(arr, pl[prec], xs, qs)
        else:
            _, l_, _ = hsma.run_trace_sequential(arr, pl[prec], xs, qs)
        lat[name] = {"p50_ms": pct(l_, 50), "p99_ms": pct(l_, 99), "offered_per_s": 0.8 * rate_of}
    e64 = energies["sequential_fp64"]
    err = {}
    for name in ("served_fp32_refined", "served_fmm_refined", "batched_fp32", "sequential_fp32",
                 "batched_fp64"):
        rel = np.abs(energies[name] - e64) / np.abs(e64)
        err[name] = {"p50": float(np.median(rel)), "p99": float(np.percentile(rel, 99)),
                     "max": float(rel.max()), "frac_le_1e-5": float(np.mean(rel <= 1e-5))}
    return {
        "requests": n,
        "desc": "N log-uniform [1e3,1e5] even, bc periodic/grounded 1/2, p in {12,16,20}, "
                "K=M=10p^2, R=2.7L; seeded Poisson trace (seed 4)",
        "pair_interactions": pairs,
        "solves_per_s": closed,
        # equal precision: the batched server against one solve per request,
        # neither refining
        "gain_batched_vs_sequential": {"fp32": closed["batched_fp32"] / closed["sequential_fp32"],
                                       "fp64": closed["batched_fp64"] / closed["sequential_fp64"]},
        # the served single-precision path (every energy within 1e-5) against
        # the plain double-precision path
        "gain_served_fp32_vs_sequential_fp64": mu32 / mu64,
        # the served path with tree plans (fast multipole method from 24576
        # particles on, same refinement) against the plain double-precision path
        "gain_served_fmm_vs_sequential_fp64": mufmm / mu64,
        "latency": lat,
        "refine_below": refine,
        "refined_in_fp64": {"requests": int(refined), "fraction": refined / n},
        "refined_in_fp64_fmm_path": {"requests": int(refined_fmm), "fraction": refined_fmm / n},
        "rel_energy_err_vs_sequential_fp64": err,
    }


def serving(args):
    """--workload serving: the serving measurement as its own JSON line."""
    sv = serving_measure(args.requests, args.refine)
    mu = sv["solves_per_s"]["served_fp32_refined"]
    rec = {
        "metric": "solves/s", "value": mu, "unit": "solves/s", "n_gpus": 1,
        "steps": sv["requests"], "warmup": 8, "ms_per_step": 1e3 / mu, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving", "serving": sv},
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


def fmm_measure(cfg, xd, qd, steps, e_direct):
    """The same workload with the fast multipole method for the near sum and
    the right-hand side (FP64, expansion order 16): ms per update step, the
    near sum's share (tree build included, HIP events), and the energy against
    the direct step of this run."""
    import torch

    from paper_1806_04801_amd import hsma
    plan = hsma.Plan(cfg["L"], cfg["bc"], cfg["p"], cfg["M"], cfg["K"], cfg["R"], precision=hsma.FP64,
                     near_mode=hsma.NEAR_TREE)
    plan.energy_forces(xd, qd)   # warm-up
    torch.cuda.synchronize()
    hsma.timing_read()
    hsma.timing_enable(True)
    t0 = time.perf_counter()
    for i in range(steps):
        e, _, _ = plan.energy_forces(xd, qd)
        print("fmm step %d done: energy %.10e" % (i, e), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    hsma.timing_enable(False)
    kt = hsma.timing_read()
    sched = plan.near_schedule(len(qd))
    info = plan.info
    plan.close()
    return {"steps": steps, "ms_per_step": 1e3 * dt, "near_ms": kt["near"][0] / max(kt["near"][1], 1),
            "rhs_ms": kt["rhs"][0] / max(kt["rhs"][1], 1), "near_kernel": "fmm" if sched["kind"] == 2 else sched,
            "order": info["tree_order"], "precision": "fp64", "energy": e,
            "rel_energy_diff_vs_direct_fp32_step": abs(e - e_direct) / abs(e_direct)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (there is no multi-GPU path); use --gpus 1",
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
    x, q = workloads.make_inputs(args.workload, n=args.n if args.n > 0 else None)
    n = len(q)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.grad:
        return adjoint_bench(args, cfg, x, q, prec)
    near_mode = {"sphere": hsma.NEAR_SPHERE, "tree": hsma.NEAR_TREE}.get(args.near, hsma.NEAR_BLOCK)
    if near_mode == hsma.NEAR_TREE:
        prec = hsma.FP64
    plan = hsma.Plan(cfg["L"], cfg["bc"], cfg["p"], cfg["M"], cfg["K"], cfg["R"], precision=prec,
                     near_mode=near_mode,
                     dipole_mode=hsma.DIPOLE_LAYERS if args.dipole == "layers" else hsma.DIPOLE_EXACT,
                     far_mode=hsma.FAR_DIRECT if args.far == "direct" else hsma.FAR_SURFACE,
                     tree_order=args.tree_order)
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
    kind = "pair-once" if sched["kind"] == 1 else "tiles"
    if near_mode == hsma.NEAR_TREE:
        kind = "tree"
    ptag = "f32" if prec == hsma.FP32_COMP else "f64"
    peak = FP32_PEAK_TFLOPS if prec == hsma.FP32_COMP else FP64_PEAK_TFLOPS
    if near_mode in (hsma.NEAR_SPHERE, hsma.NEAR_TREE):
        # tree: the pair interactions of the direct sum it replaces (the
        # multipole method evaluates far fewer; no flop roofline for it)
        evaluated = near_pairs
    else:
        evaluated = near_evaluated_pairs(n, cfg, sched)
    achieved = NEAR_FLOPS_PER_PAIR * evaluated / near_avg_s / 1e12
    other_fracs = {"flops_20_per_evaluated_pair_image": achieved / peak}
    if sched["kind"] == 1:
        # unordered cross-block pairs with both directions at 28 flops
        both = NEAR_FLOPS_PER_UNORDERED_PAIR_BOTH_DIRECTIONS * (near_pairs / 2.0)
        other_fracs["flops_28_per_unordered_pair_image_both_directions"] = both / near_avg_s / 1e12 / peak
    # the workload's name, or name and size when --n resizes it (profiles are per name)
    wtag = args.workload if args.n <= 0 else "%s_n%d" % (args.workload, n)
    counted = profiled_field(wtag, ptag, kind, "counter_tflops")
    if counted is not None:
        other_fracs["valu_flops_counted_by_rocprof"] = counted / peak
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
            "workload": wtag,
            "near_set": args.near,
            "surface_dipole": args.dipole,
            "far_field": args.far,
            "desc": cfg["desc"],
            "N": n, "bc": cfg["bc"], "p": cfg["p"], "K": cfg["K"], "M_eff": info["M_eff"],
            "R": cfg["R"], "precision": "fp32 pair sums + two-sum accumulation" if prec else "fp64",
            "pairs_per_step": {"near": near_pairs, "rhs": rhs_pairs, "surface": surf_pairs},
            "near_pairs_per_s": near_pairs / near_avg_s,
            "near_kernel": kind,
            "near_schedule": sched,
            "near_pair_images_evaluated": evaluated,
            "near_ms": 1e3 * near_avg_s,
            "near_peak_fractions": other_fracs,
            "kernel_ms_avg": {k: (v[0] / max(v[1], 1)) for k, v in kt.items()},
            "energy": energies[-1],
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": profiled_traffic(wtag, ptag, kind),
        },
    }
    if near_mode == hsma.NEAR_TREE:
        # value and near_pairs_per_s count the direct sum's pair interactions
        # (direct-equivalent rates); the multipole method has no pair count
        # to charge flops to, so it reports no roofline
        rec["roofline"] = None
        rec["config"]["value_counts"] = "direct-equivalent pair interactions (the fast multipole method " \
                                        "evaluates far fewer)"
        del rec["config"]["near_peak_fractions"]
    if host_entry is not None:
        host_entry["pairs_per_s"] = pairs_step / (host_entry["ms_per_call"] / 1e3)
        rec["config"]["host_entry"] = host_entry
    if args.fmm_steps > 0 and args.workload == "periodic1m" and args.n <= 0 and near_mode == hsma.NEAR_BLOCK:
        rec["fmm"] = fmm_measure(cfg, xd, qd, args.fmm_steps, energies[-1])
    del xd, qd, phi, F
    plan.close()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(x, q, cfg, args.cpu_targets)
    if args.serving_requests > 0 and args.workload == "periodic1m" and args.n <= 0:
        # the serving half of the metric (solves/s and p99 latency at 1e-5)
        torch.cuda.empty_cache()
        rec["serving"] = serving_measure(args.serving_requests, args.refine)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
