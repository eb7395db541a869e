#!/usr/bin/env python3
"""Throughput of the tree-code on one MI355X: particles per second per full force
evaluation (tree build + walk), Plummer sphere N = 2^20, theta = 0.75,
eps = 1/64, leapfrog dt = 1/64.

A step is one leapfrog step through the C ABI: kick, drift, full rebuild (bounding
box, keys, radix sort, reorder, cells, groups, moments), opening radii, group walk,
kick, and the float64 energy/momentum sums.  Inputs are resident on the device
before the timed region starts.  Prints one JSON line on stdout.

  python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particles/s per full force eval (build+walk), N=1M Plummer theta=0.75; p99 served"
PEAK_FP32_VECTOR_TFLOPS = 157.3      # MI355X published FP32 vector peak (256 CU x 2.4 GHz)
# Stated flops per interaction, counted from the kernel source (walk.hip):
#   particle-particle: 3 sub, 3 fma, 1 rsqrt, 3 mul, 3 fma, 1 sub            = 20
#   particle-cell:     3 sub, 3 fma, 1 rsqrt, 3 mul (rho^2, rho^3, rho^5),
#                      3 mul + 6 fma (3S r), 1 mul + 2 fma (r.3S.r), 1 mul,
#                      3 fma (potential), 2 fma + 1 mul (radial factor),
#                      6 fma (acceleration)                                  = 57
FLOPS_PP = 20
FLOPS_PC = 57
PAPER_TRAVERSE_RATE = 2.8e6          # particles/s, tree traverse only, GTX480 (Sect. 4.1)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_plummer_1m_traffic.json")
WALK_SRC = os.path.join(ROOT, "paper_1106_1900_amd", "csrc", "walk.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def walk_source_hash():
    with open(WALK_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per walk launch from the committed counter runs, if they were taken
    on the current walk kernel source; None otherwise."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("walk_source_sha256_16") != walk_source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(pos, mass, theta, eps, budget_s):
    """The oracle as it stands, single-threaded: full tree build plus the walk and
    float64 evaluation of a seeded sample of groups until about budget_s seconds
    of evaluation, scaled to a full force evaluation."""
    import numpy as np

    import oracle
    n = pos.shape[0]
    t0 = time.perf_counter()
    tree = oracle.Tree(pos, mass)
    t_build = time.perf_counter() - t0
    g = tree.groups()
    order = np.random.default_rng(11).permutation(tree.ngroups)
    done_p = 0
    done_g = 0
    t_walk = 0.0
    chunk = 64
    while t_walk < budget_s and done_g < tree.ngroups:
        sel = np.sort(order[done_g:done_g + chunk])
        t1 = time.perf_counter()
        tree.forces(theta, eps, sel)
        t_walk += time.perf_counter() - t1
        done_g += sel.size
        done_p += int(g["count"][sel].sum())
    rate_walk = done_p / t_walk
    t_full = t_build + n / rate_walk
    return {
        "value": n / t_full,
        "unit": "particles/s",
        "cores": 1,
        "kind": "oracle",
        "sample": ("single-threaded C oracle on the same Plummer N=%d input: full tree build "
                   "(%.2f s) plus walk and float64 evaluation of %d randomly chosen groups "
                   "(%d particles, %.1f s), evaluation time scaled to all %d particles"
                   % (n, t_build, done_g, done_p, t_walk, n)),
    }


def accuracy_sample(pos, mass, acc_gpu, eps, ntarget=256):
    """Relative acceleration error (Eq. (2)) of the GPU forces against the oracle's
    float64 direct summation on seeded targets."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(12)
    tgt = np.sort(rng.choice(pos.shape[0], ntarget, replace=False))
    ad, _ = oracle.direct(pos, mass, eps, tgt)
    a = acc_gpu[tgt].astype(np.float64)
    err = np.linalg.norm(a - ad, axis=1) / np.linalg.norm(ad, axis=1)
    return {"targets": int(ntarget), "median": float(np.median(err)),
            "p99": float(np.percentile(err, 99)), "reference": "oracle float64 direct summation"}


def calib_copy():
    """A plain device copy of 1 GiB (read 1 GiB, write 1 GiB) for scaling the HBM
    counters of a profiler run."""
    import torch
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("calib copy done: 1 GiB read + 1 GiB write per copy, 3 copies")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 20, help="particles (default 2^20)")
    ap.add_argument("--theta", type=float, default=0.75)
    ap.add_argument("--eps", type=float, default=1.0 / 64)
    ap.add_argument("--dt", type=float, default=1.0 / 64)
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle evaluation for the CPU baseline (0: skip)")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--calib-copy", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import numpy as np
    import torch

    import paper_1106_1900_amd as bh
    import workloads

    if args.calib_copy:
        calib_copy()

    n = args.n
    log("generating Plummer N=%d" % n)
    pos, vel, mass = workloads.plummer(n, 2)
    dpos = torch.from_numpy(pos).cuda()
    dvel = torch.from_numpy(vel).cuda()
    dmass = torch.from_numpy(mass).cuda()
    torch.cuda.synchronize()

    ctx = bh.Context(nleaf=16, ncrit=64)
    ctx.build_tree(dpos, dmass)
    ctx.set_velocities(dvel)
    acc0, _ = ctx.compute_forces(args.theta, args.eps)
    e0 = ctx.energy()
    acc0_h = acc0.cpu().numpy()

    for _ in range(args.warmup):
        ctx.leapfrog_step(args.dt)
        ctx.energy()
    torch.cuda.synchronize()
    s0 = ctx.stats()

    log("timing %d steps" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.leapfrog_step(args.dt)
        ctx.energy()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s1 = ctx.stats()
    e1 = ctx.energy()

    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed

    launches = s1.walk_kernel_launches - s0.walk_kernel_launches
    walk_ms = (s1.walk_kernel_ms_total - s0.walk_kernel_ms_total) / max(launches, 1)
    pp = (s1.total_npp - s0.total_npp) / max(launches, 1)
    pc = (s1.total_npc - s0.total_npc) / max(launches, 1)
    flops = FLOPS_PP * pp + FLOPS_PC * pc
    achieved = flops / (walk_ms * 1e-3) / 1e12 if walk_ms > 0 else 0.0
    traffic = measured_traffic()
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
                "traffic": traffic, "kernel": "walk_kernel",
                "walk_ms_per_launch": round(walk_ms, 4),
                "interactions_per_launch": {"pp": pp, "pc": pc},
                "flops_per_interaction": {"pp": FLOPS_PP, "pc": FLOPS_PC}}

    phases = {"keys": s1.ms_keys, "sort": s1.ms_sort, "move": s1.ms_move, "tree": s1.ms_tree,
              "moments": s1.ms_moments, "walk_total": s1.ms_walk}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plummer N=%d theta=%g eps=%g dt=%g leapfrog, nleaf 16, group 64"
                               % (n, args.theta, args.eps, args.dt),
                   "n": n, "theta": args.theta, "eps": args.eps, "dt": args.dt,
                   "nleaf": 16, "ncrit": 64, "seed": 2},
        "roofline": roofline,
        "interactions_per_s": (pp + pc) * launches / elapsed,
        "phases_ms_last_step": {k: round(v, 4) for k, v in phases.items()},
        "energy_error_over_timed_steps": float((e0[2] - e1[2]) / e0[2]),
        "tree": {"ncells": s1.ncells, "ngroups": s1.ngroups, "depth": s1.depth},
        "paper_reference": {"value": PAPER_TRAVERSE_RATE, "unit": "particles/s",
                            "what": "tree traverse only, 1x GTX480, N=2^20 Plummer, theta=0.75"},
    }
    if not args.no_accuracy:
        out["accuracy_vs_direct"] = accuracy_sample(pos, mass, acc0_h, args.eps)
    if args.cpu_budget > 0 and rank == 0:
        log("timing the oracle on the host (%.0f s budget)" % args.cpu_budget)
        out["cpu_baseline"] = cpu_baseline(pos, mass, args.theta, args.eps, args.cpu_budget)
    ctx.close()
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
