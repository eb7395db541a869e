#!/usr/bin/env python3
"""Throughput of the tree-code on one MI355X: particles per second per full force
evaluation (tree build + walk), Plummer sphere N = 2^20, theta = 0.75,
eps = 1/64, leapfrog dt = 1/64.

A step is one leapfrog step through the C ABI: kick, drift, full rebuild (bounding
box, keys, radix sort, reorder, cells, groups, moments), opening radii, group walk,
kick, and the float64 energy/momentum sums.  Inputs are resident on the device
before the timed region starts.  Prints one JSON line on stdout.

The line also carries the batched form ("batch": 512 Plummer clusters of
1024..65536 particles in one forest, one captured graph per step, against the same
clusters stepped one context at a time) unless --no-batch is given, and the
serving loop ("served": the 2000-request Poisson trace at 200 requests/s, each a
force evaluation plus 10 leapfrog steps, latency percentiles including queueing;
"served_constrained": the same under a 4 GiB budget; "served_plain_fifo": the
same trace served one request at a time through the plain path) unless
--no-serve, the 4,194,304-particle galaxy ("galaxy", theta 0.4) unless
--no-galaxy, and the energy error of the two-galaxy encounter over its first 125
time units at theta 0.75 and 0.5 ("merger") unless --no-merger.  Force errors are measured against float64 direct summation on
16384 seeded targets.

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


_T0 = time.perf_counter()


def log(*a):
    print("[%7.1f s]" % (time.perf_counter() - _T0), *a, file=sys.stderr, flush=True)


def walk_source_hash():
    """Fingerprint of the walk kernel: its source and its compile flags."""
    from paper_1106_1900_amd.build import SOURCE_FLAGS
    with open(WALK_SRC, "rb") as f:
        src = f.read()
    return hashlib.sha256(src + b"\0" + " ".join(SOURCE_FLAGS.get("walk.hip", ())).encode()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per walk launch from the committed counter runs, if they were taken
    on the current walk kernel (source and compile flags); None otherwise."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("walk_source_sha256_16") != walk_source_hash():
        return None
    return d.get("bytes_per_launch")


def host_cpu():
    """The host the oracle baselines ran on: CPU model and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


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
        "sample": ("single-threaded C oracle on the same N=%d input: full tree build "
                   "(%.2f s) plus walk and float64 evaluation of %d randomly chosen groups "
                   "(%d particles, %.1f s), evaluation time scaled to all %d particles"
                   % (n, t_build, done_g, done_p, t_walk, n)),
        "host": host_cpu(),
    }


def cpu_worker(index, workers, n, theta, eps, budget_s):
    """One process of the all-cores baseline: the single-threaded oracle on the
    groups with index = `index` mod `workers` (seeded order), for budget_s seconds
    of evaluation.  Touches no GPU."""
    import numpy as np

    import oracle
    import workloads
    pos, _, mass = workloads.plummer(n, 2)
    t0 = time.perf_counter()
    tree = oracle.Tree(pos, mass)
    t_build = time.perf_counter() - t0
    g = tree.groups()
    mine = np.random.default_rng(11).permutation(tree.ngroups)[index::workers]
    done_p = done_g = 0
    t_walk = 0.0
    while t_walk < budget_s and done_g < mine.size:
        sel = np.sort(mine[done_g:done_g + 64])
        t1 = time.perf_counter()
        tree.forces(theta, eps, sel)
        t_walk += time.perf_counter() - t1
        done_g += sel.size
        done_p += int(g["count"][sel].sum())
    print(json.dumps({"t_build": t_build, "t_walk": t_walk, "done_p": done_p, "done_g": done_g}),
          flush=True)


def cpu_baseline_all_cores(n, theta, eps, budget_s, workers):
    """The same oracle in one process per core over disjoint group sets: the
    evaluation rates add up; the tree build (single-threaded) is counted once."""
    import subprocess
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker",
                               str(i), str(workers), str(n), repr(theta), repr(eps),
                               repr(budget_s)], stdout=subprocess.PIPE, text=True)
             for i in range(workers)]
    res = []
    for p in procs:
        out_s, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("oracle worker failed")
        res.append(json.loads(out_s.strip().splitlines()[-1]))
    rate = sum(r["done_p"] / r["t_walk"] for r in res if r["t_walk"] > 0)
    t_build = min(r["t_build"] for r in res)
    t_full = t_build + n / rate
    return {"value": n / t_full, "unit": "particles/s", "cores": workers, "kind": "oracle",
            "sample": ("the single-threaded C oracle in %d processes over disjoint seeded group "
                       "sets of the same input, %.0f s of evaluation each (%d groups, %d particles "
                       "in all); evaluation rates summed, one tree build (%.2f s) counted"
                       % (workers, budget_s, sum(r["done_g"] for r in res),
                          sum(r["done_p"] for r in res), t_build)),
            "host": host_cpu()}


def direct_fp64(pos, mass, eps, tgt):
    """Float64 direct summation (Eq. (2)'s reference) of the accelerations of the
    target particles tgt over all sources, the self pair left out: plain torch
    element-wise arithmetic on the GPU, in chunks (independent of the library)."""
    import numpy as np
    import torch
    dev = "cuda"
    x = torch.from_numpy(np.ascontiguousarray(pos, dtype=np.float64)).to(dev)
    m = torch.from_numpy(np.ascontiguousarray(mass, dtype=np.float64)).to(dev)
    t = torch.from_numpy(np.asarray(tgt, dtype=np.int64)).to(dev)
    e2 = float(np.float32(eps)) ** 2           # the softening is a float32 parameter
    out = torch.zeros((t.shape[0], 3), dtype=torch.float64, device=dev)
    tc, sc = 128, 1 << 20
    for i0 in range(0, t.shape[0], tc):
        ti = t[i0:i0 + tc]
        xi = x[ti]                                              # [T, 3]
        acc = torch.zeros((ti.shape[0], 3), dtype=torch.float64, device=dev)
        for j0 in range(0, x.shape[0], sc):
            xj = x[j0:j0 + sc]                                  # [S, 3]
            d = xj.unsqueeze(0) - xi.unsqueeze(1)               # [T, S, 3]: x_j - x_i
            r2 = (d * d).sum(dim=2)
            s = r2 + e2
            w = torch.where(r2 > 0, m[j0:j0 + sc].unsqueeze(0) / (s * torch.sqrt(s)),
                            torch.zeros_like(s))
            jj = torch.arange(j0, j0 + xj.shape[0], device=dev)
            w = torch.where(jj.unsqueeze(0) == ti.unsqueeze(1), torch.zeros_like(w), w)
            acc += (w.unsqueeze(2) * d).sum(dim=1)
        out[i0:i0 + tc] = acc
    torch.cuda.synchronize()
    return out.cpu().numpy()


def accuracy_sample(pos, mass, acc_gpu, eps, ntarget=16384):
    """Relative acceleration error (Eq. (2)) of the GPU forces against float64
    direct summation on seeded targets."""
    import numpy as np
    rng = np.random.default_rng(12)
    tgt = np.sort(rng.choice(pos.shape[0], ntarget, replace=False))
    ad = direct_fp64(pos, mass, eps, tgt)
    a = acc_gpu[tgt].astype(np.float64)
    err = np.linalg.norm(a - ad, axis=1) / np.linalg.norm(ad, axis=1)
    return {"targets": int(ntarget), "median": float(np.median(err)),
            "p99": float(np.percentile(err, 99)), "reference": "float64 direct summation (torch)"}


def pooled_accuracy(systems, ntarget, seed):
    """Δa/a against float64 direct summation pooled over several systems: each
    entry (pos, mass, acc, eps) contributes ntarget seeded targets."""
    import numpy as np
    rng = np.random.default_rng(seed)
    errs = []
    for pos, mass, acc, eps in systems:
        k = min(ntarget, pos.shape[0])
        tgt = np.sort(rng.choice(pos.shape[0], k, replace=False))
        ad = direct_fp64(pos, mass, eps, tgt)
        na = np.linalg.norm(ad, axis=1)
        ok = na > 0
        e = np.linalg.norm(acc[tgt].astype(np.float64) - ad, axis=1)
        errs.append(e[ok] / na[ok])
    err = np.concatenate(errs)
    return {"systems": len(systems), "targets": int(err.size), "median": float(np.median(err)),
            "p99": float(np.percentile(err, 99)), "reference": "float64 direct summation (torch)"}


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


def bench_batch(k, steps, warmup, dt=1.0 / 128, seed=4, alone=True):
    """Sum of N_i over a step of all k clusters, batched (one forest, graph replay)
    against one context per cluster stepped in turn."""
    import numpy as np
    import torch

    import paper_1106_1900_amd as bh
    import workloads
    log("generating %d clusters" % k)
    cl = workloads.cluster_batch(k, seed)
    ntot = int(sum(q["n"] for q in cl))
    pos = torch.from_numpy(np.concatenate([q["pos"] for q in cl])).cuda()
    vel = torch.from_numpy(np.concatenate([q["vel"] for q in cl])).cuda()
    mass = torch.from_numpy(np.concatenate([q["mass"] for q in cl])).cuda()
    table_in = [dict(n=q["n"], theta=q["theta"], eps=q["eps"], dt=dt) for q in cl]
    ctx = bh.Context()
    ctx.batch_build(table_in, pos, mass, vel)
    ctx.batch_forces(want=False)
    ctx.batch_run(warmup)
    ctx.batch_energy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.batch_run(steps)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    en = ctx.batch_energy()
    st = ctx.stats()
    # force error of the batched form: 4 seeded clusters (smallest, largest, two
    # others), 256 targets each, at their positions after the timed steps
    xs, _, acc_b, _ = ctx.get_state()
    xs = xs.cpu().numpy()
    acc_b = acc_b.cpu().numpy()
    starts = np.concatenate([[0], np.cumsum([q["n"] for q in cl])[:-1]])
    pick = sorted({int(np.argmin([q["n"] for q in cl])), int(np.argmax([q["n"] for q in cl]))}
                  | set(np.random.default_rng(13).choice(k, 2, replace=False).tolist()))
    accuracy = pooled_accuracy([(xs[starts[c]:starts[c] + cl[c]["n"]], cl[c]["mass"],
                                 acc_b[starts[c]:starts[c] + cl[c]["n"]], cl[c]["eps"]) for c in pick],
                                256, 14)
    # the batched walk against the FP32 roofline: one eager force evaluation (graph
    # replays are not timed per kernel) at the same positions
    ctx.batch_forces(want=False)
    torch.cuda.synchronize()
    sw = ctx.stats()
    walk_flops = FLOPS_PP * sw.sum_npp + FLOPS_PC * sw.sum_npc
    walk_tflops = walk_flops / (sw.ms_walk_kernel * 1e-3) / 1e12 if sw.ms_walk_kernel > 0 else 0.0

    # leaf and group sizes tuned per class (floor(log2 N), theta), then the same
    # clusters reloaded with the tuned sizes and timed again
    log("autotuning leaf and group sizes")
    tt0 = time.perf_counter()
    table = ctx.autotune(reps=3)
    t_tune = time.perf_counter() - tt0
    tuned = [dict(q, nleaf=0, ncrit=0) for q in table_in]
    ctx.batch_build(tuned, pos, mass, vel)
    ctx.batch_forces(want=False)
    ctx.batch_run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.batch_run(steps)
    torch.cuda.synchronize()
    t_tuned = (time.perf_counter() - t0) / steps
    ctx.batch_forces(want=False)
    torch.cuda.synchronize()
    swt = ctx.stats()
    tuned_flops = FLOPS_PP * swt.sum_npp + FLOPS_PC * swt.sum_npc
    tuned_tflops = tuned_flops / (swt.ms_walk_kernel * 1e-3) / 1e12 if swt.ms_walk_kernel > 0 else 0.0
    ctx.close()

    out = {
        "workload": "%d Plummer clusters, N log-uniform in [1024, 65536] (sum %d), theta 0.75, "
                    "eps 0.04 N^-1/3, dt %g, nleaf 16, group 64" % (k, ntot, dt),
        "clusters": k, "particles": ntot, "steps": steps,
        "value": ntot / t_batch, "unit": "particles/s",
        "ms_per_step": 1e3 * t_batch,
        "max_abs_energy_error": float(np.abs(en[:, 6]).max()),
        "accuracy_vs_direct": accuracy,
        "graph_launches": int(st.graph_launches),
        "walk": {"ms_per_launch": sw.ms_walk_kernel, "interactions": {"pp": sw.sum_npp,
                                                                     "pc": sw.sum_npc},
                 "tflops": walk_tflops, "frac_of_157_3": walk_tflops / PEAK_FP32_VECTOR_TFLOPS},
        "tuned_walk": {"ms_per_launch": swt.ms_walk_kernel,
                       "interactions": {"pp": swt.sum_npp, "pc": swt.sum_npc},
                       "tflops": tuned_tflops,
                       "frac_of_157_3": tuned_tflops / PEAK_FP32_VECTOR_TFLOPS},
        "tuned_value": ntot / t_tuned,
        "tuned_ms_per_step": 1e3 * t_tuned,
        "autotune_seconds": t_tune,
        "tuning": [{"log2n": t["log2n"], "theta": round(t["theta"], 6), "nleaf": t["nleaf"],
                    "ncrit": t["ncrit"], "ms": round(t["ms"], 4),
                    "ms_default": round(t["ms_default"], 4)} for t in table],
    }
    if not alone:
        return out
    log("stepping the %d clusters one context at a time" % k)
    ones = []
    first = 0
    for q in cl:
        n = q["n"]
        c1 = bh.Context()
        c1.build_tree(pos[first:first + n], mass[first:first + n])
        c1.set_velocities(vel[first:first + n].contiguous())
        c1.compute_forces(q["theta"], q["eps"], want=False)
        ones.append(c1)
        first += n
    for _ in range(warmup):
        for c1 in ones:
            c1.leapfrog_step(dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for c1 in ones:
            c1.leapfrog_step(dt)
    torch.cuda.synchronize()
    t_one = (time.perf_counter() - t0) / steps
    for c1 in ones:
        c1.close()
    out.update({
        "one_at_a_time_particles_per_s": ntot / t_one,
        "one_at_a_time_ms_per_step": 1e3 * t_one,
        "speedup_vs_one_at_a_time": t_one / t_batch,
    })
    return out


_REQUEST_POOLS = {}


def request_inputs(count, rate, steps=10, seed=5):
    """The served trace and its inputs.  Input pools: one Plummer and one Hernquist
    sphere of 2 nmax particles on the device (kept for every run on the same
    trace).  A request of n particles takes n consecutive particles of its model
    at a seeded offset (the draws are independent, so the window is itself a
    sample of the model) with masses 1/n."""
    import numpy as np
    import torch

    import workloads
    trace = workloads.request_trace(count, rate, seed, steps=steps)
    nmax = max(q["n"] for q in trace)
    key = (nmax,)
    if key not in _REQUEST_POOLS:
        _REQUEST_POOLS.clear()
        log("generating request pools of %d particles" % nmax)
        pools = {}
        for name, gen in (("plummer", workloads.plummer), ("hernquist", workloads.hernquist)):
            p, v, _ = gen(2 * nmax, 51 if name == "plummer" else 52)
            pools[name] = (torch.from_numpy(p).cuda(), torch.from_numpy(v).cuda())
        _REQUEST_POOLS[key] = pools
    rng = np.random.default_rng(seed + 1)
    offsets = [int(rng.integers(0, nmax)) for _ in trace]
    return trace, _REQUEST_POOLS[key], offsets


def trace_workload(count, rate, steps):
    return ("%d requests, Poisson arrivals at %g/s; Plummer or Hernquist (even odds), "
            "N log-uniform in [1024, 2097152], theta 0.5 or 0.75, eps 0.01, 1 force "
            "evaluation + %d leapfrog steps of dt 1/128" % (count, rate, steps))


def bench_serve(count, rate, budget, steps=10, seed=5, max_requests=256, max_resident=0):
    """The serving loop on a Poisson trace: latency (completion - arrival, with
    queueing) percentiles, offered and served particle-force-evaluation rates."""
    import numpy as np
    import torch

    import paper_1106_1900_amd as bh
    trace, pools, offsets = request_inputs(count, rate, steps, seed)
    # requests whose final state is checked against direct summation: four
    # seeded requests below 2^18 particles
    small = [i for i, q in enumerate(trace) if q["n"] < (1 << 18)]
    check = set(np.random.default_rng(seed + 2).choice(small, min(4, len(small)),
                                                      replace=False).tolist())
    kept = {}
    srv = bh.Server(budget, max_requests=max_requests, max_resident=max_resident)
    cap = srv.stats()["capacity_particles"]
    torch.cuda.synchronize()
    t0 = srv.now()
    i = 0
    open_t = []
    last_poll = 0
    while True:
        now = srv.now() - t0
        while i < count and trace[i]["arrival"] <= now:
            q = trace[i]
            n = q["n"]
            pp, pv = pools[q["shape"]]
            o = offsets[i]
            m = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")
            out_pos = torch.empty((n, 3), dtype=torch.float64, device="cuda")
            out_acc = torch.empty((n, 3), dtype=torch.float32, device="cuda")
            tk = srv.submit(pp[o:o + n], m, pv[o:o + n], q["theta"], q["eps"], q["dt"], q["steps"],
                            arrival=t0 + q["arrival"], out_pos=out_pos, out_acc=out_acc)
            open_t.append(tk)
            if i in check:
                kept[i] = (m, out_pos, out_acc)
            i += 1
        st = srv.stats()
        if st["completed"] + st["rejected"] == count:
            break
        if st["resident_requests"] == 0 and st["queued"] == 0:
            time.sleep(max(0.0, min(0.002, trace[i]["arrival"] - (srv.now() - t0))))
            continue
        srv.step()
        if st["iterations"] - last_poll >= 16:
            # release the arrays of finished requests
            open_t = [t for t in open_t if srv.poll(t)["state"] < 2]
            last_poll = st["iterations"]
    t_end = srv.now() - t0
    st = srv.stats()
    done = [srv.poll(t) for t in range(1, count + 1)]
    first_arrival = trace[0]["arrival"]
    work = sum(q["n"] * (1 + q["steps"]) for q in trace)
    dE = [abs(d["energy"][6]) for d in done if d["state"] == 2]
    srv.close()
    torch.cuda.synchronize()
    accuracy = pooled_accuracy([(kept[i][1].cpu().numpy(), kept[i][0].cpu().numpy(),
                                 kept[i][2].cpu().numpy(), trace[i]["eps"]) for i in sorted(kept)],
                               256, 15)
    return {
        "workload": trace_workload(count, rate, steps),
        "hbm_budget_bytes": int(budget), "capacity_particles": int(cap),
        "max_resident": int(max_resident),
        "latency_p50_s": st["latency_p50"], "latency_p99_s": st["latency_p99"],
        "latency_max_s": st["latency_max"],
        "queue_wait_p50_s": st["queue_wait_p50"], "queue_wait_p99_s": st["queue_wait_p99"],
        "offered_particle_evals_per_s": work / (trace[-1]["arrival"] - first_arrival),
        "served_particle_evals_per_s": st["particle_evals"] / (t_end - first_arrival),
        "completed": st["completed"], "rejected": st["rejected"], "iterations": st["iterations"],
        "wall_s": t_end, "max_abs_energy_error": max(dE) if dE else None,
        "accuracy_vs_direct": dict(accuracy, what="final accelerations of 4 seeded requests "
                                   "below 2^18 particles at their final positions"),
    }


def bench_fifo(count, rate, steps=10, seed=5):
    """The plain path on the same trace: one request at a time in arrival order,
    each through one context (sized once for the largest request): load
    (bh_build_tree), velocities, one force evaluation, `steps` leapfrog steps and
    the final positions, accelerations and energy sums copied out (as the server
    hands back), then the next request.  Latency = completion -
    arrival with the same arrival times as the served runs."""
    import numpy as np
    import torch

    import paper_1106_1900_amd as bh
    trace, pools, offsets = request_inputs(count, rate, steps, seed)
    nmax = max(q["n"] for q in trace)
    ctx = bh.Context(max_n=nmax)
    out_pos = torch.empty((nmax, 3), dtype=torch.float64, device="cuda")
    out_acc = torch.empty((nmax, 3), dtype=torch.float32, device="cuda")
    masses = {}
    lat, wait = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, q in enumerate(trace):
        now = time.perf_counter() - t0
        if now < q["arrival"]:
            time.sleep(q["arrival"] - now)
        start = time.perf_counter() - t0
        n = q["n"]
        pp, pv = pools[q["shape"]]
        o = offsets[i]
        if n not in masses:
            masses[n] = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")
        ctx.build_tree(pp[o:o + n], masses[n])
        ctx.set_velocities(pv[o:o + n])
        ctx.compute_forces(q["theta"], q["eps"], want=False)
        for _ in range(q["steps"]):
            ctx.leapfrog_step(q["dt"])
        ctx.get_state(pos=out_pos[:n], acc=out_acc[:n])
        ctx.energy()                       # reads the step's energy sums (synchronises)
        done = time.perf_counter() - t0
        lat.append(done - q["arrival"])
        wait.append(start - q["arrival"])
    t_end = time.perf_counter() - t0
    ctx.close()
    first_arrival = trace[0]["arrival"]
    work = sum(q["n"] * (1 + q["steps"]) for q in trace)
    lat = np.array(lat)
    wait = np.array(wait)
    return {
        "workload": trace_workload(count, rate, steps),
        "path": "plain: one request at a time in arrival order, one context (bh_build_tree, "
                "bh_compute_forces, bh_leapfrog_step x %d, bh_get_state)" % steps,
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_max_s": float(lat.max()),
        "queue_wait_p50_s": float(np.percentile(wait, 50)),
        "queue_wait_p99_s": float(np.percentile(wait, 99)),
        "offered_particle_evals_per_s": work / (trace[-1]["arrival"] - first_arrival),
        "served_particle_evals_per_s": work / (t_end - first_arrival),
        "completed": count, "wall_s": t_end,
    }


def bench_small(reps=20, with_oracle=True):
    """The small Plummer workload (N = 4096, seed 1, theta 0.5, eps 0.01): one force
    evaluation plus 10 leapfrog steps of dt 1/128, repeated; beside it the same
    unit in the single-threaded oracle, and the oracle's direct sum."""
    import numpy as np
    import torch

    import paper_1106_1900_amd as bh
    import workloads
    n, theta, eps, dt, steps = 4096, 0.5, 0.01, 1.0 / 128, 10
    pos, vel, mass = workloads.plummer(n, 1)
    dpos = torch.from_numpy(pos).cuda()
    dvel = torch.from_numpy(vel).cuda()
    dmass = torch.from_numpy(mass).cuda()
    ctx = bh.Context()

    def unit():
        ctx.build_tree(dpos, dmass)
        ctx.set_velocities(dvel)
        ctx.compute_forces(theta, eps, want=False)
        for _ in range(steps):
            ctx.leapfrog_step(dt)

    for _ in range(3):
        unit()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        unit()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    ctx.close()
    out = {"workload": "plummer N=4096 seed 1, theta 0.5, eps 0.01, nleaf 16, group 64: one force "
                       "evaluation + 10 leapfrog steps of dt 1/128 (tree rebuilt each step)",
           "value": n * (1 + steps) / el, "unit": "particles/s", "ms_per_unit": 1e3 * el,
           "ms_per_force_evaluation": 1e3 * el / (1 + steps)}
    if with_oracle:
        import oracle
        p, v = pos.copy(), vel.copy()
        t0 = time.perf_counter()
        tree = oracle.Tree(p, mass)
        acc, pot, _, _ = tree.forces(theta, eps)
        for _ in range(steps):
            oracle.kdk_step(p, v, mass, acc, pot, dt, theta, eps)
        t_bh = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.direct(pos, mass, eps)
        t_direct = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n * (1 + steps) / t_bh, "unit": "particles/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "the whole unit (tree, forces, 10 leapfrog steps) in the "
                                         "single-threaded C oracle, %.2f s" % t_bh,
                               "host": host_cpu()}
        out["cpu_direct_sum"] = {"value": n / t_direct, "unit": "particles/s", "cores": 1,
                                 "kind": "oracle",
                                 "sample": "one float64 direct summation over all %d particles, "
                                           "%.2f s" % (n, t_direct)}
    return out


def bench_galaxy(steps, ntarget=16384, cpu_budget=0.0):
    """The three-component galaxy of 4,194,304 particles at theta 0.4, eps 0.02:
    leapfrog steps of dt 1/128 with the walk kernel timed, and the force error of
    the first evaluation against float64 direct summation on seeded targets."""
    import numpy as np
    import torch

    import paper_1106_1900_amd as bh
    import workloads
    log("generating the galaxy")
    pos, vel, mass = workloads.galaxy()
    n = pos.shape[0]
    theta, eps, dt = 0.4, 0.02, 1.0 / 128
    ctx = bh.Context()
    ctx.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda())
    ctx.set_velocities(torch.from_numpy(vel).cuda())
    acc0, _ = ctx.compute_forces(theta, eps)
    acc0 = acc0.cpu().numpy()
    ctx.energy()
    for _ in range(2):
        ctx.leapfrog_step(dt)
    torch.cuda.synchronize()
    s0 = ctx.stats()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.leapfrog_step(dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s1 = ctx.stats()
    e1 = ctx.energy()
    ctx.close()
    launches = s1.walk_kernel_launches - s0.walk_kernel_launches
    walk_ms = (s1.walk_kernel_ms_total - s0.walk_kernel_ms_total) / max(launches, 1)
    pp = (s1.total_npp - s0.total_npp) / max(launches, 1)
    pc = (s1.total_npc - s0.total_npc) / max(launches, 1)
    achieved = (FLOPS_PP * pp + FLOPS_PC * pc) / (walk_ms * 1e-3) / 1e12
    log("direct summation on %d targets" % ntarget)
    out = {
        "workload": "galaxy N=%d (disk 2^20, bulge 2^19, halo 2.5 2^20), theta %g, eps %g, dt 1/128"
                    % (n, theta, eps),
        "value": n * steps / el, "unit": "particles/s", "ms_per_step": 1e3 * el / steps,
        "walk_ms_per_launch": walk_ms, "interactions_per_launch": {"pp": pp, "pc": pc},
        "walk_tflops": achieved, "walk_frac_of_157_3": achieved / PEAK_FP32_VECTOR_TFLOPS,
        "energy_error": float(e1[6]),
        "accuracy_vs_direct": pooled_accuracy([(pos, mass, acc0, eps)], ntarget, 16),
    }
    if cpu_budget > 0:
        log("timing the oracle on the galaxy (%.0f s budget)" % cpu_budget)
        out["cpu_baseline"] = cpu_baseline(pos, mass, theta, eps, cpu_budget)
    return out


SWEEP_FULL = dict(ns=(1 << 15, 1 << 17, 1 << 20), thetas=(0.2, 0.3, 0.4, 0.5, 0.6, 0.75, 0.8),
                  exps=tuple(range(15, 25)), ntarget=256)
SWEEP_COMPACT = dict(ns=(1 << 15, 1 << 17), thetas=(0.4, 0.5, 0.6, 0.75), exps=(15, 17, 19, 21, 23),
                     ntarget=1024)


def bench_sweep(ns, thetas, exps, ntarget):
    """Accuracy and cost against theta at the sizes ns (Plummer, eps 1/64): Δa/a
    against float64 direct summation on ntarget seeded targets, interactions per
    particle, walk time; and one force evaluation (build + walk) against N = 2^e
    for e in exps."""
    import numpy as np
    import torch

    import paper_1106_1900_amd as bh
    import workloads
    rows = []
    for n in ns:
        pos, _, mass = workloads.plummer(n, 2)
        dp, dm = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
        ctx = bh.Context()
        ctx.build_tree(dp, dm)
        for theta in thetas:
            ctx.compute_forces(theta, 1 / 64, want=False)
            acc, _ = ctx.compute_forces(theta, 1 / 64)
            torch.cuda.synchronize()
            st = ctx.stats()
            a = pooled_accuracy([(pos, mass, acc.cpu().numpy(), 1 / 64)], ntarget, 17)
            rows.append({"n": n, "theta": theta, "median": a["median"], "p99": a["p99"],
                         "pp_per_particle": st.sum_npp / n, "pc_per_particle": st.sum_npc / n,
                         "walk_ms": st.ms_walk_kernel})
            log(rows[-1])
        ctx.close()
    scaling = []
    for e in exps:
        n = 1 << e
        pos, _, mass = workloads.plummer(n, 2)
        ctx = bh.Context()
        ctx.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda())
        ctx.compute_forces(0.75, 1 / 64, want=False)
        ctx.leapfrog_step(0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            ctx.leapfrog_step(0.0)       # rebuild and forces at the same positions
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / 5
        st = ctx.stats()
        scaling.append({"n": n, "ms_per_eval": ms, "particles_per_s": n / (ms * 1e-3),
                        "build_ms": st.ms_keys + st.ms_sort + st.ms_move + st.ms_tree + st.ms_moments,
                        "phases_ms": {"keys": st.ms_keys, "sort": st.ms_sort, "move": st.ms_move,
                                      "tree": st.ms_tree, "moments": st.ms_moments,
                                      "walk": st.ms_walk_kernel},
                        "walk_ms": st.ms_walk_kernel})
        log(scaling[-1])
        ctx.close()
    return {"workload": "Plummer seed 2, eps 1/64; accuracy at N in %s, theta in %s (%d seeded "
                        "targets vs float64 direct summation); one force evaluation (rebuild + "
                        "walk, dt = 0 step) at theta 0.75 for N = 2^e, e in %s"
                        % (list(ns), list(thetas), ntarget, list(exps)),
            "accuracy_vs_theta": rows, "scaling_theta_0_75": scaling}


def bench_active(n=1 << 20, theta=0.75, eps=1.0 / 64, reps=5):
    """Between rebuilds (block time-steps): refit against rebuild, and the walk of
    the groups holding active particles against the full walk, Plummer N, the
    active particles drawn uniformly at random."""
    import numpy as np
    import torch

    import paper_1106_1900_amd as bh
    import workloads
    pos, vel, mass = workloads.plummer(n, 2)
    ctx = bh.Context()
    ctx.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda())
    ctx.set_velocities(torch.from_numpy(vel).cuda())
    ctx.compute_forces(theta, eps, want=False)
    ctx.leapfrog_step(0.0)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    out = {"workload": "plummer N=%d theta=%g eps=%g" % (n, theta, eps)}
    out["full_step_ms"] = timed(lambda: ctx.leapfrog_step(0.0))
    out["rebuild_and_forces_ms"] = out["full_step_ms"]

    def refit_forces():
        ctx.drift(0.0)
        ctx.refit()
        ctx.compute_forces(theta, eps, want=False)
    out["refit_and_forces_ms"] = timed(refit_forces)
    ctx.drift(0.0)
    out["refit_ms"] = timed(ctx.refit)
    rows = []
    rng = np.random.default_rng(18)
    for frac in (0.001, 0.01, 0.1, 0.5, 1.0):
        act = torch.from_numpy((rng.uniform(size=n) < frac).astype(np.uint8)).cuda()
        ms = timed(lambda: ctx.compute_forces_active(theta, eps, act, want=False))
        st = ctx.stats()
        rows.append({"active_fraction": frac, "ms": ms, "walk_kernel_ms": st.ms_walk_kernel})
        log(rows[-1])
    out["active_walks"] = rows
    out["full_forces_ms"] = timed(lambda: ctx.compute_forces(theta, eps, want=False))
    ctx.close()
    return out


def bench_mac(n=1 << 20, eps=1.0 / 64, reps=5, ntarget=1024):
    """The two opening tests of Sect. 3.3 at the same theta on the Plummer sphere:
    one force evaluation (rebuild and walk at fixed positions), the walk alone,
    interactions per particle and Δa/a against float64 direct summation on
    seeded targets."""
    import torch

    import paper_1106_1900_amd as bh
    import workloads
    pos, _, mass = workloads.plummer(n, 2)
    rows = []
    for theta in (0.5, 0.75):
        for mac in (bh.MAC_EQ1, bh.MAC_MIN_DIST):
            ctx = bh.Context()
            ctx.set_mac(mac)
            ctx.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda())
            acc, _ = ctx.compute_forces(theta, eps)
            ctx.leapfrog_step(0.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.leapfrog_step(0.0)     # rebuild and forces at the same positions
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / reps
            st = ctx.stats()
            a = accuracy_sample(pos, mass, acc.cpu().numpy(), eps, ntarget)
            rows.append({"theta": theta, "mac": "eq1" if mac == bh.MAC_EQ1 else "min_dist",
                         "ms_per_eval": ms, "particles_per_s": n / (ms * 1e-3),
                         "walk_ms": st.ms_walk_kernel, "pp_per_particle": st.sum_npp / n,
                         "pc_per_particle": st.sum_npc / n, "median": a["median"], "p99": a["p99"]})
            log(rows[-1])
            ctx.close()
    return {"workload": "plummer N=%d eps=%g, %d direct-sum targets" % (n, eps, ntarget),
            "rows": rows}


def bench_block(n=1 << 20, theta=0.75, eps=1.0 / 64, dt_max=1.0 / 16, levels=5, eta=0.01,
                growth=0.1, blocks=6, workload="plummer"):
    """Block time-steps against shared steps on the Plummer sphere: the same
    span of time advanced by block steps of dt_max with up to 2^levels substeps,
    and by leapfrog steps of the finest occupied bin's size (the step a shared
    scheme needs for its most demanding particle); time, rebuilds, force
    evaluations and energy error of each."""
    import numpy as np
    import torch

    import paper_1106_1900_amd as bh
    import workloads
    if workload == "galaxy":
        pos, vel, mass = workloads.galaxy(seed=3)
        n = pos.shape[0]
    else:
        pos, vel, mass = workloads.plummer(n, 2)

    def fresh():
        ctx = bh.Context()
        ctx.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda())
        ctx.set_velocities(torch.from_numpy(vel).cuda())
        ctx.compute_forces(theta, eps, want=False)
        return ctx

    ctx = fresh()
    e0 = ctx.energy()[2]
    _, count = ctx.block_bins(dt_max, eta, eps, levels)
    rows = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(blocks):
        t1 = time.perf_counter()
        st = ctx.block_step(dt_max, eta, eps, levels, growth)
        st["ms"] = 1e3 * (time.perf_counter() - t1)
        rows.append(st)
        log({k: st[k] for k in ("ms", "rebuilt", "updates", "walked_groups", "sync_interactions",
                                "base_interactions")})
    torch.cuda.synchronize()
    block_ms = 1e3 * (time.perf_counter() - t0)
    e_block = ctx.energy()[2]
    ctx.close()

    finest = max(b for b in range(levels + 1) if count[b] > 0)
    ctx = fresh()
    steps = blocks << finest
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.leapfrog_step(dt_max / (1 << finest))
    torch.cuda.synchronize()
    shared_ms = 1e3 * (time.perf_counter() - t0)
    e_shared = ctx.energy()[2]
    ctx.close()
    return {"workload": "%s N=%d theta=%g eps=%g, %d block steps of dt_max=%g with %d levels "
                        "(eta=%g, length=eps, growth=%g) vs %d leapfrog steps of %g"
                        % (workload, n, theta, eps, blocks, dt_max, levels, eta, growth, steps,
                           dt_max / (1 << finest)),
            "bins_at_start": count[:levels + 1],
            "block": {"ms_total": block_ms, "ms_per_block_step": block_ms / blocks,
                      "rebuilds": int(sum(r["rebuilt"] for r in rows)),
                      "particle_updates": int(sum(r["updates"] for r in rows)),
                      "energy_error": (e_block - e0) / e0, "steps": rows},
            "shared": {"ms_total": shared_ms, "ms_per_step": shared_ms / steps,
                       "particle_updates": int(steps * n), "energy_error": (e_shared - e0) / e0},
            "speedup": shared_ms / block_ms}


def bench_merger(t_end=1000.0, dt=1.0 / 64, eps=0.1, thetas=(0.75, 0.5), sample=1.0):
    """The long-run energy test of the paper's merger (Sect. 4.2.2, Table 2) on the
    synthetic two-galaxy encounter of the same particle numbers: shared leapfrog
    steps of dt to t_end (graph replays), energy sampled every `sample` time units;
    dE = (E0 - Et) / E0 at the end and its largest magnitude on the way, the
    black holes' separation, and the wall time."""
    import numpy as np
    import torch

    import paper_1106_1900_amd as bh
    import workloads
    pos, vel, mass = workloads.merger()
    n = pos.shape[0]
    bhs = workloads.black_holes(n)
    per = int(round(sample / dt))
    out = {"workload": "two-galaxy encounter, %d bodies (2 x (1e5 halo + 2e4 stars + 1 black "
                       "hole)), mass ratio 1:3, parabolic orbit d0 = 40, pericentre 4; eps = %g, "
                       "dt = %g, T = %g" % (n, eps, dt, t_end), "runs": []}
    for theta in thetas:
        ctx = bh.Context()
        ctx.batch_build([dict(n=n, theta=theta, eps=eps, dt=dt)], torch.from_numpy(pos).cuda(),
                        torch.from_numpy(mass).cuda(), torch.from_numpy(vel).cuda())
        ctx.batch_forces(want=False)
        ctx.batch_energy()                 # E0
        trace, sep = [], []
        de_max = 0.0
        steps = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = 0
        while steps * dt < t_end - 1e-9:
            ctx.batch_run(per)
            steps += per
            de = float(ctx.batch_energy()[0][6])
            de_max = max(de_max, abs(de))
            k += 1
            if k % 10 == 0:
                x = ctx.get_positions()[0][torch.as_tensor(bhs, device="cuda")].cpu().numpy()
                trace.append([steps * dt, de])
                sep.append([steps * dt, float(np.linalg.norm(x[0] - x[1]))])
            if k % 100 == 0:
                log("theta %g t %.0f dE %.3e dE_max %.3e (%.1f s)"
                    % (theta, steps * dt, de, de_max, time.perf_counter() - t0))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = ctx.stats()
        out["runs"].append({"theta": theta, "steps": steps, "dE_end": de, "dE_max": de_max,
                            "wall_s": wall, "ms_per_step": 1e3 * wall / steps,
                            "particle_steps_per_s": n * steps / wall,
                            "graph_launches": st.graph_launches, "dE_every_10": trace,
                            "black_hole_separation_every_10": sep})
        ctx.close()
    return out


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
    ap.add_argument("--no-small", action="store_true", help="skip the N = 4096 workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched form")
    ap.add_argument("--batch-clusters", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving loop")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the served trace (default: the full 10 s trace)")
    ap.add_argument("--no-fifo", action="store_true",
                    help="skip the plain one-request-at-a-time leg on the served trace")
    ap.add_argument("--no-galaxy", action="store_true", help="skip the 4M galaxy workload")
    ap.add_argument("--no-merger", action="store_true",
                    help="skip the compact long-run energy test (--only merger: the full one)")
    ap.add_argument("--merger-compact-time", type=float, default=125.0,
                    help="end time of the merger run in the default line (N-body units)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the compact accuracy / scaling sweep (--only sweep: the full one)")
    ap.add_argument("--targets", type=int, default=16384,
                    help="seeded targets of the force-error check against direct summation")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-max-resident", type=int, default=1 << 25,
                    help="resident-particle limit of the served run (0: the memory budget only)")
    ap.add_argument("--serve-budget-gib", type=float, default=0.0,
                    help="device memory for the server (0: 60%% of the free memory)")
    ap.add_argument("--serve-small-budget-gib", type=float, default=4.0,
                    help="a second, constrained budget for the same trace (0: skip)")
    ap.add_argument("--only", choices=("batch", "serve", "galaxy", "sweep", "active", "mac", "block",
                                       "merger"),
                    help="run only that form and print its JSON (for profiling runs)")
    ap.add_argument("--merger-time", type=float, default=1000.0,
                    help="end time of the merger run (N-body units)")
    ap.add_argument("--cpu-worker", nargs=6, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-cores", type=int, default=0,
                    help="processes of the all-cores oracle baseline (0: min(16, cpus); -1: skip)")
    args = ap.parse_args()
    if args.cpu_worker:
        i, w, n, th, ep, b = args.cpu_worker
        cpu_worker(int(i), int(w), int(n), float(th), float(ep), float(b))
        return

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import numpy as np
    import torch

    import paper_1106_1900_amd as bh
    import workloads

    if args.calib_copy:
        calib_copy()
    if args.only == "batch":
        print(json.dumps(bench_batch(args.batch_clusters, args.batch_steps, 2, alone=False)), flush=True)
        return
    if args.only == "active":
        print(json.dumps(bench_active()), flush=True)
        return
    if args.only == "sweep":
        print(json.dumps(bench_sweep(**SWEEP_FULL)), flush=True)
        return
    if args.only == "mac":
        print(json.dumps(bench_mac()), flush=True)
        return
    if args.only == "merger":
        print(json.dumps(bench_merger(t_end=args.merger_time)), flush=True)
        return
    if args.only == "block":
        print(json.dumps(bench_block()), flush=True)
        for growth in (0.1, 0.0):
            print(json.dumps(bench_block(theta=0.4, eps=0.02, dt_max=1.0 / 16, levels=6, eta=0.01,
                                         growth=growth, blocks=3, workload="galaxy")), flush=True)
        return
    if args.only == "galaxy":
        print(json.dumps(bench_galaxy(args.steps if args.steps != 100 else 10, ntarget=args.targets,
                                      cpu_budget=args.cpu_budget)), flush=True)
        return
    if args.only == "serve":
        budget = int(args.serve_budget_gib * (1 << 30)) or int(0.6 * torch.cuda.mem_get_info()[0])
        print(json.dumps(bench_serve(args.serve_requests, args.serve_rate, budget,
                                     max_resident=args.serve_max_resident)), flush=True)
        if not args.no_fifo:
            print(json.dumps(bench_fifo(args.serve_requests, args.serve_rate)), flush=True)
        return

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
    # one event between consecutive steps on the context's stream (the current
    # stream at its creation) for the per-step distribution
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # each step computes the energy sums on the device; they are read back once
    # at the end
    evs[0].record()
    for i in range(args.steps):
        ctx.leapfrog_step(args.dt)
        evs[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    s1 = ctx.stats()
    e1 = ctx.energy()
    # the same steps replayed from a captured graph (no per-kernel host launches)
    gsteps = min(args.steps, 20)
    ctx.batch_run(1)
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    ctx.batch_run(gsteps)
    torch.cuda.synchronize()
    graph_ms = 1e3 * (time.perf_counter() - tg0) / gsteps

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
        "step_ms_p10_p50_p90": [float(np.percentile(step_ms, q)) for q in (10, 50, 90)],
        "graph_replay_ms_per_step": graph_ms,
        "energy_error_over_timed_steps": float((e0[2] - e1[2]) / e0[2]),
        "tree": {"ncells": s1.ncells, "ngroups": s1.ngroups, "depth": s1.depth},
        "paper_reference": {"value": PAPER_TRAVERSE_RATE, "unit": "particles/s",
                            "what": "tree traverse only, 1x GTX480, N=2^20 Plummer, theta=0.75"},
    }
    ctx.close()
    if not args.no_small:
        log("small workload (N = 4096)")
        out["small"] = bench_small(with_oracle=args.cpu_budget > 0 and rank == 0)
    if not args.no_batch:
        out["batch"] = bench_batch(args.batch_clusters, args.batch_steps, 2)
    if not args.no_serve:
        budget = int(args.serve_budget_gib * (1 << 30))
        if budget <= 0:
            budget = int(0.6 * torch.cuda.mem_get_info()[0])
        log("serving %d requests" % args.serve_requests)
        out["served"] = bench_serve(args.serve_requests, args.serve_rate, budget,
                                    max_resident=args.serve_max_resident)
        # the same trace under a budget that makes requests wait for admission
        small = int(args.serve_small_budget_gib * (1 << 30))
        if small > 0:
            log("serving %d requests in %.1f GiB" % (args.serve_requests, args.serve_small_budget_gib))
            out["served_constrained"] = bench_serve(args.serve_requests, args.serve_rate, small)
        if not args.no_fifo:
            log("the same %d requests one at a time (plain path)" % args.serve_requests)
            out["served_plain_fifo"] = bench_fifo(args.serve_requests, args.serve_rate)
        _REQUEST_POOLS.clear()
    if not args.no_sweep:
        log("compact accuracy and scaling sweep")
        out["sweep"] = bench_sweep(**SWEEP_COMPACT)
    if not args.no_galaxy:
        out["galaxy"] = bench_galaxy(10, ntarget=args.targets,
                                     cpu_budget=min(10.0, args.cpu_budget) if rank == 0 else 0.0)
    if not args.no_merger:
        log("merger energy test to t = %g" % args.merger_compact_time)
        out["merger"] = bench_merger(t_end=args.merger_compact_time)
    if not args.no_accuracy:
        log("direct summation on %d targets" % args.targets)
        out["accuracy_vs_direct"] = accuracy_sample(pos, mass, acc0_h, args.eps, args.targets)
    if args.cpu_budget > 0 and rank == 0:
        log("timing the oracle on the host (%.0f s budget)" % args.cpu_budget)
        out["cpu_baseline"] = cpu_baseline(pos, mass, args.theta, args.eps, args.cpu_budget)
        cores = args.cpu_cores if args.cpu_cores > 0 else min(16, os.cpu_count() or 1)
        if args.cpu_cores >= 0 and cores > 1:
            log("timing the oracle on %d host cores" % cores)
            out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(
                n, args.theta, args.eps, min(10.0, args.cpu_budget), cores)
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
