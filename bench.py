#!/usr/bin/env python3
"""Throughput benchmark of the PHIA sweep on one MI355X.

Workload (default): max-cut on a synthetic Erdos-Renyi graph G(800, 0.06)
with unit weights (J = -1 on edges, h = 0, int8 couplings), 1024 replicas x
10^4 HMC steps, linear inverse-temperature schedule, int8 MFMA quasi-gradient.
One benchmark step is one complete anneal of that workload: draw of the
initial positions, 10^4 sweep steps over all replicas (momentum refresh,
drift, readout, J.s + h, exact energy, records, kick), and the final argmin.

Prints one JSON line: spin-updates/s over the timed steps, the sweep
kernel's roofline position (HIP events on the library's stream), time to
target at 99% success (Eq. 9) against the best energy of a 10x longer run,
and the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import csv
import glob
import hashlib
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks and unit counts (per GPU).
CUS, CLOCK_HZ = 256, 2.4e9
VALU_OPS_PEAK = CUS * 64 * CLOCK_HZ          # 64 FP32/INT32 lanes per CU per clock
INT8_MFMA_PEAK = 5.0e15                      # dense int8 ops/s
BF16_MFMA_PEAK = 2.5e15
FP4_MFMA_PEAK = 10.1e15
# Arithmetic operations of one spin-update, the fixed yardstick of every
# roofline fraction here (TANH mode): drift 1, readout 1, field add 1, energy
# term 3, kick 27 (gamma x, 2|u|, e^y 17, sech^2 assembly 3 with the
# reciprocal counted once, c*d, int->float, two fma), as the sweep
# specification was first written.  Later sequences compute the same
# quantities with fewer instructions (the sech^2 now takes 24); the count is
# kept so that fractions stay comparable.  The 16-column MFMA output is
# exactly the field.
OPS_PER_SPIN_UPDATE = 33
# POLY2 mode: the kick is gamma x, u*u, one fma, max, c*d, int->float and two
# fma (8 instead of 27).
OPS_PER_SPIN_UPDATE_POLY2 = 14

WORKLOADS = {
    # name: (generator, kwargs, R, T, schedule)
    "maxcut800": dict(gen="er_maxcut", args=dict(N=800, p=0.06, seed=0), R=1024, T=10000,
                      sched=dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25),
                      desc="maxcut ER G(800,0.06) w=+1 (J=-1), h=0, 1024 replicas x 1e4 steps"),
    "sk16": dict(gen="sk_pm1", args=dict(N=16, seed=0), R=64, T=1000,
                 sched=dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=50),
                 desc="SK N=16 J=+-1, h=0, 64 replicas x 1000 steps"),
    "batch4096": dict(gen="batch", args=dict(count=4096, nmin=32, nmax=512, seed=0), R=32, T=5000,
                      sched=dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25),
                      desc="batch of 4096 instances, N uniform in [32,512], even ids SK +-1 (h=0), odd ids random "
                           "3-regular +-1 with h in {-1,0,1}; 32 replicas x 5000 steps each, one graph launch"),
    "serve": dict(gen="serve", args=dict(rate=200.0, nmin=100, nmax=4000, seed=0), R=64, T=20000,
                  sched=dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25),
                  desc="serving: Poisson arrivals at 200 req/s, planted frustrated-loop instances (a pool of 120), "
                       "N log-uniform in [100,4000], half dense / half sparse, each served as integers, as J 3/16 "
                       "(2^-4 grid, int8) and as J 129/256 (2^-8 grid, BF16 hi/lo); 64 replicas, stop at the "
                       "planted energy or 2e4 steps; beta divided by the coupling scale"),
    "tts_sweep": dict(gen="tts_sweep", args=dict(sizes=(8, 16, 32, 64, 128, 256, 512, 1024), seed=0), R=256,
                      T=1000, sched=dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25),
                      desc="time to target versus N for the Table 2 families (maxcut_dense, maxcut_d3, sk_bool, "
                           "sk_ising, sk_uniform, nae_3_sat, spin_model; fractional ones on the 2^-6 grid); 10 "
                           "instances per point, 256 replicas x max(1000, 10 N) steps per run; target: the planted "
                           "energy (nae_3_sat), the exhaustive ground state for N <= 20, else the best energy of a "
                           "20x longer run; median TTS over the instances"),
    "maxcut256": dict(gen="er_maxcut", args=dict(N=256, p=0.06, seed=0, signed=True), R=4, T=10000,
                      sched=dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25),
                      desc="maxcut ER G(256,0.06) w=+-1, h=0, few replicas (default 4) x 1e4 steps"),
    "reg3_4000": dict(gen="regular3_pm1", args=dict(N=4000, seed=0), R=64, T=10000, path="auto",
                      sched=dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25),
                      desc="random 3-regular N=4000 J=+-1, h in {-1,0,1}, 64 replicas x 1e4 steps"),
    "sk2000": dict(gen="sk_gauss_fixed", args=dict(N=2000, seed=0, frac_bits=5, bits=8), R=512, T=20000,
                   sched=dict(eps=0.2, gamma=1.0, beta0=0.02, beta1=0.6, refresh_L=25),
                   desc="SK N=2000 J~N(0,1) 8-bit fixed point (2^-5), h in [-1,1], 512 replicas x 2e4 steps"),
    "sk2000_16bit": dict(gen="sk_gauss_fixed", args=dict(N=2000, seed=0, frac_bits=12, bits=16), R=512, T=20000,
                         path="bf16hilo",
                         sched=dict(eps=0.2, gamma=1.0, beta0=0.02, beta1=0.6, refresh_L=25),
                         desc="SK N=2000 J~N(0,1) 16-bit fixed point (2^-12, BF16 hi/lo planes both non-zero), "
                              "h in [-1,1], 512 replicas x 2e4 steps"),
}


CSRC = os.path.join(ROOT, "paper_2407_10205_amd", "csrc")
# sources whose hash identifies each profiled kernel's code
KERNEL_SRCS = {"k_batch_fp4": ["phia_batch_kernel.hip", "phia_devsweep.h", "phia_devmath.h"],
               "k_sweep_valu": ["phia_valu_kernel.hip", "phia_devsweep.h", "phia_devmath.h"]}
DEFAULT_SRCS = ["phia_kernels.hip", "phia_devsweep.h", "phia_devmath.h"]
PROFILES = os.path.join(ROOT, "profiles")
COPY_BYTES = 256 << 20  # plain device copy used to calibrate the byte counters


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha(kernel=None):
    h = hashlib.sha256()
    for name in KERNEL_SRCS.get(kernel, DEFAULT_SRCS):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_file(kernel, workload_name):
    return os.path.join(PROFILES, f"{kernel}_{workload_name}_traffic.json")


def recorded_traffic(kernel, workload_name, workload, geometry):
    """HBM bytes per sweep launch from the committed counter summary, or None
    when the kernel source or the launch geometry changed since it was taken."""
    try:
        with open(traffic_file(kernel, workload_name)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha(kernel) or t.get("workload") != workload or t.get("geometry") != geometry:
        return None
    return t.get("bytes_per_launch")


def calibrate_copy():
    """A plain device copy of COPY_BYTES (reads and writes that many bytes)."""
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


def _rows(pattern):
    out = []
    for path in glob.glob(pattern, recursive=True):
        with open(path, newline="") as f:
            out.extend(csv.DictReader(f))
    return out


def summarize_profiles(root, workload, kernel="k_sweep"):
    """Turn rocprofv3 outputs under root (stats/, fetch/, write/) into the
    traffic summary: per-dispatch FETCH_SIZE and WRITE_SIZE of the sweep
    kernel, each scaled by the same counter on the calibration copy."""
    stats = _rows(os.path.join(root, "stats", "**", "*kernel_stats.csv"))
    res = {"workload": workload, "kernel": kernel, "kernel_sha": kernel_sha(kernel if kernel in KERNEL_SRCS else None),
           "copy_bytes": COPY_BYTES}
    sweeps = [row for row in stats if kernel in row.get("Name", "")]
    if sweeps:
        top = max(sweeps, key=lambda r: float(r.get("TotalDurationNs", 0)))
        res["kernel_stats"] = {k: top[k] for k in ("Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage")
                               if k in top}
    counters = {}
    for which in ("fetch", "write"):
        rows = _rows(os.path.join(root, which, "**", "*counter_collection.csv"))
        sweep, copy = [], []
        for row in rows:
            name = row.get("Kernel_Name", row.get("Kernel-Name", ""))
            val = float(row.get("Counter_Value", row.get("Counter-Value", "nan")))
            if kernel in name:
                sweep.append(val)
            elif "copy" in name.lower() or "elementwise" in name.lower():
                copy.append(val)
        if sweep and copy:
            kib_per_byte = max(copy) / COPY_BYTES  # counter units per byte moved by the copy
            counters[which] = {"sweep_counter_per_dispatch": sum(sweep) / len(sweep),
                               "copy_counter_per_dispatch": max(copy),
                               "bytes_per_launch": (sum(sweep) / len(sweep)) / kib_per_byte}
    res["counters"] = counters
    if "fetch" in counters and "write" in counters:
        res["bytes_per_launch"] = counters["fetch"]["bytes_per_launch"] + counters["write"]["bytes_per_launch"]
    return res


def make_instance(w):
    from paper_2407_10205_amd import instances as inst
    return getattr(inst, w["gen"])(**w["args"])


def make_batch(count, nmin, nmax, seed):
    """Instances of the batch workload (sizes drawn from one seeded stream)."""
    import numpy as np
    from paper_2407_10205_amd import instances as inst
    g = inst.rng(seed)
    sizes = g.integers(nmin, nmax + 1, size=count)
    out = []
    for i, n in enumerate(sizes):
        n = int(n)
        if i % 2 == 0:
            out.append(inst.sk_pm1(n, 10_000 + i))
        else:
            out.append(inst.regular3_pm1(n + (n % 2), 10_000 + i))
    return out


# Precision variants of a served instance: (multiplier of the integer
# couplings, fraction bits).  Positive scaling keeps the planted ground state;
# 3/16 stays within int8 on the 2^-4 grid, 129/256 needs 16 bits (BF16 hi/lo).
SERVE_VARIANTS = ((1, 0), (3, 4), (129, 8))


def make_requests(count, rate, nmin, nmax, seed, pool=120):
    """Arrival times and planted instances of the serving workload.  `pool`
    distinct planted instances (sizes log-uniform, dense and sparse
    alternating) are served in every precision variant; request i takes pool
    entry i mod pool, variant (i // pool) mod 3 and its own seed."""
    import numpy as np
    from paper_2407_10205_amd import instances as inst
    g = inst.rng(seed)
    gaps = g.exponential(1.0 / rate, size=count)
    arrive = np.cumsum(gaps)
    npool = min(pool, count)
    sizes = np.rint(np.exp(g.uniform(np.log(nmin), np.log(nmax), size=npool))).astype(int)
    base = []
    for k in range(npool):
        J, h, E, t = inst.planted_loops(int(sizes[k]), 20_000 + k, alpha=0.4, dense=(k % 2 == 1))
        base.append((J, h, E, k % 2 == 1))
    reqs = []
    for i in range(count):
        J, h, E, dense = base[i % npool]
        mult, f = SERVE_VARIANTS[(i // npool) % len(SERVE_VARIANTS)]
        if mult > 127 and dense and J.shape[0] > 2496:
            mult, f = SERVE_VARIANTS[1]  # BF16 hi/lo holds N <= 2496 (sparse ones take ELL)
        reqs.append(dict(arrive=float(arrive[i]), J0=J, h=h, target=E * mult, frac_bits=f,
                         scale=mult / 2.0 ** f, N=J.shape[0], dense=dense, pool=i % npool, seed=17 + i))
    return reqs


def run_serve_bench(args, w):
    """Latency and throughput of the continuous-batching server.  Problems
    defer their coupling upload to admission, so the server's memory budget
    bounds everything the requests hold on the device."""
    import numpy as np
    from paper_2407_10205_amd import phia
    t = time.perf_counter()
    reqs = make_requests(args.requests, **w["args"])
    probs = [phia.Problem(r["J0"] * r["scale"], r["h"], frac_bits=r["frac_bits"], path="auto", defer_upload=True)
             for r in reqs]
    paths = [p.info()["path_name"] for p in probs]
    log(f"prepared {len(reqs)} requests in {time.perf_counter() - t:.1f} s")
    R, T, s = w["R"], w["T"], w["sched"]
    budget = int(args.serve_budget_gib * (1 << 30))
    srv = phia.Server(budget, max_slots=args.slots, chunk_steps=args.chunk)
    tickets = []
    t0 = time.perf_counter()
    for r, p in zip(reqs, probs):
        delay = r["arrive"] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        # beta divided by the couplings' scale: every variant of an instance
        # then anneals the same real-valued dynamics, so success probabilities
        # are matched across the mix
        sr = dict(s, beta0=s["beta0"] / r["scale"], beta1=s["beta1"] / r["scale"])
        tickets.append(srv.submit(p, R, T, r["target"], seed=r["seed"], **sr))
    res = [srv.wait(tk) for tk in tickets]
    srv.close()
    for p in probs:
        p.close()
    lat = np.array([x["t_done"] - x["t_arrive"] for x in res])
    su = float(sum(R * r["N"] * x["steps_used"] for r, x in zip(reqs, res)))
    span = max(x["t_done"] for x in res) - min(x["t_arrive"] for x in res)
    ok = np.array([x["success"] for x in res], bool)
    achieved = su * OPS_PER_SPIN_UPDATE / span
    by_path = {pa: int(sum(1 for q in paths if q == pa)) for pa in sorted(set(paths))}
    cpu = None
    if not args.no_cpu:
        # the oracle on every 10th pool instance, each variant's integer form
        sample = [(reqs[k]["J0"], reqs[k]["h"]) for k in range(0, min(len(reqs), 120), 10)]
        cpu = cpu_baseline_instances(sample, R, T, s, args.cpu_seconds, "serving pool")
    out = {"metric": "spin-updates/s", "value": su / span, "unit": "spin-updates/s", "n_gpus": 1,
           "steps": len(reqs), "warmup": 0, "ms_per_step": 1000 * span / len(reqs), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "mixed (i8, bf16 hi/lo, ell)", "data": "synthetic",
           "config": {"workload": w["desc"], "requests": len(reqs), "replicas": R, "max_steps": T,
                      "slots": args.slots, "chunk_steps": args.chunk, "offered_rate_per_s": w["args"]["rate"],
                      "budget_bytes": budget, "paths": by_path, "variants": [list(v) for v in SERVE_VARIANTS]},
           "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
           "latency_p50_success_s": float(np.percentile(lat[ok], 50)) if ok.any() else None,
           "latency_p99_success_s": float(np.percentile(lat[ok], 99)) if ok.any() else None,
           "success_rate": float(ok.mean()),
           "success_rate_by_variant": [float(ok[[k for k in range(len(reqs)) if reqs[k]["frac_bits"] == f]].mean())
                                       for _, f in SERVE_VARIANTS],
           "mean_steps_used": float(np.mean([x["steps_used"] for x in res])),
           "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_OPS_PEAK, "unit": "ops/s",
                        "frac": achieved / VALU_OPS_PEAK, "traffic": None,
                        "kernel": "whole server (batched small, column-split and VALU sweeps)",
                        "ops_per_spin_update": OPS_PER_SPIN_UPDATE,
                        "note": "spin-updates of all requests x 33 over the wall-clock span from the first arrival "
                                "to the last completion (idle gaps between arrivals included)"},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def run_batch_bench(args, w):
    """Throughput of the batched sweep: one step = one anneal of the whole
    batch.  The batch plan (replica state, work tables, the instantiated
    graph) is built once, untimed; every step launches it with new seeds, and
    HIP events on its stream time the launches."""
    import numpy as np
    import torch
    from paper_2407_10205_amd import phia
    t = time.perf_counter()
    insts = make_batch(**w["args"])
    log(f"generated {len(insts)} instances in {time.perf_counter() - t:.1f} s")
    stream = torch.cuda.Stream()
    probs = [phia.Problem(J, h, path="i8", stream=stream.cuda_stream) for J, h in insts]
    n = len(probs)
    R, T, s = w["R"], w["T"], w["sched"]
    su = float(sum(p.N for p in probs)) * R * T
    t = time.perf_counter()
    plan = phia.Batch(probs, [R] * n, [T] * n, [s] * n)
    log(f"batch plan built in {time.perf_counter() - t:.1f} s")
    kinds = [p.info()["sweep_kernel"] for p in probs]

    for i in range(args.warmup):
        plan.launch([900_000 * (i + 1) + j for j in range(n)])
        plan.sync()
    torch.cuda.synchronize()
    events = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.launch([1_000_000 * (i + 1) + j for j in range(n)])
        e1.record(stream)
        events.append((e0, e1))
    plan.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = su * args.steps / wall
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    best = [p.best_exact()[0] for p in probs[:4]]
    # explicit teardown while the runtime and the stream are alive
    plan.close()
    for p in probs:
        p.close()
    torch.cuda.synchronize()
    if args.calibrate_copy:
        calibrate_copy()
    achieved = su * OPS_PER_SPIN_UPDATE / (kern_ms / 1000)
    kernel = "k_batch_fp4" if all(k == 3 for k in kinds) else "k_batch_fp4 + k_sweep_mfma (batch)"
    cpu = None
    if not args.no_cpu:
        stride = max(1, n // 256)
        sample = insts[::stride + 1] if stride > 1 else insts
        cpu = cpu_baseline_instances(sample, R, T, s, args.cpu_seconds,
                                     f"instances 0, {stride + 1}, {2 * (stride + 1)}, ... of the batch")
    out = {"metric": "spin-updates/s", "value": value, "unit": "spin-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1000 * wall / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "fp8xfp4" if kernel == "k_batch_fp4" else "i8",
           "data": "synthetic",
           "config": {"workload": w["desc"], "instances": n, "replicas": R, "hmc_steps": T, "path": "i8",
                      "operands": "FP8 spins x FP4 couplings (exact for integer couplings in the FP4 set)",
                      "schedule": s, "spin_updates_per_step": su, "sweep_kernel": kernel},
           "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_OPS_PEAK, "unit": "ops/s",
                        "frac": achieved / VALU_OPS_PEAK,
                        "traffic": recorded_traffic("k_batch_fp4", "batch4096", w["desc"], None),
                        "kernel": kernel, "kernel_ms": kern_ms, "ops_per_spin_update": OPS_PER_SPIN_UPDATE},
           "cpu_baseline": cpu, "best_energy_first4": [int(b) for b in best]}
    print(json.dumps(out), flush=True)


def tts99(t_run, p_hat, R):
    """Eq. 9 with the success probability of one launch of R replicas."""
    P = 1.0 - (1.0 - p_hat) ** R if p_hat > 0 else 0.0
    if P >= 0.99:
        return t_run
    if P <= 0:
        return float("inf")
    return t_run * math.log(0.01) / math.log(1.0 - P)


def ground_energy_exhaustive(Ji, hi):
    """Minimum over all 2^N spin states of Eq. 2 in integer units (N <= 20),
    enumerated in chunks with numpy."""
    import numpy as np
    N = Ji.shape[0]
    J64, h64 = Ji.astype(np.int64), hi.astype(np.int64)
    best = None
    chunk = 1 << min(N, 14)
    bits = np.arange(N, dtype=np.int64)
    for start in range(0, 1 << N, chunk):
        idx = np.arange(start, min(start + chunk, 1 << N), dtype=np.int64)
        S = 1 - 2 * ((idx[:, None] >> bits[None, :]) & 1)       # rows of +-1
        E2 = -(np.einsum("ri,ij,rj->r", S, J64, S)) - 2 * (S @ h64)  # 2 E (i<j sum counted twice)
        m = int(E2.min()) // 2
        best = m if best is None else min(best, m)
    return best


def run_tts_sweep(args, w):
    """Time to target of one anneal (R replicas in parallel) for each Table 2
    family and size, over several instances per point (the median TTS over
    the instances, as Sec. 3.2 reports per problem type).  One JSON line
    with every point."""
    import numpy as np
    import torch
    from paper_2407_10205_amd import instances as inst, phia

    R, s = w["R"], w["sched"]
    stream = torch.cuda.Stream()
    points = []
    t_all = time.perf_counter()
    sizes = w["args"]["sizes"] if not args.tts_sizes else tuple(int(t) for t in args.tts_sizes.split(","))
    for fam in inst.TABLE2_FAMILIES:
        for n in sizes:
            N = n + (n % 2 if fam == "maxcut_d3" else 0)
            T = max(w["T"], 10 * N)
            per = []
            for k in range(args.tts_instances):
                seed = w["args"]["seed"] + 1000 * k + n
                if fam == "nae_3_sat":
                    J, h, M, _, _ = inst.nae_3_sat(N, seed)
                else:
                    J, h = inst.table2_family(fam, N, seed)
                prob = phia.Problem(J, h, stream=stream.cuda_stream)
                f = prob.info()["frac_bits"]
                if fam == "nae_3_sat":
                    target, how = -M, "planted (every clause NAE-satisfied)"
                elif N <= 20:
                    Ji = np.rint(J * 2 ** f).astype(np.int32)
                    hi = np.rint(h * 2 ** f).astype(np.int32)
                    target, how = ground_energy_exhaustive(Ji, hi), "exhaustive"
                else:
                    prob.anneal(R, 20 * T, s["eps"], s["gamma"], beta0=s["beta0"], beta1=s["beta1"],
                                refresh_L=s["refresh_L"], seed=777)
                    target, how = int(prob.best_exact()[0]), "best of a 20x longer run"
                if k == 0:  # warm-up of this shape
                    prob.anneal(R, T, s["eps"], s["gamma"], beta0=s["beta0"], beta1=s["beta1"],
                                refresh_L=s["refresh_L"], seed=1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                prob.anneal(R, T, s["eps"], s["gamma"], beta0=s["beta0"], beta1=s["beta1"],
                            refresh_L=s["refresh_L"], seed=100 + k)
                E, _, _ = prob.replica_best()
                t_run = time.perf_counter() - t0
                info = prob.info()
                prob.close()
                p_hat = float(np.mean(E <= target))
                per.append(dict(t_run=t_run, p=p_hat, tts=tts99(t_run, p_hat, R)))
            tts = [q["tts"] for q in per]
            pt = {"family": fam, "N": N, "steps": T, "instances": len(per), "path": info["path_name"],
                  "frac_bits": f, "sweep_kernel": info["sweep_kernel"], "group": info["group"], "target": how,
                  "tts99_median_s": float(np.median(tts)), "solved_instances": int(sum(q["p"] > 0 for q in per)),
                  "replica_success_mean": float(np.mean([q["p"] for q in per])),
                  "t_run_median_s": float(np.median([q["t_run"] for q in per]))}
            points.append(pt)
            log(json.dumps(pt))
    out = {"metric": "tts99_s", "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
           "config": {"workload": w["desc"], "replicas": R, "schedule": s, "instances_per_point": args.tts_instances},
           "points": points, "wall_s": time.perf_counter() - t_all}
    print(json.dumps(out), flush=True)


def host_cpu():
    """Host CPU as the CPU-baseline leg reports it: model name, logical CPUs,
    CPUs this process may run on, and the threads the oracle uses (the
    OpenMP thread count when the environment sets one, else every allowed
    CPU)."""
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    allowed = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = allowed
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        threads = min(allowed, int(env))
    return {"model": model, "nproc": os.cpu_count() or 1, "allowed": allowed, "threads": max(1, threads)}


_ORACLE_NATIVE = None


def oracle_for_host():
    """The oracle, compiled for this host's CPU (-O3 -march=native) into a
    temporary directory; the in-tree portable build if that fails."""
    global _ORACLE_NATIVE
    from oracle import build as obuild, oracle as O
    if _ORACLE_NATIVE is None:
        import tempfile
        try:
            d = tempfile.mkdtemp(prefix="phia_oracle_")
            _ORACLE_NATIVE = obuild.build(native=True, out=os.path.join(d, "liboracle_native.so"))
        except Exception as e:  # noqa: BLE001 - fall back to the portable in-tree build
            log(f"native oracle build failed ({e}); timing the in-tree build")
            _ORACLE_NATIVE = ""
    if _ORACLE_NATIVE:
        O.use_library(_ORACLE_NATIVE)
    return O, ("-O3 -march=native" if _ORACLE_NATIVE else "-O3 -march=x86-64-v3")


def grid_units(J, h):
    import numpy as np
    f = 0
    while not np.all(np.rint(J * 2**f) == J * 2**f) or not np.all(np.rint(h * 2**f) == h * 2**f):
        f += 1
    return f, np.rint(J * 2**f).astype(np.int32), np.rint(h * 2**f).astype(np.int32)


def cpu_baseline(J, h, w, budget_s, deriv="tanh", mh=None):
    """Time the oracle on a bounded replica/step sample of the workload."""
    O, flags = oracle_for_host()
    f, Ji, hi = grid_units(J, h)
    N, T = J.shape[0], w["T"]
    s = w["sched"]
    betas = O.beta_linear(s["beta0"], s["beta1"], T)
    cpu = host_cpu()
    threads = cpu["threads"]
    # calibrate one replica on a few steps, then size the sample to the budget
    t = time.perf_counter()
    O.anneal(Ji, hi, f, 1, betas, s["eps"], s["gamma"], s["refresh_L"], 7, k1=20, threads=1, deriv=deriv, mh=mh)
    per_step = (time.perf_counter() - t) / 20
    steps = int(max(20, min(T, budget_s / max(per_step, 1e-9))))
    # more replicas (groups of `threads`, up to the workload's) until the
    # sample fills the budget
    R = min(max(w["R"], threads), threads * max(1, int(budget_s / max(steps * per_step, 1e-9))))
    t = time.perf_counter()
    O.anneal(Ji, hi, f, R, betas, s["eps"], s["gamma"], s["refresh_L"], 7, k1=steps, threads=threads, deriv=deriv,
             mh=mh)
    dt = time.perf_counter() - t
    # a fifth of the budget on one thread
    steps1 = int(max(20, min(T, budget_s / 5 / max(per_step, 1e-9))))
    R1 = max(1, min(w["R"], int(budget_s / 5 / max(steps1 * per_step, 1e-9))))
    t = time.perf_counter()
    O.anneal(Ji, hi, f, R1, betas, s["eps"], s["gamma"], s["refresh_L"], 7, k1=steps1, threads=1, deriv=deriv, mh=mh)
    dt1 = time.perf_counter() - t
    return {"value": R * N * steps / dt, "unit": "spin-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"replicas 0..{R - 1}, steps 0..{steps - 1} of the same schedule, {dt:.1f} s; oracle {flags}, "
                      f"OpenMP over replicas",
            "single_thread": {"value": R1 * N * steps1 / dt1, "unit": "spin-updates/s",
                              "sample": f"replicas 0..{R1 - 1}, steps 0..{steps1 - 1}, one thread, {dt1:.1f} s"},
            "cpu_model": cpu["model"], "nproc": cpu["nproc"], "cpus_allowed": cpu["allowed"]}


def cpu_baseline_instances(insts, R, T, sched, budget_s, what):
    """Oracle timing on a subset of a workload's instances: every sampled
    instance runs `threads` replicas (OpenMP over replicas; more, up to R,
    when the whole schedule fits) for the same number of steps of its
    schedule, sized so that the sample takes about budget_s.  Spin-updates/s
    of the sample = sum N x replicas x steps / time.  A shorter run of one
    replica per instance on one thread gives the single-thread rate."""
    O, flags = oracle_for_host()
    cpu = host_cpu()
    threads = cpu["threads"]
    units = [grid_units(J, h) for J, h in insts]
    betas = O.beta_linear(sched["beta0"], sched["beta1"], T)
    total_n = sum(u[1].shape[0] for u in units)

    def run_all(k, reps, nthr):
        t = time.perf_counter()
        for f, Ji, hi in units:
            O.anneal(Ji, hi, f, reps, betas, sched["eps"], sched["gamma"], sched["refresh_L"], 7, k1=k,
                     threads=nthr)
        return time.perf_counter() - t

    def sample(reps, nthr, budget):
        # calibrate on the whole sample at two step counts (each call also has a fixed cost:
        # set-up, initial kick, thread start), then size the run to the budget: steps first,
        # then, when the whole schedule fits, more replicas (multiples of `reps`, at most R)
        calib = 16
        t1 = run_all(calib, reps, nthr)
        t2 = run_all(16 * calib, reps, nthr)
        per_step = max((t2 - t1) / (15 * calib), 1e-12)
        fixed = max(t1 - calib * per_step, 0.0)
        steps = int(max(calib, min(T, (budget - fixed) / per_step)))
        if steps >= T:
            reps = max(reps, min(max(R, reps), reps * int(round((budget - fixed) / (T * per_step)))))
        dt = run_all(steps, reps, nthr)
        return total_n * reps * steps / dt, reps, steps, dt

    value, reps, steps, dt = sample(threads, threads, budget_s)
    v1, reps1, steps1, dt1 = sample(1, 1, budget_s / 5)
    return {"value": value, "unit": "spin-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{what}: {len(units)} instances (sum N = {total_n}), replicas 0..{reps - 1}, "
                      f"steps 0..{steps - 1} of each schedule, {dt:.1f} s; oracle {flags}, OpenMP over replicas",
            "single_thread": {"value": v1, "unit": "spin-updates/s",
                              "sample": f"the same instances, replicas 0..{reps1 - 1}, steps 0..{steps1 - 1}, "
                                        f"one thread, {dt1:.1f} s"},
            "cpu_model": cpu["model"], "nproc": cpu["nproc"], "cpus_allowed": cpu["allowed"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed complete anneals")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch4096", choices=sorted(WORKLOADS))
    ap.add_argument("--replicas", type=int, default=None, help="replica count (default: the workload's)")
    ap.add_argument("--path", default=None, choices=["i8", "bf16hilo", "fp32", "ell", "auto"],
                    help="coupling path (default: the workload's, int8 unless stated)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tts", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the geometry autotuner")
    ap.add_argument("--no-int8-check", action="store_true",
                    help="skip the int8-operand timing that accompanies an FP4-operand run")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (byte-counter calibration)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="summarise rocprofv3 outputs in DIR/{stats,fetch,write} and exit")
    ap.add_argument("--profile-kernel", default=None,
                    help="kernel name (substring) the summary covers (default: the workload's sweep kernel)")
    ap.add_argument("--geometry-out", metavar="FILE", help="write the launch geometry used to FILE")
    ap.add_argument("--deriv", default="tanh", choices=["tanh", "poly2"],
                    help="derivative factor of the kick: sech^2 (Eq. 8) or the FPGA's quadratic (POLY2 mode)")
    ap.add_argument("--mh", metavar="UP,DOWN", default=None,
                    help="accept or reject every trajectory of refresh_L steps (App. A, Table 3 state 4) and "
                         "multiply beta by UP after an acceptance, DOWN after a rejection (1,1: fixed schedule)")
    ap.add_argument("--no-incremental", action="store_true",
                    help="recompute J.s in full every step (default: flip-incremental update where the sweep has it)")
    ap.add_argument("--tts-instances", type=int, default=10, help="tts_sweep: instances per (family, N)")
    ap.add_argument("--tts-sizes", default=None, help="tts_sweep: comma-separated sizes (default: the workload's)")
    ap.add_argument("--requests", type=int, default=1000, help="serving workload: number of requests")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0, help="serving workload: device memory budget")
    ap.add_argument("--slots", type=int, default=64, help="serving workload: concurrent requests")
    ap.add_argument("--chunk", type=int, default=100, help="serving workload: steps per scheduling round")
    args = ap.parse_args()
    if args.summarize_profiles:
        kern = args.profile_kernel or ("k_batch_fp4" if args.workload == "batch4096" else "k_sweep")
        res = summarize_profiles(args.summarize_profiles, WORKLOADS[args.workload]["desc"], kern)
        geo = os.path.join(args.summarize_profiles, "geometry.json")
        if os.path.exists(geo):
            with open(geo) as f:
                res["geometry"] = json.load(f)
        print(json.dumps(res, indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); replicas are independent, "
              "so a multi-GPU run would shard them with no per-step exchange -- not built here.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2407_10205_amd import phia

    mh = None if args.mh is None else tuple(float(t) for t in args.mh.split(","))
    if mh is not None and len(mh) != 2:
        ap.error("--mh takes UP,DOWN")
    w = WORKLOADS[args.workload]
    if w["gen"] == "batch":
        run_batch_bench(args, w)
        return
    if w["gen"] == "serve":
        run_serve_bench(args, w)
        return
    if w["gen"] == "tts_sweep":
        run_tts_sweep(args, w)
        return
    J, h = make_instance(w)
    N, R, T, s = J.shape[0], args.replicas or w["R"], w["T"], w["sched"]
    if args.path is None:
        args.path = w.get("path", "i8")
    stream = torch.cuda.Stream()
    prob = phia.Problem(J, h, path=args.path, stream=stream.cuda_stream)
    if args.no_incremental:
        prob.set_incremental(False)
    tuned_us = prob.autotune(R, 200) if not args.no_tune else None
    info = None

    def one(seed, events=None):
        prob.start(R, T, s["eps"], s["gamma"], beta0=s["beta0"], beta1=s["beta1"], refresh_L=s["refresh_L"],
                   seed=seed, deriv=args.deriv, mh=mh)
        if events is not None:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            prob.run(T)
            e1.record(stream)
            events.append((e0, e1))
        else:
            prob.run(T)
        return prob.best_exact()

    for i in range(args.warmup):
        one(900 + i)
    torch.cuda.synchronize()
    events, bests = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        bests.append(one(1000 + i, events))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = prob.info()  # geometry of the timed runs
    inc_stats = None
    if info["incremental"]:
        # J.s work of the last timed run: k blocks computed over those of a
        # full product at every step
        n_inc, n_full, n_kb = prob.incremental_stats()
        nkb = info["Np"] // 64
        inc_stats = {"steps_incremental": n_inc / max(1, n_inc + n_full),
                     "kblocks_frac": (n_kb + n_full * nkb) / max(1, (n_inc + n_full) * nkb)}
    # per-replica records of the last timed run, for the success estimate
    E_last, _, _ = prob.replica_best()
    mh_stats = None
    if mh is not None:
        acc, dec, lam = prob.replica_mh()
        mh_stats = {"accept_rate": float(acc.sum()) / max(1, int(dec.sum())), "decided_per_replica": int(dec[0]),
                    "beta_multiplier_median": float(np.median(lam))}
    wall = t1 - t0
    ms_step = 1000 * wall / args.steps
    su = float(R) * N * T * args.steps
    value = su / wall
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    su_launch = float(R) * N * T
    ops_su = OPS_PER_SPIN_UPDATE_POLY2 if args.deriv == "poly2" else OPS_PER_SPIN_UPDATE
    achieved = su_launch * ops_su / (kern_ms / 1000)
    Np = info["Np"]
    mfma_ops = 2.0 * Np * Np * (math.ceil(R / info["rows_per_block"]) * info["rows_per_block"]) * T
    fp4_ops = info["sweep_kernel"] == 2  # interleaved sweep with FP4 MFMA operands
    if fp4_ops:
        Nk = math.ceil(Np / 128) * 128  # FP4 products run over 128-wide k blocks
        mfma_ops = 2.0 * Nk * Np * (math.ceil(R / info["rows_per_block"]) * info["rows_per_block"]) * T
    if inc_stats is not None:
        mfma_ops *= inc_stats["kblocks_frac"]
    mfma_peak = (FP4_MFMA_PEAK if fp4_ops else INT8_MFMA_PEAK if info["path_name"] == "i8"
                 else BF16_MFMA_PEAK * 0.5)
    geometry = {k: info[k] for k in ("group", "rows_per_block", "j_in_lds", "sweep_kernel", "group_on_one_xcd",
                                     "incremental")}
    # counter summaries are kept per kernel and per workload variant
    profile_key = (args.workload + (f"_{args.path}" if args.path != w.get("path", "i8") else "") +
                   ("_poly2" if args.deriv == "poly2" else "") + ("_mh" if mh is not None else "") +
                   ("_full" if args.no_incremental else "") + (f"_r{R}" if args.replicas else ""))
    kernel = ("k_sweep_valu" if info["sweep_kernel"] == 4 else
              "k_sweep_pp" if info["sweep_kernel"] >= 1 else "k_sweep_mfma")
    if info["sweep_kernel"] == 4:
        mfma_ops = 0.0  # J.s on the vector ALUs
    if args.geometry_out:
        with open(args.geometry_out, "w") as f:
            json.dump(geometry, f)
    roofline = {"bound": "alu", "achieved": achieved, "peak": VALU_OPS_PEAK, "unit": "ops/s",
                "frac": achieved / VALU_OPS_PEAK,
                "traffic": recorded_traffic(kernel, profile_key, w["desc"], geometry),
                "kernel": kernel,
                "kernel_ms": kern_ms, "ops_per_spin_update": ops_su,
                "mfma_executed_ops_per_s": mfma_ops / (kern_ms / 1000),
                "mfma_frac_of_peak": (mfma_ops / (kern_ms / 1000)) / mfma_peak}

    extra = {}
    if info["sweep_kernel"] == 2 and not args.no_int8_check:
        # the same geometry with int8 matrix-core operands (FP4 is exact here
        # and bit-identical, but the workload names int8): one timed anneal
        os.environ["PHIA_GEOMETRY"] = f"pp,{info['group']},{info['group_on_one_xcd']}"
        try:
            q = phia.Problem(J, h, path=args.path, stream=stream.cuda_stream)
            q.start(R, T, s["eps"], s["gamma"], beta0=s["beta0"], beta1=s["beta1"], refresh_L=s["refresh_L"],
                    seed=1000, deriv=args.deriv)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            q.run(T)
            e1.record(stream)
            torch.cuda.synchronize()
            qi = q.info()
            E8 = q.best_exact()[0]
            q.close()
            extra["int8_operands"] = {"kernel_ms": e0.elapsed_time(e1), "sweep_kernel": qi["sweep_kernel"],
                                      "group": qi["group"], "best_energy_same_seed": int(E8),
                                      "fp4_best_energy_same_seed": int(bests[0][0])}
        finally:
            os.environ.pop("PHIA_GEOMETRY", None)
    if not args.no_tts:
        # target: best energy of one run 10x longer (untimed), Eq. 9 with P per launch
        ref = phia.Problem(J, h, path=args.path, stream=stream.cuda_stream)
        if not args.no_tune:
            ref.autotune(R, 100)
        ref.anneal(R, 10 * T, s["eps"], s["gamma"], beta0=s["beta0"], beta1=s["beta1"],
                   refresh_L=s["refresh_L"], seed=4242, deriv=args.deriv, mh=mh)
        target = ref.best_exact()[0]
        ref.close()
        p_hat = float(np.mean(E_last <= target))
        P = 1.0 - (1.0 - p_hat) ** R if p_hat > 0 else 0.0
        t_run = ms_step / 1000
        if P >= 0.99:
            tts = t_run
        elif P <= 0:
            tts = float("inf")
        else:
            tts = t_run * math.log(0.01) / math.log(1.0 - P)
        extra.update({"tts99_s": tts, "target_energy": int(target), "replica_success": p_hat,
                      "best_energy_per_run": [int(b[0]) for b in bests]})
    # explicit teardown while the runtime and the stream are alive
    prob.close()
    torch.cuda.synchronize()
    if args.calibrate_copy:
        calibrate_copy()
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(J, h, w, args.cpu_seconds, args.deriv, mh)
    out = {
        "metric": "spin-updates/s", "value": value, "unit": "spin-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "fp4 (int8 couplings held exactly as E2M1)" if info["sweep_kernel"] == 2 else info["path_name"],
        "data": "synthetic",
        "config": {"workload": w["desc"], "N": N, "replicas": R, "hmc_steps": T, "path": info["path_name"],
                   "schedule": dict(s, deriv=args.deriv, **({} if mh is None else {"mh_up": mh[0], "mh_down": mh[1]})),
                   "group": info["group"], "rows_per_block": info["rows_per_block"],
                   "j_in_lds": info["j_in_lds"], "group_on_one_xcd": info["group_on_one_xcd"],
                   "incremental": info["incremental"],
                   "sweep_kernel": kernel, "autotune_us_per_step": tuned_us},
        "roofline": roofline, "cpu_baseline": cpu, **extra,
    }
    if mh_stats is not None:
        out["metropolis"] = mh_stats
    if inc_stats is not None:
        out["incremental"] = inc_stats
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
