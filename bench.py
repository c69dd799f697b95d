"""Benchmark of the ACS construction hot path on one MI355X.

Workload (one "step" = one iteration of Alg. 1 = construction of m tours,
iteration best, global update): n = 2392 cities uniform in [0, 10000)^2
(seed 2392), m = n ants, candidate lists of 32, beta = 2, q0 = 0.9,
phi = rho = 0.1, dense FP32 pheromone.  The headline value is construction
steps per second (m * (n - 1) ant moves per iteration) in the asynchronous
atomic mode; the synchronous (bit-exact) mode is timed beside it, and the
other workloads (n=198, n=1000 clustered, n=20000 with the selective memory,
a batch of 256 instances, the non-atomic variant, local-update period 16)
follow as context.

Prints one JSON line.  Only one GPU is supported; --gpus N > 1 exits.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ant construction steps/s at n=2392,m=n; tour gap vs plain ACS at equal time"
HBM_PEAK_GBS = 8000.0
N, CL = 2392, 32
KERNEL = "k_construct_async_dense_q<true, true, true>"
KERNEL_SOURCE = os.path.join(ROOT, "paper_1605_02669_amd", "csrc", "acs_kernels.hip")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_construct_async_dense_q_n2392.md")


def algorithmic_bytes(st_delta: dict, n: int, m: int, cl: int, iters: int) -> float:
    """Bytes the method must move per the per-step model of the design notes:
    per construction step cl * (4 candidate index + 4 tau + 4 eta) + 2 (d of
    the chosen edge) + 4 (tour entry) + 16 (two 4-byte read-modify-writes of
    the local update); per fallback step additionally 6 bytes (4 tau + 2 d)
    for every unvisited city scanned; per ant the closing edge (2 + 16)."""
    steps = st_delta["steps"]
    b = steps * (cl * 12 + 2 + 4 + 16)
    b += st_delta["fallback_unvisited"] * 6
    b += iters * m * (2 + 16)
    return float(b)


def measured_traffic():
    """HBM bytes per launch of the headline kernel from the committed
    rocprofv3 counter summary, or None when the kernel source has changed
    since the counters were taken (the summary records the source's hash)."""
    try:
        text = open(TRAFFIC_PROFILE).read()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    h = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not h or not t or h.group(1) != src:
        return None
    return float(t.group(1))


def run_mode(acs, xy, mode, steps, warmup, seed=0, **kw):
    import torch
    kw.setdefault("m", 0)
    kw.setdefault("cl", CL)
    col = acs.Colony(xy, mode=mode, seed=seed, **kw)
    col.iterate(max(warmup, 1))
    st0 = col.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    col.iterate(steps)  # one call: the library records events around every construction
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = col.stats()
    delta = {k: st1[k] - st0[k] for k in ("steps", "fallback", "fallback_unvisited", "greedy",
                                          "roulette", "cas_retries", "spm_hits", "spm_misses")}
    res = dict(
        seconds=t1 - t0,
        steps=delta["steps"],
        construct_ms=st1["construct_ms"],  # summed over the launches of the timed call
        launches=st1["construct_launches"],
        iterate_ms=st1["iterate_ms"],
        best=st1["best_length"],
        nn_length=st1["nn_length"],
        delta=delta,
        n=col.n, m=col.m, cl=col.cl,
    )
    col.close()
    return res


def host_cpu() -> dict:
    """The host's CPU model, logical CPUs, the CPUs this process may run on,
    and the OpenMP thread count the environment sets."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS")
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": affinity,
            "omp_num_threads": int(omp) if omp and omp.isdigit() else None}


def cpu_baseline(xy, budget_s: float = 12.0):
    """The oracle on the host cores: every core this process may use (OpenMP
    over the ants of a step; the environment's OMP_NUM_THREADS caps it where
    set, as on a shared host), then one thread (the paper's sequential
    convention)."""
    import oracle
    host = host_cpu()
    threads = host["affinity"]
    if host["omp_num_threads"]:
        threads = min(threads, host["omp_num_threads"])
    oracle.set_threads(threads)
    orc = oracle.Oracle(xy, cl=CL, seed=0)
    t0 = time.perf_counter()
    iters = 0
    while True:
        orc.iterate(1)
        iters += 1
        if time.perf_counter() - t0 > budget_s or iters >= 8:
            break
    dt = time.perf_counter() - t0
    steps = orc.counts()["steps"]
    oracle.set_threads(1)
    orc.close()
    one = oracle.Oracle(xy, cl=CL, seed=0)
    t0 = time.perf_counter()
    one.iterate(1)
    dt1 = time.perf_counter() - t0
    steps1 = one.counts()["steps"]
    one.close()
    return dict(value=steps / dt, unit="steps/s", cores=threads, kind="oracle",
                single_thread_value=steps1 / dt1, host=host,
                sample=f"{iters} synchronous iterations of the n={N}, m={N} workload "
                       f"({steps} steps, {dt:.1f} s, {threads} OpenMP threads); "
                       f"single thread: 1 iteration ({dt1:.1f} s)")


EXTRA = {
    # n=198 uniform, m=n, cl=32, dense (the paper's d198 size)
    "n198": dict(kind="uniform", n=198, kw=dict(), modes=(("sync", 20), ("async", 50))),
    # n=1000 clustered (20 Gaussian clusters), m=n, cl=32, dense
    "n1000_clustered": dict(kind="clustered", n=1000, kw=dict(), modes=(("sync", 3), ("async", 20))),
    # n=20000 uniform, m=1024, cl=16, selective memory with s=8
    "n20000_spm": dict(kind="uniform", n=20000, kw=dict(m=1024, cl=16, memory=1, spm_s=8),
               modes=(("sync", 1), ("async", 5), ("racy", 5))),
    # the headline instance without atomics (the paper's Alt) and with the
    # local update after every 16th edge only
    "n2392_alt": dict(kind="uniform", n=N, kw=dict(), modes=(("racy", 20),)),
    "n2392_period16": dict(kind="uniform", n=N, kw=dict(local_update_period=16),
                modes=(("async", 20), ("racy", 20), ("sync", 2))),
    # the in-step sequential schedule (Alg. 1 read literally) with m = n and
    # with a 64-ant colony, beside the step-snapshot schedule at m = 64
    "n2392_sequential": dict(kind="uniform", n=N, kw=dict(), modes=(("sequential", 1),)),
    "n2392_sequential_m64": dict(kind="uniform", n=N, kw=dict(m=64),
                                 modes=(("sequential", 5), ("sync", 5))),
}


def run_extra(acs, inputs, name):
    spec = EXTRA[name]
    xy = inputs.uniform(spec["n"]) if spec["kind"] == "uniform" else inputs.clustered(spec["n"])
    res = {"n": spec["n"], **{k: v for k, v in spec["kw"].items()}}
    modes = {"sync": acs.ACS_SYNC, "async": acs.ACS_ASYNC_ATOMIC, "racy": acs.ACS_ASYNC_RACY,
             "sequential": acs.ACS_SEQUENTIAL}
    for mode_name, iters in spec["modes"]:
        r = run_mode(acs, xy, modes[mode_name], iters, 1, **spec["kw"])
        res[mode_name] = {"steps_per_s": r["steps"] / r["seconds"],
                          "ms_per_iteration": r["seconds"] * 1e3 / iters,
                          "construct_ms": r["construct_ms"] / r["launches"],
                          "iterations": iters, "best": r["best"]}
    return res


def run_batch(acs, inputs, iters=5, count=256):
    """256 instances, n log-uniform in [100, 2000], half uniform and half
    clustered, m = n each, dense, asynchronous; one graph launch per
    iteration."""
    import torch
    insts = inputs.batch(count)
    t0 = time.perf_counter()
    b = acs.Batch(insts, cl=CL, seed=0)
    create_s = time.perf_counter() - t0
    b.iterate(1 + 4 + 1)  # warm-up and the launch-shape tuning (up to 4 candidates)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.iterate(iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info = b.info()
    tuning = b.tuning()
    b.close()
    return {"instances": count, "launch_shape": tuning["chosen"],
            "tuning_ms": tuning["candidates"], "n_min": int(min(len(x) for x in insts)),
            "n_max": int(max(len(x) for x in insts)),
            "steps_per_iteration": info["steps_per_iteration"], "graph": info["graph"],
            "steps_per_s": info["steps_per_iteration"] * iters / dt,
            "ms_per_iteration": dt * 1e3 / iters, "iterations": iters,
            "create_s": create_s}


def run_quality(acs, inputs, seeds=20, iters=100):
    """Best tour length after `iters` iterations over `seeds` seeds at the
    headline size, for the bit-exact synchronous mode, the asynchronous
    atomic mode (headline kernel) and the unsynchronised Alt mode (Sec. 3.1.2
    and Sec. 4.1 compare the atomic and the Alt variants this way)."""
    import numpy as np
    from scipy.stats import mannwhitneyu
    xy = inputs.uniform(N)
    arms = {"sync": acs.ACS_SYNC, "async_atomic": acs.ACS_ASYNC_ATOMIC,
            "alt": acs.ACS_ASYNC_RACY}
    res, out = {}, {"n": N, "seeds": seeds, "iterations": iters}
    for name, mode in arms.items():
        best = []
        for s in range(seeds):
            col = acs.Colony(xy, mode=mode, seed=s, cl=CL)
            col.iterate(iters)
            best.append(col.best()[1])
            lnn = col.stats()["nn_length"]
            col.close()
        r = np.array(best, dtype=np.float64)
        res[name] = r
        out[name] = {"mean": r.mean(), "sd": r.std(), "min": r.min(), "max": r.max(),
                     "vs_nn_percent": 100.0 * (r.mean() / lnn - 1.0)}
    for a, b in (("async_atomic", "sync"), ("alt", "async_atomic"), ("alt", "sync")):
        out[f"{a}_vs_{b}"] = {"gap_percent": 100.0 * (res[a].mean() / res[b].mean() - 1.0),
                              "rank_sum_p": float(mannwhitneyu(res[a], res[b]).pvalue)}
    return out


def run_ants(acs, inputs, ants=(64, 256, 1024, N), seeds=10, budget_tours=25 * N,
             budget_s=0.5):
    """Fewer ants than cities (Sec. 4, the number of ants): mean best tour
    length over `seeds` seeds for each colony size m, at an equal budget of
    constructed solutions (budget_tours / m iterations) and at equal wall
    clock (budget_s per run), asynchronous atomic mode at the headline size."""
    import numpy as np
    import torch
    xy = inputs.uniform(N)
    out = {"n": N, "seeds": seeds, "budget_tours": budget_tours, "budget_s": budget_s}
    for m in ants:
        iters = max(1, budget_tours // m)
        eq_b, eq_t, its_t = [], [], []
        for s in range(seeds):
            col = acs.Colony(xy, m=m, mode=acs.ACS_ASYNC_ATOMIC, seed=s, cl=CL)
            col.iterate(iters)
            eq_b.append(col.best()[1])
            col.close()
            col = acs.Colony(xy, m=m, mode=acs.ACS_ASYNC_ATOMIC, seed=s, cl=CL)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k = 0
            while time.perf_counter() - t0 < budget_s:
                col.iterate(1)
                k += 1
            eq_t.append(col.best()[1])
            its_t.append(k)
            col.close()
        out[f"m{m}"] = {"equal_budget": {"iterations": iters, "mean_best": float(np.mean(eq_b))},
                        "equal_time": {"iterations": float(np.mean(its_t)),
                                       "mean_best": float(np.mean(eq_t))}}
    return out


def run_colonies(acs, inputs, colonies=(1, 4, 8), seeds=5, budget_s=0.5, period=10):
    """Several colonies on the headline instance with a best-so-far exchange
    every `period` iterations (from the best colony; Sec. 2's multi-colony
    model), n ants in total, against one colony, at equal wall-clock: mean
    best tour length over `seeds` seeds."""
    import numpy as np
    import torch
    xy = inputs.uniform(N)
    out = {"n": N, "seeds": seeds, "budget_s": budget_s, "exchange_period": period}
    for c in colonies:
        best, its = [], []
        for s in range(seeds):
            b = acs.Batch([xy] * c, m=N // c, cl=CL, seed=s)
            if c > 1:
                b.set_exchange(0, period)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k = 0
            while time.perf_counter() - t0 < budget_s:
                b.iterate(1)
                k += 1
            best.append(min(b.best(i)[1] for i in range(c)))
            its.append(k)
            b.close()
        out[f"c{c}"] = {"ants_per_colony": N // c, "mean_best": float(np.mean(best)),
                        "iterations": float(np.mean(its))}
    return out


def run_local_search(acs, inputs, seeds=5, budget_s=1.0):
    """ACS with a descent after each construction against plain ACS at equal
    wall-clock on the headline instance (asynchronous atomic mode): m = n
    ants with and without the descent (2-opt and Or-opt; and with the 3-opt
    move as well), and 64-ant colonies with each descent."""
    import numpy as np
    import torch
    xy = inputs.uniform(N)
    out = {"n": N, "seeds": seeds, "budget_s": budget_s}
    for name, kw in (("plain_m2392", dict()), ("ls_m2392", dict(local_search=1)),
                     ("ls_m64", dict(local_search=1, m=64)),
                     ("ls3_m2392", dict(local_search=2)),
                     ("ls3_m64", dict(local_search=2, m=64))):
        best, its, ms = [], [], []
        for s in range(seeds):
            col = acs.Colony(xy, mode=acs.ACS_ASYNC_ATOMIC, seed=s, cl=CL, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k = 0
            while time.perf_counter() - t0 < budget_s:
                col.iterate(1)
                k += 1
            best.append(col.best()[1])
            its.append(k)
            ms.append(col.stats()["iterate_ms"])
            col.close()
        out[name] = {"mean_best": float(np.mean(best)), "iterations": float(np.mean(its)),
                     "ms_per_iteration": float(np.mean(ms))}
    return out


MFMA_BF16_PEAK_TFLOPS = 2500.0
# algorithmic flops per feature row of the 4-64-64-1 network: forward
# 2 (4*64 + 64*64 + 64); backward adds the weight and input gradients of the
# two upper layers and the first layer's weight gradient, 2 (64 + 64 + 2*4096
# + 256), plus the recomputed forward
PRIOR_FWD_FLOPS = 2 * (4 * 64 + 64 * 64 + 64)
PRIOR_BWD_FLOPS = PRIOR_FWD_FLOPS + 2 * (64 + 64 + 2 * 64 * 64 + 4 * 64)


def run_prior(acs, inputs, rows=1 << 22, reps=5, eval_seeds=10, eval_budget_s=0.5):
    """The learned prior's kernels at training scale (BF16 matrix cores), and
    the equal-wall-clock comparison with plain ACS when trained parameters
    are present."""
    import numpy as np
    import torch
    from paper_1605_02669_amd import prior
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    X = torch.randn((rows, 4), generator=g, device="cuda")
    Y = torch.rand((rows,), generator=g, device="cuda")
    P = torch.tensor(prior.init_params(0), device="cuda")
    G = torch.zeros_like(P)
    L = torch.zeros(1, device="cuda")
    acs.prior_forward(P, X)
    acs.prior_grad(P, X, Y, G, L)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    for _ in range(reps):
        acs.prior_forward(P, X)
    e[1].record()
    for _ in range(reps):
        acs.prior_grad(P, X, Y, G, L)
    e[2].record()
    torch.cuda.synchronize()
    fwd_s = e[0].elapsed_time(e[1]) / 1e3 / reps
    bwd_s = e[1].elapsed_time(e[2]) / 1e3 / reps
    fwd_tf = rows * PRIOR_FWD_FLOPS / fwd_s / 1e12
    bwd_tf = rows * PRIOR_BWD_FLOPS / bwd_s / 1e12
    out = {"rows": rows,
           "forward": {"ms": fwd_s * 1e3, "tflops": fwd_tf,
                       "mfma_frac": fwd_tf / MFMA_BF16_PEAK_TFLOPS},
           "gradient": {"ms": bwd_s * 1e3, "tflops": bwd_tf,
                        "mfma_frac": bwd_tf / MFMA_BF16_PEAK_TFLOPS},
           "peak_tflops": MFMA_BF16_PEAK_TFLOPS, "flops_per_row": [PRIOR_FWD_FLOPS, PRIOR_BWD_FLOPS]}
    if os.path.exists(prior.DEFAULT_PARAMS):
        params = torch.tensor(np.load(prior.DEFAULT_PARAMS), device="cuda")
        out["equal_time"] = prior.evaluate(params, seeds=eval_seeds, budget_s=eval_budget_s,
                                           log=lambda s: print("# " + s, file=sys.stderr,
                                                               flush=True))
    else:
        out["equal_time"] = None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sync-steps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extra", default="n198,n1000_clustered,n20000_spm,batch256,prior,n2392_alt,"
                                       "n2392_period16,n2392_sequential,n2392_sequential_m64,"
                                       "quality,ants,colonies,local_search",
                    help="other workloads timed beside the headline (comma list of "
                         "n198, n1000_clustered, n20000_spm, batch256, prior, n2392_alt, n2392_period16, "
                         "n2392_sequential, n2392_sequential_m64, quality, ants, colonies, "
                         "local_search; empty for none)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="after timing, run one plain device copy of this many MiB "
                         "(reference kernel for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: only one GPU is supported (asked for {args.gpus}); "
              "the colony runs on a single MI355X.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1605_02669_amd import acs, inputs

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    acs.load()
    xy = inputs.uniform(N)

    asy = run_mode(acs, xy, acs.ACS_ASYNC_ATOMIC, args.steps, args.warmup)
    print(f"# async: {asy['seconds']*1e3/args.steps:.3f} ms/iteration", file=sys.stderr, flush=True)
    syn = None
    if args.sync_steps > 0:
        syn = run_mode(acs, xy, acs.ACS_SYNC, args.sync_steps, 1)
        print(f"# sync: {syn['seconds']*1e3/args.sync_steps:.3f} ms/iteration", file=sys.stderr,
              flush=True)

    value = asy["steps"] / asy["seconds"]
    ms_per_step = asy["seconds"] * 1e3 / args.steps
    avg_launch_s = asy["construct_ms"] / asy["launches"] / 1e3
    bytes_per_launch = algorithmic_bytes(asy["delta"], asy["n"], asy["m"], asy["cl"],
                                         args.steps) / args.steps
    achieved = bytes_per_launch / avg_launch_s / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ACS construction, n=2392 uniform [0,1e4)^2 (seed 2392), m=n, "
                               "cl=32, beta=2, q0=0.9, phi=rho=0.1, dense FP32 pheromone, "
                               "asynchronous atomic local updates",
                   "n": asy["n"], "m": asy["m"], "cl": asy["cl"], "mode": "async_atomic"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": KERNEL,
                     "bytes_per_launch": bytes_per_launch,
                     "avg_launch_ms": avg_launch_s * 1e3},
        "sync_mode": None if syn is None else {
            "value": syn["steps"] / syn["seconds"], "unit": "steps/s",
            "ms_per_step": syn["seconds"] * 1e3 / args.sync_steps,
            "avg_construct_ms": syn["construct_ms"] / syn["launches"]},
        "fallback_share": asy["delta"]["fallback"] / max(asy["delta"]["steps"], 1),
        "cas_retry_share": asy["delta"]["cas_retries"] / max(2 * asy["delta"]["steps"], 1),
        "best_length_async": asy["best"],
        "nn_length": asy["nn_length"],
    }
    extra = {}
    for name in [x for x in args.extra.split(",") if x]:
        if name == "batch256":
            extra[name] = run_batch(acs, inputs)
        elif name == "quality":
            extra[name] = run_quality(acs, inputs)
        elif name == "ants":
            extra[name] = run_ants(acs, inputs)
        elif name == "colonies":
            extra[name] = run_colonies(acs, inputs)
        elif name == "local_search":
            extra[name] = run_local_search(acs, inputs)
        elif name == "prior":
            extra[name] = run_prior(acs, inputs)
        else:
            extra[name] = run_extra(acs, inputs, name)
        print(f"# {name}: {extra[name]}", file=sys.stderr, flush=True)
    if extra:
        out["other_workloads"] = extra
    if args.copy_calibration_mb:
        nbytes = args.copy_calibration_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(xy)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
