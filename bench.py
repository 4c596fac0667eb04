"""Throughput of the batched simplex cross-map on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one pass of the whole hot path (ingest, embedding, library draws,
gather, fused distance / top-(E+1) / prediction / Pearson kernel, rho
finalize) over the parameter-sweep workload: coupled logistic map, N=10^4,
E=1..10, tau=1..5, 20 library sizes log-spaced 100..10^4, r=250, both
directions -- 500 000 rho values and ~5e9 cross-map predictions per step.
The series are resident in device memory before the timed region starts.

The timed steps replay the call's HIP graph (the form a caller gets).  The
runtime cannot time events recorded by graph nodes, so the roofline's kernel
durations come from HIP events around each cross-map launch of a profiled
pass of the same steps right after (direct launches on the same stream); its
wall time is reported beside the graph's.

Prints one JSON line: value = cross-map predictions per second, plus
rho-realizations per second, the roofline of the cross-map kernel (binary32
flops per pair 3E-1, over the summed HIP-event duration of its launches; HBM
traffic from the committed counter summary when it matches the kernel
sources), the other workloads of the method (`workloads`: small coupled map
with plain vs batched launches, long noisy series, 64-series causal matrix),
the sweep's launch forms (`forms`: persistent, no graph, plain vs batched on
its r = 1 subset), the run-time elasticity study (`elasticity`), the same
workloads through the paper's distance indexing table (`index_table`), the
sweep and long series with nested libraries (`nested`), E-sweep sharing
(`shared_e`), the served form (`served`: capacity against the same jobs one
after another, p50/p99 job latency at several loads, a binding HBM budget),
and the CPU oracle timed on a deterministic sample of the same realizations
(all threads and one core, extrapolated to the workload, and checked against
the GPU's rho).

    python bench.py --serve-protocol 1

runs only the served form's full protocol (seven loads x 1000 jobs) and
prints its JSON.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1905_00565_amd import capi, synth  # noqa: E402

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak

# HBM bytes per cross-map launch, from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# of this bench (scaled by a plain copy of known size); valid only for the
# kernel sources it was measured on, which the file records by hash.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "crossmap_sweep_coupled_logistic_N10000_traffic.json")
KERNEL_SOURCES = ["paper_1905_00565_amd/csrc/ccm_device.h",
                  "paper_1905_00565_amd/csrc/ccm_inst.hip",
                  "paper_1905_00565_amd/csrc/ccm_inst_multi.hip",
                  "paper_1905_00565_amd/csrc/ccm_internal.h",
                  "paper_1905_00565_amd/csrc/ccm_tune.h"]


def kernel_sources_sha256() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload_name: str):
    """Counter-measured HBM bytes per launch, or None when the counters were
    taken on other kernel sources or another workload."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    if d.get("workload") != workload_name:
        return None
    return d.get("hbm_bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--r", type=int, default=250, help="realizations per L")
    ap.add_argument("--n", type=int, default=10000, help="series length")
    ap.add_argument("--flags", type=int, default=0, help="CCM_FLAG_* bits")
    ap.add_argument("--cpu-modulus", type=int, default=1000,
                    help="CPU oracle sample: realizations whose library stream state is "
                         "0 mod this (0: skip the CPU baseline)")
    ap.add_argument("--workloads", type=int, default=1,
                    help="1: also time the small, long-series and causal-matrix "
                         "workloads and the elasticity study (0: skip)")
    ap.add_argument("--legs", type=str,
                    default="small,long,matrix,elasticity,index_table,nested,shared_e,forms",
                    help="legs run with --workloads 1 (matrix-alone: the causal matrix "
                         "without its plain comparison, for profiling)")
    ap.add_argument("--serve-jobs", type=int, default=200,
                    help="jobs per load point of the served leg (0: skip it)")
    ap.add_argument("--serve-loads", type=str, default="0.5,0.8,0.95",
                    help="Poisson arrival rates as fractions of measured capacity")
    ap.add_argument("--serve-protocol", type=int, default=0,
                    help="1: run only the served form's full protocol and print it")
    ap.add_argument("--protocol-loads", type=str, default="0.1,0.3,0.5,0.7,0.8,0.9,0.95",
                    help="load points of --serve-protocol (a subset runs in less time)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the timed steps, copy this many MiB device to device "
                         "once (a plain copy of known size for calibrating the "
                         "profiler's byte counters)")
    return ap.parse_args()


def cpu_info():
    """Host cores and CPU model of the machine running the bench."""
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
    except AttributeError:
        affinity = None
    return {"nproc": os.cpu_count(), "affinity": affinity, "model": model}


def workload_pairs(w):
    """(query, candidate) pairs of the whole workload (self excluded)."""
    tot = 0
    for e in w.E:
        for t in w.tau:
            ne = w.N - (e - 1) * t
            for l in w.L:
                tot += 2 * w.r * (ne - 1) * min(l, ne)
    return tot


def cpu_baseline(w, rho_gpu, modulus=1000, single_every=12):
    """The oracle on a deterministic sample of the workload: the realizations
    whose library stream state is 0 mod `modulus` (both directions), timed on
    every host thread, and every `single_every`-th of them on one core; the
    full workload's CPU time is extrapolated by pair count.  The same sample
    is checked against the GPU's rho of the last timed step."""
    import oracle
    orc = oracle.default()
    threads = oracle.default_threads()
    tasks, picks = orc.deterministic_sample(w.X, w.Y, w.E, w.tau, w.L, w.r, w.seed, modulus)

    def cost(ts):
        preds = pairs = 0
        for t in ts:
            ne = w.N - (t[2] - 1) * t[3]
            preds += ne
            pairs += (ne - 1) * min(t[4], ne)
        return preds, pairs

    preds, pairs = cost(tasks)
    t0 = time.perf_counter()
    want = orc.realizations_threaded(tasks, threads)
    el = time.perf_counter() - t0
    sub = tasks[::single_every]
    preds1, pairs1 = cost(sub)
    t0 = time.perf_counter()
    orc.realizations_threaded(sub, threads=1)
    el1 = time.perf_counter() - t0
    got = np.asarray([rho_gpu[p] for p in picks])
    full = workload_pairs(w)
    return {"value": preds / el, "unit": "predictions/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(tasks)} realizations of the workload's {2 * len(w.E) * len(w.tau) * len(w.L) * w.r} "
                      f"(library stream state = 0 mod {modulus}, both directions; "
                      f"{pairs:.3g} pairs), {el:.1f} s on {threads} threads",
            "single_core": {"value": preds1 / el1, "unit": "predictions/s", "cores": 1,
                            "sample": f"every {single_every}th of the sample: {len(sub)} "
                                      f"realizations, {pairs1:.3g} pairs, {el1:.1f} s"},
            "cpu": cpu_info(),
            "extrapolated": {"label": "extrapolated by pair count from the sample",
                             "workload_pairs": full,
                             "step_seconds_all_threads": el * full / pairs,
                             "step_seconds_one_core": el1 * full / pairs1},
            "parity": {"realizations": len(tasks),
                       "max_abs_rho_diff_vs_gpu": float(np.max(np.abs(got - np.asarray(want))))}}


def _timed(ctx, torch, fn, reps, profile):
    """Mean wall time per call of fn (after one untimed call), and the
    library's kernel counters over the timed calls when profiling."""
    ctx.profile_enable(profile)
    fn()
    torch.cuda.synchronize()
    ctx.profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    p = ctx.profile_read(reset=True)
    if profile:
        for k in ("kernel_ms", "launches", "pairs", "flops", "predictions", "realizations"):
            p[k] = p[k] / reps
    return el, p


def _leg(ctx, torch, name, fn, reps, plain_fn=None, plain_reps=1, plain_note=None):
    """Wall time of the batched form (graph path, no profiling), one profiled
    pass for kernel throughput, and optionally the plain per-realization form."""
    el, _ = _timed(ctx, torch, fn, reps, False)
    _, p = _timed(ctx, torch, fn, 1, True)
    out = {"workload": name, "ms_per_call": el * 1e3,
           "predictions_per_sec": p["predictions"] / el,
           "rho_realizations_per_sec": p["realizations"] / el,
           "kernel_ms": p["kernel_ms"], "kernel_tflops": p["flops"] / p["kernel_ms"] / 1e9,
           "kernel_frac_of_fp32_peak": p["flops"] / p["kernel_ms"] / 1e9 / FP32_VECTOR_PEAK_TFLOPS,
           "pairs": p["pairs"]}
    if plain_fn is not None:
        b, _ = _timed(ctx, torch, plain_fn[0], plain_reps, False)
        pl, _ = _timed(ctx, torch, plain_fn[1], plain_reps, False)
        out["plain_vs_batched"] = {"subset": plain_note, "batched_ms": b * 1e3,
                                   "plain_ms": pl * 1e3, "plain_over_batched": pl / b}
    return out


def workloads_leg(ctx, torch, dev, stream, which=("small", "long", "matrix")):
    """The other configurations of the method on one GPU: the small coupled
    map (launch-bound), the long noisy series, and the 64-series causal
    matrix (one neighbour search per library series shared by its 63
    targets), each with the plain per-realization form beside the batched
    one (the matrix on its r = 1 subset)."""
    res = {}
    f64 = dict(dtype=torch.float64, device=dev)

    if "small" in which:
        w = synth.workload_small()
        X, Y = torch.tensor(w.X, device=dev), torch.tensor(w.Y, device=dev)
        a, b = torch.empty((len(w.L), w.r), **f64), torch.empty((len(w.L), w.r), **f64)

        def small(flags=0):
            return lambda: ctx.ccm_dev(X, Y, w.E[0], w.tau[0], w.L, w.r, w.seed, a, b,
                                       stream=stream, flags=flags)
        res["small"] = _leg(ctx, torch, w.name, small(), 20,
                            (small(), small(capi.CCM_FLAG_PLAIN)), 3, "the whole workload")

    if "long" in which:
        w = synth.workload_long()
        X, Y = torch.tensor(w.X, device=dev), torch.tensor(w.Y, device=dev)
        a, b = torch.empty((len(w.L), w.r), **f64), torch.empty((len(w.L), w.r), **f64)
        res["long"] = _leg(ctx, torch, w.name,
                           lambda: ctx.ccm_dev(X, Y, w.E[0], w.tau[0], w.L, w.r, w.seed, a, b,
                                               stream=stream), 1)

    if "matrix" not in which:
        return res
    m = synth.workload_matrix()
    S = torch.tensor(m["S"], device=dev)
    M = S.shape[0]
    rho = torch.empty((M, M, len(m["L"]), m["r"]), **f64)
    rho1 = torch.empty((M, M, len(m["L"]), 1), **f64)

    def matrix(r, out, flags=0):
        return lambda: ctx.ccm_matrix_dev(S, m["E"], m["tau"], m["L"], r, m["seed"], out,
                                          stream=stream, flags=flags)
    plain = None if "matrix-alone" in which else (matrix(1, rho1),
                                                     matrix(1, rho1, capi.CCM_FLAG_PLAIN))
    res["matrix"] = _leg(ctx, torch, m["name"], matrix(m["r"], rho), 1, plain, 1,
                         "r = 1 (640 neighbour searches, 40 320 rho values)")
    return res


def table_leg(ctx, torch, dev, stream, steps=3):
    """The distance indexing table (Section 3.2, flag CCM_FLAG_TABLE) on the
    sweep, the long series and the causal matrix: same results bit for bit
    as the brute-force path (tested); realizations with a short expected
    walk use it, the rest scan.  Wall time per call includes building the
    tables."""
    f64 = dict(dtype=torch.float64, device=dev)
    out = {}
    w = synth.workload_sweep()
    X, Y = torch.tensor(w.X, device=dev), torch.tensor(w.Y, device=dev)
    rho = torch.empty((2, len(w.E), len(w.tau), len(w.L), w.r), **f64)
    fn = lambda: ctx.ccm_sweep_dev(X, Y, w.E, w.tau, w.L, w.r, w.seed, rho, stream=stream,
                                   flags=capi.CCM_FLAG_TABLE)
    el, _ = _timed(ctx, torch, fn, steps, False)
    _, p = _timed(ctx, torch, fn, 1, True)
    out["sweep"] = {"workload": w.name, "ms_per_call": el * 1e3,
                    "predictions_per_sec": p["predictions"] / el,
                    "rho_realizations_per_sec": p["realizations"] / el,
                    "table_realization_share": p["table_realizations"] / p["realizations"]}
    w = synth.workload_long()
    X, Y = torch.tensor(w.X, device=dev), torch.tensor(w.Y, device=dev)
    a, b = torch.empty((len(w.L), w.r), **f64), torch.empty((len(w.L), w.r), **f64)
    fn = lambda: ctx.ccm_dev(X, Y, w.E[0], w.tau[0], w.L, w.r, w.seed, a, b, stream=stream,
                             flags=capi.CCM_FLAG_TABLE)
    el, _ = _timed(ctx, torch, fn, 1, False)
    _, p = _timed(ctx, torch, fn, 1, True)
    out["long"] = {"workload": w.name, "ms_per_call": el * 1e3,
                   "predictions_per_sec": p["predictions"] / el,
                   "table_realization_share": p["table_realizations"] / p["realizations"]}
    m = synth.workload_matrix()
    S = torch.tensor(m["S"], device=dev)
    M = S.shape[0]
    rho = torch.empty((M, M, len(m["L"]), m["r"]), **f64)
    fn = lambda: ctx.ccm_matrix_dev(S, m["E"], m["tau"], m["L"], m["r"], m["seed"], rho,
                                    stream=stream, flags=capi.CCM_FLAG_TABLE)
    el, _ = _timed(ctx, torch, fn, 1, False)
    _, p = _timed(ctx, torch, fn, 1, True)
    out["matrix"] = {"workload": m["name"], "ms_per_call": el * 1e3,
                     "predictions_per_sec": p["predictions"] / el,
                     "table_realization_share": p["table_realizations"] / p["realizations"]}
    return out


def nested_leg(ctx, torch, dev, stream, steps=3):
    """Nested libraries across L (flag CCM_FLAG_NESTED): the sweep and the
    long series with the libraries of one r drawn as prefixes of one
    ordering, so a query scans the largest library once and takes a
    snapshot at every size.  Different draws from the default (rho differs),
    tested against the oracle's nested mode."""
    f64 = dict(dtype=torch.float64, device=dev)
    out = {}
    w = synth.workload_sweep()
    X, Y = torch.tensor(w.X, device=dev), torch.tensor(w.Y, device=dev)
    rho = torch.empty((2, len(w.E), len(w.tau), len(w.L), w.r), **f64)
    fn = lambda: ctx.ccm_sweep_dev(X, Y, w.E, w.tau, w.L, w.r, w.seed, rho, stream=stream,
                                   flags=capi.CCM_FLAG_NESTED)
    el, _ = _timed(ctx, torch, fn, steps, False)
    _, p = _timed(ctx, torch, fn, 1, True)
    out["sweep"] = {"workload": w.name, "ms_per_call": el * 1e3,
                    "predictions_per_sec": p["predictions"] / el,
                    "rho_realizations_per_sec": p["realizations"] / el,
                    "pairs": p["pairs"], "kernel_ms": p["kernel_ms"],
                    "kernel_tflops": p["flops"] / p["kernel_ms"] / 1e9}
    w = synth.workload_long()
    X, Y = torch.tensor(w.X, device=dev), torch.tensor(w.Y, device=dev)
    a, b = torch.empty((len(w.L), w.r), **f64), torch.empty((len(w.L), w.r), **f64)
    fn = lambda: ctx.ccm_dev(X, Y, w.E[0], w.tau[0], w.L, w.r, w.seed, a, b, stream=stream,
                             flags=capi.CCM_FLAG_NESTED)
    el, _ = _timed(ctx, torch, fn, 1, False)
    _, p = _timed(ctx, torch, fn, 1, True)
    out["long"] = {"workload": w.name, "ms_per_call": el * 1e3,
                   "predictions_per_sec": p["predictions"] / el, "pairs": p["pairs"],
                   "kernel_tflops": p["flops"] / p["kernel_ms"] / 1e9}
    return out


def shared_e_leg(ctx, torch, dev, stream, default_ms, steps=3):
    """E-sweep sharing (flag CCM_FLAG_SHARED_E): the sweep with every E on
    E_max's common points and one library per (tau, L, r), so one scan per
    (tau, L, r, direction) yields all ten E.  Different draws from the
    default (rho differs), tested against the oracle's shared-E mode."""
    f64 = dict(dtype=torch.float64, device=dev)
    w = synth.workload_sweep()
    X, Y = torch.tensor(w.X, device=dev), torch.tensor(w.Y, device=dev)
    rho = torch.empty((2, len(w.E), len(w.tau), len(w.L), w.r), **f64)
    fn = lambda: ctx.ccm_sweep_dev(X, Y, w.E, w.tau, w.L, w.r, w.seed, rho, stream=stream,
                                   flags=capi.CCM_FLAG_SHARED_E)
    el, _ = _timed(ctx, torch, fn, steps, False)
    _, p = _timed(ctx, torch, fn, 1, True)
    return {"workload": w.name, "ms_per_call": el * 1e3,
            "predictions_per_sec": p["predictions"] / el,
            "rho_realizations_per_sec": p["realizations"] / el,
            "speedup_over_default_sweep": default_ms / (el * 1e3),
            "pairs": p["pairs"], "kernel_ms": p["kernel_ms"],
            "kernel_tflops": p["flops"] / p["kernel_ms"] / 1e9}


def elasticity_leg(ctx, torch, dev, stream, reps=3):
    """Run time as one parameter doubles, after the paper's parameter study
    (Section 4.2, Table 2): N = 4000, r = 500; each case fixes the varied
    parameter (L in 500, 1000, 2000; E or tau in 1, 2, 4) and keeps the
    baseline's lists for the other two.  Timed for both query sets: every
    embedded point (cost linear in L) and the library points only (cost
    quadratic in L, the shape of the paper's single-threaded timings)."""
    x, y = synth.coupled_logistic(4000)
    X, Y = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    base = {"L": [500, 1000, 2000], "E": [1, 2, 4], "tau": [1, 2, 4]}
    out = {"workload": "coupled-logistic N=4000 r=500, baseline L=500,1000,2000 E=1,2,4 "
                       "tau=1,2,4", "seconds": {}, "ratio_per_doubling": {}}
    for qs in (0, 1):
        key = "all_points" if qs == 0 else "library_points"
        secs = {}
        for par in ("L", "E", "tau"):
            secs[par] = []
            for v in base[par]:
                g = dict(base)
                g[par] = [v]
                rho = torch.empty((2, len(g["E"]), len(g["tau"]), len(g["L"]), 500),
                                  dtype=torch.float64, device=dev)
                fn = (lambda g=g, rho=rho: ctx.ccm_sweep_dev(X, Y, g["E"], g["tau"], g["L"], 500,
                                                             7, rho, stream=stream,
                                                             query_set=qs))
                el, _ = _timed(ctx, torch, fn, reps, False)
                secs[par].append(el)
        out["seconds"][key] = secs
        out["ratio_per_doubling"][key] = {
            par: [secs[par][1] / secs[par][0], secs[par][2] / secs[par][1]] for par in secs}
    return out


def _serve(srv, jobs, arrivals, flags=0, note=None):
    """Submit jobs at the given arrival times (seconds from now), wait for all;
    returns (makespan, latencies submit->done, stats of each job).  With a
    note, a progress line goes to stderr every 100 submissions."""
    t0 = time.perf_counter()
    tickets = []
    for k, ((X, Y, j), ta) in enumerate(zip(jobs, arrivals)):
        delay = ta - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append((srv.submit(X, Y, j["E"], j["tau"], j["L"], j["r"], j["seed"],
                                   flags=flags), j))
        if note and (k + 1) % 100 == 0:
            print(f"bench: {note}: {k + 1}/{len(jobs)} submitted", file=sys.stderr, flush=True)
    lat, stats = [], []
    for t, j in tickets:
        assert srv.wait(t) == capi.CCM_OK
        _, _, st = srv.result(t, len(j["L"]), j["r"])
        lat.append(st["t_done"] - st["t_submit"])
        stats.append(st)
    return time.perf_counter() - t0, np.asarray(lat), stats


def _max_concurrent(stats):
    ev = sorted([(s["t_admit"], 1) for s in stats] + [(s["t_done"], -1) for s in stats])
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


def load_points(ctx, jobs, capacity, loads, seed, discard):
    """Open loops of Poisson arrivals at each load x capacity: p50/p99 job
    latency (submit to result) over the jobs after the first `discard`."""
    pts = []
    with capi.Server(ctx) as srv:
        _serve(srv, jobs[:4], [0.0] * 4)                 # warm the server up
        for k, load in enumerate(loads):
            rate = load * capacity
            gaps = np.random.default_rng([seed, 17, k]).exponential(1.0 / rate, len(jobs))
            arrivals = np.cumsum(gaps) - gaps[0]
            make, lat, _ = _serve(srv, jobs, list(arrivals), note=f"load {load}")
            kept = lat[discard:]
            pts.append({"load": load, "arrival_rate_jobs_per_sec": rate, "jobs": len(jobs),
                        "discarded": discard, "throughput_jobs_per_sec": len(jobs) / make,
                        "p50_latency_ms": float(np.percentile(kept, 50) * 1e3),
                        "p99_latency_ms": float(np.percentile(kept, 99) * 1e3),
                        "mean_latency_ms": float(kept.mean() * 1e3)})
            print(f"bench: served load {load}: p50 {pts[-1]['p50_latency_ms']:.0f} ms, "
                  f"p99 {pts[-1]['p99_latency_ms']:.0f} ms", file=sys.stderr, flush=True)
    return pts


def served_leg(ctx, n_jobs, loads, n_cap=100, seed=4):
    """Served form on the job-stream workload (jobs of coupled-logistic pairs,
    N ~ U[1000, 50000], E ~ U[1, 10], tau ~ U[1, 4], 10-point L grid,
    r = 100, both directions).
      capacity: the first n_cap jobs submitted at once (closed loop), against
        the same jobs one after another through ccm() (each call batched) and
        the first three through ccm() with one launch per realization;
      load points: Poisson arrivals of n_jobs jobs at each load x capacity,
        p50/p99 latency over the jobs after the first 5%;
      budget: the closed loop again under an HBM budget of twice the largest
        job's footprint, so admission binds;
      tables: the closed loop with distance indexing tables (same results)."""
    stream = synth.job_stream(max(n_jobs, n_cap), 1.0, seed=seed)
    jobs = [(*j["make"](), j) for j in stream]
    cap_jobs = jobs[:n_cap]
    with capi.Server(ctx) as srv:
        _serve(srv, jobs[:4], [0.0] * 4)                 # warm the server up
        make_closed, _, stats = _serve(srv, cap_jobs, [0.0] * len(cap_jobs))
        make_tables, _, _ = _serve(srv, cap_jobs, [0.0] * len(cap_jobs),
                                   flags=capi.CCM_FLAG_TABLE)
    capacity = len(cap_jobs) / make_closed
    preds = sum(st["predictions"] for st in stats)
    foot = max(st["device_bytes"] for st in stats)
    with capi.Server(ctx, hbm_budget_bytes=2 * foot) as srv:
        make_budget, _, stats_b = _serve(srv, cap_jobs, [0.0] * len(cap_jobs))
    per_job = []
    for X, Y, j in cap_jobs:
        t0 = time.perf_counter()
        ctx.ccm(X, Y, j["E"], j["tau"], j["L"], j["r"], j["seed"])
        per_job.append(time.perf_counter() - t0)
    fifo = sum(per_job)
    n_plain = 3
    t0 = time.perf_counter()
    for X, Y, j in cap_jobs[:n_plain]:
        ctx.ccm(X, Y, j["E"], j["tau"], j["L"], j["r"], j["seed"], flags=capi.CCM_FLAG_PLAIN)
    fifo_plain = time.perf_counter() - t0
    points = load_points(ctx, jobs[:n_jobs], capacity, loads, seed, max(1, n_jobs // 20))
    return {
        "workload": f"job stream (seed {seed}): coupled-logistic pairs, N~U[1000,50000], "
                    "E~U[1,10], tau~U[1,4], 10-point geometric L grid, r=100",
        "capacity_jobs": len(cap_jobs),
        "capacity_jobs_per_sec": capacity,
        "closed_loop_predictions_per_sec": preds / make_closed,
        "fifo_ccm_jobs_per_sec": len(cap_jobs) / fifo,
        "served_over_fifo": capacity / (len(cap_jobs) / fifo),
        "load_points": points,
        "budget": {"hbm_budget_bytes": 2 * foot, "largest_job_bytes": foot,
                   "jobs_per_sec": len(cap_jobs) / make_budget,
                   "max_jobs_on_device": _max_concurrent(stats_b),
                   "max_jobs_on_device_unbounded": _max_concurrent(stats)},
        "capacity_jobs_per_sec_with_tables": len(cap_jobs) / make_tables,
        "tables_over_scan": make_closed / make_tables,
        "plain_subset_jobs": n_plain,
        "plain_subset_seconds": fifo_plain,
        "batched_subset_seconds": sum(per_job[:n_plain]),
        "batched_over_plain": fifo_plain / sum(per_job[:n_plain]),
    }


def serve_protocol(ctx, n_jobs=1000, loads=(0.1, 0.3, 0.5, 0.7, 0.8, 0.9, 0.95), seed=4,
                   n_cap=100):
    """The served form's full protocol: capacity from a closed loop of n_cap
    jobs, then n_jobs Poisson arrivals at each load x capacity, the first 50
    jobs of each point discarded."""
    stream = synth.job_stream(n_jobs, 1.0, seed=seed)
    jobs = [(*j["make"](), j) for j in stream]
    with capi.Server(ctx) as srv:
        _serve(srv, jobs[:4], [0.0] * 4)
        make, _, _ = _serve(srv, jobs[:n_cap], [0.0] * n_cap)
    capacity = n_cap / make
    return {"capacity_jobs_per_sec": capacity, "capacity_jobs": n_cap,
            "load_points": load_points(ctx, jobs, capacity, list(loads), seed, 50)}


def forms_leg(ctx, torch, dev, stream, default_ms, reps=2):
    """The sweep's launch forms on the same GPU: the default (one launch per
    E and wave, replayed from a HIP graph) against a persistent grid per
    launch and against direct launches without the graph; and the batched
    form against one launch per realization on the sweep's r = 1 subset
    (2000 realizations, 10 ms batched)."""
    f64 = dict(dtype=torch.float64, device=dev)
    w = synth.workload_sweep()
    X, Y = torch.tensor(w.X, device=dev), torch.tensor(w.Y, device=dev)
    rho = torch.empty((2, len(w.E), len(w.tau), len(w.L), w.r), **f64)

    def sweep(flags, r=w.r, out=rho):
        return lambda: ctx.ccm_sweep_dev(X, Y, w.E, w.tau, w.L, r, w.seed, out, stream=stream,
                                         flags=flags)
    pers, _ = _timed(ctx, torch, sweep(capi.CCM_FLAG_PERSISTENT), reps, False)
    nog, _ = _timed(ctx, torch, sweep(capi.CCM_FLAG_NO_GRAPH), reps, False)
    rho1 = torch.empty((2, len(w.E), len(w.tau), len(w.L), 1), **f64)
    b1, _ = _timed(ctx, torch, sweep(0, 1, rho1), 3, False)
    p1, _ = _timed(ctx, torch, sweep(capi.CCM_FLAG_PLAIN, 1, rho1), 1, False)
    return {"workload": w.name,
            "default_ms": default_ms, "persistent_ms": pers * 1e3, "no_graph_ms": nog * 1e3,
            "persistent_over_default": pers * 1e3 / default_ms,
            "plain_vs_batched": {"subset": "r = 1 (2000 realizations)", "batched_ms": b1 * 1e3,
                                 "plain_ms": p1 * 1e3, "plain_over_batched": p1 / b1}}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(the cross map would shard by realization: each GPU its own share of the "
              "(E, tau, L, r) realizations, rho gathered at the end)", flush=True)
        sys.exit(2)
    import torch

    w = synth.workload_sweep(n=a.n, r=a.r)
    dev = torch.device("cuda:0")
    X = torch.tensor(w.X, device=dev)
    Y = torch.tensor(w.Y, device=dev)
    rho = torch.empty((2, len(w.E), len(w.tau), len(w.L), w.r), dtype=torch.float64,
                      device=dev)
    stream = torch.cuda.current_stream()
    ctx = capi.Context(0)
    if a.serve_protocol:
        loads = [float(v) for v in a.protocol_loads.split(",") if v]
        print(json.dumps({"served_protocol": serve_protocol(ctx, loads=loads)}), flush=True)
        ctx.close()
        return

    def step():
        ctx.ccm_sweep_dev(X, Y, w.E, w.tau, w.L, w.r, w.seed, rho, stream=stream,
                          flags=a.flags)

    ctx.profile_enable(False)
    print(f"bench: warmup {a.warmup} step(s) of {w.name}", file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    for i in range(a.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    el = t1 - t0
    print(f"bench: {a.steps} steps in {el:.3f} s (graph replay)", file=sys.stderr, flush=True)

    # the same steps with every cross-map launch timed by HIP events
    n_prof = max(1, min(a.steps, 5))
    ctx.profile_enable(True)
    step()
    torch.cuda.synchronize()
    ctx.profile_read(reset=True)
    t0 = time.perf_counter()
    for i in range(n_prof):
        step()
    torch.cuda.synchronize()
    el_prof = time.perf_counter() - t0
    prof = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    for k in ("kernel_ms", "launches", "pairs", "flops", "predictions", "realizations",
              "waves"):
        prof[k] = prof[k] / n_prof * a.steps          # per timed region of a.steps steps
    print(f"bench: {n_prof} profiled steps in {el_prof:.3f} s", file=sys.stderr, flush=True)

    if a.copy_mib > 0:
        n = a.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    rh = rho.cpu().numpy()
    if not np.isfinite(rh).all():
        print("bench: warning: non-finite rho values", file=sys.stderr, flush=True)

    preds = prof["predictions"]
    realizations = prof["realizations"]
    kernel_s = prof["kernel_ms"] / 1e3
    achieved_tflops = prof["flops"] / kernel_s / 1e12 if kernel_s > 0 else 0.0
    launches = max(1, prof["launches"])
    out = {
        "metric": "cross-map predictions/sec and rho-realizations/sec",
        "value": preds / el,
        "unit": "predictions/s",
        "rho_realizations_per_sec": realizations / el,
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": el / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "N": w.N, "E": f"{w.E[0]}..{w.E[-1]}",
                   "tau": f"{w.tau[0]}..{w.tau[-1]}", "L": w.L, "r": w.r,
                   "directions": 2, "parallelism": "single GPU",
                   "realizations_per_step": realizations / a.steps,
                   "predictions_per_step": preds / a.steps},
        "roofline": {
            "bound": "alu",
            "kernel": "k_crossmap (fused distance/top-(E+1)/predict/moments)",
            "achieved": achieved_tflops,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": measured_traffic(w.name),
            "launches_per_step": launches / a.steps,
            "avg_launch_ms": prof["kernel_ms"] / launches,
            "kernel_share_of_step": kernel_s / el,
            "pairs_per_step": prof["pairs"] / a.steps,
            "waves_per_step": prof["waves"] / a.steps,
            "kernel_timing": f"HIP events around each cross-map launch, {n_prof} profiled "
                             "steps (direct launches) after the timed graph steps",
            "profiled_ms_per_step": el_prof / n_prof * 1e3,
        },
    }
    if a.workloads:
        legs = set(v for v in a.legs.split(",") if v)
        if "matrix-alone" in legs:
            legs.add("matrix")
        print("bench: other workloads and the elasticity study", file=sys.stderr, flush=True)
        which = tuple(k for k in ("small", "long", "matrix", "matrix-alone") if k in legs)
        if which:
            out["workloads"] = workloads_leg(ctx, torch, dev, stream, which)
        if "elasticity" in legs:
            out["elasticity"] = elasticity_leg(ctx, torch, dev, stream)
        if "index_table" in legs:
            out["index_table"] = table_leg(ctx, torch, dev, stream)
        if "nested" in legs:
            out["nested"] = nested_leg(ctx, torch, dev, stream)
        if "shared_e" in legs:
            out["shared_e"] = shared_e_leg(ctx, torch, dev, stream, out["ms_per_step"])
        if "forms" in legs:
            out["forms"] = forms_leg(ctx, torch, dev, stream, out["ms_per_step"])
    if a.serve_jobs > 0:
        print(f"bench: served leg, {a.serve_jobs} jobs per load", file=sys.stderr, flush=True)
        ctx.profile_enable(False)
        loads = [float(v) for v in a.serve_loads.split(",") if v]
        out["served"] = served_leg(ctx, a.serve_jobs, loads)
    if a.cpu_modulus > 0:
        print("bench: timing the CPU oracle on its sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, rh, modulus=a.cpu_modulus)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
