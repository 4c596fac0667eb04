"""Pick the cross-map kernels' launch shapes.

The hot kernel has three shape parameters per E (see ``csrc/ccm_tune.h``):
Q, the queries each lane holds; G, the library candidates evaluated per
trigger check; and W, a minimum of resident wavefronts per SIMD imposed on
the register allocator (0: none).  The E-sweep-sharing scan has the same
three per E_max (``--kind shared``).  All are compile-time, so candidates
are separate builds of the kernel translation unit.  Each build ("column")
gives every E one candidate from that E's list; every column is timed on
the same sweep and each E keeps its fastest candidate.

Two phases, so that compilation stays off the GPU host:

    python -m paper_1905_00565_amd.autotune build          # CPU: compile columns
    python -m paper_1905_00565_amd.autotune time --out T.h  # GPU: time, write table

``time`` runs one child process per column (a process loads one libccm) and
writes the chosen tables as a header in the format of ``csrc/ccm_tune.h``
(the tables of the other kind are kept as they are), plus a JSON report
next to it.  Results do not depend on the shape (the neighbour selection is
exact whatever the visiting order and grouping), so the choice is about
speed alone.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

from . import build as B

TUNE_DIR = os.path.join(B.PKG, "_tune")

# (Q, G) or (Q, G, W) candidates per E; the first is the current table's choice.
CANDIDATES = {
    1: [(3, 16, 7), (3, 16, 6), (2, 16, 7), (3, 12, 7), (2, 24, 6)],
    2: [(4, 12, 6), (4, 12, 7), (3, 12, 7), (4, 8, 7), (3, 16, 6)],
    3: [(4, 8, 6), (4, 8, 7), (3, 8, 7), (4, 6, 7), (3, 12, 6)],
    4: [(4, 6, 6), (4, 6, 7), (3, 6, 7), (4, 4, 7), (3, 8, 6)],
    5: [(3, 6, 6), (3, 6, 7), (2, 6, 7), (3, 4, 7), (2, 8, 6)],
    6: [(2, 4, 7), (3, 4, 6), (3, 4, 7), (2, 6, 6), (3, 3, 7)],
    7: [(2, 3, 7), (2, 4, 6), (2, 4, 7), (2, 6, 6), (1, 6, 8)],
    8: [(2, 4, 6), (2, 3, 6), (2, 3, 7), (1, 4, 8), (2, 2, 7)],
    9: [(2, 4, 6), (2, 3, 6), (2, 3, 7), (1, 4, 8), (2, 2, 7)],
    10: [(2, 3, 6), (2, 3, 7), (2, 2, 7), (1, 4, 8), (1, 3, 8)],
}


# E-sweep sharing, per E_max: (Q, G) or (Q, G, W); the first is the current choice.
SHARED_CANDIDATES = {
    1: [(2, 8), (4, 8), (2, 16), (1, 16), (3, 8)],
    2: [(2, 8), (4, 8), (2, 12), (3, 8), (2, 4)],
    3: [(2, 8), (3, 8), (2, 6), (2, 4), (1, 8)],
    4: [(1, 8), (2, 4), (2, 6), (2, 8), (3, 4)],
    5: [(1, 6), (2, 6), (2, 4), (1, 8), (2, 3)],
    6: [(1, 6), (1, 6, 4), (1, 4, 4), (2, 4), (1, 3)],
    7: [(1, 4), (1, 4, 3), (1, 3, 4), (1, 6), (1, 2)],
    8: [(1, 4), (1, 4, 3), (1, 3, 3), (1, 2), (1, 6)],
    9: [(1, 4), (1, 4, 3), (1, 3, 3), (1, 2), (1, 6)],
    10: [(1, 4, 3), (1, 4), (1, 3, 3), (1, 2), (1, 6)],
}
MACROS = {"default": ("CCM_TUNE_Q", "CCM_TUNE_G", "CCM_TUNE_W"),
          "shared": ("CCM_SHARED_Q", "CCM_SHARED_G", "CCM_SHARED_W")}


def columns(kind="default"):
    """Column k gives every E its k-th candidate (or its last, if it has fewer);
    a candidate is (Q, G) or (Q, G, W)."""
    cand = CANDIDATES if kind == "default" else SHARED_CANDIDATES
    n = max(len(v) for v in cand.values())
    cols = []
    for k in range(n):
        pick = [cand[e][min(k, len(cand[e]) - 1)] for e in range(1, 11)]
        q = [0] + [c[0] for c in pick]
        g = [0] + [c[1] for c in pick]
        w = [0] + [c[2] if len(c) > 2 else 0 for c in pick]
        cols.append((q, g, w))
    return cols


def _brace(v):
    return "{" + ", ".join(str(x) for x in v) + "}"


def _build_column(k, q, g, w, kind="default"):
    mq, mg, mw = MACROS[kind]
    defines = [f"-D{mq}={_brace(q)}", f"-D{mg}={_brace(g)}", f"-D{mw}={_brace(w)}"]
    col = os.path.join(TUNE_DIR, f"col{k}")
    os.makedirs(col, exist_ok=True)
    objs = []
    for src, obj, extra in B.units(defines):
        if extra:                       # a unit that holds kernels: rebuild it
            obj = os.path.join(col, os.path.basename(obj))
            B.compile_unit(src, obj, extra)
        objs.append(obj)
    lib = os.path.join(TUNE_DIR, f"libccm_{k}.so")
    res = subprocess.run([B.hipcc(), f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-o", lib,
                          *objs], capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"link failed on column {k}")
    return lib


def build_columns(jobs: int = 8, kind: str = "default"):
    B.build_library()                       # the other objects, and a current library
    os.makedirs(TUNE_DIR, exist_ok=True)
    cols = columns(kind)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        libs = list(ex.map(lambda a: _build_column(*a, kind),
                           [(k, *c) for k, c in enumerate(cols)]))
    with open(os.path.join(TUNE_DIR, "columns.json"), "w") as f:
        json.dump({"kind": kind, "columns": cols,
                   "libs": [os.path.basename(x) for x in libs]}, f)
    return libs


def time_column(r: int, n: int, kind: str = "default"):
    """Child process: time every E of the sweep (or, for the shared scan, the
    sweep of E = 1..E_max for every E_max) with the library in CCM_LIBRARY."""
    import torch
    from . import capi, synth
    w = synth.workload_sweep(n=n, r=r)
    dev = torch.device("cuda:0")
    X = torch.tensor(w.X, device=dev)
    Y = torch.tensor(w.Y, device=dev)
    ctx = capi.Context(0)
    ctx.profile_enable(True)
    out = {}
    flags = capi.CCM_FLAG_SHARED_E if kind == "shared" else 0
    for e in w.E:
        es = list(range(1, e + 1)) if kind == "shared" else [e]
        rho = torch.empty((2, len(es), len(w.tau), len(w.L), r), dtype=torch.float64, device=dev)
        st = torch.cuda.current_stream()
        ctx.ccm_sweep_dev(X, Y, es, w.tau, w.L, r, w.seed, rho, stream=st, flags=flags)
        torch.cuda.synchronize()
        ctx.profile_read(reset=True)
        ctx.ccm_sweep_dev(X, Y, es, w.tau, w.L, r, w.seed, rho, stream=st, flags=flags)
        torch.cuda.synchronize()
        p = ctx.profile_read(reset=True)
        out[e] = {"ms": p["kernel_ms"], "flops": p["flops"], "rho_sum": float(rho.sum().item())}
        print(f"E={e} {p['kernel_ms']:.2f} ms", file=sys.stderr, flush=True)
    ctx.close()
    print(json.dumps(out), flush=True)


def read_tables(path):
    """The six tables of an existing ccm_tune.h (macro name -> list)."""
    with open(path) as f:
        text = f.read()
    tables = {}
    for name in MACROS["default"] + MACROS["shared"]:
        m = re.search(r"#define " + name + r" \{([^}]*)\}", text)
        tables[name] = [int(x) for x in m.group(1).split(",")]
    return tables


def write_header(path, tables, note):
    q, g, w = (tables[m] for m in MACROS["default"])
    sq, sg, sw = (tables[m] for m in MACROS["shared"])
    text = f"""// ccm_tune.h -- launch shape of the cross-map kernel for each embedding
// dimension E (index 0 unused).  Written by paper_1905_00565_amd/autotune.py
// from timings of the E = 1..10, tau = 1..5 sweep on coupled-logistic series
// ({note}); the build may override any table with -DCCM_TUNE_Q={{...}},
// -DCCM_TUNE_G={{...}} or -DCCM_TUNE_W={{...}} (the tuner does, to time
// candidates).
//
//   kTuneQ[E]  queries per lane (a workgroup of 256 lanes holds 256*Q queries)
//   kTuneG[E]  library candidates per trigger check (one group of G distances
//              per query, then one compare against its running E+1-th key)
//   kTuneW[E]  minimum wavefronts per SIMD the compiler must fit (register
//              budget 512/W per lane); 0 leaves it free
#pragma once

#ifndef CCM_TUNE_Q
#define CCM_TUNE_Q {_brace(q)}
#endif
#ifndef CCM_TUNE_W
#define CCM_TUNE_W {_brace(w)}
#endif
#ifndef CCM_TUNE_G
#define CCM_TUNE_G {_brace(g)}
#endif

// E-sweep sharing: the scan at E_max keeps E_max (E_max + 3) / 2 keys per
// query, so its shape is chosen per E_max (index E_max):
//   kSharedQ  queries per lane;  kSharedG  candidates per trigger check;
//   kSharedW  minimum wavefronts per SIMD (0: free)
#ifndef CCM_SHARED_Q
#define CCM_SHARED_Q {_brace(sq)}
#endif
#ifndef CCM_SHARED_G
#define CCM_SHARED_G {_brace(sg)}
#endif
#ifndef CCM_SHARED_W
#define CCM_SHARED_W {_brace(sw)}
#endif

namespace ccmk {{
constexpr int kTuneQ[11] = CCM_TUNE_Q;
constexpr int kTuneG[11] = CCM_TUNE_G;
constexpr int kTuneW[11] = CCM_TUNE_W;
constexpr int kSharedQ[11] = CCM_SHARED_Q;
constexpr int kSharedG[11] = CCM_SHARED_G;
constexpr int kSharedW[11] = CCM_SHARED_W;
}}  // namespace ccmk
"""
    with open(path, "w") as f:
        f.write(text)


def time_columns(out: str, r: int, n: int, timeout: int):
    with open(os.path.join(TUNE_DIR, "columns.json")) as f:
        meta = json.load(f)
    cols, libs = meta["columns"], meta["libs"]
    kind = meta.get("kind", "default")
    results = []
    for k, lib in enumerate(libs):
        print(f"column {k}: Q={cols[k][0][1:]} G={cols[k][1][1:]} W={cols[k][2][1:]}", flush=True)
        env = dict(os.environ, CCM_LIBRARY=os.path.join(TUNE_DIR, lib))
        res = subprocess.run([sys.executable, "-u", "-m", "paper_1905_00565_amd.autotune",
                              "_child", "--r", str(r), "--n", str(n), "--kind", kind],
                             env=env, capture_output=True, text=True, timeout=timeout,
                             cwd=B.ROOT)
        if res.returncode != 0:
            sys.stderr.write(res.stderr[-4000:])
            raise RuntimeError(f"column {k} failed (exit {res.returncode})")
        results.append({int(e): v for e, v in json.loads(res.stdout.strip().splitlines()[-1]).items()})
    # every column must give the same rho (the shape changes only the speed)
    for e in range(1, 11):
        sums = {results[k][e]["rho_sum"] for k in range(len(results))}
        if len({round(s, 9) for s in sums}) != 1:
            raise RuntimeError(f"rho differs between columns at E={e}: {sums}")
    q, g, wv, report = [0], [0], [0], {}
    for e in range(1, 11):
        ms = [results[k][e]["ms"] for k in range(len(results))]
        best = min(range(len(ms)), key=lambda k: ms[k])
        q.append(cols[best][0][e])
        g.append(cols[best][1][e])
        wv.append(cols[best][2][e])
        report[e] = {"choice": [q[-1], g[-1], wv[-1]], "ms": ms,
                     "candidates": [[cols[k][i][e] for i in range(3)] for k in range(len(cols))],
                     "tflops": results[best][e]["flops"] / ms[best] / 1e9}
    current = os.path.join(B.CSRC, "ccm_tune.h")
    tables = read_tables(out if os.path.exists(out) else current)
    for name, vals in zip(MACROS[kind], (q, g, wv)):
        tables[name] = vals
    write_header(out, tables, f"N = {n}, r = {r} per (E, tau, L)")
    with open(os.path.splitext(out)[0] + ".json", "w") as f:
        json.dump(report, f, indent=1)
    for e in range(1, 11):
        print(f"E={e}: Q={q[e]} G={g[e]} W={wv[e]}  {min(report[e]['ms']):.2f} ms "
              f"({report[e]['tflops']:.1f} TFLOP/s)  candidates ms={['%.2f' % x for x in report[e]['ms']]}")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("phase", choices=["build", "time", "_child"])
    ap.add_argument("--out", default=os.path.join(B.CSRC, "ccm_tune.h"))
    ap.add_argument("--r", type=int, default=250)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--timeout", type=int, default=240)
    ap.add_argument("--kind", choices=["default", "shared"], default="default")
    a = ap.parse_args(argv)
    if a.phase == "build":
        for lib in build_columns(a.jobs, a.kind):
            print("built", lib)
    elif a.phase == "time":
        time_columns(a.out, a.r, a.n, a.timeout)
    else:
        time_column(a.r, a.n, a.kind)


if __name__ == "__main__":
    main()
