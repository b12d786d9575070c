#!/usr/bin/env python3
"""Benchmark: single-graph balanced-butterfly count on one MI355X.

One step = one full bbc_count call on a device-resident signed edge list:
validation, degree-priority relabel, signed CSR build, planning, wedge
enumeration with bucket counting, and the read-back of the exact counts.
The metric is wedges/s = W / (time per step), W being the number of
priority-filtered wedges the count enumerates (returned exactly by the call).

Prints ONE JSON line on stdout; details go to stderr.

    python bench.py [--steps K] [--warmup W] [--workload powerlaw|voting|uniform]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

WORKLOAD_DESC = {
    "powerlaw": "power-law rating graph, Chung-Lu Zipf(2.1) degrees, |U|=1,000,000 |V|=300,000, "
                "8,000,000 distinct edges, P(sign=-1)=0.2, seed 3",
    "voting": "dense voting graph, |U|=100 |V|=10,000, edge p=0.6, P(-1)=0.9*Beta(2,2) per voter, seed 2",
    "uniform": "uniform random graph, |U|=2000 |V|=1000, 20,000 distinct edges, P(-1)=0.3, seed 1",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def wedge_kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("wedge.hip", "bbc_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2308_07932_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per wedge-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", f"wedge_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_hash") != wedge_kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(g, W: int, budget_s: float):
    """Time the CPU oracle (pair enumeration, one thread) on a bounded sample of
    rows of side U and extrapolate to the whole graph by the exact inner-loop
    count of each row (sum of the degrees of its neighbours)."""
    import numpy as np

    import oracle
    deg_v = np.bincount(g.ev, minlength=g.n_v).astype(np.int64)
    row_cost = np.zeros(g.n_u, np.int64)
    np.add.at(row_cost, g.eu, deg_v[g.ev])
    total = int(row_cost.sum())
    csum = np.cumsum(row_cost)
    t0 = time.perf_counter()
    oracle.pair_count_rows(g, 0, 0, 0)  # input check + adjacency build only
    setup = time.perf_counter() - t0
    pilot_rows = int(np.searchsorted(csum, min(total, 3e7)))
    t0 = time.perf_counter()
    oracle.pair_count_rows(g, 0, 0, pilot_rows)
    tp = max(time.perf_counter() - t0 - setup, 1e-3)
    rate = csum[pilot_rows - 1] / tp if pilot_rows > 0 else 1e8
    want = min(total, rate * budget_s)
    rows = int(np.searchsorted(csum, want))
    rows = max(1, min(rows, g.n_u))
    t0 = time.perf_counter()
    oracle.pair_count_rows(g, 0, 0, rows)
    ts = time.perf_counter() - t0 - setup
    cost = int(csum[rows - 1])
    full_s = setup + ts * total / max(cost, 1)
    return {
        "value": W / full_s,
        "unit": "wedges/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"oracle pair enumeration over U rows 0..{rows - 1} of {g.n_u} "
                  f"({cost:.3g} of {total:.3g} inner steps, {ts:.1f} s, 1 thread); "
                  f"extrapolated full oracle time {full_s:.1f} s incl. {setup:.1f} s setup",
        "oracle_full_seconds_est": full_s,
    }


def bench_batched(ctx, steps: int, warmup: int, oracle_sample: int):
    """The batched workload: 20,000 graphs (sides log-uniform in [16, 4096],
    density log-uniform in [1e-3, 0.2], P(-1)=0.3) counted by one
    bbc_count_batch call per step, against a plain loop of one bbc_count call
    per graph over the same device-resident edges."""
    import numpy as np
    import torch

    import gen
    import paper_2308_07932_amd as bbc
    t0 = time.perf_counter()
    nu, nv, ne = gen.batch_graph_params(20000)
    graphs = [gen.batch_graph(i, nu[i], nv[i], ne[i]) for i in range(len(nu))]
    cat = bbc.concat_graphs(graphs)
    off = cat[2]
    log(f"batched workload: {len(graphs)} graphs, {int(off[-1])} edges, generated in "
        f"{time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    te = [torch.from_numpy(x).to(dev) for x in cat[3:]]
    torch.cuda.synchronize()
    for _ in range(warmup):
        res = ctx.count_batch(*cat[:3], *te)
    torch.cuda.synchronize()
    phase = np.zeros(4)
    t0 = time.perf_counter()
    for _ in range(steps):
        res = ctx.count_batch(*cat[:3], *te)
        for p in range(4):
            phase[p] += ctx.phase_ms(p)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    phase /= steps
    st = ctx.stats()
    assert (res.status == bbc.OK).all()
    W = int(res.wedges.sum())
    # plain loop: one bbc_count per graph, same device-resident edges
    t0 = time.perf_counter()
    plain_equal = True
    for i, g in enumerate(graphs):
        a, b = int(off[i]), int(off[i + 1])
        if a == b:
            continue
        r = ctx.count(te[0][a:b], te[1][a:b], te[2][a:b], g.n_u, g.n_v)
        plain_equal &= r == res.result(i)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    # exactness against the oracle on a seeded sample of graphs
    from oracle.gram import gram_count

    import oracle
    rng = np.random.default_rng(12345)
    sample = rng.choice(len(graphs), size=oracle_sample, replace=False)
    ok = 0
    for i in sample:
        g = graphs[i]
        if g.n_edges == 0:
            want = (0, 0)
        elif min(g.n_u, g.n_v) <= 2048:
            want = gram_count(g)
        else:
            want = oracle.count(g)
        ok += (int(res.balanced[i]), int(res.unbalanced[i])) == want
    log(f"batched: {ms:.2f} ms per batch ({len(graphs) / ms * 1e3:.0f} graphs/s); plain loop "
        f"{plain_s:.2f} s ({len(graphs) / plain_s:.0f} graphs/s), equal={plain_equal}; oracle sample "
        f"{ok}/{len(sample)}")
    return {
        "workload": "20,000 signed bipartite graphs, |U|,|V| log-uniform in [16, 4096], density "
                    "log-uniform in [1e-3, 0.2], P(sign=-1)=0.3, seeds 4 / 10000+i",
        "graphs": len(graphs), "edges": int(off[-1]), "wedges": W,
        "graphs_per_s": len(graphs) / (ms * 1e-3), "ms_per_batch": ms,
        "wedges_per_s": W / (ms * 1e-3),
        "phase_ms": {"prep": phase[1], "plan": phase[3], "wedge_kernel": phase[2]},
        "work_items": st[4], "plain_loop_graphs_per_s": len(graphs) / plain_s,
        "plain_loop_s": plain_s, "speedup_vs_plain_loop": plain_s / (ms * 1e-3),
        "plain_loop_results_equal": bool(plain_equal),
        "oracle_sample_exact": f"{ok}/{len(sample)}",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="powerlaw", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=3)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build counts one graph per GPU and has no "
              "multi-GPU path (see DESIGN.md for how it would shard).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2308_07932_amd as bbc

    t0 = time.perf_counter()
    g = gen.workload(args.workload)
    log(f"generated {g.name}: n_u={g.n_u} n_v={g.n_v} m={g.n_edges} in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    eu = torch.from_numpy(g.eu).to(dev)
    ev = torch.from_numpy(g.ev).to(dev)
    sg = torch.from_numpy(g.sign).to(dev)
    torch.cuda.synchronize()

    ctx = bbc.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    ctx.set_timing(True)
    for _ in range(args.warmup):
        r = ctx.count(eu, ev, sg, g.n_u, g.n_v)
    torch.cuda.synchronize()
    phase = np.zeros(4)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = ctx.count(eu, ev, sg, g.n_u, g.n_v)
        for p in range(4):
            phase[p] += ctx.phase_ms(p)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    phase /= args.steps
    st = ctx.stats()
    W, m, active = st[2], st[1], st[6]
    log(f"result balanced={r.balanced} unbalanced={r.unbalanced} wedges={r.wedges}")
    log(f"per step {ms:.3f} ms; device phases (ms): pipeline {phase[0]:.3f}, prep {phase[1]:.3f}, "
        f"plan {phase[3]:.3f}, wedge kernel {phase[2]:.3f}; items={st[4]} heavy_pieces={st[7]} "
        f"resplit_pieces={st[5]} active_starts={active}")

    # algorithmic bytes of the wedge kernel: 4 B per wedge (one CSR entry),
    # 16 B per middle record, 16 B per active start
    alg_bytes = 4 * W + 16 * m + 16 * active
    achieved = alg_bytes / (phase[2] * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)
    out = {
        "metric": "wedges/sec + total count time (1 GPU)",
        "value": W / (ms * 1e-3),
        "unit": "wedges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_DESC[args.workload], "n_u": g.n_u, "n_v": g.n_v,
                   "edges": g.n_edges, "wedges": W, "balanced": r.balanced,
                   "unbalanced": r.unbalanced, "parallelism": "single GPU"},
        "total_count_time_ms": ms,
        "phase_ms": {"prep": phase[1], "plan": phase[3], "wedge_kernel": phase[2],
                     "pipeline": phase[0]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": "bbc::k_wedge",
                     "algorithmic_bytes_per_launch": alg_bytes},
    }
    if not args.no_batched:
        out["batched"] = bench_batched(ctx, args.batched_steps, 1, 24)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(g, W, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
