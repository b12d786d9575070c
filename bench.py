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
    """Hash of the sources that shape the wedge step's memory traffic (its
    kernels and the planner that cuts the work into pieces)."""
    h = hashlib.sha256()
    for f in ("wedge.hip", "plan.hip", "bbc_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2308_07932_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes of the wedge step (its kernels' launches in one count) from the
    committed rocprofv3 counter summary, if it was taken on the current
    sources; else None."""
    p = os.path.join(ROOT, "profiles", f"wedge_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_hash") != wedge_kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_count")


def host_threads() -> int:
    """Threads the CPU baselines use: the host's cores, at most 16 (the share of
    the host that goes with one GPU)."""
    return max(1, min(os.cpu_count() or 1, 16))


def cpu_baseline(g, W: int, budget_s: float, small: dict):
    """The oracle timed on the host's cores.

    value: the oracle's bucket route (Algorithm 2 in the paper's order, starts
    in parallel as in Algorithm 4) over the whole power-law graph on all host
    threads, W / its wall time (its own relabel and sort included): the same
    wedges the GPU enumerates, so the two rates compare directly.  Beside it:
    the bucket route on one thread and on all threads for the small graphs,
    and the pair enumeration (what the parity tests trust) on all threads,
    whole for the small graphs and over a bounded prefix of U rows of the
    power-law graph, extrapolated by each row's exact inner-loop count."""
    import numpy as np

    import oracle
    th = host_threads()
    t0 = time.perf_counter()
    b, u, w = oracle.bucket(g, threads=th)
    t_bucket = time.perf_counter() - t0
    assert w == W, (w, W)
    small_runs = {}
    for name, gs in small.items():
        row = {}
        for threads in (1, th):
            t0 = time.perf_counter()
            oracle.bucket(gs, threads=threads)
            row[f"bucket_s_{threads}t"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.pair_count(gs, 0, threads=th)
        row[f"pairs_u_side_s_{th}t"] = time.perf_counter() - t0
        small_runs[name] = row
    # pair enumeration over a bounded prefix of U rows, all threads
    deg_v = np.bincount(g.ev, minlength=g.n_v).astype(np.int64)
    row_cost = np.zeros(g.n_u, np.int64)
    np.add.at(row_cost, g.eu, deg_v[g.ev])
    total = int(row_cost.sum())
    csum = np.cumsum(row_cost)
    t0 = time.perf_counter()
    oracle.pair_count_rows(g, 0, 0, 0, threads=th)  # input check + adjacency build only
    setup = time.perf_counter() - t0
    pilot_rows = int(np.searchsorted(csum, min(total, 3e7 * th)))
    t0 = time.perf_counter()
    oracle.pair_count_rows(g, 0, 0, pilot_rows, threads=th)
    tp = max(time.perf_counter() - t0 - setup, 1e-3)
    rate = csum[pilot_rows - 1] / tp if pilot_rows > 0 else 1e8
    rows = int(np.searchsorted(csum, min(total, rate * budget_s)))
    rows = max(1, min(rows, g.n_u))
    t0 = time.perf_counter()
    oracle.pair_count_rows(g, 0, 0, rows, threads=th)
    ts = time.perf_counter() - t0 - setup
    cost = int(csum[rows - 1])
    full_s = setup + ts * total / max(cost, 1)
    log(f"cpu: bucket route {t_bucket:.2f} s on {th} threads (W/s {W / t_bucket:.3g}); pair "
        f"enumeration est. {full_s:.1f} s on {th} threads")
    return {
        "value": W / t_bucket,
        "unit": "wedges/s",
        "cores": th,
        "kind": "oracle",
        "sample": f"whole power-law graph: the oracle's bucket route (Algorithm 2, starts in "
                  f"parallel as in Algorithm 4; its own relabel and sort included) on {th} threads, "
                  f"{t_bucket:.2f} s for the same W the GPU enumerates",
        "bucket_seconds": t_bucket,
        "small_graphs": small_runs,
        "pair_enumeration": {
            "threads": th,
            "sample": f"U rows 0..{rows - 1} of {g.n_u} ({cost:.3g} of {total:.3g} inner steps, "
                      f"{ts:.1f} s)",
            "full_seconds_est": full_s,
            "note": "the pair enumeration does sum-of-degree-squared work, not W; its time is "
                    "extrapolated from the sample by exact per-row step counts",
        },
    }


def bench_small(ctx, name: str, steps: int):
    """Whole bbc_count calls on a small device-resident workload (uniform or
    voting): time per call, the wedge kernel's HIP-event time, and its
    roofline fraction (same algorithmic bytes as the power-law line)."""
    import numpy as np
    import torch

    import gen
    g = gen.workload(name)
    dev = torch.device("cuda:0")
    eu, ev, sg = (torch.from_numpy(x).to(dev) for x in (g.eu, g.ev, g.sign))
    torch.cuda.synchronize()
    for _ in range(5):
        r = ctx.count(eu, ev, sg, g.n_u, g.n_v)
    torch.cuda.synchronize()
    phase = np.zeros(4)
    t0 = time.perf_counter()
    for _ in range(steps):
        r = ctx.count(eu, ev, sg, g.n_u, g.n_v)
        for p in range(4):
            phase[p] += ctx.phase_ms(p)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    phase /= steps
    st = ctx.stats()
    W, m, active = st[2], st[1], st[6]
    alg = 4 * W + 16 * m + 16 * active
    log(f"{name}: {ms:.3f} ms per call (wedge kernel {phase[2] * 1e3:.1f} us), W={W}")
    return {"workload": WORKLOAD_DESC[name], "edges": g.n_edges, "wedges": W,
            "balanced": r.balanced, "ms_per_call": ms, "wedges_per_s": W / (ms * 1e-3),
            "phase_ms": {"prep": phase[1], "plan": phase[3], "wedge_kernel": phase[2]},
            "wedge_kernel_roofline_frac": alg / (phase[2] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes": alg, "steps": steps}


def lds_atomic_peaks():
    """Measured LDS atomic-add ceilings of the device (probe library): adds/s
    for conflict-free u32, scattered u32 and scattered u64 adds."""
    import ctypes
    path = os.path.join(ROOT, "paper_2308_07932_amd", "libbbc_probe.so")
    lib = ctypes.CDLL(path)
    f = lib.bbc_probe_lds_atomics
    f.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_ulonglong)]
    f.restype = ctypes.c_int
    out = {}
    for pat, name in ((0, "u32_conflict_free"), (1, "u32_scattered"), (2, "u64_scattered")):
        r, ms, chk = ctypes.c_double(), ctypes.c_double(), ctypes.c_ulonglong()
        blocks, iters = 1024, 1024
        rc = f(0, pat, blocks, iters, 3, ctypes.byref(r), ctypes.byref(ms), ctypes.byref(chk))
        if rc != 0 or chk.value != blocks * 1024 * iters * 8:
            raise RuntimeError(f"LDS probe pattern {pat} failed (rc {rc})")
        out[name] = r.value
    return out


def bench_per_vertex(ctx, g, eu, ev, sg, r, steps: int):
    """Per-vertex balanced counts (BBC_PER_VERTEX | BBC_OUTPUT_ON_DEVICE) of
    the same device-resident graph: whole calls whose per-vertex array stays in
    device memory.  The output is checked by what holds at any size: each
    balanced butterfly has four vertices, so the counts sum to 4 x the balanced
    total, and the totals equal those of the plain count."""
    import torch
    rr, pv = ctx.count(eu, ev, sg, g.n_u, g.n_v, per_vertex=True,
                       per_vertex_on_device=True)  # warm-up
    torch.cuda.synchronize()
    dev_ms = wedge_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        rr, pv = ctx.count(eu, ev, sg, g.n_u, g.n_v, per_vertex=True, per_vertex_on_device=True)
        dev_ms += ctx.phase_ms(0)
        wedge_ms += ctx.phase_ms(2)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ok_sum = int(pv.sum().item()) == 4 * r.balanced
    log(f"per-vertex: {ms:.3f} ms per call (device {dev_ms / steps:.3f} ms, wedge kernel "
        f"{wedge_ms / steps:.3f} ms); sum = 4 x balanced: {ok_sum}; totals equal: {rr == r}")
    return {"ms_per_call": ms, "device_ms": dev_ms / steps, "wedge_kernel_ms": wedge_ms / steps,
            "wedges_per_s": r.wedges / (ms * 1e-3), "steps": steps,
            "output": f"{g.n_u + g.n_v} int64 counts left in device memory",
            "sum_is_4x_balanced": ok_sum, "totals_equal_plain_count": rr == r}


def bench_batched(ctx, steps: int, warmup: int, oracle_sample: int, plain_loop: bool = True):
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
    # tunables picked by the autotuner on the first 2,000 graphs of the batch
    k = 2000
    t0 = time.perf_counter()
    chosen, _ = ctx.autotune(cat[0][:k], cat[1][:k], cat[2][:k + 1], *te, repeats=2)
    tune_s = time.perf_counter() - t0
    log(f"autotune on {k} graphs ({tune_s:.1f}s): {chosen}")
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
    # the same batch again with the two pipeline segments replayed as HIP graphs
    ctx.set_param(bbc.PARAM_GRAPHS, 1)
    for _ in range(warmup):
        rg = ctx.count_batch(*cat[:3], *te)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rg = ctx.count_batch(*cat[:3], *te)
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / steps
    graph_equal = all(np.array_equal(a, b) for a, b in zip(res, rg))
    ctx.set_param(bbc.PARAM_GRAPHS, 0)
    # a small batch (the 256 graphs with the fewest edges), where launches
    # dominate: eager calls vs graph replay
    small_idx = np.argsort(np.diff(off), kind="stable")[:256]
    sg_ = [graphs[i] for i in sorted(small_idx)]
    scat = bbc.concat_graphs(sg_)
    ste = [torch.from_numpy(x).to(dev) for x in scat[3:]]
    torch.cuda.synchronize()
    small_ms = {}
    for mode in (0, 1):
        ctx.set_param(bbc.PARAM_GRAPHS, mode)
        for _ in range(3):
            ctx.count_batch(*scat[:3], *ste)
        t0 = time.perf_counter()
        for _ in range(50):
            ctx.count_batch(*scat[:3], *ste)
        small_ms[mode] = (time.perf_counter() - t0) * 1e3 / 50
    ctx.set_param(bbc.PARAM_GRAPHS, 0)
    # plain loop: one bbc_count per graph, same device-resident edges
    t0 = time.perf_counter()
    plain_equal = True
    for i, g in enumerate(graphs if plain_loop else []):
        a, b = int(off[i]), int(off[i + 1])
        if a == b:
            continue
        r = ctx.count(te[0][a:b], te[1][a:b], te[2][a:b], g.n_u, g.n_v)
        plain_equal &= r == res.result(i)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0 if plain_loop else float("nan")
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
    bench_batched.graphs = graphs
    bench_batched.results = [res.result(i) for i in range(len(graphs))]
    return {
        "workload": "20,000 signed bipartite graphs, |U|,|V| log-uniform in [16, 4096], density "
                    "log-uniform in [1e-3, 0.2], P(sign=-1)=0.3, seeds 4 / 10000+i",
        "graphs": len(graphs), "edges": int(off[-1]), "wedges": W,
        "graphs_per_s": len(graphs) / (ms * 1e-3), "ms_per_batch": ms,
        "wedges_per_s": W / (ms * 1e-3),
        "phase_ms": {"prep": phase[1], "plan": phase[3], "wedge_kernel": phase[2]},
        "work_items": st[4], "autotuned": chosen, "autotune_s": tune_s,
        "graph_replay_ms_per_batch": ms_graph,
        "graph_replay_graphs_per_s": len(graphs) / (ms_graph * 1e-3),
        "graph_replay_results_equal": bool(graph_equal),
        "small_batch_256": {"edges": int(scat[2][-1]), "eager_ms": small_ms[0],
                            "graph_replay_ms": small_ms[1]},
        "plain_loop_graphs_per_s": len(graphs) / plain_s if plain_loop else None,
        "plain_loop_s": plain_s if plain_loop else None,
        "speedup_vs_plain_loop": plain_s / (ms * 1e-3) if plain_loop else None,
        "plain_loop_results_equal": bool(plain_equal),
        "oracle_sample_exact": f"{ok}/{len(sample)}",
    }


def bench_serving(small_graphs, small_results, n_templates: int, n_requests: int,
                  load: float, seed: int = 99):
    """Serving: a Poisson stream of jobs, 80% small graphs of the batched
    workload and 20% large Chung-Lu graphs (sides log-uniform in [1e5, 2e6],
    edges log-uniform in [1e6, 3e7], P(-1) uniform in [0.1, 0.4]), submitted
    to a bbc_server at a rate that keeps the device about `load` busy; reports
    latency percentiles (submission to result) and completed graphs/s, and
    checks every result against the same graph counted alone."""
    import threading

    import numpy as np

    import gen
    import paper_2308_07932_amd as bbc
    t0 = time.perf_counter()
    params = gen.serving_large_params(n_templates)
    large = [gen.chung_lu_graph_fast(sd, nu, nv, m, p_neg=pn) for sd, nu, nv, m, pn in params]
    log(f"serving: {len(large)} large job graphs ({sum(g.n_edges for g in large)} edges) generated "
        f"in {time.perf_counter() - t0:.1f}s")
    # each large graph alone (its reference result and its service time)
    ctx = bbc.Context(0)
    alone, t_alone = [], []
    for g in large:
        ctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v)  # warm the workspace
        t1 = time.perf_counter()
        alone.append(ctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v))
        t_alone.append(time.perf_counter() - t1)
    ctx.close()
    mean_large = float(np.mean(t_alone))
    rate = load / (0.2 * mean_large)  # requests/s; small jobs cost little next to large ones
    rng = np.random.default_rng(seed)
    kinds = rng.random(n_requests) < 0.8
    pick = np.where(kinds, rng.integers(0, len(small_graphs), n_requests),
                    rng.integers(0, len(large), n_requests))
    gaps = rng.exponential(1.0 / rate, n_requests)
    results = [None] * n_requests
    with bbc.Server(0, large_workers=2) as srv:
        # warm the workers' workspaces on the largest graph and a small batch
        big = max(large, key=lambda g: g.n_edges)
        srv.poll(srv.submit(big.eu, big.ev, big.sign, big.n_u, big.n_v))
        tickets = [None] * n_requests

        def feed():
            t_next = time.perf_counter()
            for i in range(n_requests):
                t_next += gaps[i]
                d = t_next - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                g = small_graphs[pick[i]] if kinds[i] else large[pick[i]]
                tickets[i] = srv.submit(g.eu, g.ev, g.sign, g.n_u, g.n_v)

        t_start = time.perf_counter()
        th = threading.Thread(target=feed)
        th.start()
        th.join()
        for i in range(n_requests):
            results[i] = srv.poll(tickets[i], wait_ms=-1)
        t_end = time.perf_counter()
        st = srv.stats()
    lat = np.array([r.latency_ms for r in results])
    exact = 0
    for i, r in enumerate(results):
        want = small_results[pick[i]] if kinds[i] else alone[pick[i]]
        exact += r.status == bbc.OK and r.result == want
    ls, ll = lat[kinds], lat[~kinds]
    out = {
        "workload": "Poisson arrivals; 80% graphs of the batched workload, 20% Chung-Lu graphs with "
                    "|U|,|V| log-uniform in [1e5, 2e6], edges log-uniform in [1e6, 3e7], P(-1) "
                    f"uniform in [0.1, 0.4] ({len(large)} drawn graphs reused)",
        "requests": n_requests, "rate_per_s": rate, "target_load": load,
        "graphs_per_s": n_requests / (t_end - t_start),
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "small_p50_ms": float(np.percentile(ls, 50)) if ls.size else None,
        "small_p99_ms": float(np.percentile(ls, 99)) if ls.size else None,
        "large_p50_ms": float(np.percentile(ll, 50)) if ll.size else None,
        "large_p99_ms": float(np.percentile(ll, 99)) if ll.size else None,
        "large_alone_mean_ms": mean_large * 1e3,
        "batches": st["batches"], "max_batch": st["max_batch"], "peak_running": st["peak_running"],
        "peak_reserved_bytes": st["peak_reserved"],
        "exact_vs_alone": f"{exact}/{n_requests}",
    }
    log(f"serving: {n_requests} requests at {rate:.0f}/s: {out['graphs_per_s']:.0f} graphs/s, p50 "
        f"{out['p50_ms']:.2f} ms, p99 {out['p99_ms']:.2f} ms; exact {exact}/{n_requests}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="powerlaw", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-per-vertex", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the uniform and voting graphs")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--only-batched", action="store_true",
                    help="run the batched workload alone (for profiling); its line reports graphs/s")
    ap.add_argument("--no-plain-loop", action="store_true",
                    help="skip the per-graph loop of the batched workload")
    ap.add_argument("--serving-requests", type=int, default=1500)
    ap.add_argument("--serving-load", type=float, default=0.8)
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

    if args.only_batched:
        ctx = bbc.Context(0, stream=torch.cuda.current_stream().cuda_stream)
        ctx.set_timing(True)
        b = bench_batched(ctx, args.batched_steps, 1, 24, plain_loop=not args.no_plain_loop)
        print(json.dumps({"metric": "batched graphs/sec (1 GPU)", "value": b["graphs_per_s"],
                          "unit": "graphs/s", "n_gpus": 1, "steps": args.batched_steps, "warmup": 1,
                          "ms_per_step": b["ms_per_batch"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                          "data": "synthetic", "config": {"workload": b["workload"]},
                          "batched": b}), flush=True)
        ctx.close()
        return

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
    phase = np.zeros(5)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = ctx.count(eu, ev, sg, g.n_u, g.n_v)
        for p in range(5):
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

    # algorithmic bytes of the wedge step: 4 B per wedge (one CSR entry),
    # 16 B per middle record, 16 B per active start
    alg_bytes = 4 * W + 16 * m + 16 * active
    achieved = alg_bytes / (phase[2] * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)
    out = {
        "metric": "wedges/sec + total count time (1 GPU); batched graphs/sec and p50/p99 latency",
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
                     "pipeline": phase[0], "short_wedge_lists": phase[4]},
        "work": {"work_items": st[4], "heavy_pieces": st[7], "resplit_pieces": st[5],
                 "tile_pieces": {"dense_32bit": st[8], "dense_16bit_2_tiles": st[9],
                                 "dense_8bit_4_tiles": st[11], "dense_4bit_8_tiles": st[12],
                                 "hashed_runs": st[10]},
                 "one_wave_pieces": st[13]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "wedge step: bbc::k_wedge_pieces<false> (dense pieces), "
                               "k_wedge_pieces<true> (hashed), k_wedge_wave (one-wave pieces), "
                               "k_wedge (light items), one launch each per count",
                     "algorithmic_bytes_per_launch": alg_bytes,
                     # the planner's bucketing of the wedges through short middle
                     # rows (k_short_wedges, timed as its own phase) also reads
                     # wedges: the fraction with its time added to the step's
                     "frac_with_short_wedge_lists":
                         alg_bytes / ((phase[2] + phase[4]) * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    peaks = lds_atomic_peaks()
    adds = W / (phase[2] * 1e-3)  # one LDS add per wedge
    out["lds_atomics"] = {
        "achieved_adds_per_s": adds,
        "peak_adds_per_s": peaks,
        "frac_of_u32_scattered": adds / peaks["u32_scattered"],
        "probe": "1024 workgroups of 1024 threads, each with a 128 KiB LDS table, non-returning "
                 "ds_add (libbbc_probe.so)",
    }
    log(f"LDS adds: achieved {adds:.3g}/s; probe peaks {peaks}")
    if not args.no_small:
        out["configs"] = {name: bench_small(ctx, name, 50) for name in ("uniform", "voting")}
    if not args.no_per_vertex:
        out["per_vertex"] = bench_per_vertex(ctx, g, eu, ev, sg, r, 5)
    if not args.no_batched:
        out["batched"] = bench_batched(ctx, args.batched_steps, 1, 24)
        if not args.no_serving:
            out["serving"] = bench_serving(bench_batched.graphs, bench_batched.results, 4,
                                           args.serving_requests, args.serving_load)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(g, W, args.cpu_seconds,
                                           {n: gen.workload(n) for n in ("uniform", "voting")})
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
