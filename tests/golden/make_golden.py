"""Write the stored expected values under tests/golden/ from the oracle alone.

Calls only the seeded generators (gen/) and oracle/ -- never the HIP library.
Run from the repository root:

    python tests/golden/make_golden.py [--threads N] [--only NAME]

NAME (default: all of them):
  uniform, voting, powerlaw  workloads.json: balanced and unbalanced counts (pair
                             enumeration on both sides, which must agree) and W
                             (explicit enumeration of the priority-filtered wedges)
  batched                    batched_counts.csv.gz: per graph of the 20,000-graph
                             batched workload, balanced and unbalanced counts from
                             the Gram closed form and W by enumeration
  voting_pv                  voting_per_vertex.txt.gz: balanced butterflies containing
                             each vertex of the voting graph (U then V), all 10,100
  powerlaw_pv                workloads.json["powerlaw_per_vertex"]: SHA-256 of the
                             power-law graph's 1.3M per-vertex counts (little-endian
                             int64, U then V), their sum, and spot entries
"""
import argparse
import gzip
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import gen  # noqa: E402
import oracle  # noqa: E402
from oracle.gram import gram_count  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "workloads.json")
BATCHED = os.path.join(HERE, "batched_counts.csv.gz")
VOTING_PV = os.path.join(HERE, "voting_per_vertex.txt.gz")
ALL = ("uniform", "voting", "powerlaw", "batched", "voting_pv", "powerlaw_pv")


def per_vertex_digest(pv: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(pv, dtype="<i8").tobytes()).hexdigest()


def spot_indices(g, pv: np.ndarray, count: int = 48):
    """Vertices whose counts are stored one by one: the largest counts, the
    highest degrees on each side, a seeded random sample, and a few zeros."""
    n = g.n_u + g.n_v
    deg = np.bincount(np.concatenate([g.eu, g.ev.astype(np.int64) + g.n_u]), minlength=n)
    rng = np.random.default_rng(99)
    pick = set(np.argsort(-pv.astype(np.int64), kind="stable")[:count // 4].tolist())
    pick |= set(np.argsort(-deg[:g.n_u], kind="stable")[:count // 8].tolist())
    pick |= set((g.n_u + np.argsort(-deg[g.n_u:], kind="stable")[:count // 8]).tolist())
    pick |= set(rng.integers(0, n, size=count // 4).tolist())
    pick |= set(np.flatnonzero(pv == 0)[:4].tolist())
    return sorted(int(x) for x in pick)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    ap.add_argument("--only", default=None, choices=ALL)
    args = ap.parse_args()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in ("uniform", "voting", "powerlaw"):
        if args.only and name != args.only:
            continue
        g = gen.workload(name)
        t0 = time.time()
        bal, unb = oracle.count(g, threads=args.threads)   # both sides, must agree
        w = oracle.wedges(g, threads=args.threads)
        data[name] = {
            "graph": g.name,
            "n_u": g.n_u, "n_v": g.n_v, "n_edges": g.n_edges,
            "negative_edges": int(np.sum(g.sign < 0)),
            "balanced": bal, "unbalanced": unb, "wedges": w,
            "oracle_seconds": round(time.time() - t0, 1),
            "oracle_threads": args.threads,
            "writer": "tests/golden/make_golden.py (oracle.count both sides + oracle.wedges)",
        }
        print(name, data[name], flush=True)
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)

    if args.only in (None, "batched"):
        t0 = time.time()
        nu, nv, ne = gen.batch_graph_params(20000)
        with gzip.open(BATCHED, "wt") as f:
            f.write("# per graph i of the batched workload (gen.batch_graph_params(20000), "
                    "gen.batch_graph(i, ...)): balanced and unbalanced butterflies from the Gram "
                    "closed form (oracle.gram), W by enumeration (oracle.wedges); written by "
                    "tests/golden/make_golden.py\n")
            f.write("graph,n_u,n_v,n_edges,balanced,unbalanced,wedges\n")
            for i in range(len(nu)):
                g = gen.batch_graph(i, nu[i], nv[i], ne[i])
                bal, unb = gram_count(g) if g.n_edges else (0, 0)
                w = oracle.wedges(g, threads=args.threads) if g.n_edges else 0
                f.write(f"{i},{g.n_u},{g.n_v},{g.n_edges},{bal},{unb},{w}\n")
                if i % 1000 == 999:
                    print(f"batched: {i + 1} graphs, {time.time() - t0:.0f}s", flush=True)
        print(f"batched: done in {time.time() - t0:.0f}s", flush=True)

    if args.only in (None, "voting_pv"):
        g = gen.workload("voting")
        t0 = time.time()
        pv = oracle.per_vertex(g, threads=args.threads)
        with gzip.open(VOTING_PV, "wt") as f:
            f.write(f"# {g.name}: balanced butterflies containing each vertex, U (0..{g.n_u - 1}) "
                    f"then V; oracle.per_vertex; written by tests/golden/make_golden.py\n")
            f.write("\n".join(str(int(x)) for x in pv) + "\n")
        print(f"voting_pv: sum {int(pv.sum())} in {time.time() - t0:.0f}s", flush=True)

    if args.only in (None, "powerlaw_pv"):
        g = gen.workload("powerlaw")
        t0 = time.time()
        pv = oracle.per_vertex(g, threads=args.threads).astype(np.int64)
        idx = spot_indices(g, pv)
        data["powerlaw_per_vertex"] = {
            "graph": g.name,
            "sha256_le_int64": per_vertex_digest(pv),
            "sum": int(pv.sum()),
            "nonzero": int(np.count_nonzero(pv)),
            "spot": {str(i): int(pv[i]) for i in idx},
            "oracle_seconds": round(time.time() - t0, 1),
            "oracle_threads": args.threads,
            "writer": "tests/golden/make_golden.py (oracle.per_vertex)",
        }
        print("powerlaw_pv", {k: v for k, v in data["powerlaw_per_vertex"].items() if k != "spot"},
              flush=True)
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
