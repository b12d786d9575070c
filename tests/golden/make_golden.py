"""Write tests/golden/workloads.json: oracle counts of the three full-size
workloads (uniform 2000x1000/20K edges, voting 100x10000/p=0.6, power-law
1Mx300K/8M edges).  Calls only the seeded generators and oracle/ -- never the
HIP library.  Run from the repository root:

    python tests/golden/make_golden.py [--threads N] [--only NAME]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import gen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workloads.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    ap.add_argument("--only", default=None)
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


if __name__ == "__main__":
    main()
