"""Full-size parity of the batched and per-vertex paths against stored oracle
values (tests/golden/, written by tests/golden/make_golden.py from the oracle
and the seeded generators alone):

* every one of the 20,000 graphs of the batched workload, in one
  bbc_count_batch call on device-resident edges, exactly as the benchmark
  counts it: balanced, unbalanced and W per graph, element by element;
* the voting graph's per-vertex counts (Section 5.1), all 10,100 of them;
* the power-law graph's 1.3M per-vertex counts: SHA-256 of the whole vector,
  its sum and nonzero count, and stored spot entries.
"""
import gzip
import hashlib
import json
import os

import numpy as np
import pytest

import gen
import paper_2308_07932_amd as bbc

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    c = bbc.Context(0)
    yield c
    c.close()


def load_batched_golden():
    rows = []
    with gzip.open(os.path.join(GOLDEN, "batched_counts.csv.gz"), "rt") as f:
        for line in f:
            if line.startswith("#") or line.startswith("graph,"):
                continue
            rows.append([int(x) for x in line.split(",")])
    a = np.array(rows, dtype=np.int64)
    assert a.shape == (20000, 7) and (a[:, 0] == np.arange(20000)).all()
    return a


def test_full_batched_workload_matches_golden(ctx):
    import torch
    gold = load_batched_golden()
    nu, nv, ne = gen.batch_graph_params(20000)
    graphs = [gen.batch_graph(i, nu[i], nv[i], ne[i]) for i in range(len(nu))]
    assert [g.n_u for g in graphs] == gold[:, 1].tolist()
    assert [g.n_v for g in graphs] == gold[:, 2].tolist()
    assert [g.n_edges for g in graphs] == gold[:, 3].tolist()
    cat = bbc.concat_graphs(graphs)
    del graphs
    dev = torch.device("cuda:0")
    te = [torch.from_numpy(x).to(dev) for x in cat[3:]]
    torch.cuda.synchronize()
    print(f"[gpu] batched workload: 20000 graphs, {int(cat[2][-1])} edges", flush=True)
    res = ctx.count_batch(*cat[:3], *te)
    assert (res.status == bbc.OK).all()
    assert np.array_equal(res.balanced, gold[:, 4])
    assert np.array_equal(res.unbalanced, gold[:, 5])
    assert np.array_equal(res.wedges, gold[:, 6])


def test_voting_per_vertex_matches_golden(ctx):
    with gzip.open(os.path.join(GOLDEN, "voting_per_vertex.txt.gz"), "rt") as f:
        want = np.array([int(x) for x in f if not x.startswith("#")], dtype=np.int64)
    g = gen.workload("voting")
    assert want.shape == (g.n_u + g.n_v,)
    gold = json.load(open(os.path.join(GOLDEN, "workloads.json")))["voting"]
    print(f"[gpu] per-vertex {g.name}", flush=True)
    r, pv = ctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v, per_vertex=True)
    assert (r.balanced, r.unbalanced, r.wedges) == (gold["balanced"], gold["unbalanced"],
                                                    gold["wedges"])
    assert np.array_equal(pv, want)


def test_powerlaw_per_vertex_matches_golden(ctx):
    gold = json.load(open(os.path.join(GOLDEN, "workloads.json")))
    want = gold["powerlaw_per_vertex"]
    g = gen.workload("powerlaw")
    print(f"[gpu] per-vertex {g.name}", flush=True)
    r, pv = ctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v, per_vertex=True)
    assert r.balanced == gold["powerlaw"]["balanced"]
    assert pv.shape == (g.n_u + g.n_v,)
    for i, v in want["spot"].items():
        assert int(pv[int(i)]) == v, i
    assert int(pv.sum()) == want["sum"] == 4 * r.balanced
    assert int(np.count_nonzero(pv)) == want["nonzero"]
    digest = hashlib.sha256(np.ascontiguousarray(pv, dtype="<i8").tobytes()).hexdigest()
    assert digest == want["sha256_le_int64"]
