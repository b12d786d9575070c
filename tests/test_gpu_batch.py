"""Batched counting (bbc_count_batch) on the GPU: every graph of a batch must
get exactly what the oracle gives for it alone (balanced, unbalanced and W),
and invalid graphs must not disturb the others."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import gen
import oracle
from oracle.gram import gram_count
import paper_2308_07932_amd as bbc
from gen import SignedBipartiteGraph

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    c = bbc.Context(0)
    yield c
    c.close()


def expect(g):
    if g.n_edges == 0:
        return bbc.Result(0, 0, 0)
    b, u = oracle.count(g)
    return bbc.Result(b, u, oracle.wedges(g))


def mixed_graphs(seed: int, count: int):
    """Small graphs of varied shapes: random densities, stars, complete
    bipartite graphs with switched signs, tiny and empty ones."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = i % 6
        if kind == 0:
            out.append(gen.random_graph(rng, int(rng.integers(1, 60)), int(rng.integers(1, 60)),
                                        float(rng.uniform(0.02, 0.6)), p_neg=float(rng.uniform(0, 1))))
        elif kind == 1:
            a, b = int(rng.integers(1, 12)), int(rng.integers(1, 12))
            out.append(gen.complete_graph(a, b, rng.choice([1, -1], a), rng.choice([1, -1], b)))
        elif kind == 2:
            nu, nv = int(rng.integers(50, 400)), int(rng.integers(50, 400))
            m = int(rng.integers(0, min(nu * nv, 6000)))
            out.append(gen.uniform_graph(seed=1000 + i, n_u=nu, n_v=nv, n_edges=m, p_neg=0.3))
        elif kind == 3:  # a hub on each side
            nu, nv = int(rng.integers(2, 200)), int(rng.integers(2, 200))
            eu = np.concatenate([np.zeros(nv, np.int32), np.arange(1, nu, dtype=np.int32)])
            ev = np.concatenate([np.arange(nv, dtype=np.int32), np.zeros(nu - 1, np.int32)])
            s = rng.choice([1, -1], eu.shape[0]).astype(np.int8)
            out.append(SignedBipartiteGraph(nu, nv, eu, ev, s, f"hubs{i}"))
        elif kind == 4:  # no edges, sizes arbitrary
            out.append(SignedBipartiteGraph(int(rng.integers(0, 30)), int(rng.integers(0, 30)),
                                            np.zeros(0, np.int32), np.zeros(0, np.int32),
                                            np.zeros(0, np.int8), f"empty{i}"))
        else:  # a dense block in a wider graph: heavy starts with many middles
            nu, nv = int(rng.integers(300, 2000)), int(rng.integers(30, 120))
            g = gen.random_graph(rng, nu, nv, float(rng.uniform(0.2, 0.7)), p_neg=0.4)
            out.append(g)
    return out


def run_batch(ctx, graphs):
    print(f"[gpu] batch of {len(graphs)} graphs, {sum(g.n_edges for g in graphs)} edges", flush=True)
    return ctx.count_batch(*bbc.concat_graphs(graphs))


def test_batch_matches_oracle_and_single_counts(ctx):
    graphs = mixed_graphs(7, 240)
    res = run_batch(ctx, graphs)
    assert (res.status == bbc.OK).all()
    for i, g in enumerate(graphs):
        want = expect(g)
        assert res.result(i) == want, (i, g.name, res.result(i), want)
        if i % 10 == 0 and g.n_edges:
            assert ctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v) == want


def test_batch_of_one_and_repeated_calls(ctx):
    graphs = mixed_graphs(8, 60)
    first = run_batch(ctx, graphs)
    again = run_batch(ctx, graphs)
    for a, b in zip(first, again):
        assert np.array_equal(a, b)
    one = run_batch(ctx, graphs[5:6])
    assert one.result(0) == first.result(5)
    empty = ctx.count_batch(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(1, np.int64),
                            np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int8))
    assert empty.status.shape == (0,)


def test_batch_isolates_invalid_graphs(ctx):
    graphs = mixed_graphs(9, 48)
    bad = {}
    g = graphs[2]
    assert g.n_edges > 3
    ev = g.ev.copy()
    ev[1] = g.n_v  # out of range
    graphs[2] = g._replace(ev=ev)
    bad[2] = bbc.VERTEX_RANGE
    g = graphs[8]
    s = g.sign.copy()
    s[0] = 0
    graphs[8] = g._replace(sign=s)
    bad[8] = bbc.BAD_SIGN
    g = graphs[14]
    graphs[14] = g._replace(eu=np.append(g.eu, g.eu[0]), ev=np.append(g.ev, g.ev[0]),
                            sign=np.append(g.sign, np.int8(-g.sign[0])))
    bad[14] = bbc.DUPLICATE_EDGE
    g = graphs[20]
    eu = g.eu.copy()
    eu[-1] = -3
    graphs[20] = g._replace(eu=eu)
    bad[20] = bbc.VERTEX_RANGE
    res = run_batch(ctx, graphs)
    for i, gr in enumerate(graphs):
        if i in bad:
            assert res.status[i] == bad[i], (i, res.status[i])
            assert res.result(i) == bbc.Result(0, 0, 0)
        else:
            assert res.status[i] == bbc.OK
            assert res.result(i) == expect(gr), (i, gr.name)
    # a negative size is reported for that graph only
    nu, nv, off, eu, ev, sg = bbc.concat_graphs(graphs[:5])
    nu[3] = -1
    res = ctx.count_batch(nu, nv, off, eu, ev, sg)
    assert res.status[3] == bbc.INVALID_ARG and res.status[0] == bbc.OK


def test_batch_empty_side_with_edges(ctx):
    # A graph with no vertex on one side shares its id block start with the
    # next graph, so its (necessarily out-of-range) edges must be dropped, not
    # placed: its neighbours (rows longer than 64 entries) stay exact.
    rng = np.random.default_rng(77)
    dense = [gen.random_graph(rng, 90, 120, 0.7, p_neg=0.4) for _ in range(3)]
    no_v = SignedBipartiteGraph(5, 0, np.array([0, 1, 2], np.int32), np.array([0, 0, 1], np.int32),
                                np.array([1, -1, 1], np.int8), "no_v")
    no_u = SignedBipartiteGraph(0, 80, np.zeros(70, np.int32), np.arange(70, dtype=np.int32),
                                rng.choice([1, -1], 70).astype(np.int8), "no_u")
    graphs = [no_v, dense[0], no_u, dense[1], no_v, no_u, dense[2]]
    res = run_batch(ctx, graphs)
    for i, g in enumerate(graphs):
        if g.name in ("no_v", "no_u"):
            assert res.status[i] == bbc.VERTEX_RANGE, (i, res.status[i])
            assert res.result(i) == bbc.Result(0, 0, 0)
        else:
            assert res.status[i] == bbc.OK, (i, res.status[i])
            assert res.result(i) == expect(g), (i, g.name)


def test_batch_with_a_large_graph(ctx):
    # more than 16384 vertices on a side: counted on its own inside the call
    big = gen.chung_lu_graph(seed=31, n_u=40000, n_v=9000, n_edges=150000, alpha=2.1, p_neg=0.3)
    graphs = mixed_graphs(10, 30)
    graphs.insert(11, big)
    res = run_batch(ctx, graphs)
    assert (res.status == bbc.OK).all()
    for i, g in enumerate(graphs):
        assert res.result(i) == expect(g), (i, g.name)


def test_batch_long_rows_and_repeats(ctx):
    # rows sorted through LDS bitmaps: medium rows (65..4096 entries, every row
    # of a batch spans one small graph block) and rows above 4096 entries; a
    # repeated edge in such a row is reported for its graph only
    rng = np.random.default_rng(21)
    graphs = mixed_graphs(14, 12)
    graphs.insert(2, gen.complete_graph(3, 3000, rng.choice([1, -1], 3), rng.choice([1, -1], 3000)))
    graphs.insert(5, gen.complete_graph(2, 6000, rng.choice([1, -1], 2), rng.choice([1, -1], 6000)))
    big = gen.complete_graph(2, 5000)
    graphs.insert(7, big._replace(eu=np.append(big.eu, np.int32(1)), ev=np.append(big.ev, np.int32(4321)),
                                  sign=np.append(big.sign, np.int8(-1))))
    mid = gen.complete_graph(3, 2000)
    graphs.insert(9, mid._replace(eu=np.append(mid.eu, np.int32(2)), ev=np.append(mid.ev, np.int32(1234)),
                                  sign=np.append(mid.sign, np.int8(1))))
    res = run_batch(ctx, graphs)
    for i, g in enumerate(graphs):
        if i in (7, 9):
            assert res.status[i] == bbc.DUPLICATE_EDGE, (i, res.status[i])
            assert res.result(i) == bbc.Result(0, 0, 0)
        else:
            assert res.status[i] == bbc.OK, (i, res.status[i])
            assert res.result(i) == expect(g), (i, g.name)


def test_batch_device_input_matches_host(ctx):
    import torch
    graphs = mixed_graphs(11, 90)
    nu, nv, off, eu, ev, sg = bbc.concat_graphs(graphs)
    host = ctx.count_batch(nu, nv, off, eu, ev, sg)
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(x).to(dev) for x in (eu, ev, sg)]
    torch.cuda.synchronize()
    on_dev = ctx.count_batch(nu, nv, off, *t)
    for a, b in zip(host, on_dev):
        assert np.array_equal(a, b)


def test_batched_recipe_sample(ctx):
    # the batched workload's own recipe (sizes log-uniform in [16, 4096]),
    # first 400 graphs, each checked against the oracle
    nu, nv, ne = gen.batch_graph_params(20000)
    idx = [i for i in range(400) if ne[i] <= 200000]
    graphs = [gen.batch_graph(i, nu[i], nv[i], ne[i]) for i in idx]
    res = run_batch(ctx, graphs)
    assert (res.status == bbc.OK).all()
    for k, g in enumerate(graphs):
        b, u = gram_count(g) if min(g.n_u, g.n_v) <= 2048 else oracle.count(g)
        assert (int(res.balanced[k]), int(res.unbalanced[k])) == (b, u), (idx[k], g.name)
    for k in range(0, len(graphs), 25):
        assert int(res.wedges[k]) == oracle.wedges(graphs[k])


def test_graph_replay_matches_eager(ctx):
    # the pipeline's two segments captured as HIP graphs and replayed for
    # repeated shapes; eager work and synchronisations run between replays
    import torch
    graphs = mixed_graphs(12, 120)
    nu, nv, off, eu, ev, sg = bbc.concat_graphs(graphs)
    eager = ctx.count_batch(nu, nv, off, eu, ev, sg)
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(x).to(dev) for x in (eu, ev, sg)]
    torch.cuda.synchronize()
    gctx = bbc.Context(0)
    try:
        gctx.set_param(bbc.PARAM_GRAPHS, 1)
        other = gen.uniform_graph(seed=77, n_u=500, n_v=400, n_edges=9000)
        want_other = ctx.count(other.eu, other.ev, other.sign, other.n_u, other.n_v)
        for rep in range(4):
            res = gctx.count_batch(nu, nv, off, *t)
            for a, b in zip(eager, res):
                assert np.array_equal(a, b), rep
            # eager work on another context and the torch stream in between
            assert ctx.count(other.eu, other.ev, other.sign, other.n_u, other.n_v) == want_other
            x = torch.arange(1 << 20, device=dev, dtype=torch.int64)
            assert int(x.sum().item()) == (1 << 20) * ((1 << 20) - 1) // 2
            torch.cuda.synchronize()
        assert gctx.get_param(bbc.PARAM_GRAPH_CAPTURES) == 2
        assert gctx.get_param(bbc.PARAM_GRAPH_REPLAYS) == 6
        # a new shape is captured again and stays exact; single graphs and
        # per-vertex counts replay as well
        res = gctx.count_batch(nu[:60], nv[:60], off[:61], *t)
        for a, b in zip(eager, res):
            assert np.array_equal(a[:60], b)
        g = gen.voting_graph(seed=8, n_u=60, n_v=2000, p_edge=0.5)
        want = ctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v, per_vertex=True)
        for rep in range(3):
            r, pv = gctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v, per_vertex=True)
            assert r == want[0] and np.array_equal(pv, want[1]), rep
            assert gctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v) == want[0]
    finally:
        gctx.close()


def test_autotune_keeps_counts(ctx):
    graphs = mixed_graphs(13, 150)
    nu, nv, off, eu, ev, sg = bbc.concat_graphs(graphs)
    before = ctx.count_batch(nu, nv, off, eu, ev, sg)
    tctx = bbc.Context(0)
    try:
        chosen, best = tctx.autotune(nu, nv, off, eu, ev, sg, repeats=1)
        assert chosen["chunk_wedges"] in (16384, 65536, 262144, 1048576, 4194304)
        # no graph here is cut into end-vertex tiles: hash target and probe
        # limit are not searched and keep their defaults
        assert (chosen["hash_target"], chosen["probe_limit"]) == (4096, 256)
        assert chosen["light_max"] in (512, 1024, 2048)
        assert chosen["grab_div"] in (8, 16, 32)
        assert chosen["union_edges"] in (1 << 24, 1 << 26, 1 << 28, 1 << 30)
        assert tctx.get_param(bbc.PARAM_LIGHT_MAX) == chosen["light_max"]
        assert tctx.get_param(bbc.PARAM_UNION_EDGES) == chosen["union_edges"]
        assert best > 0
        assert tctx.get_param(bbc.PARAM_CHUNK_WEDGES) == chosen["chunk_wedges"]
        assert tctx.get_param(bbc.PARAM_HASH_TARGET) == chosen["hash_target"]
        after = tctx.count_batch(nu, nv, off, eu, ev, sg)
        for a, b in zip(before, after):
            assert np.array_equal(a, b)
        # one graph with split starts: tuned on bbc_count
        g = gen.chung_lu_graph(seed=11, n_u=60000, n_v=20000, n_edges=250000, p_neg=0.25)
        want = ctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v)
        chosen, best = tctx.autotune([g.n_u], [g.n_v], [0, g.n_edges], g.eu, g.ev, g.sign,
                                     repeats=1)
        assert tctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v) == want
    finally:
        tctx.close()


def test_batch_tunables_never_change_counts(ctx):
    # the light cut, grab size, union size and one-wave share change how the
    # work is cut, never a count: extreme settings (many tiny unions, almost
    # no light starts, one-record grabs, one-wave starts of any size or of at
    # most 4096 wedges) give the same per-graph results
    graphs = mixed_graphs(17, 120)
    nu, nv, off, eu, ev, sg = bbc.concat_graphs(graphs)
    want = ctx.count_batch(nu, nv, off, eu, ev, sg)
    tctx = bbc.Context(0)
    try:
        for lm, gd, ue, ws in ((16, 4, 1 << 16, 0), (2048, 64, 1 << 16, 1 << 20),
                               (512, 8, 1 << 20, 1), (1024, 32, 1 << 30, 2048)):
            tctx.set_param(bbc.PARAM_LIGHT_MAX, lm)
            tctx.set_param(bbc.PARAM_GRAB_DIV, gd)
            tctx.set_param(bbc.PARAM_UNION_EDGES, ue)
            tctx.set_param(bbc.PARAM_WAVE_SHARE, ws)
            got = tctx.count_batch(nu, nv, off, eu, ev, sg)
            for a, b in zip(want, got):
                assert np.array_equal(a, b), (lm, gd, ue, ws)
        with pytest.raises(bbc.BBCError):
            tctx.set_param(bbc.PARAM_LIGHT_MAX, 4096)
        with pytest.raises(bbc.BBCError):
            tctx.set_param(bbc.PARAM_UNION_EDGES, 100)
    finally:
        tctx.close()
    for g in graphs[:12]:
        assert want.result(graphs.index(g)) == expect(g)
