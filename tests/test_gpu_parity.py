"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Integer results must be bit-exact: balanced, unbalanced and W (the number of
priority-filtered wedges).  Inputs are seeded synthetic graphs; full-size
workloads are compared with tests/golden/workloads.json, written by
tests/golden/make_golden.py from the oracle alone.
"""
import ctypes
import json
import os

import numpy as np
import pytest

import gen
import oracle
import paper_2308_07932_amd as bbc
from gen import SignedBipartiteGraph

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    c = bbc.Context(0)
    yield c
    c.close()


def graph_from_edges(n_u, n_v, edges, name="g"):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    return SignedBipartiteGraph(n_u, n_v, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32),
                                e[:, 2].astype(np.int8), name)


def expect(g):
    b, u = oracle.count(g)
    return bbc.Result(b, u, oracle.wedges(g))


def run(ctx, g):
    print(f"[gpu] {g.name} n_u={g.n_u} n_v={g.n_v} m={g.n_edges}", flush=True)
    return ctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v)


def check(ctx, g):
    got = run(ctx, g)
    want = expect(g)
    assert got == want, (g.name, got, want)
    return got


def test_figure1_and_all_k22_signings(ctx):
    fx = json.load(open(os.path.join(GOLDEN, "fig1_butterflies.json")))
    for pat in fx["patterns"] + fx["derived"]:
        g = graph_from_edges(2, 2, pat["edges"], pat["name"])
        r = run(ctx, g)
        assert (r.balanced, r.balanced + r.unbalanced) == (pat["balanced"], pat["total"])
    import itertools
    for signs in itertools.product([1, -1], repeat=4):
        g = graph_from_edges(2, 2, [[0, 0, signs[0]], [0, 1, signs[1]], [1, 0, signs[2]],
                                    [1, 1, signs[3]]])
        r = run(ctx, g)
        assert r.balanced == (1 if signs.count(-1) % 2 == 0 else 0)
        assert r.balanced + r.unbalanced == 1


def test_random_small_graphs(ctx):
    rng = np.random.default_rng(2024)
    for i in range(120):
        nu = int(rng.integers(1, 60))
        nv = int(rng.integers(1, 60))
        g = gen.random_graph(rng, nu, nv, float(rng.uniform(0.02, 1.0)), float(rng.uniform(0, 1)))
        check(ctx, g._replace(name=f"small{i}"))


def test_uniform_sizes_across_thresholds(ctx):
    # sweeps light / hashed / dense pieces and the row-sort size classes
    for seed, (nu, nv, m) in enumerate([(50, 40, 600), (300, 200, 9000), (2000, 1000, 20000),
                                        (700, 90, 30000), (90, 3000, 60000), (5000, 5000, 100000),
                                        (20000, 300, 120000), (120, 120, 14000)]):
        check(ctx, gen.uniform_graph(seed=100 + seed, n_u=nu, n_v=nv, n_edges=m, p_neg=0.4))


def test_complete_bipartite(ctx):
    rng = np.random.default_rng(5)
    for a, b in [(2, 2), (3, 70), (64, 4096), (130, 130), (5, 9000), (300, 40)]:
        su = rng.choice([1, -1], size=a)
        sv = rng.choice([1, -1], size=b)
        g = gen.complete_graph(a, b, su, sv)
        r = run(ctx, g)
        c2 = lambda k: k * (k - 1) // 2  # noqa: E731
        assert r.balanced == c2(a) * c2(b) and r.unbalanced == 0
        # W for K_{a,b}: the side of larger degree starts, ties go to V (larger ids)
        w = b * c2(a) if b > a else a * c2(b)
        assert r.wedges == w
        # random signs: compare with the oracle
        s = rng.choice([1, -1], size=g.n_edges).astype(np.int8)
        check(ctx, g._replace(sign=s, name=f"K{a},{b}rand"))


def test_hub_and_star_shapes(ctx):
    rng = np.random.default_rng(8)
    # one U hub adjacent to every V vertex, on top of a sparse random graph
    base = gen.uniform_graph(seed=9, n_u=3000, n_v=5000, n_edges=30000, p_neg=0.3)
    hub_v = np.setdiff1d(np.arange(5000), base.ev[base.eu == 0])
    eu = np.concatenate([base.eu, np.zeros(hub_v.size, np.int32)])
    ev = np.concatenate([base.ev, hub_v.astype(np.int32)])
    sg = np.concatenate([base.sign, rng.choice([1, -1], size=hub_v.size).astype(np.int8)])
    check(ctx, SignedBipartiteGraph(3000, 5000, eu, ev, sg, "hub"))
    # star: no butterflies, no wedges kept
    star = graph_from_edges(1, 7000, [[0, v, 1 if v % 3 else -1] for v in range(7000)])
    assert run(ctx, star) == bbc.Result(0, 0, 0)


def test_small_powerlaw(ctx):
    for seed in (11, 12):
        g = gen.chung_lu_graph(seed=seed, n_u=60000, n_v=20000, n_edges=250000, p_neg=0.25)
        check(ctx, g)


def test_phase_timing(ctx):
    # HIP-event phase times: the pipeline holds preprocessing, planning and the
    # wedge step; the short-wedge bucketing (phase 4) is part of planning
    g = gen.chung_lu_graph(seed=11, n_u=60000, n_v=20000, n_edges=250000, p_neg=0.25)
    c = bbc.Context(0)
    try:
        c.set_timing(True)
        r = c.count(g.eu, g.ev, g.sign, g.n_u, g.n_v)
        assert r == expect(g)
        ph = [c.phase_ms(p) for p in range(5)]
        assert all(x >= 0 for x in ph), ph
        assert ph[1] + ph[2] + ph[3] <= ph[0] * 1.01 + 0.01, ph
        assert 0 < ph[4] <= ph[3], ph  # this graph has split starts with short middles
        with pytest.raises(bbc.BBCError):
            c.phase_ms(5)
    finally:
        c.close()


def test_resplit_path(ctx):
    # A hub start whose first end-vertex tile holds 16000 degree-2 leaves (each
    # sharing two middles with the hub) while most degree mass sits in 100
    # heavy vertices the hub cannot reach: the leaf tile goes to a hashed
    # piece, the table overflows, and the piece must be redone (here with
    # dense counters) and still count exactly.
    n_iso, n_leaf, n_heavy, n_mid = 384, 16000, 100, 20
    leaf0, heavy0 = n_iso, n_iso + n_leaf
    hub = heavy0 + n_heavy
    n_u = hub + 1
    hub_leaf0, hv0 = n_mid, n_mid + 4980
    n_v = hv0 + 4000
    eu, ev = [], []
    for j in range(n_leaf):
        a = j % n_mid
        b = (a + 1 + (j // n_mid) % (n_mid - 1)) % n_mid
        eu += [leaf0 + j, leaf0 + j]
        ev += [a, b]
    for v in range(hv0):              # hub: 20 middles + 4980 private leaves (degree 5000)
        eu.append(hub)
        ev.append(v)
    for h in range(n_heavy):          # heavy block K_{100,4000}, out of the hub's reach
        for v in range(4000):
            eu.append(heavy0 + h)
            ev.append(hv0 + v)
    rng = np.random.default_rng(1)
    g = SignedBipartiteGraph(n_u, n_v, np.array(eu, np.int32), np.array(ev, np.int32),
                             rng.choice([1, -1], size=len(eu)).astype(np.int8), "resplit")
    r = check(ctx, g)
    assert r.balanced > 0
    # A hashed run of one tile can no longer overflow by capacity when its
    # start has fewer than 2^16 middles (16-bit halves give as many slots as
    # the tile has vertices), so the redo is forced by a short probe limit;
    # a hash target above the hub's 32,000 wedges keeps its two tiles out of
    # a dense piece, in one hashed run.
    ctx.set_param(bbc.PARAM_PROBE_LIMIT, 8)
    ctx.set_param(bbc.PARAM_HASH_TARGET, 65536)
    try:
        assert run(ctx, g) == r
        assert ctx.stats()[5] > 0, "expected a hashed piece to be redone"
    finally:
        ctx.set_param(bbc.PARAM_PROBE_LIMIT, 256)
        ctx.set_param(bbc.PARAM_HASH_TARGET, 4096)


def test_forced_resplits_stay_exact(ctx):
    # A probe limit of a few slots makes nearly every hashed piece of a heavy
    # start overflow, so the halving and dense-redo paths run thousands of
    # times, interleaved with normal pieces on the same workgroups.  A smaller
    # and a larger hash target change the piece layout itself (at 512 hardly
    # any range stays hashed).
    g = gen.chung_lu_graph(seed=21, n_u=200000, n_v=60000, n_edges=1500000, alpha=2.1, p_neg=0.2)
    want = expect(g)
    base = run(ctx, g)
    assert base == want
    try:
        for target, probes in ((4096, 4), (8192, 4), (512, 2), (65536, 256)):
            ctx.set_param(bbc.PARAM_HASH_TARGET, target)
            ctx.set_param(bbc.PARAM_PROBE_LIMIT, probes)
            for _ in range(2):
                got = run(ctx, g)
                assert got == want, (target, probes, got, want)
            if probes <= 4 and target >= 4096:
                assert ctx.stats()[5] > 100, (target, probes, ctx.stats())
            if target == 512:  # nearly every range is dense, most of them packed
                assert ctx.stats()[11] + ctx.stats()[12] > ctx.stats()[10], ctx.stats()
    finally:
        ctx.set_param(bbc.PARAM_HASH_TARGET, 4096)
        ctx.set_param(bbc.PARAM_PROBE_LIMIT, 256)


def saturated_graph(n_end, end_deg, n_mid, n_pad=0, pad_deg=2, seed=0):
    """A hub on side U adjacent to every one of n_mid middles, and n_end end
    vertices of degree end_deg whose middles are all the hub's: every (hub, w)
    bucket has l + m = end_deg, the most its packed counters may hold.  A third
    of the ends have l = end_deg, a third m = end_deg, a third a mix; n_pad
    ends of degree pad_deg sit below them."""
    rng = np.random.default_rng(seed)
    eu, ev, sg = [0] * n_mid, list(range(n_mid)), [1] * n_mid
    for i in range(n_end + n_pad):
        d = end_deg if i < n_end else pad_deg
        mids = rng.choice(n_mid, size=d, replace=False)
        if i < n_end and i % 3 < 2:
            s = [1 - 2 * (i % 3)] * d
        else:
            s = rng.choice([1, -1], size=d).tolist()
        eu += [1 + i] * d
        ev += mids.tolist()
        sg += s
    return SignedBipartiteGraph(1 + n_end + n_pad, n_mid, np.array(eu, np.int32),
                                np.array(ev, np.int32), np.array(sg, np.int8),
                                f"saturated{end_deg}")


def test_packed_counters_at_their_limits(ctx):
    # 4-bit halves: 40,000 ends of degree 15 below a hub of degree 1000, one
    # piece of eight tiles (cut to the three the hub has); 8-bit halves: 100
    # ends of degree 255 above 20,000 of degree 2
    g4 = saturated_graph(40000, 15, 1000)
    check(ctx, g4)
    assert ctx.stats()[12] >= 1, ctx.stats()
    g8 = saturated_graph(100, 255, 400, n_pad=20000)
    check(ctx, g8)
    assert ctx.stats()[11] >= 1, ctx.stats()


def test_one_wave_pieces_at_their_limits(ctx):
    # starts counted by one wave alone: 4-bit halves filled to 15 (4,000 ends
    # of degree 15), 8-bit halves filled to 255, and 16-bit counters over a
    # range of exactly one slice (2,048 ends: 2,047 of degree 1 below one of
    # degree 300, which sets the width).  These graphs are small, so the
    # bound of a one-wave start by its share of the count is lifted.
    ctx.set_param(bbc.PARAM_WAVE_SHARE, 0)
    try:
        for g in (saturated_graph(4000, 15, 1000), saturated_graph(250, 255, 400)):
            check(ctx, g)
            assert ctx.stats()[13] >= 1, ctx.stats()
        rng = np.random.default_rng(12)
        eu, ev = [0] * 400, list(range(400))
        for i in range(1, 2048):
            eu.append(i)
            ev.append(i % 400)
        eu += [2048] * 300
        ev += list(range(300))
        g = SignedBipartiteGraph(2049, 400, np.array(eu, np.int32), np.array(ev, np.int32),
                                 rng.choice([1, -1], size=len(eu)).astype(np.int8), "wave16_full")
        check(ctx, g)
        assert ctx.stats()[13] >= 1, ctx.stats()
    finally:
        ctx.set_param(bbc.PARAM_WAVE_SHARE, 2048)


def test_16bit_halves_at_their_limit(ctx):
    # k = 2^16 - 1 middles, all adjacent to a start s and to ends of the same
    # degree below it (lower id): w+ with every sign +, w- with every sign -.
    # With s all +, the bucket (s, w+) holds l = 65535 and (s, w-) m = 65535,
    # the most a 16-bit half may hold (l + m <= the start's middles < 2^16);
    # with s mixed, both halves are large.  20,000 ends of degree 1 below them
    # fill the first end-vertex tile (no piece), so the live tile becomes a
    # two-tile dense piece with 16-bit halves.  With a single end the start has
    # W = 65535 wedges and is counted by one wave, with 16-bit halves too.
    # Expected counts in closed form (Lemma 2 per pair; ends of degree 1 lie
    # in no butterfly): a pair whose common middles give l symmetric and m
    # asymmetric wedges holds C(l,2) + C(m,2) balanced and l m unbalanced.
    k = 65535
    rng = np.random.default_rng(16)

    def c2(x):
        return x * (x - 1) // 2

    def graph(n_pad, end_signs, n_plus, name):
        eu = [np.arange(n_pad, dtype=np.int32)]
        ev = [rng.integers(0, k, size=n_pad).astype(np.int32)]
        sg = [rng.choice([1, -1], size=n_pad).astype(np.int8)]
        s_signs = np.where(np.arange(k) < n_plus, 1, -1).astype(np.int8)
        for i, sgn in enumerate(end_signs):
            eu.append(np.full(k, n_pad + i, np.int32))
            ev.append(np.arange(k, dtype=np.int32))
            sg.append(np.full(k, sgn, np.int8))
        eu.append(np.full(k, n_pad + len(end_signs), np.int32))  # the start, highest id
        ev.append(np.arange(k, dtype=np.int32))
        sg.append(s_signs)
        return SignedBipartiteGraph(n_pad + len(end_signs) + 1, k, np.concatenate(eu),
                                    np.concatenate(ev), np.concatenate(sg), name)

    for n_plus in (k, 40000):
        p, q = n_plus, k - n_plus
        g = graph(20000, (1, -1), n_plus, f"halves16_tiles_{n_plus}")
        got = run(ctx, g)
        # (s, w+) and (s, w-) each give l, m = p, q (in either order); (w-, w+)
        # has only asymmetric wedges
        want = bbc.Result(2 * (c2(p) + c2(q)) + c2(k), 2 * p * q, oracle.wedges(g))
        assert got == want, (g.name, got, want)
        assert ctx.stats()[9] >= 1, ctx.stats()
        assert ctx.stats()[5] == 0, ctx.stats()
    # the same start alone (W = 65535): counted by one wave when the bound by
    # its share of the count is lifted, else (its cost W_u + 8 k_u far above
    # max(4096, W / 2048)) by a workgroup piece; the same counts either way
    for share, waves in ((0, 1), (2048, 0)):
        ctx.set_param(bbc.PARAM_WAVE_SHARE, share)
        try:
            for sgn in (1, -1):
                g = graph(0, (sgn,), k, f"halves16_wave_{sgn}_{share}")
                got = run(ctx, g)
                assert got == bbc.Result(c2(k), 0, k), (g.name, got)
                assert oracle.wedges(g) == k
                assert ctx.stats()[13] == waves, ctx.stats()
        finally:
            ctx.set_param(bbc.PARAM_WAVE_SHARE, 2048)


def test_tiles_of_degree_one_ends(ctx):
    # A hub adjacent to 2000 middles, each with private leaves of degree 1
    # (80 per middle for the first 100, whose rows are then long, 30 for the
    # rest): the leaves fill the hub's first tiles, which get no piece.  Alone
    # they give no butterfly at all; with 500 ends of degree 2 above them the
    # last tile is live and must still be counted exactly.
    rng = np.random.default_rng(8)
    n_mid = 2000
    per = [80] * 100 + [30] * (n_mid - 100)
    n_leaf = sum(per)
    for n_live in (0, 500):
        eu, ev = [0] * n_mid, list(range(n_mid))
        w = 1
        for v, c in enumerate(per):
            eu += range(w, w + c)
            ev += [v] * c
            w += c
        for i in range(n_live):
            eu += [w + i] * 2
            ev += rng.choice(n_mid, size=2, replace=False).tolist()
        g = SignedBipartiteGraph(1 + n_leaf + n_live, n_mid, np.array(eu, np.int32),
                                 np.array(ev, np.int32),
                                 rng.choice([1, -1], size=len(eu)).astype(np.int8),
                                 f"dead_tiles_{n_live}")
        r = check(ctx, g)
        assert (r.balanced + r.unbalanced > 0) == (n_live > 0)
        assert r.wedges >= n_leaf


def test_param_checks(ctx):
    assert ctx.get_param(bbc.PARAM_HASH_TARGET) == 4096
    assert ctx.get_param(bbc.PARAM_PROBE_LIMIT) == 256
    assert ctx.get_param(bbc.PARAM_WAVE_SHARE) == 2048
    for p, v in ((bbc.PARAM_HASH_TARGET, 63), (bbc.PARAM_HASH_TARGET, (1 << 20) + 1),
                 (bbc.PARAM_PROBE_LIMIT, 0), (bbc.PARAM_PROBE_LIMIT, 8193),
                 (bbc.PARAM_WAVE_SHARE, -1), (bbc.PARAM_WAVE_SHARE, (1 << 20) + 1), (99, 1)):
        with pytest.raises(bbc.BBCError):
            ctx.set_param(p, v)
    assert ctx.get_param(bbc.PARAM_HASH_TARGET) == 4096
    with pytest.raises(bbc.BBCError):
        ctx.get_param(99)


def test_full_workloads_match_golden(ctx):
    gold = json.load(open(os.path.join(GOLDEN, "workloads.json")))
    for name in ("uniform", "voting", "powerlaw"):
        if name not in gold:
            pytest.fail(f"golden value for {name} missing")
        g = gen.workload(name)
        r = run(ctx, g)
        want = gold[name]
        assert g.n_edges == want["n_edges"] and int(np.sum(g.sign < 0)) == want["negative_edges"]
        assert (r.balanced, r.unbalanced, r.wedges) == (want["balanced"], want["unbalanced"],
                                                        want["wedges"]), name
    # the full power-law graph again with nearly every hashed piece redone
    g = gen.workload("powerlaw")
    ctx.set_param(bbc.PARAM_PROBE_LIMIT, 4)
    try:
        r = run(ctx, g)
        assert ctx.stats()[5] > 1000
    finally:
        ctx.set_param(bbc.PARAM_PROBE_LIMIT, 256)
    want = gold["powerlaw"]
    assert (r.balanced, r.unbalanced, r.wedges) == (want["balanced"], want["unbalanced"], want["wedges"])


def test_device_input_and_determinism(ctx):
    import torch
    g = gen.voting_graph(seed=5, n_u=60, n_v=3000, p_edge=0.5)
    want = expect(g)
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(x).to(dev) for x in (g.eu, g.ev, g.sign)]
    for _ in range(5):
        assert ctx.count(*t, g.n_u, g.n_v) == want
        assert ctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v) == want


def test_invariances_on_gpu(ctx):
    rng = np.random.default_rng(77)
    g = gen.uniform_graph(seed=31, n_u=900, n_v=700, n_edges=40000, p_neg=0.35)
    r = run(ctx, g)
    # switching at a vertex and global negation keep the balanced count
    s = g.sign.copy()
    s[g.eu == 5] *= -1
    assert run(ctx, g._replace(sign=s)).balanced == r.balanced
    assert run(ctx, g._replace(sign=(-g.sign).astype(np.int8))).balanced == r.balanced
    # transposing U and V keeps both counts
    rt = run(ctx, SignedBipartiteGraph(g.n_v, g.n_u, g.ev, g.eu, g.sign, "T"))
    assert (rt.balanced, rt.unbalanced) == (r.balanced, r.unbalanced)
    # shuffling the edge order changes nothing at all
    o = rng.permutation(g.n_edges)
    assert run(ctx, g._replace(eu=g.eu[o], ev=g.ev[o], sign=g.sign[o])) == r


def _raw(ctx, g, flags=0, pv=None):
    out = bbc._CResult(-7, -7, -7)
    rc = ctx._lib.bbc_count(ctx._h, g.n_u, g.n_v, g.n_edges, g.eu.ctypes.data, g.ev.ctypes.data,
                            g.sign.ctypes.data, flags, ctypes.byref(out), pv)
    return rc, (out.balanced, out.unbalanced, out.wedges)


def long_interval_light_graph(seed: int) -> SignedBipartiteGraph:
    """A light start u (2000 wedges) whose middle v1 holds 1100 of u's ends in one
    interval, packed into one work item with two other light starts that come
    before it in priority order (U vertices of a K(3,3) raised above their
    middles by two leaves each): the interval exceeds the kernel's queued-chunk
    length inside an item of several pieces.  v2 shares 900 of the ends, so
    every end's bucket matters.  U: 0 = u, 1..1100 = the ends, 1101..1103 = the
    K(3,3) side a; V: 0 = v1, 1 = v2, 2..1101 = leaves of u (raising its
    priority), 1102..1104 = the K(3,3) side b, 1105..1110 = leaves of side a."""
    rng = np.random.default_rng(seed)
    e = [(0, 0), (0, 1)] + [(0, 2 + i) for i in range(1100)]
    e += [(1 + i, 0) for i in range(1100)] + [(1 + i, 1) for i in range(200, 1100)]
    e += [(1101 + i, 1102 + j) for i in range(3) for j in range(3)]
    e += [(1101 + i, 1105 + 2 * i + k) for i in range(3) for k in range(2)]
    e = np.array(e)
    s = rng.choice([1, -1], len(e), p=[0.7, 0.3]).astype(np.int8)
    return SignedBipartiteGraph(1104, 1111, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), s,
                                f"long_interval_light_{seed}")


def test_long_interval_in_light_item(ctx):
    for seed in range(3):
        g = long_interval_light_graph(seed)
        check(ctx, g)
        r = ctx.count_batch(*bbc.concat_graphs([g, gen.complete_graph(4, 5), g]))
        want = bbc.Result(*oracle.count(g), oracle.wedges(g))
        assert r.result(0) == want and r.result(2) == want


def threshold_graph(seed: int) -> SignedBipartiteGraph:
    """Hubs on both sides whose degrees sit at the wedge kernel's size limits
    (short-prefix scan 16, long middle 64, queued chunk 1024, light start
    2048) over a random background, plus on each side two "leafy" starts: a
    vertex raised above every hub by fresh leaf neighbours and joined to a hub
    of degree 1300 or 1400 and one of degree 400 or 500, so that it is a light
    start (about 1700 wedges) whose interval through the first hub is longer
    than a queued chunk and shares ends with the second."""
    rng = np.random.default_rng(seed)
    n = [int(rng.integers(2500, 4000)), int(rng.integers(2500, 4000))]
    degs = [15, 16, 17, 63, 64, 65, 1023, 1024, 1025, 2047, 2049]
    pairs = set()
    hubs = [[], []]
    for side in (0, 1):
        cand = rng.choice(n[side], len(degs) + 4, replace=False)
        for h, dg in zip(cand, degs + [1300, 1400, 400, 500]):
            hubs[side].append(int(h))
            for o in rng.choice(n[1 - side], min(dg, n[1 - side]), replace=False):
                pairs.add((int(h), int(o)) if side == 0 else (int(o), int(h)))
    m_bg = int(rng.integers(5000, 20000))
    for u, v in zip(rng.integers(0, n[0], m_bg), rng.integers(0, n[1], m_bg)):
        pairs.add((int(u), int(v)))
    for side in (0, 1):
        for k in range(2):
            x = int(rng.integers(0, n[side]))
            mids = [hubs[1 - side][11 + k], hubs[1 - side][13 + k]]  # degrees 1300/1400, 400/500
            leaves = int(rng.integers(2100, 2600))
            first = n[1 - side]
            n[1 - side] += leaves
            for o in mids + list(range(first, first + leaves)):
                pairs.add((x, o) if side == 0 else (o, x))
    e = np.array(sorted(pairs))[rng.permutation(len(pairs))]
    sg = rng.choice([1, -1], len(e), p=[0.6, 0.4]).astype(np.int8)
    return SignedBipartiteGraph(n[0], n[1], e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), sg,
                                f"thresholds{seed}")


def test_size_limit_structures(ctx):
    graphs = [threshold_graph(seed) for seed in range(6)]
    for g in graphs:
        check(ctx, g)
    r = ctx.count_batch(*bbc.concat_graphs(graphs))
    for i, g in enumerate(graphs):
        assert r.result(i) == expect(g), (i, g.name)


def test_error_paths(ctx):
    g = gen.uniform_graph(seed=3, n_u=100, n_v=80, n_edges=2000)
    bad = g.ev.copy()
    bad[123] = 80
    rc, out = _raw(ctx, g._replace(ev=bad))
    assert rc == bbc.VERTEX_RANGE and out == (-7, -7, -7)
    assert "123" in ctx.last_error()
    bad = g.eu.copy()
    bad[7] = -1
    assert _raw(ctx, g._replace(eu=bad))[0] == bbc.VERTEX_RANGE
    bs = g.sign.copy()
    bs[55] = 0
    rc, out = _raw(ctx, g._replace(sign=bs))
    assert rc == bbc.BAD_SIGN and out == (-7, -7, -7)
    # duplicate pair, same sign and opposite sign
    for flip in (1, -1):
        dup = g._replace(eu=np.append(g.eu, g.eu[10]), ev=np.append(g.ev, g.ev[10]),
                         sign=np.append(g.sign, np.int8(g.sign[10] * flip)))
        rc, out = _raw(ctx, dup)
        assert rc == bbc.DUPLICATE_EDGE and out == (-7, -7, -7)
    # duplicate inside a long (bitmap-sorted) row
    k = gen.complete_graph(2, 5000)
    dup = k._replace(eu=np.append(k.eu, np.int32(1)), ev=np.append(k.ev, np.int32(4321)),
                     sign=np.append(k.sign, np.int8(-1)))
    assert _raw(ctx, dup)[0] == bbc.DUPLICATE_EDGE
    # duplicate inside a medium row whose neighbours span few ids (bitmap-sorted)
    k = gen.complete_graph(3, 2000)
    dup = k._replace(eu=np.append(k.eu, np.int32(2)), ev=np.append(k.ev, np.int32(1234)),
                     sign=np.append(k.sign, np.int8(1)))
    assert _raw(ctx, dup)[0] == bbc.DUPLICATE_EDGE
    # rows of 100 to 2000 entries whose neighbours span more than 16384 ids
    # (one-wave register sorts of 2, 4, 8 or 16 entries per lane up to 1024
    # entries, the workgroup sort above): counted exactly, and a repeated pair in
    # each is reported
    wide = graph_from_edges(5, 40000, [[u, (i * 397 + u * 13) % 40000, 1 if (i + u) % 3 else -1]
                                       for u, L in enumerate((100, 200, 400, 1000, 2000))
                                       for i in range(L)])
    check(ctx, wide)
    for row, i in ((0, 57), (1, 150), (2, 399), (3, 700), (4, 1999)):
        e = int(np.nonzero(wide.eu == row)[0][i])
        dup = wide._replace(eu=np.append(wide.eu, wide.eu[e]), ev=np.append(wide.ev, wide.ev[e]),
                            sign=np.append(wide.sign, np.int8(-wide.sign[e])))
        assert _raw(ctx, dup)[0] == bbc.DUPLICATE_EDGE, row
    # sizes and pointers
    out = bbc._CResult()
    assert ctx._lib.bbc_count(ctx._h, -1, 5, 0, None, None, None, 0, ctypes.byref(out), None) == bbc.INVALID_ARG
    assert ctx._lib.bbc_count(ctx._h, 5, 5, 3, None, None, None, 0, ctypes.byref(out), None) == bbc.INVALID_ARG
    assert ctx._lib.bbc_count(ctx._h, 5, 5, 0, None, None, None, 0, None, None) == bbc.INVALID_ARG
    assert ctx._lib.bbc_count(ctx._h, 5, 5, 0, None, None, None, 0x100, ctypes.byref(out), None) == bbc.INVALID_ARG
    assert ctx._lib.bbc_count(ctx._h, 1 << 29, 1 << 29, 0, None, None, None, 0, ctypes.byref(out), None) == bbc.TOO_LARGE
    # empty graph and one-sided graphs give zeros
    assert ctx.count(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int8), 10, 10) == (0, 0, 0)
    one = graph_from_edges(1, 50, [[0, v, 1] for v in range(50)])
    assert run(ctx, one) == (0, 0, 0)
    # the context still works after errors
    check(ctx, g)


def check_per_vertex(ctx, g, want=None, bu=None):
    r, pv = ctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v, per_vertex=True)
    if want is None:
        want = oracle.per_vertex(g).astype(np.int64)
    assert np.array_equal(pv, want), (g.name, np.nonzero(pv != want)[0][:10])
    b, u = bu if bu is not None else oracle.count(g)
    assert (r.balanced, r.unbalanced) == (b, u)
    # every balanced butterfly has two vertices on each side
    assert int(pv[:g.n_u].sum()) == 2 * b and int(pv[g.n_u:].sum()) == 2 * b
    return r, pv


def test_per_vertex_counts(ctx):
    fx = json.load(open(os.path.join(GOLDEN, "fig1_butterflies.json")))
    for pat in fx["patterns"]:
        g = graph_from_edges(2, 2, pat["edges"], pat["name"])
        r, pv = check_per_vertex(ctx, g)
        assert list(pv) == [pat["balanced"]] * 4
    rng = np.random.default_rng(41)
    for i in range(40):
        g = gen.random_graph(rng, int(rng.integers(2, 40)), int(rng.integers(2, 40)),
                             float(rng.uniform(0.1, 0.8)), p_neg=float(rng.uniform(0, 1)))
        check_per_vertex(ctx, g)
    # K_{a,b} all positive: every vertex of U lies in (a-1) C(b,2) butterflies
    g = gen.complete_graph(30, 50)
    r, pv = check_per_vertex(ctx, g)
    assert (pv[:30] == 29 * 50 * 49 // 2).all() and (pv[30:] == 49 * 30 * 29 // 2).all()


def test_per_vertex_heavy_shapes(ctx):
    # heavy starts with small end ranges (dense pieces), hubs, and a side
    # wider than one end-vertex tile (split starts)
    check_per_vertex(ctx, gen.voting_graph(seed=6, n_u=80, n_v=3000, p_edge=0.5))
    check_per_vertex(ctx, gen.chung_lu_graph(seed=11, n_u=60000, n_v=20000, n_edges=250000,
                                             p_neg=0.25))
    g = gen.chung_lu_graph(seed=21, n_u=200000, n_v=60000, n_edges=1500000, alpha=2.1, p_neg=0.2)
    want, bu = oracle.per_vertex(g).astype(np.int64), oracle.count(g)
    check_per_vertex(ctx, g, want, bu)
    ctx.set_param(bbc.PARAM_PROBE_LIMIT, 4)  # split pieces redone many times
    try:
        check_per_vertex(ctx, g, want, bu)
        assert ctx.stats()[5] > 100
    finally:
        ctx.set_param(bbc.PARAM_PROBE_LIMIT, 256)
    # the plain count is unchanged by asking for per-vertex counts
    assert ctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v)[:2] == bu


def test_per_vertex_on_device(ctx):
    # the per-vertex counts written straight into a device buffer equal the
    # host copy; on error the device buffer is left as it was
    import torch
    for g in (gen.voting_graph(seed=6, n_u=80, n_v=3000, p_edge=0.5),
              gen.chung_lu_graph(seed=11, n_u=60000, n_v=20000, n_edges=250000, p_neg=0.25)):
        r_h, pv_h = ctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v, per_vertex=True)
        r_d, pv_d = ctx.count(g.eu, g.ev, g.sign, g.n_u, g.n_v, per_vertex=True,
                              per_vertex_on_device=True)
        assert pv_d.is_cuda and r_d == r_h
        assert np.array_equal(pv_d.cpu().numpy(), pv_h)
    empty = ctx.count(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int8), 7, 5,
                      per_vertex=True, per_vertex_on_device=True)
    assert empty[0] == (0, 0, 0) and int(empty[1].abs().sum()) == 0 and empty[1].numel() == 12
    g = gen.uniform_graph(seed=3, n_u=100, n_v=80, n_edges=2000)
    bad = g.ev.copy()
    bad[5] = 80
    buf = torch.full((180,), -7, dtype=torch.int64, device="cuda:0")
    torch.cuda.synchronize()
    rc, _ = _raw(ctx, g._replace(ev=bad), bbc.PER_VERTEX | bbc.OUTPUT_ON_DEVICE, buf.data_ptr())
    assert rc == bbc.VERTEX_RANGE and bool((buf == -7).all())
    # the flag without per-vertex counts is rejected
    assert _raw(ctx, g, bbc.OUTPUT_ON_DEVICE)[0] == bbc.INVALID_ARG


def test_per_vertex_buffer_untouched_on_error(ctx):
    g = gen.uniform_graph(seed=3, n_u=100, n_v=80, n_edges=2000)
    bad = g.sign.copy()
    bad[5] = 3
    pv = np.full(180, -7, np.int64)
    out = bbc._CResult()
    p = [a.ctypes.data for a in (g.eu, g.ev, bad)]
    rc = ctx._lib.bbc_count(ctx._h, 100, 80, g.n_edges, *p, bbc.PER_VERTEX, ctypes.byref(out),
                            pv.ctypes.data)
    assert rc == bbc.BAD_SIGN and (pv == -7).all()
    assert ctx._lib.bbc_count(ctx._h, 100, 80, g.n_edges, *p[:2], g.sign.ctypes.data,
                              bbc.PER_VERTEX, ctypes.byref(out), None) == bbc.INVALID_ARG
