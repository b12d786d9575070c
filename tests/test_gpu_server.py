"""The counting service (bbc_server_*): jobs of mixed sizes submitted while
others run are batched continuously and overlap on the device; each result
must equal the oracle's count of that graph alone."""
from __future__ import annotations

import threading
import time

import numpy as np
import pytest

import gen
import oracle
import paper_2308_07932_amd as bbc
from gen import SignedBipartiteGraph

pytestmark = pytest.mark.gpu


def small_graphs(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nu, nv = int(rng.integers(2, 300)), int(rng.integers(2, 300))
        m = int(rng.integers(1, min(nu * nv, 4000)))
        out.append(gen.uniform_graph(seed=5000 + seed * 1000 + i, n_u=nu, n_v=nv, n_edges=m,
                                     p_neg=float(rng.uniform(0.05, 0.6))))
    return out


def expect(g):
    b, u = oracle.count(g)
    return bbc.Result(b, u, oracle.wedges(g))


def test_server_mixed_stream_exact():
    large = [gen.chung_lu_graph(seed=41 + i, n_u=150000, n_v=50000, n_edges=900000, alpha=2.1,
                                p_neg=0.1 + 0.1 * i) for i in range(3)]
    small = small_graphs(1, 300)
    want = {}
    for i, g in enumerate(large):
        want[("L", i)] = expect(g)
    for i, g in enumerate(small):
        want[("S", i)] = expect(g)
    with bbc.Server(0, large_workers=2) as srv:
        tickets = {}
        lock = threading.Lock()

        def feed(kind, graphs, delay):
            for i, g in enumerate(graphs):
                t = srv.submit(g.eu, g.ev, g.sign, g.n_u, g.n_v)
                with lock:
                    tickets[t] = (kind, i)
                time.sleep(delay)

        th = [threading.Thread(target=feed, args=("L", large, 0.01)),
              threading.Thread(target=feed, args=("S", small[:150], 0.0005)),
              threading.Thread(target=feed, args=("S2", small[150:], 0.0002))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        got = {}
        for t, key in tickets.items():
            r = srv.poll(t, wait_ms=-1)
            kind, i = key
            if kind == "S2":
                key = ("S", 150 + i)
            got[key] = r
        st = srv.stats()
    assert len(got) == len(want)
    for key, r in got.items():
        assert r.status == bbc.OK, (key, r)
        assert r.result == want[key], (key, r.result, want[key])
        assert r.latency_ms > 0
    assert st["submitted"] == st["completed"] == len(want)
    assert st["batched_jobs"] == len(small)
    assert st["batches"] >= 2, st  # jobs arriving during a batch went into later ones
    assert st["peak_running"] >= 2, st  # work from several jobs on the device at once


def test_server_memory_admission():
    # A budget that binds: room for about one large job.  The reservations cover
    # what the workers' workspaces really hold (they keep their arenas between
    # jobs), so the device memory the server takes, sampled while it runs,
    # stays within the budget plus a fixed slack (allocation granularity).
    import threading

    import torch
    graphs = [gen.chung_lu_graph(seed=51 + i, n_u=100000, n_v=40000, n_edges=400000, alpha=2.1,
                                 p_neg=0.3) for i in range(4)]
    fp = max(bbc.workspace_bytes(g.n_u, g.n_v, g.n_edges) + 9 * g.n_edges for g in graphs)
    budget = int(fp * 1.5)  # room for one large job at a time
    huge = gen.chung_lu_graph(seed=59, n_u=300000, n_v=100000, n_edges=3000000, alpha=2.1)
    assert bbc.workspace_bytes(huge.n_u, huge.n_v, huge.n_edges) > budget
    small = small_graphs(2, 40)
    want = [expect(g) for g in graphs + small]
    torch.cuda.synchronize()
    with bbc.Server(0, large_workers=3, memory_budget=budget) as srv:
        torch.cuda.synchronize()
        free0, total = torch.cuda.mem_get_info()
        peak = [0]
        stop = threading.Event()

        def sample():
            while not stop.is_set():
                free, _ = torch.cuda.mem_get_info()
                peak[0] = max(peak[0], free0 - free)
                stop.wait(0.001)

        th_s = threading.Thread(target=sample)
        th_s.start()
        try:
            for rnd in range(2):  # twice: the second round meets warm, resident workspaces
                tl = [srv.submit(g.eu, g.ev, g.sign, g.n_u, g.n_v) for g in graphs]
                th = srv.submit(huge.eu, huge.ev, huge.sign, huge.n_u, huge.n_v)
                ts = [srv.submit(g.eu, g.ev, g.sign, g.n_u, g.n_v) for g in small]
                rl = [srv.poll(t) for t in tl]
                rh = srv.poll(th)
                rs = [srv.poll(t) for t in ts]
                assert rh.status == bbc.OUT_OF_MEMORY
                for w, r in zip(want, rl + rs):
                    assert r.status == bbc.OK
                    assert r.result == w
        finally:
            stop.set()
            th_s.join()
        st = srv.stats()
    print(f"[gpu] admission: budget {budget}, peak device bytes taken {peak[0]}, stats {st}",
          flush=True)
    assert st["peak_reserved"] <= budget, st
    assert st["budget"] == budget
    assert peak[0] <= budget + (64 << 20), (peak[0], budget)


def test_server_reports_bad_jobs_and_keeps_going():
    good = small_graphs(3, 20)
    g = good[4]
    s = g.sign.copy()
    s[0] = 2
    bad = g._replace(sign=s)
    big_bad = gen.chung_lu_graph(seed=61, n_u=40000, n_v=20000, n_edges=100000)
    dup = big_bad._replace(eu=np.append(big_bad.eu, big_bad.eu[7]),
                           ev=np.append(big_bad.ev, big_bad.ev[7]),
                           sign=np.append(big_bad.sign, big_bad.sign[7]))
    with bbc.Server(0) as srv:
        tb = srv.submit(bad.eu, bad.ev, bad.sign, bad.n_u, bad.n_v)
        td = srv.submit(dup.eu, dup.ev, dup.sign, dup.n_u, dup.n_v)
        tg = [srv.submit(x.eu, x.ev, x.sign, x.n_u, x.n_v) for x in good]
        assert srv.poll(tb).status == bbc.BAD_SIGN
        assert srv.poll(td).status == bbc.DUPLICATE_EDGE
        for x, t in zip(good, tg):
            r = srv.poll(t)
            assert r.status == bbc.OK and r.result == expect(x)
        with pytest.raises(bbc.BBCError):
            srv.poll(tg[0])  # released after its result was taken
        empty = SignedBipartiteGraph(5, 5, np.zeros(0, np.int32), np.zeros(0, np.int32),
                                     np.zeros(0, np.int8), "empty")
        r = srv.poll(srv.submit(empty.eu, empty.ev, empty.sign, 5, 5))
        assert r.status == bbc.OK and r.result == bbc.Result(0, 0, 0)
