"""Seeded generators for signed bipartite graphs G = (U, V, E, sign).

Conventions shared by every consumer:
  * vertices of U are 0..n_u-1 and vertices of V are 0..n_v-1 (int32);
  * an edge i is (eu[i], ev[i]) with sign[i] in {+1, -1} (int8);
  * E is a set: no (u, v) pair appears twice (the problem definition takes
    E as a subset of U x V).

The workload recipes stand in for the paper's datasets (Section 6, Table 1),
none of which is available here: a small uniform graph, a dense voting-shaped
graph (few voters x many bills, like the Senate/House data) and a power-law
rating-shaped graph (like the Konect rating graphs, which the paper signs at
random).  Only numpy's PCG64 ``default_rng`` is used, so a seed fixes a graph
bit for bit on any machine with the same numpy.
"""
from __future__ import annotations

import math
from typing import NamedTuple

import numpy as np


class SignedBipartiteGraph(NamedTuple):
    n_u: int
    n_v: int
    eu: np.ndarray  # int32[E]
    ev: np.ndarray  # int32[E]
    sign: np.ndarray  # int8[E], +1 or -1
    name: str = ""

    @property
    def n_edges(self) -> int:
        return int(self.eu.shape[0])


def _signs(rng: np.random.Generator, m: int, p_neg) -> np.ndarray:
    """sign = -1 with probability p_neg (scalar or per-edge array), else +1."""
    neg = rng.random(m) < p_neg
    return np.where(neg, -1, 1).astype(np.int8)


def _pack(n_u, n_v, u, v, s, name):
    return SignedBipartiteGraph(int(n_u), int(n_v), np.ascontiguousarray(u, dtype=np.int32),
                                np.ascontiguousarray(v, dtype=np.int32),
                                np.ascontiguousarray(s, dtype=np.int8), name)


def uniform_graph(seed: int = 1, n_u: int = 2000, n_v: int = 1000, n_edges: int = 20000,
                  p_neg: float = 0.3) -> SignedBipartiteGraph:
    """Uniform random signed bipartite graph: n_edges distinct (u, v) pairs drawn
    without replacement from U x V, each sign independently -1 with p_neg."""
    rng = np.random.default_rng(seed)
    total = n_u * n_v
    if n_edges > total:
        raise ValueError("more edges than vertex pairs")
    keys = rng.choice(total, size=n_edges, replace=False)
    u = keys // n_v
    v = keys % n_v
    return _pack(n_u, n_v, u, v, _signs(rng, n_edges, p_neg), f"uniform{n_u}x{n_v}e{n_edges}s{seed}")


def voting_graph(seed: int = 2, n_u: int = 100, n_v: int = 10000, p_edge: float = 0.6,
                 neg_scale: float = 0.9) -> SignedBipartiteGraph:
    """Voting-shaped graph: every (u, v) present independently with p_edge; each
    voter u draws a bias b_u = neg_scale * Beta(2, 2) and each of its edges is
    negative with probability b_u (mean negative fraction neg_scale / 2 = 0.45).
    The edge list is returned in a random order."""
    rng = np.random.default_rng(seed)
    present = rng.random((n_u, n_v)) < p_edge
    bias = neg_scale * rng.beta(2.0, 2.0, size=n_u)
    u, v = np.nonzero(present)
    s = _signs(rng, u.shape[0], bias[u])
    order = rng.permutation(u.shape[0])
    return _pack(n_u, n_v, u[order], v[order], s[order], f"voting{n_u}x{n_v}p{p_edge}s{seed}")


def chung_lu_graph(seed: int = 3, n_u: int = 1_000_000, n_v: int = 300_000,
                   n_edges: int = 8_000_000, alpha: float = 2.1,
                   p_neg: float = 0.2) -> SignedBipartiteGraph:
    """Power-law rating-shaped graph ("fast Chung-Lu").

    Each vertex draws an expected-degree weight from Zipf(alpha), capped at the
    size of the other side.  Endpoint pairs are drawn independently with
    u ~ w_u and v ~ w_v; repeated pairs are dropped (first draw wins) and more
    pairs are drawn until exactly n_edges distinct pairs exist; the list is then
    shuffled.  Signs are iid, -1 with p_neg.
    """
    rng = np.random.default_rng(seed)
    wu = np.minimum(rng.zipf(alpha, n_u), n_v).astype(np.float64)
    wv = np.minimum(rng.zipf(alpha, n_v), n_u).astype(np.float64)
    cu = np.cumsum(wu)
    cu /= cu[-1]
    cv = np.cumsum(wv)
    cv /= cv[-1]
    kept = np.empty(0, dtype=np.int64)
    while kept.shape[0] < n_edges:
        need = n_edges - kept.shape[0]
        m = int(need * 1.25) + 1024
        u = np.minimum(np.searchsorted(cu, rng.random(m), side="right"), n_u - 1)
        v = np.minimum(np.searchsorted(cv, rng.random(m), side="right"), n_v - 1)
        keys = np.concatenate([kept, u.astype(np.int64) * n_v + v])
        _, first = np.unique(keys, return_index=True)
        first.sort()
        kept = keys[first]
    kept = kept[:n_edges]
    kept = kept[rng.permutation(n_edges)]
    u = kept // n_v
    v = kept % n_v
    return _pack(n_u, n_v, u, v, _signs(rng, n_edges, p_neg),
                 f"chunglu{n_u}x{n_v}e{n_edges}a{alpha}s{seed}")


def chung_lu_graph_fast(seed: int, n_u: int, n_v: int, n_edges: int, alpha: float = 2.1,
                        p_neg: float = 0.2) -> SignedBipartiteGraph:
    """Chung-Lu graph as chung_lu_graph (Zipf(alpha) weights capped at the
    other side's size, endpoints drawn independently in proportion to the
    weights), drawn in bulk for speed: the number of draws landing on each
    vertex is one multinomial sample per side, the two endpoint lists are
    shuffled and paired, and repeated pairs are removed by keeping a uniformly
    random n_edges of the distinct pairs (drawing more while there are too
    few).  Used for the large jobs of the serving workload (up to 3e7 edges)."""
    rng = np.random.default_rng(seed)
    wu = np.minimum(rng.zipf(alpha, n_u), n_v).astype(np.float64)
    wv = np.minimum(rng.zipf(alpha, n_v), n_u).astype(np.float64)
    pu = wu / wu.sum()
    pv = wv / wv.sum()
    kept = np.empty(0, dtype=np.int64)
    while kept.shape[0] < n_edges:
        m = int((n_edges - kept.shape[0]) * 1.3) + 1024
        u = np.repeat(np.arange(n_u, dtype=np.int64), rng.multinomial(m, pu))
        v = np.repeat(np.arange(n_v, dtype=np.int64), rng.multinomial(m, pv))
        rng.shuffle(u)
        rng.shuffle(v)
        kept = np.unique(np.concatenate([kept, u * n_v + v]))
    kept = kept[rng.permutation(kept.shape[0])[:n_edges]]
    u = kept // n_v
    v = kept % n_v
    return _pack(n_u, n_v, u, v, _signs(rng, n_edges, p_neg),
                 f"chunglufast{n_u}x{n_v}e{n_edges}a{alpha}s{seed}")


def serving_large_params(count: int, seed: int = 5):
    """Large jobs of the serving workload: |U|, |V| log-uniform in [1e5, 2e6],
    edges log-uniform in [1e6, 3e7] (at most |U||V|/4), P(-1) uniform in
    [0.1, 0.4]; returns a list of (seed, n_u, n_v, n_edges, p_neg)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nu = int(round(math.exp(rng.uniform(math.log(1e5), math.log(2e6)))))
        nv = int(round(math.exp(rng.uniform(math.log(1e5), math.log(2e6)))))
        m = int(round(math.exp(rng.uniform(math.log(1e6), math.log(3e7)))))
        out.append((100 + i, nu, nv, min(m, nu * nv // 4), float(rng.uniform(0.1, 0.4))))
    return out


def random_graph(rng: np.random.Generator, n_u: int, n_v: int, density: float,
                 p_neg: float = 0.5) -> SignedBipartiteGraph:
    """Small Erdos-Renyi-style bipartite graph for tests: each pair present with
    probability `density`, iid signs; the edge list is shuffled."""
    present = rng.random((n_u, n_v)) < density
    u, v = np.nonzero(present)
    s = _signs(rng, u.shape[0], p_neg)
    order = rng.permutation(u.shape[0])
    return _pack(n_u, n_v, u[order], v[order], s[order], f"er{n_u}x{n_v}d{density:.3f}")


def complete_graph(a: int, b: int, sign_u=None, sign_v=None) -> SignedBipartiteGraph:
    """K_{a,b}; with sign_u / sign_v (+-1 arrays) the edge (u, v) gets the sign
    sign_u[u] * sign_v[v] (a switching of the all-positive graph)."""
    u, v = np.meshgrid(np.arange(a), np.arange(b), indexing="ij")
    u = u.ravel()
    v = v.ravel()
    su = np.ones(a, dtype=np.int8) if sign_u is None else np.asarray(sign_u, dtype=np.int8)
    sv = np.ones(b, dtype=np.int8) if sign_v is None else np.asarray(sign_v, dtype=np.int8)
    s = (su[u] * sv[v]).astype(np.int8)
    return _pack(a, b, u, v, s, f"K{a},{b}")


# ---------------------------------------------------------------------------
# Many small graphs (the batched workload): per-graph parameters are drawn from
# one master stream; each graph's edges come from its own stream.

BATCH_MASTER_SEED = 4
BATCH_GRAPH_SEED0 = 10_000


def batch_graph_params(n_graphs: int, seed: int = BATCH_MASTER_SEED, lo: int = 16, hi: int = 4096,
                       dens_lo: float = 1e-3, dens_hi: float = 0.2):
    """Per-graph (n_u, n_v, n_edges): sides log-uniform in [lo, hi], density
    log-uniform in [dens_lo, dens_hi], n_edges = round(density * n_u * n_v)."""
    rng = np.random.default_rng(seed)
    nu = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n_graphs))).astype(np.int64)
    nv = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n_graphs))).astype(np.int64)
    dens = np.exp(rng.uniform(math.log(dens_lo), math.log(dens_hi), n_graphs))
    ne = np.rint(dens * nu * nv).astype(np.int64)
    return nu, nv, ne


def batch_graph(i: int, n_u: int, n_v: int, n_edges: int, p_neg: float = 0.3) -> SignedBipartiteGraph:
    """Graph i of the batched workload: n_edges distinct pairs drawn uniformly
    without replacement (seed BATCH_GRAPH_SEED0 + i)."""
    return uniform_graph(seed=BATCH_GRAPH_SEED0 + i, n_u=int(n_u), n_v=int(n_v),
                         n_edges=int(n_edges), p_neg=p_neg)


# ---------------------------------------------------------------------------

WORKLOADS = {
    "uniform": lambda: uniform_graph(),
    "voting": lambda: voting_graph(),
    "powerlaw": lambda: chung_lu_graph(),
}


def workload(name: str) -> SignedBipartiteGraph:
    """The three single-graph workloads: 'uniform' (2000x1000, 20K edges),
    'voting' (100x10000, p=0.6) and 'powerlaw' (1Mx300K, 8M edges)."""
    return WORKLOADS[name]()
