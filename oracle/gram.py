"""Closed form of the balanced count through integer matrix products (numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a same-side pair (a, c) let P = |Gamma(a) ∩ Gamma(c)| = l + m and
Q = sum over common neighbours b of sign(a,b) sign(c,b) = l - m, where l and m
count the symmetric and asymmetric wedges a-b-c (Section 4, Definitions 5-6).
Then the pair holds C(l,2) + C(m,2) = (P^2 + Q^2 - 2P) / 4 balanced and
l*m = (P^2 - Q^2) / 4 unbalanced butterflies (Lemma 2).  With the unsigned
adjacency A and the signed adjacency S of the smaller side, P = A A^T and
Q = S S^T; both are computed as float64 products, exact while every entry is
below 2^53, then summed over a < c in int64.
"""
from __future__ import annotations

import numpy as np


def gram_count(g, side: int | None = None):
    """(balanced, unbalanced) from the Gram matrices of side 0 (U) or 1 (V);
    by default the smaller side."""
    n_u, n_v = int(g.n_u), int(g.n_v)
    if side is None:
        side = 0 if n_u <= n_v else 1
    rows, cols = (g.eu, g.ev) if side == 0 else (g.ev, g.eu)
    nr, nc = (n_u, n_v) if side == 0 else (n_v, n_u)
    if nr * nc > 1 << 28:
        raise ValueError("graph too large for the dense closed form")
    s = np.zeros((nr, nc), dtype=np.float64)
    s[rows, cols] = g.sign.astype(np.float64)
    a = np.abs(s)
    p = np.rint(a @ a.T).astype(np.int64)
    q = np.rint(s @ s.T).astype(np.int64)
    iu = np.triu_indices(nr, k=1)
    pp = p[iu]
    qq = q[iu]
    num_b = pp * pp + qq * qq - 2 * pp
    num_u = pp * pp - qq * qq
    assert np.all(num_b % 4 == 0) and np.all(num_u % 4 == 0)
    return int(num_b.sum() // 4), int(num_u.sum() // 4)
