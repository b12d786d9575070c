"""CPU oracle for balanced-butterfly counting -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package.  The product library never loads it and shares no code
with it.  The C part (``oracle.c``) is compiled with gcc by :func:`build`; the
closed form of :mod:`oracle.gram` is plain numpy.

Every function takes a :class:`gen.SignedBipartiteGraph`-like object (``n_u``,
``n_v``, ``eu``, ``ev``, ``sign``) and returns Python ints.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

ERRORS = {
    -1: "invalid argument",
    -2: "vertex id out of range",
    -3: "sign not +1/-1",
    -4: "duplicate edge",
    -6: "overflow",
    -7: "out of memory",
}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, '?')}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no GPU code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I32, I64, I = ctypes.c_int32, ctypes.c_int64, ctypes.c_int
        lib.bbo_brute_force.argtypes = [I32, I32, I64, P, P, P, P, P]
        lib.bbo_pairs.argtypes = [I32, I32, I64, P, P, P, I, I, P]
        lib.bbo_pairs_rows.argtypes = [I32, I32, I64, P, P, P, I, I32, I32, I, P]
        lib.bbo_bucket.argtypes = [I32, I32, I64, P, P, P, I, P]
        lib.bbo_per_vertex.argtypes = [I32, I32, I64, P, P, P, I, P]
        lib.bbo_wedges.argtypes = [I32, I32, I64, P, P, P, I, P]
        for f in (lib.bbo_brute_force, lib.bbo_pairs, lib.bbo_pairs_rows, lib.bbo_per_vertex,
                  lib.bbo_wedges, lib.bbo_bucket):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _args(g):
    eu = np.ascontiguousarray(g.eu, dtype=np.int32)
    ev = np.ascontiguousarray(g.ev, dtype=np.int32)
    sg = np.ascontiguousarray(g.sign, dtype=np.int8)
    keep = (eu, ev, sg)
    return keep, (int(g.n_u), int(g.n_v), int(eu.shape[0]), eu.ctypes.data, ev.ctypes.data,
                  sg.ctypes.data)


def _check(rc):
    if rc != 0:
        raise OracleError(rc)


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


def brute_force(g):
    """O0 (tiny graphs): (balanced, total) by checking every pair of U vertices
    against every pair of V vertices."""
    keep, a = _args(g)
    b = np.zeros(1, np.uint64)
    t = np.zeros(1, np.uint64)
    _check(_load().bbo_brute_force(*a, b.ctypes.data, t.ctypes.data))
    del keep
    return int(b[0]), int(t[0])


def pair_count(g, side: int = 0, threads: int | None = None):
    """O1: (balanced, unbalanced) from the same-side pairs of side 0 (U) or 1 (V)."""
    keep, a = _args(g)
    out = np.zeros(2, np.uint64)
    _check(_load().bbo_pairs(*a, int(side), int(threads or default_threads()), out.ctypes.data))
    del keep
    return int(out[0]), int(out[1])


def pair_count_rows(g, side: int, x0: int, x1: int, threads: int = 1):
    """O1 restricted to rows [x0, x1) of one side (for timing a bounded sample):
    (balanced, unbalanced) over pairs {x, z}, x0 <= x < x1, z > x.  The rows are
    split over `threads` threads."""
    keep, a = _args(g)
    out = np.zeros(2, np.uint64)
    _check(_load().bbo_pairs_rows(*a, int(side), int(x0), int(x1), int(threads), out.ctypes.data))
    del keep
    return int(out[0]), int(out[1])


def count(g, threads: int | None = None):
    """Balanced and unbalanced butterfly counts; both sides are computed and
    must agree (each butterfly has one U pair and one V pair)."""
    bu = pair_count(g, 0, threads)
    bv = pair_count(g, 1, threads)
    if bu != bv:
        raise AssertionError(f"oracle sides disagree: U {bu} vs V {bv}")
    return bu


def per_vertex(g, threads: int | None = None) -> np.ndarray:
    """uint64[n_u + n_v]: balanced butterflies containing each vertex (U then V)."""
    keep, a = _args(g)
    out = np.zeros(int(g.n_u) + int(g.n_v), np.uint64)
    _check(_load().bbo_per_vertex(*a, int(threads or default_threads()), out.ctypes.data))
    del keep
    return out


def bucket(g, threads: int | None = None):
    """The bucket method on the CPU (Algorithm 2; starts in parallel as in
    Algorithm 4): (balanced, unbalanced, W)."""
    keep, a = _args(g)
    out = np.zeros(3, np.uint64)
    _check(_load().bbo_bucket(*a, int(threads or default_threads()), out.ctypes.data))
    del keep
    return int(out[0]), int(out[1]), int(out[2])


def wedges(g, threads: int | None = None) -> int:
    """W: wedges (u, v, w) whose start u outranks both v and w under the
    (degree, id) vertex priority."""
    keep, a = _args(g)
    out = np.zeros(1, np.uint64)
    _check(_load().bbo_wedges(*a, int(threads or default_threads()), out.ctypes.data))
    del keep
    return int(out[0])
