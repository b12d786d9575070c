"""Balanced-butterfly counting on AMD MI355X: Python binding of libbbc.so.

Argument marshalling only; every step of the count runs in the HIP library.
There is no CPU fallback: if the library is missing, importing works but any
call raises :class:`LibraryNotBuilt`.

    >>> import paper_2308_07932_amd as bbc
    >>> r = bbc.count(eu, ev, sign, n_u, n_v)     # numpy (host) or torch (device)
    >>> r.balanced, r.unbalanced, r.wedges

Tensors on a GPU are passed as device pointers; the call is ordered after the
work already queued on torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import NamedTuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbbc.so")
HEADER_PATH = os.path.join(_HERE, "..", "include", "bbc.h")

PENDING = 1
OK = 0
INVALID_ARG = -1
VERTEX_RANGE = -2
BAD_SIGN = -3
DUPLICATE_EDGE = -4
TOO_LARGE = -5
OVERFLOW = -6
OUT_OF_MEMORY = -7
DEVICE = -8
NOT_IMPLEMENTED = -9
INTERNAL = -10

INPUT_ON_DEVICE = 1
OUTPUT_ON_DEVICE = 2
PER_VERTEX = 4
PARAM_HASH_TARGET = 1
PARAM_PROBE_LIMIT = 2
PARAM_CHUNK_WEDGES = 3
PARAM_GRAPHS = 4
PARAM_GRAPH_CAPTURES = 5
PARAM_GRAPH_REPLAYS = 6
PARAM_LIGHT_MAX = 7
PARAM_GRAB_DIV = 8
PARAM_UNION_EDGES = 9
PARAM_WAVE_SHARE = 10

PHASE_TOTAL, PHASE_PREP, PHASE_WEDGE, PHASE_PLAN = 0, 1, 2, 3

# size of the static device scratch that bbc_count_noalloc works in (bbc.h)
NOALLOC_SCRATCH_BYTES = 256 << 20


class LibraryNotBuilt(ImportError):
    pass


class BBCError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"bbc error {code}: {message}")
        self.code = code
        self.message = message


class Result(NamedTuple):
    balanced: int
    unbalanced: int
    wedges: int


class _CResult(ctypes.Structure):
    _fields_ = [("balanced", ctypes.c_int64), ("unbalanced", ctypes.c_int64),
                ("wedges", ctypes.c_int64)]


_lib = None


def library_path() -> str:
    return LIB_PATH


def load_library():
    """Load libbbc.so (built in-tree by ``python -m paper_2308_07932_amd._build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryNotBuilt(f"{LIB_PATH} is missing; build it with "
                              "`python -m paper_2308_07932_amd._build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.bbc_create.argtypes = [ctypes.c_int, P, ctypes.POINTER(P)]
    lib.bbc_create.restype = ctypes.c_int
    lib.bbc_destroy.argtypes = [P]
    lib.bbc_destroy.restype = None
    lib.bbc_count.argtypes = [P, I32, I32, I64, P, P, P, U32, ctypes.POINTER(_CResult), P]
    lib.bbc_count.restype = ctypes.c_int
    lib.bbc_status_string.argtypes = [ctypes.c_int]
    lib.bbc_status_string.restype = ctypes.c_char_p
    lib.bbc_last_error.argtypes = [P]
    lib.bbc_last_error.restype = ctypes.c_char_p
    lib.bbc_version.argtypes = []
    lib.bbc_version.restype = ctypes.c_int
    lib.bbc_set_timing.argtypes = [P, ctypes.c_int]
    lib.bbc_set_timing.restype = ctypes.c_int
    lib.bbc_last_phase_ms.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.bbc_last_phase_ms.restype = ctypes.c_int
    lib.bbc_last_stats.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.bbc_last_stats.restype = ctypes.c_int
    lib.bbc_set_param.argtypes = [P, ctypes.c_int, I64]
    lib.bbc_set_param.restype = ctypes.c_int
    lib.bbc_get_param.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
    lib.bbc_get_param.restype = ctypes.c_int
    lib.bbc_count_noalloc.argtypes = [P, I32, I32, I64, P, P, P, U32, ctypes.POINTER(_CResult), P]
    lib.bbc_count_noalloc.restype = ctypes.c_int
    lib.bbc_count_batch.argtypes = [P, I32, P, P, P, P, P, P, U32, P, P]
    lib.bbc_count_batch.restype = ctypes.c_int
    lib.bbc_autotune.argtypes = [P, I32, P, P, P, P, P, P, U32, I32,
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    lib.bbc_autotune.restype = ctypes.c_int
    lib.bbc_workspace_bytes.argtypes = [I32, I32, I64]
    lib.bbc_workspace_bytes.restype = ctypes.c_int64
    lib.bbc_server_create.argtypes = [P, ctypes.POINTER(P)]
    lib.bbc_server_create.restype = ctypes.c_int
    lib.bbc_server_submit.argtypes = [P, I32, I32, I64, P, P, P, ctypes.POINTER(ctypes.c_uint64)]
    lib.bbc_server_submit.restype = ctypes.c_int
    lib.bbc_server_poll.argtypes = [P, ctypes.c_uint64, I32, ctypes.POINTER(_CResult),
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    lib.bbc_server_poll.restype = ctypes.c_int
    lib.bbc_server_stats.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.bbc_server_stats.restype = ctypes.c_int
    lib.bbc_server_destroy.argtypes = [P]
    lib.bbc_server_destroy.restype = None
    _lib = lib
    return lib


def declared_symbols() -> list[str]:
    """Function names declared in include/bbc.h."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bbc_[a-z_]+)\s*\(", text)))


def status_string(code: int) -> str:
    return load_library().bbc_status_string(int(code)).decode()


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _prepare(eu, ev, sign):
    """Return (pointers, keepalive, on_device, n_edges)."""
    if _is_torch(eu):
        import torch  # noqa: F401  (only needed for tensors)
        ts = (eu, ev, sign)
        if not all(_is_torch(t) for t in ts):
            raise TypeError("eu, ev and sign must all be torch tensors or all be arrays")
        dev = {t.device.type for t in ts}
        if len(dev) != 1:
            raise ValueError("eu, ev and sign must live on the same device")
        want = ("int32", "int32", "int8")
        ts = tuple(t.contiguous() for t in ts)
        for t, w in zip(ts, want):
            if str(t.dtype) != f"torch.{w}":
                raise TypeError(f"expected torch.{w}, got {t.dtype}")
        n = int(ts[0].numel())
        if int(ts[1].numel()) != n or int(ts[2].numel()) != n:
            raise ValueError("eu, ev and sign must have the same length")
        on_dev = ts[0].is_cuda
        return tuple(t.data_ptr() for t in ts), ts, on_dev, n
    arrs = (np.ascontiguousarray(eu, dtype=np.int32), np.ascontiguousarray(ev, dtype=np.int32),
            np.ascontiguousarray(sign, dtype=np.int8))
    n = int(arrs[0].shape[0])
    if arrs[1].shape[0] != n or arrs[2].shape[0] != n:
        raise ValueError("eu, ev and sign must have the same length")
    return tuple(a.ctypes.data for a in arrs), arrs, False, n


class Context:
    """A libbbc context: device, stream and a reusable device workspace."""

    def __init__(self, device: int = 0, stream: int | None = None):
        lib = load_library()
        h = ctypes.c_void_p()
        rc = lib.bbc_create(int(device), ctypes.c_void_p(stream) if stream else None,
                            ctypes.byref(h))
        if rc != OK:
            raise BBCError(rc, f"bbc_create(device={device}): {status_string(rc)}")
        self._lib = lib
        self._h = h
        self.device = int(device)
        self.stream = stream

    def close(self):
        if getattr(self, "_h", None):
            self._lib.bbc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_param(self, param: int, value: int):
        rc = self._lib.bbc_set_param(self._h, int(param), int(value))
        if rc != OK:
            raise BBCError(rc, f"parameter {param} = {value} rejected")

    def get_param(self, param: int) -> int:
        v = ctypes.c_int64()
        rc = self._lib.bbc_get_param(self._h, int(param), ctypes.byref(v))
        if rc != OK:
            raise BBCError(rc, f"unknown parameter {param}")
        return int(v.value)

    def set_timing(self, on: bool = True):
        self._lib.bbc_set_timing(self._h, 1 if on else 0)

    def phase_ms(self, phase: int) -> float:
        v = ctypes.c_double()
        rc = self._lib.bbc_last_phase_ms(self._h, int(phase), ctypes.byref(v))
        if rc != OK:
            raise BBCError(rc, "no phase timing for the last call (enable set_timing)")
        return float(v.value)

    def stats(self) -> list[int]:
        a = (ctypes.c_int64 * 14)()
        self._lib.bbc_last_stats(self._h, a, 14)
        return list(a)

    def last_error(self) -> str:
        return self._lib.bbc_last_error(self._h).decode()

    def count_raw(self, n_u: int, n_v: int, n_edges: int, p_u: int, p_v: int, p_s: int,
                  flags: int = 0, per_vertex_ptr: int | None = None) -> Result:
        """Pointer-level entry (ints are addresses); raises BBCError on failure."""
        out = _CResult()
        rc = self._lib.bbc_count(self._h, int(n_u), int(n_v), int(n_edges), p_u, p_v, p_s,
                                 int(flags), ctypes.byref(out), per_vertex_ptr)
        if rc != OK:
            raise BBCError(rc, self.last_error() or status_string(rc))
        return Result(int(out.balanced), int(out.unbalanced), int(out.wedges))

    def count(self, eu, ev, sign, n_u: int, n_v: int, per_vertex: bool = False,
              per_vertex_on_device: bool = False):
        """Count the balanced butterflies of the signed bipartite graph given by
        edges (eu[i], ev[i]) with sign[i] in {+1, -1}.  Returns a Result, or
        (Result, per-vertex int64 array) when per_vertex is set: a numpy array,
        or with per_vertex_on_device a torch tensor on the context's device."""
        ptrs, keep, on_dev, n = _prepare(eu, ev, sign)
        flags = INPUT_ON_DEVICE if on_dev else 0
        pv = None
        pv_ptr = None
        if per_vertex and per_vertex_on_device:
            import torch
            flags |= PER_VERTEX | OUTPUT_ON_DEVICE
            pv = torch.empty(int(n_u) + int(n_v), dtype=torch.int64,
                             device=torch.device("cuda", self.device))
            pv_ptr = pv.data_ptr()
        elif per_vertex:
            flags |= PER_VERTEX
            pv = np.zeros(int(n_u) + int(n_v), dtype=np.int64)
            pv_ptr = pv.ctypes.data
        if on_dev or (per_vertex and per_vertex_on_device):
            # torch's pending work on these buffers is done before the library's
            # stream reads or writes them (the call itself ends synchronized)
            import torch
            dev = keep[0].device if on_dev else torch.device("cuda", self.device)
            cur = torch.cuda.current_stream(dev)
            if self.stream is None or int(cur.cuda_stream) != int(self.stream):
                cur.synchronize()
        r = self.count_raw(n_u, n_v, n, *ptrs, flags=flags, per_vertex_ptr=pv_ptr)
        del keep
        return (r, pv) if per_vertex else r

    def count_noalloc(self, eu, ev, sign, n_u: int, n_v: int, per_vertex_out=None) -> Result:
        """bbc_count_noalloc: the count without any allocation in the library.
        eu, ev, sign are torch tensors on the context's device; per_vertex_out,
        if given, is a caller-allocated int64 device tensor of n_u + n_v
        entries that receives the per-vertex counts."""
        ptrs, keep, on_dev, n = _prepare(eu, ev, sign)
        if not on_dev:
            raise ValueError("count_noalloc takes device tensors")
        flags = INPUT_ON_DEVICE
        pv_ptr = None
        if per_vertex_out is not None:
            if str(per_vertex_out.dtype) != "torch.int64" or not per_vertex_out.is_cuda or \
                    int(per_vertex_out.numel()) != int(n_u) + int(n_v):
                raise ValueError("per_vertex_out must be an int64 device tensor of n_u + n_v entries")
            flags |= PER_VERTEX | OUTPUT_ON_DEVICE
            pv_ptr = per_vertex_out.data_ptr()
        import torch
        cur = torch.cuda.current_stream(keep[0].device)
        if self.stream is None or int(cur.cuda_stream) != int(self.stream):
            cur.synchronize()
        out = _CResult()
        rc = self._lib.bbc_count_noalloc(self._h, int(n_u), int(n_v), int(n), *ptrs, int(flags),
                                         ctypes.byref(out), pv_ptr)
        del keep
        if rc != OK:
            raise BBCError(rc, self.last_error() or status_string(rc))
        return Result(int(out.balanced), int(out.unbalanced), int(out.wedges))

    def autotune(self, n_u, n_v, edge_offset, eu, ev, sign, repeats: int = 2):
        """bbc_autotune on a batch (or one graph): returns ({chunk_wedges,
        hash_target, probe_limit, light_max, grab_div, union_edges}, best call
        ms); the settings stay on the context."""
        nu = np.ascontiguousarray(n_u, dtype=np.int32)
        nv = np.ascontiguousarray(n_v, dtype=np.int32)
        off = np.ascontiguousarray(edge_offset, dtype=np.int64)
        ptrs, keep, on_dev, n = _prepare(eu, ev, sign)
        if on_dev:
            import torch
            cur = torch.cuda.current_stream(keep[0].device)
            if self.stream is None or int(cur.cuda_stream) != int(self.stream):
                cur.synchronize()
        ch = (ctypes.c_int64 * 6)()
        best = ctypes.c_double()
        rc = self._lib.bbc_autotune(self._h, int(nu.shape[0]), nu.ctypes.data, nv.ctypes.data,
                                    off.ctypes.data, *ptrs, INPUT_ON_DEVICE if on_dev else 0,
                                    int(repeats), ch, ctypes.byref(best))
        del keep
        if rc != OK:
            raise BBCError(rc, self.last_error() or status_string(rc))
        return {"chunk_wedges": int(ch[0]), "hash_target": int(ch[1]),
                "probe_limit": int(ch[2]), "light_max": int(ch[3]), "grab_div": int(ch[4]),
                "union_edges": int(ch[5])}, float(best.value)

    def count_batch(self, n_u, n_v, edge_offset, eu, ev, sign) -> "BatchResult":
        """Count many graphs in one call (bbc_count_batch): n_u, n_v (n_graphs
        entries), edge_offset (n_graphs + 1) and the concatenated local-id edge
        arrays (numpy, or torch CUDA tensors).  Returns a BatchResult."""
        return _count_batch(self, n_u, n_v, edge_offset, eu, ev, sign)


class BatchResult(NamedTuple):
    """Per-graph outputs of count_batch (numpy arrays of length n_graphs)."""
    balanced: np.ndarray
    unbalanced: np.ndarray
    wedges: np.ndarray
    status: np.ndarray

    def result(self, g: int) -> Result:
        return Result(int(self.balanced[g]), int(self.unbalanced[g]), int(self.wedges[g]))


def concat_graphs(graphs):
    """Concatenate graphs (objects with n_u, n_v, eu, ev, sign) into the batch
    layout: (n_u, n_v, edge_offset, eu, ev, sign) as numpy arrays."""
    nu = np.array([g.n_u for g in graphs], dtype=np.int32)
    nv = np.array([g.n_v for g in graphs], dtype=np.int32)
    lens = np.array([len(g.eu) for g in graphs], dtype=np.int64)
    off = np.zeros(len(graphs) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    cat = (lambda xs, dt: np.concatenate([np.asarray(x, dtype=dt) for x in xs])
           if len(xs) else np.zeros(0, dtype=dt))
    return (nu, nv, off, cat([g.eu for g in graphs], np.int32), cat([g.ev for g in graphs], np.int32),
            cat([g.sign for g in graphs], np.int8))


def _count_batch(ctx, n_u, n_v, edge_offset, eu, ev, sign) -> BatchResult:
    nu = np.ascontiguousarray(n_u, dtype=np.int32)
    nv = np.ascontiguousarray(n_v, dtype=np.int32)
    off = np.ascontiguousarray(edge_offset, dtype=np.int64)
    G = int(nu.shape[0])
    if nv.shape[0] != G or off.shape[0] != G + 1:
        raise ValueError("n_u and n_v need n_graphs entries and edge_offset n_graphs + 1")
    ptrs, keep, on_dev, n = _prepare(eu, ev, sign)
    if G and int(off[-1]) > n:
        raise ValueError("edge_offset points past the edge arrays")
    if on_dev:
        import torch
        cur = torch.cuda.current_stream(keep[0].device)
        if ctx.stream is None or int(cur.cuda_stream) != int(ctx.stream):
            cur.synchronize()
    out = (_CResult * max(G, 1))()
    st = np.zeros(max(G, 1), dtype=np.int32)
    rc = ctx._lib.bbc_count_batch(ctx._h, G, nu.ctypes.data, nv.ctypes.data, off.ctypes.data,
                                  *ptrs, INPUT_ON_DEVICE if on_dev else 0, out, st.ctypes.data)
    del keep
    if rc != OK:
        raise BBCError(rc, ctx.last_error() or status_string(rc))
    arr = np.frombuffer(out, dtype=np.int64).reshape(-1, 3)[:G]
    return BatchResult(arr[:, 0].copy(), arr[:, 1].copy(), arr[:, 2].copy(), st[:G].copy())


class _CServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("large_workers", ctypes.c_int32),
                ("memory_budget", ctypes.c_int64), ("small_side", ctypes.c_int32),
                ("max_batch_graphs", ctypes.c_int32)]


class JobResult(NamedTuple):
    status: int
    result: Result
    latency_ms: float


def workspace_bytes(n_u: int, n_v: int, n_edges: int) -> int:
    return int(load_library().bbc_workspace_bytes(int(n_u), int(n_v), int(n_edges)))


class Server:
    """bbc_server: jobs submitted at any time, small ones counted in continuous
    batches, large ones on concurrent streams, admitted by device memory."""

    def __init__(self, device: int = 0, large_workers: int = 0, memory_budget: int = 0,
                 small_side: int = 0, max_batch_graphs: int = 0):
        lib = load_library()
        cfg = _CServerConfig(int(device), int(large_workers), int(memory_budget), int(small_side),
                             int(max_batch_graphs))
        h = ctypes.c_void_p()
        rc = lib.bbc_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != OK:
            raise BBCError(rc, f"bbc_server_create: {status_string(rc)}")
        self._lib = lib
        self._h = h

    def submit(self, eu, ev, sign, n_u: int, n_v: int) -> int:
        """Queue one graph (host arrays, copied); returns its ticket."""
        ptrs, keep, on_dev, n = _prepare(eu, ev, sign)
        if on_dev:
            raise TypeError("the server takes host arrays")
        t = ctypes.c_uint64()
        rc = self._lib.bbc_server_submit(self._h, int(n_u), int(n_v), n, *ptrs, ctypes.byref(t))
        del keep
        if rc != OK:
            raise BBCError(rc, f"bbc_server_submit: {status_string(rc)}")
        return int(t.value)

    def poll(self, ticket: int, wait_ms: int = -1):
        """JobResult when the job is done (the ticket is then released), else None."""
        out = _CResult()
        st = ctypes.c_int32()
        lat = ctypes.c_double()
        rc = self._lib.bbc_server_poll(self._h, int(ticket), int(wait_ms), ctypes.byref(out),
                                       ctypes.byref(st), ctypes.byref(lat))
        if rc == PENDING:
            return None
        if rc != OK:
            raise BBCError(rc, f"bbc_server_poll({ticket}): {status_string(rc)}")
        return JobResult(int(st.value), Result(int(out.balanced), int(out.unbalanced),
                                               int(out.wedges)), float(lat.value))

    def stats(self) -> dict:
        a = (ctypes.c_int64 * 12)()
        self._lib.bbc_server_stats(self._h, a, 12)
        keys = ("submitted", "completed", "batches", "batched_jobs", "max_batch", "peak_reserved",
                "peak_running", "budget", "waiting", "reserved", "trims", "retries")
        return dict(zip(keys, (int(x) for x in a)))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.bbc_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default: dict[int, Context] = {}


def default_context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def count(eu, ev, sign, n_u: int, n_v: int, per_vertex: bool = False, device: int = 0):
    """Module-level convenience: count on the default context of `device`."""
    return default_context(device).count(eu, ev, sign, n_u, n_v, per_vertex=per_vertex)


def version() -> int:
    return int(load_library().bbc_version())
