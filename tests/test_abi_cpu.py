"""Host-side checks of the C ABI library (no GPU work is launched here)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2308_07932_amd as bbc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(bbc.LIB_PATH):
        from paper_2308_07932_amd import _build
        _build.build()
    return bbc.load_library()


def test_exports_every_declared_symbol(lib):
    names = bbc.declared_symbols()
    assert {"bbc_create", "bbc_destroy", "bbc_count", "bbc_status_string",
            "bbc_last_error"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", bbc.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(bbc_\w+)", out))
    for n in names:
        assert n in exported, n
        assert hasattr(lib, n)


def test_status_strings_and_version(lib):
    for code in range(0, -11, -1):
        s = bbc.status_string(code)
        assert s and s != "unknown status"
    assert bbc.status_string(5) == "unknown status"
    assert bbc.version() >= 10000


def test_create_argument_checks(lib):
    # NULL out pointer is rejected before any device query
    assert lib.bbc_create(0, None, None) == bbc.INVALID_ARG
    lib.bbc_destroy(None)  # NULL-safe


def test_param_calls_reject_null_context(lib):
    v = ctypes.c_int64()
    assert lib.bbc_set_param(None, 1, 4096) == bbc.INVALID_ARG
    assert lib.bbc_get_param(None, 1, ctypes.byref(v)) == bbc.INVALID_ARG


def test_no_device_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    h = ctypes.c_void_p()
    assert lib.bbc_create(0, None, ctypes.byref(h)) == bbc.DEVICE


def test_binding_rejects_mismatched_lengths():
    with pytest.raises(ValueError):
        bbc._prepare(np.zeros(3, np.int32), np.zeros(2, np.int32), np.ones(3, np.int8))


def test_product_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2308_07932_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\bimport oracle\b|from oracle\b|liboracle|bbo_", text), f


def test_batch_call_rejects_null_context(lib):
    import numpy as np
    nu = np.ones(1, np.int32)
    off = np.zeros(2, np.int64)
    assert lib.bbc_count_batch(None, 1, nu.ctypes.data, nu.ctypes.data, off.ctypes.data,
                               None, None, None, 0, None, None) == bbc.INVALID_ARG


def test_concat_graphs_layout():
    import numpy as np
    import gen
    gs = [gen.uniform_graph(seed=i, n_u=10 + i, n_v=8, n_edges=5 * i) for i in range(4)]
    nu, nv, off, eu, ev, sg = bbc.concat_graphs(gs)
    assert list(nu) == [10, 11, 12, 13] and list(nv) == [8] * 4
    assert list(off) == [0, 0, 5, 15, 30]
    for i, g in enumerate(gs):
        assert np.array_equal(eu[off[i]:off[i + 1]], g.eu)
        assert np.array_equal(sg[off[i]:off[i + 1]], g.sign)


def test_server_argument_checks(lib):
    import ctypes
    cfg = bbc._CServerConfig(0, 99, 0, 0, 0)  # too many workers
    h = ctypes.c_void_p()
    assert lib.bbc_server_create(ctypes.byref(cfg), ctypes.byref(h)) == bbc.INVALID_ARG
    assert lib.bbc_server_create(None, None) == bbc.INVALID_ARG
    t = ctypes.c_uint64()
    assert lib.bbc_server_submit(None, 1, 1, 0, None, None, None, ctypes.byref(t)) == bbc.INVALID_ARG
    out = bbc._CResult()
    st = ctypes.c_int32()
    assert lib.bbc_server_poll(None, 1, 0, ctypes.byref(out), ctypes.byref(st), None) == bbc.INVALID_ARG
    lib.bbc_server_destroy(None)


def test_workspace_estimate():
    assert bbc.workspace_bytes(-1, 5, 5) == -1
    assert bbc.workspace_bytes(1 << 30, 0, 5) == -1
    # edges: the CSR's 2m entries and its 1024 pad entries keep 32-bit positions
    assert bbc.workspace_bytes(1000, 1000, (1 << 31) - 1024) == -1
    assert bbc.workspace_bytes(1000, 1000, (1 << 31) - 1025) > 0
    a = bbc.workspace_bytes(1000, 1000, 10000)
    b = bbc.workspace_bytes(1000, 1000, 100000)
    c = bbc.workspace_bytes(100000, 1000, 100000)
    assert 0 < a < b < c


def test_noalloc_scratch_size_matches_header():
    text = open(bbc.HEADER_PATH).read()
    m = re.search(r"#define\s+BBC_NOALLOC_SCRATCH_BYTES\s+\((\d+)ull\s*<<\s*(\d+)\)", text)
    assert m, "BBC_NOALLOC_SCRATCH_BYTES not found in bbc.h"
    assert int(m.group(1)) << int(m.group(2)) == bbc.NOALLOC_SCRATCH_BYTES
