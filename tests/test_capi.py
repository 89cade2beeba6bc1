"""C-ABI checks that need no GPU: the built library loads, exports every function the
header declares, and rejects invalid arguments on the host before touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "speedann.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sa_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def B():
    from paper_2201_13007_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libspeedann.so is not built; run __graft_entry__.build()")
    return binding


def test_exports_match_header(B):
    names = declared_functions()
    assert "sa_search" in names and "sa_build_graph" in names and "sa_knn" in names
    L = B.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(B.EXPORTS) == names


def test_default_params(B):
    p = B.SearchParams()
    B.lib().sa_default_params(C.byref(p))
    assert p.sync == 2 and abs(p.rho - 0.8) < 1e-7 and p.staged == 1 and p.static_I == 0


def _err(B):
    return B.lib().sa_last_error().decode()


def test_validation_errors_without_device(B):
    L = B.lib()
    fake = 1 << 20   # an aligned non-null address; never dereferenced on these paths
    out = C.c_void_p(0)
    # index creation touches no device
    assert L.sa_index_create(fake, 100, 30, 32, 0, fake, 16, 0, C.byref(out)) == -1
    assert "multiple of 4" in _err(B)
    assert L.sa_index_create(fake, 100, 32, 32, 0, fake, 65, 0, C.byref(out)) == -1
    assert "R=65" in _err(B)
    assert L.sa_index_create(fake, 100, 32, 32, 0, fake, 16, 100, C.byref(out)) == -1
    assert "entry" in _err(B)
    assert L.sa_index_create(fake, 100, 32, 32, 7, fake, 16, 0, C.byref(out)) == -1
    assert L.sa_index_create(fake, 100, 32, 32, 0, fake, 16, 5, C.byref(out)) == 0
    ix = out
    # not analysed: no integer range, so the search accumulates in double
    lo, hi = C.c_int32(0), C.c_int32(0)
    assert L.sa_index_integer_range(ix, C.byref(lo), C.byref(hi)) == 0
    assert L.sa_index_integer_range(None, None, None) == 0
    assert L.sa_index_analyze(None, None) == -1 and "NULL" in _err(B)
    p = B.SearchParams()
    L.sa_default_params(C.byref(p))
    # k > L, M > 16, L > 1024
    for (k, Lq, M) in ((11, 10, 1), (10, 10, 17), (10, 2000, 1), (0, 10, 1)):
        assert L.sa_search(ix, fake, 4, 32, k, Lq, M, C.byref(p), fake, fake, None, fake, 1 << 30, None) == -1
    # a workspace that is too small is reported before any launch
    assert L.sa_search_workspace_bytes(ix, 1000, 10, 64, 4, C.byref(p)) > 0
    p.rho = float("nan")
    assert L.sa_search(ix, fake, 4, 32, 10, 64, 4, C.byref(p), fake, fake, None, fake, 1 << 30, None) == -1
    assert "rho" in _err(B)
    # batches: every query is checked before anything is allocated; no re-rank
    import numpy as np
    bL = np.array([64, 10, 64], np.int32)
    bk = np.array([10, 20, 10], np.int32)
    bM = np.array([1, 1, 4], np.int32)
    bh = C.c_void_p(0)
    L.sa_default_params(C.byref(p))
    assert L.sa_batch_create(ix, 3, bL.ctypes.data, bk.ctypes.data, bM.ctypes.data, C.byref(p), C.byref(bh)) == -1
    assert "query 1" in _err(B) and not bh.value
    p.rerank = -1
    bk[1] = 5
    qx = C.c_void_p(0)   # bf16 codes with no float32 vectors: nothing to re-rank with
    assert L.sa_index_create_q(fake, 1, None, 32, None, 32, 100, 32, 0, fake, 16, 5, C.byref(qx)) == 0
    assert L.sa_batch_create(qx, 3, bL.ctypes.data, bk.ctypes.data, bM.ctypes.data, C.byref(p), C.byref(bh)) != 0
    assert "float32 vectors" in _err(B)
    L.sa_index_destroy(qx)
    p.rerank = 0
    assert L.sa_batch_create(ix, 3, None, bk.ctypes.data, bM.ctypes.data, C.byref(p), C.byref(bh)) == -1
    assert L.sa_batch_workspace_bytes(None) == 0
    # serving: defaults and configuration checks before any device call
    cfg = B.ServerConfig()
    L.sa_server_default_config(C.byref(cfg))
    assert (cfg.slots, cfg.max_batch, cfg.k_max) == (8, 1024, 100) and cfg.workspace_bytes == 1 << 30
    sh = C.c_void_p(0)
    cfg.slots = 17
    assert L.sa_server_create(ix, None, C.byref(cfg), C.byref(sh)) == -1 and "slots" in _err(B)
    cfg.slots, cfg.k_max = 2, 0
    assert L.sa_server_create(ix, None, C.byref(cfg), C.byref(sh)) == -1 and "k_max" in _err(B)
    assert L.sa_server_submit(None, fake, 10, 64, 1, 0) == -1
    assert L.sa_batch_describe(None, None, 0) < 0
    L.sa_index_destroy(ix)
    # exact kNN argument checks
    assert L.sa_knn(fake, 10, 32, 32, fake, 3, 32, 0, 0, 0, fake, fake, None) == -1
    assert L.sa_knn(fake, 10, 32, 32, fake, 3, 32, 300, 0, 0, fake, fake, None) == -1
    assert L.sa_knn(fake + 4, 10, 32, 32, fake, 3, 32, 5, 0, 0, fake, fake, None) == -1
    assert "aligned" in _err(B)
    used = C.c_int32(7)
    assert L.sa_knn_ex(fake, 10, 32, 32, fake, 3, 32, 5, 0, 0, fake, fake, 3, C.byref(used), None) == -1
    assert "path" in _err(B) and used.value == 0
    # reduced precision: bad dtype, fp8 without scales, re-rank without float32 vectors
    assert L.sa_quantize(fake, 10, 32, 32, 0, fake, 32, fake, None) == -1
    assert "dtype" in _err(B)
    h = C.c_void_p(0)
    assert L.sa_index_create_q(fake, 2, None, 32, None, 32, 10, 32, 0, fake, 16, 0, C.byref(h)) == -1
    assert "scale" in _err(B)
    assert L.sa_index_create_q(fake, 1, None, 32, None, 32, 10, 32, 0, fake, 16, 0, C.byref(h)) == 0
    pr = B.SearchParams()
    L.sa_default_params(C.byref(pr))
    assert pr.rerank == 0
    pr.rerank = -1
    assert L.sa_search(h, fake, 4, 32, 10, 64, 1, C.byref(pr), fake, fake, None, fake, 1 << 30, None) == -1
    assert "float32 vectors" in _err(B)
    L.sa_index_destroy(h)
    assert L.sa_prune(fake, 10, 32, 32, 0, fake, 65, 16, 1, fake, None) == -1
    e = C.c_int32(0)
    assert L.sa_build_graph(fake, 1, 32, 32, 0, 16, 16, 0, 0, 1, 4, 4, fake, C.byref(e), None, None, None) == -1
    assert L.sa_build_graph(fake, 100, 32, 32, 0, 16, 16, 1, 1, 1, 4, 17, fake, C.byref(e), None, None, None) == -1
    assert "hub_keep_local" in _err(B)
