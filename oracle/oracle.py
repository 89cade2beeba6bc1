"""ctypes front end of the C oracle (see oracle.c for the passages each function follows).

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

L2, IP = 0, 1
SYNC_BSP, SYNC_STATIC, SYNC_ADAPTIVE = 0, 1, 2
ALGO_BFIS, ALGO_TOPM, ALGO_SPEEDANN = 0, 1, 2


STATS_DTYPE = np.dtype([("global_steps", "<i8"), ("substeps", "<i8"), ("expansions", "<i8"),
                        ("dist_comps", "<i8"), ("merges", "<i8"), ("flags", "<i8")])
# or_trace: the smallest relative gap between neighbouring keys a decision depended on,
# where it was seen, and how many expansions / added entries were recorded
TRACE_DTYPE = np.dtype([("min_gap", "<f8"), ("gap_step", "<i8"), ("gap_dist", "<f4", (2,)),
                        ("gap_id", "<i4", (2,)), ("n_exp", "<i8"), ("n_keys", "<i8")])


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP over independent queries)."""
    with _lock:
        if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
            return _LIB_PATH
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
               "-Wno-unused-parameter", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
        return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB_PATH)
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        st = np.ctypeslib.ndpointer(STATS_DTYPE, flags="C_CONTIGUOUS")
        i64, i32, dbl = C.c_int64, C.c_int32, C.c_double
        L.or_distance.argtypes = [f32p, f32p, C.c_int, C.c_int]
        L.or_distance.restype = C.c_float
        L.or_knn.argtypes = [f32p, i64, C.c_int, i64, f32p, i64, i64, C.c_int, C.c_int, C.c_int, i32p, f32p]
        L.or_knn.restype = None
        L.or_knn_self.argtypes = [f32p, i64, C.c_int, i64, f32p, i64, i64, C.c_int, C.c_int, i32p, i32p, f32p]
        L.or_knn_self.restype = None
        L.or_search_batch.argtypes = [C.c_int, f32p, i64, C.c_int, i64, C.c_int, i32p, C.c_int, i32, f32p, i64,
                                      i64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, dbl, C.c_int, C.c_int,
                                      i32p, f32p, st]
        L.or_search_batch.restype = C.c_int
        tr = np.ctypeslib.ndpointer(TRACE_DTYPE, flags="C_CONTIGUOUS")
        L.or_search_batch_traced.argtypes = L.or_search_batch.argtypes + [tr, i32p, f32p, i32p, i64, i64]
        L.or_search_batch_traced.restype = C.c_int
        L.or_medoid.argtypes = [f32p, i64, C.c_int, i64]
        L.or_medoid.restype = i64
        L.or_prune.argtypes = [f32p, i64, C.c_int, i64, C.c_int, i32p, C.c_int, C.c_int, C.c_int, i32p]
        L.or_prune.restype = None
        L.or_repair.argtypes = [f32p, i64, C.c_int, i64, C.c_int, i32p, C.c_int, i32, C.c_int, C.c_int, C.c_int,
                                C.POINTER(C.c_int64)]
        L.or_repair.restype = i64
        L.or_reverse_edges.argtypes = [f32p, i64, C.c_int, i64, C.c_int, i32p, C.c_int]
        L.or_reverse_edges.restype = i64
        L.or_reachable.argtypes = [i32p, C.c_int, i64, i32, u8p]
        vp = C.c_void_p
        L.or_quantize.argtypes = [f32p, i64, C.c_int, i64, C.c_int, vp, f32p]
        L.or_quantize.restype = None
        L.or_dequantize.argtypes = [vp, f32p, i64, C.c_int, C.c_int, f32p]
        L.or_dequantize.restype = None
        L.or_rerank.argtypes = [f32p, C.c_int, i64, C.c_int, f32p, i64, i64, i32p, C.c_int, C.c_int, i32p, f32p]
        L.or_rerank.restype = None
        L.or_reachable.restype = i64
        _lib = L
    return _lib


def _metric(m) -> int:
    if isinstance(m, str):
        return {"l2": L2, "ip": IP}[m]
    return int(m)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def distance(a, b, metric="l2") -> float:
    a, b = _f32(a).ravel(), _f32(b).ravel()
    return float(lib().or_distance(a, b, a.shape[0], _metric(metric)))


def knn(base, queries, k, metric="l2", exclude_self=False):
    """Exact top-k by key (distance, id) over all base vectors (linear scan)."""
    base, queries = _f32(base), _f32(queries)
    n, d = base.shape
    nq = queries.shape[0]
    ids = np.empty((nq, k), np.int32)
    dists = np.empty((nq, k), np.float32)
    lib().or_knn(base, n, d, d, queries, nq, d, k, _metric(metric), int(exclude_self), ids, dists)
    return ids, dists


def knn_self(base, rows, k, metric="l2"):
    """Exact top-k of the listed base rows, each excluding itself."""
    base = _f32(base)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    n, d = base.shape
    q = np.ascontiguousarray(base[rows])
    ids = np.empty((rows.shape[0], k), np.int32)
    dists = np.empty((rows.shape[0], k), np.float32)
    lib().or_knn_self(base, n, d, d, q, rows.shape[0], d, k, _metric(metric), rows, ids, dists)
    return ids, dists


def search(algo, base, adj, entry, queries, k, L, M=1, metric="l2", sync="adaptive", static_I=0,
           rho=0.8, staged=True, max_substeps=0, trace=None):
    """Run one of the search algorithms for every query.  algo: "bfis" (Algorithm 1),
    "topm" (Top-M, M fixed or staged) or "speedann" (Algorithm 3, lockstep).
    trace=(cap_exp, cap_keys): also return a Trace of every query (see oracle.c)."""
    base, queries = _f32(base), _f32(queries)
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    n, d = base.shape
    R = adj.shape[1]
    nq = queries.shape[0]
    a = {"bfis": ALGO_BFIS, "topm": ALGO_TOPM, "speedann": ALGO_SPEEDANN}[algo]
    s = {"bsp": SYNC_BSP, "static": SYNC_STATIC, "adaptive": SYNC_ADAPTIVE}[sync] if isinstance(sync, str) else int(sync)
    ids = np.empty((nq, k), np.int32)
    dists = np.empty((nq, k), np.float32)
    stats = np.zeros(nq, STATS_DTYPE)
    args = (a, base, n, d, d, _metric(metric), adj, R, int(entry), queries, nq, d, int(k), int(L), int(M), s,
            int(static_I), float(rho), int(bool(staged)), int(max_substeps), ids, dists, stats)
    if trace is None:
        rc = lib().or_search_batch(*args)
    else:
        ce, ck = (int(x) for x in trace)
        tr = Trace(np.zeros(nq, TRACE_DTYPE), np.zeros((nq, max(ce, 1), 4), np.int32),
                   np.zeros((nq, max(ck, 1)), np.float32), np.zeros((nq, max(ck, 1)), np.int32))
        rc = lib().or_search_batch_traced(*args, tr.summary, tr.expansions, tr.key_dist, tr.key_id, ce, ck)
    if rc & 2:
        raise MemoryError("oracle search: allocation failed")
    return (ids, dists, stats) if trace is None else (ids, dists, stats, tr)


class Trace:
    """Per-query record of an oracle search: summary (TRACE_DTYPE: the smallest relative gap
    between neighbouring keys of distinct vertices in any sorted list, within the places
    that decide what is kept, the local step and keys where it was seen, and the counts),
    expansions[q, i] = (local step, worker, vertex, entries added) and the added entries'
    keys in order, each up to the capacity asked for."""

    def __init__(self, summary, expansions, key_dist, key_id):
        self.summary, self.expansions, self.key_dist, self.key_id = summary, expansions, key_dist, key_id


def bfis(base, adj, entry, queries, k, L, metric="l2"):
    return search("bfis", base, adj, entry, queries, k, L, 1, metric)


def topm(base, adj, entry, queries, k, L, M, staged=False, metric="l2"):
    return search("topm", base, adj, entry, queries, k, L, M, metric, staged=staged)


def speedann(base, adj, entry, queries, k, L, T, sync="adaptive", static_I=0, rho=0.8, staged=True,
             metric="l2", max_substeps=0):
    return search("speedann", base, adj, entry, queries, k, L, T, metric, sync, static_I, rho, staged,
                  max_substeps)


def medoid(base) -> int:
    base = _f32(base)
    n, d = base.shape
    return int(lib().or_medoid(base, n, d, d))


def prune(base, cand, R, mode="rng", metric="l2"):
    base = _f32(base)
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    n, d = base.shape
    adj = np.empty((n, R), np.int32)
    lib().or_prune(base, n, d, d, _metric(metric), cand, cand.shape[1], int(R), {"knn": 0, "rng": 1}[mode], adj)
    return adj


def default_hubs(n: int) -> int:
    return max(1, n // 256)


def repair(base, adj, entry, keep_local=1, metric="l2", hubs=None, hub_keep_local=4):
    """Connectivity repair in place; returns (bridges added, component count)."""
    base = _f32(base)
    assert adj.dtype == np.int32 and adj.flags.c_contiguous
    n, d = base.shape
    if hubs is None:
        hubs = default_hubs(n)
    nc = C.c_int64(0)
    added = lib().or_repair(base, n, d, d, _metric(metric), adj, adj.shape[1], int(entry), int(keep_local),
                            int(hubs), int(hub_keep_local), C.byref(nc))
    if added < 0:
        raise RuntimeError("repair: no reachable vertex has a free slot")
    return int(added), int(nc.value)


def reverse_edges(base, adj, metric="l2"):
    """Adds reverse edges in place (see oracle.c); returns the number added."""
    base = _f32(base)
    assert adj.dtype == np.int32 and adj.flags.c_contiguous
    n, d = base.shape
    return int(lib().or_reverse_edges(base, n, d, d, _metric(metric), adj, adj.shape[1]))


def reachable(adj, entry):
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    n = adj.shape[0]
    mark = np.zeros(n, np.uint8)
    cnt = lib().or_reachable(adj, adj.shape[1], n, int(entry), mark)
    return int(cnt), mark.astype(bool)


def build_graph(base, knn_k, R, prune_mode="rng", do_repair=True, keep_local=1, metric="l2", reverse=None,
                hubs=None, hub_keep_local=4):
    """Exact knn_k-NN candidates, row pruning to R, medoid entry; with do_repair, reverse
    edges (unless reverse=False) and the connectivity repair.  Returns (adj, entry, info)."""
    base = _f32(base)
    entry = medoid(base)
    cand, _ = knn(base, base, knn_k, metric, exclude_self=True)
    adj = prune(base, cand, R, prune_mode, metric)
    info = {"bridges": 0, "components": None, "reverse": 0}
    if reverse is None:
        reverse = do_repair
    if reverse:
        info["reverse"] = reverse_edges(base, adj, metric)
    if do_repair:
        info["bridges"], info["components"] = repair(base, adj, entry, keep_local, metric, hubs, hub_keep_local)
    return adj, entry, info


def recall(found_ids, true_ids, k=None) -> np.ndarray:
    """Per-query Recall = |R' & R| / K (Sec. 2.1); padding ids (-1) never count."""
    found_ids = np.asarray(found_ids)
    true_ids = np.asarray(true_ids)
    if k is None:
        k = true_ids.shape[1]
    out = np.empty(found_ids.shape[0])
    for i in range(found_ids.shape[0]):
        t = set(int(x) for x in true_ids[i, :k] if x >= 0)
        f = set(int(x) for x in found_ids[i, :k] if x >= 0)
        out[i] = len(t & f) / float(k)
    return out


DTYPES = {"f32": 0, "bf16": 1, "fp8": 2}


def quantize(x, dtype):
    """Codes (uint16 for bf16, uint8 for fp8 e4m3) and per-vector scales of the rows of x."""
    x = _f32(x)
    n, d = x.shape
    codes = np.empty((n, d), np.uint16 if dtype == "bf16" else np.uint8)
    scale = np.empty(n, np.float32)
    lib().or_quantize(x, n, d, d, DTYPES[dtype], codes.ctypes.data, scale)
    return codes, scale


def dequantize(codes, scale, dtype):
    """The float32 vectors the codes stand for (scale * value, one float rounding)."""
    codes = np.ascontiguousarray(codes)
    scale = np.ascontiguousarray(scale, dtype=np.float32)
    n, d = codes.shape
    out = np.empty((n, d), np.float32)
    lib().or_dequantize(codes.ctypes.data, scale, n, d, DTYPES[dtype], out)
    return out


def rerank(base, queries, cand, k, metric="l2"):
    """Exact re-rank of each query's candidate ids (-1 padded) on float32 base: first k by key."""
    base, queries = _f32(base), _f32(queries)
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    nq, L = cand.shape
    ids = np.empty((nq, k), np.int32)
    dists = np.empty((nq, k), np.float32)
    lib().or_rerank(base, base.shape[1], base.shape[1], _metric(metric), queries, nq, queries.shape[1], cand, L, k,
                    ids, dists)
    return ids, dists


def graph_order(adj, entry, mode="bfs"):
    """Vertex renumbering (the GPU counterpart of the neighbour grouping of Sec. 4.4):
    perm[i] = original id of new vertex i.  "degree": in-degree descending, equal
    in-degrees by id.  "bfs": breadth-first from entry, neighbours in row order, every
    vertex taken when first seen; unreachable vertices after, by id.  Plain Python."""
    adj = np.asarray(adj)
    n = adj.shape[0]
    if mode == "degree":
        indeg = np.zeros(n, np.int64)
        for row in adj:
            for u in row:
                if 0 <= u < n:
                    indeg[u] += 1
        return np.array(sorted(range(n), key=lambda v: (-indeg[v], v)), np.int32)
    seen = [False] * n
    order = [int(entry)]
    seen[entry] = True
    head = 0
    while head < len(order):
        for u in adj[order[head]]:
            u = int(u)
            if 0 <= u < n and not seen[u]:
                seen[u] = True
                order.append(u)
        head += 1
    order += [v for v in range(n) if not seen[v]]
    return np.array(order, np.int32)


def permute(base, adj, entry, perm):
    """The index in the new numbering: rows base[perm[i]], adjacency rows adj[perm[i]]
    with every id u replaced by its new id, and the new entry."""
    perm = np.asarray(perm, np.int64)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    a = np.asarray(adj)[perm]
    a2 = np.where(a >= 0, inv[np.maximum(a, 0)], -1).astype(np.int32)
    return np.ascontiguousarray(np.asarray(base)[perm]), a2, int(inv[entry])
