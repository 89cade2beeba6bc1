"""Python binding of libspeedann (include/speedann.h): argument marshalling only.

Device memory and streams come from PyTorch (ROCm); every step of the search, the
exact kNN and the graph construction runs in the library.  There is no CPU fallback:
if the built library or a gfx950 device is missing, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspeedann.so")

SA_L2, SA_IP = 0, 1
SYNC = {"bsp": 0, "static": 1, "adaptive": 2}
QFLAG_MAX_STEPS, QFLAG_CAPACITY, QFLAG_SPILLED = 1, 2, 4

EXPORTS = ["sa_last_error", "sa_default_params", "sa_knn", "sa_knn_ex", "sa_quantize", "sa_index_create_q", "sa_medoid", "sa_prune", "sa_reverse_edges",
           "sa_repair", "sa_build_graph", "sa_index_create", "sa_index_destroy", "sa_search_workspace_bytes", "sa_search",
           "sa_batch_create", "sa_batch_destroy", "sa_batch_workspace_bytes", "sa_batch_upload", "sa_batch_run",
           "sa_batch_tune", "sa_batch_set_config", "sa_batch_classes", "sa_batch_class_options", "sa_batch_set_class",
           "sa_batch_describe", "sa_server_default_config",
           "sa_server_create", "sa_server_destroy", "sa_server_submit", "sa_server_poll", "sa_server_replay",
           "sa_server_stats", "sa_graph_order", "sa_permute_rows", "sa_permute_graph", "sa_index_set_id_map",
           "sa_gather_probe", "sa_knn_last_rescanned", "sa_index_analyze", "sa_index_integer_range",
           "sa_search_noalloc"]


class SearchParams(C.Structure):
    _fields_ = [("sync", C.c_int32), ("static_I", C.c_int32), ("rho", C.c_double), ("staged", C.c_int32),
                ("max_substeps", C.c_int32), ("lds_hash_slots", C.c_int32), ("ws_hash_slots", C.c_int32),
                ("rerank", C.c_int32), ("ws_hash_init", C.c_int32)]


class ServerConfig(C.Structure):
    _fields_ = [("slots", C.c_int32), ("max_batch", C.c_int32), ("max_pending", C.c_int32), ("k_max", C.c_int32),
                ("workspace_bytes", C.c_size_t)]


# sa_query_stats as a numpy/torch view: 6 int32 + 2 uint64 = 40 bytes
STATS_FIELDS = ["global_steps", "substeps", "expansions", "dist_comps", "merges", "flags"]
STATS_BYTES = 40


class SpeedAnnError(RuntimeError):
    pass


_lib = None


def lib():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SpeedAnnError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
        L.sa_last_error.restype = C.c_char_p
        L.sa_default_params.argtypes = [C.POINTER(SearchParams)]
        L.sa_knn.argtypes = [vp, i64, i32, i64, vp, i64, i64, i32, i32, i32, vp, vp, vp]
        L.sa_knn_ex.argtypes = [vp, i64, i32, i64, vp, i64, i64, i32, i32, i32, vp, vp, i32, C.POINTER(C.c_int32), vp]
        L.sa_knn_last_rescanned.argtypes = []
        L.sa_knn_last_rescanned.restype = i64
        L.sa_index_analyze.argtypes = [vp, vp]
        L.sa_index_integer_range.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.sa_index_integer_range.restype = i32
        L.sa_medoid.argtypes = [vp, i64, i32, i64, C.POINTER(C.c_int32), vp]
        L.sa_prune.argtypes = [vp, i64, i32, i64, i32, vp, i32, i32, i32, vp, vp]
        L.sa_reverse_edges.argtypes = [vp, i64, i32, i64, i32, vp, i32, C.POINTER(C.c_int64), vp]
        L.sa_repair.argtypes = [vp, i64, i32, i64, i32, vp, i32, i32, i32, i32, i32, C.POINTER(C.c_int64),
                                C.POINTER(C.c_int64), vp]
        L.sa_build_graph.argtypes = [vp, i64, i32, i64, i32, i32, i32, i32, i32, i32, i32, i32, vp,
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int64), vp]
        L.sa_index_create.argtypes = [vp, i64, i32, i64, i32, vp, i32, i32, C.POINTER(vp)]
        L.sa_index_create_q.argtypes = [vp, i32, vp, i64, vp, i64, i64, i32, i32, vp, i32, i32, C.POINTER(vp)]
        L.sa_quantize.argtypes = [vp, i64, i32, i64, i32, vp, i64, vp, vp]
        L.sa_index_destroy.argtypes = [vp]
        L.sa_index_destroy.restype = None
        L.sa_search_workspace_bytes.argtypes = [vp, i64, i32, i32, i32, C.POINTER(SearchParams)]
        L.sa_search_workspace_bytes.restype = sz
        L.sa_search.argtypes = [vp, vp, i64, i64, i32, i32, i32, C.POINTER(SearchParams), vp, vp, vp, vp, sz, vp]
        L.sa_search_noalloc.argtypes = [vp, vp, i64, i64, i32, i32, i32, C.POINTER(SearchParams), vp, vp, vp, vp]
        L.sa_batch_create.argtypes = [vp, i64, vp, vp, vp, C.POINTER(SearchParams), C.POINTER(vp)]
        L.sa_batch_destroy.argtypes = [vp]
        L.sa_batch_destroy.restype = None
        L.sa_batch_workspace_bytes.argtypes = [vp]
        L.sa_batch_workspace_bytes.restype = sz
        L.sa_batch_upload.argtypes = [vp, vp, sz, vp]
        L.sa_batch_run.argtypes = [vp, vp, i64, vp, vp, i64, vp, vp, sz, vp]
        L.sa_batch_tune.argtypes = [vp, vp, i64, vp, vp, i64, vp, sz, i32, vp]
        L.sa_batch_set_config.argtypes = [vp, i32, i32]
        L.sa_batch_classes.argtypes = [vp]
        L.sa_batch_classes.restype = i32
        L.sa_batch_class_options.argtypes = [vp, i32, vp, i32, C.POINTER(i32), C.POINTER(i32)]
        L.sa_batch_set_class.argtypes = [vp, i32, i32, i32]
        L.sa_batch_describe.argtypes = [vp, C.c_char_p, sz]
        L.sa_batch_describe.restype = i64
        L.sa_server_default_config.argtypes = [C.POINTER(ServerConfig)]
        L.sa_server_default_config.restype = None
        L.sa_server_create.argtypes = [vp, C.POINTER(SearchParams), C.POINTER(ServerConfig), C.POINTER(vp)]
        L.sa_server_destroy.argtypes = [vp]
        L.sa_server_destroy.restype = None
        L.sa_server_submit.argtypes = [vp, vp, i32, i32, i32, C.c_uint64]
        L.sa_server_poll.argtypes = [vp, i32, vp, vp, vp, i64, vp, vp, i32]
        L.sa_server_poll.restype = i32
        L.sa_server_replay.argtypes = [vp, vp, i64, i64, vp, vp, vp, vp, vp, vp, i64, vp, C.POINTER(C.c_int64)]
        L.sa_server_stats.argtypes = [vp] + [C.POINTER(C.c_int64)] * 5
        L.sa_graph_order.argtypes = [vp, i64, i32, i32, i32, vp, vp]
        L.sa_permute_rows.argtypes = [vp, i64, i64, vp, vp, vp]
        L.sa_permute_graph.argtypes = [vp, i64, i32, vp, vp, vp, vp]
        L.sa_index_set_id_map.argtypes = [vp, vp]
        L.sa_gather_probe.argtypes = [vp, i64, i32, i64, i64, i32, C.c_uint32, vp, vp]
        for name in ("sa_knn", "sa_knn_ex", "sa_quantize", "sa_index_create_q", "sa_medoid", "sa_prune", "sa_reverse_edges", "sa_repair", "sa_build_graph", "sa_index_create",
                     "sa_search", "sa_search_noalloc", "sa_batch_create", "sa_batch_upload", "sa_batch_run", "sa_batch_tune",
                     "sa_batch_set_config", "sa_batch_class_options", "sa_batch_set_class", "sa_server_create",
                     "sa_server_submit", "sa_server_replay",
                     "sa_server_stats", "sa_graph_order", "sa_permute_rows", "sa_permute_graph",
                     "sa_index_set_id_map", "sa_gather_probe"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise SpeedAnnError(f"{what} failed ({rc}): {lib().sa_last_error().decode()}")


def _metric(m) -> int:
    return {"l2": SA_L2, "ip": SA_IP}[m] if isinstance(m, str) else int(m)


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _mat(x: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise SpeedAnnError(f"{name} must be a device tensor")
    if x.dtype != torch.float32 or x.dim() != 2:
        raise SpeedAnnError(f"{name} must be a 2-d float32 tensor")
    if x.stride(1) != 1:
        x = x.contiguous()
    return x


def pad_dim(x: torch.Tensor) -> torch.Tensor:
    """Pads rows with zero columns to a multiple of 4 (zero columns change no distance)."""
    d = x.shape[1]
    if d % 4 == 0 and x.stride(0) % 4 == 0 and x.data_ptr() % 16 == 0:
        return x
    d4 = (d + 3) // 4 * 4
    out = torch.zeros((x.shape[0], d4), dtype=x.dtype, device=x.device)
    out[:, :d] = x
    return out


KNN_PATHS = {"auto": 0, "scan": 1, "mfma": 2}


def knn(base: torch.Tensor, queries: torch.Tensor, k: int, metric="l2", exclude_self=False, stream=None,
        path="auto", return_path=False):
    """Exact top-k by (distance, id) over all rows of base (linear scan on the GPU).

    path: "scan" (double precision, any data), "mfma" (bf16 matrix cores: integer-valued
    data, or finite floats with d <= 1024 and k <= 96; exact either way), "auto" (mfma
    where it applies).  With return_path the path that ran is returned as a third value."""
    base = pad_dim(_mat(base, "base"))
    queries = base if (exclude_self and queries is None) else pad_dim(_mat(queries, "queries"))
    nq = queries.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int32, device=base.device)
    dists = torch.empty((nq, k), dtype=torch.float32, device=base.device)
    used = C.c_int32(0)
    _check(lib().sa_knn_ex(base.data_ptr(), base.shape[0], base.shape[1], base.stride(0), queries.data_ptr(), nq,
                           queries.stride(0), k, _metric(metric), int(exclude_self), ids.data_ptr(),
                           dists.data_ptr(), KNN_PATHS[path], C.byref(used), _stream(stream)), "sa_knn_ex")
    if return_path:
        names = {v: n for n, v in KNN_PATHS.items()}
        return ids, dists, names[int(used.value)]
    return ids, dists


def knn_last_rescanned() -> int:
    """Queries of the last knn call on this thread that the float MFMA form handed to the scan."""
    return int(lib().sa_knn_last_rescanned())


def medoid(base: torch.Tensor, stream=None) -> int:
    base = pad_dim(_mat(base, "base"))
    out = C.c_int32(0)
    _check(lib().sa_medoid(base.data_ptr(), base.shape[0], base.shape[1], base.stride(0), C.byref(out),
                           _stream(stream)), "sa_medoid")
    return int(out.value)


def prune(base: torch.Tensor, cand: torch.Tensor, R: int, mode="rng", metric="l2", stream=None) -> torch.Tensor:
    base = pad_dim(_mat(base, "base"))
    cand = cand.to(torch.int32).contiguous()
    adj = torch.empty((base.shape[0], R), dtype=torch.int32, device=base.device)
    _check(lib().sa_prune(base.data_ptr(), base.shape[0], base.shape[1], base.stride(0), _metric(metric),
                          cand.data_ptr(), cand.shape[1], R, {"knn": 0, "rng": 1}[mode], adj.data_ptr(),
                          _stream(stream)), "sa_prune")
    return adj


def reverse_edges(base: torch.Tensor, adj: torch.Tensor, metric="l2", stream=None) -> int:
    """Reverse-edge insertion in place; returns the number of edges added."""
    base = pad_dim(_mat(base, "base"))
    assert adj.dtype == torch.int32 and adj.is_contiguous()
    a = C.c_int64(0)
    _check(lib().sa_reverse_edges(base.data_ptr(), base.shape[0], base.shape[1], base.stride(0), _metric(metric),
                                  adj.data_ptr(), adj.shape[1], C.byref(a), _stream(stream)), "sa_reverse_edges")
    return int(a.value)


def default_hubs(n: int) -> int:
    """Hub count of the repair: one per 256 vertices."""
    return max(1, n // 256)


def repair(base: torch.Tensor, adj: torch.Tensor, entry: int, keep_local=1, metric="l2", hubs=None,
           hub_keep_local=4, stream=None):
    """Connectivity repair of adj in place; returns (bridges, components)."""
    base = pad_dim(_mat(base, "base"))
    assert adj.dtype == torch.int32 and adj.is_contiguous()
    if hubs is None:
        hubs = default_hubs(base.shape[0])
    b, c = C.c_int64(0), C.c_int64(0)
    _check(lib().sa_repair(base.data_ptr(), base.shape[0], base.shape[1], base.stride(0), _metric(metric),
                           adj.data_ptr(), adj.shape[1], int(entry), int(keep_local), int(hubs), int(hub_keep_local),
                           C.byref(b), C.byref(c), _stream(stream)), "sa_repair")
    return int(b.value), int(c.value)


def build_graph(base: torch.Tensor, knn_k: int, R: int, prune_mode="rng", do_repair=True, keep_local=1,
                metric="l2", hubs=None, hub_keep_local=4, stream=None):
    """Returns (adj, entry, info) built on the GPU."""
    base = pad_dim(_mat(base, "base"))
    n = base.shape[0]
    if hubs is None:
        hubs = default_hubs(n)
    adj = torch.empty((n, R), dtype=torch.int32, device=base.device)
    entry, b, c = C.c_int32(0), C.c_int64(0), C.c_int64(0)
    _check(lib().sa_build_graph(base.data_ptr(), n, base.shape[1], base.stride(0), _metric(metric), knn_k, R,
                                {"knn": 0, "rng": 1}[prune_mode], int(bool(do_repair)), int(keep_local),
                                int(hubs), int(hub_keep_local), adj.data_ptr(), C.byref(entry), C.byref(b), C.byref(c), _stream(stream)),
           "sa_build_graph")
    return adj, int(entry.value), {"bridges": int(b.value), "components": int(c.value)}


def make_params(sync="adaptive", static_I=0, rho=0.8, staged=True, max_substeps=0, lds_hash_slots=0,
                ws_hash_slots=0, rerank=0, ws_hash_init=0) -> SearchParams:
    p = SearchParams()
    lib().sa_default_params(C.byref(p))
    p.sync = SYNC[sync] if isinstance(sync, str) else int(sync)
    p.static_I = int(static_I)
    p.rho = float(rho)
    p.staged = int(bool(staged))
    p.max_substeps = int(max_substeps)
    p.lds_hash_slots = int(lds_hash_slots)
    p.ws_hash_slots = int(ws_hash_slots)
    p.rerank = int(rerank)
    p.ws_hash_init = int(ws_hash_init)
    return p


DTYPES = {"f32": 0, "bf16": 1, "fp8": 2}


def quantize(x: torch.Tensor, dtype: str, stream=None):
    """Reduced-precision copy of the rows of x: (codes, scales).  Codes are int16 (bf16
    patterns) or uint8 (fp8 e4m3), rows padded to a multiple of 4 with code 0."""
    x = pad_dim(_mat(x, "vectors"))
    n, d = x.shape
    codes = torch.empty((n, d), dtype=torch.int16 if dtype == "bf16" else torch.uint8, device=x.device)
    scale = torch.empty(n, dtype=torch.float32, device=x.device)
    _check(lib().sa_quantize(x.data_ptr(), n, d, x.stride(0), DTYPES[dtype], codes.data_ptr(), codes.stride(0),
                             scale.data_ptr(), _stream(stream)), "sa_quantize")
    return codes, scale


@dataclass
class SearchResult:
    ids: torch.Tensor
    dists: torch.Tensor
    stats: torch.Tensor | None   # (nq, 10) int32 view of sa_query_stats, or None

    def stat(self, name: str) -> torch.Tensor:
        return self.stats[:, STATS_FIELDS.index(name)]

    def times(self) -> torch.Tensor:
        """(t_start, t_end) device real-time counter values per query (100 MHz)."""
        return self.stats.view(torch.int64)[:, 3:5]


class Index:
    """A graph index over device arrays (borrowed: keep vec and adj alive)."""

    def __init__(self, vec: torch.Tensor, adj: torch.Tensor, entry: int, metric="l2", dtype="f32", codes=None,
                 scale=None, id_map: torch.Tensor | None = None, analyze=True):
        """vec: float32 vectors.  dtype "bf16" / "fp8": the search reads codes and scale (from
        quantize(vec, dtype), made here when not given) and vec serves the re-rank.
        id_map: for a renumbered index (reorder), new id -> original id of the results.
        analyze (float32 storage): scan the vectors once so that integer-valued data can be
        searched with float32 accumulation (sa_index_analyze; results unchanged)."""
        vec = pad_dim(_mat(vec, "vectors"))
        if adj.dtype != torch.int32 or not adj.is_cuda or not adj.is_contiguous():
            raise SpeedAnnError("adj must be a contiguous int32 device tensor")
        self.vec, self.adj, self.entry, self.metric, self.dtype = vec, adj, int(entry), metric, dtype
        h = C.c_void_p(0)
        if dtype == "f32":
            _check(lib().sa_index_create(vec.data_ptr(), vec.shape[0], vec.shape[1], vec.stride(0), _metric(metric),
                                         adj.data_ptr(), adj.shape[1], self.entry, C.byref(h)), "sa_index_create")
        else:
            if codes is None:
                codes, scale = quantize(vec, dtype)
            self.codes, self.scale = codes, scale
            _check(lib().sa_index_create_q(codes.data_ptr(), DTYPES[dtype], scale.data_ptr(), codes.stride(0),
                                           vec.data_ptr(), vec.stride(0), vec.shape[0], vec.shape[1],
                                           _metric(metric), adj.data_ptr(), adj.shape[1], self.entry, C.byref(h)),
                   "sa_index_create_q")
        self._h = h
        self._ws = {}   # stream handle -> workspace
        self._lib = lib()   # kept for __del__, which may run after module teardown
        if dtype == "f32" and analyze:
            _check(lib().sa_index_analyze(h, _stream(None)), "sa_index_analyze")
        self.id_map = id_map
        if id_map is not None:
            if id_map.dtype != torch.int32 or not id_map.is_cuda or id_map.numel() != vec.shape[0]:
                raise SpeedAnnError("id_map must be an int32 device tensor of n entries")
            _check(lib().sa_index_set_id_map(h, id_map.data_ptr()), "sa_index_set_id_map")

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(self, "_lib", None)
        if h is not None and h.value and L is not None:
            L.sa_index_destroy(h)
            self._h = None

    @property
    def integer_range(self):
        """(lo, hi) when the analysed float32 vectors are integers searched with float32
        accumulation, else None."""
        lo, hi = C.c_int32(0), C.c_int32(0)
        return (lo.value, hi.value) if lib().sa_index_integer_range(self._h, C.byref(lo), C.byref(hi)) else None

    def workspace_bytes(self, nq, k, L, M, params: SearchParams) -> int:
        return int(lib().sa_search_workspace_bytes(self._h, nq, k, L, M, C.byref(params)))

    def workspace(self, nbytes: int, stream=None) -> torch.Tensor:
        """Zero-filled device workspace of the searches on `stream` (default: the current
        one); sa_search leaves it zero-filled.  One per stream, so that searches on
        different streams never share one, allocated and zeroed on its stream: a buffer
        replaced by a larger one goes back to torch's pool on the stream whose searches
        used it, which reuses it only after them."""
        s = stream if stream is not None else torch.cuda.current_stream()
        key = int(s.cuda_stream)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            with torch.cuda.stream(s):
                ws = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=self.vec.device)
            self._ws[key] = ws
        return ws

    def search(self, queries: torch.Tensor, k: int, L: int, M: int = 1, params: SearchParams | None = None,
               stats=False, stream=None, out=None, **kw) -> SearchResult:
        if params is None:
            params = make_params(**kw)
        queries = pad_dim(_mat(queries, "queries"))
        if queries.shape[1] != self.vec.shape[1]:
            raise SpeedAnnError("query dimension does not match the index")
        nq = queries.shape[0]
        dev = self.vec.device
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
            dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
            st = torch.empty((nq, STATS_BYTES // 4), dtype=torch.int32, device=dev) if stats else None
        else:
            ids, dists, st = out
        nbytes = self.workspace_bytes(nq, k, L, M, params)
        ws = self.workspace(nbytes, stream)
        _check(lib().sa_search(self._h, queries.data_ptr(), nq, queries.stride(0), k, L, M, C.byref(params),
                               ids.data_ptr(), dists.data_ptr(), st.data_ptr() if st is not None else None,
                               ws.data_ptr(), ws.numel(), _stream(stream)), "sa_search")
        return SearchResult(ids, dists, st)

    def search_noalloc(self, queries: torch.Tensor, k: int, L: int, M: int = 1, out=None,
                       params: SearchParams | None = None, stream=None, **kw) -> SearchResult:
        """sa_search_noalloc: the search with the library's static device workspace.  The
        library allocates nothing; with out=(ids, dists, stats or None) given, neither does
        this call (queries must then be contiguous with d a multiple of 4)."""
        if params is None:
            params = make_params(**kw)
        if out is None:
            queries = pad_dim(_mat(queries, "queries"))
            nq, dev = queries.shape[0], self.vec.device
            out = (torch.empty((nq, k), dtype=torch.int32, device=dev),
                   torch.empty((nq, k), dtype=torch.float32, device=dev), None)
        ids, dists, st = out
        nq = ids.shape[0]
        _check(lib().sa_search_noalloc(self._h, queries.data_ptr(), nq, queries.stride(0), k, L, M, C.byref(params),
                                       ids.data_ptr(), dists.data_ptr(), st.data_ptr() if st is not None else None,
                                       _stream(stream)), "sa_search_noalloc")
        return SearchResult(ids, dists, st)


class Batch:
    """A batch of queries with per-query (L, k, M) over an Index (sa_batch_*).

    run() enqueues only kernel launches and events on the current (or given) stream, so
    it can be captured in a torch.cuda.CUDAGraph and replayed."""

    def __init__(self, index: "Index", L, k, M, params: SearchParams | None = None, **kw):
        import numpy as np
        self.index = index
        Ls = np.ascontiguousarray(np.asarray(L, dtype=np.int32))
        ks = np.ascontiguousarray(np.asarray(k, dtype=np.int32))
        Ms = np.ascontiguousarray(np.asarray(M, dtype=np.int32))
        if not (Ls.shape == ks.shape == Ms.shape) or Ls.ndim != 1:
            raise SpeedAnnError("L, k and M must be 1-d arrays of one length")
        self.nq = int(Ls.shape[0])
        self.kmax = int(ks.max()) if self.nq else 1
        self.k = ks
        if params is None:
            params = make_params(**kw)
        self.params = params
        h = C.c_void_p()
        _check(lib().sa_batch_create(index._h, self.nq, Ls.ctypes.data, ks.ctypes.data, Ms.ctypes.data,
                                     C.byref(params), C.byref(h)), "sa_batch_create")
        self._h = h
        self._lib = lib()
        nbytes = int(lib().sa_batch_workspace_bytes(h))
        self.ws = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=index.vec.device)
        _check(lib().sa_batch_upload(h, self.ws.data_ptr(), self.ws.numel(), _stream(None)), "sa_batch_upload")

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(self, "_lib", None)
        if h is not None and h.value and L is not None:
            L.sa_batch_destroy(h)
            self._h = None

    def outputs(self, stats=False):
        dev = self.index.vec.device
        ids = torch.full((self.nq, self.kmax), -1, dtype=torch.int32, device=dev)
        dists = torch.full((self.nq, self.kmax), float("inf"), dtype=torch.float32, device=dev)
        st = torch.empty((self.nq, STATS_BYTES // 4), dtype=torch.int32, device=dev) if stats else None
        return ids, dists, st

    def run(self, queries: torch.Tensor, out=None, stats=False, stream=None) -> SearchResult:
        queries = pad_dim(_mat(queries, "queries"))
        if queries.shape[0] != self.nq:
            raise SpeedAnnError("the batch was planned for a different number of queries")
        ids, dists, st = out if out is not None else self.outputs(stats)
        _check(lib().sa_batch_run(self._h, queries.data_ptr(), queries.stride(0), ids.data_ptr(), dists.data_ptr(),
                                  ids.stride(0), st.data_ptr() if st is not None else None, self.ws.data_ptr(),
                                  self.ws.numel(), _stream(stream)), "sa_batch_run")
        return SearchResult(ids, dists, st)

    def tune(self, queries: torch.Tensor, reps: int = 3, stream=None) -> dict:
        queries = pad_dim(_mat(queries, "queries"))
        ids, dists, _ = self.outputs()
        _check(lib().sa_batch_tune(self._h, queries.data_ptr(), queries.stride(0), ids.data_ptr(), dists.data_ptr(),
                                   ids.stride(0), self.ws.data_ptr(), self.ws.numel(), int(reps), _stream(stream)),
               "sa_batch_tune")
        return self.describe()["tuning"]

    def set_config(self, streams: int, lds_hash_slots: int = 0):
        _check(lib().sa_batch_set_config(self._h, int(streams), int(lds_hash_slots)), "sa_batch_set_config")

    def classes(self) -> int:
        return int(lib().sa_batch_classes(self._h))

    def class_options(self, cls: int):
        """(lds_hash_slots settings class cls may take, whether it may run persistent)"""
        import numpy as np
        vals = np.zeros(8, np.int32)
        cnt, pers = C.c_int32(), C.c_int32()
        _check(lib().sa_batch_class_options(self._h, int(cls), vals.ctypes.data, 8, C.byref(cnt), C.byref(pers)),
               "sa_batch_class_options")
        return [int(v) for v in vals[:cnt.value]], bool(pers.value)

    def set_class(self, cls: int, lds_hash_slots: int, persistent: bool):
        _check(lib().sa_batch_set_class(self._h, int(cls), int(lds_hash_slots), int(bool(persistent))),
               "sa_batch_set_class")

    def describe(self) -> dict:
        import json
        n = int(lib().sa_batch_describe(self._h, None, 0))
        if n < 0:
            _check(n, "sa_batch_describe")
        buf = C.create_string_buffer(n)
        lib().sa_batch_describe(self._h, buf, n)
        return json.loads(buf.value.decode())


class Server:
    """The serving loop (sa_server_*) over a resident Index: submit / poll from host
    threads, or replay a timed arrival trace natively."""

    def __init__(self, index: "Index", params: SearchParams | None = None, slots=None, max_batch=None,
                 max_pending=None, k_max=None, workspace_bytes=None, **kw):
        cfg = ServerConfig()
        lib().sa_server_default_config(C.byref(cfg))
        for name, v in (("slots", slots), ("max_batch", max_batch), ("max_pending", max_pending),
                        ("k_max", k_max), ("workspace_bytes", workspace_bytes)):
            if v is not None:
                setattr(cfg, name, int(v))
        self.cfg = cfg
        self.index = index
        if params is None:
            params = make_params(**kw)
        h = C.c_void_p()
        _check(lib().sa_server_create(index._h, C.byref(params), C.byref(cfg), C.byref(h)), "sa_server_create")
        self._h = h
        self._lib = lib()
        self.d = index.vec.shape[1]

    def close(self):
        h = getattr(self, "_h", None)
        L = getattr(self, "_lib", None)
        if h is not None and h.value and L is not None:
            L.sa_server_destroy(h)
            self._h = None

    __del__ = close

    def _row(self, q):
        import numpy as np
        q = np.ascontiguousarray(q, dtype=np.float32).reshape(-1)
        if q.shape[0] < self.d:
            q = np.concatenate([q, np.zeros(self.d - q.shape[0], np.float32)])
        return q

    def submit(self, query, k: int, L: int, M: int, tag: int):
        q = self._row(query)
        _check(lib().sa_server_submit(self._h, q.ctypes.data, int(k), int(L), int(M), int(tag)), "sa_server_submit")

    def poll(self, max_n=256, wait_us=1000):
        """[(tag, ids, dists, t_submit_ns, t_done_ns)] of up to max_n finished requests."""
        import numpy as np
        km = self.cfg.k_max
        tags = np.empty(max_n, np.uint64)
        ids = np.empty((max_n, km), np.int32)
        dists = np.empty((max_n, km), np.float32)
        ts = np.empty(max_n, np.int64)
        td = np.empty(max_n, np.int64)
        n = lib().sa_server_poll(self._h, max_n, tags.ctypes.data, ids.ctypes.data, dists.ctypes.data, km,
                                 ts.ctypes.data, td.ctypes.data, int(wait_us))
        if n < 0:
            _check(n, "sa_server_poll")
        return [(int(tags[i]), ids[i], dists[i], int(ts[i]), int(td[i])) for i in range(n)]

    def replay(self, queries, k, L, M, arrival_ns):
        """Native load replay: returns (ids, dists, latency_ns, wall_ns); row i of ids has
        its first k[i] entries."""
        import numpy as np
        q = np.ascontiguousarray(queries, dtype=np.float32)
        if q.shape[1] < self.d:
            q = np.ascontiguousarray(np.pad(q, ((0, 0), (0, self.d - q.shape[1]))))
        n = q.shape[0]
        ks = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (n,)))
        Ls = np.ascontiguousarray(np.broadcast_to(np.asarray(L, np.int32), (n,)))
        Ms = np.ascontiguousarray(np.broadcast_to(np.asarray(M, np.int32), (n,)))
        arr = np.ascontiguousarray(arrival_ns, dtype=np.int64)
        km = self.cfg.k_max
        ids = np.full((n, km), -1, np.int32)
        dists = np.full((n, km), np.inf, np.float32)
        lat = np.zeros(n, np.int64)
        wall = C.c_int64(0)
        _check(lib().sa_server_replay(self._h, q.ctypes.data, n, q.shape[1], ks.ctypes.data, Ls.ctypes.data,
                                      Ms.ctypes.data, arr.ctypes.data, ids.ctypes.data, dists.ctypes.data, km,
                                      lat.ctypes.data, C.byref(wall)), "sa_server_replay")
        return ids, dists, lat, int(wall.value)

    def stats(self) -> dict:
        v = [C.c_int64(0) for _ in range(5)]
        _check(lib().sa_server_stats(self._h, *[C.byref(x) for x in v]), "sa_server_stats")
        return dict(zip(["completed", "batches", "launches", "max_batch", "sum_batch"], [x.value for x in v]))


ORDERS = {"degree": 0, "bfs": 1}


def graph_order(adj: torch.Tensor, entry: int, mode="bfs", stream=None) -> torch.Tensor:
    """perm (int32, device): perm[i] = original id of new vertex i (sa_graph_order)."""
    assert adj.dtype == torch.int32 and adj.is_contiguous() and adj.is_cuda
    perm = torch.empty(adj.shape[0], dtype=torch.int32, device=adj.device)
    _check(lib().sa_graph_order(adj.data_ptr(), adj.shape[0], adj.shape[1], int(entry), ORDERS[mode],
                                perm.data_ptr(), _stream(stream)), "sa_graph_order")
    return perm


def permute_rows(src: torch.Tensor, perm: torch.Tensor, stream=None) -> torch.Tensor:
    src = src.contiguous()
    dst = torch.empty_like(src)
    row_bytes = src.element_size() * (src.numel() // max(1, src.shape[0]))
    _check(lib().sa_permute_rows(src.data_ptr(), src.shape[0], row_bytes, perm.data_ptr(), dst.data_ptr(),
                                 _stream(stream)), "sa_permute_rows")
    return dst


def permute_graph(adj: torch.Tensor, perm: torch.Tensor, stream=None):
    """(adj in the new numbering, inv) with inv[perm[i]] = i."""
    out = torch.empty_like(adj)
    inv = torch.empty_like(perm)
    _check(lib().sa_permute_graph(adj.data_ptr(), adj.shape[0], adj.shape[1], perm.data_ptr(), inv.data_ptr(),
                                  out.data_ptr(), _stream(stream)), "sa_permute_graph")
    return out, inv


def reorder(base: torch.Tensor, adj: torch.Tensor, entry: int, mode="bfs"):
    """(base, adj, entry, perm) of the renumbered index; an Index over them built with
    id_map=perm returns original ids."""
    perm = graph_order(adj, entry, mode)
    base2 = permute_rows(pad_dim(_mat(base, "base")), perm)
    adj2, inv = permute_graph(adj, perm)
    torch.cuda.synchronize()
    return base2, adj2, int(inv[entry].item()), perm


def gather_ceiling(vec: torch.Tensor, iters=64, waves=8192, reps=5, seed=1) -> dict:
    """Random whole-row gather bandwidth over vec (sa_gather_probe), best-of-reps median."""
    vec = pad_dim(_mat(vec, "vectors"))
    n, d = vec.shape
    lpv = 1
    while lpv < 64 and 4 * lpv < d // 4:
        lpv *= 2
    sink = torch.empty(waves * 64, dtype=torch.float32, device=vec.device)
    s = torch.cuda.current_stream()
    ms = []
    for r in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        _check(lib().sa_gather_probe(vec.data_ptr(), n, d, vec.stride(0), int(iters), int(waves), int(seed + r),
                                     sink.data_ptr(), int(s.cuda_stream)), "sa_gather_probe")
        b.record()
        torch.cuda.synchronize()
        if r:
            ms.append(a.elapsed_time(b))
    rows = waves * iters * (64 // lpv)
    t = sorted(ms)[len(ms) // 2]
    return {"GBs": rows * d * 4 / (t / 1e3) / 1e9, "rows": rows, "row_bytes": d * 4, "ms": t}
