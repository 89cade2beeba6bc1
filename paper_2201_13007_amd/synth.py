"""Seeded synthetic workloads shaped like the paper's datasets (Table 3: SIFT 1M x 128,
DEEP 96-d, GIST 960-d).  The paper's datasets are public benchmark files that are not
available here; these generators stand in for them with the same shapes and a value
distribution of the same kind (integers 0..255 for SIFT, unit-norm floats for DEEP).

This module holds only random number generation: no distance, search or graph
arithmetic.  Both the CPU oracle and the GPU path take their inputs from here.

Seeding: every stream is ``numpy.random.default_rng([2201, 13007, config, stream])``
(PCG64).  Streams: 0 mixture parameters, 1 base labels, 2 base noise, 3 query labels,
4 query noise, 5 per-query parameters.  Rows are drawn sequentially, so a workload
with fewer base points is exactly a prefix of the larger one.
"""
from __future__ import annotations

import dataclasses
import numpy as np

SEED_PREFIX = (2201, 13007)

# stream ids
S_MIX, S_BASE_LABEL, S_BASE_NOISE, S_Q_LABEL, S_Q_NOISE, S_QPARAM = range(6)

_CHUNK = 1 << 16


def rng(config: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([SEED_PREFIX[0], SEED_PREFIX[1], int(config), int(stream)])


@dataclasses.dataclass
class Workload:
    name: str
    base: np.ndarray          # (n, d) float32, C-contiguous
    queries: np.ndarray       # (nq, d) float32
    metric: str               # "l2" | "ip"
    k: int
    graph_knn: int            # candidate list size for graph construction
    graph_R: int              # out-degree cap
    graph_prune: str          # "knn" (keep the R nearest) | "rng" (relative-neighbourhood rule)
    graph_repair: bool        # make every vertex reachable from the entry point
    info: dict


def _mixture_rows(config, n, means, sigma, label_stream, noise_stream):
    """means[label] + sigma * N(0, 1), labels uniform over components, in float64."""
    ncomp, d = means.shape
    labels = rng(config, label_stream).integers(0, ncomp, size=n)
    g = rng(config, noise_stream)
    out = np.empty((n, d), dtype=np.float64)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        out[s:e] = means[labels[s:e]] + sigma * g.standard_normal((e - s, d))
    return out, labels


def tiny(n: int = 10_000, nq: int = 100, d: int = 32) -> Workload:
    """Config 1: iid uniform[0,1) float32, 16-NN graph, entry = medoid, k=10."""
    base = rng(1, S_BASE_NOISE).random((n, d), dtype=np.float32)
    queries = rng(1, S_Q_NOISE).random((nq, d), dtype=np.float32)
    return Workload("tiny-uniform-10k-d32", np.ascontiguousarray(base), np.ascontiguousarray(queries),
                    "l2", 10, 16, 16, "knn", False, {"config": 1})


def sift_like(n: int = 1_000_000, nq: int = 10_000, d: int = 128, ncomp: int = 256,
              sigma: float = 20.0) -> Workload:
    """Config 2: 256-component isotropic Gaussian mixture, means uniform in [0,255],
    sigma 20, rounded to nearest (ties to even) and clipped to 0..255, stored as float32."""
    means = rng(2, S_MIX).uniform(0.0, 255.0, size=(ncomp, d))
    xb, lb = _mixture_rows(2, n, means, sigma, S_BASE_LABEL, S_BASE_NOISE)
    xq, lq = _mixture_rows(2, nq, means, sigma, S_Q_LABEL, S_Q_NOISE)
    base = np.clip(np.rint(xb), 0, 255).astype(np.float32)
    queries = np.clip(np.rint(xq), 0, 255).astype(np.float32)
    return Workload(f"sift-like-{n}x{d}", base, queries, "l2", 10, 64, 32, "rng", True,
                    {"config": 2, "ncomp": ncomp, "sigma": sigma, "base_labels": lb, "query_labels": lq})


def deep_like(n: int = 1_000_000, nq: int = 10_000, d: int = 96, ncomp: int = 512,
              sigma: float = 1.0, decay: float = 1.0, config: int = 3) -> Workload:
    """Config 3 (and 5 with 1024 components): a Gaussian mixture in coordinates whose
    variance falls as 1 / i^decay (i = 1..d), the way it does in PCA-compressed
    descriptors: means N(0, I), x = (mean + sigma N(0, I)) * i^(-decay/2) per coordinate,
    then scaled to unit l2 norm; inner-product metric.  With decay 0 the mixture is
    isotropic and, at sigma 1 and 1M points, about as hard to navigate as 96-d noise."""
    means = rng(config, S_MIX).standard_normal((ncomp, d))
    xb, lb = _mixture_rows(config, n, means, sigma, S_BASE_LABEL, S_BASE_NOISE)
    xq, lq = _mixture_rows(config, nq, means, sigma, S_Q_LABEL, S_Q_NOISE)
    sd = (np.arange(d) + 1.0) ** (-0.5 * decay)
    xb *= sd
    xq *= sd
    xb /= np.linalg.norm(xb, axis=1, keepdims=True)
    xq /= np.linalg.norm(xq, axis=1, keepdims=True)
    return Workload(f"deep-like-{n}x{d}", xb.astype(np.float32), xq.astype(np.float32), "ip", 10, 64, 32,
                    "rng", True, {"config": config, "ncomp": ncomp, "sigma": sigma, "decay": decay,
                                  "base_labels": lb, "query_labels": lq})


def gist_like(n: int = 1_000_000, nq: int = 20_000, d: int = 960, ncomp: int = 128,
              sigma: float = 0.1) -> Workload:
    """Config 4: means uniform [0,1]^960, sigma 0.1, no clipping; per-query (L, k, M)."""
    means = rng(4, S_MIX).uniform(0.0, 1.0, size=(ncomp, d))
    xb, lb = _mixture_rows(4, n, means, sigma, S_BASE_LABEL, S_BASE_NOISE)
    xq, lq = _mixture_rows(4, nq, means, sigma, S_Q_LABEL, S_Q_NOISE)
    g = rng(4, S_QPARAM)
    L = np.rint(np.exp(g.uniform(np.log(32.0), np.log(1024.0), size=nq))).astype(np.int32)
    k = g.choice(np.array([1, 10, 100], dtype=np.int32), size=nq)
    M = g.choice(np.array([1, 4, 8], dtype=np.int32), size=nq)
    return Workload(f"gist-like-{n}x{d}", xb.astype(np.float32), xq.astype(np.float32), "l2", 10, 64, 32,
                    "rng", True, {"config": 4, "ncomp": ncomp, "sigma": sigma, "L": L, "k": k, "M": M,
                                  "base_labels": lb, "query_labels": lq})


def integer_grid(n: int, d: int, nq: int, hi: int = 16, config: int = 90, lo: int = 0) -> Workload:
    """Integer-valued vectors (uniform over lo..hi-1) for order-independent exact
    distances in tests; with a narrow range, duplicates and exact distance ties are
    common by design."""
    base = rng(config, S_BASE_NOISE).integers(lo, hi, size=(n, d)).astype(np.float32)
    queries = rng(config, S_Q_NOISE).integers(lo, hi, size=(nq, d)).astype(np.float32)
    return Workload(f"int-grid-{n}x{d}", base, queries, "l2", 10, 16, 16, "knn", False, {"config": config})
