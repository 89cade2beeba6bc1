"""Benchmark: QPS and p50/p99 latency at recall@10 = 0.99 on the SIFT-shaped 1M x 128
workload (synthetic: 256-component Gaussian mixture rounded to 0..255), one GPU.

A step is one pass of the whole search over the batch of 10,000 queries: one launch of
the search kernel with the index and the queries already resident in HBM.  Setup (not
timed): generate the data, build the graph on the GPU (exact 64-NN, relative-
neighbourhood pruning to R = 32, connectivity repair, medoid entry), exact ground truth
on the GPU, and the operating point: for each walker count M the smallest L of the sweep
whose mean recall@10 reaches 0.99; the point with the highest QPS is timed.

With --workload deep: the DEEP-shaped 1M x 96 inner-product workload (512-component
mixture with per-coordinate variance 1/i, scaled to unit norm) searched over float32, bf16 and fp8-e4m3 vector storage,
with and without the exact float32 re-rank of the final list.  Each form is timed at its
own operating point (smallest swept L reaching recall@10 0.99) and compared with the
float32 path at equal L: recall, QPS and the error of the returned distances against
FP64.

With --workload gist: the GIST-shaped 1M x 960 batch (128-component mixture, sigma 0.1),
20,000 queries each with its own L (log-uniform in [32, 1024], raised to k), k in
{1, 10, 100} and M in {1, 4, 8}, searched as one batch: planned into classes, tuned,
captured in a HIP graph and replayed.  A step is one replay.  The plain path for the
same results, one search call per distinct (L, k, M), is timed beside it.

With --workload serve: the served DEEP-shaped 10M x 96 index (1024-component mixture,
coordinate variance 1/i, unit norm) stored as bf16 with an exact float32 re-rank of the
final list, resident on the GPU behind the serving loop.  Recall targets {0.9, 0.99,
0.999} are mapped to L on a calibration sample; each request draws a target; Poisson
arrival traces at 10k-500k queries/s are replayed natively and p50 / p99 latency
(completion minus scheduled arrival) and achieved throughput are reported per rate.
The 10M graph is built from exact 64-NN candidates computed on the matrix cores in
1M-row chunks (--serve-graph partition: from overlapping partitions instead, each
point's two nearest of 2048 sampled centroids with exact kNN inside each partition).

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# the served workload runs up to 16 micro-batches at once, the batched one up to 8
# streams: give each its own hardware queue (HIP's default is 4; streams beyond the queue count share queues and serialise
# their kernels).  Read when the runtime starts, so set here, over any inherited value.
if "--workload" in sys.argv and ("serve" in sys.argv or "gist" in sys.argv):
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

# the synchronisation schedules of the paper the latency candidates use (Sec. 4.3)
SYNCS = {"adaptive": dict(sync="adaptive", rho=0.8, staged=True),
         "bsp": dict(sync="bsp", staged=True),
         "static8": dict(sync="static", static_I=8, staged=True)}

L_SWEEP = [32, 48, 64, 80, 96, 112, 128, 144, 160, 176, 192, 208, 224, 240, 256, 272, 288, 304, 320, 336, 352, 384,
           416, 448, 480, 512]
M_SWEEP = [1, 2, 4, 8, 16]
TARGET = 0.99
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def recall_at_k(ids, gt, k):
    import torch
    hit = (ids[:, :k, None] == gt[:, None, :k]).any(-1).sum(1)
    return (hit.float() / k)


# every source that goes into the search kernels: measured traffic is reported only while
# these files are unchanged
SEARCH_SOURCES = ("search.hip", "sa_internal.h", "search_body.h", "search_single.h", "search_single_f32.hip",
                  "search_multi.h", "search_multi_f32.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in SEARCH_SOURCES:
        with open(os.path.join(ROOT, "paper_2201_13007_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload_key):
    """HBM traffic per launch measured with rocprofv3 counters (profiles/), if it was taken
    on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "search_kernel_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("kernel_source") != kernel_source_hash() or t.get("workload") != workload_key:
        return None
    return t


def lscpu_model():
    """CPU model, sockets, cores and threads from lscpu (model name from /proc/cpuinfo if
    lscpu is missing)."""
    import subprocess
    f = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for ln in out.splitlines():
            key, _, v = ln.partition(":")
            f[key.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    model = f.get("Model name", "")
    if not model:
        try:
            with open("/proc/cpuinfo") as fh:
                model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
        except OSError:
            pass
    if f.get("Socket(s)"):
        model += (f"; {f.get('Socket(s)')} socket(s) x {f.get('Core(s) per socket', '?')} cores x "
                  f"{f.get('Thread(s) per core', '?')} threads, {f.get('CPU(s)', '?')} logical CPUs")
    return model


def cpu_oracle(w, base_h, adj_h, entry, perm, gt, gpu_ids, k, point, seconds, lat_queries=1000, bfis_L=None,
               lockstep=None):
    """The oracle timed on the host cores, on the index the GPU searches (renumbered, ids
    mapped back), as a reported baseline.
      point = (M, L, sync keywords): the GPU's timed operating point.  Throughput: Algorithm
        3 in lockstep over a growing prefix of the queries, one query per OpenMP thread, until
        about `seconds` of wall time; its ids are compared with the GPU's.  Latency: the first
        lat_queries queries one at a time (one thread), host wall time.
      bfis_L: Algorithm 1 at its own smallest swept L reaching the recall target (the
        sweep's one-walker point): throughput on all cores over a prefix, recall@k of that
        prefix, and one-thread latency as above.
      lockstep = (M, L, sync keywords): the GPU's best batch-1 point, one-thread latency."""
    import oracle
    M, L, skw = point
    nq = w.queries.shape[0]
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    back = (lambda ids: np.where(ids >= 0, perm[np.maximum(ids, 0)], -1)) if perm is not None else (lambda ids: ids)

    def throughput(run, budget):
        done, t, bs, outs = 0, 0.0, 256, []
        while t < budget and done < nq:
            n1 = min(bs, nq - done)
            s0 = time.perf_counter()
            outs.append(run(w.queries[done:done + n1]))
            t += time.perf_counter() - s0
            done += n1
            bs = min(bs * 2, 4096)
        return done, t, back(np.concatenate(outs))

    def latency(run, count):
        count = min(count, nq)
        lat = np.empty(count)
        for i in range(count):
            s0 = time.perf_counter()
            run(w.queries[i:i + 1])
            lat[i] = (time.perf_counter() - s0) * 1e3
        return {"latency_p50_ms": round(float(np.percentile(lat, 50)), 4),
                "latency_p99_ms": round(float(np.percentile(lat, 99)), 4), "latency_queries": int(count)}

    def alg3(Mx, Lx, kw):
        return lambda q: oracle.speedann(base_h, adj_h, entry, q, k, Lx, Mx, metric=w.metric, **kw)[0]

    done, t, ids = throughput(alg3(M, L, skw), seconds)
    same = float((ids == gpu_ids[:done]).all(1).mean())
    cpu = {"value": round(done / t, 1), "unit": "queries/s", "cores": nthreads, "kind": "oracle",
           "sample": f"first {done} of the {nq} queries, the index the GPU searches"
                     + (" (renumbered, ids mapped back)" if perm is not None else "")
                     + f", f32 vectors, M={M}, L={L}, schedule {skw}: lockstep emulation of Algorithm 3 in plain C, "
                     f"one query per OpenMP thread",
           "cpu_model": lscpu_model(),
           "ids_equal_gpu": same,
           **latency(alg3(M, L, skw), lat_queries)}
    cpu["latency_sample"] = f"first {cpu['latency_queries']} queries one at a time, one thread, host wall time"
    if bfis_L:
        run = lambda q: oracle.bfis(base_h, adj_h, entry, q, k, bfis_L, metric=w.metric)[0]
        done_b, t_b, ids_b = throughput(run, seconds / 2)
        cpu["bfis"] = {"algorithm": "Algorithm 1 (best-first search, one walker)", "L": int(bfis_L),
                       "qps": round(done_b / t_b, 1), "queries": int(done_b),
                       "recall@10": round(float(oracle.recall(ids_b, gt[:done_b], k).mean()), 5),
                       **latency(run, lat_queries)}
    if lockstep is not None and (tuple(lockstep[:2]) != (M, L) or lockstep[2] != skw):
        M2, L2, kw2 = lockstep
        cpu["lockstep_point"] = {"M": int(M2), "L": int(L2), "sync": kw2, **latency(alg3(M2, L2, kw2), lat_queries)}
    log(f"cpu oracle: {cpu['value']} q/s on {nthreads} threads ({done} queries, {t:.1f}s), ids equal to the GPU's "
        f"for {same:.4f} of them; one thread p50 {cpu['latency_p50_ms']} ms"
        + (f"; Algorithm 1 at L={bfis_L}: {cpu['bfis']['qps']} q/s, p50 {cpu['bfis']['latency_p50_ms']} ms"
           if bfis_L else ""))
    return cpu


def timed_launches(torch, fn, reps):
    """Per-launch device times (ms) of fn() on torch's current stream, which is the stream
    the search runs on."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in evs])


STORAGE_BYTES = {"f32": 4, "bf16": 2, "fp8": 1}


def deep_main(args, torch, B, synth, dev):
    t0 = time.time()
    w = synth.deep_like(n=args.n, nq=args.nq)
    log(f"data {w.name}: {w.base.shape} + {w.queries.shape} queries in {time.time() - t0:.1f}s")
    base = torch.from_numpy(w.base).to(dev)
    queries = torch.from_numpy(w.queries).to(dev)
    k, d, R = w.k, w.base.shape[1], w.graph_R
    nq = args.nq

    t0 = time.time()
    adj, entry, ginfo = B.build_graph(base, w.graph_knn, R, w.graph_prune, w.graph_repair, keep_local=1,
                                      metric=w.metric)
    torch.cuda.synchronize()
    t_graph = time.time() - t0
    log(f"graph built in {t_graph:.1f}s: entry {entry}, {ginfo}")
    t0 = time.time()
    gt, _ = B.knn(base, queries, k, metric=w.metric)
    torch.cuda.synchronize()
    log(f"ground truth in {time.time() - t0:.2f}s")

    # default: two walkers merging after every step (one wavefront), the fastest form found
    M = args.M or 2
    skw = SYNCS[args.sync if args.sync != "all" else ("bsp" if M == 2 else "adaptive")]
    forms = [("f32", 0), ("bf16", 0), ("bf16", -1), ("fp8", 0), ("fp8", -1)]
    index = {s: B.Index(base, adj, entry, metric=w.metric, dtype=s) for s in ("f32", "bf16", "fp8")}
    base64 = w.base.astype(np.float64)
    q64 = w.queries.astype(np.float64)

    def run(storage, rr, L, stats=False, out=None):
        p = B.make_params(rerank=rr, **skw)
        return index[storage].search(queries, k, L, M, params=p, stats=stats, out=out)

    def measure(storage, rr, L, reps):
        r = run(storage, rr, L, stats=True)
        ids = r.ids
        rec = recall_at_k(ids, gt, k).mean().item()
        out = (torch.empty_like(r.ids), torch.empty_like(r.dists), None)
        run(storage, rr, L, out=out)
        ms = timed_launches(torch, lambda: run(storage, rr, L, out=out), reps)
        # returned distances against FP64 inner products of the same (query, id) pairs
        ih, dh = ids.cpu().numpy(), r.dists.cpu().numpy().astype(np.float64)
        ok = ih >= 0
        exact = -np.einsum("qd,qkd->qk", q64, base64[np.where(ok, ih, 0)])
        err = np.abs(dh - exact)[ok]
        st = r.stats.cpu().numpy()
        return {"storage": storage, "rerank": "whole list" if rr < 0 else "none", "L": L,
                "recall": round(rec, 5), "ms": round(float(np.median(ms)), 4),
                "qps": round(nq / float(np.median(ms)) * 1e3),
                "dist_err_max": float(f"{err.max():.3e}"), "dist_err_mean": float(f"{err.mean():.3e}"),
                "dist_comps": round(float(st[:, 3].mean()), 1), "expansions": round(float(st[:, 2].mean()), 1),
                "flagged": int(((st[:, 5] & 3) != 0).sum())}, st, ms

    # each form's operating point
    points, at_f32 = [], []
    for storage, rr in forms:
        hit = None
        for L in ([args.L] if args.L else L_SWEEP):
            row, _, _ = measure(storage, rr, L, 3)
            log(f"{storage:4s} rerank={row['rerank']:10s} L={L:4d} recall={row['recall']:.4f} "
                f"qps={row['qps']:>9} err max {row['dist_err_max']:.2e} mean {row['dist_err_mean']:.2e}")
            if row["recall"] >= TARGET:
                hit = row
                break
        points.append(hit if hit else row)
    L32 = points[0]["L"]
    for storage, rr in forms:
        row, _, _ = measure(storage, rr, L32, 3)
        at_f32.append(row)

    # the fastest form at the target is timed over the full step count
    ok_points = [p for p in points if p["recall"] >= TARGET]
    best = max(ok_points, key=lambda p: p["qps"]) if ok_points else max(points, key=lambda p: p["recall"])
    storage, rr, L = best["storage"], (-1 if best["rerank"] != "none" else 0), best["L"]
    row, stats, _ = measure(storage, rr, L, 1)
    out = (torch.empty((nq, k), dtype=torch.int32, device=dev), torch.empty((nq, k), dtype=torch.float32, device=dev),
           None)
    for _ in range(args.warmup):
        run(storage, rr, L, out=out)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    launch_ms = timed_launches(torch, lambda: run(storage, rr, L, out=out), args.steps)
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1e3 / args.steps
    qps = nq / (ms_per_step / 1e3)
    log(f"timed {storage} rerank={best['rerank']} M={M} L={L}: {ms_per_step:.3f} ms/step, QPS {qps:,.0f}")

    # algorithmic bytes of the search: per distance one stored row (+ its fp8 scale), per
    # expansion one adjacency row, the query, and (re-rank) the float32 rows of the list
    D = stats[:, 3].astype(np.float64)
    E = stats[:, 2].astype(np.float64)
    row_bytes = d * STORAGE_BYTES[storage] + (4 if storage == "fp8" else 0)
    bytes_launch = float((D * row_bytes + E * R * 4 + d * 4 + k * 8).sum())
    if rr:
        bytes_launch += float(nq * L * (d * 4 + 4))
    achieved = bytes_launch / (launch_ms.mean() / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "algorithmic_bytes_per_launch": round(bytes_launch),
                "kernel_ms": round(float(launch_ms.mean()), 4),
                "note": "search and re-rank launches timed together" if rr else "search launch"}
    cpu = None
    if not args.no_cpu:
        r32 = index["f32"].search(queries, k, L32, M, **skw)
        cpu = cpu_oracle(w, w.base, adj.cpu().numpy(), entry, None, gt.cpu().numpy(), r32.ids.cpu().numpy(), k,
                         (M, L32, skw), args.cpu_seconds, args.cpu_latency_queries)
    res = {
        "metric": "QPS and recall@10 by vector storage (fp32 / bf16 / fp8-e4m3, exact fp32 re-rank), "
                  "distance error vs FP64, 1M×96 DEEP-shaped inner product, 1 GPU",
        "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f64", "bf16": "bf16 storage, f64 accumulate",
                  "fp8": "fp8-e4m3 storage, f64 accumulate"}[storage],
        "data": "synthetic",
        "config": {
            "workload": f"deep-like {args.n}x{d} (512-component mixture, sigma 1, coordinate variance 1/i, "
                        f"unit norm), {nq} queries, k={k}, inner product",
            "graph": f"exact 64-NN, relative-neighbourhood prune to R={R}, repair (keep_local 1), medoid entry",
            "graph_build_s": round(t_graph, 1), "M": M, **skw,
            "timed": {"storage": storage, "rerank": best["rerank"], "L": L, "recall@10": row["recall"]},
            "operating_points": points,
            "at_f32_L": at_f32,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def build_graph_logged(torch, B, base, knn_k, R, prune_mode, chunk=100_000, metric="l2"):
    """The steps of sa_build_graph (medoid entry, exact knn_k-NN candidates, pruning,
    reverse edges, repair), with the candidate search cut into row chunks so that each
    finished chunk is logged.  A chunk's rows search the whole base with k = knn_k + 1
    and drop their own id, which leaves the same knn_k candidates as excluding it."""
    n = base.shape[0]
    entry = B.medoid(base)
    cand = torch.empty((n, knn_k), dtype=torch.int32, device=base.device)
    t0 = time.time()
    for s0 in range(0, n, chunk):
        e0 = min(n, s0 + chunk)
        ids, _ = B.knn(base, base[s0:e0], knn_k + 1, metric=metric)
        own = torch.arange(s0, e0, device=base.device, dtype=torch.int32)[:, None]
        keep = ids != own
        # rows where the own id is not among the knn_k + 1 keep their first knn_k
        first = torch.cumsum(keep.to(torch.int32), 1) <= knn_k
        cand[s0:e0] = ids[keep & first].view(e0 - s0, knn_k)
        torch.cuda.synchronize()
        log(f"candidates: rows {e0:,} of {n:,} in {time.time() - t0:.1f}s")
    adj = B.prune(base, cand, R, prune_mode, metric=metric)
    B.reverse_edges(base, adj, metric=metric)
    bridges, comps = B.repair(base, adj, entry, keep_local=1, metric=metric)
    torch.cuda.synchronize()
    return adj, entry, {"bridges": bridges, "components": comps}


def ordered_keys(torch, dists, ids):
    """(distance, id) as sortable int64 keys, as the library orders its lists."""
    b = dists.contiguous().view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    neg = b >= 0x80000000
    o = torch.where(neg, (~b) & 0xFFFFFFFF, b | 0x80000000)
    o = torch.where(dists == 0, torch.full_like(o, 0x80000000), o)
    return (o << 32) | (ids.to(torch.int64) & 0xFFFFFFFF)


def build_graph_partitioned(torch, B, base, knn_k, R, prune_mode, metric, parts=2048, seed=5):
    """Approximate kNN candidates from overlapping partitions, then the library's pruning,
    reverse edges, repair and medoid entry.  Each point joins the partitions of its two
    nearest of `parts` sampled centroids; exact kNN inside every partition gives each
    point two candidate lists, merged by (distance, id) without duplicates."""
    n = base.shape[0]
    dev = base.device
    t0 = time.time()
    entry = B.medoid(base)
    cidx = torch.from_numpy(np.sort(np.random.default_rng([2201, 13007, seed]).choice(n, parts, replace=False)))
    cent = base.index_select(0, cidx.to(dev)).contiguous()
    assign, _ = B.knn(cent, base, 2, metric=metric)
    flat = assign.reshape(-1).to(torch.int64)
    pts = torch.arange(n, device=dev, dtype=torch.int64).repeat_interleave(2)
    col = torch.arange(2, device=dev, dtype=torch.int64).repeat(n)
    order = torch.argsort(flat, stable=True)
    flat, pts, col = flat[order], pts[order], col[order]
    counts = torch.bincount(flat, minlength=parts).cpu().numpy()
    starts = np.concatenate([[0], np.cumsum(counts)])
    keys = torch.full((n, 2 * knn_k), -1, dtype=torch.int64, device=dev)   # -1 = empty (largest unsigned)
    log(f"partitions: {parts}, sizes {counts.min()}..{counts.max()} in {time.time() - t0:.1f}s")
    for p in range(parts):
        a, b = int(starts[p]), int(starts[p + 1])
        if b - a < 2:
            continue
        mem, c = pts[a:b], col[a:b]
        kk = min(knn_k + 1, b - a)
        ids, d = B.knn(base.index_select(0, mem), base.index_select(0, mem), kk, metric=metric)
        gid = mem[ids.to(torch.int64)]
        own = gid == mem[:, None]
        kept = (~own) & (torch.cumsum((~own).to(torch.int32), 1) <= knn_k)
        rows = torch.full((b - a, knn_k), -1, dtype=torch.int64, device=dev)
        cnt = kept.sum(1)
        pos = torch.cumsum(kept.to(torch.int64), 1) - 1
        r_i, c_i = torch.nonzero(kept, as_tuple=True)
        rows[r_i, pos[r_i, c_i]] = ordered_keys(torch, d[r_i, c_i], gid[r_i, c_i])
        keys[mem[:, None], c[:, None] * knn_k + torch.arange(knn_k, device=dev)[None, :]] = rows
        if (p + 1) % 256 == 0:
            torch.cuda.synchronize()
            log(f"partition kNN: {p + 1} of {parts} in {time.time() - t0:.1f}s")
    # merge the two lists of every point: unsigned order = (distance, id); drop repeats
    u = keys ^ (-0x8000000000000000)          # signed order of the unsigned keys
    u, _ = torch.sort(u, dim=1)
    dup = torch.zeros_like(u, dtype=torch.bool)
    dup[:, 1:] = u[:, 1:] == u[:, :-1]
    u = torch.where(dup, torch.full_like(u, 0x7FFFFFFFFFFFFFFF), u)
    u, _ = torch.sort(u, dim=1)
    k0 = u[:, :knn_k] ^ (-0x8000000000000000)
    cand = torch.where(k0 == -1, torch.full_like(k0, -1), k0 & 0xFFFFFFFF).to(torch.int32).contiguous()
    del keys, u, dup
    torch.cuda.synchronize()
    log(f"candidates merged in {time.time() - t0:.1f}s; empty slots {(cand < 0).sum().item()}")
    adj = B.prune(base, cand, R, prune_mode, metric=metric)
    B.reverse_edges(base, adj, metric=metric)
    torch.cuda.synchronize()
    log(f"pruned and reversed in {time.time() - t0:.1f}s")
    bridges, comps = B.repair(base, adj, entry, keep_local=1, metric=metric)
    torch.cuda.synchronize()
    return adj, entry, {"bridges": bridges, "components": comps}


def serve_main(args, torch, B, synth, dev):
    t0 = time.time()
    w = synth.deep_like(n=args.n, nq=args.nq, ncomp=1024, config=5)
    log(f"data {w.name} (1024 components): {w.base.shape} + {w.queries.shape} queries in {time.time() - t0:.1f}s")
    base = torch.from_numpy(w.base).to(dev)
    queries = torch.from_numpy(w.queries).to(dev)
    d, R, k, Ms = w.base.shape[1], w.graph_R, 10, args.serve_M
    skw = SYNCS[args.serve_sync]
    t0 = time.time()
    if args.serve_graph == "exact":
        adj, entry, ginfo = build_graph_logged(torch, B, base, w.graph_knn, R, w.graph_prune, chunk=1_000_000,
                                               metric=w.metric)
    else:
        adj, entry, ginfo = build_graph_partitioned(torch, B, base, w.graph_knn, R, w.graph_prune, w.metric)
    t_graph = time.time() - t0
    log(f"graph built in {t_graph:.1f}s: entry {entry}, {ginfo}")
    t0 = time.time()
    gt, _ = B.knn(base, queries, k, metric=w.metric)
    torch.cuda.synchronize()
    gth = gt.cpu().numpy()
    log(f"ground truth in {time.time() - t0:.1f}s")
    ix = B.Index(base, adj, entry, metric=w.metric, dtype="bf16")

    # recall target -> L, calibrated on the queries that are served
    nc = args.nq   # every query the replays cycle through, so the targets hold for them
    sweep = {}
    for L in [16, 24, 32, 48, 64, 80, 96, 112, 128, 160, 192, 224, 256, 320, 384, 448, 512, 640, 768, 896, 1024]:
        r = ix.search(queries[:nc], k, L, Ms, rerank=-1, **skw)
        rec = recall_at_k(r.ids, gt[:nc], k).mean().item()
        sweep[L] = round(rec, 5)
        log(f"calibration M={Ms} {args.serve_sync} L={L}: recall@10 {rec:.4f}")
    targets = [0.9, 0.99, 0.999]
    tL = {}
    for t in targets:
        # a tenth of the remaining error as margin: each target's requests are a random
        # part of the queries, whose recall scatters around the calibrated mean
        ok = [L for L, rc in sweep.items() if rc >= t + 0.1 * (1 - t)]
        tL[t] = min(ok) if ok else max(sweep)
    log(f"target -> L: {tL}")

    # single-request latency: one query per search call, host wall time, on a sample
    single = {}
    q1 = torch.empty((1, k), dtype=torch.int32, device=dev), torch.empty((1, k), dtype=torch.float32, device=dev), None
    for Lx in sorted(set(tL.values())):
        for Mx, sx in ((1, args.serve_sync), (2, "bsp"), (4, args.serve_sync), (16, args.serve_sync)):
            for i in range(5):
                ix.search(queries[i:i + 1], k, Lx, Mx, rerank=-1, out=q1, **SYNCS[sx])
            torch.cuda.synchronize()
            lat1 = []
            for i in range(100):
                s0 = time.perf_counter()
                ix.search(queries[i:i + 1], k, Lx, Mx, rerank=-1, out=q1, **SYNCS[sx])
                torch.cuda.synchronize()
                lat1.append((time.perf_counter() - s0) * 1e3)
            single[f"L{Lx}_M{Mx}" + ("" if sx == args.serve_sync else f"_{sx}")] = round(float(np.percentile(lat1, 50)), 3)
    log(f"single-request p50 latency (ms): {single}")

    srv = B.Server(ix, slots=args.serve_slots, max_batch=1024, k_max=k, workspace_bytes=8 << 30, rerank=-1, **skw)
    rng = np.random.default_rng([2201, 13007, 5, 9])
    qh = w.queries
    rows = []
    for rate in [int(x) for x in args.rates.split(",") if x]:
        n = int(min(200_000, max(5000, rate)))   # about one second of arrivals
        qi = np.arange(n) % args.nq
        tgt = rng.integers(0, 3, size=n)
        Lr = np.array([tL[targets[t]] for t in tgt], np.int32)
        arrival = np.cumsum(rng.exponential(1e9 / rate, size=n)).astype(np.int64)
        st0 = srv.stats()
        ids, dists, lat, wall = srv.replay(qh[qi], k, Lr, Ms, arrival)
        st1 = srv.stats()
        hit = (ids[:, :k, None] == gth[qi][:, None, :k]).any(-1).mean(1)
        lat_ms = lat / 1e6
        row = {"offered_qps": rate, "requests": n, "achieved_qps": round(n / (wall / 1e9), 1),
               "p50_ms": round(float(np.percentile(lat_ms, 50)), 4),
               "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
               "mean_batch": round((st1["sum_batch"] - st0["sum_batch"]) / max(1, st1["batches"] - st0["batches"]), 1),
               "by_target": {}}
        for j, t in enumerate(targets):
            m = tgt == j
            row["by_target"][str(t)] = {"L": tL[t], "recall@10": round(float(hit[m].mean()), 5),
                                        "p50_ms": round(float(np.percentile(lat_ms[m], 50)), 4),
                                        "p99_ms": round(float(np.percentile(lat_ms[m], 99)), 4)}
        rows.append(row)
        log(f"rate {rate:>7}/s: achieved {row['achieved_qps']:,.0f}/s, p50 {row['p50_ms']:.3f} ms, "
            f"p99 {row['p99_ms']:.3f} ms, mean batch {row['mean_batch']}, "
            f"0.99-target p50/p99 {row['by_target']['0.99']['p50_ms']:.3f}/{row['by_target']['0.99']['p99_ms']:.3f} ms")
    srv.close()
    sustained = [r for r in rows if r["achieved_qps"] >= 0.95 * r["offered_qps"]]
    top = max(sustained, key=lambda r: r["offered_qps"]) if sustained else rows[0]
    res = {
        "metric": "p50/p99 latency and QPS at recall@10=0.99 under Poisson load, 10M×96 DEEP-shaped bf16 "
                  "(exact fp32 re-rank), served, 1 GPU",
        "value": top["achieved_qps"], "unit": "queries/s", "n_gpus": 1, "steps": len(rows), "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 storage, f64 accumulate", "data": "synthetic",
        "config": {
            "workload": f"deep-like {args.n}x{d} (1024-component mixture, sigma 1, coordinate variance 1/i, unit "
                        f"norm), inner product, {args.nq} distinct queries cycled, k={k}",
            "graph": (f"exact 64-NN (matrix cores, 1M-row chunks)" if args.serve_graph == "exact" else
                      "approximate 64-NN candidates from 2048 overlapping partitions") +
                     f", relative-neighbourhood prune to R={R}, reverse edges, repair, medoid entry",
            "graph_build_s": round(t_graph, 1), "M": Ms, **skw, "rerank": "whole list", "calibration": sweep,
            "target_to_L": {str(t): L for t, L in tL.items()},
            "server": {"slots": args.serve_slots, "max_batch": 1024, "workspace_bytes": 8 << 30,
                       "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES", "default")},
            "single_request_p50_ms": single,
            "rates": rows,
            "value_is": "achieved throughput at the highest offered rate sustained (>= 95% achieved)",
            "p50_ms_at_0.99": top["by_target"]["0.99"]["p50_ms"], "p99_ms_at_0.99": top["by_target"]["0.99"]["p99_ms"],
        },
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


def gist_main(args, torch, B, synth, dev):
    t0 = time.time()
    w = synth.gist_like(n=args.n, nq=args.nq)
    log(f"data {w.name}: {w.base.shape} + {w.queries.shape} queries in {time.time() - t0:.1f}s")
    base = torch.from_numpy(w.base).to(dev)
    queries = torch.from_numpy(w.queries).to(dev)
    d, R, nq = w.base.shape[1], w.graph_R, args.nq
    kq = w.info["k"].astype(np.int32)
    Lq = np.maximum(w.info["L"], kq).astype(np.int32)
    Mq = w.info["M"].astype(np.int32)
    t0 = time.time()
    adj, entry, ginfo = build_graph_logged(torch, B, base, w.graph_knn, R, w.graph_prune)
    t_graph = time.time() - t0
    log(f"graph built in {t_graph:.1f}s: entry {entry}, {ginfo}")
    t0 = time.time()
    gt, _ = B.knn(base, queries, int(kq.max()))
    torch.cuda.synchronize()
    log(f"ground truth (k={int(kq.max())}) in {time.time() - t0:.1f}s")

    ix = B.Index(base, adj, entry)
    bt = B.Batch(ix, Lq, kq, Mq, rho=0.8)
    tuning = bt.tune(queries, reps=2)
    log(f"tuning: {tuning}")
    desc = bt.describe()
    for c in desc["classes"]:
        log(f"class M={c['M']} slots/lane={c['slots_per_lane']} queries={c['queries']} L_max={c['L_max']} "
            f"stream={c['stream']} lds_hash_slots={c['lds_hash_slots']} persistent={c['persistent']}")

    # one run with counters: recall and the bytes of the roofline
    r = bt.run(queries, stats=True)
    torch.cuda.synchronize()
    ids = r.ids.cpu().numpy()
    stats = r.stats.cpu().numpy()
    gth = gt.cpu().numpy()
    rec = np.array([np.isin(ids[q, :kq[q]], gth[q, :kq[q]]).mean() for q in range(nq)])
    recall_by_k = {str(int(kk)): round(float(rec[kq == kk].mean()), 5) for kk in np.unique(kq)}
    log(f"recall@k by k: {recall_by_k}, mean {rec.mean():.4f}")

    # capture one run in a HIP graph and replay it
    out = bt.outputs()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bt.run(queries, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bt.run(queries, out=out)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    written = np.arange(ids.shape[1])[None, :] < kq[:, None]
    assert (out[0].cpu().numpy()[written] == ids[written]).all(), "graph replay differs from the eager run"
    t_start = time.perf_counter()
    launch_ms = timed_launches(torch, g.replay, args.steps)
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1e3 / args.steps
    qps = nq / (ms_per_step / 1e3)
    log(f"graph replay: {ms_per_step:.3f} ms per batch, {qps:,.0f} queries/s")

    # the plain path: one search call per distinct (L, k, M), same results
    groups = {}
    for q in range(nq):
        groups.setdefault((int(Lq[q]), int(kq[q]), int(Mq[q])), []).append(q)
    gq = {key: torch.tensor(v, dtype=torch.int64, device=dev) for key, v in groups.items()}
    gqueries = {key: queries.index_select(0, v).contiguous() for key, v in gq.items()}

    def plain():
        res = {}
        for (L1, k1, M1), qv in gqueries.items():
            res[(L1, k1, M1)] = ix.search(qv, k1, L1, M1, rho=0.8)
        return res

    res = plain()
    torch.cuda.synchronize()
    for (L1, k1, M1), rr in res.items():
        sel = groups[(L1, k1, M1)]
        assert (rr.ids.cpu().numpy() == ids[sel, :k1]).all(), "plain path and batch differ"
    t1 = time.perf_counter()
    ev = timed_launches(torch, plain, 1)
    plain_ms = (time.perf_counter() - t1) * 1e3
    log(f"plain path: {len(groups)} search calls, {plain_ms:.1f} ms wall, {ev[0]:.1f} ms on the stream")

    D = stats[:, 3].astype(np.float64)
    E = stats[:, 2].astype(np.float64)
    bytes_launch = float((D * d * 4 + E * R * 4 + d * 4 + kq * 8).sum())
    achieved = bytes_launch / (launch_ms.mean() / 1e3) / 1e9
    t = stats.view(np.int64)[:, 3:5]
    svc_ms = (t[:, 1] - t[:, 0]) / 1e5
    res = {
        "metric": "QPS of a mixed (L, k, M) batch in one captured HIP graph, recall@k vs exact, "
                  "1M×960 GIST-shaped, 1 GPU",
        "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {
            "workload": f"gist-like {args.n}x{d} (128-component mixture, sigma 0.1), {nq} queries, L log-uniform "
                        f"[32, 1024] raised to k, k in {{1, 10, 100}}, M in {{1, 4, 8}}, l2",
            "graph": f"exact 64-NN, relative-neighbourhood prune to R={R}, repair (keep_local 1), medoid entry",
            "graph_build_s": round(t_graph, 1), "sync": "adaptive", "rho": 0.8, "staged": True,
            "recall_at_k_by_k": recall_by_k, "recall_mean": round(float(rec.mean()), 5),
            "classes": desc["classes"], "tuning": tuning,
            "plain_path": {"search_calls": len(groups), "ms_wall": round(plain_ms, 2),
                           "ms_stream": round(float(ev[0]), 2),
                           "qps": round(nq / (plain_ms / 1e3), 1)},
            "p50_ms_in_batch": round(float(np.percentile(svc_ms, 50)), 4),
            "p99_ms_in_batch": round(float(np.percentile(svc_ms, 99)), 4),
            "flagged_queries": int(((stats[:, 5] & 3) != 0).sum()),
        },
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                     "algorithmic_bytes_per_launch": round(bytes_launch),
                     "kernel_ms": round(float(launch_ms.mean()), 4), "note": "one graph replay (all classes)"},
        "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=0, help="base vectors (0: 1,000,000; 10,000,000 for serve)")
    ap.add_argument("--nq", type=int, default=0, help="queries (0: 10,000; 20,000 for gist)")
    ap.add_argument("--latency-queries", type=int, default=2000)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall time of the oracle's throughput leg (Algorithm 1's leg takes half of it)")
    ap.add_argument("--cpu-latency-queries", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--M", type=int, default=0, help="time this walker count only (0: sweep)")
    ap.add_argument("--L", type=int, default=0, help="with --M, time this L (0: sweep)")
    ap.add_argument("--sync", choices=["all", "adaptive", "bsp", "static8"], default="all",
                    help="schedules to sweep: all = adaptive at every M and M = 2 merging after every step")
    ap.add_argument("--sweep-json", default="")
    ap.add_argument("--order", choices=["none", "degree", "bfs"], default="bfs",
                    help="vertex renumbering of the SIFT-shaped index (setup, not timed)")
    ap.add_argument("--workload", choices=["sift", "deep", "gist", "serve"], default="sift")
    ap.add_argument("--serve-M", type=int, default=1, help="walkers per served request")
    ap.add_argument("--serve-sync", choices=["adaptive", "bsp", "static8"], default="adaptive",
                    help="schedule of the served requests (bsp with --serve-M 2: two walkers in one wavefront)")
    ap.add_argument("--serve-slots", type=int, default=16, help="server micro-batch slots")
    ap.add_argument("--serve-graph", choices=["exact", "partition"], default="exact",
                    help="10M graph candidates: exact kNN (matrix cores, row chunks) or overlapping partitions")
    ap.add_argument("--rates", default="10000,50000,100000,200000,300000,400000,500000",
                    help="Poisson arrival rates to replay")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after timing, run a plain elementwise copy of this many MiB (read and written "
                         "once) so that a profiler run can scale its byte counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the search shards by query across GPUs with no exchange "
              "(see the design notes), and no multi-GPU figure is produced here.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2201_13007_amd import binding as B
    from paper_2201_13007_amd import synth

    assert torch.cuda.is_available(), "no GPU"
    B.lib()
    dev = torch.device("cuda:0")
    if args.nq <= 0:
        args.nq = 20_000 if args.workload == "gist" else 10_000
    if args.n <= 0:
        args.n = 10_000_000 if args.workload == "serve" else 1_000_000
    if args.workload == "deep":
        return deep_main(args, torch, B, synth, dev)
    if args.workload == "gist":
        return gist_main(args, torch, B, synth, dev)
    if args.workload == "serve":
        return serve_main(args, torch, B, synth, dev)

    t0 = time.time()
    w = synth.sift_like(n=args.n, nq=args.nq)
    log(f"data {w.name}: {w.base.shape} + {w.queries.shape} queries in {time.time() - t0:.1f}s")
    base = torch.from_numpy(w.base).to(dev)
    queries = torch.from_numpy(w.queries).to(dev)
    k = w.k

    t0 = time.time()
    adj, entry, ginfo = B.build_graph(base, w.graph_knn, w.graph_R, w.graph_prune, w.graph_repair, keep_local=1)
    torch.cuda.synchronize()
    t_graph = time.time() - t0
    deg = (adj >= 0).sum(1).float()
    log(f"graph built in {t_graph:.1f}s: entry {entry}, mean degree {deg.mean().item():.2f}, {ginfo}")

    t0 = time.time()
    gt, _ = B.knn(base, queries, k)
    torch.cuda.synchronize()
    log(f"ground truth in {time.time() - t0:.2f}s")

    perm = None
    if args.order != "none":
        t0 = time.time()
        base, adj, entry, perm = B.reorder(base, adj, entry, args.order)
        log(f"renumbered ({args.order} order) in {time.time() - t0:.1f}s")
    ix = B.Index(base, adj, entry, metric=w.metric, id_map=perm)
    int_range = ix.integer_range
    log(f"integer range of the vectors: {int_range}")
    params = {}

    def run(M, L, stats=False, q=queries, out=None, sync="adaptive"):
        p = params.get((M, L, sync))
        if p is None:
            p = params[(M, L, sync)] = B.make_params(**SYNCS[sync])
        return ix.search(q, k, L, M, params=p, stats=stats, out=out)

    def time_launches(M, L, reps, sync="adaptive"):
        out = run(M, L, sync=sync)
        out = (out.ids, out.dists, None)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in evs:
            a.record()
            run(M, L, out=out, sync=sync)
            b.record()
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in evs]

    # ---------------------------------------------------------------- operating points
    # candidates: the adaptive schedule at every M, and two walkers merging after every
    # local step (Top-2, which the single-worker kernel runs in one wavefront)
    sweep = []
    Ms = [args.M] if args.M else M_SWEEP
    cands = [(Mx, sx) for Mx in Ms for sx in (["adaptive"] if args.sync == "all" else [args.sync])]
    if args.sync == "all" and (not args.M or args.M == 2):
        cands.append((2, "bsp"))
    best = None
    for M, sync in cands:
        Ls = [args.L] if args.L else L_SWEEP
        for L in Ls:
            r = run(M, L, stats=True, sync=sync)
            rec = recall_at_k(r.ids, gt, k).mean().item()
            ms = sorted(time_launches(M, L, 3, sync))[1]
            st = r.stats[:, :6].double().mean(0).tolist()
            row = {"M": M, "sync": sync, "L": L, "recall": round(rec, 5), "ms": round(ms, 3), "qps": round(args.nq / ms * 1e3),
                   "dist_comps": round(st[3], 1), "expansions": round(st[2], 1), "substeps": round(st[1], 1),
                   "spilled": float((r.stats[:, 5] & 4 != 0).float().mean().item()),
                   "flagged": int((r.stats[:, 5] & 3 != 0).sum().item())}
            sweep.append(row)
            log(f"M={M:2d} {sync:8s} L={L:4d} recall={rec:.4f} {ms:8.3f} ms/batch qps={row['qps']:>9} "
                f"D={row['dist_comps']:.0f} E={row['expansions']:.0f} sub={row['substeps']:.0f} "
                f"spill={row['spilled']:.2f} flagged={row['flagged']}")
            if rec >= TARGET:
                if best is None or row["qps"] > best["qps"]:
                    best = row
                break
    if args.sweep_json:
        with open(args.sweep_json, "w") as f:
            json.dump(sweep, f, indent=1)
    reached = best is not None
    if not reached:
        best = max(sweep, key=lambda r: (r["recall"], r["qps"]))
        log(f"recall {TARGET} not reached; timing the best-recall point {best}")
    M, L, SYNC = best["M"], best["L"], best["sync"]

    # ---------------------------------------------------------------- timed region
    r = run(M, L, stats=True, sync=SYNC)
    torch.cuda.synchronize()
    stats = r.stats.cpu().numpy()
    recall = recall_at_k(r.ids, gt, k).mean().item()
    out = (torch.empty_like(r.ids), torch.empty_like(r.dists), None)
    for _ in range(args.warmup):
        run(M, L, out=out, sync=SYNC)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for a, b in evs:
        a.record()
        run(M, L, out=out, sync=SYNC)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    launch_ms = np.array([a.elapsed_time(b) for a, b in evs])
    ms_per_step = wall * 1e3 / args.steps
    qps = args.nq / (ms_per_step / 1e3)
    log(f"timed M={M} {SYNC} L={L}: {ms_per_step:.3f} ms/step, kernel {launch_ms.mean():.3f} ms, QPS {qps:,.0f}")

    # in-batch service time of each query (device real-time counter, 100 MHz)
    t = stats.view(np.int64)[:, 3:5]
    svc_ms = (t[:, 1] - t[:, 0]) / 1e5
    if args.copy_calibration_mib > 0:
        src = torch.ones(args.copy_calibration_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log(f"copy calibration: 3 x {args.copy_calibration_mib} MiB read + written")

    # ---------------------------------------------------------------- batch-1 latency
    # one query per launch, host wall time: every M's operating point (the smallest swept L
    # at the recall target) on a short sample, then the best-p50 point on the full sample
    nl = min(args.latency_queries, args.nq)
    one = (torch.empty((1, k), dtype=torch.int32, device=dev), torch.empty((1, k), dtype=torch.float32, device=dev),
           None)

    def batch1(Mx, Lx, count, sync="adaptive"):
        for i in range(min(20, count)):
            run(Mx, Lx, q=queries[i:i + 1], out=one, sync=sync)
        torch.cuda.synchronize()
        lat = []
        for i in range(count):
            q1 = queries[i:i + 1]
            s0 = time.perf_counter()
            run(Mx, Lx, q=q1, out=one, sync=sync)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - s0) * 1e3)
        return np.array(lat) if lat else np.array([float("nan")])

    # candidates: every M at its adaptive operating point, and for the latency widths
    # M = 8, 16 the other schedules of the paper at their own smallest L reaching the target
    # (merging after every local step is Top-M; within one workgroup a merge is cheap)
    ops = {(s["M"], s["sync"]): s["L"] for s in sweep if s["recall"] >= TARGET} if reached else {(M, SYNC): L}
    op_recall = {(s["M"], s["sync"]): s["recall"] for s in sweep if s["recall"] >= TARGET}
    if reached and nl > 0 and not args.M and args.sync == "all":
        for Mx in (8, 16):
            for sync in ("bsp", "static8"):
                for Lx in L_SWEEP:
                    rec = recall_at_k(run(Mx, Lx, sync=sync).ids, gt, k).mean().item()
                    if rec >= TARGET:
                        ops[(Mx, sync)] = Lx
                        op_recall[(Mx, sync)] = round(rec, 5)
                        log(f"operating point M={Mx} {sync}: L={Lx} recall {rec:.4f}")
                        break
    lat_by_M = {}
    if nl > 0:
        for (Mx, sync), Lx in sorted(ops.items()):
            a = batch1(Mx, Lx, min(300, nl), sync)
            key = str(Mx) if sync == "adaptive" else f"{Mx}-{sync}"
            lat_by_M[key] = {"M": Mx, "sync": sync, "L": Lx, "recall@10": op_recall.get((Mx, sync)),
                             "p50_ms": round(float(np.percentile(a, 50)), 4),
                             "p99_ms": round(float(np.percentile(a, 99)), 4), "queries": len(a)}
            log(f"batch-1 latency sample M={Mx} {sync} L={Lx}: p50 {lat_by_M[key]['p50_ms']:.3f} ms")
    best_key = min(lat_by_M, key=lambda c: lat_by_M[c]["p50_ms"]) if lat_by_M else None
    Mlat, sync_lat = (lat_by_M[best_key]["M"], lat_by_M[best_key]["sync"]) if best_key else (M, SYNC)
    Llat = ops.get((Mlat, sync_lat), L)
    lat = batch1(Mlat, Llat, nl, sync_lat)
    log(f"batch-1 latency M={Mlat} {sync_lat} L={Llat}: p50 {np.percentile(lat, 50):.3f} ms, "
        f"p99 {np.percentile(lat, 99):.3f} ms")

    # ---------------------------------------------------------------- roofline
    d, R = w.base.shape[1], w.graph_R
    D = stats[:, 3].astype(np.float64)
    E = stats[:, 2].astype(np.float64)
    bytes_launch = float((D * d * 4 + E * R * 4 + d * 4 + k * 8).sum())
    achieved = bytes_launch / (launch_ms.mean() / 1e3) / 1e9
    workload_key = f"sift-like-{args.n}x{d}-nq{args.nq}-M{M}-{SYNC}-L{L}-order-{args.order}"
    tr = load_traffic(workload_key)
    gc = B.gather_ceiling(base)
    log(f"gather ceiling: {gc['GBs']:.0f} GB/s for random {gc['row_bytes']}-byte rows")
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": tr["bytes_per_launch"] if tr else None,
                "algorithmic_bytes_per_launch": round(bytes_launch),
                "kernel_ms": round(float(launch_ms.mean()), 4),
                "gather_ceiling_GBs": round(gc["GBs"], 1),
                "frac_of_gather_ceiling": round(achieved / gc["GBs"], 4)}

    # ---------------------------------------------------------------- CPU oracle baseline
    cpu = None
    if not args.no_cpu:
        cpu = cpu_oracle(w, base.cpu().numpy(), adj.cpu().numpy(), entry,
                         perm.cpu().numpy() if perm is not None else None, gt.cpu().numpy(), r.ids.cpu().numpy(), k,
                         (M, L, SYNCS[SYNC]), args.cpu_seconds, args.cpu_latency_queries,
                         bfis_L=ops.get((1, "adaptive")), lockstep=(Mlat, Llat, SYNCS[sync_lat]))

    res = {
        "metric": "QPS and p50/p99 latency at recall@10=0.99, 1M×128 SIFT-shaped, 1 GPU",
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if int_range else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"sift-like {args.n}x{d} (256-component mixture, sigma 20, 0..255), {args.nq} queries, k={k}",
            "accumulation": (f"float32, exact: the vectors and queries are integers in {list(int_range)}, so every partial "
                             f"sum is an integer below 2^24" if int_range else "double, rounded once to float32"),
            "graph": f"exact 64-NN, relative-neighbourhood prune to R={R}, repair (keep_local 1), medoid entry",
            "graph_build_s": round(t_graph, 1),
            "vertex_order": args.order,
            "M": M, "L": L, **SYNCS[SYNC],
            "recall@10": round(recall, 5), "target_reached": reached,
            "storage": "f32 vectors, int32 adjacency",
            "p50_ms_batch1": round(float(np.percentile(lat, 50)), 4),
            "p99_ms_batch1": round(float(np.percentile(lat, 99)), 4),
            "batch1_point": {"M": Mlat, "L": Llat, "sync": sync_lat, "recall@10": op_recall.get((Mlat, sync_lat)),
                             "queries": nl},
            "batch1_by_M": {str(m): v for m, v in sorted(lat_by_M.items())},
            "p50_ms_in_batch": round(float(np.percentile(svc_ms, 50)), 4),
            "p99_ms_in_batch": round(float(np.percentile(svc_ms, 99)), 4),
            "flagged_queries": int(((stats[:, 5] & 3) != 0).sum()),
            "dist_comps_per_query": round(float(D.mean()), 1),
            "expansions_per_query": round(float(E.mean()), 1),
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
