"""GPU parity for batches with per-query (L, k, M) (sa_batch_*).

Every query of a batch must give exactly what the oracle gives for it alone with its own
(L, k, M): ids and counters exact, distances within 1e-5 relative.  The batch must equal
sa_search per query under every configuration the autotuner can pick, and a HIP graph
captured from a run must replay to the same result.
"""
import numpy as np
import pytest

import oracle
import parity
from paper_2201_13007_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2201_13007_amd import binding
    binding.lib()
    return binding


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def gist():
    # GIST-shaped mix at small size: L log-uniform in [32, 1024], k in {1, 10, 100}, M in
    # {1, 4, 8}, L raised to k where it falls below
    w = synth.gist_like(n=4000, nq=96)
    adj, entry, _ = oracle.build_graph(w.base, 32, 24, "rng", do_repair=True)
    L = np.maximum(w.info["L"], w.info["k"]).astype(np.int32)
    return w, adj, entry, L, w.info["k"].astype(np.int32), w.info["M"].astype(np.int32)


@pytest.mark.parametrize("init", [0, 256])
def test_batch_matches_oracle_per_query(B, gist, init):
    # init = 256: the one-walker classes start in a 256-slot visited table and grow it
    w, adj, entry, L, k, M = gist
    print(f"case: batch gist-4000x960 nq={len(L)} mixed L/k/M ws_hash_init={init}", flush=True)
    ix = B.Index(dev(w.base), dev(adj), entry)
    bt = B.Batch(ix, L, k, M, rho=0.8, ws_hash_init=init)
    r = bt.run(dev(w.queries), stats=True)
    gids, gd, gst = host(r.ids), host(r.dists), host(r.stats)
    if init:
        assert ((gst[M == 1, 5] & 4) != 0).any()
    for q in range(len(L)):
        kq = int(k[q])
        e = parity.oracle_search(w.base, adj, entry, w.queries[q:q + 1], kq, int(L[q]), int(M[q]), rho=0.8)
        parity.compare((gids[q:q + 1, :kq], gd[q:q + 1, :kq], gst[q:q + 1]), e, exact=False, base=w.base,
                       queries=w.queries[q:q + 1], label=f"query {q} (L={L[q]} k={kq} M={M[q]})")
        assert (gids[q, kq:] == -1).all(), "entries past k must stay unwritten"


def test_batch_equals_search_under_every_config(B, gist):
    w, adj, entry, L, k, M = gist
    ix = B.Index(dev(w.base), dev(adj), entry)
    q = dev(w.queries)
    want_ids = np.full((len(L), int(k.max())), -1, np.int32)
    want_d = np.full((len(L), int(k.max())), np.inf, np.float32)
    for i in range(len(L)):
        r = ix.search(q[i:i + 1], int(k[i]), int(L[i]), int(M[i]), rho=0.8)
        want_ids[i, :k[i]] = host(r.ids)[0]
        want_d[i, :k[i]] = host(r.dists)[0]
    bt = B.Batch(ix, L, k, M, rho=0.8)
    for streams in (1, 2, 4, 8):
        for lds in (0, -1, 4096):
            print(f"case: batch config streams={streams} lds_hash_slots={lds}", flush=True)
            bt.set_config(streams, lds)
            r = bt.run(q)
            np.testing.assert_array_equal(host(r.ids), want_ids)
            np.testing.assert_array_equal(host(r.dists), want_d)
    # every candidate the tuner may pick: each class in each of its LDS settings, in both
    # forms (one workgroup per query, persistent), on one stream and on eight
    opts = [bt.class_options(c) for c in range(bt.classes())]
    assert all(o[1] for o in opts)
    for persistent in (False, True):
        for j in range(max(len(o[0]) for o in opts)):
            for c, (vals, _) in enumerate(opts):
                bt.set_class(c, vals[j % len(vals)], persistent)
            for streams in (1, 8):
                print(f"case: batch classes persistent={persistent} lds option {j} streams={streams}", flush=True)
                bt.set_config(streams, 0)   # the stream count (and the default table, set again below)
                for c, (vals, _) in enumerate(opts):
                    bt.set_class(c, vals[j % len(vals)], persistent)
                r = bt.run(q)
                np.testing.assert_array_equal(host(r.ids), want_ids)
                np.testing.assert_array_equal(host(r.dists), want_d)
    with pytest.raises(B.SpeedAnnError, match="room"):
        bt.set_class(0, 777, False)
    print("case: batch tune", flush=True)
    t = bt.tune(q, reps=1)
    assert len(t["classes"]) == bt.classes()
    for c, cands in enumerate(t["classes"]):
        assert len(cands) == 2 * len(opts[c][0])
        assert {(x["lds_hash_slots"], x["persistent"]) for x in cands} == {(v, p) for v in opts[c][0] for p in (0, 1)}
    assert {x["plan"] for x in t["plans"]} == {"per_query", "persistent", "mixed"}
    best = min(t["plans"], key=lambda x: x["ms"])
    assert t["chosen"]["plan"] == best["plan"] and t["chosen"]["streams"] == best["streams"]
    r = bt.run(q)
    np.testing.assert_array_equal(host(r.ids), want_ids)
    d = bt.describe()
    assert sum(c["queries"] for c in d["classes"]) == len(L)
    assert {c["M"] for c in d["classes"]} == set(M.tolist())


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_graph_replay(B, gist, persistent):
    # persistent: every class takes its queries from a device counter, which the last
    # workgroup of each launch sets back to zero; replays and eager runs must keep working
    w, adj, entry, L, k, M = gist
    ix = B.Index(dev(w.base), dev(adj), entry)
    q = dev(w.queries)
    bt = B.Batch(ix, L, k, M, rho=0.8)
    bt.set_config(4, 0)
    for c in range(bt.classes()):
        bt.set_class(c, bt.class_options(c)[0][0], persistent)
    eager = bt.run(q)
    e_ids, e_d = host(eager.ids), host(eager.dists)
    out = bt.outputs()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bt.run(q, out=out)          # warm on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    print(f"case: batch captured in a graph, 3 replays, persistent={persistent}", flush=True)
    with torch.cuda.graph(g):
        bt.run(q, out=out)
    written = np.arange(e_ids.shape[1])[None, :] < k[:, None]   # row q gets its first k[q] entries
    for rep in range(3):
        out[0].fill_(-7)
        out[1].fill_(-7.0)
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(out[0])[written], e_ids[written], err_msg=f"replay {rep}")
        np.testing.assert_array_equal(host(out[1])[written], e_d[written], err_msg=f"replay {rep}")
        assert (host(out[0])[~written] == -7).all()
        # eager work between replays
        again = bt.run(q)
        np.testing.assert_array_equal(host(again.ids), e_ids)


@pytest.mark.parametrize("sync", ["adaptive", "bsp"])
def test_batch_one_class_and_sift(B, sync):
    # bsp: two walkers merging after every step, which run in one wavefront
    w = synth.sift_like(n=5000, nq=40)
    adj, entry, _ = oracle.build_graph(w.base, 32, 24, "rng", do_repair=True)
    L = np.full(40, 96, np.int32)
    k = np.full(40, 10, np.int32)
    M = np.full(40, 2, np.int32)
    ix = B.Index(dev(w.base), dev(adj), entry)
    bt = B.Batch(ix, L, k, M, sync=sync)
    eids, ed, est = oracle.speedann(w.base, adj, entry, w.queries, 10, 96, 2, sync=sync)
    vals, _ = bt.class_options(0)
    # bsp: the packed wavefront (default) and, with an LDS table, one wavefront per walker
    assert len(vals) >= 2
    for lds in vals:
        for persistent in (False, True):
            print(f"case: batch sift-5000 one class M=2 L=96 {sync} lds={lds} persistent={persistent}", flush=True)
            bt.set_class(0, lds, persistent)
            r = bt.run(dev(w.queries), stats=True)
            np.testing.assert_array_equal(host(r.ids), eids)
            np.testing.assert_array_equal(host(r.dists), ed)   # integer data: exact
            for j, name in enumerate(["global_steps", "substeps", "expansions", "dist_comps", "merges"]):
                np.testing.assert_array_equal(host(r.stats)[:, j], est[name], err_msg=name)


def test_batch_errors(B, gist):
    w, adj, entry, L, k, M = gist
    ix = B.Index(dev(w.base), dev(adj), entry)
    bad = k.copy()
    bad[5] = L[5] + 1
    with pytest.raises(B.SpeedAnnError, match="query 5"):
        B.Batch(ix, L, bad, M)
    bt = B.Batch(ix, L, k, M)
    with pytest.raises(B.SpeedAnnError, match="different number"):
        bt.run(dev(w.queries[:10]))


def test_knn_gist_shaped(B):
    # the exact kNN behind the GIST-shaped ground truth and graph: d = 960, k = 100
    w = synth.gist_like(n=3000, nq=17)
    print("case: knn gist-3000x960 k=100", flush=True)
    ids, d = B.knn(dev(w.base), dev(w.queries), 100)
    eids, ed = oracle.knn(w.base, w.queries, 100)
    np.testing.assert_array_equal(host(ids), eids)
    np.testing.assert_allclose(host(d), ed, rtol=1e-6)


def test_chunked_graph_build_equals_library(B):
    # bench.py builds the GIST-shaped graph in logged row chunks; it must equal sa_build_graph
    import bench
    w = synth.gist_like(n=5000, nq=1)
    base = dev(w.base)
    print("case: chunked graph build gist-5000x960 vs sa_build_graph", flush=True)
    adj, entry, info = B.build_graph(base, 64, 32, "rng", True, keep_local=1)
    adj2, entry2, info2 = bench.build_graph_logged(torch, B, base, 64, 32, "rng", chunk=1500)
    assert entry == entry2 and info == info2
    np.testing.assert_array_equal(host(adj), host(adj2))


@pytest.mark.parametrize("rr", [-1, 30])
def test_batch_rerank_bf16(B, rr):
    # a re-ranked batch over bf16 codes equals sa_search with the same re-rank, per query
    w = synth.deep_like(n=6000, nq=48)
    adj, entry, _ = oracle.build_graph(w.base, 32, 24, "rng", do_repair=True, metric="ip")
    rng = np.random.default_rng([2201, 13007, 79])
    k = rng.choice(np.array([1, 10, 20], np.int32), size=48)
    L = np.maximum(rng.integers(32, 200, size=48), 30).astype(np.int32)
    M = rng.choice(np.array([1, 4], np.int32), size=48)
    ix = B.Index(dev(w.base), dev(adj), entry, metric="ip", dtype="bf16")
    q = dev(w.queries)
    print(f"case: batch bf16 deep-6000 rerank={rr}", flush=True)
    bt = B.Batch(ix, L, k, M, rerank=rr)
    r = bt.run(q)
    gi, gd = host(r.ids), host(r.dists)
    for i in range(48):
        a = ix.search(q[i:i + 1], int(k[i]), int(L[i]), int(M[i]), rerank=rr)
        np.testing.assert_array_equal(gi[i, :k[i]], host(a.ids)[0], err_msg=f"query {i}")
        np.testing.assert_array_equal(gd[i, :k[i]], host(a.dists)[0], err_msg=f"query {i}")
