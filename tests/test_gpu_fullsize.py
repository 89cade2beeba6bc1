"""Full-size checks on the SIFT-shaped 1M x 128 workload (graph built on the GPU).

The configuration bench.py times (breadth-first renumbering, two walkers merging after
every local step, staged, L = 192, k = 10) is compared with the oracle id for id,
distance for distance and counter for counter on all 10,000 queries: the oracle searches
the relabelled graph (the search of a renumbered index is the search of the relabelled
graph) and its ids are mapped back.  The graph build itself is too large for the oracle;
its kNN rows are checked on a sample, and the graph on properties that hold at any size.
Data are integer-valued, so every distance is exact and compared bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2201_13007_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def full():
    from paper_2201_13007_amd import binding as B
    B.lib()
    w = synth.sift_like()
    base = torch.from_numpy(w.base).cuda()
    print("case: full-size graph build 1M x 128", flush=True)
    adj, entry, info = B.build_graph(base, w.graph_knn, w.graph_R, w.graph_prune, w.graph_repair, keep_local=1)
    torch.cuda.synchronize()
    return B, w, base, adj, entry, info


def test_fullsize_knn_rows_sampled(full):
    B, w, base, adj, entry, info = full
    rows = np.random.default_rng(7).choice(w.base.shape[0], 12, replace=False).astype(np.int32)
    eids, ed = oracle.knn_self(w.base, rows, 64)
    # the self-join that graph construction runs (matrix-core path on these integer data)
    print("case: full-size 64-NN self-join, 12 sampled rows checked", flush=True)
    ids, dd, used = B.knn(base, None, 64, exclude_self=True, return_path=True)
    assert used == "mfma"
    ids, dd = ids.cpu().numpy(), dd.cpu().numpy()
    np.testing.assert_array_equal(ids[rows], eids)
    np.testing.assert_array_equal(dd[rows], ed)
    del ids, dd
    # both paths on the sampled rows as separate queries (their own id comes first)
    for path in ("mfma", "scan"):
        print(f"case: full-size exact 65-NN of 12 sampled vertices, path={path}", flush=True)
        gids, gd = B.knn(base, base[torch.from_numpy(rows).long().cuda()], 65, path=path)
        gids, gd = gids.cpu().numpy(), gd.cpu().numpy()
        for i, v in enumerate(rows):
            keep = gids[i] != v
            np.testing.assert_array_equal(gids[i][keep][:64], eids[i])
            np.testing.assert_array_equal(gd[i][keep][:64], ed[i])


def test_fullsize_graph_properties(full):
    B, w, base, adj, entry, info = full
    a = adj.cpu().numpy()
    n, R = a.shape
    assert entry == oracle.medoid(w.base)
    assert info["components"] == 256
    assert ((a >= -1) & (a < n)).all()
    valid = a >= 0
    # padding only at the end of a row, no self loops, no repeated id in a row
    assert (np.diff(valid.astype(np.int8), axis=1) <= 0).all()
    assert not (a == np.arange(n)[:, None]).any()
    srt = np.sort(np.where(valid, a, -1 - np.arange(R)[None, :]), axis=1)
    assert not ((srt[:, 1:] == srt[:, :-1]) & (srt[:, 1:] >= 0)).any()
    cnt, _ = oracle.reachable(a, entry)
    assert cnt == n


@pytest.mark.parametrize("M", [1, 2])
def test_fullsize_search_sampled(full, M):
    B, w, base, adj, entry, info = full
    ix = B.Index(base, adj, entry)
    q = torch.from_numpy(w.queries).cuda()
    print(f"case: full-size search M={M} L=384 all 10000 queries", flush=True)
    r = ix.search(q, 10, 384, M, stats=True, sync="adaptive", rho=0.8, staged=True)
    ids, d, st = r.ids.cpu().numpy(), r.dists.cpu().numpy(), r.stats.cpu().numpy()
    assert (st[:, 5] & 3 == 0).all()
    # sorted by key, distinct, ids in range, no padding (the graph is connected)
    assert (ids >= 0).all() and (ids < w.base.shape[0]).all()
    keys = d.astype(np.float64) * 2**32 + ids
    assert (np.diff(keys, axis=1) > 0).all()
    sample = np.random.default_rng(3).choice(w.queries.shape[0], 60, replace=False)
    # distances equal the oracle's distance of the returned ids
    for qi in sample[:20]:
        for j in range(10):
            assert d[qi, j] == oracle.distance(w.queries[qi], w.base[ids[qi, j]])
    # recall against the oracle's exact kNN of sampled queries, and dominance
    gt, gd = oracle.knn(w.base, w.queries[sample], 10)
    rec = oracle.recall(ids[sample], gt).mean()
    print(f"   sampled recall@10 = {rec:.4f}", flush=True)
    assert rec >= 0.97
    assert (d[sample] >= gd).all()


def test_fullsize_search_renumbered(full):
    # the configuration bench.py times: the index renumbered in breadth-first order,
    # results mapped back to original ids
    B, w, base, adj, entry, info = full
    base2, adj2, entry2, perm = B.reorder(base, adj, entry, "bfs")
    p = perm.cpu().numpy()
    assert np.array_equal(np.sort(p), np.arange(w.base.shape[0]))
    ix = B.Index(base2, adj2, entry2, id_map=perm)
    q = torch.from_numpy(w.queries).cuda()
    print("case: full-size search renumbered (bfs) M=1 L=384 all 10000 queries", flush=True)
    r = ix.search(q, 10, 384, 1, stats=True)
    ids, d, st = r.ids.cpu().numpy(), r.dists.cpu().numpy(), r.stats.cpu().numpy()
    assert (st[:, 5] & 3 == 0).all()
    assert (ids >= 0).all() and (ids < w.base.shape[0]).all()
    sample = np.random.default_rng(4).choice(w.queries.shape[0], 60, replace=False)
    for qi in sample[:20]:
        for j in range(10):
            assert d[qi, j] == oracle.distance(w.queries[qi], w.base[ids[qi, j]])
    gt, gd = oracle.knn(w.base, w.queries[sample], 10)
    rec = oracle.recall(ids[sample], gt).mean()
    print(f"   sampled recall@10 = {rec:.4f}", flush=True)
    assert rec >= 0.97
    assert (d[sample] >= gd).all()


def test_fullsize_bench_config_equals_oracle(full):
    # exactly the timed configuration: renumbered index with an id map, M = 2 merging
    # after every local step, staged, L = 192, k = 10, float32 accumulation (integer data)
    B, w, base, adj, entry, info = full
    base2, adj2, entry2, perm = B.reorder(base, adj, entry, "bfs")
    ix = B.Index(base2, adj2, entry2, id_map=perm)
    assert ix.integer_range is not None
    q = torch.from_numpy(w.queries).cuda()
    print("case: full-size bench configuration M=2 bsp staged L=192, all 10000 queries vs oracle", flush=True)
    r = ix.search(q, 10, 192, 2, stats=True, sync="bsp", staged=True)
    torch.cuda.synchronize()
    ids, d = r.ids.cpu().numpy(), r.dists.cpu().numpy()
    st = r.stats.cpu().numpy()
    assert (st[:, 5] & 3 == 0).all()
    p = perm.cpu().numpy()
    # the oracle's index: the original graph relabelled by the oracle, which must be the
    # renumbered index the GPU holds
    b2, a2, e2 = oracle.permute(w.base, adj.cpu().numpy(), entry, p)
    assert e2 == entry2
    np.testing.assert_array_equal(a2, adj2.cpu().numpy())
    np.testing.assert_array_equal(b2, base2.cpu().numpy())
    eids, ed, est = oracle.speedann(b2, a2, entry2, w.queries, 10, 192, 2, sync="bsp", staged=True)
    eids = np.where(eids >= 0, p[np.maximum(eids, 0)], -1)
    bad = np.nonzero((ids != eids).any(1))[0]
    assert bad.size == 0, f"{bad.size} queries differ, first {bad[:5]}"
    np.testing.assert_array_equal(d, ed)
    for j, name in enumerate(("global_steps", "substeps", "expansions", "dist_comps", "merges")):
        np.testing.assert_array_equal(st[:, j], est[name], err_msg=name)
    gt, _ = B.knn(base, q, 10)
    rec = oracle.recall(ids, gt.cpu().numpy()).mean()
    print(f"   recall@10 = {rec:.4f}", flush=True)
    assert rec >= 0.99
