"""GPU parity for vertex renumbering (sa_graph_order, sa_permute_rows, sa_permute_graph,
sa_index_set_id_map): orders and permuted arrays bit-exact against the oracle, and a
search of the renumbered index equal to the oracle's search of the renumbered graph
with its ids mapped back."""
import numpy as np
import pytest

import oracle
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
def sift():
    w = synth.sift_like(n=6000, nq=50)
    adj, entry, _ = oracle.build_graph(w.base, 32, 24, "rng", do_repair=True)
    return w, adj, entry


@pytest.mark.parametrize("mode", ["degree", "bfs"])
def test_order_and_permutation_match_oracle(B, sift, mode):
    w, adj, entry = sift
    print(f"case: graph order {mode} sift-6000", flush=True)
    perm = B.graph_order(dev(adj), entry, mode)
    want = oracle.graph_order(adj, entry, mode)
    np.testing.assert_array_equal(host(perm), want)
    b2, a2, e2 = oracle.permute(w.base, adj, entry, want)
    np.testing.assert_array_equal(host(B.permute_rows(dev(w.base), perm)), b2)
    ga2, inv = B.permute_graph(dev(adj), perm)
    np.testing.assert_array_equal(host(ga2), a2)
    assert int(host(inv)[entry]) == e2


@pytest.mark.parametrize("M", [1, 4])
def test_renumbered_search_matches_oracle(B, sift, M):
    w, adj, entry = sift
    base2, adj2, entry2, perm = B.reorder(dev(w.base), dev(adj), entry, "bfs")
    ph = host(perm)
    b2, a2, e2 = oracle.permute(w.base, adj, entry, ph)
    assert e2 == entry2
    print(f"case: renumbered search bfs M={M}", flush=True)
    ix = B.Index(base2, adj2, entry2, id_map=perm)
    r = ix.search(dev(w.queries), 10, 96, M, stats=True)
    eids, ed, est = oracle.speedann(b2, a2, e2, w.queries, 10, 96, M)
    want = np.where(eids >= 0, ph[np.maximum(eids, 0)], -1)
    np.testing.assert_array_equal(host(r.ids), want)
    np.testing.assert_array_equal(host(r.dists), ed)       # integer data: exact
    np.testing.assert_array_equal(host(r.stats)[:, 3], est["dist_comps"])


def test_renumbered_batch_and_rerank(B, sift):
    w, adj, entry = sift
    base2, adj2, entry2, perm = B.reorder(dev(w.base), dev(adj), entry, "degree")
    ix = B.Index(base2, adj2, entry2, dtype="bf16", id_map=perm)
    q = dev(w.queries)
    L = np.full(50, 64, np.int32)
    L[::3] = 200
    k = np.full(50, 10, np.int32)
    M = np.where(np.arange(50) % 2 == 0, 1, 4).astype(np.int32)
    print("case: renumbered bf16 batch with re-rank", flush=True)
    r = B.Batch(ix, L, k, M, rerank=-1).run(q)
    gi = host(r.ids)
    for i in range(50):
        a = ix.search(q[i:i + 1], 10, int(L[i]), int(M[i]), rerank=-1)
        np.testing.assert_array_equal(gi[i], host(a.ids)[0], err_msg=f"query {i}")
    # ids come back in the original numbering: recompute their distances there
    d = ((w.base[gi[:, 0]] - w.queries) ** 2).sum(1)
    np.testing.assert_allclose(host(r.dists)[:, 0], d, rtol=1e-6)
