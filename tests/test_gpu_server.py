"""GPU tests of the serving loop (sa_server_*): every request's result is the one
sa_search gives for it alone (and, on a sample, the oracle's), whatever micro-batch
it was served in, under submit / poll and under a timed replay with overlapping
micro-batches and a workspace budget that splits the load."""
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
def deep():
    w = synth.deep_like(n=8000, nq=160)
    adj, entry, _ = oracle.build_graph(w.base, 32, 24, "rng", do_repair=True, metric="ip")
    rng = np.random.default_rng([2201, 13007, 77])
    k = rng.choice(np.array([1, 10, 20], np.int32), size=160)
    L = np.maximum(rng.integers(32, 300, size=160), k).astype(np.int32)
    M = rng.choice(np.array([1, 2, 4, 8], np.int32), size=160)
    return w, adj, entry, k, L, M


def alone(B, ix, w, k, L, M):
    q = dev(w.queries)
    out = []
    for i in range(len(k)):
        r = ix.search(q[i:i + 1], int(k[i]), int(L[i]), int(M[i]))
        out.append((host(r.ids)[0], host(r.dists)[0]))
    return out


def test_server_submit_poll_equals_alone(B, deep):
    w, adj, entry, k, L, M = deep
    ix = B.Index(dev(w.base), dev(adj), entry, metric="ip", dtype="bf16")
    want = alone(B, ix, w, k, L, M)
    print("case: server submit/poll deep-8k bf16, 160 mixed requests, slots 3, max_batch 16", flush=True)
    srv = B.Server(ix, slots=3, max_batch=16, k_max=20)
    for i in range(len(k)):
        srv.submit(w.queries[i], k[i], L[i], M[i], tag=1000 + i)
    got = {}
    for _ in range(2000):
        for tag, ids, dists, ts, td in srv.poll(64, 2000):
            got[tag] = (ids.copy(), dists.copy(), td - ts)
        if len(got) == len(k):
            break
    assert len(got) == len(k)
    for i in range(len(k)):
        ids, dists, lat = got[1000 + i]
        np.testing.assert_array_equal(ids[:k[i]], want[i][0], err_msg=f"request {i}")
        np.testing.assert_array_equal(dists[:k[i]], want[i][1], err_msg=f"request {i}")
        assert lat > 0
    st = srv.stats()
    assert st["completed"] == len(k) and st["max_batch"] <= 16 and st["batches"] >= len(k) // 16
    srv.close()


def test_server_replay_overlap_and_budget(B, deep):
    w, adj, entry, k, L, M = deep
    ix = B.Index(dev(w.base), dev(adj), entry, metric="ip")
    want = alone(B, ix, w, k, L, M)
    # a budget of a few requests per slot: micro-batches split by memory, not by count
    one = ix.workspace_bytes(1, 20, 1024, 16, B.make_params())
    print(f"case: server replay, 4 slots x {4 * one} bytes, Poisson arrivals 50k/s", flush=True)
    srv = B.Server(ix, slots=4, max_batch=64, k_max=20, workspace_bytes=16 * one)
    rng = np.random.default_rng([2201, 13007, 78])
    arrival = np.cumsum(rng.exponential(1e9 / 50_000, size=len(k))).astype(np.int64)
    ids, dists, lat, wall = srv.replay(w.queries, k, L, M, arrival)
    for i in range(len(k)):
        np.testing.assert_array_equal(ids[i, :k[i]], want[i][0], err_msg=f"request {i}")
        np.testing.assert_array_equal(dists[i, :k[i]], want[i][1], err_msg=f"request {i}")
    assert (lat > 0).all() and wall > 0
    st = srv.stats()
    assert st["completed"] == len(k)
    srv.close()


def test_server_matches_oracle_sample(B, deep):
    w, adj, entry, k, L, M = deep
    ix = B.Index(dev(w.base), dev(adj), entry, metric="ip")
    srv = B.Server(ix, slots=2, max_batch=8, k_max=20)
    n = 24
    print("case: server vs oracle, 24 requests burst", flush=True)
    ids, dists, lat, wall = srv.replay(w.queries[:n], k[:n], L[:n], M[:n], np.zeros(n, np.int64))
    for i in range(n):
        ki = int(k[i])
        e = parity.oracle_search(w.base, adj, entry, w.queries[i:i + 1], ki, int(L[i]), int(M[i]), metric="ip")
        parity.compare((ids[i:i + 1, :ki], dists[i:i + 1, :ki], None), e, exact=False, base=w.base,
                       queries=w.queries[i:i + 1], metric="ip", atol=1e-6, label=f"request {i}")
    srv.close()


def test_server_errors(B, deep):
    w, adj, entry, k, L, M = deep
    ix = B.Index(dev(w.base), dev(adj), entry, metric="ip")
    with pytest.raises(B.SpeedAnnError, match="workspace_bytes"):
        B.Server(ix, workspace_bytes=1 << 16)
    srv = B.Server(ix, slots=1, max_batch=4, k_max=10, max_pending=2)
    with pytest.raises(B.SpeedAnnError, match="k_max"):
        srv.submit(w.queries[0], 20, 64, 1, 0)
    srv.close()


def test_server_rerank_bf16(B, deep):
    w, adj, entry, k, L, M = deep
    ix = B.Index(dev(w.base), dev(adj), entry, metric="ip", dtype="bf16")
    q = dev(w.queries)
    n = 64
    want = []
    for i in range(n):
        r = ix.search(q[i:i + 1], int(k[i]), int(L[i]), int(M[i]), rerank=-1)
        want.append((host(r.ids)[0], host(r.dists)[0]))
    print("case: server bf16 with whole-list re-rank, 64 requests at 100k/s", flush=True)
    srv = B.Server(ix, slots=4, max_batch=16, k_max=20, rerank=-1)
    arrival = (np.arange(n) * 10_000).astype(np.int64)
    ids, dists, lat, wall = srv.replay(w.queries[:n], k[:n], L[:n], M[:n], arrival)
    for i in range(n):
        np.testing.assert_array_equal(ids[i, :k[i]], want[i][0], err_msg=f"request {i}")
        np.testing.assert_array_equal(dists[i, :k[i]], want[i][1], err_msg=f"request {i}")
    srv.close()


def test_server_renumbered_index(B, deep):
    # a renumbered index behind the server returns original ids, equal to its own searches
    w, adj, entry, k, L, M = deep
    base2, adj2, entry2, perm = B.reorder(dev(w.base), dev(adj), entry, "bfs")
    ix = B.Index(base2, adj2, entry2, metric="ip", id_map=perm)
    q = dev(w.queries)
    n = 48
    want = [host(ix.search(q[i:i + 1], int(k[i]), int(L[i]), int(M[i])).ids)[0] for i in range(n)]
    print("case: server over a renumbered index, 48 requests", flush=True)
    srv = B.Server(ix, slots=4, max_batch=8, k_max=20)
    ids, dists, lat, wall = srv.replay(w.queries[:n], k[:n], L[:n], M[:n], (np.arange(n) * 20_000).astype(np.int64))
    for i in range(n):
        np.testing.assert_array_equal(ids[i, :k[i]], want[i], err_msg=f"request {i}")
    # original numbering: the distances are those of the original rows
    np.testing.assert_allclose(dists[:n, 0], -(w.base[ids[:n, 0]] * w.queries[:n]).sum(1), rtol=1e-5, atol=1e-6)
    srv.close()
