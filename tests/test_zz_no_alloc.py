"""sa_search_noalloc (the search with the library's static device workspace, for callers
that cannot allocate) against sa_search with a caller workspace: the same ids, distances
and counters, on two calls in a row, the second with fewer queries, fewer walkers and a
smaller L; and the capacity error."""
import numpy as np
import pytest

import oracle
from paper_2201_13007_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_noalloc_equals_search():
    from paper_2201_13007_amd import binding as B
    B.lib()
    w = synth.sift_like(n=20_000, nq=300)
    adj, entry, _ = oracle.build_graph(w.base, 64, 32, "rng", do_repair=True)
    ix = B.Index(torch.from_numpy(w.base).cuda(), torch.from_numpy(adj).cuda(), entry)
    q_all = torch.from_numpy(w.queries).cuda()
    for nq, L, M, sync in ((300, 192, 2, "bsp"), (37, 96, 1, "adaptive"), (200, 100, 4, "adaptive")):
        print(f"case: noalloc nq={nq} L={L} M={M} {sync}", flush=True)
        q = q_all[:nq].contiguous()
        want = ix.search(q, 10, L, M, stats=True, sync=sync)
        st = torch.empty((nq, B.STATS_BYTES // 4), dtype=torch.int32, device="cuda")
        out = (torch.empty((nq, 10), dtype=torch.int32, device="cuda"),
               torch.empty((nq, 10), dtype=torch.float32, device="cuda"), st)
        got = ix.search_noalloc(q, 10, L, M, out=out, sync=sync)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.ids.cpu().numpy(), want.ids.cpu().numpy())
        np.testing.assert_array_equal(got.dists.cpu().numpy(), want.dists.cpu().numpy())   # integer data: exact
        np.testing.assert_array_equal(got.stats.cpu().numpy()[:, :6], want.stats.cpu().numpy()[:, :6])
    # beyond the 64 MiB array: a clear error, nothing launched
    big = torch.zeros((20_000, 128), dtype=torch.float32, device="cuda")
    with pytest.raises(B.SpeedAnnError, match="scratch"):
        ix.search_noalloc(big, 10, 192, 2, sync="bsp")
