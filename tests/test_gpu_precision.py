"""GPU parity for reduced-precision vector storage (bf16, fp8 e4m3 with per-vector scales)
and for the exact float32 re-rank of the final list.

The oracle quantizes from the format definitions; the codes must match bit for bit.  A
search over stored codes must equal the oracle's search over the dequantized vectors
(ids and counters exact, distances within 1e-5 relative); a re-ranked search must equal
the oracle's final list re-ranked on the float32 vectors.
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
def deep():
    w = synth.deep_like(n=8000, nq=60)
    adj, entry, _ = oracle.build_graph(w.base, 32, 24, "rng", do_repair=True, metric="ip")
    return w, adj, entry


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_quantize_codes_match_oracle(B, dtype):
    w = synth.deep_like(n=3000, nq=1)
    x = w.base.copy()
    x[0] = 0.0            # zero vector: scale 1, codes 0
    x[1] *= 1e4           # large and small magnitudes
    x[2] *= 1e-4
    x[3, ::2] = -x[3, ::2]
    print(f"case: quantize {dtype} 3000x96", flush=True)
    codes, scale = B.quantize(dev(x), dtype)
    ec, es = oracle.quantize(x, dtype)
    got = host(codes).view(np.uint16 if dtype == "bf16" else np.uint8)
    np.testing.assert_array_equal(got, ec)
    np.testing.assert_array_equal(host(scale), es)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
@pytest.mark.parametrize("M", [1, 4])
def test_search_over_codes(B, deep, dtype, M):
    w, adj, entry = deep
    codes, scale = oracle.quantize(w.base, dtype)
    deq = oracle.dequantize(codes, scale, dtype)
    print(f"case: search deep-8k ip {dtype} M={M} L=64", flush=True)
    ix = B.Index(dev(w.base), dev(adj), entry, metric="ip", dtype=dtype)
    r = ix.search(dev(w.queries), 10, 64, M, stats=True, rho=0.9)
    e = parity.oracle_search(deq, adj, entry, w.queries, 10, 64, M, rho=0.9, metric="ip")
    acc = parity.compare((host(r.ids), host(r.dists), host(r.stats)), e, exact=False, base=deq, queries=w.queries,
                         metric="ip", atol=1e-6, label=f"{dtype} M={M}")
    if acc:
        print(f"   {len(acc)} queries parted at a near tie: {acc[:10]}", flush=True)


def test_search_over_codes_l2_integer(B):
    # integer data: bf16 holds 0..255 exactly, so the search equals the float32 search bit for bit
    w = synth.sift_like(n=6000, nq=40)
    adj, entry, _ = oracle.build_graph(w.base, 32, 24, "rng", do_repair=True)
    print("case: search sift-6k l2 bf16 M=2 L=96", flush=True)
    ix = B.Index(dev(w.base), dev(adj), entry, dtype="bf16")
    r = ix.search(dev(w.queries), 10, 96, 2, stats=True)
    eids, ed, est = oracle.speedann(w.base, adj, entry, w.queries, 10, 96, 2)
    np.testing.assert_array_equal(host(r.ids), eids)
    np.testing.assert_array_equal(host(r.dists), ed)


@pytest.mark.parametrize("dtype", ["f32", "fp8"])
@pytest.mark.parametrize("M,rr", [(1, -1), (1, 20), (4, -1), (8, 30)])
def test_rerank(B, deep, dtype, M, rr):
    w, adj, entry = deep
    L = 64
    if dtype == "f32":
        searched = w.base
    else:
        codes, scale = oracle.quantize(w.base, dtype)
        searched = oracle.dequantize(codes, scale, dtype)
    print(f"case: re-rank {dtype} M={M} rerank={rr}", flush=True)
    ix = B.Index(dev(w.base), dev(adj), entry, metric="ip", dtype=dtype)
    r = ix.search(dev(w.queries), 10, L, M, rho=0.9, rerank=rr)
    final, _, _ = oracle.speedann(searched, adj, entry, w.queries, L if rr < 0 else rr, L, M, rho=0.9, metric="ip")
    eids, ed = oracle.rerank(w.base, w.queries, final, 10, metric="ip")
    np.testing.assert_array_equal(host(r.ids), eids)
    np.testing.assert_allclose(host(r.dists), ed, rtol=1e-5, atol=1e-6)
    # the workspace is zero again after the re-rank
    assert int(ix.workspace(0).count_nonzero().item()) == 0


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_rerank_after_table_growth(B, deep, dtype):
    # one walker starting in a 128-slot visited table grows it several times; the re-rank
    # list at the end of the slot list must come through unchanged
    w, adj, entry = deep
    L = 64
    searched = w.base if dtype == "f32" else oracle.dequantize(*oracle.quantize(w.base, dtype), dtype)
    print(f"case: re-rank {dtype} after visited-table growth", flush=True)
    ix = B.Index(dev(w.base), dev(adj), entry, metric="ip", dtype=dtype)
    r = ix.search(dev(w.queries), 10, L, 1, rho=0.9, rerank=-1, ws_hash_init=128, stats=True)
    assert ((host(r.stats)[:, 5] & 4) != 0).all()
    final, _, _ = oracle.speedann(searched, adj, entry, w.queries, L, L, 1, rho=0.9, metric="ip")
    eids, ed = oracle.rerank(w.base, w.queries, final, 10, metric="ip")
    np.testing.assert_array_equal(host(r.ids), eids)
    np.testing.assert_allclose(host(r.dists), ed, rtol=1e-5, atol=1e-6)
    assert int(ix.workspace(0).count_nonzero().item()) == 0


def test_rerank_needs_room_and_vectors(B, deep):
    w, adj, entry = deep
    ix = B.Index(dev(w.base), dev(adj), entry, metric="ip", dtype="fp8")
    with pytest.raises(B.SpeedAnnError, match="8192"):
        ix.search(dev(w.queries[:4]), 10, 64, 1, rerank=-1, ws_hash_slots=4096)
