"""The GPU-vs-oracle comparison helper (tests/parity.py), exercised on the CPU with
results written by hand: a difference is accepted only where the oracle's trajectory
decided between keys within the tolerance, and only if the other list is itself valid."""
import numpy as np
import pytest

import parity


def path_graph(coords):
    n = len(coords)
    base = np.array(coords, np.float32)[:, None]
    adj = np.full((n, 2), -1, np.int32)
    for i in range(n):
        nb = [j for j in (i - 1, i + 1) if 0 <= j < n]
        adj[i, :len(nb)] = nb
    return base, adj


def test_near_tie_divergence_accepted():
    # vertices 1 and 2 are at squared distances 0.25 and 0.25 + 2e-7 from the query
    base, adj = path_graph([0.0, 1.0, 2.0000002, 3.0, 5.0, 8.0])
    q = np.array([[1.5]], np.float32)
    e = parity.oracle_search(base, adj, 0, q, 2, 4, 1)
    assert e[0][0].tolist() == [1, 2]
    assert e[3].summary["min_gap"][0] <= parity.RTOL
    # another implementation whose rounding put vertex 2 first
    gpu = (np.array([[2, 1]], np.int32), np.array([[0.25, np.float32(0.25000003)]], np.float32), None)
    acc = parity.compare(gpu, e, exact=False, base=base, queries=q)
    assert acc == [0]
    # the same difference is a failure when the data are integers (exact distances)
    with pytest.raises(AssertionError, match="beyond a near tie"):
        parity.compare(gpu, e, exact=True)
    # and when the other list is not valid (not sorted by key)
    bad = (np.array([[2, 1]], np.int32), np.array([[0.25000003, 0.25]], np.float32), None)
    with pytest.raises(AssertionError, match="beyond a near tie"):
        parity.compare(bad, e, exact=False, base=base, queries=q)


def test_divergence_without_near_tie_rejected():
    base, adj = path_graph([0.0, 1.0, 2.0, 3.0, 5.0, 8.0])
    q = np.array([[0.9]], np.float32)
    e = parity.oracle_search(base, adj, 0, q, 2, 4, 1)
    assert e[0][0].tolist() == [1, 0]
    assert e[3].summary["min_gap"][0] > parity.RTOL
    gpu = (np.array([[1, 2]], np.int32), np.array([[0.01, 1.21]], np.float32), None)
    with pytest.raises(AssertionError, match="smallest key gap"):
        parity.compare(gpu, e, exact=False, base=base, queries=q)


def test_counters_and_distances_checked():
    base, adj = path_graph([0.0, 1.0, 2.0, 3.0, 5.0, 8.0])
    q = np.array([[2.6]], np.float32)
    e = parity.oracle_search(base, adj, 0, q, 2, 4, 1)
    st = np.zeros((1, 10), np.int32)
    for j, name in enumerate(parity.COUNTERS):
        st[0, j] = e[2][name][0]
    parity.compare((e[0].copy(), e[1].copy(), st), e, exact=True)
    st[0, 3] += 1
    with pytest.raises(AssertionError, match="dist_comps"):
        parity.compare((e[0].copy(), e[1].copy(), st), e, exact=True)
    d = e[1].copy()
    d[0, 1] = np.nextafter(d[0, 1], np.float32(np.inf))
    with pytest.raises(AssertionError):
        parity.compare((e[0].copy(), d, None), e, exact=True)
    parity.compare((e[0].copy(), d, None), e, exact=False)
