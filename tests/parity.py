"""Comparison of a GPU search with the oracle's, with a report of where they part.

The result of a graph search is defined by its trajectory (Algorithm 1: which candidate
is expanded next depends on the order of the keys in the list), so two correct
implementations whose distances differ in the last bit can return different ids.  The
bar is therefore:

* integer-valued data (every distance exact in any summation order): ids, distances and
  counters bit for bit;
* float data: ids and counters exactly, distances within `rtol` relative, except for a
  query whose oracle trajectory took a decision between two keys of distinct vertices
  within `rtol` of each other (the oracle's trace records the smallest such gap).  Such a
  query may differ; its GPU list must still be a valid result: sorted by key, distinct
  ids, each distance within `rtol` of the oracle's distance of that id.

A failure message names the first queries that differ, their lists, and the smallest key
gap the oracle saw for each (the step and the two keys), so that a rounding near-tie and a
wrong step are told apart.
"""
import numpy as np

import oracle

RTOL = 1e-5
COUNTERS = ("global_steps", "substeps", "expansions", "dist_comps", "merges")


def oracle_search(base, adj, entry, queries, k, L, M, **kw):
    """oracle.speedann with the decision trace (summary only)."""
    return oracle.search("speedann", base, adj, entry, queries, k, L, M, trace=(0, 0), **kw)


def _gap_text(tr, q):
    s = tr.summary[q]
    if not np.isfinite(s["min_gap"]):
        return "no two keys were ever compared"
    return (f"smallest key gap {s['min_gap']:.3g} after local step {int(s['gap_step'])} between "
            f"({s['gap_dist'][0]!r}, {int(s['gap_id'][0])}) and ({s['gap_dist'][1]!r}, {int(s['gap_id'][1])})")


def compare(gpu, orc, exact, base=None, queries=None, metric="l2", counters=True, rtol=RTOL, atol=0.0,
            label=""):
    """gpu: (ids, dists, stats as the binding returns them, or None); orc: (ids, dists,
    stats, trace) from oracle_search.  base / queries (float data only) let a query that
    parted on a near-tie be checked for validity.  atol: an absolute floor for distances
    near zero (inner products).  Returns the queries accepted as near-tie divergences."""
    gids, gd, gst = gpu
    eids, ed, est, tr = orc
    differ = np.nonzero((gids != eids).any(1))[0]
    accepted = []
    lines = []
    for q in differ:
        tie = (not exact) and tr is not None and tr.summary["min_gap"][q] <= rtol
        if tie and base is not None:
            ok = _valid(gids[q], gd[q], base, queries[q], metric, rtol, atol)
            tie = tie and ok
        if tie:
            accepted.append(int(q))
        else:
            lines.append(f"  query {q}: gpu {gids[q].tolist()} oracle {eids[q].tolist()}; "
                         + (_gap_text(tr, q) if tr is not None else "no trace"))
    assert not lines, f"{label}: {len(lines)} queries differ beyond a near tie:\n" + "\n".join(lines[:5])
    same = np.setdiff1d(np.arange(gids.shape[0]), accepted)
    if exact:
        np.testing.assert_array_equal(gd[same], ed[same], err_msg=label)
    else:
        np.testing.assert_allclose(gd[same], ed[same], rtol=rtol, atol=atol, err_msg=label)
    if counters and gst is not None:
        for j, name in enumerate(COUNTERS):
            np.testing.assert_array_equal(gst[same, j], est[name][same], err_msg=f"{label} {name}")
    return accepted


def _valid(ids, dists, base, q, metric, rtol, atol):
    ok = ids >= 0
    if len(set(ids[ok].tolist())) != int(ok.sum()):
        return False
    keys = list(zip(dists[ok].tolist(), ids[ok].tolist()))
    if keys != sorted(keys):
        return False
    for i, d in zip(ids[ok], dists[ok]):
        want = oracle.distance(q, base[i], metric)
        if abs(d - want) > atol + rtol * abs(want):
            return False
    return True
