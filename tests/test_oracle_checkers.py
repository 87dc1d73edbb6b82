"""The invariant checkers reject wrong trees.

check_spanning_tree and check_cycle_property pin other results (the cycle
property characterises the unique MST under the key K, Section 2), so each is
shown here to raise on trees that are wrong in the ways a plausible bug would
make them wrong: a heavier reconnecting edge in place of a tree edge, a
repeated edge, a cycle, a missing or extra edge, an orientation or range
error, and weights that are not those of the edges.
"""
import numpy as np
import pytest

import oracle
from paper_2207_00514_amd import workloads as W


def _tree(n=60, dim=2, seed=5, kind="uniform"):
    pts = W.small_random(n, dim, seed, kind)
    return pts, oracle.prim(pts)


def _with(mst, edges, d2=None):
    e = np.ascontiguousarray(np.asarray(edges, np.int32).reshape(-1, 2))
    if d2 is None:
        d2 = mst.d2[: e.shape[0]]
    d2 = np.asarray(d2, np.float32)
    return oracle.MST(e, d2, np.sqrt(d2).astype(np.float32))


def _swap_for_heavier(pts, mst, k):
    """Remove tree edge k and reconnect the two parts with the lightest
    other crossing pair: still a spanning tree, strictly heavier under K."""
    n = pts.shape[0]
    keep = np.delete(mst.edges, k, axis=0)
    par = np.arange(n)

    def find(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x

    for a, b in keep.tolist():
        par[find(a)] = find(b)
    side = np.array([find(i) for i in range(n)])
    D = oracle.pair_d2_matrix(pts)
    removed = tuple(mst.edges[k].tolist())
    best = None
    for u in range(n):
        for v in range(u + 1, n):
            if side[u] != side[v] and (u, v) != removed:
                key = (int(D[u, v].view(np.uint32)), u, v)
                if best is None or key < best:
                    best = key
    u, v = best[1], best[2]
    e = np.vstack([keep, [[u, v]]])
    d2 = np.concatenate([np.delete(mst.d2, k), [D[u, v]]])
    return _with(mst, e, d2)


def test_checkers_accept_the_mst():
    pts, t = _tree()
    oracle.check_spanning_tree(len(pts), t.edges)
    oracle.check_cycle_property(pts, t)


@pytest.mark.parametrize("k", [0, 17, 58])
def test_cycle_check_rejects_a_heavier_reconnecting_edge(k):
    pts, t = _tree()
    bad = _swap_for_heavier(pts, t, k)
    oracle.check_spanning_tree(len(pts), bad.edges)  # still a spanning tree
    with pytest.raises(AssertionError):
        oracle.check_cycle_property(pts, bad)


def test_cycle_check_rejects_a_heavier_edge_under_ties():
    # unit grid: many equal D, so the swap changes only the index tie-break
    pts = W.integer_grid(6, 2)
    t = oracle.prim(pts)
    bad = _swap_for_heavier(pts, t, 3)
    assert np.array_equal(np.sort(bad.d2), np.sort(t.d2))  # same weights, wrong tie-break
    with pytest.raises(AssertionError):
        oracle.check_cycle_property(pts, bad)


def test_cycle_check_rejects_understated_weights():
    pts, t = _tree()
    d2 = t.d2.copy()
    d2[-1] = d2[0]  # claims the heaviest edge is as light as the lightest
    with pytest.raises(AssertionError):
        oracle.check_cycle_property(pts, _with(t, t.edges, d2))


def test_cycle_check_rejects_a_disconnected_edge_set():
    pts, t = _tree()
    e = t.edges.copy()
    e[-1] = e[0]  # repeated edge: n - 1 edges, one component fewer joined
    with pytest.raises(AssertionError):
        oracle.check_cycle_property(pts, _with(t, e, t.d2))


def test_spanning_check_rejects_a_repeated_edge():
    pts, t = _tree()
    e = t.edges.copy()
    e[5] = e[4]
    with pytest.raises(AssertionError):
        oracle.check_spanning_tree(len(pts), e)


def test_spanning_check_rejects_a_cycle():
    n = 6
    e = np.array([[0, 1], [1, 2], [0, 2], [3, 4], [4, 5]], np.int32)  # triangle, {3,4,5} cut off
    with pytest.raises(AssertionError):
        oracle.check_spanning_tree(n, e)


def test_spanning_check_rejects_wrong_counts_orientation_and_range():
    pts, t = _tree()
    n = len(pts)
    with pytest.raises(AssertionError):
        oracle.check_spanning_tree(n, t.edges[:-1])
    with pytest.raises(AssertionError):
        oracle.check_spanning_tree(n, np.vstack([t.edges, [[0, n - 1]]]))
    flipped = t.edges.copy()
    flipped[3] = flipped[3][::-1]
    with pytest.raises(AssertionError):
        oracle.check_spanning_tree(n, flipped)
    out = t.edges.copy()
    out[7, 1] = n
    with pytest.raises(AssertionError):
        oracle.check_spanning_tree(n, out)


def test_mreach_cycle_check_rejects_a_heavier_edge():
    pts = W.small_random(50, 3, 9, "uniform")
    core2 = oracle.core_bruteforce(pts, 3)
    t = oracle.prim_mreach(pts, core2)
    oracle.check_cycle_property(pts, t, core2)
    # a tree that is the EMST, not the mutual-reachability MST: its weights
    # under M are replaced by M so only its edge choice is wrong
    e = oracle.prim(pts).edges
    M = np.maximum(np.maximum(oracle.pair_d2_matrix(pts), core2[:, None]), core2[None, :]).astype(np.float32)
    alt = _with(t, e, M[e[:, 0], e[:, 1]])
    assert set(map(tuple, e.tolist())) != set(map(tuple, t.edges.tolist()))
    oracle.check_spanning_tree(len(pts), alt.edges)
    with pytest.raises(AssertionError):
        oracle.check_cycle_property(pts, alt, core2)
