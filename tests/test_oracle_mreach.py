"""Pins of the mutual-reachability oracle (Section 4, "Mutual reachability
distance"; Section 3, "Non-Euclidean metrics").

core(u) is the distance to the k_pts-th nearest neighbour counting u itself;
M(u, v) = max(core2(u), core2(v), D(u, v)) in squared terms; the tree is the
MST under (bits(M), min, max).  Pinned here against: numpy brute force
(sorting every row of the D matrix; Kruskal over all pairs), the k_pts = 1
reduction to the Euclidean MST stated by the paper, a closed form on a line,
and the cycle property.  CPU only."""
import numpy as np
import pytest

import oracle
from paper_2207_00514_amd import workloads as W

CLOUDS = [(n, dim, seed, kind)
          for kind in ("uniform", "int", "dup", "outlier")
          for dim in (2, 3)
          for n, seed in ((7, 1), (64, 2), (300, 3))]


def same(a, b):
    return np.array_equal(np.asarray(a).view(np.uint32), np.asarray(b).view(np.uint32))


def same_mst(a, b):
    return np.array_equal(a.edges, b.edges) and same(a.d2, b.d2) and same(a.w, b.w)


@pytest.mark.parametrize("n,dim,seed,kind", CLOUDS)
@pytest.mark.parametrize("k", [1, 2, 3, 6])
def test_core_distances_equal_row_sorts(n, dim, seed, kind, k):
    pts = W.small_random(n, dim, seed, kind)
    if k > n:
        pytest.skip("k_pts > n")
    ref = oracle.core_bruteforce(pts, k)
    assert same(oracle.core_distances(pts, k, "brute"), ref)
    assert same(oracle.core_distances(pts, k, "kd"), ref)


def test_core_distances_k1_is_zero_and_monotone_in_k():
    pts = W.small_random(500, 3, 9, "dup")
    prev = oracle.core_distances(pts, 1)
    assert (prev == 0).all()
    for k in (2, 3, 8, 17, 500):
        cur = oracle.core_distances(pts, k)
        assert (cur >= prev).all()
        prev = cur
    # k = n: the farthest point from each u
    D = oracle.pair_d2_matrix(pts)
    assert same(prev, D.max(axis=1))


def test_core_kd_thread_count_independent():
    pts = W.make("clustered3d_2m", 30_000)
    a = oracle.core_distances(pts, 5, "kd", threads=1)
    b = oracle.core_distances(pts, 5, "kd", threads=8)
    assert same(a, b)
    sub = pts[:2000]
    assert same(oracle.core_distances(sub, 5, "kd", threads=4), oracle.core_bruteforce(sub, 5))


@pytest.mark.parametrize("n,dim,seed,kind", CLOUDS)
def test_k1_reduces_to_the_euclidean_mst(n, dim, seed, kind):
    pts = W.small_random(n, dim, seed, kind)
    core2 = oracle.core_distances(pts, 1)
    assert same_mst(oracle.prim_mreach(pts, core2), oracle.prim(pts))
    assert same_mst(oracle.kdboruvka_mreach(pts, core2), oracle.kdboruvka(pts))


@pytest.mark.parametrize("n,dim,seed,kind", [c for c in CLOUDS if c[0] <= 64])
@pytest.mark.parametrize("k", [2, 3, 5])
def test_prim_mreach_equals_bruteforce_kruskal(n, dim, seed, kind, k):
    pts = W.small_random(n, dim, seed, kind)
    if k > n:
        pytest.skip("k_pts > n")
    core2 = oracle.core_bruteforce(pts, k)
    ref = oracle.kruskal_bruteforce(pts, core2)
    got = oracle.prim_mreach(pts, core2)
    assert same_mst(got, ref)
    oracle.check_spanning_tree(n, got.edges)
    oracle.check_cycle_property(pts, got, core2)


@pytest.mark.parametrize("n,dim,seed,kind", CLOUDS)
@pytest.mark.parametrize("k", [2, 4, 16])
def test_kdboruvka_mreach_equals_prim_mreach(n, dim, seed, kind, k):
    pts = W.small_random(n, dim, seed, kind)
    if k > n:
        pytest.skip("k_pts > n")
    core2 = oracle.core_distances(pts, k)
    a = oracle.prim_mreach(pts, core2)
    b = oracle.kdboruvka_mreach(pts, core2, threads=4)
    assert same_mst(a, b)


def test_kdboruvka_mreach_medium_clouds():
    for n, dim, seed, kind, k in ((3000, 3, 11, "uniform", 4), (3500, 2, 12, "int", 8),
                                  (3000, 3, 13, "outlier", 16)):
        pts = W.small_random(n, dim, seed, kind)
        core2 = oracle.core_distances(pts, k)
        assert same_mst(oracle.kdboruvka_mreach(pts, core2, threads=8), oracle.prim_mreach(pts, core2))


@pytest.mark.parametrize("n", [5, 6, 11, 40])
def test_closed_form_unit_line(n):
    """Points 0, 1, ..., n-1 on a line.  k_pts = 2: every core is 1, so every
    M is max(1, D) and the tree is the chain.  k_pts = 3: interior cores are
    1, the two end cores are 2 (D 4).  Kruskal takes the interior chain at
    M = 1, then among the M = 4 pairs (0, 1) first for vertex 0 and, for
    vertex n-1, (n-3, n-1) before (n-2, n-1) by the smaller index."""
    pts = np.zeros((n, 3), np.float32)
    pts[:, 0] = np.arange(n, dtype=np.float32)
    core2 = oracle.core_distances(pts, 2)
    assert (core2 == 1).all()
    t = oracle.prim_mreach(pts, core2)
    assert t.edges.tolist() == [[i, i + 1] for i in range(n - 1)]
    assert (t.w == 1).all()
    core3 = oracle.core_distances(pts, 3)
    assert core3[0] == 4 and core3[-1] == 4 and (core3[1:-1] == 1).all()
    t3 = oracle.prim_mreach(pts, core3)
    expect = sorted([[i, i + 1] for i in range(1, n - 2)] + [[0, 1], [n - 3, n - 1]],
                    key=lambda e: (4 if e in ([0, 1], [n - 3, n - 1]) else 1, e[0], e[1]))
    assert t3.edges.tolist() == expect
    assert t3.total_weight == float(n + 1)


def test_mreach_weights_dominate_euclidean():
    """M >= D pairwise, so the MST under M weighs at least the EMST, and
    every tree weight is at least both end points' core distances."""
    pts = W.small_random(1500, 3, 21, "uniform")
    for k in (2, 5, 12):
        t, core2 = oracle.mreach_mst(pts, k)
        assert t.total_weight >= oracle.prim(pts).total_weight
        assert (t.d2 >= np.maximum(core2[t.edges[:, 0]], core2[t.edges[:, 1]])).all()
