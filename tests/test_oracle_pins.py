"""Pins for the CPU oracle: each test checks it against something other than
itself -- exact arithmetic, closed forms, a textbook algorithm written
independently (Kruskal), a library routine (scipy), the paper's worked
example (Figure 4) and invariants (spanning, cycle property, round bound).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2207_00514_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def same_tree(a, b):
    assert a.edges.shape == b.edges.shape
    np.testing.assert_array_equal(a.edges, b.edges)
    np.testing.assert_array_equal(a.d2.view(np.uint32), b.d2.view(np.uint32))
    np.testing.assert_array_equal(a.w.view(np.uint32), b.w.view(np.uint32))


# ---------------------------------------------------------------------------
# D, the float32 squared distance


def test_sqdist_exact_on_integers(oracle_lib):
    rng = np.random.default_rng(0)
    for dim in (2, 3):
        for _ in range(200):
            a = rng.integers(-1000, 1000, dim).astype(np.float32)
            b = rng.integers(-1000, 1000, dim).astype(np.float32)
            exact = int(sum((int(x) - int(y)) ** 2 for x, y in zip(a, b)))
            assert oracle_lib.sqdist(a, b) == np.float32(exact)


def test_sqdist_symmetric_bitwise(oracle_lib):
    rng = np.random.default_rng(1)
    for dim in (2, 3):
        for _ in range(500):
            a = rng.standard_normal(dim).astype(np.float32)
            b = rng.standard_normal(dim).astype(np.float32)
            assert oracle_lib.sqdist(a, b).view(np.uint32) == oracle_lib.sqdist(b, a).view(np.uint32)


def test_sqdist_within_rounding_bound(oracle_lib):
    # |fl(D) - D_exact| <= (dim + 2) u D_exact + O(u^2), u = 2^-24
    rng = np.random.default_rng(2)
    u = Fraction(1, 2 ** 24)
    for dim in (2, 3):
        for _ in range(300):
            a = rng.random(dim).astype(np.float32)
            b = rng.random(dim).astype(np.float32)
            exact = sum((Fraction(float(x)) - Fraction(float(y))) ** 2 for x, y in zip(a, b))
            got = Fraction(float(oracle_lib.sqdist(a, b)))
            assert abs(got - exact) <= (dim + 3) * u * exact


def test_sqdist_keeps_denormals(oracle_lib):
    a = np.array([1e-20, 0.0, 0.0], np.float32)
    b = np.zeros(3, np.float32)
    d = oracle_lib.sqdist(a, b)
    assert d != 0.0 and d < np.finfo(np.float32).tiny  # a denormal result
    assert d == np.float32(1e-20) * np.float32(1e-20)


def test_sqdist_uses_every_coordinate_and_the_left_to_right_order(oracle_lib):
    # drop-a-term / wrong-order mutations change these exact results
    a = np.array([0.0, 0.0, 3.0], np.float32)
    assert oracle_lib.sqdist(a, np.zeros(3, np.float32)) == 9.0
    # (2^24 + 1 + 1) depends on the order of the float32 additions:
    # s = 2^24; s + 1 -> 2^24 (tie to even); s + 1 -> 2^24
    p = np.array([4096.0, 1.0, 1.0], np.float32)
    assert oracle_lib.sqdist(p, np.zeros(3, np.float32)) == np.float32(2 ** 24)


# ---------------------------------------------------------------------------
# whole-tree results on small inputs


CASES = [(n, dim, seed, kind)
         for kind in ("uniform", "int", "dup", "outlier")
         for dim in (2, 3)
         for n, seed in ((0, 0), (1, 1), (2, 2), (3, 3), (17, 4), (64, 5), (150, 6))]


@pytest.mark.parametrize("n,dim,seed,kind", CASES)
def test_prim_equals_bruteforce_kruskal(oracle_lib, n, dim, seed, kind):
    pts = W.small_random(n, dim, seed, kind)
    a = oracle_lib.prim(pts)
    b = oracle_lib.kruskal_bruteforce(pts)
    same_tree(a, b)
    oracle_lib.check_spanning_tree(n, a.edges)


@pytest.mark.parametrize("n,dim,seed,kind", CASES)
def test_kdboruvka_equals_prim(oracle_lib, n, dim, seed, kind):
    pts = W.small_random(n, dim, seed, kind)
    same_tree(oracle_lib.kdboruvka(pts), oracle_lib.prim(pts))


@pytest.mark.parametrize("seed", range(6))
def test_kdboruvka_equals_prim_medium(oracle_lib, seed):
    dim = 2 + seed % 2
    kind = ("uniform", "int", "dup")[seed % 3]
    pts = W.small_random(1500 + 97 * seed, dim, 100 + seed, kind)
    same_tree(oracle_lib.kdboruvka(pts), oracle_lib.prim(pts))


def test_kdboruvka_threads_do_not_change_the_result(oracle_lib):
    pts = W.small_random(20000, 3, 7, "dup")
    a = oracle_lib.kdboruvka(pts, threads=1)
    b = oracle_lib.kdboruvka(pts, threads=4)
    same_tree(a, b)


def test_prim_matches_scipy_when_weights_are_distinct(oracle_lib):
    from scipy.sparse.csgraph import minimum_spanning_tree
    used = 0
    for seed in range(40):
        for dim in (2, 3):
            pts = W.small_random(100, dim, 200 + seed)
            D = oracle_lib.pair_d2_matrix(pts)
            iu = np.triu_indices(len(pts), 1)
            if len(np.unique(D[iu])) != len(iu[0]) or not (D[iu] > 0).all():
                continue  # float32 ties: the MST under real weights is not unique
            used += 1
            T = minimum_spanning_tree(np.triu(D.astype(np.float64), 1)).tocoo()
            ref = sorted((min(a, b), max(a, b)) for a, b in zip(T.row.tolist(), T.col.tolist()))
            got = sorted(map(tuple, oracle_lib.prim(pts).edges.tolist()))
            assert got == ref
    assert used >= 10


def test_total_weight_close_to_real_euclidean_mst(oracle_lib):
    from scipy.sparse.csgraph import minimum_spanning_tree
    from scipy.spatial.distance import cdist
    pts = W.small_random(400, 3, 11)
    real = minimum_spanning_tree(np.triu(cdist(pts.astype(np.float64), pts.astype(np.float64)), 1)).sum()
    got = oracle_lib.prim(pts).total_weight
    assert abs(got - real) <= 1e-5 * real


def test_cycle_property(oracle_lib):
    for seed, kind in enumerate(("uniform", "int", "dup", "outlier")):
        pts = W.small_random(90, 2 + seed % 2, 300 + seed, kind)
        oracle_lib.check_cycle_property(pts, oracle_lib.kdboruvka(pts))


# ---------------------------------------------------------------------------
# closed forms


def test_identical_points_give_a_star_at_vertex_zero(oracle_lib):
    for n in (2, 5, 300):
        for f in (oracle_lib.prim, oracle_lib.kdboruvka):
            t = f(W.identical(n))
            np.testing.assert_array_equal(t.edges, np.stack([np.zeros(n - 1), np.arange(1, n)], 1))
            assert (t.d2 == 0).all() and (t.w == 0).all()


def _grid_reference(pts):
    """Kruskal over the unit grid edges only, ordered by (min, max): every
    MST edge of a unit integer grid has length 1."""
    n = len(pts)
    index = {tuple(p): i for i, p in enumerate(pts.astype(np.int64).tolist())}
    cand = []
    for i, p in enumerate(pts.astype(np.int64).tolist()):
        for k in range(len(p)):
            q = list(p)
            q[k] += 1
            j = index.get(tuple(q))
            if j is not None:
                cand.append((min(i, j), max(i, j)))
    cand.sort()
    par = list(range(n))

    def find(x):
        while par[x] != x:
            x = par[x]
        return x

    out = []
    for a, b in cand:
        ra, rb = find(a), find(b)
        if ra != rb:
            par[rb] = ra
            out.append((a, b))
    return sorted(out)


@pytest.mark.parametrize("k,dim", [(2, 2), (7, 2), (30, 2), (5, 3), (12, 3)])
def test_integer_grid(oracle_lib, k, dim):
    pts = W.integer_grid(k, dim, seed=k)
    for f in (oracle_lib.prim, oracle_lib.kdboruvka):
        t = f(pts)
        assert (t.d2 == 1.0).all()
        assert t.total_weight == float(k ** dim - 1)
        assert sorted(map(tuple, t.edges.tolist())) == _grid_reference(pts)


def test_collinear_chain(oracle_lib):
    for n in (2, 3, 50, 2000):
        pts = W.collinear(n, 2, seed=n)
        pos = pts[:, 0].astype(np.int64)
        inv = np.argsort(pos)
        ref = sorted((min(a, b), max(a, b)) for a, b in zip(inv[:-1].tolist(), inv[1:].tolist()))
        t = oracle_lib.kdboruvka(pts)
        assert sorted(map(tuple, t.edges.tolist())) == ref
        assert t.total_weight == float(n - 1)


def test_two_far_clusters_have_one_crossing_edge(oracle_lib):
    pts = W.two_clusters(200, 3, seed=3)
    side = pts[:, 0] > 50
    t = oracle_lib.kdboruvka(pts)
    cross = [(u, v) for u, v in t.edges.tolist() if side[u] != side[v]]
    assert len(cross) == 1
    D = oracle_lib.pair_d2_matrix(pts)
    A, B = np.nonzero(~side)[0], np.nonzero(side)[0]
    best = min((int(D[a, b].view(np.uint32)), min(a, b), max(a, b)) for a in A for b in B)
    assert cross[0] == best[1:]


def test_two_points(oracle_lib):
    pts = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]], np.float32)
    t = oracle_lib.prim(pts)
    assert t.edges.tolist() == [[0, 1]] and t.d2[0] == 9.0 and t.w[0] == 3.0


def test_fewer_than_two_points(oracle_lib):
    for n in (0, 1):
        t = oracle_lib.kdboruvka(np.zeros((n, 3), np.float32))
        assert t.edges.shape == (0, 2)


# ---------------------------------------------------------------------------
# round structure of Boruvka (Section 2: at most ceil(log2 n) rounds, every
# round at least halves the number of components)


@pytest.mark.parametrize("n,kind", [(1000, "uniform"), (3000, "int"), (2048, "dup")])
def test_round_bound(oracle_lib, n, kind):
    t = oracle_lib.kdboruvka(W.small_random(n, 3, 9, kind))
    assert 1 <= t.rounds <= math.ceil(math.log2(n))
    c = list(t.comps) + [1]
    assert c[0] == n
    for a, b in zip(c[:-1], c[1:]):
        assert b <= a // 2


# ---------------------------------------------------------------------------
# binary radix tree + label propagation: the paper's Figure 4


def _fig4():
    with open(os.path.join(GOLDEN, "fig4_label_reduction.json")) as f:
        return json.load(f)


def _figure_ranges(g):
    """Leaf range of each named internal node of the figure's tree."""
    rng = {}

    def span(ref):
        if ref.startswith("L"):
            i = int(ref[1:])
            return (i, i)
        name = ref[1:]
        l, r = (span(c) for c in g["internal"][name]["children"])
        assert l[1] + 1 == r[0]
        rng[name] = (l[0], r[1])
        return rng[name]

    span("n" + g["root"])
    return rng


def test_radix_tree_of_fig4_codes_has_the_figure_topology(oracle_lib):
    g = _fig4()
    tree = oracle_lib.radix_tree(g["codes"])
    rng = _figure_ranges(g)
    assert set(tree) == set(rng.values())
    for name, node in g["internal"].items():
        kids = []
        for c in node["children"]:
            kids.append((int(c[1:]), int(c[1:])) if c.startswith("L") else rng[c[1:]])
        assert tree[rng[name]] == tuple(kids)


def test_label_reduction_of_fig4(oracle_lib):
    g = _fig4()
    colours = {"green": 0, "red": 4, "orange": 5}
    leaf = [colours[c] for c in g["leaf_colours"]]
    tree = oracle_lib.radix_tree(g["codes"])
    labels = oracle_lib.reduce_labels(tree, leaf)
    rng = _figure_ranges(g)
    for name, node in g["internal"].items():
        want = oracle_lib.INVALID if node["colour"] == "gray" else colours[node["colour"]]
        assert labels[rng[name]] == want, name


def test_radix_tree_duplicates_split_by_index(oracle_lib):
    # equal codes: the tree over them is the radix tree of their indices
    tree = oracle_lib.radix_tree([5, 5, 5, 5])
    assert tree[(0, 3)] == ((0, 1), (2, 3))
    tree = oracle_lib.radix_tree([1, 2, 2, 2])
    assert tree[(0, 3)] == ((0, 0), (1, 3))
    assert tree[(1, 3)] == ((1, 1), (2, 3))


def test_label_reduction_matches_bruteforce_on_random_trees(oracle_lib):
    rng = np.random.default_rng(5)
    for _ in range(30):
        n = int(rng.integers(2, 60))
        codes = np.sort(rng.integers(0, 16, n)).tolist()
        leaf = rng.integers(0, 3, n).tolist()
        tree = oracle_lib.radix_tree(codes, 4)
        labels = oracle_lib.reduce_labels(tree, leaf)
        for (lo, hi), lab in labels.items():
            s = set(leaf[lo:hi + 1])
            assert lab == (s.pop() if len(s) == 1 else oracle_lib.INVALID)


# ---------------------------------------------------------------------------
# per-point nearest neighbour in another component


def test_nearest_other_on_a_line(oracle_lib):
    # points x = 0..9; components {0..3}, {4..6}, {7..9}
    pts = np.zeros((10, 2), np.float32)
    pts[:, 0] = np.arange(10)
    lab = np.array([0] * 4 + [4] * 3 + [7] * 3)
    d2, j = oracle_lib.nearest_other_bruteforce(pts, lab)
    want_j = [4, 4, 4, 4, 3, 3, 7, 6, 6, 6]
    want_d = [16, 9, 4, 1, 1, 4, 1, 1, 4, 9]
    assert j.tolist() == want_j
    assert d2.tolist() == want_d


def test_nearest_other_tie_goes_to_smaller_index(oracle_lib):
    # point 1 at the origin, two other-component points at distance 1
    pts = np.array([[1, 0], [0, 0], [-1, 0]], np.float32)
    d2, j = oracle_lib.nearest_other_bruteforce(pts, [0, 1, 2])
    assert j[1] == 0 and d2[1] == 1.0
    d2, j = oracle_lib.nearest_other_bruteforce(pts, [5, 5, 5])
    assert (j == -1).all() and np.isinf(d2).all()
