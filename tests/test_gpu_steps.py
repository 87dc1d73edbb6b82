"""Single steps of a Boruvka round on the GPU against brute force, and the
kernels' distance and weight functions against the oracle's.

A round (Section 3, Figure 3) is run from a given partition through the C
ABI test hook emst_test_round; each step is then checked on its own:

  bound      (Optimization 2) finite, at least the component's shortest
             outgoing D, and the D of a real pair leaving the component;
  candidate  (Algorithm 2) the (D, j)-nearest point outside the component
             if that lies within the bound, else none;
  stages A+B (the tie-break of Section 2) the component's minimum outgoing
             edge under (D, min, max);
  merge      ("Merging components together") the new partition is the
             connected components of the old one joined by the chosen
             edges, and their number is reported.
"""
import numpy as np
import pytest

import oracle
from paper_2207_00514_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

VARIANTS = (0, 5, 7, 8, 10, 11, 13)
BIG = 1 << 40


@pytest.fixture(scope="module")
def ctx():
    import paper_2207_00514_amd as emst
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    return emst.Context(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def bits(x):
    return np.asarray(x, np.float32).view(np.uint32).astype(np.int64)


def components_of(comp, edges):
    """Union-find over the partition `comp` joined by `edges`; returns a
    canonical labelling (smallest member index)."""
    n = len(comp)
    par = np.arange(n)

    def find(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x

    first = {}
    for i, c in enumerate(comp.tolist()):
        if c in first:
            a, b = find(i), find(first[c])
            par[max(a, b)] = min(a, b)
        else:
            first[c] = i
    for u, v in edges:
        a, b = find(int(u)), find(int(v))
        par[max(a, b)] = min(a, b)
    return np.array([find(i) for i in range(n)])


def canonical(labels):
    _, first = np.unique(labels, return_index=True)
    rep = {int(labels[f]): int(f) for f in first}
    return np.array([rep[int(x)] for x in labels])


def boruvka_partition(pts, rounds):
    """The partition after `rounds` Boruvka rounds, by brute force: each
    component joins along its minimum outgoing edge under (D, min, max)."""
    n = len(pts)
    comp = np.arange(n)
    D = bits(oracle.pair_d2_matrix(pts))
    for _ in range(rounds):
        d2, j = oracle.nearest_other_bruteforce(pts, comp)
        if (j < 0).all():
            break
        best = {}
        for i in range(n):
            if j[i] < 0:
                continue
            k = (int(D[i, j[i]]), min(i, int(j[i])), max(i, int(j[i])))
            c = int(comp[i])
            if c not in best or k < best[c]:
                best[c] = k
        comp = components_of(comp, [(k[1], k[2]) for k in best.values()])
    return comp


def partitions(pts, seed):
    n = len(pts)
    rng = np.random.default_rng(seed)
    yield "random", rng.integers(0, max(2, n // 7), n)
    yield "two", (np.arange(n) % 2)
    cells = np.floor(pts[:, :2] * 4.0).astype(np.int64)
    yield "cells", (cells[:, 0] * 97 + cells[:, 1]) % n
    for r in (1, 2):
        p = boruvka_partition(pts, r)
        if len(np.unique(p)) >= 2:
            yield f"boruvka{r}", p


_BRUTE = {}


def brute(pts, comp, key=None):
    """D bits of all pairs and the (D, j)-nearest outside point of every
    point, cached per case."""
    if key is not None and key in _BRUTE:
        return _BRUTE[key]
    D = bits(oracle.pair_d2_matrix(pts))
    d2, j = oracle.nearest_other_bruteforce(pts, comp)
    if key is not None:
        _BRUTE[key] = (D, d2, j)
    return D, d2, j


_PARTS = {}


def cached_partitions(pts, seed, key):
    if key not in _PARTS:
        _PARTS[key] = [(name, np.asarray(c)) for name, c in partitions(pts, seed) if len(np.unique(c)) >= 2]
    return _PARTS[key]


def check_round(pts, comp, got, shared_bound=False, key=None):
    n = len(pts)
    comp = np.asarray(comp)
    D, d2, j = brute(pts, comp, key)
    same = comp[:, None] == comp[None, :]
    out_min = np.where(same, BIG, D).min(axis=1)          # per point: shortest D leaving its component
    bound = bits(host(got["bound"]))
    comps = np.unique(comp)
    # bound: one value per component, finite, >= the shortest outgoing D,
    # equal to the D of a pair leaving the component
    for c in comps:
        m = comp == c
        b = np.unique(bound[m])
        assert b.size == 1, f"component {c}: several bounds"
        assert b[0] < bits(np.inf), f"component {c}: no bound"
        assert b[0] >= out_min[m].min(), f"component {c}: bound below its shortest edge"
        leaving = np.where(same[m], BIG, D[m])
        assert (leaving == b[0]).any(), f"component {c}: bound is not the length of a leaving pair"
    # candidate: the (D, j)-nearest outside point, if within the bound
    cj = host(got["cand_j"])
    cd = bits(host(got["cand_d"]))
    if not shared_bound:
        within = bits(d2) <= bound
        np.testing.assert_array_equal(cj, np.where(within, j, -1))
        np.testing.assert_array_equal(cd, np.where(within, bits(d2), bits(np.inf)))
    else:
        # variant 11 lowers the bound while the round runs, so a point whose
        # nearest outside point is longer than its component's edge may stop
        # early, with nothing or with a farther outside point; whatever it
        # reports is an outside point at its true D, never nearer than the
        # nearest
        found = np.nonzero(cj >= 0)[0]
        assert (comp[cj[found]] != comp[found]).all()
        np.testing.assert_array_equal(cd[found], D[found, cj[found]])
        assert ((cd[found] > bits(d2)[found]) | ((cd[found] == bits(d2)[found]) & (cj[found] >= j[found]))).all()
        assert (cd[cj < 0] == bits(np.inf)).all()
    # stages A and B: the component's minimum under (D, min, max)
    cu, cv, cd2 = host(got["comp_u"]), host(got["comp_v"]), bits(host(got["comp_d2"]))
    chosen = []
    for c in comps:
        idx = np.nonzero(comp == c)[0]
        keys = [(int(D[i, j[i]]), min(i, int(j[i])), max(i, int(j[i]))) for i in idx if j[i] >= 0]
        k = min(keys)
        for i in idx:
            assert (int(cd2[i]), int(cu[i]), int(cv[i])) == k, f"component {c}: edge {k}"
        chosen.append((k[1], k[2]))
    # merge: the components of the old partition joined by the chosen edges
    want = components_of(comp, chosen)
    np.testing.assert_array_equal(canonical(host(got["comp_out"])), canonical(want))
    assert got["ncomp"] == len(np.unique(want))


CASES = [(n, dim, seed) for n, dim, seed in ((3, 2, 1), (64, 3, 2), (257, 2, 3), (1500, 3, 4), (4096, 3, 5))]


@pytest.mark.parametrize("n,dim,seed", CASES)
@pytest.mark.parametrize("variant", VARIANTS)
def test_one_round_steps(ctx, n, dim, seed, variant):
    kinds = ("uniform", "int", "dup", "outlier")
    pts = W.small_random(n, dim, seed, kinds[seed % 4])
    for name, comp in cached_partitions(pts, seed, (n, dim, seed)):
        for rnd in (1, 2):
            print(f"case n={n} dim={dim} seed={seed} variant={variant} partition={name} round={rnd}", flush=True)
            got = ctx.test_round(dev(pts), torch.from_numpy(comp.astype(np.int32)), rnd, variant)
            torch.cuda.synchronize()
            check_round(pts, comp, got, shared_bound=variant == 11, key=(n, dim, seed, name))


def test_one_round_steps_on_ties(ctx):
    """Unit grid: every candidate ties with several others at D = 1."""
    pts = W.integer_grid(40, 2, seed=3)
    for name, comp in partitions(pts, 9):
        got = ctx.test_round(dev(pts), torch.from_numpy(comp.astype(np.int32)), 1, 13)
        torch.cuda.synchronize()
        check_round(pts, comp, got)


@pytest.mark.timeout(600)
def test_one_round_with_a_query_list(ctx):
    """From 3 * 2^18 points on, variant 13 searches from a query list in the
    third round on.  Sampled points are checked against a brute-force scan
    over every point, the smallest components in full, and the merge by its
    properties."""
    n = 800_000
    pts = W.clustered3d(n, seed=41)
    cells = np.floor(pts * 12.0).astype(np.int64)
    comp = ((cells[:, 0] * 12 + cells[:, 1]) * 12 + cells[:, 2]) % n
    got = ctx.test_round(dev(pts), torch.from_numpy(comp.astype(np.int32)), 3, 13)
    torch.cuda.synchronize()
    bound = bits(host(got["bound"]))
    cj, cd = host(got["cand_j"]), bits(host(got["cand_d"]))
    rng = np.random.default_rng(42)

    def nearest_other(i):
        d = bits(oracle.sqdist_pairs(np.repeat(pts[i:i + 1], n, axis=0), pts))
        d = np.where(comp == comp[i], BIG, d)
        k = d * (n + 1) + np.arange(n)
        j = int(np.argmin(k))
        return (int(d[j]), j) if d[j] < BIG else (None, -1)

    for i in rng.choice(n, 150, replace=False).tolist():
        d, j = nearest_other(i)
        if d is not None and d <= bound[i]:
            assert (int(cd[i]), int(cj[i])) == (d, j), f"point {i}"
        else:
            assert cj[i] == -1, f"point {i}"
    labels, counts = np.unique(comp, return_counts=True)
    cu, cv, cd2 = host(got["comp_u"]), host(got["comp_v"]), bits(host(got["comp_d2"]))
    for c in labels[np.argsort(counts)[:3]]:
        idx = np.nonzero(comp == c)[0]
        keys = []
        for i in idx.tolist():
            d, j = nearest_other(i)
            keys.append((d, min(i, j), max(i, j)))
        k = min(keys)
        assert (int(cd2[idx[0]]), int(cu[idx[0]]), int(cv[idx[0]])) == k, f"component {c}"
    # the merge: the reported partition is the old one joined by the chosen edges
    edges = set(zip(cu.tolist(), cv.tolist()))
    want = components_of(comp, sorted(edges))
    np.testing.assert_array_equal(canonical(host(got["comp_out"])), canonical(want))
    assert got["ncomp"] == len(np.unique(want))


# ---------------------------------------------------------------------------
# distance and weight functions


def _pair_sets(rng, m, dim):
    yield "uniform", rng.random((m, dim)), rng.random((m, dim))
    yield "wide", rng.normal(0, 1e15, (m, dim)), rng.normal(0, 1e15, (m, dim))
    yield "denormal", rng.random((m, dim)) * 1e-39, rng.random((m, dim)) * 1e-39
    yield "integer", rng.integers(-2 ** 20, 2 ** 20, (m, dim)), rng.integers(-2 ** 20, 2 ** 20, (m, dim))
    base = rng.random((m, dim)) * 1e3
    yield "close", base, base * (1 + rng.normal(0, 1e-7, (m, dim)))
    yield "mixed", rng.random((m, dim)) * 10.0 ** rng.integers(-30, 15, (m, 1)), rng.random((m, dim))


@pytest.mark.parametrize("dim", [2, 3])
def test_device_distances_equal_the_oracle(ctx, dim):
    rng = np.random.default_rng(100 + dim)
    m = 1 << 23
    for name, a, b in _pair_sets(rng, m, dim):
        a, b = a.astype(np.float32), b.astype(np.float32)
        print(f"distances {name} dim={dim} m={m}", flush=True)
        sq, box, w = ctx.test_distances(dev(a), dev(b))
        ref = oracle.sqdist_pairs(a, b)
        np.testing.assert_array_equal(host(sq).view(np.uint32), ref.view(np.uint32), err_msg=name)
        np.testing.assert_array_equal(host(box).view(np.uint32), ref.view(np.uint32), err_msg=name)
        np.testing.assert_array_equal(host(w).view(np.uint32), oracle.weights(ref).view(np.uint32), err_msg=name)


def test_device_weights_on_every_non_negative_float(ctx):
    """Every float32 from +0 to +inf: the weight is the oracle's correctly
    rounded square root, bit for bit."""
    last = 0x7F800000
    chunk = 1 << 27
    buf = torch.empty(chunk, dtype=torch.float32, device="cuda")
    for first in range(0, last + 1, chunk):
        count = min(chunk, last + 1 - first)
        ctx.test_weights(first, count, out=buf[:count])
        got = host(buf[:count]).view(np.uint32)
        x = np.arange(first, first + count, dtype=np.uint32).view(np.float32)
        want = oracle.weights(x).view(np.uint32)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, f"bits {first + int(bad[0]):#x}: {got[bad[0]]:#x} vs {want[bad[0]]:#x}"
