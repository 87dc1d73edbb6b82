"""Parity of the mutual-reachability path (HDBSCAN*, Section 4 "Mutual
reachability distance") with the CPU oracle, through the C ABI.

Bar: squared core distances bit-exact; the tree under (bits(M), min, max)
bit-exact in edges, M and weights, with M = max(core2(u), core2(v), D)."""
import numpy as np
import pytest

import oracle
from paper_2207_00514_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2207_00514_amd as emst
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    return emst.Context(0)


def dev(pts):
    return torch.from_numpy(np.ascontiguousarray(pts, np.float32)).cuda()


def same(a, b):
    return np.array_equal(np.asarray(a).view(np.uint32), np.asarray(b).view(np.uint32))


def assert_same_tree(got, ref, tag):
    e, w, d2 = got
    assert e.shape == ref.edges.shape, tag
    bad = np.nonzero((e != ref.edges).any(axis=1))[0]
    assert bad.size == 0, f"{tag}: {bad.size} edges differ, first {e[bad[:3]]} vs {ref.edges[bad[:3]]}"
    assert same(d2, ref.d2), tag
    assert same(w, ref.w), tag


def gpu_core(ctx, pts, k):
    c = ctx.core_distances(dev(pts), k)
    torch.cuda.synchronize()
    return c.cpu().numpy()


def gpu_tree(ctx, pts, k):
    e, w, d2, core2 = ctx.build_mreach(dev(pts), k)
    torch.cuda.synchronize()
    return (e.cpu().numpy(), w.cpu().numpy(), d2.cpu().numpy()), core2.cpu().numpy()


SMALL = [(n, dim, seed, kind)
         for kind in ("uniform", "int", "dup", "outlier")
         for dim in (2, 3)
         for n, seed in ((3, 1), (65, 2), (1000, 3), (3001, 4))]


@pytest.mark.parametrize("n,dim,seed,kind", SMALL)
@pytest.mark.parametrize("k", [1, 2, 3, 8, 17, 64])
def test_core_distances_small(ctx, n, dim, seed, kind, k):
    if k > n:
        pytest.skip("k_pts > n")
    pts = W.small_random(n, dim, seed, kind)
    print(f"case n={n} dim={dim} kind={kind} k={k}", flush=True)
    ref = oracle.core_bruteforce(pts, k) if n <= 1000 else oracle.core_distances(pts, k, "kd", threads=8)
    assert same(gpu_core(ctx, pts, k), ref)


@pytest.mark.parametrize("n,dim,seed,kind", SMALL)
@pytest.mark.parametrize("k", [1, 2, 5, 16])
def test_mreach_tree_small(ctx, n, dim, seed, kind, k):
    if k > n:
        pytest.skip("k_pts > n")
    pts = W.small_random(n, dim, seed, kind)
    print(f"case n={n} dim={dim} kind={kind} k={k}", flush=True)
    core2 = oracle.core_distances(pts, k, "kd", threads=8)
    got, gcore = gpu_tree(ctx, pts, k)
    assert same(gcore, core2)
    assert_same_tree(got, oracle.prim_mreach(pts, core2), f"mreach n={n} d={dim} {kind} k={k}")


def test_k1_equals_the_emst(ctx):
    for n, dim, seed, kind in ((5000, 3, 7, "uniform"), (4000, 2, 8, "dup")):
        pts = W.small_random(n, dim, seed, kind)
        got, core2 = gpu_tree(ctx, pts, 1)
        assert (core2 == 0).all()
        e, w, d2 = ctx.build(dev(pts))
        torch.cuda.synchronize()
        assert np.array_equal(got[0], e.cpu().numpy())
        assert same(got[1], w.cpu().numpy()) and same(got[2], d2.cpu().numpy())


def test_unit_line_closed_form(ctx):
    n = 40
    pts = np.zeros((n, 3), np.float32)
    pts[:, 0] = np.arange(n, dtype=np.float32)
    (e, w, _), core2 = gpu_tree(ctx, pts, 3)
    assert core2[0] == 4 and core2[-1] == 4 and (core2[1:-1] == 1).all()
    expect = [[i, i + 1] for i in range(1, n - 2)] + [[0, 1], [n - 3, n - 1]]
    assert e.tolist() == sorted(expect, key=lambda x: (4 if x in ([0, 1], [n - 3, n - 1]) else 1, x[0], x[1]))
    assert float(np.sum(w.astype(np.float64))) == float(n + 1)


@pytest.mark.parametrize("k", [2, 4, 16])
def test_mreach_medium_clouds(ctx, k):
    for wl, n in (("clustered3d_2m", 60_000), ("uniform2d_10k", 10_000), ("cosmology3d_37m", 80_000)):
        pts = W.make(wl, n)
        print(f"case {wl} n={n} k={k}", flush=True)
        core2 = oracle.core_distances(pts, k, "kd", threads=16)
        got, gcore = gpu_tree(ctx, pts, k)
        assert same(gcore, core2)
        assert_same_tree(got, oracle.kdboruvka_mreach(pts, core2, threads=16), f"{wl} k={k}")


def test_mreach_clustered3d_2m(ctx):
    """Full-size cloud, k_pts = 4: cores and the whole tree against the
    OpenMP oracle."""
    pts = W.make("clustered3d_2m")
    core2 = oracle.core_distances(pts, 4, "kd", threads=16)
    got, gcore = gpu_tree(ctx, pts, 4)
    assert same(gcore, core2)
    assert_same_tree(got, oracle.kdboruvka_mreach(pts, core2, threads=16), "clustered3d_2m k=4")


def test_mreach_one_sweep_size(ctx):
    """5,000,000 cosmology-recipe points, k_pts = 8: from 2^22 points on the
    Morton and edge sorts are one-sweep radix passes (the edge order in an
    odd number of them); cores and the whole tree against the oracle."""
    pts = W.make("cosmology3d_37m", 5_000_000)
    core2 = oracle.core_distances(pts, 8, "kd", threads=16)
    got, gcore = gpu_tree(ctx, pts, 8)
    assert same(gcore, core2)
    assert_same_tree(got, oracle.kdboruvka_mreach(pts, core2, threads=16), "cosmology3d n=5,000,000 k=8")


def test_errors(ctx):
    import paper_2207_00514_amd as emst
    pts = dev(W.small_random(100, 3, 1))
    for k in (0, 65, 101):
        with pytest.raises(emst.EmstError) as ei:
            ctx.core_distances(pts, k)
        assert ei.value.name == "EMST_EINVAL"
        with pytest.raises(emst.EmstError) as ei:
            ctx.build_mreach(pts, k)
        assert ei.value.name == "EMST_EINVAL"
    one = dev(np.ones((1, 3), np.float32))
    c = ctx.core_distances(one, 1)
    torch.cuda.synchronize()
    assert c.cpu().numpy().tolist() == [0.0]
    e, w, d2, core2 = ctx.build_mreach(one, 1)
    torch.cuda.synchronize()
    assert e.shape == (0, 2) and core2.cpu().numpy().tolist() == [0.0]
    bad = W.small_random(50, 2, 3)
    bad[3, 1] = np.nan
    with pytest.raises(emst.EmstError) as ei:
        ctx.build_mreach(dev(bad), 2)
    assert ei.value.name == "EMST_ENONFINITE"
    # the context still works
    p = W.small_random(300, 3, 4)
    got, _ = gpu_tree(ctx, p, 3)
    assert_same_tree(got, oracle.prim_mreach(p, oracle.core_bruteforce(p, 3)), "after errors")
