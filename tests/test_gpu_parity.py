"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: the edge set, the squared distances and the weights are bit-exact
(integer indices equal, float32 bit patterns equal), and the FP64 total
weight is equal; edges come in canonical (D, min, max) order."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2207_00514_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
# every traversal shape the library offers (emst_set_traversal); all give the same tree
VARIANTS = (0, 5, 7, 8, 10, 11, 13)


@pytest.fixture(scope="module")
def ctx():
    import paper_2207_00514_amd as emst
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    return emst.Context(0)


def run(ctx, pts, variant=None):
    if variant is not None:
        ctx.set_traversal(variant)
    e, w, d2 = ctx.build(torch.from_numpy(np.ascontiguousarray(pts, np.float32)).cuda())
    torch.cuda.synchronize()
    return e.cpu().numpy(), w.cpu().numpy(), d2.cpu().numpy()


def assert_same(got, ref, tag=""):
    e, w, d2 = got
    assert e.shape == ref.edges.shape, tag
    bad = np.nonzero((e != ref.edges).any(axis=1))[0]
    assert bad.size == 0, f"{tag}: {bad.size} edges differ, first at {bad[:5]}: {e[bad[:3]]} vs {ref.edges[bad[:3]]}"
    np.testing.assert_array_equal(d2.view(np.uint32), ref.d2.view(np.uint32), err_msg=tag)
    np.testing.assert_array_equal(w.view(np.uint32), ref.w.view(np.uint32), err_msg=tag)
    total = float(np.cumsum(w.astype(np.float64))[-1]) if len(w) else 0.0
    assert total == ref.total_weight, tag


SMALL = [(n, dim, seed, kind)
         for kind in ("uniform", "int", "dup", "outlier")
         for dim in (2, 3)
         for n, seed in ((2, 1), (3, 2), (5, 3), (64, 4), (65, 5), (257, 6), (1000, 7), (4099, 8))]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("n,dim,seed,kind", SMALL)
def test_small_clouds(ctx, n, dim, seed, kind, variant):
    pts = W.small_random(n, dim, seed, kind)
    print(f"case n={n} dim={dim} seed={seed} kind={kind} variant={variant}", flush=True)
    assert_same(run(ctx, pts, variant), oracle.prim(pts), f"{kind} n={n} d={dim}")


@pytest.mark.parametrize("dim,span", [(2, 6000), (3, 600)])
def test_short_runs_of_equal_edge_lengths(ctx, dim, span):
    """Integer coordinates over a wide range: a few pairs of MST edges share
    their smaller endpoint u and have exactly equal D, so the (D, u)-sorted
    edge order needs its in-place v fix-up; heavy-tie inputs (grids,
    duplicates) take the full sort instead."""
    ties_seen = 0
    for seed in range(6):
        rng = np.random.default_rng(500 + seed)
        pts = rng.integers(0, span, (3000, dim)).astype(np.float32)
        ref = oracle.prim(pts)
        print(f"case dim={dim} seed={500 + seed}", flush=True)
        assert_same(run(ctx, pts), ref, f"int-wide dim={dim} seed={seed}")
        k = (ref.d2.view(np.uint32).astype(np.uint64) << np.uint64(32)) | ref.edges[:, 0].astype(np.uint64)
        k = np.sort(k)
        ties_seen += int((k[1:] == k[:-1]).sum())
    assert ties_seen > 0


@pytest.mark.parametrize("variant", VARIANTS)
def test_closed_forms(ctx, variant):
    cases = {
        "identical": W.identical(1000),
        "grid2d": W.integer_grid(40, 2, seed=1),
        "grid3d": W.integer_grid(13, 3, seed=2),
        "collinear": W.collinear(3000, 2, seed=3),
        "dups": W.duplicates(300, 7, 3, seed=4),
        "two_clusters": W.two_clusters(2000, 3, seed=5),
    }
    for name, pts in cases.items():
        print(f"case {name} variant={variant}", flush=True)
        assert_same(run(ctx, pts, variant), oracle.emst(pts, threads=8), name)


@pytest.mark.parametrize("variant", VARIANTS)
def test_denormal_and_wide_range_coordinates(ctx, variant):
    rng = np.random.default_rng(3)
    tiny = (rng.random((500, 3)) * 1e-19).astype(np.float32)   # D is denormal
    assert_same(run(ctx, tiny, variant), oracle.prim(tiny), "denormal")
    under = (rng.random((500, 3)) * 1e-22).astype(np.float32)  # many D underflow to 0
    assert_same(run(ctx, under, variant), oracle.prim(under), "underflow")
    big = (rng.random((500, 3)) * 1e18).astype(np.float32)     # D near 1e36, finite
    assert_same(run(ctx, big, variant), oracle.prim(big), "large")
    neg = (rng.standard_normal((800, 2)) * 1e3).astype(np.float32)
    assert_same(run(ctx, neg, variant), oracle.prim(neg), "negative")
    off = (1000.0 + rng.random((800, 3)) * 1e-3).astype(np.float32)  # small extent far from 0
    assert_same(run(ctx, off, variant), oracle.prim(off), "offset")


def test_fewer_than_two_points(ctx):
    for n in (0, 1):
        e, w, d2 = run(ctx, np.zeros((n, 3), np.float32))
        assert e.shape == (0, 2) and w.shape == (0,)


def test_errors(ctx):
    import paper_2207_00514_amd as emst
    bad = np.zeros((10, 3), np.float32)
    bad[4, 1] = np.nan
    with pytest.raises(emst.EmstError) as ei:
        run(ctx, bad)
    assert ei.value.name == "EMST_ENONFINITE"
    bad[4, 1] = np.inf
    with pytest.raises(emst.EmstError) as ei:
        run(ctx, bad)
    assert ei.value.name == "EMST_ENONFINITE"
    huge = np.zeros((10, 3), np.float32)
    huge[0, 0] = 3e38
    huge[1, 0] = -3e38
    with pytest.raises(emst.EmstError) as ei:
        run(ctx, huge)
    assert ei.value.name == "EMST_ERANGE"
    with pytest.raises(emst.EmstError) as ei:
        run(ctx, np.zeros((10, 4), np.float32))
    assert ei.value.name == "EMST_EINVAL"
    # undersized workspace through the raw ABI
    import ctypes
    pts = torch.rand(100, 3, device="cuda")
    out = [torch.empty(99, 2, dtype=torch.int32, device="cuda"), torch.empty(99, device="cuda")]
    ws = torch.empty(emst.workspace_bytes(100, 3), dtype=torch.uint8, device="cuda")
    rc = emst.lib().emst_build(ctx._h, ctypes.c_void_p(pts.data_ptr()), 100, 3,
                               ctypes.c_void_p(out[0].data_ptr()), ctypes.c_void_p(out[1].data_ptr()),
                               None, ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(1000),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -4
    # the context still works afterwards
    pts = W.small_random(300, 3, 1)
    assert_same(run(ctx, pts), oracle.prim(pts), "after errors")


def test_variants_counting_and_repeats_agree(ctx):
    pts = W.clustered3d(60_000, seed=9)
    ref = oracle.kdboruvka(pts, threads=8)
    for variant in VARIANTS:
        for counting in (False, True):
            ctx.set_counting(counting)
            print(f"variant={variant} counting={counting}", flush=True)
            for rep in range(2):
                assert_same(run(ctx, pts, variant), ref, f"v{variant} c{counting} r{rep}")
            if counting:
                st = ctx.stats()
                assert st["child_tests"] > 0 and st["leaf_tests"] > 0
    ctx.set_counting(False)


def test_round_structure(ctx):
    pts = W.clustered3d(100_000, seed=10)
    run(ctx, pts)
    st = ctx.stats()
    n = len(pts)
    assert 1 <= st["rounds"] <= math.ceil(math.log2(n))
    c = st["components"] + [1]
    assert c[0] == n
    for a, b in zip(c[:-1], c[1:]):
        assert b <= a // 2
    assert st["tree_height"] <= 96


# ---------------------------------------------------------------------------
# stages


def test_fig4_tree_and_label_propagation(ctx):
    g = json.load(open(os.path.join(GOLDEN, "fig4_label_reduction.json")))
    codes = torch.tensor(g["codes"], dtype=torch.int64, device="cuda")
    colours = {"green": 0, "red": 4, "orange": 5}
    leaf = torch.tensor([colours[c] for c in g["leaf_colours"]], dtype=torch.int32, device="cuda")
    left, right, label, root = ctx.test_tree_from_codes(codes, leaf)
    left, right, label = left.cpu().tolist(), right.cpu().tolist(), label.cpu().numpy().view(np.uint32)
    ref = oracle.radix_tree(g["codes"])
    ref_lab = oracle.reduce_labels(ref, [colours[c] for c in g["leaf_colours"]])

    def rng(ref_child):
        return (-ref_child - 1, -ref_child - 1) if ref_child < 0 else (ref_child,)

    ranges = {}

    def span(k):
        if k < 0:
            return (-k - 1, -k - 1)
        lo = span(left[k])[0]
        hi = span(right[k])[1]
        ranges[k] = (lo, hi)
        return (lo, hi)

    assert span(root) == (0, 7)
    assert set(ranges.values()) == set(ref)
    for k, rr in ranges.items():
        assert (span(left[k]), span(right[k])) == ref[rr]
        want = ref_lab[rr]
        assert (label[k] == 0xFFFFFFFF) if want == oracle.INVALID else (label[k] == want)
        # node k splits between leaves k and k+1
        assert span(left[k])[1] == k


def test_tree_and_labels_on_random_codes(ctx):
    rng = np.random.default_rng(4)
    for trial in range(20):
        n = int(rng.integers(2, 3000))
        hi = [4, 64, 2 ** 20, 2 ** 62][trial % 4]
        codes = np.sort(rng.integers(0, hi, n, dtype=np.int64))
        leaf = rng.integers(0, 1 + trial, n).astype(np.int32)
        left, right, label, root = ctx.test_tree_from_codes(torch.from_numpy(codes).cuda(),
                                                            torch.from_numpy(leaf).cuda())
        left, right = left.cpu().numpy(), right.cpu().numpy()
        label = label.cpu().numpy().view(np.uint32)
        # ranges bottom-up via the split rule: node k covers [lo, hi] with k in it
        ref = oracle.radix_tree(codes.tolist()) if n <= 400 else None
        stack = [(root, None)]
        spans = {}

        def span(k):
            if k < 0:
                return (-k - 1, -k - 1)
            if k in spans:
                return spans[k]
            a, b = span(left[k]), span(right[k])
            assert a[1] + 1 == b[0] and a[1] == k
            spans[k] = (a[0], b[1])
            return spans[k]

        import sys
        sys.setrecursionlimit(100000)
        assert span(root) == (0, n - 1)
        assert len(spans) == n - 1
        for k, (lo, hi_) in spans.items():
            s = set(leaf[lo:hi_ + 1].tolist())
            assert label[k] == (s.pop() if len(s) == 1 else 0xFFFFFFFF)
            if ref is not None:
                assert (span(left[k]), span(right[k])) == ref[(lo, hi_)]


def test_radix_sort(ctx):
    rng = np.random.default_rng(5)
    # 8,388,608 keys and up run the 16-item tile shape; from 4,194,304 keys
    # on a pass is one launch with look-back across tiles
    for n in (2, 100, 2047, 2048, 2049, 100_000, 3_000_001, 4_194_303, 4_194_304, 4_194_305, 8_388_608,
              9_000_001):
        keys = rng.integers(0, 2 ** 63, n, dtype=np.int64)
        keys[: n // 3] = keys[0]  # many equal keys: stability matters
        if n > 10:
            keys[5] = -1  # top bit set (uint64 0xFFFF...)
        vals = np.arange(n, dtype=np.int32)
        k = torch.from_numpy(keys).cuda()
        v = torch.from_numpy(vals).cuda()
        ctx.test_radix_sort(k, v)
        order = np.argsort(keys.view(np.uint64), kind="stable")
        np.testing.assert_array_equal(k.cpu().numpy(), keys[order])
        np.testing.assert_array_equal(v.cpu().numpy(), vals[order])


# ---------------------------------------------------------------------------
# full workloads


def test_uniform2d_10k(ctx):
    pts = W.uniform2d()
    ref = oracle.prim(pts)
    for variant in VARIANTS:
        assert_same(run(ctx, pts, variant), ref, f"uniform2d_10k v{variant}")


def test_query_list_threshold(ctx):
    """Variant 13 compacts the searching points into a query list from
    3 * 2^18 points on and skips inside the traversal below: both sides of the
    threshold, 2D and 3D, with integer coordinates (many equal lengths)."""
    for n in (786_431, 786_432):
        for pts in (W.clustered3d(n, seed=31), np.floor(W.uniform2d(n, seed=32) * 2000.0).astype(np.float32)):
            print(f"query list n={n} dim={pts.shape[1]}", flush=True)
            ref = oracle.kdboruvka(pts, threads=16)
            assert_same(run(ctx, pts, 13), ref, f"n={n} dim={pts.shape[1]}")
            st = ctx.stats()
            q = st["queries_round"]
            assert all(x == n for x in q[:2])
            if n >= 786_432:
                assert any(x < n for x in q[2:])  # a list ran
            else:
                assert all(x == n for x in q)


def test_scan_fold_threshold(ctx):
    """Up to 1024 tiles of 2048 positions the round kernels compute the
    tile carries and list offsets themselves, above it one-workgroup scan
    kernels do; the merge kernels' root-list segments grow from 1024 to
    1280 entries across the same sizes.  Both sides, variant 13."""
    for n in (1024 * 2048, 1024 * 2048 + 1):
        pts = W.clustered3d(n, seed=33)
        print(f"scan fold n={n}", flush=True)
        ref = oracle.kdboruvka(pts, threads=16)
        assert_same(run(ctx, pts, 13), ref, f"n={n}")


def test_clustered3d_2m(ctx):
    pts = W.clustered3d()
    ref = oracle.kdboruvka(pts, threads=16)
    for variant in VARIANTS:
        print(f"clustered3d_2m variant={variant}", flush=True)
        assert_same(run(ctx, pts, variant), ref, f"clustered3d_2m v{variant}")


# ---------------------------------------------------------------------------
# batches


def run_batched(ctx, clouds):
    ts = [torch.from_numpy(np.ascontiguousarray(c, np.float32)).cuda() for c in clouds]
    out = ctx.build_batched(ts)
    torch.cuda.synchronize()
    return [(e.cpu().numpy(), w.cpu().numpy(), d.cpu().numpy()) for e, w, d in out]


@pytest.mark.parametrize("variant", [0, 5, 7, 8, 10, 13])
def test_batched_small_mixed(ctx, variant):
    ctx.set_traversal(variant)
    rng = np.random.default_rng(11)
    clouds = []
    for c in range(40):
        n = int(rng.choice([0, 1, 2, 3, 17, 64, 300, 1500]))
        dim = int(rng.choice([2, 3]))
        kind = ("uniform", "int", "dup", "outlier")[c % 4]
        clouds.append(W.small_random(n, dim, 1000 + c, kind))
    res = run_batched(ctx, clouds)
    for c, (pts, got) in enumerate(zip(clouds, res)):
        assert_same(got, oracle.prim(pts), f"cloud {c} n={len(pts)} d={pts.shape[1]} variant {variant}")
    ctx.set_traversal(10)


def test_batched_equals_solo(ctx):
    clouds = W.batched_clouds(n_clouds=24, seed=21, lo=500, hi=20_000)
    res = run_batched(ctx, clouds)
    for c, (pts, got) in enumerate(zip(clouds, res)):
        solo = run(ctx, pts)
        for a, b in zip(got, solo):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"cloud {c}"


def test_batched_graph_replays_equal_eager(ctx):
    """Rounds from the third on replayed from a captured graph (one per
    context, reused across calls): several calls in a row, with eager work of
    another context and synchronisations between them, each equal to the
    eager batched result, then a second shape (a new capture)."""
    import paper_2207_00514_amd as emst
    g = emst.Context(0)
    g.set_graphs(True)
    other = emst.Context(0)
    for shape in range(2):
        clouds = W.batched_clouds(n_clouds=48 if shape == 0 else 12, seed=81 + shape, lo=2000, hi=60_000)
        ctx.set_traversal(-1)
        ref = run_batched(ctx, clouds)
        for rep in range(4):
            print(f"graph replay shape={shape} rep={rep}", flush=True)
            got = run_batched(g, clouds)
            for c, (a, b) in enumerate(zip(got, ref)):
                for x, y in zip(a, b):
                    assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), f"shape {shape} rep {rep} cloud {c}"
            assert g.stats()["rounds"] == ctx.stats()["rounds"]
            pts = W.small_random(3000, 3, 90 + rep)
            assert_same(run(other, pts), oracle.prim(pts), "eager work between replays")
    # a batch large enough for the query-list rounds
    clouds = W.batched_clouds(n_clouds=20, seed=83, lo=40_000, hi=80_000)
    ref = run_batched(ctx, clouds)
    for rep in range(2):
        got = run_batched(g, clouds)
        for c, (a, b) in enumerate(zip(got, ref)):
            assert all(np.array_equal(x.view(np.uint8), y.view(np.uint8)) for x, y in zip(a, b)), f"cloud {c}"


def test_batched_errors(ctx):
    import paper_2207_00514_amd as emst
    clouds = [W.small_random(100, 3, 1), W.small_random(50, 2, 2)]
    clouds[1][7, 0] = np.nan
    with pytest.raises(emst.EmstError) as ei:
        run_batched(ctx, clouds)
    assert ei.value.name == "EMST_ENONFINITE" and "cloud 1" in str(ei.value)
    # two single points: no edges at all
    res = run_batched(ctx, [np.zeros((1, 3), np.float32), np.ones((1, 2), np.float32)])
    assert all(r[0].shape == (0, 2) for r in res)
    # the context still works
    pts = W.small_random(300, 3, 1)
    assert_same(run(ctx, pts), oracle.prim(pts), "after batch errors")


@pytest.mark.timeout(600)
def test_batched_512_clouds(ctx):
    """The 512-cloud batch (log-uniform sizes 1e3..2e5, half 2D uniform, half
    3D mixtures, about 2e7 points; above 2^23 keys the radix sort runs its
    16-item tiles): every cloud against the oracle."""
    clouds = W.batched_clouds()
    ctx.set_traversal(-1)
    res = run_batched(ctx, clouds)
    for c, (pts, got) in enumerate(zip(clouds, res)):
        if c % 64 == 0:
            print(f"batched cloud {c} n={len(pts)} dim={pts.shape[1]}", flush=True)
        assert_same(got, oracle.emst(pts, threads=16), f"cloud {c} n={len(pts)} dim={pts.shape[1]}")


@pytest.mark.timeout(900)
def test_cosmology3d_37m(ctx):
    """The full 37M-point cosmology-like cloud through emst_build, edge by
    edge against the oracle's kd-tree Boruvka: Morton codes (no rank-space
    switch), the one-sweep radix passes, the scan kernels above 1024 tiles
    and the query-list rounds all run at this size."""
    import time
    t0 = time.perf_counter()
    pts = W.make("cosmology3d_37m")
    print(f"cosmology3d_37m generated in {time.perf_counter() - t0:.1f} s", flush=True)
    ctx.set_traversal(-1)
    got = run(ctx, pts)
    st = ctx.stats()
    n = len(pts)
    assert st["rank_codes"] == 0
    assert st["traversal_variant"] == 13
    assert any(q < n for q in st["queries_round"][2:]), "no query-list round ran"
    t0 = time.perf_counter()
    ref = oracle.kdboruvka(pts, threads=min(16, os.cpu_count() or 1))
    print(f"oracle {time.perf_counter() - t0:.1f} s", flush=True)
    assert_same(got, ref, "cosmology3d_37m")


def test_one_sweep_odd_pass_count(ctx):
    """5,000,000 points: from 2^22 keys on every radix pass is one launch
    with look-back across tiles.  With 23 bits of point index the edge order
    takes 7 passes (3 on the index, 4 on the length), so the sorted edges
    end in the second buffer; the Morton sort takes 8 passes in 3D and 4
    (32-bit codes) in 2D."""
    for pts in (W.clustered3d(5_000_000, seed=41), W.uniform2d(5_000_000, seed=42)):
        print(f"one-sweep n={len(pts)} dim={pts.shape[1]}", flush=True)
        got = run(ctx, pts, 13)
        ref = oracle.kdboruvka(pts, threads=min(16, os.cpu_count() or 1))
        assert_same(got, ref, f"n=5,000,000 dim={pts.shape[1]}")


def test_tree_boxes_are_exact(ctx):
    """Every internal node's box is exactly the min/max of its leaves."""
    import sys
    sys.setrecursionlimit(100000)
    for seed, n in ((1, 2), (2, 3), (3, 777), (4, 5000), (5, 40000)):
        pts = W.small_random(n, 3, seed, ("uniform", "dup", "int", "outlier")[seed % 4])
        left, right, lo, hi, root = ctx.test_tree_boxes(torch.from_numpy(pts).cuda())
        left, right = left.cpu().numpy(), right.cpu().numpy()
        lo, hi = lo.cpu().numpy(), hi.cpu().numpy()
        mn = np.zeros((n - 1, 3), np.float32)
        mx = np.zeros((n - 1, 3), np.float32)
        seen = np.zeros(n, bool)
        # post-order without recursion
        order, stack = [], [root]
        while stack:
            k = stack.pop()
            order.append(k)
            for c in (left[k], right[k]):
                if c >= 0:
                    stack.append(c)
        for k in reversed(order):
            boxes = []
            for c in (left[k], right[k]):
                if c < 0:
                    seen[-c - 1] = True
                    boxes.append((pts[-c - 1], pts[-c - 1]))
                else:
                    boxes.append((mn[c], mx[c]))
            mn[k] = np.minimum(boxes[0][0], boxes[1][0])
            mx[k] = np.maximum(boxes[0][1], boxes[1][1])
        assert seen.all() and len(order) == n - 1
        np.testing.assert_array_equal(lo, mn)
        np.testing.assert_array_equal(hi, mx)


def test_skewed_density_rank_space_codes(ctx):
    """Extreme density contrast (most points inside a few Morton cells of
    the outlier-set scene box): the build switches to rank-space codes and
    the tree is the oracle's."""
    for n in (60_000, 250_000):
        pts = W.make("skewed3d_2m", n)
        print(f"case skewed3d n={n}", flush=True)
        got = run(ctx, pts)
        assert ctx.stats()["rank_codes"] == 1
        assert_same(got, oracle.emst(pts, threads=16), f"skewed3d n={n}")
    pts = W.make("clustered3d_2m", 60_000)
    run(ctx, pts)
    assert ctx.stats()["rank_codes"] == 0


def test_skewed3d_2m(ctx):
    pts = W.make("skewed3d_2m")
    got = run(ctx, pts)
    assert ctx.stats()["rank_codes"] == 1
    assert_same(got, oracle.kdboruvka(pts, threads=16), "skewed3d_2m")


def test_skewed3d_rank_space_one_sweep(ctx):
    """5,000,000 skewed points: the rank-space rebuild's per-axis sorts (4
    passes each) and the rank-space Morton sort run as one-sweep passes."""
    pts = W.skewed3d(5_000_000)
    got = run(ctx, pts)
    assert ctx.stats()["rank_codes"] == 1
    assert_same(got, oracle.kdboruvka(pts, threads=16), "skewed3d n=5,000,000")
