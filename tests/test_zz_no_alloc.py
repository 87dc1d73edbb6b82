"""emst_build_noalloc (the entry point for callers that cannot allocate
device memory) against emst_build, through the C ABI: bit-identical edges,
squared distances and weights on two calls in a row, the second with a
smaller cloud, and the size limit of its static workspace."""
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


def host(res):
    e, w, d2 = res
    torch.cuda.synchronize()
    return e.cpu().numpy(), w.cpu().numpy(), d2.cpu().numpy()


def assert_identical(a, b, tag):
    assert a[0].shape == b[0].shape, tag
    assert np.array_equal(a[0], b[0]), f"{tag}: edges differ"
    assert np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32)), f"{tag}: weights differ"
    assert np.array_equal(a[2].view(np.uint32), b[2].view(np.uint32)), f"{tag}: d2 differ"


def test_noalloc_equals_build_on_two_calls(ctx):
    """Two calls in a row, the second smaller: the static workspace keeps
    the first call's contents, which the second must not depend on."""
    big = W.clustered3d(200_000, seed=21)
    small = W.uniform2d(30_000, seed=22)
    for tag, pts in (("clustered3d 200000", big), ("uniform2d 30000", small)):
        print(f"noalloc: {tag}", flush=True)
        t = torch.from_numpy(pts).cuda()
        got = host(ctx.build_noalloc(t))
        ref = host(ctx.build(t))
        assert_identical(got, ref, tag)
    # the smaller cloud also against the oracle, edge by edge
    o = oracle.emst(small, threads=8)
    assert np.array_equal(got[0], o.edges)
    assert np.array_equal(got[2].view(np.uint32), o.d2.view(np.uint32))
    assert np.array_equal(got[1].view(np.uint32), o.w.view(np.uint32))


def test_noalloc_repeat_and_preallocated_outputs(ctx):
    """The same cloud twice into caller-allocated outputs, after a larger
    call left the workspace dirty: identical each time."""
    pts = torch.from_numpy(W.clustered3d(50_000, seed=23)).cuda()
    m = pts.shape[0] - 1
    out = (torch.empty((m, 2), dtype=torch.int32, device="cuda"), torch.empty(m, device="cuda"),
           torch.empty(m, device="cuda"))
    ref = host(ctx.build(pts))
    for k in range(2):
        assert_identical(host(ctx.build_noalloc(pts, out=out)), ref, f"repeat {k}")


def test_noalloc_limit_and_degenerate_sizes(ctx):
    import paper_2207_00514_amd as emst
    lim = emst.NOALLOC_WORKSPACE_BYTES
    n_ok = 1
    while emst.workspace_bytes(2 * n_ok, 3) <= lim:
        n_ok *= 2
    n_bad = n_ok
    while emst.workspace_bytes(n_bad, 3) <= lim:
        n_bad += n_ok // 8
    pts = torch.zeros((n_bad, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(emst.EmstError) as ei:
        ctx.build_noalloc(pts)
    assert ei.value.name == "EMST_ENOMEM" and "static workspace" in str(ei.value)
    # 0 and 1 points: no edges
    for n in (0, 1):
        e, w, d2 = ctx.build_noalloc(torch.zeros((n, 3), dtype=torch.float32, device="cuda"))
        assert e.shape == (0, 2)
    # the largest size that fits still equals emst_build
    while emst.workspace_bytes(n_ok + 4096, 3) <= lim:
        n_ok += 4096
    big = torch.from_numpy(W.small_random(n_ok, 3, 24)).cuda()
    assert_identical(host(ctx.build_noalloc(big)), host(ctx.build(big)), f"n={n_ok}")
