"""The traversal autotuner and the continuous-batching server, on the GPU.

Autotuning only chooses among traversal variants that compute the same
tree, so every tuned call must still equal the oracle; the table must
round-trip through the C ABI and be applied by mode, dimension and size.
The server must return for every request exactly the tree of that request
solved alone, whatever it was batched with."""
import json

import numpy as np
import pytest

import oracle
from paper_2207_00514_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(pts):
    return torch.from_numpy(np.ascontiguousarray(pts, np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in t]


def same_tree(a, b):
    return (np.array_equal(a[0], b[0]) and np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32))
            and np.array_equal(a[2].view(np.uint32), b[2].view(np.uint32)))


def oracle_tree(pts):
    """(edges, weights, d2) of the CPU oracle for one cloud."""
    ref = oracle.emst(np.ascontiguousarray(pts, np.float32), threads=16)
    return ref.edges, ref.w, ref.d2


def test_autotune_table_round_trip_and_results():
    import paper_2207_00514_amd as emst
    from paper_2207_00514_amd import autotune
    ctx = emst.Context(0)
    text = autotune.autotune(ctx, single_sizes=(3000, 30000), dims=(3,), repeats=1)
    table = json.loads(text)["entries"]
    assert [e["n_min"] for e in table] == [0, int((3000 * 30000) ** 0.5)]
    assert all((e["variant"], e["lds_depth"]) in autotune.SINGLE_CANDIDATES for e in table)
    back = json.loads(ctx.get_autotune())["entries"]
    key = lambda e: (e["mode"], e["dim"], e["n_min"], e["variant"], e["lds_depth"])  # noqa: E731
    assert [key(e) for e in back] == [key(e) for e in table]
    for n in (3000, 30000):
        pts = W.clustered3d(n)
        got = host(ctx.build(dev(pts)))
        e = table[0] if n < table[1]["n_min"] else table[1]
        assert ctx.stats()["traversal_variant"] == e["variant"]
        assert ctx.stats()["traversal_lds_depth"] == (e["lds_depth"] if e["variant"] == 13 else 0)
        ref = oracle.emst(pts, threads=8)
        assert np.array_equal(got[0], ref.edges) and np.array_equal(got[2].view(np.uint32), ref.d2.view(np.uint32))
    # the saved table configures a new context
    ctx2 = emst.Context(0, autotune_json=text)
    assert json.loads(ctx2.get_autotune())["entries"] == back


def test_autotune_lookup_by_mode_dim_and_size():
    import paper_2207_00514_amd as emst
    table = {"entries": [
        {"mode": "single", "dim": 3, "n_min": 0, "variant": 7},
        {"mode": "single", "dim": 3, "n_min": 5000, "variant": 5},
        {"mode": "single", "dim": 2, "n_min": 0, "variant": 8},
        {"mode": "batched", "dim": 3, "n_min": 0, "variant": 0}]}
    ctx = emst.Context(0, autotune_json=json.dumps(table))
    for pts, want in ((W.clustered3d(1000), 7), (W.clustered3d(6000), 5), (W.uniform2d(3000), 8)):
        host(ctx.build(dev(pts)))
        assert ctx.stats()["traversal_variant"] == want
    clouds = W.batched_clouds(n_clouds=5, seed=41, lo=200, hi=3000)
    res = ctx.build_batched([dev(c) for c in clouds])
    torch.cuda.synchronize()
    assert ctx.stats()["traversal_variant"] == 0
    for c, r in zip(clouds, res):
        ref = oracle.prim(c)
        assert np.array_equal(r[0].cpu().numpy(), ref.edges)
    # an explicit variant overrides the table
    ctx.set_traversal(10)
    host(ctx.build(dev(W.clustered3d(6000))))
    assert ctx.stats()["traversal_variant"] == 10


def test_lds_depth_axis():
    """The LDS ring depth of variant 13 (table key lds_depth, or
    emst_set_lds_depth): every depth gives the oracle's tree, alone and in a
    batch, and the table's depth applies by size."""
    import paper_2207_00514_amd as emst
    table = {"entries": [
        {"mode": "single", "dim": 3, "n_min": 0, "variant": 13, "lds_depth": 4},
        {"mode": "single", "dim": 3, "n_min": 5000, "variant": 13, "lds_depth": 16},
        {"mode": "batched", "dim": 3, "n_min": 0, "variant": 13, "lds_depth": 16}]}
    ctx = emst.Context(0, autotune_json=json.dumps(table))
    for pts, want in ((W.clustered3d(1000, seed=5), 4), (W.clustered3d(60_000, seed=6), 16)):
        got = host(ctx.build(dev(pts)))
        assert ctx.stats()["traversal_lds_depth"] == want
        ref = oracle.emst(pts, threads=8)
        assert np.array_equal(got[0], ref.edges) and np.array_equal(got[2].view(np.uint32), ref.d2.view(np.uint32))
    pts = W.clustered3d(900_000, seed=7)  # query-list rounds
    ref = oracle.emst(pts, threads=16)
    for d in (4, 8, 16):
        ctx.set_lds_depth(d)
        got = host(ctx.build(dev(pts)))
        assert ctx.stats()["traversal_lds_depth"] == d
        assert np.array_equal(got[0], ref.edges), f"depth {d}"
    ctx.set_lds_depth(0)
    clouds = W.batched_clouds(n_clouds=8, seed=42, lo=500, hi=20_000)
    res = ctx.build_batched([dev(c) for c in clouds])
    torch.cuda.synchronize()
    assert ctx.stats()["traversal_lds_depth"] == 16
    for c, r in zip(clouds, res):
        assert np.array_equal(r[0].cpu().numpy(), oracle.emst(c, threads=8).edges)
    for bad in (1, 2, 3, 5, 32, -1):
        with pytest.raises(emst.EmstError):
            ctx.set_lds_depth(bad)
    with pytest.raises(emst.EmstError):
        ctx.set_autotune('{"entries": [{"mode": "single", "dim": 3, "n_min": 0, "variant": 13, "lds_depth": 6}]}')


def test_autotune_bad_tables():
    import paper_2207_00514_amd as emst
    ctx = emst.Context(0)
    good = '{"entries": [{"mode": "single", "dim": 3, "n_min": 0, "variant": 7}]}'
    ctx.set_autotune(good)
    for bad in ("{", '{"entries": [{"mode": "x", "dim": 3, "n_min": 0, "variant": 7}]}',
                '{"entries": [{"mode": "single", "dim": 4, "n_min": 0, "variant": 7}]}',
                '{"entries": [{"mode": "single", "dim": 3, "n_min": 0, "variant": 99}]}',
                '{"entries": [{"mode": "single", "dim": 3, "n_min": 0, "variant": 12}]}',
                '{"entries": []} trailing'):
        with pytest.raises(emst.EmstError) as ei:
            ctx.set_autotune(bad)
        assert ei.value.name == "EMST_EINVAL"
        assert json.loads(ctx.get_autotune())["entries"][0]["variant"] == 7
    with pytest.raises(emst.EmstError):
        emst.Context(0, autotune_json="not json")
    ctx.set_autotune(None)
    assert json.loads(ctx.get_autotune()) == {"entries": []}


def test_only_the_offered_traversal_shapes_are_accepted():
    import paper_2207_00514_amd as emst
    ctx = emst.Context(0)
    for v in (-1, 0, 5, 7, 8, 10, 11, 13):
        ctx.set_traversal(v)
    for v in (-2, 1, 2, 3, 4, 6, 9, 12, 14, 31, 32):
        with pytest.raises(emst.EmstError) as ei:
            ctx.set_traversal(v)
        assert ei.value.name == "EMST_EINVAL"


def test_serving_results_equal_alone_and_in_the_mix():
    import paper_2207_00514_amd as emst
    from paper_2207_00514_amd import serve
    sizes = np.clip(W.request_sizes(48, seed=51), 500, 40_000).astype(int)
    # one request above the query-list threshold (3 * 2^18 points), so a
    # batch holding it runs the list rounds
    sizes[20] = 900_000
    reqs = [serve.Request(rid=i, points=W.request_cloud(int(n), seed=1000 + i)) for i, n in enumerate(sizes)]
    rng = np.random.default_rng(52)
    arrivals = np.cumsum(rng.exponential(0.002, len(reqs))).tolist()
    server = serve.Server(workers=2, budget_bytes=1 << 30, max_batch=16)
    serve.replay(server, reqs, arrivals)
    assert all(r.error is None for r in reqs)
    assert len({r.batch for r in reqs}) < len(reqs), "no request was batched with another"
    alone = emst.Context(0)
    for r in reqs:
        print(f"request {r.rid} n={len(r.points)}", flush=True)
        solo = host(alone.build(dev(r.points)))
        assert same_tree((r.edges, r.weights, r.d2), solo), f"request {r.rid}"
        assert same_tree((r.edges, r.weights, r.d2), oracle_tree(r.points)), f"request {r.rid} vs oracle"


def test_serving_rejects_a_request_over_its_share():
    from paper_2207_00514_amd import serve
    server = serve.Server(workers=2, budget_bytes=64 << 20, max_batch=8)
    big = serve.Request(rid=0, points=W.request_cloud(400_000, seed=7))
    small = serve.Request(rid=1, points=W.request_cloud(5_000, seed=8))
    serve.replay(server, [big, small], [0.0, 0.001])
    assert big.error is not None and "share" in big.error
    assert small.error is None and small.edges.shape == (4_999, 2)


def _solve_all(solver, ctx, limit=400):
    done = {}
    for _ in range(limit):
        solver.step()
        for s in list(solver._pending):
            state, _ = solver.poll(s)
            if state != 1:
                done[s] = state
        if all(solver.poll(s)[0] != 1 for s in solver._pending):
            break
    return done


def test_solver_round_granular_admission_equals_alone():
    import paper_2207_00514_amd as emst
    ctx = emst.Context(0)
    alone = emst.Context(0)
    solver = emst.Solver(ctx, 512 << 20, max_slots=16)
    clouds = [W.small_random(n, d, 70 + i, k) for i, (n, d, k) in enumerate(
        [(3000, 3, "uniform"), (20000, 2, "uniform"), (1, 3, "uniform"), (0, 2, "uniform"),
         (5000, 3, "dup"), (40000, 3, "outlier"), (2, 2, "int"), (12000, 3, "int")])]
    # a request above the query-list threshold (3 * 2^18 points) joins too
    clouds.append(W.clustered3d(800_000, seed=79))
    first = [solver.admit(dev(c), tag=i) for i, c in enumerate(clouds[:4])]
    assert None not in first
    solver.step()
    solver.step()
    later = [solver.admit(dev(c), tag=4 + i) for i, c in enumerate(clouds[4:])]  # join mid-flight
    assert None not in later
    slots = first + later
    _solve_all(solver, ctx)
    for i, (s, c) in enumerate(zip(slots, clouds)):
        state, tag = solver.poll(s)
        assert state == 2 and tag == i
        got = host(solver.take(s))
        if len(c) < 2:
            assert got[0].shape == (0, 2)
            continue
        assert same_tree(got, host(alone.build(dev(c)))), f"cloud {i}"
        assert same_tree(got, oracle_tree(c)), f"cloud {i} vs oracle"
    solver.close()


def test_solver_take_many_equals_alone():
    """ready() lists finished slots by cohort and position; take_many copies
    them back to back, each request's rows equal to its build alone; a
    failed slot is refused by take_many and taken alone."""
    import paper_2207_00514_amd as emst
    ctx = emst.Context(0)
    alone = emst.Context(0)
    solver = emst.Solver(ctx, 256 << 20, max_slots=16)
    clouds = [W.small_random(n, d, 90 + i, k) for i, (n, d, k) in enumerate(
        [(4000, 3, "uniform"), (1, 3, "uniform"), (9000, 2, "dup"), (2, 3, "int"), (15000, 3, "outlier")])]
    bad = W.small_random(300, 2, 99)
    bad[3, 0] = np.nan
    slots = [solver.admit(dev(c), tag=i) for i, c in enumerate(clouds[:3])]
    f = solver.admit(dev(bad), tag=99)
    solver.step()
    slots += [solver.admit(dev(c), tag=3 + i) for i, c in enumerate(clouds[3:])]  # a second cohort
    assert None not in slots and f is not None
    _solve_all(solver, ctx)
    ready = solver.ready()
    assert sorted(ready) == sorted(slots + [f])
    with pytest.raises(emst.EmstError) as ei:
        solver.take_many([f] + slots)
    assert ei.value.name == "EMST_EINVAL"
    with pytest.raises(emst.EmstError) as ei:
        solver.take(f)
    assert ei.value.name == "EMST_ENONFINITE"
    order = [s for s in solver.ready()]
    assert sorted(order) == sorted(slots)
    e, w, d, offs = solver.take_many(order)
    e, w, d = host((e, w, d))
    for k, s in enumerate(order):
        c = clouds[slots.index(s)]
        a, b = offs[k], offs[k + 1]
        assert b - a == max(len(c) - 1, 0)
        got = (e[a:b], w[a:b], d[a:b])
        if len(c) < 2:
            continue
        assert same_tree(got, host(alone.build(dev(c)))), f"slot {s}"
    assert solver.ready() == []
    solver.close()


def test_solver_budget_busy_and_failures():
    import paper_2207_00514_amd as emst
    ctx = emst.Context(0)
    one = emst.Solver.slot_bytes(20000, 3)
    solver = emst.Solver(ctx, 2 * one + emst.Solver.slot_bytes(500, 3) + 4096, max_slots=8)
    a = solver.admit(dev(W.small_random(20000, 3, 1)))
    b = solver.admit(dev(W.small_random(20000, 3, 2)))
    assert a is not None and b is not None
    assert solver.admit(dev(W.small_random(20000, 3, 3))) is None        # budget full: EBUSY
    with pytest.raises(emst.EmstError) as ei:
        solver.admit(dev(W.small_random(60000, 3, 4)))                  # larger than the budget
    assert ei.value.name == "EMST_ENOMEM"
    _solve_all(solver, ctx)
    host(solver.take(a))
    c = solver.admit(dev(W.small_random(20000, 3, 3)))                   # fits again
    assert c is not None
    bad = W.small_random(500, 3, 5)
    bad[7, 2] = np.inf
    f = solver.admit(dev(bad))
    assert f is not None
    _solve_all(solver, ctx)
    assert solver.poll(f)[0] == -2
    with pytest.raises(emst.EmstError) as ei:
        solver.take(f)
    assert ei.value.name == "EMST_ENONFINITE"
    for s, seed in ((b, 2), (c, 3)):
        pts = W.small_random(20000, 3, seed)
        assert np.array_equal(host(solver.take(s))[0], oracle.emst(pts, threads=8).edges)
    solver.close()


def test_solver_server_results_equal_alone():
    import paper_2207_00514_amd as emst
    from paper_2207_00514_amd import serve
    sizes = np.clip(W.request_sizes(40, seed=61), 500, 30_000).astype(int)
    reqs = [serve.Request(rid=i, points=W.request_cloud(int(n), seed=2000 + i)) for i, n in enumerate(sizes)]
    rng = np.random.default_rng(62)
    arrivals = np.cumsum(rng.exponential(0.003, len(reqs))).tolist()
    server = serve.SolverServer(budget_bytes=512 << 20, max_slots=32)
    serve.replay(server, reqs, arrivals)
    assert all(r.error is None for r in reqs)
    alone = emst.Context(0)
    for r in reqs:
        assert same_tree((r.edges, r.weights, r.d2), host(alone.build(dev(r.points)))), f"request {r.rid}"
        assert same_tree((r.edges, r.weights, r.d2), oracle_tree(r.points)), f"request {r.rid} vs oracle"
