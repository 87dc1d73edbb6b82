"""CPU oracle for the EMST hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it and shares no code with it.

Contents
--------
* ``prim``          dense O(n^2) Prim under the key K (C, ``emst_oracle.c``)
* ``kdboruvka``     Boruvka over a kd-tree, serial or OpenMP (C)
* ``sqdist``        the float32 squared distance D for one pair (C);
                    ``sqdist_pairs`` for many, ``weights`` the reported
                    weight sqrtf(D)
* ``kruskal_bruteforce``  all n(n-1)/2 keys sorted, then union-find (numpy)
* ``nearest_other_bruteforce``  per-point nearest neighbour in another
                    component under (D, j) (numpy), the per-point step of
                    Section 3 ("Finding the shortest outgoing edge")
* ``radix_tree`` / ``reduce_labels``  the binary radix tree over sorted keys
                    and the bottom-up label propagation of Section 3,
                    Optimization 1 (pure Python; small inputs)
* invariant checkers: spanning tree, cycle property, round structure.
* mutual reachability (Section 4, "Mutual reachability distance"):
  ``core_distances`` (brute force by sorting, or a kd-tree k-nearest
  search), ``prim_mreach`` / ``kdboruvka_mreach`` / ``mreach_mst`` (the MST
  under M(u, v) = max(core2(u), core2(v), D(u, v)) and the same tie-break),
  and the numpy checks ``core_bruteforce`` / ``kruskal_bruteforce(core2=)``.

The key K(u, v) = (bits(D(u, v)), min(u, v), max(u, v)) is the paper's
tie-break (Section 2, Boruvka's algorithm) applied to the float32 squared
distance; the tree minimising it is unique.  Pins for every function live in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "emst_oracle.c")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (contraction off, IEEE semantics)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        f32p = ctypes.POINTER(ctypes.c_float)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.oracle_sqdist.argtypes = [f32p, f32p, ctypes.c_int]
        L.oracle_sqdist.restype = ctypes.c_float
        L.oracle_sqdist_pairs.argtypes = [f32p, f32p, ctypes.c_int64, ctypes.c_int, f32p]
        L.oracle_sqdist_pairs.restype = None
        L.oracle_weights.argtypes = [f32p, ctypes.c_int64, f32p]
        L.oracle_weights.restype = None
        L.oracle_prim.argtypes = [f32p, ctypes.c_int64, ctypes.c_int, i32p, f32p]
        L.oracle_prim.restype = ctypes.c_int
        L.oracle_kdboruvka.argtypes = [f32p, ctypes.c_int64, ctypes.c_int, i32p, f32p,
                                       ctypes.c_int, i64p, i64p]
        L.oracle_kdboruvka.restype = ctypes.c_int
        L.oracle_canonicalize.argtypes = [ctypes.c_int64, i32p, f32p, f32p]
        L.oracle_canonicalize.restype = ctypes.c_int
        L.oracle_total_weight.argtypes = [ctypes.c_int64, f32p]
        L.oracle_total_weight.restype = ctypes.c_double
        L.oracle_prim_mreach.argtypes = [f32p, ctypes.c_int64, ctypes.c_int, f32p, i32p, f32p]
        L.oracle_prim_mreach.restype = ctypes.c_int
        L.oracle_kdboruvka_mreach.argtypes = [f32p, ctypes.c_int64, ctypes.c_int, f32p, i32p, f32p,
                                              ctypes.c_int, i64p, i64p]
        L.oracle_kdboruvka_mreach.restype = ctypes.c_int
        for f in ("oracle_core_brute", "oracle_core_kd"):
            getattr(L, f).argtypes = [f32p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, f32p, ctypes.c_int]
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _points(points) -> np.ndarray:
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float32))
    if pts.ndim != 2:
        raise ValueError("points must be [n, dim]")
    return pts


def sqdist(a, b) -> np.float32:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float32))
    return np.float32(lib().oracle_sqdist(_p(a, ctypes.c_float), _p(b, ctypes.c_float), a.shape[0]))


def sqdist_pairs(a, b) -> np.ndarray:
    """D of every pair of rows: a, b [m, dim] float32 -> [m] float32."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float32))
    assert a.shape == b.shape and a.ndim == 2
    out = np.empty(a.shape[0], np.float32)
    lib().oracle_sqdist_pairs(_p(a, ctypes.c_float), _p(b, ctypes.c_float), a.shape[0], a.shape[1],
                              _p(out, ctypes.c_float))
    return out


def weights(d2) -> np.ndarray:
    """The reported edge weights: sqrtf(d2), correctly rounded."""
    d = np.ascontiguousarray(np.asarray(d2, dtype=np.float32).reshape(-1))
    out = np.empty_like(d)
    lib().oracle_weights(_p(d, ctypes.c_float), d.shape[0], _p(out, ctypes.c_float))
    return out


class MST:
    """Canonical EMST: edges [m, 2] int32 (u < v), d2 [m] float32, w [m]
    float32 = sqrtf(d2), sorted by K."""

    def __init__(self, edges, d2, w, rounds=None, comps=None):
        self.edges, self.d2, self.w = edges, d2, w
        self.rounds, self.comps = rounds, comps

    @property
    def total_weight(self) -> float:
        """FP64 left-to-right sum of w in canonical order."""
        return float(lib().oracle_total_weight(self.w.shape[0], _p(self.w, ctypes.c_float)))


def canonicalize(edges, d2) -> MST:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2)).copy()
    d = np.ascontiguousarray(np.asarray(d2, dtype=np.float32).reshape(-1)).copy()
    w = np.empty_like(d)
    rc = lib().oracle_canonicalize(d.shape[0], _p(e, ctypes.c_int32), _p(d, ctypes.c_float),
                                   _p(w, ctypes.c_float))
    if rc != 0:
        raise RuntimeError(f"oracle_canonicalize failed: {rc}")
    return MST(e, d, w)


def prim(points) -> MST:
    pts = _points(points)
    n, dim = pts.shape
    m = max(n - 1, 0)
    e = np.zeros((m, 2), np.int32)
    d = np.zeros(m, np.float32)
    rc = lib().oracle_prim(_p(pts, ctypes.c_float), n, dim, _p(e, ctypes.c_int32), _p(d, ctypes.c_float))
    if rc != 0:
        raise RuntimeError(f"oracle_prim failed: {rc}")
    return canonicalize(e, d)


def kdboruvka(points, threads: int = 1) -> MST:
    pts = _points(points)
    n, dim = pts.shape
    m = max(n - 1, 0)
    e = np.zeros((m, 2), np.int32)
    d = np.zeros(m, np.float32)
    rounds = np.zeros(1, np.int64)
    comps = np.zeros(64, np.int64)
    rc = lib().oracle_kdboruvka(_p(pts, ctypes.c_float), n, dim, _p(e, ctypes.c_int32),
                                _p(d, ctypes.c_float), int(threads), _p(rounds, ctypes.c_int64),
                                _p(comps, ctypes.c_int64))
    if rc != 0:
        raise RuntimeError(f"oracle_kdboruvka failed: {rc}")
    out = canonicalize(e, d)
    out.rounds = int(rounds[0])
    out.comps = comps[:out.rounds].copy()
    return out


def emst(points, threads: int = 1) -> MST:
    """The oracle's answer for any size: Prim for small n, kd-Boruvka above."""
    pts = _points(points)
    if pts.shape[0] <= 4000:
        return prim(pts)
    return kdboruvka(pts, threads=threads)


# ----------------------------------------------------------------------------
# mutual reachability (Section 4, "Mutual reachability distance")


def core_distances(points, k_pts: int, method: str = "kd", threads: int = 1) -> np.ndarray:
    """Squared core distance of every point: the k_pts-th smallest of the
    values D(u, v) over all v, the point itself (D = 0) included."""
    pts = _points(points)
    n, dim = pts.shape
    out = np.zeros(n, np.float32)
    if n == 0:
        return out
    fn = lib().oracle_core_kd if method == "kd" else lib().oracle_core_brute
    rc = fn(_p(pts, ctypes.c_float), n, dim, int(k_pts), _p(out, ctypes.c_float), int(threads))
    if rc != 0:
        raise RuntimeError(f"core distances failed: {rc}")
    return out


def prim_mreach(points, core2) -> MST:
    pts = _points(points)
    c = np.ascontiguousarray(np.asarray(core2, dtype=np.float32))
    n, dim = pts.shape
    m = max(n - 1, 0)
    e = np.zeros((m, 2), np.int32)
    d = np.zeros(m, np.float32)
    rc = lib().oracle_prim_mreach(_p(pts, ctypes.c_float), n, dim, _p(c, ctypes.c_float),
                                  _p(e, ctypes.c_int32), _p(d, ctypes.c_float))
    if rc != 0:
        raise RuntimeError(f"oracle_prim_mreach failed: {rc}")
    return canonicalize(e, d)


def kdboruvka_mreach(points, core2, threads: int = 1) -> MST:
    pts = _points(points)
    c = np.ascontiguousarray(np.asarray(core2, dtype=np.float32))
    n, dim = pts.shape
    m = max(n - 1, 0)
    e = np.zeros((m, 2), np.int32)
    d = np.zeros(m, np.float32)
    rounds = np.zeros(1, np.int64)
    comps = np.zeros(64, np.int64)
    rc = lib().oracle_kdboruvka_mreach(_p(pts, ctypes.c_float), n, dim, _p(c, ctypes.c_float),
                                       _p(e, ctypes.c_int32), _p(d, ctypes.c_float), int(threads),
                                       _p(rounds, ctypes.c_int64), _p(comps, ctypes.c_int64))
    if rc != 0:
        raise RuntimeError(f"oracle_kdboruvka_mreach failed: {rc}")
    out = canonicalize(e, d)
    out.rounds = int(rounds[0])
    out.comps = comps[:out.rounds].copy()
    return out


def mreach_mst(points, k_pts: int, threads: int = 1):
    """(MST under M, squared core distances) for any size."""
    pts = _points(points)
    core2 = core_distances(pts, k_pts, "kd", threads)
    if pts.shape[0] <= 4000:
        return prim_mreach(pts, core2), core2
    return kdboruvka_mreach(pts, core2, threads), core2


def core_bruteforce(points, k_pts: int) -> np.ndarray:
    """numpy: the k_pts-th smallest entry of every row of the D matrix."""
    D = pair_d2_matrix(points)
    return np.sort(D, axis=1)[:, k_pts - 1].astype(np.float32)


# ----------------------------------------------------------------------------
# numpy brute force (small n)


def pair_d2_matrix(points) -> np.ndarray:
    """All-pairs D as float32, evaluated coordinate by coordinate in the
    fixed order with numpy float32 elementwise arithmetic (no fusion)."""
    pts = _points(points)
    a = pts[:, None, :]
    b = pts[None, :, :]
    dk = a[..., 0] - b[..., 0]
    s = dk * dk
    for k in range(1, pts.shape[1]):
        dk = a[..., k] - b[..., k]
        s = s + dk * dk
    return s.astype(np.float32)


def kruskal_bruteforce(points, core2=None) -> MST:
    """Kruskal (Section 2): sort all pairs by K, add every pair that joins
    two different components (union-find).  With core2, the weight of a
    pair is M = max(core2[u], core2[v], D)."""
    pts = _points(points)
    n = pts.shape[0]
    if n < 2:
        return canonicalize(np.zeros((0, 2), np.int32), np.zeros(0, np.float32))
    D = pair_d2_matrix(pts)
    if core2 is not None:
        c = np.asarray(core2, dtype=np.float32)
        D = np.maximum(np.maximum(D, c[:, None]), c[None, :]).astype(np.float32)
    iu, ju = np.triu_indices(n, k=1)
    w = D[iu, ju].view(np.uint32)
    order = np.lexsort((ju, iu, w))  # primary w, then min (=iu), then max (=ju)
    par = list(range(n))

    def find(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x

    out_e, out_d = [], []
    for k in order:
        a, b = int(iu[k]), int(ju[k])
        ra, rb = find(a), find(b)
        if ra != rb:
            par[max(ra, rb)] = min(ra, rb)
            out_e.append((a, b))
            out_d.append(D[a, b])
            if len(out_e) == n - 1:
                break
    return canonicalize(np.array(out_e, np.int32).reshape(-1, 2), np.array(out_d, np.float32))


def nearest_other_bruteforce(points, labels):
    """Per point i: the j with labels[j] != labels[i] minimising (D, j);
    returns (d2 float32 [n] with +inf for none, j int64 [n] with -1)."""
    pts = _points(points)
    lab = np.asarray(labels).reshape(-1)
    D = pair_d2_matrix(pts).view(np.uint32).astype(np.int64)
    n = pts.shape[0]
    same = lab[:, None] == lab[None, :]
    D[same] = np.int64(1) << 40
    key = D * (n + 1) + np.arange(n)[None, :]
    j = key.argmin(axis=1)
    kmin = key[np.arange(n), j]
    none = (kmin >> 0) >= (np.int64(1) << 40) * (n + 1)
    d2 = pair_d2_matrix(pts)[np.arange(n), j]
    d2 = np.where(none, np.float32(np.inf), d2).astype(np.float32)
    j = np.where(none, -1, j)
    return d2, j


# ----------------------------------------------------------------------------
# invariants


def check_spanning_tree(n: int, edges) -> None:
    e = np.asarray(edges).reshape(-1, 2)
    assert e.shape[0] == max(n - 1, 0), f"expected {max(n - 1, 0)} edges, got {e.shape[0]}"
    if n < 2:
        return
    assert (e[:, 0] < e[:, 1]).all(), "edges must satisfy u < v"
    assert (e[:, 0] >= 0).all() and (e[:, 1] < n).all(), "index out of range"
    par = np.arange(n)

    def find(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x

    for a, b in e.tolist():
        ra, rb = find(a), find(b)
        assert ra != rb, f"edge ({a},{b}) closes a cycle"
        par[max(ra, rb)] = min(ra, rb)


def check_cycle_property(points, mst: MST, core2=None) -> None:
    """Every non-tree pair's key exceeds the largest key on its tree path
    (the cycle property that characterises the unique MST under K; with
    core2, under the key of M).  The edge set must also be a spanning tree
    (check_spanning_tree) and its d2 must be the weights of its own edges:
    the path keys come from the points, not from the tree."""
    pts = _points(points)
    n = pts.shape[0]
    check_spanning_tree(n, mst.edges)
    if n < 2:
        return
    W = pair_d2_matrix(pts)
    if core2 is not None:
        c = np.asarray(core2, dtype=np.float32)
        W = np.maximum(np.maximum(W, c[:, None]), c[None, :]).astype(np.float32)
    D = W.view(np.uint32).astype(np.int64)
    e = np.asarray(mst.edges).reshape(-1, 2)
    # the tree's own weights must be the weights of its edges: the keys below
    # are taken from the points, never from the tree
    claimed = np.asarray(mst.d2, dtype=np.float32).view(np.uint32).astype(np.int64)
    assert np.array_equal(claimed, D[e[:, 0], e[:, 1]]), "tree weights differ from the weights of its edges"
    adj = [[] for _ in range(n)]
    for u, v in e.tolist():
        d = int(D[u, v])
        adj[u].append((v, d))
        adj[v].append((u, d))
    B = np.int64(n + 1)
    for s in range(n):
        # max key on the path from s to every vertex (BFS over the tree)
        mx = np.full(n, -1, np.int64)
        mx[s] = -2
        stack = [s]
        while stack:
            x = stack.pop()
            for y, d in adj[x]:
                if mx[y] == -1:
                    k = (int(d) * B + min(x, y)) * B + max(x, y)
                    mx[y] = max(int(mx[x]), k)
                    stack.append(y)
        assert (mx != -1).all(), f"vertex {int(np.argmax(mx == -1))} is not reachable from {s}"
        ys = np.arange(s + 1, n)
        keys = (D[s, ys] * B + s) * B + ys
        assert (keys >= mx[ys]).all(), f"cycle property violated from vertex {s}"


# ----------------------------------------------------------------------------
# binary radix tree and label propagation (small inputs, pure Python)

INVALID = -1


def radix_tree(codes, code_bits: int = 64):
    """Binary radix tree over sorted codes with equal codes separated by
    their sorted index.  Every internal node is a leaf range [lo, hi] split
    where the first bit (from the most significant one) of the augmented key
    (code, index) changes.  Returns {(lo, hi): ((llo, lhi), (rlo, rhi))}."""
    codes = [int(c) for c in codes]
    n = len(codes)
    assert all(codes[i] <= codes[i + 1] for i in range(n - 1)), "codes must be sorted"
    ibits = max(1, (n - 1).bit_length())
    keys = [(c << ibits) | i for i, c in enumerate(codes)]
    tree = {}

    def build(lo, hi):
        if lo == hi:
            return
        x = keys[lo] ^ keys[hi]
        top = x.bit_length() - 1
        split = lo
        while split < hi and not ((keys[split + 1] >> top) & 1):
            split += 1
        tree[(lo, hi)] = ((lo, split), (split + 1, hi))
        build(lo, split)
        build(split + 1, hi)

    if n >= 2:
        build(0, n - 1)
    return tree


def reduce_labels(tree, leaf_labels):
    """Internal label = the children's common label, else INVALID
    (Section 3, Optimization 1).  Returns {(lo, hi): label}."""
    out = {}

    def lab(node):
        lo, hi = node
        if lo == hi:
            return int(leaf_labels[lo])
        if node in out:
            return out[node]
        l, r = tree[node]
        a, b = lab(l), lab(r)
        out[node] = a if (a == b and a != INVALID) else INVALID
        return out[node]

    for node in tree:
        lab(node)
    return out
