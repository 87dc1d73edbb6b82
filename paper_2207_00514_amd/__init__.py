"""Single-tree Boruvka EMST on MI355X (gfx950).

A thin ctypes binding over ``libemst.so`` (C ABI in ``include/emst.h``):
argument marshalling only, every step of the EMST runs in the HIP kernels.
PyTorch provides device memory and streams.

    import torch, paper_2207_00514_amd as emst
    pts = torch.rand(10_000, 3, device="cuda")
    edges, weights, d2 = emst.build(pts)

The library is required: if ``libemst.so`` is missing or fails to load,
every call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import contextlib
import ctypes
import os

from . import workloads  # noqa: F401  (seeded input generators)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libemst.so")

EMST_OK = 0
EMST_EBUSY = -6
ERRORS = {
    -1: "EMST_EINVAL", -2: "EMST_ENONFINITE", -3: "EMST_ERANGE", -4: "EMST_ENOMEM",
    -5: "EMST_EHIP", -6: "EMST_EBUSY", -7: "EMST_EINTERNAL",
}

EXPORTS = [
    "emst_create", "emst_destroy", "emst_last_error", "emst_workspace_bytes", "emst_build",
    "emst_set_profiling", "emst_set_counting", "emst_set_traversal", "emst_get_stats",
    "emst_test_tree_from_codes", "emst_test_radix_sort",
    "emst_workspace_bytes_batched", "emst_build_batched", "emst_test_tree_boxes",
    "emst_core_distances", "emst_build_mreach", "emst_set_autotune", "emst_get_autotune",
    "emst_solver_slot_bytes", "emst_solver_create", "emst_solver_destroy", "emst_solver_admit",
    "emst_solver_step", "emst_solver_poll", "emst_solver_ready", "emst_solver_take",
    "emst_solver_take_many",
    "emst_test_round", "emst_test_distances", "emst_test_weights",
    "emst_set_graphs", "emst_set_lds_depth", "emst_build_noalloc",
]


class EmstError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("dim", ctypes.c_int32), ("rounds", ctypes.c_int32),
        ("components", ctypes.c_int64 * 64), ("tree_height", ctypes.c_int32),
        ("traversal_launches", ctypes.c_int32), ("traversal_ms", ctypes.c_double),
        ("traversal_ms_round", ctypes.c_double * 64), ("tree_ms", ctypes.c_double),
        ("rounds_ms", ctypes.c_double), ("finalize_ms", ctypes.c_double),
        ("total_ms", ctypes.c_double), ("child_tests", ctypes.c_int64),
        ("leaf_tests", ctypes.c_int64), ("child_tests_round", ctypes.c_int64 * 64),
        ("leaf_tests_round", ctypes.c_int64 * 64), ("dist_evals", ctypes.c_int64),
        ("traversal_variant", ctypes.c_int32), ("rank_codes", ctypes.c_int32),
        ("queries_round", ctypes.c_int64 * 64), ("records_touched_round", ctypes.c_int64 * 64),
        ("traversal_lds_depth", ctypes.c_int32), ("pad_", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        r = self.rounds
        return dict(
            n=self.n, dim=self.dim, rounds=r, components=list(self.components[:r]),
            tree_height=self.tree_height, traversal_ms=self.traversal_ms,
            traversal_ms_round=list(self.traversal_ms_round[:r]), tree_ms=self.tree_ms,
            rounds_ms=self.rounds_ms, finalize_ms=self.finalize_ms, total_ms=self.total_ms,
            child_tests=self.child_tests, leaf_tests=self.leaf_tests,
            child_tests_round=list(self.child_tests_round[:r]),
            leaf_tests_round=list(self.leaf_tests_round[:r]), dist_evals=self.dist_evals,
            traversal_variant=self.traversal_variant, rank_codes=self.rank_codes,
            queries_round=list(self.queries_round[:r]),
            records_touched_round=list(self.records_touched_round[:r]),
            traversal_lds_depth=self.traversal_lds_depth,
        )


_lib = None


def lib():
    """Load libemst.so (raises if it is missing: no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "or python -m paper_2207_00514_amd._build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
        L.emst_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.c_char_p]
        L.emst_create.restype = i32
        L.emst_destroy.argtypes = [vp]
        L.emst_destroy.restype = None
        L.emst_last_error.argtypes = [vp]
        L.emst_last_error.restype = ctypes.c_char_p
        L.emst_workspace_bytes.argtypes = [i64, i32]
        L.emst_workspace_bytes.restype = sz
        L.emst_build.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp, sz, vp]
        L.emst_core_distances.argtypes = [vp, vp, i64, i32, i32, vp, vp, sz, vp]
        L.emst_core_distances.restype = i32
        L.emst_build_mreach.argtypes = [vp, vp, i64, i32, i32, vp, vp, vp, vp, vp, sz, vp]
        L.emst_build_mreach.restype = i32
        L.emst_build.restype = i32
        L.emst_build_noalloc.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp]
        L.emst_build_noalloc.restype = i32
        for f in ("emst_set_profiling", "emst_set_counting", "emst_set_traversal", "emst_set_graphs",
                  "emst_set_lds_depth"):
            getattr(L, f).argtypes = [vp, i32]
            getattr(L, f).restype = i32
        L.emst_set_autotune.argtypes = [vp, ctypes.c_char_p]
        L.emst_set_autotune.restype = i32
        L.emst_get_autotune.argtypes = [vp, ctypes.c_char_p, sz, ctypes.POINTER(sz)]
        L.emst_get_autotune.restype = i32
        L.emst_solver_slot_bytes.argtypes = [i64, i32]
        L.emst_solver_slot_bytes.restype = sz
        L.emst_solver_create.argtypes = [vp, vp, sz, i32, ctypes.POINTER(vp)]
        L.emst_solver_create.restype = i32
        L.emst_solver_destroy.argtypes = [vp]
        L.emst_solver_destroy.restype = None
        L.emst_solver_admit.argtypes = [vp, vp, i64, i32, i64, vp, ctypes.POINTER(i32)]
        L.emst_solver_admit.restype = i32
        L.emst_solver_step.argtypes = [vp, vp, ctypes.POINTER(i32)]
        L.emst_solver_step.restype = i32
        L.emst_solver_poll.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.emst_solver_poll.restype = i32
        L.emst_solver_ready.argtypes = [vp, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]
        L.emst_solver_ready.restype = i32
        L.emst_solver_take_many.argtypes = [vp, ctypes.POINTER(i32), i32, vp, vp, vp, ctypes.POINTER(i64), vp]
        L.emst_solver_take_many.restype = i32
        L.emst_solver_take.argtypes = [vp, i32, vp, vp, vp, vp]
        L.emst_solver_take.restype = i32
        L.emst_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.emst_get_stats.restype = i32
        L.emst_workspace_bytes_batched.argtypes = [i64, ctypes.c_int32]
        L.emst_workspace_bytes_batched.restype = sz
        L.emst_build_batched.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.c_int32, vp, vp, vp, ctypes.POINTER(ctypes.c_int64), vp, sz, vp]
        L.emst_build_batched.restype = i32
        L.emst_test_tree_from_codes.argtypes = [vp, vp, i64, vp, vp, vp, vp,
                                                ctypes.POINTER(ctypes.c_int32), vp, sz, vp]
        L.emst_test_tree_from_codes.restype = i32
        L.emst_test_tree_boxes.argtypes = [vp, vp, i64, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int32), vp, sz, vp]
        L.emst_test_tree_boxes.restype = i32
        L.emst_test_radix_sort.argtypes = [vp, vp, vp, i64, vp, sz, vp]
        L.emst_test_radix_sort.restype = i32
        L.emst_test_round.argtypes = [vp, vp, i64, i32, vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp,
                                      vp, vp, ctypes.POINTER(ctypes.c_int64), vp, sz, vp]
        L.emst_test_round.restype = i32
        L.emst_test_distances.argtypes = [vp, vp, vp, i64, i32, vp, vp, vp, vp]
        L.emst_test_distances.restype = i32
        L.emst_test_weights.argtypes = [vp, ctypes.c_uint32, i64, vp, vp]
        L.emst_test_weights.restype = i32
        _lib = L
    return _lib


# emst_build_noalloc's static workspace (EMST_NOALLOC_WORKSPACE_BYTES)
NOALLOC_WORKSPACE_BYTES = 64 << 20


def workspace_bytes(n: int, dim: int) -> int:
    return int(lib().emst_workspace_bytes(int(n), int(dim)))


def workspace_bytes_batched(total_points: int, n_clouds: int) -> int:
    return int(lib().emst_workspace_bytes_batched(int(total_points), int(n_clouds)))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """One emst_ctx on one HIP device."""

    def __init__(self, device: int = 0, autotune_json: str | None = None):
        import torch
        self.device = int(device)
        torch.cuda.init()
        h = ctypes.c_void_p()
        rc = lib().emst_create(ctypes.byref(h), self.device,
                               autotune_json.encode() if autotune_json is not None else None)
        if rc != EMST_OK:
            raise EmstError(rc, "emst_create failed")
        self._h = h
        self._ws = None

    def close(self):
        if getattr(self, "_h", None):
            lib().emst_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != EMST_OK:
            raise EmstError(rc, lib().emst_last_error(self._h).decode())

    def set_profiling(self, on: bool = True):
        self._check(lib().emst_set_profiling(self._h, int(bool(on))))

    def set_lds_depth(self, depth: int):
        """LDS stack ring entries per lane of variant 13 (4, 8, 16; 0 = the
        autotune table's choice, else 8)."""
        self._check(lib().emst_set_lds_depth(self._h, int(depth)))

    def set_graphs(self, on: bool = True):
        """Batches: replay captured pairs of rounds (see emst_set_graphs)."""
        self._check(lib().emst_set_graphs(self._h, int(bool(on))))

    def set_counting(self, on: bool = True):
        self._check(lib().emst_set_counting(self._h, int(bool(on))))

    def set_traversal(self, variant: int):
        self._check(lib().emst_set_traversal(self._h, int(variant)))

    def set_autotune(self, table_json: str | None):
        """Install a traversal-shape table (JSON, see include/emst.h); None
        clears it."""
        self._check(lib().emst_set_autotune(self._h, table_json.encode() if table_json is not None else None))

    def get_autotune(self) -> str:
        n = ctypes.c_size_t()
        self._check(lib().emst_get_autotune(self._h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(lib().emst_get_autotune(self._h, buf, n.value, ctypes.byref(n)))
        return buf.value.decode()

    def stats(self) -> dict:
        s = Stats()
        self._check(lib().emst_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def workspace(self, n: int, dim: int):
        """A cached device workspace of at least emst_workspace_bytes(n, dim)."""
        import torch
        need = workspace_bytes(n, dim) + 256
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def _ws_ptr(self, n: int, dim: int):
        ws = self.workspace(n, dim)
        return ctypes.c_void_p((ws.data_ptr() + 255) & ~255), ctypes.c_size_t(workspace_bytes(n, dim))

    def test_tree_from_codes(self, codes, leaf_labels, stream=None):
        """Hierarchy + one label propagation on sorted uint64 codes (int64
        tensor, bit pattern) and int32 leaf labels; returns (left, right,
        label, root) -- see include/emst_test.h."""
        import torch
        n = codes.shape[0]
        left = torch.empty(n - 1, dtype=torch.int32, device=codes.device)
        right = torch.empty_like(left)
        label = torch.empty_like(left)
        root = ctypes.c_int32()
        ws, wsb = self._ws_ptr(n, 3)
        self._check(lib().emst_test_tree_from_codes(
            self._h, ctypes.c_void_p(codes.data_ptr()), int(n), ctypes.c_void_p(leaf_labels.data_ptr()),
            ctypes.c_void_p(left.data_ptr()), ctypes.c_void_p(right.data_ptr()),
            ctypes.c_void_p(label.data_ptr()), ctypes.byref(root), ws, wsb, _stream_handle(stream)))
        return left, right, label, root.value

    def test_tree_boxes(self, points, stream=None):
        """Tree of emst_build on points [n, 3]; returns (left, right, lo, hi,
        root) -- see include/emst_test.h."""
        import torch
        n = points.shape[0]
        left = torch.empty(n - 1, dtype=torch.int32, device=points.device)
        right = torch.empty_like(left)
        lo = torch.empty((n - 1, 3), dtype=torch.float32, device=points.device)
        hi = torch.empty_like(lo)
        root = ctypes.c_int32()
        ws, wsb = self._ws_ptr(n, 3)
        self._check(lib().emst_test_tree_boxes(
            self._h, ctypes.c_void_p(points.data_ptr()), int(n), ctypes.c_void_p(left.data_ptr()),
            ctypes.c_void_p(right.data_ptr()), ctypes.c_void_p(lo.data_ptr()), ctypes.c_void_p(hi.data_ptr()),
            ctypes.byref(root), ws, wsb, _stream_handle(stream)))
        return left, right, lo, hi, root.value

    def test_radix_sort(self, keys, vals, stream=None):
        """Sort (keys int64 bit patterns as uint64, vals int32) in place."""
        n = keys.shape[0]
        ws, wsb = self._ws_ptr(max(n, 2), 3)
        self._check(lib().emst_test_radix_sort(
            self._h, ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()), int(n),
            ws, wsb, _stream_handle(stream)))

    def test_round(self, points, comp, round_: int = 1, variant: int = 13, stream=None):
        """One Boruvka round from the partition `comp` (int32 [n], input
        order); returns a dict of per-point tensors (bound, cand_d, cand_j,
        comp_d2, comp_u, comp_v, comp_out) and ncomp -- see
        include/emst_test.h."""
        import torch
        points = self._check_points(points)
        n, dim = points.shape
        dev = points.device
        f = lambda: torch.empty(n, dtype=torch.float32, device=dev)  # noqa: E731
        i = lambda: torch.empty(n, dtype=torch.int32, device=dev)  # noqa: E731
        out = dict(bound=f(), cand_d=f(), cand_j=i(), comp_d2=f(), comp_u=i(), comp_v=i(), comp_out=i())
        comp = comp.to(device=dev, dtype=torch.int32).contiguous()
        nc = ctypes.c_int64(0)
        ws, wsb = self._ws_ptr(n, dim)
        P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
        self._check(lib().emst_test_round(
            self._h, P(points), int(n), int(dim), P(comp), int(round_), int(variant), P(out["bound"]),
            P(out["cand_d"]), P(out["cand_j"]), P(out["comp_d2"]), P(out["comp_u"]), P(out["comp_v"]),
            P(out["comp_out"]), ctypes.byref(nc), ws, wsb, _stream_handle(stream)))
        out["ncomp"] = nc.value
        return out

    def test_distances(self, a, b, stream=None):
        """(D, box distance to the one-point box, weight) of the kernels for
        every pair of rows of a and b ([m, dim] float32)."""
        import torch
        a, b = self._check_points(a), self._check_points(b)
        m, dim = a.shape
        sq, box, w = (torch.empty(m, dtype=torch.float32, device=a.device) for _ in range(3))
        P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
        self._check(lib().emst_test_distances(self._h, P(a), P(b), int(m), int(dim), P(sq), P(box), P(w),
                                              _stream_handle(stream)))
        return sq, box, w

    def test_weights(self, first: int, count: int, out=None, stream=None):
        """The kernels' weight function on the float32 bit patterns first ..
        first + count - 1."""
        import torch
        if out is None:
            out = torch.empty(count, dtype=torch.float32, device=f"cuda:{self.device}")
        self._check(lib().emst_test_weights(self._h, ctypes.c_uint32(int(first)), int(count),
                                            ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def build(self, points, out=None, want_d2: bool = True, stream=None):
        """EMST of points [n, dim] (float32, on this context's device).
        Returns (edges int32 [n-1, 2], weights float32 [n-1], d2 float32 [n-1]
        or None), sorted by (D, min index, max index)."""
        import torch
        if not isinstance(points, torch.Tensor) or points.device.type != "cuda":
            raise TypeError("points must be a CUDA (HIP) torch tensor")
        if points.dtype != torch.float32 or points.dim() != 2:
            raise TypeError("points must be float32 [n, dim]")
        points = points.contiguous()
        n, dim = points.shape
        m = max(n - 1, 0)
        if out is None:
            edges = torch.empty((m, 2), dtype=torch.int32, device=points.device)
            weights = torch.empty(m, dtype=torch.float32, device=points.device)
            d2 = torch.empty(m, dtype=torch.float32, device=points.device) if want_d2 else None
        else:
            edges, weights, d2 = out
        ws_bytes = workspace_bytes(n, dim) if dim in (2, 3) else 0
        ws = self.workspace(n, dim if dim in (2, 3) else 3)
        base = ws.data_ptr()
        aligned = (base + 255) & ~255
        rc = lib().emst_build(self._h, ctypes.c_void_p(points.data_ptr()), int(n), int(dim),
                              ctypes.c_void_p(edges.data_ptr()), ctypes.c_void_p(weights.data_ptr()),
                              ctypes.c_void_p(d2.data_ptr() if d2 is not None else 0),
                              ctypes.c_void_p(aligned), ctypes.c_size_t(ws_bytes),
                              _stream_handle(stream))
        self._check(rc)
        return edges, weights, d2

    def build_noalloc(self, points, out=None, want_d2: bool = True, stream=None):
        """emst_build_noalloc: as build(), with the library's static device
        workspace instead of a caller workspace (no device allocation in the
        call; at most NOALLOC_WORKSPACE_BYTES of workspace, so a few hundred
        thousand points).  `out` = (edges, weights, d2 or None) preallocated
        by the caller; without it the outputs are allocated here, before the
        call."""
        import torch
        if not isinstance(points, torch.Tensor) or points.device.type != "cuda":
            raise TypeError("points must be a CUDA (HIP) torch tensor")
        if points.dtype != torch.float32 or points.dim() != 2:
            raise TypeError("points must be float32 [n, dim]")
        points = points.contiguous()
        n, dim = points.shape
        m = max(n - 1, 0)
        if out is None:
            edges = torch.empty((m, 2), dtype=torch.int32, device=points.device)
            weights = torch.empty(m, dtype=torch.float32, device=points.device)
            d2 = torch.empty(m, dtype=torch.float32, device=points.device) if want_d2 else None
        else:
            edges, weights, d2 = out
        rc = lib().emst_build_noalloc(self._h, ctypes.c_void_p(points.data_ptr()), int(n), int(dim),
                                      ctypes.c_void_p(edges.data_ptr()), ctypes.c_void_p(weights.data_ptr()),
                                      ctypes.c_void_p(d2.data_ptr() if d2 is not None else 0),
                                      _stream_handle(stream))
        self._check(rc)
        return edges, weights, d2

    @staticmethod
    def _check_points(points):
        import torch
        if not isinstance(points, torch.Tensor) or points.device.type != "cuda":
            raise TypeError("points must be a CUDA (HIP) torch tensor")
        if points.dtype != torch.float32 or points.dim() != 2:
            raise TypeError("points must be float32 [n, dim]")
        return points.contiguous()

    def core_distances(self, points, k_pts: int, stream=None):
        """Squared core distances [n] (float32, input order) of the mutual
        reachability metric: the k_pts-th smallest D from each point, the
        point itself counted."""
        import torch
        points = self._check_points(points)
        n, dim = points.shape
        core2 = torch.empty(n, dtype=torch.float32, device=points.device)
        ws, wsb = self._ws_ptr(n, dim if dim in (2, 3) else 3)
        self._check(lib().emst_core_distances(self._h, ctypes.c_void_p(points.data_ptr()), int(n), int(dim),
                                              int(k_pts), ctypes.c_void_p(core2.data_ptr()), ws, wsb,
                                              _stream_handle(stream)))
        return core2

    def build_mreach(self, points, k_pts: int, want_d2: bool = True, stream=None):
        """MST under the mutual reachability M = max(core2(u), core2(v), D).
        Returns (edges [n-1, 2], weights sqrtf(M) [n-1], M [n-1] or None,
        core2 [n]) sorted by (M, min index, max index)."""
        import torch
        points = self._check_points(points)
        n, dim = points.shape
        m = max(n - 1, 0)
        dev = points.device
        edges = torch.empty((m, 2), dtype=torch.int32, device=dev)
        weights = torch.empty(m, dtype=torch.float32, device=dev)
        d2 = torch.empty(m, dtype=torch.float32, device=dev) if want_d2 else None
        core2 = torch.empty(n, dtype=torch.float32, device=dev)
        ws, wsb = self._ws_ptr(n, dim if dim in (2, 3) else 3)
        self._check(lib().emst_build_mreach(
            self._h, ctypes.c_void_p(points.data_ptr()), int(n), int(dim), int(k_pts),
            ctypes.c_void_p(edges.data_ptr()), ctypes.c_void_p(weights.data_ptr()),
            ctypes.c_void_p(d2.data_ptr() if d2 is not None else 0), ctypes.c_void_p(core2.data_ptr()),
            ws, wsb, _stream_handle(stream)))
        return edges, weights, d2, core2

    def build_batched(self, clouds, want_d2: bool = True, stream=None):
        """EMSTs of a list of clouds ([n_c, dim_c] float32 tensors on this
        device, dims 2 or 3, mixed allowed) in one batched pass.  Returns a
        list of (edges, weights, d2) per cloud (views into shared outputs,
        cloud-local indices)."""
        import torch
        dev = torch.device(f"cuda:{self.device}")
        flat = [c.contiguous().reshape(-1) for c in clouds]
        sizes = [int(c.shape[0]) for c in clouds]
        dims = [int(c.shape[1]) if c.dim() == 2 else 0 for c in clouds]
        points = torch.cat(flat) if flat else torch.empty(0, device=dev)
        return self.build_batched_flat(points, sizes, dims, want_d2=want_d2, stream=stream)

    def build_batched_flat(self, points, sizes, dims, want_d2: bool = True, stream=None):
        """Low-level form: `points` is the flat float32 concatenation, `sizes`
        and `dims` the per-cloud point counts and dimensions."""
        import torch
        B = len(sizes)
        offs = (ctypes.c_int64 * (B + 1))()
        for c in range(B):
            offs[c + 1] = offs[c] + int(sizes[c])
        dims_c = (ctypes.c_int32 * max(B, 1))(*[int(d) for d in dims])
        eoffs = (ctypes.c_int64 * (B + 1))()
        total = int(offs[B])
        m = sum(max(int(n) - 1, 0) for n in sizes)
        dev = points.device
        edges = torch.empty((m, 2), dtype=torch.int32, device=dev)
        weights = torch.empty(m, dtype=torch.float32, device=dev)
        d2 = torch.empty(m, dtype=torch.float32, device=dev) if want_d2 else None
        wsb = workspace_bytes_batched(total, max(B, 1))
        if self._ws is None or self._ws.numel() < wsb + 256:
            self._ws = torch.empty(wsb + 256, dtype=torch.uint8, device=dev)
        base = (self._ws.data_ptr() + 255) & ~255
        rc = lib().emst_build_batched(
            self._h, ctypes.c_void_p(points.data_ptr() if points.numel() else 0), offs, dims_c, int(B),
            ctypes.c_void_p(edges.data_ptr() if m else 0), ctypes.c_void_p(weights.data_ptr() if m else 0),
            ctypes.c_void_p(d2.data_ptr() if (d2 is not None and m) else 0), eoffs, ctypes.c_void_p(base),
            ctypes.c_size_t(wsb), _stream_handle(stream))
        self._check(rc)
        out = []
        for c in range(B):
            a, b = int(eoffs[c]), int(eoffs[c + 1])
            out.append((edges[a:b], weights[a:b], d2[a:b] if d2 is not None else None))
        return out


_default = {}


def context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def build(points, **kw):
    """EMST of a device tensor with the default context of its device."""
    return context(points.device.index or 0).build(points, **kw)


class Solver:
    """Round-granular continuous batching on one context (emst_solver_*):
    ``admit`` requests at any time; ``step`` starts the requests admitted
    since the last step as one cohort and moves every cohort whose phase
    has completed on by one phase; ``ready`` lists the finished slots;
    ``take`` returns a finished result exactly as ``build`` (written on
    ``stream``, by default the current stream)."""

    def __init__(self, ctx: "Context", budget_bytes: int, max_slots: int = 64):
        import torch
        self.ctx = ctx
        self._mem = torch.empty(int(budget_bytes) + 256, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        base = (self._mem.data_ptr() + 255) & ~255
        h = ctypes.c_void_p()
        ctx._check(lib().emst_solver_create(ctx._h, ctypes.c_void_p(base), ctypes.c_size_t(int(budget_bytes)),
                                            int(max_slots), ctypes.byref(h)))
        self._h = h
        self._pending = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().emst_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def slot_bytes(n: int, dim: int) -> int:
        return int(lib().emst_solver_slot_bytes(int(n), int(dim)))

    def admit(self, points, tag: int = 0, stream=None):
        """Slot of the admitted request, or None if no slot or budget is free
        right now (EMST_EBUSY)."""
        points = Context._check_points(points)
        n, dim = points.shape
        slot = ctypes.c_int32(-1)
        rc = lib().emst_solver_admit(self._h, ctypes.c_void_p(points.data_ptr()), int(n), int(dim), int(tag),
                                     _stream_handle(stream), ctypes.byref(slot))
        if rc == EMST_EBUSY:
            return None
        self.ctx._check(rc)
        self._pending[slot.value] = (int(n), points.device)
        return slot.value

    def step(self, stream=None) -> int:
        fin = ctypes.c_int32(0)
        self.ctx._check(lib().emst_solver_step(self._h, _stream_handle(stream), ctypes.byref(fin)))
        return fin.value

    def poll(self, slot: int):
        state = ctypes.c_int32(0)
        tag = ctypes.c_int64(0)
        self.ctx._check(lib().emst_solver_poll(self._h, int(slot), ctypes.byref(state), ctypes.byref(tag)))
        return state.value, tag.value

    def ready(self):
        """Slots whose request finished or failed and is not taken yet."""
        cap = max(len(self._pending), 1)
        buf = (ctypes.c_int32 * cap)()
        count = ctypes.c_int32(0)
        self.ctx._check(lib().emst_solver_ready(self._h, buf, cap, ctypes.byref(count)))
        return list(buf[:count.value])

    def take_many(self, slots, want_d2: bool = True, stream=None):
        """Finished results of `slots` (all state 2; ``ready`` order copies
        in the fewest pieces), concatenated: edges [M, 2], weights [M], d2
        [M] or None, and offsets (k + 1 ints: request i owns rows
        offsets[i]:offsets[i+1])."""
        import torch
        slots = [int(s) for s in slots]
        total = sum(max(self._pending[s][0] - 1, 0) for s in slots)
        device = f"cuda:{self.ctx.device}"
        with torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext():
            edges = torch.empty((total, 2), dtype=torch.int32, device=device)
            weights = torch.empty(total, dtype=torch.float32, device=device)
            d2 = torch.empty(total, dtype=torch.float32, device=device) if want_d2 else None
        arr = (ctypes.c_int32 * max(len(slots), 1))(*slots)
        offs = (ctypes.c_int64 * (len(slots) + 1))()
        self.ctx._check(lib().emst_solver_take_many(self._h, arr, len(slots), ctypes.c_void_p(edges.data_ptr()),
                                                    ctypes.c_void_p(weights.data_ptr()),
                                                    ctypes.c_void_p(d2.data_ptr() if d2 is not None else 0),
                                                    offs, _stream_handle(stream)))
        for s in slots:
            self._pending.pop(s)
        return edges, weights, d2, list(offs)

    def take(self, slot: int, want_d2: bool = True, stream=None):
        import torch
        n, device = self._pending.pop(slot)
        m = max(n - 1, 0)
        with torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext():
            edges = torch.empty((m, 2), dtype=torch.int32, device=device)
            weights = torch.empty(m, dtype=torch.float32, device=device)
            d2 = torch.empty(m, dtype=torch.float32, device=device) if want_d2 else None
        self.ctx._check(lib().emst_solver_take(self._h, int(slot), ctypes.c_void_p(edges.data_ptr()),
                                               ctypes.c_void_p(weights.data_ptr()),
                                               ctypes.c_void_p(d2.data_ptr() if d2 is not None else 0),
                                               _stream_handle(stream)))
        return edges, weights, d2
