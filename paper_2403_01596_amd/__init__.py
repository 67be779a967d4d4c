"""MI355X near-field P2P operator: Python binding of libp2p (include/p2p.h).

Argument marshalling only: every step of the plan build, the apply and the
reverse pass runs in the HIP library; PyTorch provides device memory and the
stream.  If the library is not built, importing works but the first call raises
(there is no other path to the result).

    plan = Plan(xyz, ids, k, dtype=torch.complex64, layout="tiles")
    y = plan.apply(q)                       # y = A_near q
    dq, dx = plan.backward(q, grad_y)
    y = P2PFunction.apply(xyz, q, plan)     # differentiable in q and xyz
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libp2p.so")

P2P_C64, P2P_C128 = 1, 2
LAYOUTS = {"tiles": 0, "csr": 1}
_STATUS = {0: "ok", 1: "invalid argument", 2: "value out of range", 3: "dtype does not match the plan",
           4: "out of device memory", 5: "HIP runtime error", 6: "invalid plan"}


class P2PError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (%d): %s" % (_STATUS.get(status, "?"), status, message))
        self.status = status


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("layout", ctypes.c_int), ("max_rhs", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("tune_cache", ctypes.c_char_p)]


class _Info(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_boxes", ctypes.c_int64), ("n_nbr", ctypes.c_int64),
                ("n_slots", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("n_zero_pairs", ctypes.c_int64),
                ("tile_entries", ctypes.c_int64), ("device_bytes", ctypes.c_int64), ("t_max", ctypes.c_int32),
                ("quantum_exp", ctypes.c_int32), ("d_mean", ctypes.c_double), ("max_sep", ctypes.c_double),
                ("n_close_pairs", ctypes.c_int64), ("n_targets", ctypes.c_int64), ("n_near_boxes", ctypes.c_int64)]


class _Info2D(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_boxes", ctypes.c_int64), ("layout_bytes", ctypes.c_int64),
                ("n_slots", ctypes.c_int64), ("n_src_entries", ctypes.c_int64), ("t_max", ctypes.c_int32),
                ("record_len", ctypes.c_int32), ("collect_ms", ctypes.c_double), ("transfer_ms", ctypes.c_double)]


_lib = None


def lib():
    """The loaded libp2p; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libp2p.so is not built (python -m paper_2403_01596_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    P, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.p2p_box_ids.argtypes = [P, i64, P, f64, P, P]
    L.p2p_box_ids_noalloc.argtypes = [P, i64, P, f64, P, P]
    L.p2p_leaf_level.argtypes = [P, i64, P, f64, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(f64),
                                 ctypes.POINTER(i32), P]
    L.p2p_plan_create.argtypes = [P, P, i64, f64, ctypes.POINTER(_Opts), P, ctypes.POINTER(ctypes.c_void_p)]
    L.p2p_plan_create_grid.argtypes = [P, i64, P, f64, f64, ctypes.POINTER(_Opts), P, ctypes.POINTER(ctypes.c_void_p)]
    L.p2p_plan_create_st.argtypes = [P, i64, P, i64, P, f64, f64, ctypes.POINTER(_Opts), P,
                                     ctypes.POINTER(ctypes.c_void_p)]
    L.p2p_plan_info.argtypes = [P, ctypes.POINTER(_Info)]
    L.p2p_plan_export.argtypes = [P, P, P, P, P, P]
    L.p2p_apply.argtypes = [P, P, P, i32, ctypes.c_int, P]
    L.p2p_apply_backward.argtypes = [P, P, P, P, P, i32, ctypes.c_int, P]
    L.p2p_plan_destroy.argtypes = [P]
    L.p2p_batch_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), i32, i32, ctypes.POINTER(ctypes.c_void_p)]
    L.p2p_batch_apply.argtypes = [P, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), P]
    L.p2p_batch_tune.argtypes = [P, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                 ctypes.c_char_p, P, ctypes.POINTER(ctypes.c_int32)]
    L.p2p_batch_timing.argtypes = [P, ctypes.c_int]
    L.p2p_batch_timing_read.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.p2p_batch_destroy.argtypes = [P]
    L.p2p_plan_timing.argtypes = [P, ctypes.c_int]
    L.p2p_plan_timing_read.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.p2p2d_collect.argtypes = [ctypes.c_int, P, P, i64, i32, i32, ctypes.POINTER(ctypes.c_void_p)]
    L.p2p2d_transfer.argtypes = [P, P]
    L.p2p2d_run.argtypes = [P, P, P]
    L.p2p2d_info.argtypes = [P, ctypes.POINTER(_Info2D)]
    L.p2p2d_destroy.argtypes = [P]
    L.p2p2d_layout.argtypes = [P, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(i64), P]
    L.p2p_apply_log2d.argtypes = [P, P, P, P]
    L.p2p_last_error.restype = ctypes.c_char_p
    L.p2p_status_str.restype = ctypes.c_char_p
    L.p2p_status_str.argtypes = [ctypes.c_int]
    for name in ("p2p_box_ids", "p2p_box_ids_noalloc", "p2p_leaf_level", "p2p_plan_create", "p2p_plan_create_grid", "p2p_plan_create_st", "p2p_plan_info", "p2p_plan_export", "p2p_apply",
                 "p2p_apply_backward", "p2p_plan_destroy", "p2p_plan_timing", "p2p_plan_timing_read",
                 "p2p_batch_create", "p2p_batch_apply", "p2p_batch_tune", "p2p_batch_timing",
                 "p2p_batch_timing_read", "p2p_batch_destroy", "p2p2d_collect", "p2p2d_transfer", "p2p2d_run",
                 "p2p2d_info", "p2p2d_destroy", "p2p_apply_log2d", "p2p2d_layout"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise P2PError(rc, lib().p2p_last_error().decode(errors="replace"))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _cuda(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    return t.contiguous()


def box_ids(xyz: torch.Tensor, origin, h: float) -> torch.Tensor:
    """floor((xyz - origin) / h) per axis, int32 [n, 3], computed on the device."""
    xyz = _cuda(xyz, torch.float64, "xyz")
    n = xyz.shape[0]
    ids = torch.empty((n, 3), dtype=torch.int32, device=xyz.device)
    o = (ctypes.c_double * 3)(*[float(v) for v in origin])
    _check(lib().p2p_box_ids(_ptr(xyz), n, o, float(h), _ptr(ids), _stream()))
    return ids


def leaf_level(xyz: torch.Tensor, origin, size: float, ct: int = 15, min_level: int = 1):
    """The tree height whose leaf boxes (2^(L-1) per axis over the cube [origin,
    origin + size)^3) hold at most ct points each, smallest from min_level on:
    returns (level, h, t_max).  The paper's clustering-threshold loop (section 3.1)."""
    xyz = _cuda(xyz, torch.float64, "xyz")
    o = (ctypes.c_double * 3)(*[float(v) for v in origin])
    lv, h, t = ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32()
    _check(lib().p2p_leaf_level(_ptr(xyz), xyz.shape[0], o, float(size), int(ct), int(min_level), ctypes.byref(lv),
                                ctypes.byref(h), ctypes.byref(t), _stream()))
    return lv.value, h.value, t.value


def box_ids_noalloc(xyz: torch.Tensor, origin, h: float, out: torch.Tensor) -> torch.Tensor:
    """box_ids into the caller's int32 [n, 3] tensor, through the library's entry point
    that allocates nothing (p2p_box_ids_noalloc)."""
    xyz = _cuda(xyz, torch.float64, "xyz")
    n = xyz.shape[0]
    if not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != torch.int32 or \
            tuple(out.shape) != (n, 3) or not out.is_contiguous():
        raise TypeError("out must be a contiguous int32 CUDA tensor of shape (%d, 3)" % n)
    o = (ctypes.c_double * 3)(*[float(v) for v in origin])
    _check(lib().p2p_box_ids_noalloc(_ptr(xyz), n, o, float(h), _ptr(out), _stream()))
    return out


class Plan:
    """Near-field plan of one point set: boxes, neighbour lists and source lists on the device."""

    def __init__(self, xyz: torch.Tensor, ids: torch.Tensor, k: float, dtype=torch.complex64, layout: str = "tiles",
                 max_rhs: int = 1, tune_cache: Optional[str] = None):
        if dtype not in (torch.complex64, torch.complex128):
            raise TypeError("dtype must be complex64 or complex128")
        # the positions the plan copies: P2PFunction checks that it is given these
        self._xyz_src, self._xyz_version = xyz, getattr(xyz, "_version", None)
        xyz = _cuda(xyz, torch.float64, "xyz")
        if ids is not None:
            ids = _cuda(ids, torch.int32, "ids")
        if xyz.dim() != 2 or xyz.shape[1] != 3 or (ids is not None and ids.shape != xyz.shape):
            raise ValueError("xyz and ids must both be [n, 3]")
        self.dtype = dtype
        self.layout = layout
        self.k = float(k)
        self.n = xyz.shape[0]
        sets = getattr(self, "_sets", None)  # (n_targets, sources) from from_sets
        self.n_targets = self.n if sets is None else sets[0]
        self.n_sources = self.n if sets is None else sets[1].shape[0]
        self.max_rhs = int(max_rhs)
        self.device = xyz.device
        opts = _Opts(P2P_C64 if dtype == torch.complex64 else P2P_C128, LAYOUTS[layout], self.max_rhs, 0,
                     tune_cache.encode() if tune_cache else None)
        h = ctypes.c_void_p()
        if sets is not None:  # distinct target and source sets (from_sets): xyz holds the targets
            src = _cuda(sets[1], torch.float64, "sources")
            org = (ctypes.c_double * 3)(*self._grid[0])
            _check(lib().p2p_plan_create_st(_ptr(xyz), self.n_targets, _ptr(src), self.n_sources, org,
                                            float(self._grid[1]), self.k, ctypes.byref(opts), _stream(),
                                            ctypes.byref(h)))
            self.n = self.n_targets + self.n_sources
        elif ids is None:  # leaf grid given by from_grid
            org = (ctypes.c_double * 3)(*self._grid[0])
            _check(lib().p2p_plan_create_grid(_ptr(xyz), self.n, org, float(self._grid[1]), self.k,
                                              ctypes.byref(opts), _stream(), ctypes.byref(h)))
        else:
            _check(lib().p2p_plan_create(_ptr(xyz), _ptr(ids), self.n, self.k, ctypes.byref(opts), _stream(),
                                         ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_grid(cls, xyz: torch.Tensor, origin, h: float, k: float, dtype=torch.complex64, layout: str = "tiles",
                  max_rhs: int = 1, tune_cache: Optional[str] = None) -> "Plan":
        """The plan with leaf-box ids floor((xyz - origin) / h) computed inside the build."""
        self = cls.__new__(cls)
        self._grid = ([float(v) for v in origin], float(h))
        cls.__init__(self, xyz, None, k, dtype=dtype, layout=layout, max_rhs=max_rhs, tune_cache=tune_cache)
        return self

    @classmethod
    def from_sets(cls, targets: torch.Tensor, sources: torch.Tensor, origin, h: float, k: float,
                  dtype=torch.complex64, layout: str = "tiles", max_rhs: int = 1) -> "Plan":
        """A plan whose targets and sources are distinct point sets, both on the leaf
        grid (origin, h): apply(q) takes q [n_sources(, m)] and returns y
        [n_targets(, m)].  No reverse pass."""
        self = cls.__new__(cls)
        self._grid = ([float(v) for v in origin], float(h))
        sources = _cuda(sources, torch.float64, "sources")
        if sources.dim() != 2 or sources.shape[1] != 3:
            raise ValueError("sources must be [n, 3]")
        self._sets = (targets.shape[0], sources)
        cls.__init__(self, targets, None, k, dtype=dtype, layout=layout, max_rhs=max_rhs)
        self._sets = None
        return self

    @property
    def handle(self):
        if self._h is None:
            raise P2PError(6, "plan has been closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.p2p_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = _Info()
        _check(lib().p2p_plan_info(self.handle, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in _Info._fields_}

    def export(self) -> dict:
        import numpy as np
        inf = self.info()
        B, n = inf["n_boxes"], inf["n_points"]
        out = dict(box_key=np.empty(B, np.uint64), box_start=np.empty(B + 1, np.int32), perm=np.empty(n, np.int32),
                   nbr_start=np.empty(B + 1, np.int32), nbr_idx=np.empty(inf["n_nbr"], np.int32))
        p = lambda a: ctypes.c_void_p(a.ctypes.data)
        _check(lib().p2p_plan_export(self.handle, p(out["box_key"]), p(out["box_start"]), p(out["perm"]),
                                     p(out["nbr_start"]), p(out["nbr_idx"])))
        return out

    def check_positions(self, xyz: torch.Tensor):
        """Raises unless xyz holds the positions the plan was built from.

        The plan keeps its own copy of the positions (sorted, with the quantised
        form of FP32 plans), so positions that moved after the build, in place or
        in another tensor, would give y and dx for the old ones.
        """
        src = self._xyz_src
        if src._version != self._xyz_version:
            raise ValueError("the positions this plan was built from were modified in place since; "
                             "build a new plan for the new positions")
        if xyz is not src:
            if xyz.shape != src.shape or xyz.device != src.device or not torch.equal(xyz.detach(), src.detach()):
                raise ValueError("xyz differs from the positions this plan was built from; build a new plan")

    def apply_log2d(self, q: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """The paper's 2-D potential -ln(r) / (2 pi) over this plan's near pairs (points in
        the plane z = 0 with quadtree ids (bx, by, 0)); q real float64 [n].  FP64 plans."""
        q = _cuda(q, torch.float64, "q")
        if q.shape != (self.n,):
            raise ValueError("q must be [n]")
        y = torch.empty_like(q) if out is None else out
        _check(lib().p2p_apply_log2d(self.handle, _ptr(q), _ptr(y), _stream()))
        return y

    def timing(self, enable: bool = True):
        """Record HIP events around the sweep kernels of later apply/backward calls."""
        _check(lib().p2p_plan_timing(self.handle, 1 if enable else 0))

    def timing_read(self):
        """(summed sweep milliseconds, calls timed) since the last read."""
        ms, calls = ctypes.c_double(), ctypes.c_int64()
        _check(lib().p2p_plan_timing_read(self.handle, ctypes.byref(ms), ctypes.byref(calls)))
        return ms.value, calls.value

    def _rhs(self, q: torch.Tensor, name="q", rows=None):
        q = _cuda(q, self.dtype, name)
        rows = self.n if rows is None else rows
        if q.dim() not in (1, 2) or q.shape[0] != rows:
            raise ValueError("%s must be [%d] or [%d, m]" % (name, rows, rows))
        return q

    def apply(self, q: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        q = self._rhs(q, rows=self.n_sources)
        m = 1 if q.dim() == 1 else q.shape[1]
        shape = (self.n_targets,) + tuple(q.shape[1:])
        y = torch.empty(shape, dtype=q.dtype, device=q.device) if out is None else out
        if tuple(y.shape) != shape or y.dtype != q.dtype or not y.is_contiguous():
            raise ValueError("out must be a contiguous %s tensor of shape %s" % (q.dtype, shape))
        dt = P2P_C64 if self.dtype == torch.complex64 else P2P_C128
        _check(lib().p2p_apply(self.handle, _ptr(q), _ptr(y), m, dt, _stream()))
        return y

    def backward(self, q: torch.Tensor, grad_y: torch.Tensor, want_dq: bool = True, want_dx: bool = True):
        dt = P2P_C64 if self.dtype == torch.complex64 else P2P_C128
        if self.n_targets != self.n or self.n_sources != self.n:  # distinct sets: the library refuses
            _check(lib().p2p_apply_backward(self.handle, None, None, None, None, 1, dt, _stream()))
        q = self._rhs(q)
        gy = self._rhs(grad_y, "grad_y")
        if gy.shape != q.shape:
            raise ValueError("grad_y must be shaped like q")
        m = 1 if q.dim() == 1 else q.shape[1]
        dq = torch.empty_like(q) if want_dq else None
        dx = torch.empty((self.n, 3), dtype=torch.float64, device=q.device) if want_dx else None
        dt = P2P_C64 if self.dtype == torch.complex64 else P2P_C128
        _check(lib().p2p_apply_backward(self.handle, _ptr(q), _ptr(gy), _ptr(dq), _ptr(dx), m, dt, _stream()))
        return dq, dx


class Batch:
    """Several complex64 plans served together for nrhs right-hand sides on the matrix cores.

    One product launch per apply that reads the strengths in each plan's point
    order, no allocation inside the library call and no synchronisation, so
    apply_into can be captured in a graph.  The
    plans must outlive the batch and must have been created with max_rhs >= nrhs.
    """

    def __init__(self, plans, nrhs: int):
        self.plans = list(plans)
        self.nrhs = int(nrhs)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().p2p_batch_create(arr, len(self.plans), self.nrhs, ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise P2PError(6, "batch has been closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.p2p_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, ts, name):
        if len(ts) != len(self.plans):
            raise ValueError("one %s per plan" % name)
        out = []
        for t, p in zip(ts, self.plans):
            if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous():
                raise TypeError("%s must be contiguous complex64 CUDA tensors" % name)
            if tuple(t.shape) != (p.n, self.nrhs):
                raise ValueError("%s must be [n_i, nrhs]" % name)
            out.append(t.data_ptr())
        return (ctypes.c_void_p * len(out))(*out)

    def apply_into(self, qs, ys):
        _check(lib().p2p_batch_apply(self.handle, self._ptrs(qs, "q"), self._ptrs(ys, "y"), _stream()))
        return ys

    def apply(self, qs):
        return self.apply_into(qs, [torch.empty_like(q) for q in qs])

    def tune(self, qs, ys, cache_path: Optional[str] = None):
        """Times the launch shapes on these inputs and keeps the fastest; returns (rhs per item, waves per block)."""
        chosen = (ctypes.c_int32 * 2)()
        path = cache_path.encode() if cache_path else None
        _check(lib().p2p_batch_tune(self.handle, self._ptrs(qs, "q"), self._ptrs(ys, "y"), path, _stream(), chosen))
        return chosen[0], chosen[1]

    def timing(self, enable: bool = True):
        _check(lib().p2p_batch_timing(self.handle, 1 if enable else 0))

    def timing_read(self):
        ms, calls = ctypes.c_double(), ctypes.c_int64()
        _check(lib().p2p_batch_timing_read(self.handle, ctypes.byref(ms), ctypes.byref(calls)))
        return ms.value, calls.value


def apply(plan: Plan, q: torch.Tensor) -> torch.Tensor:
    return plan.apply(q)


METHODS_2D = {"indexing": 0, "repetition": 1}


class Quad2D:
    """One of the paper's two GPU layouts for its 2-D experiment (sections 3.2, 3.3):
    collected on the host from host arrays, copied to the device, swept by its own
    kernel.  xy: numpy float64 [n, 2] in the unit square; q: numpy float64 [n]."""

    def __init__(self, method: str, xy, q, level: int, ct: int = 15):
        import numpy as np
        self.xy = np.ascontiguousarray(xy, dtype=np.float64)
        self.q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        if self.xy.ndim != 2 or self.xy.shape[1] != 2 or self.q.shape[0] != self.xy.shape[0]:
            raise ValueError("xy must be [n, 2] and q [n]")
        self.n = self.xy.shape[0]
        h = ctypes.c_void_p()
        _check(lib().p2p2d_collect(METHODS_2D[method], ctypes.c_void_p(self.xy.ctypes.data),
                                   ctypes.c_void_p(self.q.ctypes.data), self.n, int(level), int(ct), ctypes.byref(h)))
        self._h = h

    def transfer(self):
        _check(lib().p2p2d_transfer(self._h, _stream()))

    def run(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        y = torch.empty(self.n, dtype=torch.float64, device="cuda") if out is None else out
        _check(lib().p2p2d_run(self._h, _ptr(y), _stream()))
        return y

    def info(self) -> dict:
        inf = _Info2D()
        _check(lib().p2p2d_info(self._h, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in _Info2D._fields_}

    def layout(self) -> dict:
        """The collected host layout as numpy views (a copy), by array name."""
        import numpy as np
        data, nbytes = ctypes.c_void_p(), ctypes.c_int64()
        offs = (ctypes.c_int64 * 9)()
        _check(lib().p2p2d_layout(self._h, ctypes.byref(data), ctypes.byref(nbytes), offs))
        raw = np.ctypeslib.as_array((ctypes.c_char * nbytes.value).from_address(data.value)).view(np.uint8).copy()
        inf = self.info()
        n, B = inf["n_points"], inf["n_boxes"]

        def arr(i, dt, count):
            return raw[offs[i]:offs[i] + np.dtype(dt).itemsize * count].view(dt)

        if inf["record_len"] == 0:
            return dict(target_xy=arr(0, np.float64, 2 * n).reshape(n, 2), source_xy=arr(1, np.float64, 2 * n).reshape(n, 2),
                        target_idx=arr(2, np.int32, n), target_start=arr(3, np.int32, B + 1),
                        source_idx=arr(4, np.int32, inf["n_src_entries"]), source_start=arr(5, np.int32, B + 1),
                        q=arr(6, np.float64, n))
        R = inf["record_len"]
        return dict(records=arr(7, np.float64, n * R).reshape(n, R), record_target=arr(8, np.int32, n))

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.p2p2d_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class P2PFunction(torch.autograd.Function):
    """y = A_near(xyz) q, differentiable in q and in the positions.

    The plan fixes the near-field pair set (the ids) and holds the positions it was
    built from; xyz must hold those positions (the tensor the plan was built from,
    unmodified, or one equal to it), else forward raises.  Gradients follow the
    real-loss convention grad = dL/dRe + i dL/dIm.
    """

    @staticmethod
    def forward(ctx, xyz: torch.Tensor, q: torch.Tensor, plan: Plan):
        plan.check_positions(xyz)
        ctx.plan = plan
        ctx.save_for_backward(q)
        return plan.apply(q)

    @staticmethod
    def backward(ctx, grad_y: torch.Tensor):
        (q,) = ctx.saved_tensors
        want_dx, want_dq = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        dq, dx = ctx.plan.backward(q, grad_y.contiguous(), want_dq=want_dq, want_dx=want_dx)
        return dx, dq, None
