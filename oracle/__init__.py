"""FP64 CPU oracle for the near-field P2P operator (ctypes binding of oracle.cpp).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does, and this
package imports nothing from the product.

Pins (tests/test_oracle_*.py): numpy brute force over all pairs on small inputs,
closed forms (two points, the 3x3x3 lattice, the r -> 0 limit of Im G, the
spherical-mean identity of the Helmholtz kernel), invariants (reciprocity,
translation, k = 0 realness, neighbour counts on full grids) and, for the
gradients, exact finite differences in q, dual numbers and the translation,
rotation and scaling identities in x.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.cpp with g++ (no FMA contraction, OpenMP)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               _SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    L = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.orc_box_ids.argtypes = [P, i64, P, f64, P]
    L.orc_morton.argtypes = [i32, i32, i32]
    L.orc_morton.restype = ctypes.c_uint64
    L.orc_plan_build.argtypes = [P, i64, ctypes.POINTER(ctypes.c_void_p)]
    L.orc_plan_free.argtypes = [P]
    L.orc_plan_nboxes.argtypes = [P]
    L.orc_plan_nboxes.restype = i64
    L.orc_plan_nnbr.argtypes = [P]
    L.orc_plan_nnbr.restype = i64
    L.orc_plan_export.argtypes = [P, P, P, P, P, P]
    L.orc_plan_stats.argtypes = [P, P, P, P, P]
    L.orc_apply.argtypes = [P, P, f64, P, ctypes.c_int, P, ctypes.c_int]
    L.orc_apply_rows.argtypes = [P, P, f64, P, ctypes.c_int, P, i64, P, ctypes.c_int]
    L.orc_backward.argtypes = [P, P, f64, P, P, ctypes.c_int, P, P, ctypes.c_int]
    L.orc_dual_dx.argtypes = [P, P, f64, P, ctypes.c_int, i64, ctypes.c_int, P]
    L.orc2d_apply.argtypes = [P, P, i64, i32, P, ctypes.c_int]
    L.orc2d_stats.argtypes = [P, i64, i32, P, P, P, P]
    _lib = L
    return L


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _c128(q: np.ndarray) -> np.ndarray:
    q = np.asarray(q)
    if q.ndim == 1:
        q = q[:, None]
    return np.ascontiguousarray(q.astype(np.complex128))


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError("%s failed with status %d" % (what, rc))


def morton(ix: int, iy: int, iz: int) -> int:
    return int(_load().orc_morton(ix, iy, iz))


def box_ids(xyz: np.ndarray, origin, h: float) -> np.ndarray:
    L = _load()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    ids = np.empty((xyz.shape[0], 3), np.int32)
    _check(L.orc_box_ids(_ptr(xyz), xyz.shape[0], _ptr(o), float(h), _ptr(ids)), "orc_box_ids")
    return ids


class Plan:
    """Box table and neighbour lists of one point set (ids are the leaf-box coordinates)."""

    def __init__(self, ids: np.ndarray):
        L = _load()
        self._ids = np.ascontiguousarray(ids, dtype=np.int32)
        self.n = self._ids.shape[0]
        h = ctypes.c_void_p()
        _check(L.orc_plan_build(_ptr(self._ids), self.n, ctypes.byref(h)), "orc_plan_build")
        self._h = h
        self.n_boxes = int(L.orc_plan_nboxes(h))
        self.n_nbr = int(L.orc_plan_nnbr(h))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_plan_free(self._h)
            self._h = None

    def tables(self):
        """box_key u64[B], box_start i32[B+1], perm i32[N], nbr_start i32[B+1], nbr_idx i32[nnz]."""
        bk = np.empty(self.n_boxes, np.uint64)
        bs = np.empty(self.n_boxes + 1, np.int32)
        pm = np.empty(self.n, np.int32)
        ns = np.empty(self.n_boxes + 1, np.int32)
        ni = np.empty(self.n_nbr, np.int32)
        _load().orc_plan_export(self._h, _ptr(bk), _ptr(bs), _ptr(pm), _ptr(ns), _ptr(ni))
        return dict(box_key=bk, box_start=bs, perm=pm, nbr_start=ns, nbr_idx=ni)

    def stats(self, xyz: np.ndarray):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _load().orc_plan_stats(self._h, _ptr(xyz), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return dict(n_pairs=a.value, n_zero_pairs=b.value, t_max=c.value)

    def apply(self, xyz: np.ndarray, k: float, q: np.ndarray, threads: int = 0) -> np.ndarray:
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        qq = _c128(q)
        y = np.empty_like(qq)
        _check(_load().orc_apply(self._h, _ptr(xyz), float(k), _ptr(qq), qq.shape[1], _ptr(y), threads),
               "orc_apply")
        return y

    def apply_rows(self, xyz: np.ndarray, k: float, q: np.ndarray, rows, threads: int = 0) -> np.ndarray:
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        qq = _c128(q)
        rr = np.ascontiguousarray(rows, dtype=np.int64)
        y = np.empty((rr.shape[0], qq.shape[1]), np.complex128)
        _check(_load().orc_apply_rows(self._h, _ptr(xyz), float(k), _ptr(qq), qq.shape[1], _ptr(rr), rr.shape[0],
                                      _ptr(y), threads), "orc_apply_rows")
        return y

    def backward(self, xyz: np.ndarray, k: float, q: np.ndarray, g: np.ndarray, want_dq=True, want_dx=True,
                 threads: int = 0):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        qq, gg = _c128(q), _c128(g)
        dq = np.empty_like(qq) if want_dq else None
        dx = np.empty((self.n, 3), np.float64) if want_dx else None
        _check(_load().orc_backward(self._h, _ptr(xyz), float(k), _ptr(qq), _ptr(gg), qq.shape[1], _ptr(dq),
                                    _ptr(dx), threads), "orc_backward")
        return dq, dx

    def dual_dx(self, xyz: np.ndarray, k: float, q: np.ndarray, i: int, a: int) -> float:
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        qq = _c128(q)
        out = ctypes.c_double()
        _check(_load().orc_dual_dx(self._h, _ptr(xyz), float(k), _ptr(qq), qq.shape[1], int(i), int(a),
                                   ctypes.byref(out)), "orc_dual_dx")
        return out.value

    def near_rows(self, i: int) -> np.ndarray:
        """Original indices of every point near point i (i included)."""
        t = self.tables()
        pos = np.empty(self.n, np.int64)
        pos[t["perm"]] = np.arange(self.n)
        T = np.searchsorted(t["box_start"], pos[i], side="right") - 1
        rows = []
        for e in range(t["nbr_start"][T], t["nbr_start"][T + 1]):
            S = t["nbr_idx"][e]
            rows.append(t["perm"][t["box_start"][S]:t["box_start"][S + 1]])
        return np.concatenate(rows)


# ----------------------------------------------------------------------------
# the paper's two-dimensional setting (a quadtree over the unit square)
# ----------------------------------------------------------------------------
def apply2d(xy: np.ndarray, q: np.ndarray, level: int, threads: int = 0) -> np.ndarray:
    """y_i = sum over the nine boxes around i's leaf box (quadtree of height level on
    the unit square), x_j != x_i, of -ln|x_i - x_j| / (2 pi) q_j; q, y real."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    qq = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    y = np.empty(xy.shape[0], np.float64)
    _check(_load().orc2d_apply(_ptr(xy), _ptr(qq), xy.shape[0], int(level), _ptr(y), threads), "orc2d_apply")
    return y


def stats2d(xy: np.ndarray, level: int) -> dict:
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    a, b, c, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    _check(_load().orc2d_stats(_ptr(xy), xy.shape[0], int(level), ctypes.byref(a), ctypes.byref(b),
                               ctypes.byref(c), ctypes.byref(d)), "orc2d_stats")
    return dict(n_pairs=a.value, n_zero_pairs=b.value, t_max=c.value, n_boxes=d.value)
