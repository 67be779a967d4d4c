"""Seeded synthetic inputs for the near-field P2P operator.

This module holds input recipes only: point clouds, complex source strengths and
the uniform leaf grid (box ids) that the plan consumes.  It contains none of the
operator's arithmetic (no Morton keys, no neighbour search, no kernel
evaluation), so that the oracle and the HIP path can both be fed from it without
sharing any of the method's code.

The paper draws its points at random (section 3.1: randomly generated inputs;
section 4: points distributed at random over a plate).  The workloads below keep
that and lift it to three dimensions: a unit cube (volume), the unit sphere and an
ellipsoid (surfaces, where box occupancy varies strongly).  Every array comes from
``numpy.random.default_rng(seed)`` (PCG64) in a fixed draw order: positions first,
then the real parts of the strengths, then the imaginary parts.  complex64
strengths are rounded from the same float64 draws.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

GRID_BITS = 21            # box ids live in [0, 2**21) on every axis
ID_LIMIT = 1 << GRID_BITS


# ----------------------------------------------------------------------------
# point clouds
# ----------------------------------------------------------------------------
def uniform_cube(n: int, rng: np.random.Generator) -> np.ndarray:
    """n points uniform in [0, 1)^3, float64 [n, 3]."""
    return rng.random((n, 3))


def sphere_surface(n: int, rng: np.random.Generator) -> np.ndarray:
    """n points uniform on the unit sphere (normalised Gaussian vectors)."""
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def ellipsoid_surface(n: int, rng: np.random.Generator, axes=(1.0, 0.5, 0.25)) -> np.ndarray:
    """n points uniform (by area) on the ellipsoid with semi-axes ``axes``.

    A unit-sphere point u maps to (a u_x, b u_y, c u_z); the map stretches area by
    sqrt((b c u_x)^2 + (a c u_y)^2 + (a b u_z)^2), so a candidate is accepted with
    that factor divided by its maximum.  Candidates are drawn in batches until n
    are accepted; the accepted points keep their draw order.
    """
    a, b, c = (float(v) for v in axes)
    fmax = max(b * c, a * c, a * b)
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = int(1.3 * (n - out.shape[0]) / 0.55) + 1024
        u = sphere_surface(m, rng)
        f = np.sqrt((b * c * u[:, 0]) ** 2 + (a * c * u[:, 1]) ** 2 + (a * b * u[:, 2]) ** 2)
        keep = rng.random(m) * fmax < f
        out = np.concatenate([out, u[keep] * np.array([a, b, c])])
    return np.ascontiguousarray(out[:n])


def strengths(n: int, m: int, rng: np.random.Generator, dtype=np.complex128) -> np.ndarray:
    """Complex strengths with real and imaginary parts ~ N(0, 1), shape [n, m]."""
    re = rng.standard_normal((n, m))
    im = rng.standard_normal((n, m))
    if dtype == np.complex64:
        out = np.empty((n, m), np.complex64)
        out.real = re.astype(np.float32)
        out.imag = im.astype(np.float32)
        return out
    return re + 1j * im


# ----------------------------------------------------------------------------
# leaf grid
# ----------------------------------------------------------------------------
def leaf_ids(xyz: np.ndarray, origin, h: float) -> np.ndarray:
    """Integer leaf-box coordinates floor((x - o) / h), int32 [n, 3]."""
    o = np.asarray(origin, dtype=np.float64).reshape(1, 3)
    ids = np.floor((xyz - o) / h)
    if ids.size and (ids.min() < 0 or ids.max() >= ID_LIMIT):
        raise ValueError("leaf grid does not fit in [0, 2^21) per axis")
    return ids.astype(np.int32)


def count_boxes(ids: np.ndarray) -> int:
    """Number of distinct leaf boxes that hold at least one point."""
    if ids.shape[0] == 0:
        return 0
    lin = (ids[:, 0].astype(np.int64) << 42) | (ids[:, 1].astype(np.int64) << 21) | ids[:, 2].astype(np.int64)
    lin.sort()
    return int(1 + np.count_nonzero(lin[1:] != lin[:-1]))


def grid_for_density(xyz: np.ndarray, d_target: float, tol: float = 0.02, max_iter: int = 80):
    """Leaf size h (and origin) whose mean occupancy of non-empty boxes is d_target.

    Bisection on log h; the origin is the bounding-box minimum minus h/2.
    Returns (h, origin, ids, achieved D).
    """
    lo_pt = xyz.min(axis=0)
    extent = float((xyz.max(axis=0) - lo_pt).max())
    n = xyz.shape[0]
    h_lo, h_hi = extent * 1e-5, extent * 2.0
    best = None
    for _ in range(max_iter):
        h = math.sqrt(h_lo * h_hi)
        origin = lo_pt - h / 2
        ids = leaf_ids(xyz, origin, h)
        d = n / count_boxes(ids)
        if best is None or abs(d / d_target - 1) < abs(best[3] / d_target - 1):
            best = (h, origin, ids, d)
        if abs(d / d_target - 1) <= tol:
            break
        if d < d_target:
            h_lo = h
        else:
            h_hi = h
    return best


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Instance:
    name: str
    xyz: np.ndarray          # float64 [n, 3]
    ids: np.ndarray          # int32 [n, 3]
    q: np.ndarray            # complex [n, m]
    k: float
    h: float
    origin: np.ndarray
    d_mean: float            # N / non-empty boxes

    @property
    def n(self) -> int:
        return self.xyz.shape[0]

    @property
    def m(self) -> int:
        return self.q.shape[1]


def _finish(name, xyz, rng, m, dtype, k, h=None, origin=None, d_target=None):
    if h is None:
        h, origin, ids, d = grid_for_density(xyz, d_target)
    else:
        origin = np.asarray(origin, dtype=np.float64)
        ids = leaf_ids(xyz, origin, h)
        d = xyz.shape[0] / max(1, count_boxes(ids))
    q = strengths(xyz.shape[0], m, rng, dtype)
    return Instance(name, np.ascontiguousarray(xyz), np.ascontiguousarray(ids), q, float(k), float(h),
                    np.asarray(origin, np.float64), float(d))


def cube(n: int, grid: int, k: float, seed: int = 0, m: int = 1, dtype=np.complex128, name="cube") -> Instance:
    """Uniform unit cube on a full grid^3 leaf grid (h = 1/grid, origin 0)."""
    rng = np.random.default_rng(seed)
    xyz = uniform_cube(n, rng)
    return _finish(name, xyz, rng, m, dtype, k, h=1.0 / grid, origin=(0.0, 0.0, 0.0))


def sphere(n: int, d_target: float, k: float, seed: int = 0, m: int = 1, dtype=np.complex64,
           name="sphere") -> Instance:
    rng = np.random.default_rng(seed)
    xyz = sphere_surface(n, rng)
    return _finish(name, xyz, rng, m, dtype, k, d_target=d_target)


def ellipsoid(n: int, d_target: float, k: Optional[float] = None, seed: int = 0, m: int = 1,
              dtype=np.complex64, name="ellipsoid") -> Instance:
    """Ellipsoid (1, 0.5, 0.25).  k=None picks k = pi / (2h): a leaf box is a quarter wavelength."""
    rng = np.random.default_rng(seed)
    xyz = ellipsoid_surface(n, rng)
    h, origin, ids, d = grid_for_density(xyz, d_target)
    kk = math.pi / (2 * h) if k is None else k
    q = strengths(n, m, rng, dtype)
    return Instance(name, xyz, ids, q, float(kk), float(h), origin, float(d))


# The five workloads of the operator's evaluation, by what they are.
def plain_f64_cube() -> Instance:
    """8192 points uniform in the unit cube, 8^3 leaf grid, k = 2 pi * 4, complex128, 1 RHS."""
    return cube(8192, 8, 2 * math.pi * 4, seed=0, m=1, dtype=np.complex128, name="cube8192_g8_k8pi_c128")


def sphere_2m() -> Instance:
    """2M points on the unit sphere, ~32 per non-empty box, k = 2 pi * 64, complex64, 1 RHS."""
    return sphere(2_000_000, 32, 2 * math.pi * 64, seed=0, m=1, dtype=np.complex64, name="sphere2M_D32_k128pi")


def ellipsoid_4m(d_target: int) -> Instance:
    """4M points on the (1, .5, .25) ellipsoid, D in {16, 32, 64}, box = lambda/4, complex64."""
    return ellipsoid(4_000_000, d_target, None, seed=0, m=1, dtype=np.complex64,
                     name="ellipsoid4M_D%d" % d_target)


def multi_rhs_main(m: int = 64) -> Instance:
    """1M sphere points, ~32 per box, k = 2 pi * 32, m complex64 RHS."""
    return sphere(1_000_000, 32, 2 * math.pi * 32, seed=0, m=m, dtype=np.complex64, name="sphere1M_D32_m%d" % m)


def uneven_sizes(count: int = 16) -> List[int]:
    """Instance sizes n_j = round(1e4 * 20^(j/15)), 10k .. 200k points."""
    return [int(round(1e4 * 20.0 ** (j / (count - 1)))) for j in range(count)]


def multi_rhs_batch(m: int = 64, count: int = 16, scale: float = 1.0) -> List[Instance]:
    """The uneven batch: sphere instances of the sizes above (times ``scale``), seeds 1..count."""
    out = []
    for j, nj in enumerate(uneven_sizes(count)):
        nn = max(64, int(round(nj * scale)))
        out.append(sphere(nn, 32, 2 * math.pi * 32, seed=j + 1, m=m, dtype=np.complex64,
                          name="sphere%d_D32_m%d_s%d" % (nn, m, j + 1)))
    return out


def grad_cube_500k() -> Instance:
    """500k points uniform in the unit cube, 25^3 grid (~32 per box), k = 2 pi * 16, complex64."""
    return cube(500_000, 25, 2 * math.pi * 16, seed=0, m=1, dtype=np.complex64, name="cube500k_g25_k32pi")
