"""Pins for the oracle's forward near-field sum (CPU only).

Each check fixes something the oracle could plausibly get wrong: the dense
all-pairs sum (a dropped or extra neighbour box, a wrong skip rule), closed forms
on hand-built configurations, the r -> 0 limit of the imaginary part (the sign of
the phase), the spherical-mean identity of the Helmholtz kernel (the magnitude,
the wavenumber scaling), reciprocity, translation invariance and the k = 0
Laplace limit.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from _brute import dense_apply, dense_pair_count


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def G(r, k):
    return np.exp(1j * k * r) / (4 * np.pi * r)


# --------------------------------------------------------------------------
# dense brute force
# --------------------------------------------------------------------------
def small_cases():
    rng = np.random.default_rng(5)
    cube = W.cube(1500, 5, 7.3, seed=1, m=1)
    yield "cube_g5", cube.xyz, cube.ids, cube.k, cube.q
    sph = W.sphere(2000, 8, 2 * math.pi * 3, seed=2, m=2, dtype=np.complex128)
    yield "sphere_D8_m2", sph.xyz, sph.ids, sph.k, sph.q
    # duplicates at distinct indices and a few collinear points
    x = rng.random((600, 3))
    x[100:110] = x[0]
    x[200] = x[201]
    ids = W.leaf_ids(x, (0, 0, 0), 0.25)
    yield "duplicates", x, ids, 11.0, W.strengths(600, 1, rng)
    # ids that do not follow the positions: the near field is defined by the ids
    x = rng.random((700, 3))
    ids = rng.integers(0, 4, size=(700, 3)).astype(np.int32)
    yield "ids_not_positions", x, ids, 2.5, W.strengths(700, 1, rng)
    # hollow grid, boundary and empty boxes, k = 0
    x = rng.random((900, 3)) * 6
    keep = ~np.all((x >= 1) & (x < 5), axis=1)
    x = x[keep]
    ids = W.leaf_ids(x, (0, 0, 0), 1.0)
    yield "hollow_k0", x, ids, 0.0, W.strengths(x.shape[0], 1, rng)


@pytest.mark.parametrize("case", list(small_cases()), ids=lambda c: c[0])
def test_matches_dense_brute_force(case):
    _, xyz, ids, k, q = case
    P = oracle.Plan(ids)
    y = P.apply(xyz, k, q)
    yb = dense_apply(xyz, ids, k, q)
    assert rel_l2(y, yb) < 1e-13
    np.testing.assert_allclose(y, yb, rtol=1e-11, atol=1e-12 * np.abs(yb).max())
    st = P.stats(xyz)
    assert st["n_pairs"] == dense_pair_count(xyz, ids)


def test_pair_counts_add_up():
    inst = W.cube(3000, 6, 1.0, seed=4)
    P = oracle.Plan(inst.ids)
    t = P.tables()
    nb = np.diff(t["box_start"])
    total = sum(int(nb[T]) * int(sum(nb[S] for S in t["nbr_idx"][t["nbr_start"][T]:t["nbr_start"][T + 1]]))
                for T in range(P.n_boxes))
    st = P.stats(inst.xyz)
    assert st["n_pairs"] + st["n_zero_pairs"] == total
    assert st["n_zero_pairs"] == inst.n  # distinct random points: only the self pairs
    assert st["t_max"] == nb.max()


def test_pair_count_full_grid_expectation():
    # Uniform points on a full g^3 grid: E[n_pairs] = (3g - 2)^3 N (N - 1) / g^6.
    inst = W.plain_f64_cube()
    P = oracle.Plan(inst.ids)
    g, n = 8, inst.n
    expect = (3 * g - 2) ** 3 * n * (n - 1) / g ** 6
    assert abs(P.stats(inst.xyz)["n_pairs"] / expect - 1) < 0.03


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k", [0.0, 1.7, 40.0])
def test_two_points(k):
    r = 0.0123
    x = np.array([[0.1, 0.2, 0.3], [0.1 + r * 0.6, 0.2 + r * 0.8, 0.3]])
    ids = np.zeros((2, 3), np.int32)
    q = np.array([[1.5 - 0.5j], [-0.25 + 2.0j]])
    y = oracle.Plan(ids).apply(x, k, q)
    rr = np.sqrt(((x[0] - x[1]) ** 2).sum())
    assert abs(y[0, 0] - q[1, 0] * G(rr, k)) < 1e-14 * abs(y[0, 0])
    assert abs(y[1, 0] - q[0, 0] * G(rr, k)) < 1e-14 * abs(y[1, 0])
    # the same two points in boxes two apart do not interact
    ids2 = np.array([[0, 0, 0], [2, 0, 0]], np.int32)
    assert np.all(oracle.Plan(ids2).apply(x, k, q) == 0)


@pytest.mark.parametrize("k", [0.0, 3.0, 25.0])
def test_lattice_3x3x3(k):
    a = 0.37
    ax = np.arange(3)
    cells = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3)
    x = cells * a + 0.01
    y = oracle.Plan(cells.astype(np.int32)).apply(x, k, np.ones((27, 1)))
    centre = np.flatnonzero((cells == 1).all(axis=1))[0]
    corner = np.flatnonzero((cells == 0).all(axis=1))[0]
    s2, s3 = math.sqrt(2), math.sqrt(3)
    want_c = 6 * G(a, k) + 12 * G(s2 * a, k) + 8 * G(s3 * a, k)
    want_k = 3 * G(a, k) + 3 * G(s2 * a, k) + 1 * G(s3 * a, k)
    assert abs(y[centre, 0] - want_c) < 1e-13 * abs(want_c)
    assert abs(y[corner, 0] - want_k) < 1e-13 * abs(want_k)


@pytest.mark.parametrize("k", [0.5, 10.0, 300.0])
def test_imaginary_part_limit(k):
    # Im exp(ikr)/(4 pi r) = sin(kr)/(4 pi r) -> k / (4 pi) as r -> 0 (outgoing wave, +ikr).
    r = 1e-7
    x = np.array([[0.5, 0.5, 0.5], [0.5 + r, 0.5, 0.5]])
    y = oracle.Plan(np.zeros((2, 3), np.int32)).apply(x, k, np.array([[0.0], [1.0]]))
    assert abs(y[0, 0].imag - k / (4 * np.pi)) < 1e-9 * k / (4 * np.pi)
    assert abs(y[0, 0].real * 4 * np.pi * r - 1) < 1e-9


@pytest.mark.parametrize("ka,rho_over_a", [(0.0, 2.5), (2.5, 2.5), (7.0, 3.0)])
def test_spherical_mean(ka, rho_over_a):
    # The mean of exp(ik|x-y|)/(4 pi |x-y|) over y on a sphere of radius a, for |x - c| = rho > a,
    # is exp(ik rho)/(4 pi rho) * sin(ka)/(ka).  Sources carry quadrature weights
    # (Gauss-Legendre in cos(theta) times the trapezoid rule in phi).
    a = 0.05
    k = ka / a
    nt, nph = 48, 96
    u, wu = np.polynomial.legendre.leggauss(nt)
    ph = 2 * np.pi * np.arange(nph) / nph
    U, PH = np.meshgrid(u, ph, indexing="ij")
    st = np.sqrt(1 - U ** 2)
    c = np.array([0.3, 0.4, 0.5])
    src = c + a * np.stack([st * np.cos(PH), st * np.sin(PH), U], axis=-1).reshape(-1, 3)
    w = (np.repeat(wu, nph) / 2 / nph).astype(np.complex128)
    e = np.array([0.48, -0.6, 0.64])
    tgt = c + rho_over_a * a * e / np.linalg.norm(e)
    x = np.vstack([tgt, src])
    q = np.concatenate([[0.0], w])[:, None]
    y = oracle.Plan(np.zeros((x.shape[0], 3), np.int32)).apply_rows(x, k, q, [0])
    rho = rho_over_a * a
    sinc = 1.0 if ka == 0 else math.sin(ka) / ka
    want = G(rho, k) * sinc
    assert abs(y[0, 0] - want) < 1e-11 * abs(G(rho, k))


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------
def dyadic_cloud(n, seed, scale_bits=20):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << scale_bits, size=(n, 3)) / float(1 << scale_bits)


def test_reciprocity():
    inst = W.sphere(3000, 16, 2 * math.pi * 5, seed=9, dtype=np.complex128)
    P = oracle.Plan(inst.ids)
    rng = np.random.default_rng(1)
    u = W.strengths(inst.n, 1, rng)
    v = W.strengths(inst.n, 1, rng)
    lhs = (u[:, 0] * P.apply(inst.xyz, inst.k, v)[:, 0]).sum()
    rhs = (v[:, 0] * P.apply(inst.xyz, inst.k, u)[:, 0]).sum()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_translation_invariance():
    x = dyadic_cloud(2500, 2)
    ids = W.leaf_ids(x, (0, 0, 0), 0.125)
    q = W.strengths(2500, 1, np.random.default_rng(3))
    P = oracle.Plan(ids)
    y0 = P.apply(x, 9.0, q)
    # shift positions, keep the ids
    y1 = P.apply(x + np.array([0.375, -0.25, 2.0]), 9.0, q)
    assert np.array_equal(y0, y1)
    # shift positions and ids together by whole boxes
    s = np.array([3, 0, 17])
    y2 = oracle.Plan(ids + s.astype(np.int32)).apply(x + s * 0.125, 9.0, q)
    # the Morton order (and so the summation order) changes with the ids
    assert rel_l2(y2, y0) < 1e-14


def test_k_zero_is_real_laplace():
    inst = W.cube(2000, 6, 0.0, seed=6)
    P = oracle.Plan(inst.ids)
    y = P.apply(inst.xyz, 0.0, inst.q)
    yr = P.apply(inst.xyz, 0.0, inst.q.real.astype(np.complex128))
    yi = P.apply(inst.xyz, 0.0, inst.q.imag.astype(np.complex128))
    assert np.all(yr.imag == 0) and np.all(yi.imag == 0)
    np.testing.assert_allclose(y, yr + 1j * yi, rtol=1e-14, atol=1e-14 * np.abs(y).max())
    # Laplace kernel 1/(4 pi r), brute force
    yb = dense_apply(inst.xyz, inst.ids, 0.0, inst.q)
    assert rel_l2(y, yb) < 1e-13


def test_columns_and_threads_and_rows():
    inst = W.cube(4000, 7, 12.0, seed=8, m=3)
    P = oracle.Plan(inst.ids)
    y = P.apply(inst.xyz, inst.k, inst.q, threads=4)
    for c in range(3):
        assert np.array_equal(y[:, c:c + 1], P.apply(inst.xyz, inst.k, inst.q[:, c:c + 1], threads=1))
    rows = np.array([0, 17, 3999, 1234])
    assert np.array_equal(P.apply_rows(inst.xyz, inst.k, inst.q, rows), y[rows])
