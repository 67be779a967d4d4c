"""Pins of the oracle's two-dimensional setting (the paper's own: a quadtree of
height L over the unit square, nine neighbour boxes, real potentials), CPU only.

Reading taken for the kernel the paper leaves unwritten: G(r) = -ln(r) / (2 pi).
Each pin is chosen so that a plausible mistake fails it:
  - dense all-pairs brute force in numpy, no boxes or sorting (neighbour set,
    sign, log, factor 1/(2 pi), skip rule);
  - two points in one box, and in boxes two apart (zero);
  - the 3x3 lattice: the centre sees 4 G(a) + 4 G(sqrt(2) a);
  - symmetry u^T A v = v^T A u;
  - translation by whole boxes that keeps the Morton order (bitwise equal);
  - halving every coordinate and adding a level keeps the boxes, and turns every
    term G(r) into G(r) + ln(2) / (2 pi): y changes by ln(2)/(2 pi) times the sum
    of the near strengths;
  - full-grid neighbour counts: corner 4, edge 6, interior 9, sum (3g - 2)^2.
"""
import math

import numpy as np
import pytest

import oracle


def brute(xy, q, level):
    side = 2.0 ** (level - 1)
    b = np.floor(xy * side)
    near = np.all(np.abs(b[:, None, :] - b[None, :, :]) <= 1, axis=2)
    d = xy[:, None, :] - xy[None, :, :]
    r = np.sqrt((d * d).sum(axis=2))
    mask = near & (r > 0)
    G = np.zeros_like(r)
    G[mask] = -np.log(r[mask]) / (2 * np.pi)
    return G @ q


@pytest.mark.parametrize("n,level,seed", [(2000, 4, 0), (2000, 6, 1), (1500, 8, 2), (300, 2, 3), (400, 1, 4)])
def test_brute_force(n, level, seed):
    rng = np.random.default_rng(seed)
    xy = rng.random((n, 2))
    q = rng.standard_normal(n)
    y = oracle.apply2d(xy, q, level)
    ref = brute(xy, q, level)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-13
    st = oracle.stats2d(xy, level)
    side = 2.0 ** (level - 1)
    b = np.floor(xy * side)
    near = np.all(np.abs(b[:, None, :] - b[None, :, :]) <= 1, axis=2)
    assert st["n_pairs"] + st["n_zero_pairs"] == int(near.sum())


def test_duplicates_and_faces():
    rng = np.random.default_rng(5)
    xy = rng.random((1200, 2))
    xy[100:110] = xy[7]                       # coincident points: skipped
    xy[200:220, 0] = 0.5                      # exactly on a box face
    xy[220:230] = np.array([0.25, 0.75])
    q = rng.standard_normal(xy.shape[0])
    for level in (3, 5):
        y = oracle.apply2d(xy, q, level)
        assert np.linalg.norm(y - brute(xy, q, level)) / np.linalg.norm(y) < 1e-13


def test_two_points():
    a = np.array([[0.30, 0.40], [0.33, 0.44]])  # r = 0.05, same box at level 2
    y = oracle.apply2d(a, np.array([2.0, -3.0]), 2)
    g = -math.log(0.05) / (2 * math.pi)
    assert abs(y[0] - g * -3.0) < 1e-15 and abs(y[1] - g * 2.0) < 1e-15
    far = np.array([[0.1, 0.1], [0.6, 0.1]])  # boxes 0 and 2 at level 3 (side 4)
    assert np.all(oracle.apply2d(far, np.array([1.0, 1.0]), 3) == 0.0)


def test_lattice_centre():
    level = 3                                 # 4 x 4 boxes of side a = 1/4
    a = 0.25
    pts = np.array([[(i + 0.5) * a, (j + 0.5) * a] for j in range(4) for i in range(4)])
    y = oracle.apply2d(pts, np.ones(16), level)
    centre = 1 * 4 + 1                        # box (1, 1): all 8 neighbours present
    expect = 4 * (-math.log(a)) / (2 * math.pi) + 4 * (-math.log(math.sqrt(2) * a)) / (2 * math.pi)
    assert abs(y[centre] - expect) < 1e-14


def test_symmetry():
    rng = np.random.default_rng(6)
    xy = rng.random((1500, 2))
    u, v = rng.standard_normal(1500), rng.standard_normal(1500)
    lhs = u @ oracle.apply2d(xy, v, 5)
    rhs = v @ oracle.apply2d(xy, u, 5)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_translation_by_whole_boxes():
    rng = np.random.default_rng(7)
    level = 5
    xy = np.floor(rng.random((1500, 2)) * 2.0 ** 29) / 2.0 ** 30  # multiples of 2^-30 in [0, 0.5): shifts are exact
    q = rng.standard_normal(1500)
    # 8 boxes on each axis: every id (below 8 before) gains the same high bit, so the
    # Morton order of boxes and of each neighbour list, and with it the order of
    # summation, stays the same
    shift = np.array([8, 8]) / 2.0 ** (level - 1)
    assert np.array_equal(oracle.apply2d(xy, q, level), oracle.apply2d(xy + shift, q, level))


def test_halving_adds_log2():
    rng = np.random.default_rng(8)
    level = 4
    xy = rng.random((1500, 2))
    q = rng.standard_normal(1500)
    y = oracle.apply2d(xy, q, level)
    y2 = oracle.apply2d(xy / 2, q, level + 1)  # same boxes, every distance halved
    # sum of the near strengths of each point (r != 0), by brute force on the mask
    side = 2.0 ** (level - 1)
    b = np.floor(xy * side)
    near = np.all(np.abs(b[:, None, :] - b[None, :, :]) <= 1, axis=2)
    np.fill_diagonal(near, False)
    s = near.astype(float) @ q
    assert np.allclose(y2, y + math.log(2) / (2 * math.pi) * s, rtol=0, atol=1e-12 * np.abs(y).max())


def test_full_grid_neighbour_counts():
    g = 8
    level = 4                                 # 8 x 8 boxes
    pts = np.array([[(i + 0.5) / g, (j + 0.5) / g] for j in range(g) for i in range(g)])
    st = oracle.stats2d(pts, level)
    # one point per box: ordered near pairs with r != 0 = sum over boxes of (neighbours - 1)
    assert st["n_boxes"] == g * g
    assert st["n_pairs"] + st["n_zero_pairs"] == (3 * g - 2) ** 2
    assert st["n_zero_pairs"] == g * g
    y = oracle.apply2d(pts, np.ones(g * g), level)
    # the number of neighbours shows in the sum of unit strengths at distance scale:
    # corner boxes have 3 neighbours, edge boxes 5, interior 8 (self excluded)
    a = 1.0 / g
    g1, g2 = -math.log(a) / (2 * math.pi), -math.log(math.sqrt(2) * a) / (2 * math.pi)
    assert abs(y[0] - (2 * g1 + g2)) < 1e-14
    assert abs(y[1] - (3 * g1 + 2 * g2)) < 1e-14
    assert abs(y[g + 1] - (4 * g1 + 4 * g2)) < 1e-14


def test_out_of_plate_is_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.apply2d(np.array([[0.5, 1.0]]), np.ones(1), 3)
