"""Pins for the oracle's box table and neighbour lists (CPU only).

The paper keeps boxes in Morton order (section 3.2) and lets each box see its
adjacent boxes, itself included (section 3.2: nine in 2-D; here 27 in 3-D).
These tests re-derive every table by constructions that share nothing with the
oracle: bit strings for the Morton key, an all-pairs scan for neighbours, and
closed-form counts on full grids.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def morton_by_strings(ix, iy, iz):
    """Interleave the binary digits as text: z y x per level, most significant level first."""
    bx, by, bz = (format(v, "021b") for v in (ix, iy, iz))
    return int("".join(bz[i] + by[i] + bx[i] for i in range(21)), 2)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_morton_matches_bit_strings(seed):
    rng = np.random.default_rng(seed)
    pts = rng.integers(0, 1 << 21, size=(200, 3))
    pts[0] = (0, 0, 0)
    pts[1] = ((1 << 21) - 1,) * 3
    pts[2] = (1, 0, 0)
    for ix, iy, iz in pts:
        assert oracle.morton(int(ix), int(iy), int(iz)) == morton_by_strings(int(ix), int(iy), int(iz))
    assert oracle.morton(1, 0, 0) == 1 and oracle.morton(0, 1, 0) == 2 and oracle.morton(0, 0, 1) == 4


def full_grid_ids(g, per_box=1, seed=0):
    rng = np.random.default_rng(seed)
    ax = np.arange(g)
    cells = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3)
    ids = np.repeat(cells, per_box, axis=0)
    return ids[rng.permutation(ids.shape[0])].astype(np.int32)


@pytest.mark.parametrize("g", [2, 3, 5, 8])
def test_full_grid_neighbour_counts(g):
    ids = full_grid_ids(g, per_box=2)
    P = oracle.Plan(ids)
    t = P.tables()
    assert P.n_boxes == g ** 3
    # sum over boxes of the neighbourhood size is (3g - 2)^3 on a full grid
    assert P.n_nbr == (3 * g - 2) ** 3
    counts = np.diff(t["nbr_start"])
    # decode each box's ids from its first point
    first = ids[t["perm"][t["box_start"][:-1]]]
    interior = np.sum((first > 0) & (first < g - 1), axis=1)  # axes not on the boundary
    expect = 3 ** interior * 2 ** (3 - interior)  # 8 corner, 12 edge, 18 face, 27 interior
    if g == 1:
        expect[:] = 1
    assert np.array_equal(counts, expect)
    if g >= 3:
        assert sorted(set(expect.tolist())) == [8, 12, 18, 27]


def brute_tables(ids):
    """Box table and neighbour lists by an all-pairs scan over distinct boxes."""
    keys = np.array([morton_by_strings(*map(int, r)) for r in ids], dtype=object)
    order = sorted(range(len(ids)), key=lambda i: (keys[i], i))
    box_key, box_start, box_ids = [], [], []
    for p, i in enumerate(order):
        if not box_key or keys[i] != box_key[-1]:
            box_key.append(keys[i])
            box_start.append(p)
            box_ids.append(ids[i])
    box_start.append(len(ids))
    B = len(box_key)
    bi = np.array(box_ids, dtype=np.int64).reshape(B, 3)
    nbr = []
    for T in range(B):
        near = [S for S in range(B) if np.abs(bi[S] - bi[T]).max() <= 1]
        nbr.append(near)  # ascending box index == ascending key
    return np.array(box_key, dtype=np.uint64), np.array(box_start), np.array(order), nbr


@pytest.mark.parametrize("case", ["random_sparse", "clustered", "extremes", "one_box", "one_per_box", "hollow"])
def test_tables_match_all_pairs_scan(case):
    rng = np.random.default_rng(7)
    lim = 1 << 21
    if case == "random_sparse":
        ids = rng.integers(0, 6, size=(300, 3))
    elif case == "clustered":
        ids = rng.integers(0, 3, size=(400, 3)) + np.array([1000, 77, 5])
    elif case == "extremes":
        ids = np.array([[0, 0, 0], [lim - 1, lim - 1, lim - 1], [1, 1, 1], [lim - 2, lim - 1, lim - 1],
                        [0, 0, 1], [lim - 1, 0, 0], [0, 0, 0]])
    elif case == "one_box":
        ids = np.tile([[3, 4, 5]], (50, 1))
    elif case == "one_per_box":
        ids = full_grid_ids(4)
    else:  # a 5^3 grid with its centre 3^3 emptied out
        ids = full_grid_ids(5, per_box=2)
        ids = ids[~np.all((ids >= 1) & (ids <= 3), axis=1)]
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    P = oracle.Plan(ids)
    t = P.tables()
    bk, bs, perm, nbr = brute_tables(ids)
    assert np.array_equal(t["box_key"], bk)
    assert np.array_equal(t["box_start"], bs)
    assert np.array_equal(t["perm"], perm)
    flat = [S for lst in nbr for S in lst]
    assert np.array_equal(t["nbr_idx"], np.array(flat, dtype=np.int32))
    assert np.array_equal(np.diff(t["nbr_start"]), [len(x) for x in nbr])


def test_perm_is_stable_sort_of_keys():
    ids = np.random.default_rng(3).integers(0, 4, size=(2000, 3)).astype(np.int32)
    t = oracle.Plan(ids).tables()
    keys = np.array([oracle.morton(*map(int, r)) for r in ids], dtype=np.uint64)
    sk = keys[t["perm"]]
    assert np.all(sk[1:] >= sk[:-1])
    tie = sk[1:] == sk[:-1]
    assert np.all(t["perm"][1:][tie] > t["perm"][:-1][tie])
    assert sorted(t["perm"].tolist()) == list(range(ids.shape[0]))


def test_empty_and_single():
    P = oracle.Plan(np.zeros((0, 3), np.int32))
    assert P.n_boxes == 0 and P.n_nbr == 0
    assert P.apply(np.zeros((0, 3)), 1.0, np.zeros((0, 1), np.complex128)).shape == (0, 1)
    P1 = oracle.Plan(np.zeros((1, 3), np.int32))
    y = P1.apply(np.zeros((1, 3)), 3.0, np.ones((1, 1), np.complex128))
    assert y[0, 0] == 0


@pytest.mark.parametrize("bad", [[-1, 0, 0], [0, 1 << 21, 0], [0, 0, -5]])
def test_ids_out_of_range_rejected(bad):
    ids = np.array([[0, 0, 0], bad], dtype=np.int32)
    with pytest.raises(oracle.OracleError):
        oracle.Plan(ids)


def test_box_ids_helper():
    rng = np.random.default_rng(11)
    xyz = rng.random((1000, 3)) * 3 - 1
    o = np.array([-1.25, -1.5, -1.125])
    h = 0.1
    ids = oracle.box_ids(xyz, o, h)
    assert np.array_equal(ids, W.leaf_ids(xyz, o, h))
    # every point lies in the half-open cell its id names (up to the rounding of (x - o) / h)
    lo = o + ids * h
    assert np.all(xyz >= lo - 1e-12) and np.all(xyz < lo + h + 1e-12)
    with pytest.raises(oracle.OracleError):
        oracle.box_ids(xyz, o + 1.0, h)  # negative ids
