"""Close pairs in the FP32 path: planted pairs at r = 2^-k h, compared row by row.

The FP32 kernels take coordinate differences from fixed-point coordinates whose
quantum is about 2^-29 h; a pair a few quanta apart would carry a large relative
error in its term, and such a term dominates its row.  Every near pair closer
than 2^20 quanta therefore takes its difference from the FP64 coordinates, inside
the kernels.
These tests plant pairs at r = 2^-k h for k = 8 .. 40 in a 200k-point ellipsoid
(64 points per box, box = a quarter wavelength, the density sweep's densest
case): inside one box, and straddling a box face (where the two points are in
different boxes).  The pairs below one quantum (k >= 30) sit on one fixed-point
position across a face, the case where an uncorrected kernel divides by zero.
Every planted row is compared with the FP64 oracle on its own, and the whole
output too.  Forward (both layouts), reverse pass and the matrix-core path.
Dense clusters (hundreds of mutually close points, one of them across a box
face) give a box more close pairs than the sweep's queue holds at once.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2403_01596_amd as p2p
import workloads as W
from gpu_helpers import dev, rel_l2

pytestmark = pytest.mark.gpu
KS = list(range(8, 41))


def planted(seed=3):
    """The ellipsoid plus planted pairs; returns (xyz, ids, q, k, h, rows of planted points)."""
    base = W.ellipsoid(200_000, 64, seed=seed, dtype=np.complex64)
    rng = np.random.default_rng(seed)
    h, o = base.h, base.origin
    pts, rows = [base.xyz], []
    n = base.n
    anchors = rng.choice(n, 2 * len(KS), replace=False)
    for j, kk in enumerate(KS):
        r = h * 2.0 ** -kk
        # inside a box: a partner r away in a random direction, same box
        a = base.xyz[anchors[2 * j]]
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        b = a + r * u
        if np.any(np.floor((b - o) / h) != np.floor((a - o) / h)):
            b = a - r * u
        # across a face: two points r apart around the x face of another anchor's box
        c = base.xyz[anchors[2 * j + 1]].copy()
        face = o[0] + (np.floor((c[0] - o[0]) / h) + 1) * h
        c1, c2 = c.copy(), c.copy()
        c1[0] = face - r / 2
        c2[0] = face + r / 2
        pts.append(np.stack([b, c1, c2]))
        rows += [anchors[2 * j], n + 3 * j, n + 3 * j + 1, n + 3 * j + 2]
    xyz = np.ascontiguousarray(np.concatenate(pts))
    ids = W.leaf_ids(xyz, o, h)
    q = W.strengths(xyz.shape[0], 1, rng, np.complex64)
    return xyz, ids, q, base.k, h, np.array(rows)


@pytest.fixture(scope="module")
def case():
    xyz, ids, q, k, h, rows = planted()
    orc = oracle.Plan(ids)
    yref = orc.apply(xyz, k, q)
    print("planted: %d points, %d planted rows" % (xyz.shape[0], rows.size), flush=True)
    return xyz, ids, q, k, h, rows, orc, yref


def row_errors(got, ref, rows):
    g, r = got[rows].reshape(rows.size, -1), ref[rows].reshape(rows.size, -1)
    return np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)


def test_planted_rows_cross_the_face(case):
    xyz, ids, q, k, h, rows, orc, yref = case
    # the face pairs really straddle the face: distinct boxes, adjacent along x
    face = rows.reshape(-1, 4)[:, 2:]
    assert np.all(ids[face[:, 1], 0] == ids[face[:, 0], 0] + 1)


@pytest.mark.parametrize("layout", ["tiles", "csr"])
def test_forward_planted(case, layout):
    xyz, ids, q, k, h, rows, orc, yref = case
    P = p2p.Plan(dev(xyz, torch.float64), dev(ids, torch.int32), k, dtype=torch.complex64, layout=layout)
    info = P.info()
    y = P.apply(dev(q)).cpu().numpy().reshape(-1, 1)
    assert np.isfinite(y).all()
    e_rows = row_errors(y, yref, rows)
    e_all = rel_l2(y, yref)
    print("  %s: %d close pairs, quantum 2^%d (h 2^%.1f); planted rows: max %.2e; whole %.2e" % (
        layout, info["n_close_pairs"], info["quantum_exp"], math.log2(h), e_rows.max(), e_all), flush=True)
    assert info["n_close_pairs"] >= 4 * len(KS)
    assert e_rows.max() <= 1e-5
    assert e_all <= 1e-6
    P.close()


def test_backward_planted(case):
    xyz, ids, q, k, h, rows, orc, yref = case
    g = W.strengths(xyz.shape[0], 1, np.random.default_rng(9), np.complex64)
    dq_ref, dx_ref = orc.backward(xyz, k, q, g)
    P = p2p.Plan(dev(xyz, torch.float64), dev(ids, torch.int32), k, dtype=torch.complex64, layout="csr")
    dq, dx = P.backward(dev(q), dev(g))
    dq, dx = dq.cpu().numpy().reshape(-1, 1), dx.cpu().numpy()
    assert np.isfinite(dq).all() and np.isfinite(dx).all()
    eq, ex = row_errors(dq, dq_ref, rows), row_errors(dx, dx_ref, rows)
    print("  reverse pass, planted rows: dq max %.2e, dx max %.2e; whole dq %.2e dx %.2e" % (
        eq.max(), ex.max(), rel_l2(dq, dq_ref), rel_l2(dx, dx_ref)), flush=True)
    assert eq.max() <= 1e-5 and ex.max() <= 1e-5
    assert rel_l2(dq, dq_ref) <= 1e-6 and rel_l2(dx, dx_ref) <= 1e-5
    P.close()


def test_matrix_cores_planted(case):
    xyz, ids, q, k, h, rows, orc, yref = case
    m = 16
    qm = W.strengths(xyz.shape[0], m, np.random.default_rng(11), np.complex64)
    ref = orc.apply(xyz, k, qm)
    P = p2p.Plan(dev(xyz, torch.float64), dev(ids, torch.int32), k, dtype=torch.complex64, layout="csr",
                 max_rhs=m)
    y = P.apply(dev(qm)).cpu().numpy()
    assert np.isfinite(y).all()
    e_rows = row_errors(y, ref, rows)
    print("  matrix cores, %d columns: planted rows max %.2e, whole %.2e" % (m, e_rows.max(), rel_l2(y, ref)),
          flush=True)
    assert e_rows.max() <= 1e-5 and rel_l2(y, ref) <= 1e-6
    P.close()


def test_f64_planted(case):
    xyz, ids, q, k, h, rows, orc, yref = case
    P = p2p.Plan(dev(xyz, torch.float64), dev(ids, torch.int32), k, dtype=torch.complex128, layout="csr")
    y = P.apply(dev(q.astype(np.complex128))).cpu().numpy().reshape(-1, 1)
    e_rows = row_errors(y, yref, rows)
    print("  FP64: planted rows max %.2e, whole %.2e" % (e_rows.max(), rel_l2(y, yref)), flush=True)
    assert e_rows.max() <= 1e-12 and rel_l2(y, yref) <= 1e-12
    assert P.info()["n_close_pairs"] == 0
    P.close()


def clustered(seed=5):
    """A 30k-point sphere plus three clusters of 150 points each within 2^-20 h
    (about 500 quanta) of an anchor, one straddling a box face: every cluster point
    has ~149 close partners, far more than one group's close-pair queue takes at once.
    At that distance a term from the fixed-point coordinates would be off by about
    1e-3 of itself."""
    base = W.sphere(30_000, 32, 2 * math.pi * 8, seed=seed, dtype=np.complex64)
    rng = np.random.default_rng(seed)
    h, o = base.h, base.origin
    pts, rows = [base.xyz], []
    n = base.n
    for j, a in enumerate(rng.choice(n, 3, replace=False)):
        c = base.xyz[a].copy()
        if j == 2:  # centred on the x face of its box
            c[0] = o[0] + (np.floor((c[0] - o[0]) / h) + 1) * h
        cl = c + h * 2.0 ** -20 * rng.uniform(-1, 1, (150, 3))
        pts.append(cl)
        rows += list(range(n + 150 * j, n + 150 * (j + 1)))
    xyz = np.ascontiguousarray(np.concatenate(pts))
    ids = W.leaf_ids(xyz, o, h)
    q = W.strengths(xyz.shape[0], 1, rng, np.complex64)
    return xyz, ids, q, base.k, np.array(rows)


def near_terms(xyz, ids, k, i):
    """Row i's near sources (r != 0, by the definition) with G(r_ij), G'(r_ij) and
    the differences x_i - x_j, in FP64."""
    near = np.flatnonzero(np.all(np.abs(ids - ids[i]) <= 1, axis=1))
    d = xyz[i] - xyz[near]
    r = np.sqrt((d * d).sum(1))
    m = r > 0
    near, d, r = near[m], d[m], r[m]
    e = np.exp(1j * k * r)
    return near, e / (4 * np.pi * r), e * (1j * k * r - 1) / (4 * np.pi * r * r), d


def abs_row_sums(xyz, ids, k, rows, q, g=None):
    """Per row: sum_j |G_ij| |q_j| (forward; per column for several) and, with g, the
    same for dq (|g_j|) and sum_j |G'_ij| |u_ij| for dx: the sizes of the terms a
    floating-point sum of the row cannot be more exact than."""
    fw, dqs, dxs = [], [], []
    for i in rows:
        near, G, Gp, d = near_terms(xyz, ids, k, i)
        fw.append(np.abs(G) @ np.abs(q[near].reshape(near.size, -1)))
        if g is not None:
            dqs.append(np.abs(G) @ np.abs(g[near].reshape(near.size, -1)))
            u = np.conj(g[i, 0]) * q[near, 0] + np.conj(g[near, 0]) * q[i, 0]
            dxs.append(float(np.abs(Gp * u).sum()))
    return np.array(fw), np.array(dqs), np.array(dxs)


def err_over_abs(got, ref, rows, scale):
    g, r = got[rows].reshape(rows.size, -1), ref[rows].reshape(rows.size, -1)
    return np.linalg.norm(g - r, axis=1) / np.linalg.norm(scale.reshape(rows.size, -1), axis=1)


@pytest.fixture(scope="module")
def clusters():
    xyz, ids, q, k, rows = clustered()
    orc = oracle.Plan(ids)
    print("clusters: %d points, %d cluster rows" % (xyz.shape[0], rows.size), flush=True)
    return xyz, ids, q, k, rows, orc, orc.apply(xyz, k, q)


# Cluster rows cancel heavily (sum_j |terms| reaches hundreds of times |y_i|), so
# their error is bounded against the size of their terms: FP32 sums of exact-
# difference terms stay near 1e-7 of it (an FP32 emulation on the CPU gives at most
# 9e-8); a close pair taken from the fixed-point coordinates would be ~1e-3 off.
ABS_TOL = 1e-6


@pytest.mark.parametrize("layout", ["tiles", "csr"])
def test_forward_clusters(clusters, layout):
    xyz, ids, q, k, rows, orc, yref = clusters
    # the face cluster really spans two boxes
    assert np.unique(ids[rows[300:], 0]).size == 2
    P = p2p.Plan(dev(xyz, torch.float64), dev(ids, torch.int32), k, dtype=torch.complex64, layout=layout)
    info = P.info()
    y = P.apply(dev(q)).cpu().numpy().reshape(-1, 1)
    assert np.isfinite(y).all()
    fw, _, _ = abs_row_sums(xyz, ids, k, rows, q.astype(np.complex128))
    e_abs = err_over_abs(y, yref, rows, fw)
    print("  %s: %d close pairs; cluster rows: error / sum|terms| max %.2e, relative max %.2e; whole %.2e" % (
        layout, info["n_close_pairs"], e_abs.max(), row_errors(y, yref, rows).max(), rel_l2(y, yref)), flush=True)
    assert info["n_close_pairs"] >= 3 * 150 * 149
    assert e_abs.max() <= ABS_TOL and rel_l2(y, yref) <= 1e-6
    P.close()


def test_backward_clusters(clusters):
    xyz, ids, q, k, rows, orc, yref = clusters
    g = W.strengths(xyz.shape[0], 1, np.random.default_rng(13), np.complex64)
    dq_ref, dx_ref = orc.backward(xyz, k, q, g)
    P = p2p.Plan(dev(xyz, torch.float64), dev(ids, torch.int32), k, dtype=torch.complex64, layout="tiles")
    dq, dx = P.backward(dev(q), dev(g))
    dq, dx = dq.cpu().numpy().reshape(-1, 1), dx.cpu().numpy()
    _, sq, sx = abs_row_sums(xyz, ids, k, rows, q.astype(np.complex128), g.astype(np.complex128))
    eq, ex = err_over_abs(dq, dq_ref, rows, sq), err_over_abs(dx, dx_ref, rows, sx)
    print("  reverse pass, cluster rows: error / sum|terms| dq max %.2e, dx max %.2e; whole dq %.2e dx %.2e" % (
        eq.max(), ex.max(), rel_l2(dq, dq_ref), rel_l2(dx, dx_ref)), flush=True)
    assert eq.max() <= ABS_TOL and ex.max() <= ABS_TOL
    assert rel_l2(dq, dq_ref) <= 1e-6 and rel_l2(dx, dx_ref) <= 1e-5
    P.close()


def test_matrix_cores_clusters(clusters):
    xyz, ids, q, k, rows, orc, yref = clusters
    m = 8
    qm = W.strengths(xyz.shape[0], m, np.random.default_rng(17), np.complex64)
    ref = orc.apply(xyz, k, qm)
    P = p2p.Plan(dev(xyz, torch.float64), dev(ids, torch.int32), k, dtype=torch.complex64, layout="csr",
                 max_rhs=m)
    y = P.apply(dev(qm)).cpu().numpy()
    fw, _, _ = abs_row_sums(xyz, ids, k, rows, qm.astype(np.complex128))
    e_abs = err_over_abs(y, ref, rows, fw)
    print("  matrix cores, %d columns: cluster rows error / sum|terms| max %.2e, whole %.2e" % (
        m, e_abs.max(), rel_l2(y, ref)), flush=True)
    assert e_abs.max() <= ABS_TOL and rel_l2(y, ref) <= 1e-6
    P.close()


def lane_pairs(seed=8):
    """Isolated boxes (ids three apart: no neighbour boxes) of 2 to 100 random points
    and one pair 2^-22 h apart at positions (i, j) of the box's point order, which
    is the input order; the pairs cover every row and half-wavefront boundary of
    the plan build's own-box test and random positions.  Returns (xyz, ids, q, k,
    rows of the paired points)."""
    rng = np.random.default_rng(seed)
    h, k = 1.0 / 64, 2 * math.pi * 4
    pts, rows, box, start = [], [], 0, 0
    for s in [2, 3, 16, 17, 31, 32, 33, 47, 48, 63, 64, 65, 90, 100]:
        pairs = {(0, 1), (0, s - 1), (s - 2, s - 1)}
        for step in (1, 15, 16, 17, 31, 32, 33, 48, 64):
            pairs |= {(i, i + step) for i in range(0, s - step, 7)}
        while len(pairs) < min(60, s * (s - 1) // 2):
            i, j = sorted(rng.choice(s, 2, replace=False))
            pairs.add((int(i), int(j)))
        for i, j in sorted(pairs):
            cell = 3 * np.array([box % 32, box // 32 % 32, box // 1024])
            p = (cell + rng.uniform(0.05, 0.95, (s, 3))) * h
            u = rng.standard_normal(3)
            p[j] = p[i] + h * 2.0 ** -22 * u / np.linalg.norm(u)
            pts.append(p)
            rows += [start + i, start + j]
            start += s
            box += 1
    xyz = np.ascontiguousarray(np.concatenate(pts))
    ids = W.leaf_ids(xyz, np.zeros(3), h)
    q = W.strengths(xyz.shape[0], 1, rng, np.complex64)
    return xyz, ids, q, k, np.array(rows)


@pytest.mark.parametrize("layout", ["tiles", "csr"])
def test_own_box_pair_at_every_lane_offset(layout):
    # a box with no close neighbour box is marked for the close-pair path only by
    # the plan build's test of its own points: a pair it missed would be summed
    # from the fixed-point coordinates, 2^7 quanta apart, about 1e-2 off
    xyz, ids, q, k, rows = lane_pairs()
    print("lane pairs: %d points, %d boxes, %d paired rows" % (xyz.shape[0], W.count_boxes(ids), rows.size),
          flush=True)
    P = p2p.Plan(dev(xyz, torch.float64), dev(ids, torch.int32), k, dtype=torch.complex64, layout=layout)
    y = P.apply(dev(q)).cpu().numpy().reshape(-1, 1)
    P.close()
    qq = q.astype(np.complex128)
    yref = np.zeros((xyz.shape[0], 1), np.complex128)
    for i in rows:
        near, G, _, _ = near_terms(xyz, ids, k, i)
        yref[i, 0] = G @ qq[near]
    fw, _, _ = abs_row_sums(xyz, ids, k, rows, qq)
    e_abs = err_over_abs(y, yref, rows, fw)
    print("  %s: paired rows error / sum|terms| max %.2e" % (layout, e_abs.max()), flush=True)
    assert e_abs.max() <= ABS_TOL
