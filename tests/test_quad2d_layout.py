"""The paper's two layouts for its 2-D experiment, as collected on the host by the
library (sections 3.2 and 3.3), rebuilt here in numpy and compared exactly.  Host
logic only: no device is involved in the collection.

Indexing (section 3.2): target and source coordinates, the points of every box
of the quadtree (all 4^(L-1) boxes, Morton order, input order inside a box) with
their box offsets, the neighbour sources of every box (the nine boxes around it
in ascending key order, each box's points in that same order) with their
offsets, and the potentials.  Repetition (section 3.3): per target, in box order,
[x, y, count, (x, y, q) of each neighbour source], padded with zeros to
3 + 3 max(9 CT, largest neighbourhood) doubles.
"""
import numpy as np
import pytest

import paper_2403_01596_amd as p2p


def morton2(bx, by):
    k = np.zeros(bx.shape, np.int64)
    for b in range(16):
        k |= ((bx >> b) & 1) << (2 * b)
        k |= ((by >> b) & 1) << (2 * b + 1)
    return k


def expected(xy, q, level, ct):
    side = 2 ** (level - 1)
    b = np.floor(xy * side).astype(np.int64)
    key = morton2(b[:, 0], b[:, 1])
    order = np.argsort(key, kind="stable")
    boxes = side * side
    counts = np.bincount(key, minlength=boxes)
    start = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    # box key -> (x, y)
    kx = np.array([sum(((k >> (2 * i)) & 1) << i for i in range(16)) for k in range(boxes)])
    ky = np.array([sum(((k >> (2 * i + 1)) & 1) << i for i in range(16)) for k in range(boxes)])
    src, sstart, nbrs = [], [0], []
    for kk in range(boxes):
        nb = sorted(int(morton2(np.array([kx[kk] + dx]), np.array([ky[kk] + dy]))[0])
                    for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                    if 0 <= kx[kk] + dx < side and 0 <= ky[kk] + dy < side)
        nbrs.append(nb)
        idx = np.concatenate([order[start[s]:start[s + 1]] for s in nb]) if nb else np.zeros(0, np.int64)
        src.append(idx)
        sstart.append(sstart[-1] + idx.size)
    return order.astype(np.int32), start, np.concatenate(src).astype(np.int32), np.array(sstart, np.int32), nbrs


@pytest.mark.parametrize("n,level,seed", [(700, 3, 0), (300, 5, 1), (2000, 2, 2), (50, 6, 3), (1, 4, 4)])
def test_indexing_layout(n, level, seed):
    rng = np.random.default_rng(seed)
    xy = rng.random((n, 2))
    xy[: n // 10, 0] = 0.5  # on a box face
    q = rng.standard_normal(n)
    Q = p2p.Quad2D("indexing", xy, q, level)
    got, inf = Q.layout(), Q.info()
    tidx, tstart, sidx, sstart, _ = expected(xy, q, level, 15)
    assert inf["n_boxes"] == 4 ** (level - 1)
    assert np.array_equal(got["target_xy"], xy) and np.array_equal(got["source_xy"], xy)
    assert np.array_equal(got["q"], q)
    assert np.array_equal(got["target_idx"], tidx) and np.array_equal(got["target_start"], tstart)
    assert np.array_equal(got["source_idx"], sidx) and np.array_equal(got["source_start"], sstart)
    assert inf["t_max"] == int(np.diff(tstart).max())
    assert inf["n_slots"] == int(sum(np.diff(tstart)[b] * (sstart[b + 1] - sstart[b]) for b in range(tstart.size - 1)))
    Q.close()


@pytest.mark.parametrize("n,level,seed,ct", [(700, 3, 0, 15), (300, 5, 1, 15), (400, 4, 2, 2), (1, 2, 3, 15)])
def test_repetition_layout(n, level, seed, ct):
    rng = np.random.default_rng(seed)
    xy = rng.random((n, 2))
    q = rng.standard_normal(n)
    Q = p2p.Quad2D("repetition", xy, q, level, ct=ct)
    got, inf = Q.layout(), Q.info()
    tidx, tstart, sidx, sstart, _ = expected(xy, q, level, ct)
    smax = max(9 * ct, int(np.diff(sstart)[np.diff(tstart) > 0].max()))
    R = 3 + 3 * smax
    assert inf["record_len"] == R and got["records"].shape == (n, R)
    assert np.array_equal(got["record_target"], tidx)
    boxes = tstart.size - 1
    t = 0
    for b in range(boxes):
        src = sidx[sstart[b]:sstart[b + 1]]
        for k in range(tstart[b], tstart[b + 1]):
            rec = got["records"][t]
            i = tidx[k]
            assert rec[0] == xy[i, 0] and rec[1] == xy[i, 1] and rec[2] == src.size
            body = np.stack([xy[src, 0], xy[src, 1], q[src]], axis=1).ravel()
            assert np.array_equal(rec[3:3 + body.size], body)
            assert not rec[3 + body.size:].any()
            t += 1
    assert t == n
    # the layout's size: eq. 8's 8 N (3 + 27 CT) bytes when no box exceeds CT, plus
    # the record-to-row index
    if smax == 9 * ct:
        assert inf["layout_bytes"] >= 8 * n * (3 + 27 * ct) + 4 * n
    Q.close()


def test_collection_errors():
    with pytest.raises(p2p.P2PError) as e:
        p2p.Quad2D("indexing", np.array([[0.5, 1.0]]), np.ones(1), 3)
    assert e.value.status == 2
    with pytest.raises(p2p.P2PError) as e:
        p2p.Quad2D("repetition", np.array([[0.5, 0.5]]), np.ones(1), 0)
    assert e.value.status == 2
    with pytest.raises(p2p.P2PError) as e:
        p2p.Quad2D("repetition", np.array([[0.5, 0.5]]), np.ones(1), 3, ct=0)
    assert e.value.status == 1
