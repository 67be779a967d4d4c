"""The leaf level from the clustering threshold (paper section 3.1: the tree height
is raised until no leaf box holds more than CT points), against the definition
recomputed with numpy: ids floor((x - o) / h) at each height, the largest box
count, the first height at or above the start whose count is at most CT."""
import math

import numpy as np
import pytest
import torch

import paper_2403_01596_amd as p2p
import workloads as W

pytestmark = pytest.mark.gpu


def reference(xyz, origin, size, ct, lmin):
    for L in range(lmin, 23):
        h = math.ldexp(size, 1 - L)
        ids = np.floor((xyz - origin) / h).astype(np.int64)
        key = (ids[:, 0] << 42) | (ids[:, 1] << 21) | ids[:, 2]
        t = int(np.unique(key, return_counts=True)[1].max())
        if t <= ct:
            return L, h, t
    return None


def cube_of(xyz):
    o = xyz.min(axis=0) - 1e-9
    return o, (float((xyz.max(axis=0) - o).max()) + 1e-9) * (1 + 1e-9)


@pytest.mark.parametrize("kind,n,ct,lmin", [("sphere", 200_000, 15, 1), ("sphere", 50_000, 64, 3),
                                             ("cube", 300_000, 15, 1), ("cube", 7, 1, 1), ("cube", 1, 15, 5)])
def test_level_matches_definition(kind, n, ct, lmin):
    rng = np.random.default_rng(n + ct)
    xyz = W.sphere_surface(n, rng) if kind == "sphere" else rng.random((n, 3))
    origin, size = cube_of(xyz)
    print("leaf level: %s n=%d ct=%d from %d" % (kind, n, ct, lmin), flush=True)
    xd = torch.from_numpy(xyz).cuda()
    L, h, t = p2p.leaf_level(xd, origin, size, ct, lmin)
    Lr, hr, tr = reference(xyz, origin, size, ct, lmin)
    print("  level %d h %.6g t %d (reference %d, %d)" % (L, h, t, Lr, tr), flush=True)
    assert (L, t) == (Lr, tr) and h == hr
    # the plan's own ids for that h have exactly that occupancy
    ids = p2p.box_ids(xd, origin, h).cpu().numpy().astype(np.int64)
    key = (ids[:, 0] << 42) | (ids[:, 1] << 21) | ids[:, 2]
    assert int(np.unique(key, return_counts=True)[1].max()) == t


def test_level_errors():
    rng = np.random.default_rng(3)
    xyz = rng.random((1000, 3))
    xd = torch.from_numpy(xyz).cuda()
    with pytest.raises(p2p.P2PError) as e:  # a point outside the cube
        p2p.leaf_level(xd, (0.0, 0.0, 0.0), 0.5, 15)
    assert e.value.status == 2
    dup = xyz.copy()
    dup[:20] = dup[0]  # 20 coincident points never split below CT = 15
    with pytest.raises(p2p.P2PError) as e:
        p2p.leaf_level(torch.from_numpy(dup).cuda(), (0.0, 0.0, 0.0), 1.0, 15)
    assert e.value.status == 2
    with pytest.raises(p2p.P2PError):
        p2p.leaf_level(xd, (0.0, 0.0, 0.0), 1.0, 0)
    assert p2p.leaf_level(torch.empty((0, 3), dtype=torch.float64, device="cuda"), (0, 0, 0), 1.0, 15, 4) == \
        (4, 0.125, 0)
