"""The paper's 2-D experiment on the GPU: the Indexing kernel (thread per box), the
Repetition kernel (thread per target) and this library's sweep (wavefront per
box, both source layouts) against the FP64 oracle, on quadtrees from dense (a
few hundred points per box) to sparse (most boxes empty), with duplicates and
points on box faces.  FP64 throughout: relative L2 error <= 1e-12."""
import numpy as np
import pytest
import torch

import oracle
import paper_2403_01596_amd as p2p
from gpu_helpers import dev, rel_l2

pytestmark = pytest.mark.gpu

CASES = [  # (n, level, seed): D = n / 4^(level - 1)
    (20000, 4, 0),     # D ~ 312, neighbourhoods of ~2800 sources
    (16384, 7, 1),     # D = 4: the paper's N = 4 x boxes
    (4096, 9, 2),      # D = 1/16: most boxes empty
    (3000, 1, 3),      # one box
    (1, 5, 4),         # one point
]


def points(n, seed):
    rng = np.random.default_rng(seed)
    xy = rng.random((n, 2))
    if n > 100:
        xy[10:20] = xy[3]             # coincident points
        xy[30:60, 0] = 0.5            # on a box face
    return xy, rng.standard_normal(n)


@pytest.mark.parametrize("n,level,seed", CASES)
def test_three_routes(n, level, seed):
    xy, q = points(n, seed)
    ref = oracle.apply2d(xy, q, level)
    print("2-D n=%d L=%d" % (n, level), flush=True)
    for method in ("indexing", "repetition"):
        Q = p2p.Quad2D(method, xy, q, level)
        Q.transfer()
        y = Q.run().cpu().numpy()
        err = rel_l2(y, ref) if n > 1 else float(np.abs(y - ref).max())
        print("  %s: rel L2 %.2e, layout %d bytes" % (method, err, Q.info()["layout_bytes"]), flush=True)
        assert err <= 1e-12
        Q.close()
    xyz = np.zeros((n, 3))
    xyz[:, :2] = xy
    for layout in ("tiles", "csr"):
        P = p2p.Plan.from_grid(dev(xyz), (0.0, 0.0, 0.0), 2.0 ** (1 - level), 0.0, dtype=torch.complex128,
                               layout=layout)
        y = P.apply_log2d(dev(q)).cpu().numpy()
        err = rel_l2(y, ref) if n > 1 else float(np.abs(y - ref).max())
        print("  sweep %s: rel L2 %.2e" % (layout, err), flush=True)
        assert err <= 1e-12
        P.close()


def test_run_before_transfer_and_bad_plan():
    xy, q = points(500, 7)
    Q = p2p.Quad2D("indexing", xy, q, 3)
    with pytest.raises(p2p.P2PError) as e:
        Q.run()
    assert e.value.status == 6
    Q.close()
    xyz = np.zeros((500, 3))
    xyz[:, :2] = xy
    P = p2p.Plan.from_grid(dev(xyz), (0, 0, 0), 0.25, 0.0, dtype=torch.complex64)
    with pytest.raises(p2p.P2PError) as e:
        P.apply_log2d(dev(q))
    assert e.value.status == 3
    P.close()


def test_repeated_runs_and_transfers():
    xy, q = points(16384, 8)
    ref = oracle.apply2d(xy, q, 7)
    Q = p2p.Quad2D("repetition", xy, q, 7)
    for _ in range(2):
        Q.transfer()
        a = Q.run()
        b = Q.run()
        assert torch.equal(a, b)
        assert rel_l2(a.cpu().numpy(), ref) <= 1e-12
    Q.close()
