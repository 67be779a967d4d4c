"""Many right-hand sides on the matrix cores, uneven batches in one launch, graph
capture and the autotuner -- against the FP64 oracle (relative L2 <= 1e-5 per
instance and per column block)."""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2403_01596_amd as p2p
import workloads as W
from cases import plan_cases
from gpu_helpers import dev, gpu_plan, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5


def strengths(n, m, seed):
    return W.strengths(n, m, np.random.default_rng(seed), np.complex64)


@pytest.mark.parametrize("layout", ["csr", "tiles"])
@pytest.mark.parametrize("m", [6, 12, 16, 20, 33, 64, 71])
def test_single_plan_many_rhs(layout, m):
    inst = W.sphere(30000, 32, 2 * math.pi * 10, seed=61)
    q = strengths(inst.n, m, 7)
    P = gpu_plan(inst.xyz, inst.ids, inst.k, layout=layout, max_rhs=m)
    y = P.apply(dev(q))
    torch.cuda.synchronize()
    yref = oracle.Plan(inst.ids).apply(inst.xyz, inst.k, q)
    err = rel_l2(y.cpu().numpy(), yref)
    print("m=%d %s rel L2 %.3e" % (m, layout, err), flush=True)
    assert err <= TOL
    # every column block on its own
    for c0 in range(0, m, 16):
        assert rel_l2(y.cpu().numpy()[:, c0:c0 + 16], yref[:, c0:c0 + 16]) <= TOL


@pytest.mark.parametrize("case", list(plan_cases()), ids=lambda c: c[0])
@pytest.mark.parametrize("layout", ["csr", "tiles"])
@pytest.mark.parametrize("m", [64, 24])
def test_plan_cases_many_rhs(case, layout, m):
    """Every parity case on the matrix-core path: m = 64 takes the fast form (whole
    64-column items, 32-bit offsets), m = 24 the general one (clamped columns).
    Covers duplicates and coincident points across boxes (the masked form
    everywhere), boxes over 16 targets, lists over one LDS group and one point."""
    name, xyz, ids, k = case
    q = strengths(xyz.shape[0], m, 9)
    P = gpu_plan(xyz, ids, k, layout=layout, max_rhs=m)
    y = P.apply(dev(q)).cpu().numpy()
    yref = oracle.Plan(ids).apply(xyz, k, q)
    if np.linalg.norm(yref) == 0:
        assert np.all(y == 0)
        return
    err = rel_l2(y, yref)
    print("%s %s m=%d rel L2 %.3e" % (name, layout, m, err), flush=True)
    assert err <= TOL


def test_many_rhs_laplace_and_dense_boxes():
    inst = W.cube(12000, 3, 0.0, seed=62, dtype=np.complex64)  # > 64 targets per box, k = 0
    q = strengths(inst.n, 32, 8)
    P = gpu_plan(inst.xyz, inst.ids, 0.0, layout="csr", max_rhs=32)
    y = P.apply(dev(q)).cpu().numpy()
    assert rel_l2(y, oracle.Plan(inst.ids).apply(inst.xyz, 0.0, q)) <= TOL


def uneven_instances(m):
    sizes = [2000, 5000, 9000, 15000, 24000, 40000]
    out = []
    for j, nj in enumerate(sizes):
        inst = W.sphere(nj, 32, 2 * math.pi * 6, seed=70 + j)
        out.append((inst, strengths(nj, m, 100 + j)))
    return out


@pytest.mark.parametrize("layout", ["csr", "tiles"])
def test_uneven_batch_one_launch(layout):
    m = 64
    data = uneven_instances(m)
    plans = [gpu_plan(i.xyz, i.ids, i.k, layout=layout, max_rhs=m) for i, _ in data]
    B = p2p.Batch(plans, m)
    qs = [dev(q) for _, q in data]
    ys = B.apply(qs)
    torch.cuda.synchronize()
    for (inst, q), y in zip(data, ys):
        err = rel_l2(y.cpu().numpy(), oracle.Plan(inst.ids).apply(inst.xyz, inst.k, q))
        print("n=%d rel L2 %.3e" % (inst.n, err), flush=True)
        assert err <= TOL
    B.close()


def test_graph_capture_replays():
    m = 64
    data = uneven_instances(m)[:4]
    plans = [gpu_plan(i.xyz, i.ids, i.k, layout="csr", max_rhs=m) for i, _ in data]
    B = p2p.Batch(plans, m)
    qs = [dev(q) for _, q in data]
    ys = [torch.empty_like(q) for q in qs]
    eager = [y.clone() for y in B.apply(qs)]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.apply_into(qs, ys)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        B.apply_into(qs, ys)
    for rep in range(3):
        for y in ys:
            y.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for y, e in zip(ys, eager):
            assert torch.equal(y, e), rep
        # eager work between replays, and new strengths read by the next replay
        for q in qs:
            q.mul_(2.0)
        eager = [e * 2.0 for e in eager]
        torch.cuda.synchronize()
    B.close()


@pytest.mark.parametrize("m", [64, 12])
def test_tuner_and_cache(tmp_path, m):
    data = uneven_instances(m)[:3]
    plans = [gpu_plan(i.xyz, i.ids, i.k, layout="csr", max_rhs=m) for i, _ in data]
    B = p2p.Batch(plans, m)
    qs = [dev(q) for _, q in data]
    ys = [torch.empty_like(q) for q in qs]
    ref = [y.clone() for y in B.apply(qs)]
    cache = str(tmp_path / "tune.txt")
    w, p = B.tune(qs, ys, cache)
    assert (w in (32, 64) if m > 32 else w == 16) and p in (1, 2, 4)
    assert os.path.exists(cache) and open(cache).read().count("\n") == 1
    # the same key comes back from the file without a second entry
    assert B.tune(qs, ys, cache) == (w, p)
    assert open(cache).read().count("\n") == 1
    out = B.apply(qs)
    torch.cuda.synchronize()
    # launch shapes change scheduling only, not the order of the sums
    for a, b in zip(out, ref):
        assert torch.equal(a, b)
    B.close()


def test_batch_errors():
    inst = W.sphere(3000, 32, 10.0, seed=1)
    P64 = gpu_plan(inst.xyz, inst.ids, inst.k, dtype=torch.complex128, max_rhs=16)
    with pytest.raises(p2p.P2PError) as e:
        p2p.Batch([P64], 16)
    assert e.value.status == 3
    P1 = gpu_plan(inst.xyz, inst.ids, inst.k, max_rhs=8)
    with pytest.raises(p2p.P2PError) as e:
        p2p.Batch([P1], 16)
    assert e.value.status == 1
    Pc = gpu_plan(inst.xyz, inst.ids, inst.k, layout="csr", max_rhs=16)
    Pt = gpu_plan(inst.xyz, inst.ids, inst.k, layout="tiles", max_rhs=16)
    with pytest.raises(p2p.P2PError):
        p2p.Batch([Pc, Pt], 16)
