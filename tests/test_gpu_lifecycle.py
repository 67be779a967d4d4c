"""Plan and batch lifetime on the GPU: double destroy, device allocation failure
(P2P_TEST_FAIL_ALLOC), destroy right after asynchronous work on another stream,
positions that moved after the plan was built, and the autotuner cache read at
plan creation."""
import math

import numpy as np
import pytest
import torch

import paper_2403_01596_amd as p2p
import workloads as W
from gpu_helpers import dev, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def inst():
    return W.sphere(20000, 32, 2 * math.pi * 8, seed=2, m=1, dtype=np.complex64)


def tensors(inst):
    return dev(inst.xyz, torch.float64), dev(inst.ids, torch.int32), dev(inst.q[:, 0].copy())


def test_double_destroy_is_reported(inst):
    xyz, ids, q = tensors(inst)
    P = p2p.Plan(xyz, ids, inst.k)
    h = P.handle
    L = p2p.lib()
    assert L.p2p_plan_destroy(h) == 0
    assert L.p2p_plan_destroy(h) == 6
    assert L.p2p_apply(h, q.data_ptr(), q.data_ptr(), 1, 1, None) == 6
    P._h = None
    m = 16
    P = p2p.Plan(xyz, ids, inst.k, layout="csr", max_rhs=m)
    B = p2p.Batch([P], m)
    hb = B.handle
    assert L.p2p_batch_destroy(hb) == 0
    assert L.p2p_batch_destroy(hb) == 6
    B._h = None
    P.close()


def test_allocation_failure(inst, monkeypatch):
    xyz, ids, q = tensors(inst)
    ref = p2p.Plan(xyz, ids, inst.k, layout="csr").apply(q).cpu().numpy()
    # a build's device allocations, in order: the persistent arrays, the scratch
    # block, the dense cell table (optional: without it the neighbour search
    # bisects the box keys instead) and the neighbour lists
    got = []
    for nth in range(1, 6):
        monkeypatch.setenv("P2P_TEST_FAIL_ALLOC", str(nth))
        try:
            P = p2p.Plan(xyz, ids, inst.k, layout="csr")
        except p2p.P2PError as e:
            got.append(e.status)
            assert "allocation" in str(e)
            continue
        y = P.apply(q).cpu().numpy()
        P.close()
        assert np.array_equal(y, ref)
        got.append(0)
    monkeypatch.delenv("P2P_TEST_FAIL_ALLOC")
    print("  statuses with the n-th allocation failing, n = 1..5:", got, flush=True)
    assert got == [4, 4, 0, 4, 0]
    P = p2p.Plan(xyz, ids, inst.k, layout="csr")
    assert np.array_equal(P.apply(q).cpu().numpy(), ref)
    P.close()


def test_destroy_after_work_on_another_stream(inst):
    xyz, ids, q = tensors(inst)
    ref = p2p.Plan(xyz, ids, inst.k, layout="csr").apply(q).cpu().numpy()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    outs = []
    with torch.cuda.stream(s):
        for _ in range(3):
            P = p2p.Plan(xyz, ids, inst.k, layout="csr")
            outs.append(P.apply(q))
            P.close()  # waits for the apply just enqueued, then hands the memory back
    torch.cuda.current_stream().wait_stream(s)
    for y in outs:
        assert np.array_equal(y.cpu().numpy(), ref)


def test_moved_positions_are_rejected(inst):
    xyz, ids, q = tensors(inst)
    xg = xyz.clone().requires_grad_(True)
    P = p2p.Plan(xg, ids, inst.k)
    y = p2p.P2PFunction.apply(xg, q, P)
    y2 = p2p.P2PFunction.apply(xg.detach().clone(), q, P)  # equal positions in another tensor
    assert torch.equal(y, y2)
    moved = xg.detach().clone()
    moved[5, 0] += 1e-4
    with pytest.raises(ValueError):
        p2p.P2PFunction.apply(moved, q, P)
    with torch.no_grad():
        xg[5, 0] += 1e-4  # an optimizer step, in place
    with pytest.raises(ValueError):
        p2p.P2PFunction.apply(xg, q, P)
    P.close()


def test_tune_cache_read_at_creation(inst, tmp_path):
    xyz, ids, _ = tensors(inst)
    m = 64
    q = dev(W.strengths(inst.n, m, np.random.default_rng(4), np.complex64))
    cache = str(tmp_path / "tune.txt")
    P1 = p2p.Plan(xyz, ids, inst.k, layout="csr", max_rhs=m)
    B = p2p.Batch([P1], m)
    y1 = torch.empty_like(q)
    shape = B.tune([q], [y1], cache)
    B.apply_into([q], [y1])
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].split("\t")[1:3] == [str(shape[0]), str(shape[1])]
    P2 = p2p.Plan(xyz, ids, inst.k, layout="csr", max_rhs=m, tune_cache=cache)
    y2 = P2.apply(q)
    assert rel_l2(y2.cpu().numpy(), y1.cpu().numpy()) < 1e-6
    B.close()
    P1.close()
    P2.close()
