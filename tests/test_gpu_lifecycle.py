"""Plan and batch lifetime on the GPU: double destroy, device allocation failure
(P2P_TEST_FAIL_ALLOC), destroy right after asynchronous work on another stream,
builds, applies and releases enqueued without host waits (the build returns
before its last kernels end, the release hands memory back behind the work that
used it), a plan used on another stream right after its build, positions that
moved after the plan was built, and the autotuner cache read at plan creation."""
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
            P.close()  # hands the memory back behind the apply just enqueued
    torch.cuda.current_stream().wait_stream(s)
    for y in outs:
        assert np.array_equal(y.cpu().numpy(), ref)


def grid_tensors(inst):
    return (dev(inst.xyz, torch.float64), [float(v) for v in inst.origin], inst.h,
            dev(inst.q[:, 0].copy()))


def test_steps_without_host_waits(inst):
    # two geometries of different sizes in turn, so that each build takes blocks
    # another plan released while its apply could still be running
    other = W.sphere(26000, 16, 2 * math.pi * 6, seed=3, m=1, dtype=np.complex64)
    geoms = [grid_tensors(inst), grid_tensors(other)]
    ks = [inst.k, other.k]
    refs = []
    for g, k in zip(geoms, ks):
        xyz, org, h, q = g
        P = p2p.Plan.from_grid(xyz, org, h, k, layout="csr")
        torch.cuda.synchronize()
        refs.append(P.apply(q).cpu().numpy())
        torch.cuda.synchronize()
        P.close()
        torch.cuda.synchronize()
    outs = []
    for step in range(12):
        xyz, org, h, q = geoms[step % 2]
        P = p2p.Plan.from_grid(xyz, org, h, ks[step % 2], layout="csr" if step % 4 < 2 else "tiles")
        outs.append(P.apply(q))
        P.close()
    torch.cuda.synchronize()
    for step, y in enumerate(outs):
        assert np.array_equal(y.cpu().numpy(), refs[step % 2]), step


def test_plan_used_on_another_stream_right_after_build(inst):
    xyz, org, h, q = grid_tensors(inst)
    P = p2p.Plan.from_grid(xyz, org, h, inst.k, layout="csr")
    torch.cuda.synchronize()
    ref = P.apply(q).cpu().numpy()
    info_ref = P.info()
    export_ref = P.export()
    P.close()
    s_build, s_use = torch.cuda.Stream(), torch.cuda.Stream()
    s_build.wait_stream(torch.cuda.current_stream())
    s_use.wait_stream(torch.cuda.current_stream())
    for rep in range(3):
        with torch.cuda.stream(s_build):
            P = p2p.Plan.from_grid(xyz, org, h, inst.k, layout="csr")
        if rep == 0:  # host reads of the plan right after the build
            assert P.info() == info_ref
            got = P.export()
            assert all(np.array_equal(got[key], export_ref[key]) for key in export_ref)
        with torch.cuda.stream(s_use):
            y = P.apply(q)
        s_use.synchronize()
        assert np.array_equal(y.cpu().numpy(), ref), rep
        with torch.cuda.stream(s_use):
            P.close()
    torch.cuda.synchronize()


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
