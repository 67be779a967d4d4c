"""GPU apply y = A_near q against the FP64 oracle.

Bars: relative L2 error <= 1e-12 for the FP64 path and <= 1e-5 for the FP32 path
(complex64 strengths promoted exactly to complex128 for the oracle).
"""
import ctypes
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2403_01596_amd as p2p
import workloads as W
from cases import plan_cases
from gpu_helpers import dev, gpu_apply, gpu_plan, rel_l2

pytestmark = pytest.mark.gpu

CASES = list(plan_cases())
TOL = {torch.complex128: 1e-12, torch.complex64: 1e-5}


def strengths(n, m, dtype, seed=99):
    q = W.strengths(n, m, np.random.default_rng(seed), np.complex64 if dtype == torch.complex64 else np.complex128)
    return q


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["f64", "f32"])
@pytest.mark.parametrize("layout", ["tiles", "csr"])
def test_apply_matches_oracle(case, dtype, layout):
    name, xyz, ids, k = case
    print("apply", name, dtype, layout, flush=True)
    q = strengths(xyz.shape[0], 1, dtype)
    y = gpu_apply(gpu_plan(xyz, ids, k, dtype=dtype, layout=layout), q, dtype)
    yref = oracle.Plan(ids).apply(xyz, k, q)
    if np.linalg.norm(yref) == 0:
        assert np.all(y == 0)
        return
    err = rel_l2(y, yref)
    print("  rel L2 %.3e" % err, flush=True)
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["f64", "f32"])
@pytest.mark.parametrize("layout", ["tiles", "csr"])
@pytest.mark.parametrize("m", [3, 5, 7, 11, 15])
def test_multiple_rhs(dtype, layout, m):
    # complex64 plans: up to 5 columns in launches of 4, 2 and 1 (3 = 2 + 1, 5 = 4 + 1), from 6
    # columns on the matrix cores; complex128 plans: launches of 8, 4, 2 and 1 (7 = 4 + 2 + 1,
    # 11 = 8 + 2 + 1, 15 = 8 + 4 + 2 + 1)
    inst = W.sphere(30000, 32, 2 * math.pi * 10, seed=11)
    q = strengths(inst.n, m, dtype, seed=5)
    P = gpu_plan(inst.xyz, inst.ids, inst.k, dtype=dtype, layout=layout, max_rhs=m)
    y = gpu_apply(P, q, dtype)
    yref = oracle.Plan(inst.ids).apply(inst.xyz, inst.k, q)
    for c in range(m):
        assert rel_l2(y[:, c], yref[:, c]) <= TOL[dtype], c
    # the same columns one at a time give the same numbers up to rounding
    P1 = gpu_plan(inst.xyz, inst.ids, inst.k, dtype=dtype, layout=layout)
    y1 = np.stack([gpu_apply(P1, np.ascontiguousarray(q[:, c:c + 1]), dtype)[:, 0] for c in range(m)], axis=1)
    assert rel_l2(y, y1) <= TOL[dtype]


def test_deterministic_and_layouts_agree():
    inst = W.ellipsoid(40000, 32, seed=3)
    q = strengths(inst.n, 1, torch.complex64)
    Pt = gpu_plan(inst.xyz, inst.ids, inst.k, layout="tiles")
    Pc = gpu_plan(inst.xyz, inst.ids, inst.k, layout="csr")
    y1 = gpu_apply(Pt, q, torch.complex64)
    y2 = gpu_apply(Pt, q, torch.complex64)
    y3 = gpu_apply(Pc, q, torch.complex64)
    assert np.array_equal(y1, y2)
    # the two layouts visit the same sources in the same order
    assert np.array_equal(y1, y3)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["f64", "f32"])
def test_invariants_on_gpu_output(dtype):
    inst = W.sphere(30000, 24, 2 * math.pi * 6, seed=12, dtype=np.complex128)
    P = gpu_plan(inst.xyz, inst.ids, inst.k, dtype=dtype)
    rng = np.random.default_rng(2)
    u = strengths(inst.n, 1, dtype, seed=31)
    v = strengths(inst.n, 1, dtype, seed=32)
    au = gpu_apply(P, u, dtype)[:, 0]
    av = gpu_apply(P, v, dtype)[:, 0]
    lhs = (u[:, 0].astype(np.complex128) * av).sum()
    rhs = (v[:, 0].astype(np.complex128) * au).sum()
    # reciprocity: u^T A v = v^T A u
    assert abs(lhs - rhs) <= 10 * TOL[dtype] * np.sqrt(np.sum(np.abs(u) ** 2) * np.sum(np.abs(av) ** 2))
    # k = 0: a real operator
    P0 = gpu_plan(inst.xyz, inst.ids, 0.0, dtype=dtype)
    yr = gpu_apply(P0, u.real.astype(u.dtype), dtype)
    assert np.all(yr.imag == 0)


def test_sphere_2m_sampled_rows():
    """The 2M-point sphere at full size, in the benchmark's launch configuration:
    FP32 and FP64 paths on 4000 sampled rows against the oracle row by row."""
    inst = W.sphere_2m()
    print("sphere 2M generated", flush=True)
    rows = np.random.default_rng(0).choice(inst.n, 4000, replace=False)
    orc = oracle.Plan(inst.ids)
    yref = orc.apply_rows(inst.xyz, inst.k, inst.q, rows)
    for dtype in (torch.complex64, torch.complex128):
        P = gpu_plan(inst.xyz, inst.ids, inst.k, dtype=dtype)
        y = gpu_apply(P, inst.q, dtype)
        err = rel_l2(y[rows], yref)
        print("  %s rel L2 on sampled rows %.3e" % (dtype, err), flush=True)
        assert err <= TOL[dtype]
        inf = P.info()
        assert inf["n_boxes"] > 50000 and inf["t_max"] > 64
        del P


@pytest.mark.parametrize("layout", ["csr", "tiles"])
@pytest.mark.parametrize("m", [1, 5, 7])
def test_graph_capture_of_apply_and_backward(layout, m):
    """p2p_apply and p2p_apply_backward allocate nothing and do not synchronise, so a
    HIP graph can hold them: three replays, with eager work and new inputs between
    them, each equal bitwise to an eager call on the same inputs.  Five columns take
    launches of 4 and 1 columns in both passes; seven take the matrix cores forward
    and launches of 4, 2 and 1 columns backward."""
    inst = W.sphere(40000, 32, 2 * math.pi * 10, seed=77)
    P = gpu_plan(inst.xyz, inst.ids, inst.k, layout=layout, max_rhs=m)
    q = dev(W.strengths(inst.n, m, np.random.default_rng(4), np.complex64))
    g = dev(W.strengths(inst.n, m, np.random.default_rng(3), np.complex64))
    y = torch.empty_like(q)
    dq = torch.empty_like(q)
    dx = torch.empty((inst.n, 3), dtype=torch.float64, device="cuda")
    lib = p2p.lib()

    def calls():
        s = torch.cuda.current_stream().cuda_stream
        p = lambda t: ctypes.c_void_p(t.data_ptr())
        assert lib.p2p_apply(P.handle, p(q), p(y), m, 1, ctypes.c_void_p(s)) == 0
        assert lib.p2p_apply_backward(P.handle, p(q), p(g), p(dq), p(dx), m, 1, ctypes.c_void_p(s)) == 0

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        calls()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        calls()
    for rep in range(3):
        q.mul_(1.5)
        g.add_(0.25)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = (y.clone(), dq.clone(), dx.clone())
        ey = P.apply(q)
        edq, edx = P.backward(q, g)
        torch.cuda.synchronize()
        assert torch.equal(got[0], ey), rep
        assert torch.equal(got[1], edq), rep
        assert torch.equal(got[2], edx), rep
