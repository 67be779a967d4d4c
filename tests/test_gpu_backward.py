"""GPU reverse pass (dq, dx) against the oracle's gradients and through autograd.

Loss L = sum |y|^2, upstream g = 2 y.  Bars as for the forward pass: relative L2
error <= 1e-12 (FP64 path) and <= 1e-5 (FP32 path), dq and dx separately.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2403_01596_amd as p2p
import workloads as W
from gpu_helpers import dev, gpu_plan, rel_l2

pytestmark = pytest.mark.gpu

TOL = {torch.complex128: 1e-12, torch.complex64: 1e-5}


def cases():
    yield "cube_g6", W.cube(6000, 6, 2 * math.pi * 2, seed=41, dtype=np.complex128)
    yield "sphere_D32", W.sphere(30000, 32, 2 * math.pi * 10, seed=42, dtype=np.complex128)
    yield "cube_k0", W.cube(4000, 5, 0.0, seed=43, dtype=np.complex128)
    yield "dense_g3", W.cube(9000, 3, 5.0, seed=44, dtype=np.complex128)


@pytest.mark.parametrize("case", list(cases()), ids=lambda c: c[0])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["f64", "f32"])
@pytest.mark.parametrize("layout", ["tiles", "csr"])
def test_backward_matches_oracle(case, dtype, layout):
    name, inst = case
    print("backward", name, dtype, layout, flush=True)
    npd = np.complex64 if dtype == torch.complex64 else np.complex128
    q = inst.q.astype(npd)
    orc = oracle.Plan(inst.ids)
    y = orc.apply(inst.xyz, inst.k, q)
    g = (2 * y).astype(npd)
    dq_ref, dx_ref = orc.backward(inst.xyz, inst.k, q, g)
    P = gpu_plan(inst.xyz, inst.ids, inst.k, dtype=dtype, layout=layout)
    dq, dx = P.backward(dev(q), dev(g))
    torch.cuda.synchronize()
    e_q = rel_l2(dq.cpu().numpy(), dq_ref)
    e_x = rel_l2(dx.cpu().numpy(), dx_ref)
    print("  dq %.3e dx %.3e" % (e_q, e_x), flush=True)
    assert e_q <= TOL[dtype]
    assert e_x <= TOL[dtype]
    # each output alone
    dq1, none = P.backward(dev(q), dev(g), want_dx=False)
    none2, dx1 = P.backward(dev(q), dev(g), want_dq=False)
    assert none is None and none2 is None
    assert torch.equal(dq1, dq) and torch.equal(dx1, dx)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["f64", "f32"])
def test_autograd_function(dtype):
    inst = W.cube(5000, 5, 2 * math.pi * 3, seed=45, dtype=np.complex128)
    npd = np.complex64 if dtype == torch.complex64 else np.complex128
    xyz = dev(inst.xyz).requires_grad_(True)
    q = dev(inst.q.astype(npd)).requires_grad_(True)
    P = p2p.Plan(xyz.detach(), dev(inst.ids), inst.k, dtype=dtype)
    y = p2p.P2PFunction.apply(xyz, q, P)
    loss = (y.abs() ** 2).sum()
    loss.backward()
    orc = oracle.Plan(inst.ids)
    qq = inst.q.astype(npd)
    yref = orc.apply(inst.xyz, inst.k, qq)
    dq_ref, dx_ref = orc.backward(inst.xyz, inst.k, qq, 2 * yref)
    assert rel_l2(q.grad.cpu().numpy(), dq_ref) <= TOL[dtype]
    assert rel_l2(xyz.grad.cpu().numpy(), dx_ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["f64", "f32"])
@pytest.mark.parametrize("layout", ["tiles", "csr"])
@pytest.mark.parametrize("m", [2, 7])
def test_multi_rhs_backward(dtype, layout, m):
    # columns go in launches of 4, 2 and 1 (7 = 4 + 2 + 1); dx sums over all of them
    npd = np.complex128 if dtype == torch.complex128 else np.complex64
    inst = W.sphere(20000, 32, 2 * math.pi * 8, seed=46, m=m, dtype=np.complex128)
    orc = oracle.Plan(inst.ids)
    q = inst.q.astype(npd)
    g = (2 * orc.apply(inst.xyz, inst.k, q)).astype(npd)
    dq_ref, dx_ref = orc.backward(inst.xyz, inst.k, q, g)
    P = gpu_plan(inst.xyz, inst.ids, inst.k, dtype=dtype, layout=layout, max_rhs=m)
    for want_dq, want_dx in ((True, True), (True, False), (False, True)):
        dq, dx = P.backward(dev(q), dev(g), want_dq=want_dq, want_dx=want_dx)
        torch.cuda.synchronize()
        if want_dq:
            assert rel_l2(dq.cpu().numpy(), dq_ref) <= TOL[dtype]
        if want_dx:
            assert rel_l2(dx.cpu().numpy(), dx_ref) <= TOL[dtype]


def test_dx_against_finite_differences_on_gpu():
    """The GPU reverse pass (FP64) against central differences of the GPU forward
    pass: L = sum |y|^2 with the ids held fixed, each difference rebuilding the plan
    for the moved point.  Step 1e-3 as the evaluation prescribes, then a Richardson
    step (1e-3 and 5e-4) that removes the O(h^2) truncation term."""
    inst = W.cube(3000, 6, 2 * math.pi * 3, seed=9, dtype=np.complex128)
    ids = dev(inst.ids, torch.int32)
    q = dev(inst.q)

    def loss(x):
        P = p2p.Plan(dev(x, torch.float64), ids, inst.k, dtype=torch.complex128, layout="csr")
        y = P.apply(q)
        val = float((y.abs() ** 2).sum().item())
        P.close()
        return val

    P = gpu_plan(inst.xyz, inst.ids, inst.k, dtype=torch.complex128, layout="csr")
    y = P.apply(q)
    _, dx = P.backward(q, 2 * y, want_dq=False)
    dx = dx.cpu().numpy()
    P.close()

    def fd(i, a, h):
        xp = inst.xyz.copy()
        xm = inst.xyz.copy()
        xp[i, a] += h
        xm[i, a] -= h
        return (loss(xp) - loss(xm)) / (2 * h)

    rng = np.random.default_rng(3)
    errs_plain, errs_rich = [], []
    for i in rng.choice(inst.n, 6, replace=False):
        scale = np.abs(dx[i]).max()
        for a in range(3):
            d1 = fd(i, a, 1e-3)
            d2 = fd(i, a, 5e-4)
            errs_plain.append(abs(d1 - dx[i, a]) / scale)
            errs_rich.append(abs((4 * d2 - d1) / 3 - dx[i, a]) / scale)
    print("finite differences: median %.2e (h = 1e-3), max %.2e (Richardson)" % (
        np.median(errs_plain), max(errs_rich)), flush=True)
    # measured: median 1.1e-4 and max 1.2e-7; the truncation term is ~ (h / r_nn)^2
    assert np.median(errs_plain) < 2e-3
    assert max(errs_rich) < 1e-5
