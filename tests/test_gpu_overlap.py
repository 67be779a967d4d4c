"""The near field beside other work: an apply and a reverse pass on a stream of
their own while another stream runs matrix products (a far-field stand-in; the
paper's section 1 notes that the P2P operator does not depend on the far field, so
the two can overlap).  Results must be bitwise those of the same calls alone."""
import math

import numpy as np
import pytest
import torch

import paper_2403_01596_amd as p2p
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,layout", [(torch.complex64, "csr"), (torch.complex64, "tiles"),
                                          (torch.complex128, "csr")])
def test_concurrent_with_other_stream(dtype, layout):
    inst = W.sphere(200_000, 32, 2 * math.pi * 16, seed=21, dtype=np.complex64)
    print("overlap: n=%d %s %s" % (inst.n, dtype, layout), flush=True)
    xyz = torch.from_numpy(inst.xyz).cuda()
    q = torch.from_numpy(inst.q[:, 0].copy()).cuda().to(dtype)
    plan = p2p.Plan.from_grid(xyz, [float(v) for v in inst.origin], inst.h, inst.k, dtype=dtype, layout=layout)
    y_ref = plan.apply(q)
    dq_ref, dx_ref = plan.backward(q, q)
    torch.cuda.synchronize()
    s_near, s_far = torch.cuda.Stream(), torch.cuda.Stream()
    a = torch.randn(256, 128, 128, device="cuda")
    b = torch.randn(256, 128, 128, device="cuda")
    c = torch.empty_like(a)
    y = torch.empty_like(y_ref)
    for _ in range(3):
        with torch.cuda.stream(s_far):
            for _ in range(20):
                torch.bmm(a, b, out=c)
        with torch.cuda.stream(s_near):
            plan.apply(q, y)
            dq, dx = plan.backward(q, q)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
        assert torch.equal(dq, dq_ref) and torch.equal(dx, dx_ref)
    plan.close()
