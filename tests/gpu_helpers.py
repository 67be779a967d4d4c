"""Shared helpers for the GPU tests: device transfer, error metric, plan construction."""
import numpy as np
import torch

import paper_2403_01596_amd as p2p


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def gpu_plan(xyz, ids, k, dtype=torch.complex64, layout="tiles", max_rhs=1):
    return p2p.Plan(dev(xyz, torch.float64), dev(ids, torch.int32), k, dtype=dtype, layout=layout, max_rhs=max_rhs)


def gpu_apply(plan, q, dtype):
    qd = dev(q.astype(np.complex64 if dtype == torch.complex64 else np.complex128))
    y = plan.apply(qd)
    torch.cuda.synchronize()
    return y.cpu().numpy()
