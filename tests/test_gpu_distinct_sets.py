"""Plans of distinct target and source sets (the paper keeps the two in separate
arrays, section 3.1): y_i = sum over sources j near target i, t_i != s_j, of
G(|t_i - s_j|) q_j.  Reference: the oracle on the union of both sets with zero
strengths on the targets, whose rows for the targets are that sum by definition."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2403_01596_amd as p2p
import workloads as W
from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu
ORIGIN, H = np.array([-1.05, -1.05, -1.05]), 0.06


def sets(nt, ns, seed):
    rng = np.random.default_rng(seed)
    t = W.sphere_surface(nt, rng)
    s = W.sphere_surface(ns, rng)
    if nt > 10 and ns > 10:
        s[:5] = t[:5]                        # sources on targets: skipped (r = 0)
        s[5:10] = t[5:10] + 1e-9             # and very close to them
    return t, s


def reference(t, s, k, q):
    both = np.concatenate([t, s])
    qb = np.concatenate([np.zeros((t.shape[0],) + q.shape[1:], q.dtype), q])
    ids = W.leaf_ids(both, ORIGIN, H)
    return oracle.Plan(ids).apply(both, k, qb.reshape(both.shape[0], -1))[:t.shape[0]]


@pytest.mark.parametrize("dtype,layout", [(torch.complex64, "csr"), (torch.complex64, "tiles"),
                                          (torch.complex128, "csr"), (torch.complex128, "tiles")])
@pytest.mark.parametrize("m", [1, 3, 8])
def test_distinct_sets_match_oracle(dtype, layout, m):
    t, s = sets(30_000, 45_000, 7)
    k = 2 * math.pi * 6
    rng = np.random.default_rng(m)
    q = W.strengths(s.shape[0], m, rng, np.complex64)
    if dtype == torch.complex128:
        q = q.astype(np.complex128)
    print("distinct sets: %s %s m=%d" % (dtype, layout, m), flush=True)
    P = p2p.Plan.from_sets(torch.from_numpy(t).cuda(), torch.from_numpy(s).cuda(), ORIGIN, H, k, dtype=dtype,
                           layout=layout, max_rhs=m)
    qd = torch.from_numpy(q if m > 1 else q[:, 0].copy()).cuda()
    y = P.apply(qd).cpu().numpy().reshape(t.shape[0], m)
    ref = reference(t, s, k, q)
    err = rel_l2(y, ref)
    print("  rel L2 %.2e" % err, flush=True)
    assert err <= (1e-5 if dtype == torch.complex64 else 1e-12)
    P.close()


def test_pair_count_and_refusals():
    t, s = sets(3000, 4000, 11)
    P = p2p.Plan.from_sets(torch.from_numpy(t).cuda(), torch.from_numpy(s).cuda(), ORIGIN, H, 10.0,
                           dtype=torch.complex64, layout="csr")
    info = P.info()
    ti, si = W.leaf_ids(t, ORIGIN, H).astype(np.int64), W.leaf_ids(s, ORIGIN, H).astype(np.int64)
    near = np.all(np.abs(ti[:, None, :] - si[None, :, :]) <= 1, axis=2)
    zero = np.all(t[:, None, :] == s[None, :, :], axis=2)
    assert info["n_targets"] == 3000 and info["n_points"] == 7000
    assert info["n_pairs"] == int((near & ~zero).sum()) and info["n_zero_pairs"] == int((near & zero).sum())
    q = torch.zeros(4000, dtype=torch.complex64, device="cuda")
    with pytest.raises(p2p.P2PError):
        P.backward(q, q)
    with pytest.raises(p2p.P2PError):
        p2p.Batch([P], 8)
    P.close()
    # no targets, or no sources: valid, trivially
    E = p2p.Plan.from_sets(torch.empty((0, 3), dtype=torch.float64, device="cuda"), torch.from_numpy(s).cuda(),
                           ORIGIN, H, 10.0)
    assert E.apply(torch.ones(4000, dtype=torch.complex64, device="cuda")).shape == (0,)
    E.close()
    F = p2p.Plan.from_sets(torch.from_numpy(t).cuda(), torch.empty((0, 3), dtype=torch.float64, device="cuda"),
                           ORIGIN, H, 10.0)
    y = F.apply(torch.empty(0, dtype=torch.complex64, device="cuda"))
    assert y.shape == (3000,) and bool((y == 0).all())
    F.close()
