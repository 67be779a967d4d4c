"""Full-size workloads, in the launch configurations the benchmark uses, against the
FP64 oracle.

- 4M points on the (1, 0.5, 0.25) ellipsoid at 16, 32 and 64 points per box with
  k = pi / (2h), both layouts, FP32: pair counts exact, every row of the output;
- the multi-right-hand-side batch (1M sphere points plus 16 uneven instances,
  64 columns each) in one tuned launch: every row of the 1M instance; for the 16
  small ones sampled rows plus the rows of each instance's closest pairs;
- the 500k-point cube's reverse pass (dq and dx), FP32 and FP64, against the
  oracle's full reverse pass, and its FP64 dx against central differences (step
  1e-3, and a Richardson step) of the loss sum |y|^2 computed on the GPU;
- 2^25 points in the unit cube on a 100^3 grid (a million boxes, a replicated
  list of about 900M entries, close to the 2^31 limit of the 32-bit list
  offsets), both layouts, FP32: tables against the oracle's, sampled rows.

Bars: relative L2 error <= 1e-5 (FP32 path), <= 1e-12 (FP64 path).
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


def closest_rows(xyz, count):
    """Rows of the points with the closest neighbours (both points of each pair)."""
    from scipy.spatial import cKDTree

    d, j = cKDTree(xyz).query(xyz, k=2)
    order = np.argsort(d[:, 1])[:count]
    return np.unique(np.concatenate([order, j[order, 1]]))


@pytest.mark.parametrize("d", [16, 32, 64])
def test_ellipsoid_4m(d):
    inst = W.ellipsoid_4m(d)
    print("ellipsoid 4M D=%d generated" % d, flush=True)
    orc = oracle.Plan(inst.ids)
    st = orc.stats(inst.xyz)
    yref = orc.apply(inst.xyz, inst.k, inst.q)
    print("  oracle done", flush=True)
    close = closest_rows(inst.xyz, 200)
    xyz, ids, q = dev(inst.xyz, torch.float64), dev(inst.ids, torch.int32), dev(inst.q)
    for layout in ("tiles", "csr"):
        P = p2p.Plan(xyz, ids, inst.k, dtype=torch.complex64, layout=layout)
        info = P.info()
        assert info["n_boxes"] == orc.n_boxes and info["n_nbr"] == orc.n_nbr
        assert info["n_pairs"] == st["n_pairs"] and info["t_max"] == st["t_max"]
        y = P.apply(q).cpu().numpy()
        err = rel_l2(y, yref)
        err_close = rel_l2(y[close], yref[close])
        print("  %s: %d pairs, %d close-pair entries, rel L2 over every row %.3e, closest-pair rows %.3e" % (
            layout, info["n_pairs"], info["n_close_pairs"], err, err_close), flush=True)
        assert err <= TOL[torch.complex64] and err_close <= TOL[torch.complex64]
        P.close()


def test_multi_rhs_batch_full(tmp_path):
    m = 64
    insts = [W.multi_rhs_main(m)] + W.multi_rhs_batch(m)
    print("batch of %d instances generated" % len(insts), flush=True)
    plans = [gpu_plan(i.xyz, i.ids, i.k, layout="csr", max_rhs=m) for i in insts]
    qs = [dev(i.q) for i in insts]
    ys = [torch.empty_like(q) for q in qs]
    B = p2p.Batch(plans, m)
    B.tune(qs, ys, str(tmp_path / "tune.txt"))
    for y in ys:
        y.fill_(float("nan"))
    B.apply_into(qs, ys)
    torch.cuda.synchronize()
    worst = 0.0
    for j, (inst, y) in enumerate(zip(insts, ys)):
        got = y.cpu().numpy()
        assert np.isfinite(got).all()
        if j == 0:  # the 1M instance: every row
            ref = oracle.Plan(inst.ids).apply(inst.xyz, inst.k, inst.q)
            err = rel_l2(got, ref)
            print("  1M instance, %d columns, every row: rel L2 %.3e" % (m, err), flush=True)
        else:
            rows = np.unique(np.concatenate([np.random.default_rng(j).choice(inst.n, min(inst.n, 300), replace=False),
                                             closest_rows(inst.xyz, 20)]))
            ref = oracle.Plan(inst.ids).apply_rows(inst.xyz, inst.k, inst.q, rows)
            err = rel_l2(got[rows], ref)
        worst = max(worst, err)
        assert err <= TOL[torch.complex64], (j, inst.n, err)
    print("  worst per-instance rel L2 %.3e" % worst, flush=True)
    B.close()
    for pl in plans:
        pl.close()


def test_cube_500k_reverse_pass():
    inst = W.grad_cube_500k()
    orc = oracle.Plan(inst.ids)
    g64 = W.strengths(inst.n, 1, np.random.default_rng(5), np.complex128)
    for dtype in (torch.complex64, torch.complex128):
        npd = np.complex64 if dtype == torch.complex64 else np.complex128
        q, g = inst.q.astype(npd), g64.astype(npd)
        dq_ref, dx_ref = orc.backward(inst.xyz, inst.k, q, g)
        P = gpu_plan(inst.xyz, inst.ids, inst.k, dtype=dtype, layout="csr")
        dq, dx = P.backward(dev(q), dev(g))
        torch.cuda.synchronize()
        e_q = rel_l2(dq.cpu().numpy(), dq_ref)
        e_x = rel_l2(dx.cpu().numpy(), dx_ref)
        print("  %s dq %.3e dx %.3e" % (dtype, e_q, e_x), flush=True)
        assert e_q <= TOL[dtype] and e_x <= TOL[dtype]
        P.close()


def test_cube_33m_both_layouts():
    n, grid = 1 << 25, 100
    k = 2 * math.pi * grid / 4  # boxes of a quarter wavelength
    inst = W.cube(n, grid, k, seed=12, dtype=np.complex64)
    print("cube 2^25 generated", flush=True)
    orc = oracle.Plan(inst.ids)
    rows = np.random.default_rng(12).choice(n, 400, replace=False)
    yref = orc.apply_rows(inst.xyz, k, inst.q, rows)
    xyz, ids, q = dev(inst.xyz, torch.float64), dev(inst.ids, torch.int32), dev(inst.q)
    for layout in ("csr", "tiles"):
        P = p2p.Plan(xyz, ids, k, dtype=torch.complex64, layout=layout)
        info = P.info()
        assert info["n_boxes"] == orc.n_boxes and info["n_nbr"] == orc.n_nbr
        y = P.apply(q)
        torch.cuda.synchronize()
        err = rel_l2(y.cpu().numpy()[rows], yref)
        print("  %s: %d boxes, list %d entries, rel L2 on sampled rows %.3e" % (
            layout, info["n_boxes"], info["tile_entries"], err), flush=True)
        assert err <= TOL[torch.complex64]
        P.close()
        del y


def test_cube_500k_dx_finite_differences():
    inst = W.grad_cube_500k()
    q = dev(inst.q.astype(np.complex128))
    ids = dev(inst.ids, torch.int32)

    def loss(x):
        P = p2p.Plan(dev(x, torch.float64), ids, inst.k, dtype=torch.complex128, layout="csr")
        val = float((P.apply(q).abs() ** 2).sum().item())
        P.close()
        return val

    P = gpu_plan(inst.xyz, inst.ids, inst.k, dtype=torch.complex128, layout="csr")
    _, dx = P.backward(q, 2 * P.apply(q), want_dq=False)
    dx = dx.cpu().numpy()
    P.close()
    rng = np.random.default_rng(5)
    errs_plain, errs_rich = [], []
    for i in rng.choice(inst.n, 6, replace=False):
        scale = np.abs(dx[i]).max()
        for a in range(3):
            d = []
            for h in (1e-3, 5e-4):
                xp, xm = inst.xyz.copy(), inst.xyz.copy()
                xp[i, a] += h
                xm[i, a] -= h
                d.append((loss(xp) - loss(xm)) / (2 * h))
            errs_plain.append(abs(d[0] - dx[i, a]) / scale)
            errs_rich.append(abs((4 * d[1] - d[0]) / 3 - dx[i, a]) / scale)
    print("  500k cube, finite differences: median %.2e (h = 1e-3), median %.2e max %.2e (Richardson)" % (
        np.median(errs_plain), np.median(errs_rich), max(errs_rich)), flush=True)
    # Truncation: the step-1e-3 difference errs by ~ (h / r)^2 for a point whose nearest
    # neighbour is r away, about (1e-3 / 0.007)^2 = 2e-2 at this density; Richardson leaves
    # ~ (h / r)^4, about 4e-4, larger for the few points with a much closer neighbour.
    assert np.median(errs_plain) < 2e-2
    assert np.median(errs_rich) < np.median(errs_plain) / 4
    assert max(errs_rich) < 4e-3
