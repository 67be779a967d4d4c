"""Error model of the FP32 path, emulated in FP64 with the oracle (CPU only).

The FP32 kernels take coordinate differences from fixed-point coordinates: each
coordinate rounded to a multiple of a quantum 2^e, with e the smallest exponent
for which the largest per-axis separation of a near pair (from the boxes'
bounding boxes) stays below 2^(e + 30).  These tests pin, on the 2M-point sphere
at 32 points per box (k = 2 pi 64), what that rounding alone does to the result,
and what the close-pair correction leaves:
  - every row of the oracle on rounded coordinates against the oracle on the
    exact ones: the rounding alone costs a few 1e-6 over the whole output, most of
    it from the closest pairs (the term of a pair r apart moves by up to about
    sqrt(3) 2^e / r);
  - the same with every near pair closer than 2^20 quanta put back to its exact
    term (what the plan's correction entries do): below 2e-7.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.slow
CLOSE_QUANTA = 2 ** 20


def quantum_exponent(xyz, tables):
    """Smallest e with max separation of a near pair (bounding boxes) below 2^(e + 30)."""
    bs, perm, ns, ni = tables["box_start"], tables["perm"], tables["nbr_start"], tables["nbr_idx"]
    xs = xyz[perm]
    lo = np.minimum.reduceat(xs, bs[:-1], axis=0)
    hi = np.maximum.reduceat(xs, bs[:-1], axis=0)
    T = np.repeat(np.arange(bs.size - 1), np.diff(ns))
    sep = float(np.max(np.maximum(hi[ni] - lo[T], hi[T] - lo[ni])))
    return math.frexp(sep)[1] - 30


@pytest.fixture(scope="module")
def sphere():
    inst = W.sphere_2m()
    orc = oracle.Plan(inst.ids)
    e = quantum_exponent(inst.xyz, orc.tables())
    y = orc.apply(inst.xyz, inst.k, inst.q)[:, 0]
    return inst, orc, e, y


def kernel(d, k):
    r = np.sqrt((d * d).sum(axis=1))
    return np.exp(1j * k * r) / (4 * np.pi * r)


def test_rounding_alone(sphere):
    inst, orc, e, y = sphere
    xq = np.rint(inst.xyz * 2.0 ** -e) * 2.0 ** e
    yq = orc.apply(xq, inst.k, inst.q)[:, 0]
    err = np.linalg.norm(yq - y) / np.linalg.norm(y)
    print("quantum 2^%d: rounding alone %.3e" % (e, err))
    assert e == -34
    assert 1e-6 < err < 1e-5


def test_rounding_with_close_pairs_exact(sphere):
    from scipy.spatial import cKDTree

    inst, orc, e, y = sphere
    X = np.rint(inst.xyz * 2.0 ** -e)          # fixed-point coordinates (integers)
    xq = X * 2.0 ** e
    yq = orc.apply(xq, inst.k, inst.q)[:, 0]
    pairs = cKDTree(X).query_pairs(CLOSE_QUANTA, output_type="ndarray")
    i, j = pairs[:, 0], pairs[:, 1]
    near = np.all(np.abs(inst.ids[i] - inst.ids[j]) <= 1, axis=1)
    D = X[i] - X[j]
    keep = near & ((D * D).sum(axis=1) < float(CLOSE_QUANTA) ** 2) & np.any(inst.xyz[i] != inst.xyz[j], axis=1)
    i, j = i[keep], j[keep]
    dq = xq[i] - xq[j]
    g_exact = kernel(inst.xyz[i] - inst.xyz[j], inst.k)
    g_round = np.where(np.any(dq != 0, axis=1), kernel(np.where(dq == 0, 1.0, dq), inst.k), 0)
    dg = g_exact - g_round
    q = inst.q[:, 0].astype(np.complex128)
    yc = yq.copy()
    np.add.at(yc, i, dg * q[j])
    np.add.at(yc, j, dg * q[i])
    err = np.linalg.norm(yc - y) / np.linalg.norm(y)
    print("%d close ordered pairs; rounding with them exact %.3e" % (2 * i.size, err))
    assert 1000 < 2 * i.size < 20000
    assert err < 2e-7
