"""Pins for the oracle's reverse pass (CPU only).

Loss L = sum |y|^2 with y = A_near q, upstream g = 2 y (the gradient of a real
loss with respect to a complex tensor is dL/dRe + i dL/dIm).  The oracle's
closed-form gradients are checked against:
  * central differences in q, which are exact for a quadratic loss;
  * forward-mode dual numbers through the forward sum, in x;
  * central differences in x (step 1e-3 as the evaluation prescribes, with a
    Richardson step for a tighter bound);
  * the identities of a loss that depends on distances only: the gradients sum
    to zero (translation), sum x_i x dx_i = 0 (rotation), and at k = 0,
    sum x_i . dx_i = -2 L (the Laplace kernel is homogeneous of degree -1).
Ids are held fixed throughout: the near-field pair set does not move with x.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def cases():
    yield "cube", W.cube(1500, 5, 7.0, seed=21, m=1, dtype=np.complex128)
    yield "sphere_m2", W.sphere(1800, 8, 2 * math.pi * 2, seed=22, m=2, dtype=np.complex128)
    yield "cube_k0", W.cube(1200, 4, 0.0, seed=23, m=1, dtype=np.complex128)


CASES = list(cases())


def loss_rows(P, xyz, k, q, rows):
    y = P.apply_rows(xyz, k, q, rows)
    return float((np.abs(y) ** 2).sum())


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_dq_exact_differences(case):
    _, inst = case
    P = oracle.Plan(inst.ids)
    y = P.apply(inst.xyz, inst.k, inst.q)
    dq, _ = P.backward(inst.xyz, inst.k, inst.q, 2 * y, want_dx=False)
    rng = np.random.default_rng(0)
    for j in rng.choice(inst.n, 12, replace=False):
        rows = P.near_rows(j)
        for c in range(inst.m):
            for part, unit in (("re", 1.0), ("im", 1j)):
                qp = inst.q.copy()
                qm = inst.q.copy()
                qp[j, c] += unit
                qm[j, c] -= unit
                # L is quadratic in q: the central difference with step 1 is exact
                fd = 0.5 * (loss_rows(P, inst.xyz, inst.k, qp, rows) - loss_rows(P, inst.xyz, inst.k, qm, rows))
                got = dq[j, c].real if part == "re" else dq[j, c].imag
                scale = np.abs(dq[j]).max()
                assert abs(got - fd) < 1e-10 * scale, (j, c, part, got, fd)
    # and the adjoint identity dq = conj(A conj(g))
    ref = np.conj(P.apply(inst.xyz, inst.k, np.conj(2 * y)))
    assert np.linalg.norm(dq - ref) < 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_dx_dual_numbers(case):
    _, inst = case
    P = oracle.Plan(inst.ids)
    y = P.apply(inst.xyz, inst.k, inst.q)
    _, dx = P.backward(inst.xyz, inst.k, inst.q, 2 * y, want_dq=False)
    rng = np.random.default_rng(1)
    for i in rng.choice(inst.n, 10, replace=False):
        for a in range(3):
            d = P.dual_dx(inst.xyz, inst.k, inst.q, i, a)
            assert abs(dx[i, a] - d) < 1e-10 * np.abs(dx[i]).max(), (i, a, dx[i, a], d)


@pytest.mark.parametrize("case", CASES[:2], ids=lambda c: c[0])
def test_dx_finite_differences(case):
    _, inst = case
    P = oracle.Plan(inst.ids)
    y = P.apply(inst.xyz, inst.k, inst.q)
    _, dx = P.backward(inst.xyz, inst.k, inst.q, 2 * y, want_dq=False)
    rng = np.random.default_rng(2)

    def fd(i, a, h, rows):
        xp = inst.xyz.copy()
        xm = inst.xyz.copy()
        xp[i, a] += h
        xm[i, a] -= h
        return (loss_rows(P, xp, inst.k, inst.q, rows) - loss_rows(P, xm, inst.k, inst.q, rows)) / (2 * h)

    errs_plain, errs_rich = [], []
    for i in rng.choice(inst.n, 8, replace=False):
        rows = P.near_rows(i)
        for a in range(3):
            d1 = fd(i, a, 1e-3, rows)
            d2 = fd(i, a, 5e-4, rows)
            rich = (4 * d2 - d1) / 3
            scale = np.abs(dx[i]).max()
            errs_plain.append(abs(d1 - dx[i, a]) / scale)
            errs_rich.append(abs(rich - dx[i, a]) / scale)
    # truncation error of the step-1e-3 difference is ~ (h / r_nn)^2; Richardson removes that term
    assert np.median(errs_plain) < 1e-2
    assert max(errs_rich) < 1e-4
    assert np.median(errs_rich) < np.median(errs_plain)


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_dx_identities(case):
    _, inst = case
    P = oracle.Plan(inst.ids)
    y = P.apply(inst.xyz, inst.k, inst.q)
    _, dx = P.backward(inst.xyz, inst.k, inst.q, 2 * y, want_dq=False)
    mag = np.abs(dx).sum()
    assert np.abs(dx.sum(axis=0)).max() < 1e-12 * mag
    c = inst.xyz - inst.xyz.mean(axis=0)
    torque = np.cross(c, dx).sum(axis=0)
    assert np.abs(torque).max() < 1e-12 * (np.abs(c).max() * mag)
    if inst.k == 0.0:
        L = float((np.abs(y) ** 2).sum())
        assert abs((inst.xyz * dx).sum() + 2 * L) < 1e-11 * L
