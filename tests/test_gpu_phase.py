"""Parity across the range of phases k r.

The FP64 path reduces the phase in turns to a quarter turn around the nearest
half turn and evaluates sine and cosine from polynomials; the FP32 path takes
the phase in turns in FP32.  These cases push k r well past the few turns of
the benchmark workloads:

- FP64, 8192 uniform points on the 8^3 grid, leaf boxes of 2.5 to 20 wavelengths
  (largest near-pair phase about 9 to 70 turns), both layouts: relative L2 error
  <= 1e-12 against the oracle.  The phase itself is rounded in FP64 on both
  sides, which bounds the disagreement by about 4 pi 2^-53 times the largest
  phase in turns; that stays below 1e-13 here.
- FP32, leaf boxes of 1/4, 1/2, 1 and 4 wavelengths (the method's near field
  uses boxes of a fraction of a wavelength): relative L2 error <= 1e-5.  The
  FP32 path's phase error grows with the phase (its relative rounding is about
  2^-24), so the largest boxes are the ones that approach the bar.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_helpers import gpu_apply, gpu_plan, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("box_wavelengths", [2.5, 20.0])
@pytest.mark.parametrize("layout", ["tiles", "csr"])
def test_f64_large_phase(box_wavelengths, layout):
    h = 1.0 / 8
    k = 2 * math.pi * box_wavelengths / h
    inst = W.cube(8192, 8, k, seed=4, dtype=np.complex128)
    max_turns = k * math.sqrt(3) * 2 * h / (2 * math.pi)
    print("f64 box %.1f wavelengths, largest phase %.1f turns, %s" % (box_wavelengths, max_turns, layout), flush=True)
    y = gpu_apply(gpu_plan(inst.xyz, inst.ids, k, dtype=torch.complex128, layout=layout), inst.q, torch.complex128)
    yref = oracle.Plan(inst.ids).apply(inst.xyz, k, inst.q)
    err = rel_l2(y, yref)
    print("  rel L2 %.3e" % err, flush=True)
    assert err <= 1e-12


@pytest.mark.parametrize("box_wavelengths", [0.25, 0.5, 1.0, 4.0])
def test_f32_phase_regime(box_wavelengths):
    h = 1.0 / 8
    k = 2 * math.pi * box_wavelengths / h
    inst = W.cube(8192, 8, k, seed=4, dtype=np.complex64)
    y = gpu_apply(gpu_plan(inst.xyz, inst.ids, k, dtype=torch.complex64, layout="csr"), inst.q, torch.complex64)
    yref = oracle.Plan(inst.ids).apply(inst.xyz, k, inst.q.astype(np.complex128))
    err = rel_l2(y, yref)
    print("f32 box %.2f wavelengths: rel L2 %.3e" % (box_wavelengths, err), flush=True)
    assert err <= 1e-5
