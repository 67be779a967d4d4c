"""The seeded generators are deterministic and produce the intended shapes (CPU only)."""
import hashlib
import json
import math
import os

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_recorded_digests():
    with open(os.path.join(HERE, "golden", "inputs_sha256.json")) as f:
        rec = json.load(f)
    made = {
        "cube8192_g8_k8pi_c128": W.plain_f64_cube(),
        "sphere20k_D32": W.sphere(20000, 32, 2 * math.pi * 8, seed=0, name="sphere20k_D32"),
        "ellipsoid20k_D16": W.ellipsoid(20000, 16, seed=0, name="ellipsoid20k_D16"),
        "cube5000_g5_c64": W.cube(5000, 5, 2 * math.pi * 2, seed=0, dtype=np.complex64, name="cube5000_g5_c64"),
    }
    assert set(made) == set(rec)
    for name, inst in made.items():
        assert digest(inst.xyz, inst.ids, inst.q) == rec[name]["sha256"], name
        assert inst.h == rec[name]["h"]


def test_density_and_surfaces():
    s = W.sphere(50000, 32, 10.0, seed=3)
    assert abs(s.d_mean / 32 - 1) <= 0.02
    assert np.allclose(np.linalg.norm(s.xyz, axis=1), 1.0)
    e = W.ellipsoid(50000, 16, seed=4)
    assert abs(e.d_mean / 16 - 1) <= 0.02
    a, b, c = 1.0, 0.5, 0.25
    f = (e.xyz[:, 0] / a) ** 2 + (e.xyz[:, 1] / b) ** 2 + (e.xyz[:, 2] / c) ** 2
    assert np.allclose(f, 1.0)
    assert e.k == pytest.approx(math.pi / (2 * e.h))
    assert s.q.dtype == np.complex64 and e.q.dtype == np.complex64


def test_cube_grid_and_sizes():
    c = W.plain_f64_cube()
    assert c.ids.min() == 0 and c.ids.max() == 7 and c.q.dtype == np.complex128
    assert np.array_equal(c.ids, np.floor(c.xyz * 8).astype(np.int32))
    sizes = W.uneven_sizes()
    assert sizes[0] == 10000 and sizes[-1] == 200000 and len(sizes) == 16
