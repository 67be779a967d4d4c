"""Small seeded point sets for the parity tests (sizes the oracle finishes in seconds).

Each case: (name, xyz float64 [n,3], ids int32 [n,3], k).  Together they span
several tiles of the kernels (boxes with more than 64 targets and neighbourhoods
of more than 512 sources), ragged tails, empty and boundary boxes, duplicates,
ids that disagree with positions, k = 0 and extreme ids.
"""
import math

import numpy as np

import workloads as W


def plan_cases():
    rng = np.random.default_rng(123)
    lim = 1 << 21
    c1 = W.plain_f64_cube()
    yield "cube8192_g8", c1.xyz, c1.ids, c1.k
    s = W.sphere(20000, 32, 2 * math.pi * 8, seed=5)
    yield "sphere20k_D32", s.xyz, s.ids, s.k
    e = W.ellipsoid(20000, 16, seed=6)
    yield "ellipsoid20k_D16", e.xyz, e.ids, e.k
    # dense boxes: more than 64 targets per box and long neighbourhood lists
    d = W.cube(12000, 3, 3.0, seed=7)
    yield "dense_g3", d.xyz, d.ids, d.k
    x = rng.random((3000, 3))
    x[10:20] = x[5]
    yield "duplicates", x, W.leaf_ids(x, (0, 0, 0), 0.2), 9.0
    x = rng.random((2500, 3))
    ids = rng.integers(0, 5, size=(2500, 3)).astype(np.int32)
    yield "ids_not_positions", x, ids, 4.0
    # coincident points whose ids put them in adjacent boxes
    x = rng.random((2000, 3))
    ids = W.leaf_ids(x, (0, 0, 0), 0.25)
    x[1000:1010] = x[0:10]
    ids[1000:1010] = ids[0:10] + np.array([1, 0, 0], np.int32)
    yield "coincident_across_boxes", x, ids, 6.0
    x = rng.random((4000, 3)) * 6
    x = x[~np.all((x >= 1) & (x < 5), axis=1)]
    yield "hollow_k0", x, W.leaf_ids(x, (0, 0, 0), 1.0), 0.0
    ids = np.array([[0, 0, 0], [lim - 1, lim - 1, lim - 1], [1, 1, 1], [lim - 2, lim - 1, lim - 1],
                    [0, 0, 1], [lim - 1, 0, 0], [0, 0, 0]], np.int32)
    x = ids.astype(np.float64) * 1e-3 + 1e-4
    yield "extreme_ids", x, ids, 1.0
    x = rng.random((300, 3)) * 0.01
    yield "one_box", x, np.tile(np.array([[7, 8, 9]], np.int32), (300, 1)), 30.0
    yield "single", np.array([[0.25, 0.5, 0.75]]), np.zeros((1, 3), np.int32), 2.0
