"""Writes the stored values under tests/golden/ from the seeded generators and the oracle only.

    python tests/golden/make_golden.py

inputs_sha256.json: SHA-256 of the arrays the small workloads produce (draw order and
dtypes of the generators are part of the recipe).
"""
import hashlib
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def small_instances():
    yield W.plain_f64_cube()
    yield W.sphere(20000, 32, 2 * math.pi * 8, seed=0, name="sphere20k_D32")
    yield W.ellipsoid(20000, 16, seed=0, name="ellipsoid20k_D16")
    yield W.cube(5000, 5, 2 * math.pi * 2, seed=0, dtype=np.complex64, name="cube5000_g5_c64")


def main():
    out = {}
    for inst in small_instances():
        out[inst.name] = dict(sha256=digest(inst.xyz, inst.ids, inst.q), n=inst.n, h=inst.h, k=inst.k,
                              d_mean=inst.d_mean)
    with open(os.path.join(HERE, "inputs_sha256.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
