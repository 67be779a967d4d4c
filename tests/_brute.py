"""Dense all-pairs evaluation of the near-field sum, for small inputs only.

A pin for the oracle, built differently from it: no Morton keys, no sort, no box
table, no neighbour lists.  The near relation is read straight off the ids of
every pair of points (paper, sections 3.2-3.3: a target sees the sources of its
own and the adjacent boxes; here in 3-D, 27 boxes), and the sum is one dense
matrix product.
"""
import numpy as np


def near_mask(ids):
    ids = np.asarray(ids, dtype=np.int64)
    diff = np.abs(ids[:, None, :] - ids[None, :, :]).max(axis=2)
    return diff <= 1


def dense_matrix(xyz, ids, k):
    d = xyz[:, None, :] - xyz[None, :, :]
    nonzero = np.any(d != 0.0, axis=2)
    mask = near_mask(ids) & nonzero
    r = np.sqrt((d * d).sum(axis=2))
    r_safe = np.where(mask, r, 1.0)
    g = np.exp(1j * k * r_safe) / (4.0 * np.pi * r_safe)
    return np.where(mask, g, 0.0), mask


def dense_apply(xyz, ids, k, q):
    a, _ = dense_matrix(xyz, ids, k)
    q = np.asarray(q, dtype=np.complex128)
    if q.ndim == 1:
        q = q[:, None]
    return a @ q


def dense_pair_count(xyz, ids):
    _, mask = dense_matrix(xyz, ids, 0.0)
    return int(mask.sum())
