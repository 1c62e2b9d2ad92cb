"""Compact storage of fields with the symmetries of the separable workload.

The 256^3 separable run (uniform D, no-flux box, blob at the box centre) is
mapped onto itself by the 48 symmetries of the cube: the mirror i -> n-1-i on
each axis and every permutation of the axes.  Its field is therefore fixed by
the values on the fundamental domain 0 <= a <= b <= c < n/2, which is
C(n/2 + 2, 3) voxels (357,760 at n = 256) instead of n^3.

Pure indexing: no arithmetic of the method lives here.
"""

from __future__ import annotations

import numpy as np


def _domain(n):
    h = n // 2
    a, b, c = np.meshgrid(np.arange(h), np.arange(h), np.arange(h), indexing="ij")
    keep = (a <= b) & (b <= c)
    return a[keep], b[keep], c[keep]


def pack_cube(u):
    """Values of a cube-symmetric field (n even) on the fundamental domain."""
    n = u.shape[0]
    if u.shape != (n, n, n) or n % 2:
        raise ValueError("pack_cube needs an (n, n, n) field with n even")
    a, b, c = _domain(n)
    return np.ascontiguousarray(u[a, b, c])


def unpack_cube(vals, n, dtype=np.float64):
    """The full (n, n, n) field from its fundamental-domain values."""
    h = n // 2
    a, b, c = _domain(n)
    if vals.shape != a.shape:
        raise ValueError("value count does not match the fundamental domain of n")
    table = np.empty((h, h, h), dtype=dtype)
    table[a, b, c] = vals
    fold = np.minimum(np.arange(n), n - 1 - np.arange(n)).astype(np.int16)
    out = np.empty((n, n, n), dtype=dtype)
    for i in range(n):  # plane by plane, to keep the sort buffers small
        t = np.stack(np.broadcast_arrays(np.full((n, n), fold[i], np.int16), fold[:, None], fold[None, :]))
        t.sort(axis=0)
        out[i] = table[t[0], t[1], t[2]]
    return out
