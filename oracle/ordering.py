"""Fill-reducing orderings for the oracle (test infrastructure only).

The paper requires a reordering phase that reduces fill and gathers the
factor's nonzeros bottom-right (Section 1, Section 2.1, Fig. 2) but names no
algorithm.  The reading used here is a geometric nested dissection of the
structured grid with a fixed, deterministic rule:

* a box is a half-open range along each of the three axes;
* a box whose volume is at most 8, or whose extents are all at most 2, is a
  leaf and its points are listed in increasing grid index x + nx*(y + ny*z);
* otherwise the longest axis is cut (ties go to the lowest axis) at
  m = lo + (hi - lo) // 2: the plane at m is the separator, [lo, m) the first
  part and [m+1, hi) the second part; the order is first part, second part,
  separator (the separator listed in increasing grid index).

A permutation ``perm`` maps new position -> original index: the permuted
matrix is A[perm][:, perm].
"""
from __future__ import annotations

import numpy as np


def natural(n):
    return np.arange(n, dtype=np.int32)


def nd_grid(dims):
    """Geometric nested dissection of an nx x ny x nz grid (nz = 1 for 2D)."""
    dims = tuple(int(v) for v in dims) + (1,) * (3 - len(dims))
    nx, ny, nz = dims
    out = []

    def box_points(lo, hi):
        zs = np.arange(lo[2], hi[2], dtype=np.int64)
        ys = np.arange(lo[1], hi[1], dtype=np.int64)
        xs = np.arange(lo[0], hi[0], dtype=np.int64)
        # z slowest, x fastest == increasing grid index
        pts = xs[None, None, :] + nx * (ys[None, :, None] + ny * zs[:, None, None])
        return pts.reshape(-1)

    def rec(lo, hi):
        ext = [hi[d] - lo[d] for d in range(3)]
        if min(ext) <= 0:
            return
        vol = ext[0] * ext[1] * ext[2]
        if vol <= 8 or max(ext) <= 2:
            out.append(box_points(lo, hi))
            return
        d = int(np.argmax(ext))  # argmax returns the lowest axis on ties
        m = lo[d] + (hi[d] - lo[d]) // 2
        hi1 = list(hi); hi1[d] = m
        lo2 = list(lo); lo2[d] = m + 1
        los = list(lo); los[d] = m
        his = list(hi); his[d] = m + 1
        rec(lo, hi1)
        rec(lo2, hi)
        out.append(box_points(los, his))

    rec([0, 0, 0], [nx, ny, nz])
    perm = np.concatenate(out) if out else np.zeros(0, dtype=np.int64)
    return perm.astype(np.int32)


def is_permutation(perm, n):
    perm = np.asarray(perm)
    if perm.shape != (n,):
        return False
    seen = np.zeros(n, dtype=bool)
    if n and (perm.min() < 0 or perm.max() >= n):
        return False
    seen[perm] = True
    return bool(seen.all())


def inverse(perm):
    perm = np.asarray(perm, dtype=np.int64)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.shape[0], dtype=np.int64)
    return inv.astype(np.int32)
