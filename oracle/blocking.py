"""Diagonal block feature and irregular blocking for the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``diag_block_ptr``   -- Algorithm 2 (Section 4.2): blockptr[i] is the number
  of entries of the filled symmetric pattern inside the leading i x i
  submatrix.  It counts, per column, the entries below the diagonal at the
  row where they sit; then blockptr[i+1] = blockptr[i] + 2*num[i] + 1 (the
  row's lower entries, their mirror images and the diagonal).
* ``irregular_blocking`` -- the 1000-point sampling of the feature curve
  (blockptr over its last entry) and Algorithm 3 (Section 4.3).
* ``regular_blocking`` -- fixed-size 2D blocking (Section 3.2).

Readings where the text is incomplete (each is listed in the design notes):

R1  the loop of Algorithm 3 advances i by ``advance`` (1 = the literal
    pseudo-code, the default; ``step`` is the alternative the prose allows);
R2  the loop runs while i + step <= Sp (the printed bound would read past the
    sample array); k and l start at 0; N is appended as the last boundary when
    the loop did not end on it;
R3  Sp = min(1000, N) intervals; sample s sits at row pos(s) = floor(s*N/Sp),
    s = 0..Sp, so samples are distinct rows even for N < 1000;
R4  the threshold is step over the number of sample intervals (the printed
    name of that count is garbled) and the comparison is "greater or equal",
    evaluated exactly in integers:
        (blockptr[pos(i+step)] - blockptr[pos(i)]) * Sp >= step * blockptr[N]
    which is pct[i+step] - pct[i] >= step/Sp multiplied through by
    Sp*blockptr[N] > 0;
R5  fine blocks go to dense regions, as Algorithm 3 does (one sentence of
    Section 1 states the opposite; the abstract, Section 4 and the conclusion
    agree with the algorithm).
"""
from __future__ import annotations

import numpy as np


def diag_block_ptr(n, colptr, rowidx):
    """Algorithm 2: diagonal block pointer from a CSC pattern of S.

    Works on the lower-CSC form (diagonal included) or the full symmetric CSC;
    only entries strictly below the diagonal are counted.
    """
    colptr = np.asarray(colptr, dtype=np.int64)
    rowidx = np.asarray(rowidx, dtype=np.int64)
    col_of = np.repeat(np.arange(n, dtype=np.int64), np.diff(colptr))
    below = rowidx > col_of
    num = np.bincount(rowidx[below], minlength=n).astype(np.int64)
    blockptr = np.zeros(n + 1, dtype=np.int64)
    blockptr[1:] = np.cumsum(2 * num + 1)
    return blockptr


def sample_rows(N, sample_points=1000):
    """Rows of the Sp+1 uniform samples (reading R3)."""
    sp = min(int(sample_points), int(N))
    s = np.arange(sp + 1, dtype=np.int64)
    return (s * np.int64(N)) // np.int64(sp), sp


def irregular_blocking(blockptr, sample_points=1000, step=2, max_num=3, advance=1):
    """Structure-aware blocking (Section 4.3, Algorithm 3); returns ptr (int64).

    The feature curve is read at the Sp + 1 sample rows.  Every window of
    ``step`` sample intervals, its start moving by ``advance`` samples, is
    tested once, in order: it is dense when its increment of the curve is at
    least step/Sp of the total.  The window's end row becomes a boundary when
    the window is dense, or when the ``max_num`` windows before it passed
    without a boundary; N closes the last block.
    """
    blockptr = np.asarray(blockptr, dtype=np.int64)
    N = blockptr.shape[0] - 1
    if N == 0:
        return np.zeros(1, dtype=np.int64)
    rows, sp = sample_rows(N, sample_points)
    total = int(blockptr[N])
    starts = np.arange(0, sp - step + 1, advance, dtype=np.int64)
    ends = rows[starts + step]
    increment = blockptr[ends] - blockptr[rows[starts]]
    # increment / total >= step / Sp, multiplied through by Sp * total > 0
    dense = increment * sp >= step * total
    ptr = [0]
    passed = 0
    for end, is_dense in zip(ends.tolist(), dense.tolist()):
        if is_dense or passed >= max_num:
            ptr.append(end)
            passed = 0
        else:
            passed += 1
    if ptr[-1] != N:
        ptr.append(N)
    return np.asarray(ptr, dtype=np.int64)


def regular_blocking(N, b):
    """Blocks of b rows; the last block takes the remainder."""
    pts = list(range(0, int(N), int(b)))
    pts.append(int(N))
    if len(pts) >= 2 and pts[-2] == pts[-1]:
        pts.pop()
    return np.asarray(pts, dtype=np.int64)


def block_of_rows(N, ptr):
    """Block id of every row for a boundary array ptr."""
    sizes = np.diff(np.asarray(ptr, dtype=np.int64))
    return np.repeat(np.arange(sizes.shape[0], dtype=np.int64), sizes)


def nonempty_blocks(n, colptr, rowidx, ptr):
    """Non-empty blocks of S (both triangles) and their entry counts.

    Returns (bi, bj, nnz) sorted by (bj, bi): block (bi, bj) holds rows
    [ptr[bi], ptr[bi+1]) and columns [ptr[bj], ptr[bj+1]).
    """
    bid = block_of_rows(n, ptr)
    p = int(np.asarray(ptr).shape[0] - 1)
    col_of = np.repeat(np.arange(n, dtype=np.int64), np.diff(colptr))
    r = np.asarray(rowidx, dtype=np.int64)
    br = bid[r]
    bc = bid[col_of]
    off = r != col_of
    # lower part at (br, bc); its mirror at (bc, br); the diagonal once
    keys = np.concatenate([br * p + bc, (bc * p + br)[off]])
    uk, cnt = np.unique(keys, return_counts=True)
    bi = uk // p
    bj = uk % p
    order = np.lexsort((bi, bj))
    return bi[order], bj[order], cnt[order]
