"""Oracle of macrocell value ranges and transfer-function majorants (empty-space skipping).

Empty-space skipping is an optimisation of the local render, not part of the
paper; skipping must not change any result.  Reading (C13):

* A brick's owned cells are tiled by macrocells of ``mc`` cells per axis,
  starting at the owned lower corner; the last macrocell may be partial.
* The value range of macrocell m (per axis) is min/max over stored voxels
  [mc*m - 1, mc*m + mc] (owned-relative voxel indices), clipped to the stored
  range.  Every trilinear corner of a sample whose point lies in the macrocell
  (or, for the outermost macrocells, up to half a voxel outside the owned box)
  falls in that window, so the 8-corner interpolant lies inside [min, max].
* The majorant is the largest transfer-function opacity over table entries
  [floor(x_min) - 1, ceil(x_max) + 1] intersected with [0, N-1], where
  x = clamp((v - lo) / (hi - lo), 0, 1) (N - 1) is the table coordinate of a
  range end.  A majorant of 0 means every opacity the sample could produce is
  exactly 0, so the segment is an exact no-op.

Both are written here from their plain definitions: the range is an exact
min/max of stored values, and the table coordinates are taken in FP64.  A
kernel that decides the entry range in FP32 may differ from this only in a
macrocell whose x_min or x_max lies within FP32 rounding of an integer
(``entry_decision_ambiguous``); there both choices are valid majorants.
"""

from __future__ import annotations

import numpy as np


def macrocell_grid(owned_lo, owned_hi, mc):
    return tuple(-(-(h - l) // mc) for l, h in zip(owned_lo, owned_hi))


def macrocell_ranges(data, owned_lo, owned_hi, ghost_lo, mc=16):
    """min/max per macrocell -> (Mz, My, Mx, 2) float32 (exact: F16/F32 values)."""
    Mx, My, Mz = macrocell_grid(owned_lo, owned_hi, mc)
    sz = (data.shape[2], data.shape[1], data.shape[0])
    out = np.empty((Mz, My, Mx, 2), dtype=np.float32)

    def win(m, a):
        a0 = max(0, mc * m - 1 + ghost_lo[a])
        a1 = min(sz[a] - 1, mc * m + mc + ghost_lo[a])
        return a0, a1 + 1

    for mz in range(Mz):
        z0, z1 = win(mz, 2)
        for my in range(My):
            y0, y1 = win(my, 1)
            for mx in range(Mx):
                x0, x1 = win(mx, 0)
                blk = data[z0:z1, y0:y1, x0:x1]
                out[mz, my, mx, 0] = np.min(blk)
                out[mz, my, mx, 1] = np.max(blk)
    return out


def tf_coord(v, lo, hi, n):
    """Table coordinate x = clamp((v - lo) / (hi - lo), 0, 1) (N - 1), FP64 (C7)."""
    u = (np.asarray(v, dtype=np.float64) - float(lo)) / (float(hi) - float(lo))
    return np.clip(u, 0.0, 1.0) * (n - 1)


def _entries(xmin, xmax, n):
    e0 = np.maximum(np.floor(xmin).astype(np.int64) - 1, 0)
    e1 = np.minimum(np.ceil(xmax).astype(np.int64) + 1, n - 1)
    return e0, e1


def entry_range(ranges, n, lo=0.0, hi=1.0):
    """First and last table entry a majorant covers, [floor(x_min) - 1, ceil(x_max) + 1]
    clipped to [0, N - 1], from (..., 2) ranges -> two int64 arrays (...)."""
    return _entries(tf_coord(ranges[..., 0], lo, hi, n), tf_coord(ranges[..., 1], lo, hi, n), n)


def majorants(ranges, tf, lo=0.0, hi=1.0):
    """Majorant opacity per macrocell from (..., 2) ranges -> float32 (...)."""
    tf = np.asarray(tf, dtype=np.float32)
    n = tf.shape[0]
    e0, e1 = entry_range(ranges, n, lo, hi)
    out = np.empty(ranges.shape[:-1], dtype=np.float32)
    flat0, flat1, fo = e0.ravel(), e1.ravel(), out.reshape(-1)
    for i in range(fo.size):
        fo[i] = tf[flat0[i]:flat1[i] + 1, 3].max()
    return out


def entry_decision_ambiguous(ranges, n, lo=0.0, hi=1.0, eps=1e-4):
    """True where moving a range end's table coordinate by +-``eps`` entries changes
    the entry range, so that a decision taken in FP32 may pick the neighbouring
    entry.  An end outside (lo, hi) is clamped to x = 0 or N - 1 exactly in any
    precision, so it does not move."""
    xs = []
    for k in (0, 1):
        v = np.asarray(ranges[..., k], dtype=np.float64)
        x = tf_coord(v, lo, hi, n)
        free = (v > lo) & (v < hi)
        xs.append((np.where(free, x - eps, x), np.where(free, x + eps, x)))
    a0, a1 = _entries(xs[0][0], xs[1][0], n)
    b0, b1 = _entries(xs[0][1], xs[1][1], n)
    return (a0 != b0) | (a1 != b1)
