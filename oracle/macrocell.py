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
  [floor(x_min) - 1, ceil(x_max) + 1] intersected with [0, N-1], where x is the
  table coordinate of the range ends.  A majorant of 0 means every opacity the
  sample could produce is exactly 0, so the segment is an exact no-op.

The entry range is an integer decided from floating point, so it is taken in
FP32 with the same operation order the GPU kernel uses:
u = (v - lo) / (hi - lo) (IEEE division), clamp to [0, 1], x = u * (N - 1).
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


def _tf_coord32(v, lo, hi, n):
    v = np.asarray(v, dtype=np.float32)
    u = (v - np.float32(lo)) / (np.float32(hi) - np.float32(lo))
    u = np.minimum(np.maximum(u, np.float32(0.0)), np.float32(1.0))
    return u * np.float32(n - 1)


def majorants(ranges, tf, lo=0.0, hi=1.0):
    """Majorant opacity per macrocell from (…, 2) ranges -> float32 (…)."""
    tf = np.asarray(tf, dtype=np.float32)
    n = tf.shape[0]
    xmin = _tf_coord32(ranges[..., 0], lo, hi, n)
    xmax = _tf_coord32(ranges[..., 1], lo, hi, n)
    e0 = np.maximum(np.floor(xmin).astype(np.int64) - 1, 0)
    e1 = np.minimum(np.ceil(xmax).astype(np.int64) + 1, n - 1)
    out = np.empty(ranges.shape[:-1], dtype=np.float32)
    flat0, flat1, fo = e0.ravel(), e1.ravel(), out.reshape(-1)
    for i in range(fo.size):
        fo[i] = tf[flat0[i]:flat1[i] + 1, 3].max()
    return out
