"""FP64 oracle of deep (multi-fragment) partial frames and their compositing.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper section 5.1.1 (Compositing) allows a rank to emit possibly multiple RGBA-z
fragments per pixel; section 2.1 explains why one fragment per pixel is only
enough when each rank's data is convex.  Paper Fig. 6 deals interleaved boxes to
ranks, which makes every rank's data non-convex.

Reading (deep frames):
* A rank's world is a set of disjoint convex bricks.  Its deep frame holds, per
  pixel, one fragment for every brick the pixel's ray hits (the brick's partial
  fragment of the single-fragment path), sorted front to back by (depth, fragment
  id).  The fragment id is intrinsic: rank * 65536 + the brick's index in the
  rank's world.
* Layer i of a pixel holds its i-th fragment; layers past the pixel's count are
  empty (RGBA 0, depth +inf, id -1).
* Compositing merges every rank's fragments per pixel by (depth, fragment id) and
  applies the same front-to-back "over" as the single-fragment compositor (C12):
  C_rgba += T rgba_i, T *= 1 - alpha_i; depth = the nearest fragment's depth.
Because every brick is convex and the bricks are disjoint, this equals compositing
every brick's fragment, which is the unsplit image (the split invariant), for any
dealing of bricks to ranks.
"""

from __future__ import annotations

import numpy as np

FID_RANK = 65536  # fragment id = rank * FID_RANK + brick index


def deep_frame(rgba, depth, fids, capacity=None):
    """Pack one rank's per-brick fragments into a deep frame.

    rgba: (B, P, 4), depth: (B, P) -- fragment of brick b at pixel p (+inf when the
    ray misses the brick); fids: (B,) intrinsic fragment ids.  Returns
    (count (P,), rgba (L, P, 4), depth (L, P), fid (L, P)) with L = capacity (at
    least B, default B).
    """
    rgba = np.asarray(rgba, dtype=np.float64)
    depth = np.asarray(depth, dtype=np.float64)
    B, P = depth.shape
    L = B if capacity is None else int(capacity)
    assert L >= B
    fids = np.asarray(fids, dtype=np.int64)
    count = np.isfinite(depth).sum(axis=0)
    out_rgba = np.zeros((L, P, 4))
    out_depth = np.full((L, P), np.inf)
    out_fid = np.full((L, P), -1, dtype=np.int64)
    for p in range(P):
        live = [b for b in range(B) if np.isfinite(depth[b, p])]
        live.sort(key=lambda b: (depth[b, p], fids[b]))
        for i, b in enumerate(live):
            out_rgba[i, p] = rgba[b, p]
            out_depth[i, p] = depth[b, p]
            out_fid[i, p] = fids[b]
    return count, out_rgba, out_depth, out_fid


def composite_deep(parts):
    """Composite deep frames (a list of (count, rgba, depth, fid)) per pixel.

    Returns (rgba (P, 4), depth (P,)) in FP64.
    """
    P = parts[0][0].shape[0]
    out = np.zeros((P, 4))
    zmin = np.full(P, np.inf)
    for p in range(P):
        frags = []
        for count, rgba, depth, fid in parts:
            for i in range(int(count[p])):
                frags.append((float(depth[i, p]), int(fid[i, p]), rgba[i, p]))
        frags.sort(key=lambda f: (f[0], f[1]))
        C = np.zeros(4)
        T = 1.0
        for _, _, f in frags:
            C += T * f
            T *= 1.0 - f[3]
        out[p] = C
        if frags:
            zmin[p] = frags[0][0]
    return out, zmin
