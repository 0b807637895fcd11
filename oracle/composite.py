"""FP64 oracle of sort-last, depth-ordered compositing of RGBA-z fragments.

Paper section 2.1 (Data Parallel Rendering): each rank reduces its rendering to
one fragment (colour, opacity, depth) per pixel and the fragments are merged at
the end.  Paper section 5.1.1 (Compositing): because every fragment carries a
depth, the compositor sorts each pixel's fragments and composites them front to
back, so no fixed compositing order across ranks is needed.

Reading (C12): per pixel, take the fragments with finite depth (an empty
fragment has depth +inf and RGBA 0); sort ascending by (depth, fragment id),
where the id is intrinsic to the fragment (its rank / brick), not its position
in the input list; then T = 1, C = 0 and for each fragment the premultiplied
"over" acts on all four channels alike: C_rgba += T*rgba_i, T *= (1 - alpha_i).
The output alpha sum_i T_i alpha_i equals 1 - prod_i (1 - alpha_i) in exact
arithmetic; accumulating it like the colour makes one fragment composite to
itself bit for bit in any precision.  Depth = min depth (+inf when no fragment
is present).
"""

from __future__ import annotations

import numpy as np


def composite(rgba, depth, ids=None):
    """Composite K fragments per pixel.

    rgba: (K, ..., 4), depth: (K, ...), ids: (K,) intrinsic fragment ids
    (default 0..K-1).  Returns (rgba (..., 4), depth (...)) in FP64.
    """
    rgba = np.asarray(rgba, dtype=np.float64)
    depth = np.asarray(depth, dtype=np.float64)
    K = depth.shape[0]
    pix_shape = depth.shape[1:]
    rgba = rgba.reshape(K, -1, 4)
    depth = depth.reshape(K, -1)
    P = depth.shape[1]
    ids = np.arange(K) if ids is None else np.asarray(ids)
    idk = np.broadcast_to(ids[:, None], (K, P))
    order = np.lexsort((idk, depth), axis=0)  # primary key depth, then id
    C = np.zeros((P, 4))
    T = np.ones(P)
    cols = np.arange(P)
    for r in range(K):
        k = order[r]
        z = depth[k, cols]
        f = rgba[k, cols]
        present = np.isfinite(z)
        C += np.where(present[:, None], T[:, None] * f, 0.0)
        T = np.where(present, T * (1.0 - f[:, 3]), T)
    out = C
    zmin = np.min(depth, axis=0) if K else np.full(P, np.inf)
    return out.reshape(pix_shape + (4,)), zmin.reshape(pix_shape)
