"""Seeded synthetic partial frames standing in for remote ranks (inputs only).

Each synthetic rank r covers one screen rectangle (coverage fraction ~ U[0.2, 0.8],
aspect ~ U[0.5, 2], seeded position, clipped), like the projection of a convex
brick.  Inside it the premultiplied colour is alpha * colour_r with per-pixel
alpha = 0.05 + 0.55 * u and depth uniform inside the rank's depth slab; outside
it the fragment is empty: (0, 0, 0, 0) at depth +inf.  Depth slabs: the front
half partitions [0.1, t_min - 0.01], the back half [t_max + 0.01, t_max + 10],
assigned to ranks by a seeded permutation, so the local frame (depths in
[t_min, t_max]) lands in the middle of the sort.
"""

from __future__ import annotations

import numpy as np


def frame_params(n, width, height, t_min, t_max, seed):
    rng = np.random.default_rng(seed)
    n_front = n // 2
    n_back = n - n_front
    front = np.linspace(0.1, t_min - 0.01, n_front + 1)
    back = np.linspace(t_max + 0.01, t_max + 10.0, n_back + 1)
    slabs = [(front[i], front[i + 1]) for i in range(n_front)] + \
            [(back[i], back[i + 1]) for i in range(n_back)]
    perm = rng.permutation(n)
    out = []
    for r in range(n):
        p = 0.2 + 0.6 * rng.random()
        asp = 0.5 + 1.5 * rng.random()
        area = p * width * height
        rw = int(round(min(width, np.sqrt(area * asp))))
        rh = int(round(min(height, area / max(rw, 1))))
        x0 = int(rng.integers(0, max(1, width - rw + 1)))
        y0 = int(rng.integers(0, max(1, height - rh + 1)))
        col = rng.random(3)
        z0, z1 = slabs[perm[r]]
        out.append(dict(rect=(x0, y0, min(width, x0 + rw), min(height, y0 + rh)),
                        color=col, slab=(float(z0), float(z1)), seed=int(rng.integers(1 << 62))))
    return out


def synthetic_frames(n, width, height, t_min, t_max, seed, device="cpu", rgba_out=None, depth_out=None):
    """Fill ``n`` synthetic frames (torch tensors (n, H, W, 4) and (n, H, W), float32).

    ``rgba_out``/``depth_out`` may be views into larger preallocated buffers.
    Returns (rgba, depth, params).
    """
    import torch

    params = frame_params(n, width, height, t_min, t_max, seed)
    if rgba_out is None:
        rgba_out = torch.empty((n, height, width, 4), dtype=torch.float32, device=device)
    if depth_out is None:
        depth_out = torch.empty((n, height, width), dtype=torch.float32, device=device)
    for r, prm in enumerate(params):
        x0, y0, x1, y1 = prm["rect"]
        g = torch.Generator(device="cpu").manual_seed(prm["seed"] & 0x7FFFFFFFFFFFFFFF)
        hh, ww = y1 - y0, x1 - x0
        u = torch.rand((2, hh, ww), generator=g, dtype=torch.float32).to(device)
        alpha = 0.05 + 0.55 * u[0]
        z0, z1 = prm["slab"]
        rgba_out[r].zero_()
        depth_out[r].fill_(float("inf"))
        col = torch.tensor(prm["color"], dtype=torch.float32, device=device)
        rgba_out[r, y0:y1, x0:x1, :3] = alpha[..., None] * col
        rgba_out[r, y0:y1, x0:x1, 3] = alpha
        depth_out[r, y0:y1, x0:x1] = z0 + (z1 - z0) * u[1]
    return rgba_out, depth_out, params
