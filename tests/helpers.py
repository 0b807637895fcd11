"""Small shared fixtures for tests (inputs only; no method arithmetic)."""

import math

import numpy as np

from synth import Camera, make_blobs, make_tf, make_volume_small


def axis_camera(dims, axis=0, sign=-1.0, dist=2.5, size=9, fovy=30.0):
    """Camera on a box axis through the box centre; the centre pixel (odd size) looks along -axis*sign."""
    nx, ny, nz = dims
    h = 1.0 / max(dims)
    c = np.array([nx * h, ny * h, nz * h]) / 2
    e = c.copy()
    e[axis] -= sign * dist
    up = (0.0, 0.0, 1.0) if axis != 2 else (0.0, 1.0, 0.0)
    return Camera(tuple(e), tuple(c), up, fovy, size, size)


def diag_camera(dims, dist=2.5, size=9, fovy=30.0):
    h = 1.0 / max(dims)
    c = np.array(dims, dtype=float) * h / 2
    d = np.ones(3) / math.sqrt(3.0)
    return Camera(tuple(c + dist * d), tuple(c), (0.0, 0.0, 1.0), fovy, size, size)


def random_volume(dims, seed, nb=4, noise=0.02, dtype=np.float32):
    b = make_blobs(dims, seed, nb, (0.15, 0.4))
    return make_volume_small(dims, b, seed + 7, noise, dtype)


def constant_tf(rgb, a, n=256):
    tf = np.empty((n, 4), dtype=np.float32)
    tf[:, :3] = rgb
    tf[:, 3] = a
    return tf


def linear_alpha_tf(rgb=(0.3, 0.6, 0.9), n=256):
    tf = np.empty((n, 4), dtype=np.float64)
    tf[:, :3] = rgb
    tf[:, 3] = np.arange(n) / (n - 1)
    return tf


def rand_tf(seed, n=256):
    return make_tf(seed, n)
