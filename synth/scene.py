"""Cameras, transfer-function tables and brick partitions (inputs only)."""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Camera:
    """Pinhole camera: eye, look-at centre, up vector, vertical FOV in degrees, image size."""
    eye: tuple
    center: tuple
    up: tuple
    fovy_deg: float
    width: int
    height: int


@dataclass
class Brick:
    """One rank's share of the world: owned global cells [lo, hi) plus stored ghost layers.

    The stored array covers global voxels [lo - ghost_lo, hi + ghost_hi) per axis
    (x, y, z order in the tuples; the array itself is (z, y, x)).
    """
    lo: tuple
    hi: tuple
    ghost_lo: tuple = (0, 0, 0)
    ghost_hi: tuple = (0, 0, 0)
    data: np.ndarray | None = field(default=None, repr=False)

    @property
    def stored_lo(self):
        return tuple(l - g for l, g in zip(self.lo, self.ghost_lo))

    @property
    def stored_hi(self):
        return tuple(h + g for h, g in zip(self.hi, self.ghost_hi))

    @property
    def stored_dims(self):
        return tuple(b - a for a, b in zip(self.stored_lo, self.stored_hi))


def make_tf(seed, n_entries=256, n_ctrl=6):
    """Piecewise-linear RGBA table from ``n_ctrl`` seeded control points.

    x0 = 0, x1 ~ U[0.05, 0.25], x2..x4 sorted U[x1, 1], x5 = 1.  Opacity is 0 at
    x0 and x1 (a transparent floor, so empty space exists) and U[0.2, 1] at the
    rest; RGB ~ U[0, 1]^3 per control point.  Entry i sits at value i/(N-1).
    Returns float32 (N, 4).
    """
    rng = np.random.default_rng(seed)
    x1 = 0.05 + 0.2 * rng.random()
    mids = np.sort(x1 + (1.0 - x1) * rng.random(n_ctrl - 3))
    xs = np.concatenate([[0.0, x1], mids, [1.0]])
    alpha = np.concatenate([[0.0, 0.0], 0.2 + 0.8 * rng.random(n_ctrl - 2)])
    rgb = rng.random((n_ctrl, 3))
    e = np.arange(n_entries) / (n_entries - 1)
    tf = np.empty((n_entries, 4))
    for c in range(3):
        tf[:, c] = np.interp(e, xs, rgb[:, c])
    tf[:, 3] = np.interp(e, xs, alpha)
    return tf.astype(np.float32)


def world_box(dims):
    nx, ny, nz = (int(v) for v in dims)
    h = 1.0 / max(nx, ny, nz)
    return np.array([nx * h, ny * h, nz * h])


def orbit_camera(dims, width, height, az_deg=30.0, el_deg=20.0, dist=2.5, fovy=60.0):
    ext = world_box(dims)
    c = ext / 2
    lmax = ext.max()
    az, el = math.radians(az_deg), math.radians(el_deg)
    d = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    eye = c + dist * lmax * d
    return Camera(tuple(eye), tuple(c), (0.0, 0.0, 1.0), fovy, width, height)


def fibonacci_cameras(dims, n, width, height, dist=2.5, fovy=60.0):
    """``n`` cameras on a Fibonacci sphere around the box centre, looking at it."""
    ext = world_box(dims)
    c = ext / 2
    lmax = ext.max()
    cams = []
    for i in range(n):
        z = 1.0 - (2 * i + 1) / n
        phi = i * math.pi * (3.0 - math.sqrt(5.0))
        r = math.sqrt(max(0.0, 1.0 - z * z))
        d = np.array([r * math.cos(phi), r * math.sin(phi), z])
        up = (0.0, 1.0, 0.0) if abs(z) > 0.99 else (0.0, 0.0, 1.0)
        cams.append(Camera(tuple(c + dist * lmax * d), tuple(c), up, fovy, width, height))
    return cams


def even_split(dims, parts):
    """Split the cell box into parts[0] x parts[1] x parts[2] equal bricks (x, y, z)."""
    cuts = [np.linspace(0, n, p + 1).round().astype(int) for n, p in zip(dims, parts)]
    out = []
    for k in range(parts[2]):
        for j in range(parts[1]):
            for i in range(parts[0]):
                lo = (int(cuts[0][i]), int(cuts[1][j]), int(cuts[2][k]))
                hi = (int(cuts[0][i + 1]), int(cuts[1][j + 1]), int(cuts[2][k + 1]))
                out.append((lo, hi))
    return out


def _kd(lo, hi, n, rng, out):
    if n == 1:
        out.append((tuple(lo), tuple(hi)))
        return
    nl = n // 2
    ext = [b - a for a, b in zip(lo, hi)]
    ax = int(np.argmax(ext))
    frac = min(0.85, max(0.15, nl / n * (0.6 + 0.8 * rng.random())))
    cut = int(round(lo[ax] + frac * ext[ax]))
    cut = min(max(cut, lo[ax] + 2), hi[ax] - 2)
    l_hi = list(hi)
    l_hi[ax] = cut
    r_lo = list(lo)
    r_lo[ax] = cut
    _kd(lo, l_hi, nl, rng, out)
    _kd(r_lo, hi, n - nl, rng, out)


def kd_split(dims, n, seed, max_ratio=4.0, max_tries=1000):
    """Seeded k-d partition of the cell box into ``n`` uneven bricks.

    Recursive: split ``n`` leaves into floor(n/2) and the rest on the longest
    axis at the integer plane nearest lo + clamp(n_l/n * U[0.6, 1.4], .15, .85) * extent.
    Redraw (seed + 1, ...) until max/min brick volume <= ``max_ratio``.
    """
    for t in range(max_tries):
        rng = np.random.default_rng(seed + t)
        out = []
        _kd([0, 0, 0], [int(d) for d in dims], n, rng, out)
        vols = [np.prod([b - a for a, b in zip(lo, hi)]) for lo, hi in out]
        if max(vols) / min(vols) <= max_ratio:
            return out
    raise RuntimeError("k-d split: no draw met the volume-ratio bound")


def brick_ghosts(dims, lo, hi, width=1):
    """Ghost layers: ``width`` on faces interior to the domain, 0 on global faces."""
    glo = tuple(width if l > 0 else 0 for l in lo)
    ghi = tuple(width if h < n else 0 for h, n in zip(hi, dims))
    return glo, ghi


def extract_brick(volume, dims, lo, hi, ghost=1):
    """Copy a brick's stored region (owned cells + ghost layers) out of a global volume."""
    glo, ghi = brick_ghosts(dims, lo, hi, ghost)
    b = Brick(tuple(lo), tuple(hi), glo, ghi)
    (x0, y0, z0), (x1, y1, z1) = b.stored_lo, b.stored_hi
    b.data = np.ascontiguousarray(volume[z0:z1, y0:y1, x0:x1])
    return b


def pixel_subset(width, height, stride=8, tiles=4, tile=64, seed=0):
    """Seeded sample of pixel coordinates: every ``stride``-th pixel plus full tiles.

    Returns (px, py) int arrays without duplicates.
    """
    ys, xs = np.mgrid[0:height:stride, 0:width:stride]
    px, py = [xs.ravel()], [ys.ravel()]
    rng = np.random.default_rng(seed)
    for _ in range(tiles):
        tx = int(rng.integers(0, max(1, width - tile + 1)))
        ty = int(rng.integers(0, max(1, height - tile + 1)))
        yy, xx = np.mgrid[ty:min(height, ty + tile), tx:min(width, tx + tile)]
        px.append(xx.ravel())
        py.append(yy.ravel())
    lin = np.unique(np.concatenate(py) * width + np.concatenate(px))
    return (lin % width).astype(np.int64), (lin // width).astype(np.int64)
