"""Scalar-volume generators (inputs only).

Layout convention shared by every consumer: a volume of global dims
``(nx, ny, nz)`` is a C-contiguous array of shape ``(nz, ny, nx)`` (x fastest).
Voxel ``(i, j, k)`` sits at the centre of cell ``[i, i+1) x [j, j+1) x [k, k+1)``;
with ``h = 1 / max(nx, ny, nz)`` its world position is ``((i+.5)h, (j+.5)h, (k+.5)h)``.

Field = clamp(sum of anisotropic Gaussian blobs + noise, 0, 1), where
blob(p) = a * exp(-1/2 * sum_axis ((p_axis - c_axis) / s_axis)^2).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class BlobSet:
    centers: np.ndarray  # (n, 3) world units, x/y/z
    sigmas: np.ndarray   # (n, 3) world units
    amps: np.ndarray     # (n,)


def make_blobs(dims, seed, n, s_range, a_range=(1.0, 1.0), log_uniform=False):
    """Draw ``n`` blobs with centres uniform in the world box (numpy default_rng)."""
    nx, ny, nz = (int(v) for v in dims)
    h = 1.0 / max(nx, ny, nz)
    ext = np.array([nx * h, ny * h, nz * h])
    rng = np.random.default_rng(seed)
    centers = rng.random((n, 3)) * ext
    if log_uniform:
        lo, hi = np.log(s_range[0]), np.log(s_range[1])
        sigmas = np.exp(lo + (hi - lo) * rng.random((n, 3)))
    else:
        sigmas = s_range[0] + (s_range[1] - s_range[0]) * rng.random((n, 3))
    amps = a_range[0] + (a_range[1] - a_range[0]) * rng.random(n)
    return BlobSet(centers, sigmas, amps)


def perturb_blobs(blobs: BlobSet, seed, dist=0.02):
    """Move every blob centre by ``dist`` along a seeded unit vector."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=blobs.centers.shape)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return BlobSet(blobs.centers + dist * v, blobs.sigmas.copy(), blobs.amps.copy())


def _axis_gauss(n, h, c, s):
    x = (np.arange(n, dtype=np.float64) + 0.5) * h
    return np.exp(-0.5 * ((x[None, :] - c[:, None]) / s[:, None]) ** 2)  # (nb, n)


def blobs_field(dims, blobs: BlobSet, z_range=None):
    """FP64 sum of blobs at voxel centres, shape (nz', ny, nx) for slices z_range."""
    nx, ny, nz = (int(v) for v in dims)
    h = 1.0 / max(nx, ny, nz)
    z0, z1 = (0, nz) if z_range is None else z_range
    gx = _axis_gauss(nx, h, blobs.centers[:, 0], blobs.sigmas[:, 0])
    gy = _axis_gauss(ny, h, blobs.centers[:, 1], blobs.sigmas[:, 1])
    gz = _axis_gauss(nz, h, blobs.centers[:, 2], blobs.sigmas[:, 2])[:, z0:z1]
    # separable: sum_b a_b gz[b,k] gy[b,j] gx[b,i]
    gzy = (blobs.amps[:, None, None] * gz[:, :, None] * gy[:, None, :]).reshape(len(blobs.amps), -1)
    return (gzy.T @ gx).reshape(z1 - z0, ny, nx)


def white_noise(dims, seed, amp):
    """Per-voxel uniform noise ``amp * (2u - 1)``; u from the counter-based Philox generator."""
    nx, ny, nz = (int(v) for v in dims)
    g = np.random.Generator(np.random.Philox(key=seed))
    u = g.random((nz, ny, nx))
    return amp * (2.0 * u - 1.0)


def _fbm_lattices(dims, seed, periods):
    nx, ny, nz = (int(v) for v in dims)
    lats = []
    for o, p in enumerate(periods):
        rng = np.random.default_rng([seed, o])
        shape = (nz // p + 2, ny // p + 2, nx // p + 2)
        lats.append(2.0 * rng.random(shape) - 1.0)
    return lats


def _octave_weights(periods, gain):
    w = np.array([gain ** o for o in range(len(periods))])
    return w / w.sum()


def _axis_interp(n, p):
    x = (np.arange(n, dtype=np.float64) + 0.5) / p
    m = np.floor(x).astype(np.int64)
    return m, x - m


def fbm_field(dims, seed, amp, periods, gain=0.5, z_range=None):
    """Value-noise fBm (numpy FP64): octaves of trilinearly interpolated lattice noise.

    Octave ``o`` has lattice period ``periods[o]`` voxels and weight ``gain**o``
    (weights normalised to sum 1, then scaled by ``amp``).  Halving the period
    while halving the amplitude gives the 1/f amplitude spectrum (power ~ 1/f^2)
    of turbulence-like fields.
    """
    nx, ny, nz = (int(v) for v in dims)
    z0, z1 = (0, nz) if z_range is None else z_range
    out = np.zeros((z1 - z0, ny, nx))
    for lat, w, p in zip(_fbm_lattices(dims, seed, periods), _octave_weights(periods, gain), periods):
        mx, fx = _axis_interp(nx, p)
        my, fy = _axis_interp(ny, p)
        mz, fz = _axis_interp(nz, p)
        mz, fz = mz[z0:z1], fz[z0:z1]
        a = lat[:, :, mx] * (1 - fx) + lat[:, :, mx + 1] * fx
        a = a[:, my, :] * (1 - fy)[None, :, None] + a[:, my + 1, :] * fy[None, :, None]
        a = a[mz] * (1 - fz)[:, None, None] + a[mz + 1] * fz[:, None, None]
        out += amp * w * a
    return out


def make_volume_small(dims, blobs: BlobSet, noise_seed, noise_amp=0.02, dtype=np.float32):
    """Blobs + white noise, clamped to [0, 1], rounded once to ``dtype`` (F32 or F16)."""
    v = blobs_field(dims, blobs)
    if noise_amp:
        v += white_noise(dims, noise_seed, noise_amp)
    return np.clip(v, 0.0, 1.0).astype(dtype)


def make_volume_large(dims, blobs: BlobSet, fbm_seed, fbm_amp, periods, gain=0.5,
                      device="cpu", dtype="float16", z_chunk=64):
    """Blobs + fBm for multi-GB volumes, evaluated with torch in FP32 on ``device``.

    Same recipe as the FP64 path; rounding differs, which is harmless because the
    oracle and the GPU path both read the bytes this returns.  Returns a torch
    tensor of shape (nz, ny, nx) on ``device``.
    """
    import torch

    nx, ny, nz = (int(v) for v in dims)
    h = 1.0 / max(nx, ny, nz)
    tdt = getattr(torch, dtype)
    out = torch.empty((nz, ny, nx), dtype=tdt, device=device)
    f32 = torch.float32

    def axis_g(n, c, s):
        x = (torch.arange(n, dtype=torch.float64) + 0.5) * h
        g = torch.exp(-0.5 * ((x[None, :] - torch.from_numpy(c)[:, None]) / torch.from_numpy(s)[:, None]) ** 2)
        return g.to(f32).to(device)

    gx = axis_g(nx, blobs.centers[:, 0], blobs.sigmas[:, 0])
    gy = axis_g(ny, blobs.centers[:, 1], blobs.sigmas[:, 1])
    gz = axis_g(nz, blobs.centers[:, 2], blobs.sigmas[:, 2])
    amps = torch.from_numpy(blobs.amps).to(f32).to(device)
    lats = [torch.from_numpy(l).to(f32).to(device) for l in _fbm_lattices(dims, fbm_seed, periods)]
    ws = _octave_weights(periods, gain)
    axes = []
    for p in periods:
        per = []
        for n in (nx, ny, nz):
            m, f = _axis_interp(n, p)
            per.append((torch.from_numpy(m).to(device), torch.from_numpy(f).to(f32).to(device)))
        axes.append(per)
    nb = len(blobs.amps)
    for z0 in range(0, nz, z_chunk):
        z1 = min(nz, z0 + z_chunk)
        gzy = (amps[:, None, None] * gz[:, z0:z1, None] * gy[:, None, :]).reshape(nb, -1)
        v = (gzy.T @ gx).reshape(z1 - z0, ny, nx)
        for lat, w, ((mx, fx), (my, fy), (mz, fz)) in zip(lats, ws, axes):
            mzc, fzc = mz[z0:z1], fz[z0:z1]
            zlo, zhi = int(mzc.min()), int(mzc.max()) + 2
            sub = lat[zlo:zhi]
            a = sub[:, :, mx] * (1 - fx) + sub[:, :, mx + 1] * fx
            a = a[:, my, :] * (1 - fy)[None, :, None] + a[:, my + 1, :] * fy[None, :, None]
            mzl = mzc - zlo
            a = a[mzl] * (1 - fzc)[:, None, None] + a[mzl + 1] * fzc[:, None, None]
            v += float(fbm_amp * w) * a
        out[z0:z1] = v.clamp_(0.0, 1.0).to(tdt)
    return out
