"""FP64 oracle of the L2-loss gradient w.r.t. the density grid and the TF table.

Differentiation is not in the paper; it follows from the local-render reading
of ``render.py`` (ERT off, whole volume as one brick).  Loss (C16):
L = mean over (camera, pixel, channel in RGBA) of (I - I*)^2.

Per ray with samples s = 0..S-1, T_s the transmittance before sample s,
a_s = 1 - exp(-tau_s), colour c_s, C = sum_s T_s a_s c_s and alpha = 1 - T_S,
and with g_C = dL/dC, g_a = dL/dalpha and the exclusive suffix
C_{>s} = sum_{j>s} T_j a_j c_j:

  dL/dc_s   = T_s a_s g_C
  dL/dtau_s = g_C . (T_{s+1} c_s - C_{>s}) + g_a T_S
  dL/dA_s   = dL/dtau_s * D * l_s

(the derivative of T_s a_s w.r.t. tau_s is T_s e_s = T_{s+1}; every later
term carries T_j, whose derivative is -T_j; and dalpha/dtau_s = T_S).  TF entries
j, j+1 receive the lerp weights (1-w, w); the sample value v receives
(tf[j+1]-tf[j]) (N-1)/(hi-lo) (0 where u is clamped), and each of the eight
trilinear corners receives its trilinear weight.
"""

from __future__ import annotations

import numpy as np

from .render import RenderParams, camera_rays, clip_box


def _corners(dims, g):
    """Flat (z,y,x) indices (R,8), weights (R,8) and fractions (R,3) of the trilinear
    stencil (C2); corner c = 4 dz + 2 dy + dx."""
    R = g.shape[0]
    i0 = np.empty((R, 3), dtype=np.int64)
    fr = np.empty((R, 3))
    for a in range(3):
        n = dims[a]
        ga = np.clip(g[:, a], 0.0, n - 1.0)
        ia = np.minimum(np.floor(ga), n - 2).astype(np.int64)
        i0[:, a] = ia
        fr[:, a] = ga - ia
    nx, ny = dims[0], dims[1]
    idx = np.empty((R, 8), dtype=np.int64)
    wt = np.empty((R, 8))
    c = 0
    for dz in (0, 1):
        wz = fr[:, 2] if dz else 1.0 - fr[:, 2]
        for dy in (0, 1):
            wy = fr[:, 1] if dy else 1.0 - fr[:, 1]
            for dx in (0, 1):
                wx = fr[:, 0] if dx else 1.0 - fr[:, 0]
                idx[:, c] = ((i0[:, 2] + dz) * ny + (i0[:, 1] + dy)) * nx + (i0[:, 0] + dx)
                wt[:, c] = wz * wy * wx
                c += 1
    return idx, wt, fr


def _lerp_value(vals, fr):
    """Trilinear value from the 8 corner values (stencil order of _corners) and the
    fractions fr = (fx, fy, fz), as nested lerps a + f (b - a): exact on constant
    stencils, so a sample among voxels at a clamp bound sits exactly on it."""

    def lerp(a, b, f):
        return a + f * (b - a)

    c00 = lerp(vals[:, 0], vals[:, 1], fr[:, 0])
    c01 = lerp(vals[:, 2], vals[:, 3], fr[:, 0])
    c10 = lerp(vals[:, 4], vals[:, 5], fr[:, 0])
    c11 = lerp(vals[:, 6], vals[:, 7], fr[:, 0])
    return lerp(lerp(c00, c01, fr[:, 1]), lerp(c10, c11, fr[:, 1]), fr[:, 2])


def _tf_parts(tf, v, lo, hi):
    n = tf.shape[0]
    raw = (v - lo) / (hi - lo)
    u = np.clip(raw, 0.0, 1.0)
    x = u * (n - 1)
    j = np.minimum(np.floor(x), n - 2).astype(np.int64)
    w = x - j
    rgba = (1.0 - w)[:, None] * tf[j] + w[:, None] * tf[j + 1]
    inside = (raw >= 0.0) & (raw <= 1.0)
    return rgba, j, w, inside


def _trace(vol_flat, dims, tf, params, o, d, record):
    dims = tuple(int(v) for v in dims)
    h = 1.0 / max(dims)
    dt = params.step_voxels * h
    D = params.density
    R = o.shape[0]
    t_in, t_out, hit = clip_box(o, d, np.zeros(3), np.array(dims, dtype=np.float64) * h)
    C = np.zeros((R, 3))
    T = np.ones(R)
    s0 = np.floor(t_in / dt)
    s1 = np.ceil(t_out / dt) - 1.0
    act = np.nonzero(hit)[0]
    steps = []
    k = 0
    while act.size:
        s = s0[act] + k
        ell = np.maximum(np.minimum((s + 1.0) * dt, t_out[act]) - np.maximum(s * dt, t_in[act]), 0.0)
        p = o[act] + ((s + 0.5) * dt)[:, None] * d[act]
        idx, wt, fr = _corners(dims, p / h - 0.5)
        v = _lerp_value(vol_flat[idx], fr)
        rgba, j, w, inside = _tf_parts(tf, v, params.tf_lo, params.tf_hi)
        tau = D * rgba[:, 3] * ell
        e = np.exp(-tau)
        a = -np.expm1(-tau)
        Tb = T[act].copy()
        C[act] += (Tb * a)[:, None] * rgba[:, :3]
        T[act] = Tb * e
        if record:
            steps.append((act, ell, idx, wt, rgba, j, w, inside, Tb, a, e))
        act = act[~(s >= s1[act])]
        k += 1
    img = np.zeros((R, 4))
    img[:, :3] = C
    img[:, 3] = np.where(hit, 1.0 - T, 0.0)
    return img, T, steps


def forward_image(volume, dims, tf, params: RenderParams, cams, chunk=1 << 15):
    """Rendered images (ncam, H, W, 4), ERT ignored (always off for training)."""
    vol_flat = np.asarray(volume, dtype=np.float64).ravel()
    tf = np.asarray(tf, dtype=np.float64)
    out = []
    for cam in cams:
        py, px = np.mgrid[0:cam.height, 0:cam.width]
        px, py = px.ravel(), py.ravel()
        img = np.empty((px.size, 4))
        for c0 in range(0, px.size, chunk):
            o, d = camera_rays(cam, px[c0:c0 + chunk], py[c0:c0 + chunk])
            img[c0:c0 + chunk] = _trace(vol_flat, dims, tf, params, o, d, False)[0]
        out.append(img.reshape(cam.height, cam.width, 4))
    return np.stack(out)


def loss_and_grad(volume, dims, tf, params: RenderParams, cams, target, chunk=4096, n_elems=None, pixels=None):
    """L2 loss and its gradients (FP64).

    ``target``: (ncam, H, W, 4), or per camera (P, 4) when ``pixels`` gives each
    camera's (px, py) subset.  ``n_elems`` overrides the mean's denominator
    (default: every target channel).
    Returns (loss, grad_volume (same shape as volume), grad_tf (N, 4), images).
    """
    vol_flat = np.asarray(volume, dtype=np.float64).ravel()
    tf = np.asarray(tf, dtype=np.float64)
    n = tf.shape[0]
    slope_scale = (n - 1) / (params.tf_hi - params.tf_lo)
    D = params.density
    gV = np.zeros_like(vol_flat)
    gT = np.zeros_like(tf)
    if pixels is None:
        target = np.asarray(target, dtype=np.float64)
    else:
        target = [np.asarray(t, dtype=np.float64) for t in target]
    if n_elems is None:
        n_elems = sum(np.size(t) for t in target)
    loss = 0.0
    images = []
    for ci, cam in enumerate(cams):
        if pixels is None:
            py, px = np.mgrid[0:cam.height, 0:cam.width]
            px, py = px.ravel(), py.ravel()
        else:
            px, py = (np.asarray(a) for a in pixels[ci])
        tgt = target[ci].reshape(-1, 4)
        img = np.empty((px.size, 4))
        for c0 in range(0, px.size, chunk):
            sl = slice(c0, c0 + chunk)
            o, d = camera_rays(cam, px[sl], py[sl])
            im, T_end, steps = _trace(vol_flat, dims, tf, params, o, d, True)
            img[sl] = im
            diff = im - tgt[sl]
            loss += np.sum(diff * diff) / n_elems
            gI = 2.0 * diff / n_elems
            gC, ga = gI[:, :3], gI[:, 3]
            suffix = np.zeros((o.shape[0], 3))  # C_{>s}
            for (act, ell, idx, wt, rgba, j, w, inside, Tb, a, e) in reversed(steps):
                c = rgba[:, :3]
                T_next = Tb * e
                g_c = (Tb * a)[:, None] * gC[act]
                g_tau = np.sum(gC[act] * (T_next[:, None] * c - suffix[act]), axis=1) + ga[act] * T_end[act]
                g_A = g_tau * D * ell
                suffix[act] += (Tb * a)[:, None] * c
                g4 = np.concatenate([g_c, g_A[:, None]], axis=1)
                np.add.at(gT, j, (1.0 - w)[:, None] * g4)
                np.add.at(gT, j + 1, w[:, None] * g4)
                dtf = (tf[j + 1] - tf[j]) * slope_scale
                g_v = np.where(inside, np.sum(g4 * dtf, axis=1), 0.0)
                np.add.at(gV, idx.ravel(), (g_v[:, None] * wt).ravel())
        images.append(img.reshape(cam.height, cam.width, 4) if pixels is None else img)
    return loss, gV.reshape(np.shape(volume)), gT, (np.stack(images) if pixels is None else images)
