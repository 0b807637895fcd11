"""FP64 oracle of iso-surface fragments mixed with the emission-absorption march.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper renders iso-surfaces through the same data-parallel pipeline as volumes
(Fig. 1c, Fig. 3c, Fig. 4): a rank's local render only has to give colour and
depth per pixel (section 5.1.2), and the compositor needs nothing else (section
5.1.1).  How a local renderer finds the surface is left open; this is the
reading (C20), on top of C1-C11 and C19 of ``render.py``:

* The field is the trilinear interpolant of C2 sampled at the lattice midpoints
  q_s = o + (s + 1/2) dt d of C6.  A sample's side is v_s >= v_iso.
* Consecutive samples (s-1, s) form the pair at lattice point t_s = s dt.  A brick
  tests the pairs whose lattice point lies in [t_in, t_out): the pairs of
  consecutive segments it processes, plus (s_a - 1, s_a) when its first processed
  segment s_a starts exactly at t_in (sample s_a - 1 then lies half a step before
  the brick, inside its ghost layer).  Every lattice point on a ray's path
  through the volume lies in one brick, so each pair is tested exactly once.
* Per processed segment s, in order: if its pair is tested and the two sides
  differ, the ray hits the surface and segment s adds no emission; otherwise the
  segment is integrated as in C8-C9 and ERT is tested (C10).
* Hit point, in voxel-centre coordinates: g = g_{s-1} + f (g_s - g_{s-1}),
  f = (v_iso - v_{s-1}) / (v_s - v_{s-1}).
* Shading: albedo = RGB of the TF at v_iso (C7); n = gradient of the trilinear
  patch at g (cell and fractions by the clamp rule of C2); c = albedo (k_a +
  k_d |n . d| / |n|), with |n . d| / |n| taken as 1 where n = 0.
* The surface is opaque: C += T c and T = 0, so alpha = 1.  Depth stays t_in
  (C11), which keeps the compositing order of convex bricks.  The hit segment
  counts as a processed sample (C19).
Pairs use global sample positions and each is tested by one brick, so a split
volume composites to the unsplit image (the split invariant holds).

Skipping (an optimisation, must not change results; C21): a macrocell may be
skipped only if its majorant is 0 and its value range lies on one side of v_iso
by a margin m = 1e-6 max(|min|, |max|) (FP32 trilinear values stay within a few
ulps of the range), written here in FP64 from that definition.  ``iso_classes``
encodes it per macrocell: the majorant where positive; else 0 (skippable, every
sample below v_iso), -1 (skippable, every sample at or above v_iso) or 1 (must be
sampled).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .render import RenderParams, camera_rays, clip_box, tf_lookup, trilinear


@dataclass
class IsoParams:
    value: float
    ambient: float = 0.25
    diffuse: float = 0.75


def trilinear_grad(data, stored_lo, dims, g):
    """Gradient (voxel units) of the trilinear patch (C2 cell and fractions) at g (R,3)."""
    R = g.shape[0]
    sz = (data.shape[2], data.shape[1], data.shape[0])
    i0 = np.empty((R, 3), dtype=np.int64)
    fr = np.empty((R, 3))
    for a in range(3):
        n = dims[a]
        ga = np.clip(g[:, a], 0.0, n - 1.0)
        ia = np.minimum(np.floor(ga), n - 2).astype(np.int64)
        fr[:, a] = ga - ia
        loc = ia - stored_lo[a]
        assert np.all(loc >= 0) and np.all(loc + 1 < sz[a]), "gradient corner outside stored brick"
        i0[:, a] = loc
    x0, y0, z0 = i0[:, 0], i0[:, 1], i0[:, 2]
    fx, fy, fz = fr[:, 0], fr[:, 1], fr[:, 2]

    def V(dz, dy, dx):
        return data[z0 + dz, y0 + dy, x0 + dx].astype(np.float64)

    # v = sum over corners of w_x w_y w_z V, with w = 1 - f or f; differentiate one factor
    wx = (1.0 - fx, fx)
    wy = (1.0 - fy, fy)
    wz = (1.0 - fz, fz)
    gx = np.zeros(R)
    gy = np.zeros(R)
    gz = np.zeros(R)
    for dz in (0, 1):
        for dy in (0, 1):
            gx += wy[dy] * wz[dz] * (V(dz, dy, 1) - V(dz, dy, 0))
    for dz in (0, 1):
        for dx in (0, 1):
            gy += wx[dx] * wz[dz] * (V(dz, 1, dx) - V(dz, 0, dx))
    for dy in (0, 1):
        for dx in (0, 1):
            gz += wx[dx] * wy[dy] * (V(1, dy, dx) - V(0, dy, dx))
    return np.stack([gx, gy, gz], axis=1)


def march_rays_iso(data, stored_lo, dims, owned_lo, owned_hi, tf, params: RenderParams, iso: IsoParams, o, d):
    """Emission-absorption march with an opaque iso-surface (C20) through one brick.

    Returns (rgba (R,4), depth (R,), samples (R,) int64, margin (R,)), where margin
    is the smallest |v - v_iso| over the samples whose side was taken (how close
    the ray came to deciding a pair the other way).
    """
    dims = tuple(int(v) for v in dims)
    h = 1.0 / max(dims)
    dt = params.step_voxels * h
    D = params.density
    theta = params.ert
    vi = float(iso.value)
    box_lo = np.array(owned_lo, dtype=np.float64) * h
    box_hi = np.array(owned_hi, dtype=np.float64) * h
    R = o.shape[0]
    t_in, t_out, hit = clip_box(o, d, box_lo, box_hi)
    C = np.zeros((R, 3))
    T = np.ones(R)
    nsamp = np.zeros(R, dtype=np.int64)
    margin = np.full(R, np.inf)
    albedo = tf_lookup(tf, np.array([vi]), params.tf_lo, params.tf_hi)[0, :3]
    s0 = np.floor(t_in / dt)
    s1 = np.ceil(t_out / dt) - 1.0
    # the first processed segment, and whether the pair at its start is this brick's
    ell0 = np.minimum((s0 + 1.0) * dt, t_out) - np.maximum(s0 * dt, t_in)
    sa = np.where(ell0 > 0.0, s0, s0 + 1.0)
    has_prev = hit & (sa * dt >= t_in)
    prev_v = np.zeros(R)
    idx = np.nonzero(has_prev)[0]
    if idx.size:
        p = o[idx] + ((sa[idx] - 0.5) * dt)[:, None] * d[idx]
        prev_v[idx] = trilinear(data, stored_lo, dims, p / h - 0.5)
        margin[idx] = np.abs(prev_v[idx] - vi)
    act = np.nonzero(hit)[0]
    k = 0
    while act.size:
        s = s0[act] + k
        seg_lo = np.maximum(s * dt, t_in[act])
        seg_hi = np.minimum((s + 1.0) * dt, t_out[act])
        ell = seg_hi - seg_lo
        valid = ell > 0.0
        tm = (s + 0.5) * dt
        v = np.zeros(act.size)
        if valid.any():
            p = o[act[valid]] + tm[valid, None] * d[act[valid]]
            v[valid] = trilinear(data, stored_lo, dims, p / h - 0.5)
        margin[act[valid]] = np.minimum(margin[act[valid]], np.abs(v[valid] - vi))
        # the pair (s-1, s): a change of side is the surface
        cross = valid & has_prev[act] & ((v >= vi) != (prev_v[act] >= vi))
        ci = np.nonzero(cross)[0]
        if ci.size:
            rays = act[ci]
            vp, vs = prev_v[rays], v[ci]
            f = (vi - vp) / (vs - vp)
            gp = (o[rays] + ((s[ci] - 0.5) * dt)[:, None] * d[rays]) / h - 0.5
            gs = (o[rays] + ((s[ci] + 0.5) * dt)[:, None] * d[rays]) / h - 0.5
            gh = gp + f[:, None] * (gs - gp)
            n = trilinear_grad(data, stored_lo, dims, gh)
            nn = np.linalg.norm(n, axis=1)
            with np.errstate(divide="ignore", invalid="ignore"):
                cosv = np.where(nn > 0.0, np.abs(np.sum(n * d[rays], axis=1)) / nn, 1.0)
            c = albedo[None, :] * (iso.ambient + iso.diffuse * cosv)[:, None]
            C[rays] += T[rays, None] * c
            T[rays] = 0.0
            nsamp[rays] += 1
        # emission-absorption of every other processed segment (C8-C9)
        ea = valid & ~cross
        rgba = np.zeros((act.size, 4))
        if ea.any():
            rgba[ea] = tf_lookup(tf, v[ea], params.tf_lo, params.tf_hi)
        tau = np.where(ea, D * rgba[:, 3] * ell, 0.0)
        e = np.exp(-tau)
        a = -np.expm1(-tau)
        C[act] += (T[act] * a)[:, None] * rgba[:, :3]
        T[act] *= e
        nsamp[act] += ea
        prev_v[act[ea]] = v[ea]
        has_prev[act[ea]] = True
        done = (s >= s1[act]) | cross
        if theta < 1.0:
            done |= ea & (1.0 - T[act] >= theta)
        act = act[~done]
        k += 1
    rgba = np.zeros((R, 4))
    rgba[:, :3] = C
    rgba[:, 3] = np.where(hit, 1.0 - T, 0.0)
    depth = np.where(hit, t_in, np.inf)
    return rgba, depth, nsamp, margin


def render_brick_iso(data, stored_lo, dims, owned_lo, owned_hi, tf, params, iso, cam, px=None, py=None,
                     chunk=1 << 16):
    """One brick's partial frame with the iso-surface; per-pixel arrays.

    Without ``px``/``py`` every pixel in row-major order.  Returns (rgba (R,4),
    depth (R,), samples (R,), margin (R,)).
    """
    if px is None:
        py_, px_ = np.mgrid[0:cam.height, 0:cam.width]
        px, py = px_.ravel(), py_.ravel()
    px = np.asarray(px)
    py = np.asarray(py)
    R = px.size
    out = (np.empty((R, 4)), np.empty(R), np.empty(R, dtype=np.int64), np.empty(R))
    for c0 in range(0, R, chunk):
        c1 = min(R, c0 + chunk)
        o, d = camera_rays(cam, px[c0:c1], py[c0:c1])
        res = march_rays_iso(data, stored_lo, dims, owned_lo, owned_hi, tf, params, iso, o, d)
        for dst, src in zip(out, res):
            dst[c0:c1] = src
    return out


def render_image_iso(volume, dims, tf, params, iso, cam, px=None, py=None):
    """Unsplit render with the iso-surface: the whole global volume as one brick."""
    return render_brick_iso(volume, (0, 0, 0), dims, (0, 0, 0), tuple(dims), tf, params, iso, cam, px, py)


def iso_classes(ranges, majorant, iso_value):
    """Skip class per macrocell (C21) from (..., 2) ranges and majorants -> float32,
    from the plain definition in FP64: the majorant where positive; else 0 when
    max < v_iso - m, -1 when min > v_iso + m, 1 otherwise, m = 1e-6 max(|min|, |max|)."""
    lo = np.asarray(ranges[..., 0], dtype=np.float64)
    hi = np.asarray(ranges[..., 1], dtype=np.float64)
    maj = np.asarray(majorant, dtype=np.float32)
    v = float(iso_value)
    m = 1e-6 * np.maximum(np.abs(lo), np.abs(hi))
    below = hi < v - m
    above = lo > v + m
    out = np.where(maj > 0, maj, np.where(below, np.float32(0.0), np.where(above, np.float32(-1.0),
                                                                                np.float32(1.0))))
    return out.astype(np.float32)


def iso_class_ambiguous(ranges, iso_value, ulps=4):
    """True where a range end lies within a few FP32 ulps of v_iso -+ m, so that the
    class decided in FP32 may differ from the FP64 one (both are valid: the margin
    m covers the FP32 rounding of trilinear values either way)."""
    lo = np.asarray(ranges[..., 0], dtype=np.float64)
    hi = np.asarray(ranges[..., 1], dtype=np.float64)
    v = float(iso_value)
    m = 1e-6 * np.maximum(np.abs(lo), np.abs(hi))
    tol = ulps * float(np.spacing(np.float32(max(abs(v), 1e-30))))
    return (np.abs(hi - (v - m)) <= tol) | (np.abs(lo - (v + m)) <= tol)
