"""FP64 oracle of the per-rank local render (one brick -> one RGBA-z fragment per pixel).

The paper requires only that the local device produce colour and depth for each
pixel (section 5.1.2, Rendering; section 5.1.1 asks every fragment to carry RGBA
and depth).  The quadrature below is the reading this project adopts for that
local render; each step names its convention:

C1 grid    voxel (i,j,k) is the centre of cell [i,i+1)^3; h = 1/max(n); the world
           box is [0, n*h] per axis.
C2 sample  voxel-centre coordinate g = p/h - 0.5, clamped per axis to [0, n-1]
           (clamp-to-edge at the *global* domain), i0 = min(floor(g), n-2),
           f = g - i0, eight-corner trilinear.
C3 bricks  a brick owns global cells [lo, hi) and clips rays to [lo*h, hi*h];
           it stores one ghost voxel layer on faces shared with another brick.
C4 rays    pinhole through pixel centres, row 0 at the top, unit directions.
C5 clip    slab test; t_in = max(t_near, 0), t_out = t_far; hit iff t_out > t_in.
C6 lattice segment s is [s*dt, (s+1)*dt] in t, anchored at the eye, dt = step*h;
           a brick uses s in [floor(t_in/dt), ceil(t_out/dt) - 1], clips each to
           [t_in, t_out] (length l_s, dropped if <= 0) and evaluates the field
           once at the lattice midpoint (s+0.5)*dt.  Segment factors multiply
           exactly across brick faces, which makes splitting exact.
C7 TF      N entries, entry i at value lo + i*(hi-lo)/(N-1); u = clamp((v-lo)/(hi-lo),0,1),
           x = u*(N-1), j = min(floor(x), N-2), w = x - j, rgba = lerp(tf[j], tf[j+1], w).
C8 extinction sigma = D*A, tau = sigma*l, e = exp(-tau), a = -expm1(-tau).
C9 accumulate  C += T*a*rgb; T *= e (front to back, premultiplied); alpha = 1 - T.
C10 ERT    after each processed segment stop once 1 - T >= theta (theta >= 1: off).
C11 depth  t_in for a hit, +inf for a miss (empty fragment (0,0,0,0)).
C19 count  logical samples = processed segments with l_s > 0, skipped or not.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class RenderParams:
    step_voxels: float = 0.5
    ert: float = 0.99
    density: float = 20.0
    tf_lo: float = 0.0
    tf_hi: float = 1.0


def _normalize(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def camera_basis(cam):
    """Forward, right and up unit vectors of a pinhole camera (C4)."""
    eye = np.asarray(cam.eye, dtype=np.float64)
    f = _normalize(np.asarray(cam.center, dtype=np.float64) - eye)
    r = _normalize(np.cross(f, np.asarray(cam.up, dtype=np.float64)))
    u = np.cross(r, f)
    return f, r, u


def camera_rays(cam, px, py):
    """Ray origins and unit directions through pixel centres (C4); row 0 is the top."""
    f, r, u = camera_basis(cam)
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    th = math.tan(math.radians(cam.fovy_deg) / 2.0)
    aspect = cam.width / cam.height
    x = (2.0 * (px + 0.5) / cam.width - 1.0) * th * aspect
    y = (1.0 - 2.0 * (py + 0.5) / cam.height) * th
    d = _normalize(f[None, :] + x[:, None] * r[None, :] + y[:, None] * u[None, :])
    o = np.broadcast_to(np.asarray(cam.eye, dtype=np.float64), d.shape).copy()
    return o, d


def clip_box(o, d, box_lo, box_hi):
    """Slab test (C5).  Returns t_in, t_out and the hit mask (t_out > t_in, strict)."""
    R = o.shape[0]
    t_near = np.full(R, -np.inf)
    t_far = np.full(R, np.inf)
    ok = np.ones(R, dtype=bool)
    for a in range(3):
        da = d[:, a]
        zero = da == 0.0
        outside = (o[:, a] < box_lo[a]) | (o[:, a] > box_hi[a])
        ok &= ~(zero & outside)
        with np.errstate(divide="ignore", invalid="ignore"):
            t0 = (box_lo[a] - o[:, a]) / da
            t1 = (box_hi[a] - o[:, a]) / da
        tn = np.where(zero, -np.inf, np.minimum(t0, t1))
        tf = np.where(zero, np.inf, np.maximum(t0, t1))
        t_near = np.maximum(t_near, tn)
        t_far = np.minimum(t_far, tf)
    t_in = np.maximum(t_near, 0.0)
    t_out = t_far
    hit = ok & (t_out > t_in)
    return t_in, t_out, hit


def trilinear(data, stored_lo, dims, g):
    """Trilinear sample (C2) of a stored brick at global voxel-centre coordinates g (R,3).

    ``data`` is the stored array (z, y, x) covering global voxels starting at
    ``stored_lo`` (x, y, z).  Every corner index must lie in the stored range;
    this assertion is what proves that one ghost layer suffices.
    """
    R = g.shape[0]
    vals = data
    sz = (data.shape[2], data.shape[1], data.shape[0])
    i0 = np.empty((R, 3), dtype=np.int64)
    fr = np.empty((R, 3))
    for a in range(3):
        n = dims[a]
        ga = np.clip(g[:, a], 0.0, n - 1.0)
        ia = np.minimum(np.floor(ga), n - 2).astype(np.int64)
        fr[:, a] = ga - ia
        loc = ia - stored_lo[a]
        assert np.all(loc >= 0) and np.all(loc + 1 < sz[a]), "trilinear corner outside stored brick"
        i0[:, a] = loc
    x0, y0, z0 = i0[:, 0], i0[:, 1], i0[:, 2]
    fx, fy, fz = fr[:, 0], fr[:, 1], fr[:, 2]

    def V(dz, dy, dx):
        return vals[z0 + dz, y0 + dy, x0 + dx].astype(np.float64)

    # lerp form a + f (b - a): equal corners give exactly their value, so a sample
    # inside a constant region (e.g. a plateau at the TF range end) is exact
    def lerp(a, b, f):
        return a + f * (b - a)

    c00 = lerp(V(0, 0, 0), V(0, 0, 1), fx)
    c01 = lerp(V(0, 1, 0), V(0, 1, 1), fx)
    c10 = lerp(V(1, 0, 0), V(1, 0, 1), fx)
    c11 = lerp(V(1, 1, 0), V(1, 1, 1), fx)
    return lerp(lerp(c00, c01, fy), lerp(c10, c11, fy), fz)


def tf_lookup(tf, v, lo, hi):
    """Piecewise-linear transfer-function lookup (C7).  Returns (R,4) RGBA in FP64."""
    tf = np.asarray(tf, dtype=np.float64)
    n = tf.shape[0]
    u = np.clip((v - lo) / (hi - lo), 0.0, 1.0)
    x = u * (n - 1)
    j = np.minimum(np.floor(x), n - 2).astype(np.int64)
    w = (x - j)[:, None]
    return (1.0 - w) * tf[j] + w * tf[j + 1]


def march_rays(data, stored_lo, dims, owned_lo, owned_hi, tf, params: RenderParams, o, d):
    """Emission-absorption march of rays (o, d) through one brick (C5-C11, C19).

    Returns (rgba (R,4), depth (R,), samples (R,) int64).
    """
    dims = tuple(int(v) for v in dims)
    h = 1.0 / max(dims)
    dt = params.step_voxels * h
    D = params.density
    theta = params.ert
    box_lo = np.array(owned_lo, dtype=np.float64) * h
    box_hi = np.array(owned_hi, dtype=np.float64) * h
    R = o.shape[0]
    t_in, t_out, hit = clip_box(o, d, box_lo, box_hi)
    C = np.zeros((R, 3))
    T = np.ones(R)
    nsamp = np.zeros(R, dtype=np.int64)
    s0 = np.floor(t_in / dt)
    s1 = np.ceil(t_out / dt) - 1.0
    act = np.nonzero(hit)[0]
    k = 0
    while act.size:
        s = s0[act] + k
        seg_lo = np.maximum(s * dt, t_in[act])
        seg_hi = np.minimum((s + 1.0) * dt, t_out[act])
        ell = seg_hi - seg_lo
        valid = ell > 0.0
        tm = (s + 0.5) * dt
        rgba = np.zeros((act.size, 4))
        if valid.any():
            p = o[act[valid]] + tm[valid, None] * d[act[valid]]
            v = trilinear(data, stored_lo, dims, p / h - 0.5)
            rgba[valid] = tf_lookup(tf, v, params.tf_lo, params.tf_hi)
        tau = np.where(valid, D * rgba[:, 3] * ell, 0.0)
        e = np.exp(-tau)
        a = -np.expm1(-tau)
        C[act] += (T[act] * a)[:, None] * rgba[:, :3]
        T[act] *= e
        nsamp[act] += valid
        done = s >= s1[act]
        if theta < 1.0:
            done |= valid & (1.0 - T[act] >= theta)
        act = act[~done]
        k += 1
    rgba = np.zeros((R, 4))
    rgba[:, :3] = C
    rgba[:, 3] = np.where(hit, 1.0 - T, 0.0)
    depth = np.where(hit, t_in, np.inf)
    return rgba, depth, nsamp


def march_rays_thresholds(data, stored_lo, dims, owned_lo, owned_hi, tf, params: RenderParams, o, d, thetas):
    """The march of ``march_rays`` evaluated for several termination thresholds at
    once (C10): one pass continues until the largest threshold stops a ray, and
    each threshold keeps the accumulators as they stood after the segment at which
    1 - T first reached it.  Returns a list of (rgba, depth, samples), one per
    threshold; each equals ``march_rays`` with that threshold.
    """
    dims = tuple(int(v) for v in dims)
    h = 1.0 / max(dims)
    dt = params.step_voxels * h
    D = params.density
    thetas = [float(th) for th in thetas]
    box_lo = np.array(owned_lo, dtype=np.float64) * h
    box_hi = np.array(owned_hi, dtype=np.float64) * h
    R = o.shape[0]
    t_in, t_out, hit = clip_box(o, d, box_lo, box_hi)
    C = np.zeros((R, 3))
    T = np.ones(R)
    nsamp = np.zeros(R, dtype=np.int64)
    # per threshold: whether it has stopped the ray, and the state it stopped at
    stopped = [np.zeros(R, dtype=bool) for _ in thetas]
    keep = [(np.zeros((R, 3)), np.ones(R), np.zeros(R, dtype=np.int64)) for _ in thetas]
    s0 = np.floor(t_in / dt)
    s1 = np.ceil(t_out / dt) - 1.0
    act = np.nonzero(hit)[0]
    k = 0
    while act.size:
        s = s0[act] + k
        seg_lo = np.maximum(s * dt, t_in[act])
        seg_hi = np.minimum((s + 1.0) * dt, t_out[act])
        ell = seg_hi - seg_lo
        valid = ell > 0.0
        tm = (s + 0.5) * dt
        rgba = np.zeros((act.size, 4))
        if valid.any():
            p = o[act[valid]] + tm[valid, None] * d[act[valid]]
            v = trilinear(data, stored_lo, dims, p / h - 0.5)
            rgba[valid] = tf_lookup(tf, v, params.tf_lo, params.tf_hi)
        tau = np.where(valid, D * rgba[:, 3] * ell, 0.0)
        e = np.exp(-tau)
        a = -np.expm1(-tau)
        C[act] += (T[act] * a)[:, None] * rgba[:, :3]
        T[act] *= e
        nsamp[act] += valid
        last = s >= s1[act]
        for i, th in enumerate(thetas):
            new = ~stopped[i][act] & (last | (th < 1.0) & valid & (1.0 - T[act] >= th))
            rows = act[new]
            keep[i][0][rows] = C[rows]
            keep[i][1][rows] = T[rows]
            keep[i][2][rows] = nsamp[rows]
            stopped[i][rows] = True
        act = act[~np.all([st[act] for st in stopped], axis=0)]
        k += 1
    out = []
    for Ck, Tk, nk in keep:
        rgba = np.zeros((R, 4))
        rgba[:, :3] = Ck
        rgba[:, 3] = np.where(hit, 1.0 - Tk, 0.0)
        out.append((rgba, np.where(hit, t_in, np.inf), nk))
    return out


def render_brick_thresholds(data, stored_lo, dims, owned_lo, owned_hi, tf, params, cam, px, py, thetas,
                            chunk=1 << 16):
    """``render_brick`` on the pixels (px, py) for several termination thresholds in
    one march per ray (``march_rays_thresholds``); a list of (rgba, depth, samples)."""
    px = np.asarray(px)
    py = np.asarray(py)
    R = px.size
    res = [(np.empty((R, 4)), np.empty(R), np.empty(R, dtype=np.int64)) for _ in thetas]
    for c0 in range(0, R, chunk):
        c1 = min(R, c0 + chunk)
        o, d = camera_rays(cam, px[c0:c1], py[c0:c1])
        for (rg, dp, ns), (r2, d2, n2) in zip(res, march_rays_thresholds(
                data, stored_lo, dims, owned_lo, owned_hi, tf, params, o, d, thetas)):
            rg[c0:c1], dp[c0:c1], ns[c0:c1] = r2, d2, n2
    return res


def render_brick(data, stored_lo, dims, owned_lo, owned_hi, tf, params, cam, px=None, py=None,
                 chunk=1 << 16):
    """Render one brick's partial frame (or a pixel subset of it).

    Without ``px``/``py`` returns full images rgba (H,W,4), depth (H,W), samples (H,W);
    with them returns per-pixel arrays in the given order.
    """
    full = px is None
    if full:
        py_, px_ = np.mgrid[0:cam.height, 0:cam.width]
        px, py = px_.ravel(), py_.ravel()
    px = np.asarray(px)
    py = np.asarray(py)
    R = px.size
    rgba = np.empty((R, 4))
    depth = np.empty(R)
    ns = np.empty(R, dtype=np.int64)
    for c0 in range(0, R, chunk):
        c1 = min(R, c0 + chunk)
        o, d = camera_rays(cam, px[c0:c1], py[c0:c1])
        rgba[c0:c1], depth[c0:c1], ns[c0:c1] = march_rays(
            data, stored_lo, dims, owned_lo, owned_hi, tf, params, o, d)
    if full:
        return (rgba.reshape(cam.height, cam.width, 4), depth.reshape(cam.height, cam.width),
                ns.reshape(cam.height, cam.width))
    return rgba, depth, ns


def render_image(volume, dims, tf, params, cam, px=None, py=None):
    """Unsplit render: the whole global volume as one brick."""
    return render_brick(volume, (0, 0, 0), dims, (0, 0, 0), tuple(dims), tf, params, cam, px, py)
