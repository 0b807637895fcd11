"""FP64 oracle of data-parallel volumetric path tracing.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper motivates data-parallel rendering that goes beyond one fragment per
rank: illumination such as volumetric shadows needs rays that visit content on
other ranks (section 2.2; Fig. 7, thunderstorm with volumetric shadows), and its
path tracer forwards each ray to the rank holding the content it meets next, so
every ray finds its true interactions wherever it was spawned (section 5.2,
Barney; the wave-front exchange of section 2.2).  The estimator a rank runs on
the rays it holds is not given; this is the reading (C22), on the field of C1-C2
and the transfer function of C7:

* Medium: extinction sigma(x) = D A(v(x)); single-scattering albedo = the TF's
  RGB at v(x); isotropic phase function 1/(4 pi); no emission.  Light: one
  directional light (radiance L_l, travelling along l_dir) and a constant
  environment radiance L_e seen by rays leaving the volume box.
* Majorant: piecewise constant on the global grid of 16^3-cell blocks: block b
  has sigma_bar_b = D m_b, with m_b the transfer-function majorant (C13, decided
  in FP32) of the value range over voxels [16 b - 1, 16 b + 16] per axis.  The
  grid is global, so the tentative collisions of a path do not depend on how the
  volume is split into bricks; a block with m_b = 0 holds no tentative collision.
* Random numbers: Philox4x32-10 (``rng.py``), key (seed, 0x243F6A88), counter
  (path, event, kind, step).  Path id = (row * width + column) * spp + sample;
  event e counts the tentative collisions of the path; one draw per event gives
  u0 (free flight), u1 (real or null), u2, u3 (new direction).
* Camera ray through the pixel centre (C4), started at its entry t_in into the
  volume box; a ray that misses the box sees L_e.
* Delta tracking: from x along w, walk the blocks (a 3D DDA), accumulating
  sigma_bar_b times the length in each, until the sum reaches tau = -ln(u0); the
  tentative point q is where it does.  If the walk leaves the box first, the path
  leaves: it adds thr L_e.  Otherwise q is real when u1 < sigma(q) / sigma_bar(q)
  (the majorant of the block holding q's cell; 0 / 0 counts as null); else null,
  and the flight goes on from q.
* At the k-th real collision (k = 0, 1, ...): thr *= albedo(q); a shadow ray from
  q towards the light (-l_dir) estimates the transmittance by ratio tracking:
  flights of optical length -ln(u) (u from counter (path, e, 1, step)) under the
  same block majorants, T *= 1 - sigma / sigma_bar at each tentative point, until
  a flight leaves the box; the path adds thr L_l T / (4 pi).  After B real collisions the path ends; else it
  leaves q in the isotropic direction z = 1 - 2 u2, phi = 2 pi u3.
* Pixel radiance = mean over its spp paths of the sum of the path's
  contributions (NEE terms in collision order, then the environment term).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .render import RenderParams, camera_rays, clip_box, tf_lookup, trilinear
from .rng import philox4x32, uniforms

KEY1 = 0x243F6A88


@dataclass
class PathParams:
    light_dir: tuple = (-0.45, -0.55, -0.7)
    light_rgb: tuple = (3.0, 2.8, 2.5)
    env_rgb: tuple = (0.15, 0.2, 0.3)
    max_bounces: int = 3
    spp: int = 1
    seed: int = 1


def _draw(pid, e, kind, step, seed):
    n = pid.shape[0]
    ctr = np.stack([pid, e, np.full(n, kind), step], axis=1).astype(np.uint64)
    key = np.stack([np.full(n, seed), np.full(n, KEY1)], axis=1).astype(np.uint64)
    return uniforms(philox4x32(ctr, key))


BLOCK = 16


def _entry_range32(ranges, n, lo, hi):
    """The majorant's table-entry range [floor(x_min) - 1, ceil(x_max) + 1] with the
    table coordinates taken in FP32: u = (v - lo) / (hi - lo), clamp to [0, 1],
    x = u (N - 1).  Any entry range that covers the values gives an unbiased
    estimator, but the tentative collisions, and so the paths, depend on sigma_bar
    itself; the estimator is defined with this FP32 decision so that a path is one
    definite sequence of events (an integer decided in the kernel's precision)."""
    f32 = np.float32
    out = []
    for k in (0, 1):
        v = np.asarray(ranges[..., k], dtype=f32)
        u = (v - f32(lo)) / (f32(hi) - f32(lo))
        out.append(np.minimum(np.maximum(u, f32(0.0)), f32(1.0)) * f32(n - 1))
    e0 = np.maximum(np.floor(out[0]).astype(np.int64) - 1, 0)
    e1 = np.minimum(np.ceil(out[1]).astype(np.int64) + 1, n - 1)
    return e0, e1


def block_majorants(volume, dims, tf, params: RenderParams):
    """sigma_bar per 16^3-cell block of the global grid -> (Mz, My, Mx) FP64: D times
    the largest TF opacity over the entry range of the block's value range (C13
    windows, one voxel of apron)."""
    from .macrocell import macrocell_ranges
    rng = macrocell_ranges(volume, (0, 0, 0), tuple(int(v) for v in dims), (0, 0, 0), BLOCK)
    a = np.asarray(tf, dtype=np.float32)[:, 3]
    e0, e1 = _entry_range32(rng, a.shape[0], params.tf_lo, params.tf_hi)
    m = np.array([a[i:j + 1].max() for i, j in zip(e0.ravel(), e1.ravel())], dtype=np.float32)
    return params.density * m.reshape(e0.shape).astype(np.float64)


def _block_of(q, dims, h):
    cell = np.clip(np.floor(q / h).astype(np.int64), 0, np.array(dims) - 1)
    return cell // BLOCK


def _flight(x, w, target, grid, dims, h):
    """Delta-tracking flight under the block majorants: distance t along w from x
    at which the accumulated sigma_bar * length reaches target (inf if the walk
    leaves the box first), and the smallest |accumulated - target| at a block
    boundary (how close a block or exit decision came to going the other way)."""
    n = x.shape[0]
    dims_a = np.array(dims, dtype=np.int64)
    box_hi = dims_a * h
    t_box = _exit_distance(x, w, box_hi)
    blk = _block_of(x, dims, h)
    t = np.zeros(n)
    acc = np.zeros(n)
    out = np.full(n, np.inf)
    margin = np.full(n, np.inf)
    act = np.arange(n)
    while act.size:
        b = blk[act]
        lo = b * BLOCK * h
        hi = np.minimum((b + 1) * BLOCK, dims_a) * h
        xa, wa = x[act], w[act]
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = np.where(wa > 0, (hi - xa) / wa, np.where(wa < 0, (lo - xa) / wa, np.inf))
        t_next = ta.min(axis=1)
        seg_end = np.minimum(t_next, t_box[act])
        sb = grid[b[:, 2], b[:, 1], b[:, 0]]
        gain = sb * (seg_end - t[act])
        hit = acc[act] + gain >= target[act]
        hi_idx = act[hit]
        out[hi_idx] = t[hi_idx] + (target[hi_idx] - acc[hi_idx]) / sb[hit]
        miss = ~hit
        mi = act[miss]
        acc[mi] += gain[miss]
        t[mi] = seg_end[miss]
        margin[mi] = np.minimum(margin[mi], np.abs(acc[mi] - target[mi]))
        go_on = miss & (seg_end < t_box[act])
        step = (ta == t_next[:, None]) & go_on[:, None]
        blk[act] = b + np.where(step, np.sign(wa).astype(np.int64), 0)
        act = act[go_on]
    return out, margin


def _exit_distance(x, w, box_hi):
    """Distance from points x inside the box [0, box_hi] to its exit along w."""
    t = np.full(x.shape[0], np.inf)
    for a in range(3):
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = np.where(w[:, a] > 0, (box_hi[a] - x[:, a]) / w[:, a],
                          np.where(w[:, a] < 0, -x[:, a] / w[:, a], np.inf))
        t = np.minimum(t, ta)
    return t


def _medium(volume, dims, tf, params, q):
    h = 1.0 / max(dims)
    v = trilinear(volume, (0, 0, 0), dims, q / h - 0.5)
    rgba = tf_lookup(tf, v, params.tf_lo, params.tf_hi)
    return params.density * rgba[:, 3], rgba[:, :3]


def trace_paths(volume, dims, tf, params: RenderParams, pp: PathParams, o, d, pid):
    """Radiance (N,3) of the paths (o, d, pid), and the decision margin (N,): the
    smallest of |u1 - sigma/sigma_bar| and sigma_bar |t - exit| over the path."""
    dims = tuple(int(v) for v in dims)
    h = 1.0 / max(dims)
    box_hi = np.array(dims, dtype=np.float64) * h
    grid = block_majorants(volume, dims, tf, params)
    tf = np.asarray(tf, dtype=np.float64)
    B = int(pp.max_bounces)
    ldir = -np.asarray(pp.light_dir, dtype=np.float64)
    ldir = ldir / np.linalg.norm(ldir)
    L_l = np.asarray(pp.light_rgb, dtype=np.float64)
    L_e = np.asarray(pp.env_rgb, dtype=np.float64)
    N = o.shape[0]
    L = np.zeros((N, 3))
    margin = np.full(N, np.inf)
    t_in, _, hit = clip_box(o, d, np.zeros(3), box_hi)
    L[~hit] = L_e
    act = np.nonzero(hit)[0]
    x = o[act] + t_in[act, None] * d[act]
    w = d[act].copy()
    thr = np.ones((act.size, 3))
    e = np.zeros(act.size, dtype=np.int64)
    bounce = np.zeros(act.size, dtype=np.int64)
    while act.size:
        u = _draw(pid[act], e, 0, np.zeros(act.size, dtype=np.int64), pp.seed)
        t, fm = _flight(x, w, -np.log(u[:, 0]), grid, dims, h)
        margin[act] = np.minimum(margin[act], fm)
        leave = ~np.isfinite(t)
        L[act[leave]] += thr[leave] * L_e
        keep = ~leave
        act, x, w, thr, e, bounce, u, t = (a[keep] for a in (act, x, w, thr, e, bounce, u, t))
        if not act.size:
            break
        q = x + t[:, None] * w
        sigma, alb = _medium(volume, dims, tf, params, q)
        bq = _block_of(q, dims, h)
        sq = grid[bq[:, 2], bq[:, 1], bq[:, 0]]
        with np.errstate(divide="ignore", invalid="ignore"):
            ratio = np.where(sq > 0, sigma / sq, 0.0)
        margin[act] = np.minimum(margin[act], np.abs(u[:, 1] - ratio))
        real = u[:, 1] < ratio
        ri = np.nonzero(real)[0]
        if ri.size:
            thr[ri] *= alb[ri]
            T = _shadow(volume, dims, tf, params, q[ri], ldir, pid[act[ri]], e[ri], pp.seed, grid, margin,
                        act[ri])
            L[act[ri]] += thr[ri] * (L_l[None, :] * (T / (4.0 * math.pi))[:, None])
            bounce[ri] += 1
            z = 1.0 - 2.0 * u[ri, 2]
            rr = np.sqrt(np.maximum(0.0, 1.0 - z * z))
            phi = 2.0 * math.pi * u[ri, 3]
            w[ri] = np.stack([rr * np.cos(phi), rr * np.sin(phi), z], axis=1)
        x = q
        e = e + 1
        done = real & (bounce >= B)
        act, x, w, thr, e, bounce = (a[~done] for a in (act, x, w, thr, e, bounce))
    return L, margin


def _shadow(volume, dims, tf, params, y0, l, pid, e, seed, grid, margin, rays):
    """Ratio-tracking transmittance from y0 along l to the box exit, under the
    block majorants."""
    dims = tuple(int(v) for v in dims)
    h = 1.0 / max(dims)
    n = y0.shape[0]
    T = np.ones(n)
    y = y0.copy()
    lv = np.broadcast_to(l, y0.shape)
    idx = np.arange(n)
    k = 0
    while idx.size:
        u = _draw(pid[idx], e[idx], 1, np.full(idx.size, k), seed)[:, 0]
        t, fm = _flight(y[idx], lv[idx], -np.log(u), grid, dims, h)
        margin[rays[idx]] = np.minimum(margin[rays[idx]], fm)
        out = ~np.isfinite(t)
        idx = idx[~out]
        t = t[~out]
        if not idx.size:
            break
        y[idx] = y[idx] + t[:, None] * l[None, :]
        sigma, _ = _medium(volume, dims, tf, params, y[idx])
        b = _block_of(y[idx], dims, h)
        sb = grid[b[:, 2], b[:, 1], b[:, 0]]
        with np.errstate(divide="ignore", invalid="ignore"):
            T[idx] *= np.where(sb > 0, 1.0 - sigma / sb, 1.0)
        k += 1
    return T


def render_path(volume, dims, tf, params: RenderParams, pp: PathParams, cam, px=None, py=None):
    """Pixel radiance (R,3) averaged over spp paths, and the per-pixel decision margin (R,)."""
    if px is None:
        py_, px_ = np.mgrid[0:cam.height, 0:cam.width]
        px, py = px_.ravel(), py_.ravel()
    px = np.asarray(px)
    py = np.asarray(py)
    R = px.size
    spp = int(pp.spp)
    o, d = camera_rays(cam, px, py)
    pix = (py.astype(np.int64) * cam.width + px).astype(np.int64)
    pid = (pix[:, None] * spp + np.arange(spp)[None, :]).ravel()
    L, mg = trace_paths(volume, dims, tf, params, pp, np.repeat(o, spp, axis=0), np.repeat(d, spp, axis=0), pid)
    return L.reshape(R, spp, 3).mean(axis=1), mg.reshape(R, spp).min(axis=1)
