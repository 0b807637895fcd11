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
* Majorant: one constant sigma_bar = D max_j A_j over the table, so the tentative
  collisions of a path do not depend on how the volume is split into bricks.
* Random numbers: Philox4x32-10 (``rng.py``), key (seed, 0x243F6A88), counter
  (path, event, kind, step).  Path id = (row * width + column) * spp + sample;
  event e counts the tentative collisions of the path; one draw per event gives
  u0 (free flight), u1 (real or null), u2, u3 (new direction).
* Camera ray through the pixel centre (C4), started at its entry t_in into the
  volume box; a ray that misses the box sees L_e.
* Delta tracking: from x along w, the tentative point is q = x + t w with
  t = -ln(u0) / sigma_bar.  If t >= the distance to the box exit, the path
  leaves: it adds thr L_e.  Otherwise q is real when u1 < sigma(q) / sigma_bar;
  else null, and the flight goes on from q.
* At the k-th real collision (k = 0, 1, ...): thr *= albedo(q); a shadow ray from
  q towards the light (-l_dir) estimates the transmittance by ratio tracking,
  steps s = -ln(u) / sigma_bar with u from counter (path, e, 1, step), T *=
  1 - sigma / sigma_bar until the accumulated length reaches the box exit; the
  path adds thr L_l T / (4 pi).  After B real collisions the path ends; else it
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
    tf = np.asarray(tf, dtype=np.float64)
    sbar = params.density * float(tf[:, 3].max())
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
        t = -np.log(u[:, 0]) / sbar if sbar > 0 else np.full(act.size, np.inf)
        t_exit = _exit_distance(x, w, box_hi)
        if sbar > 0:
            margin[act] = np.minimum(margin[act], sbar * np.abs(t - t_exit))
        leave = t >= t_exit
        L[act[leave]] += thr[leave] * L_e
        keep = ~leave
        act, x, w, thr, e, bounce, u, t = (a[keep] for a in (act, x, w, thr, e, bounce, u, t))
        if not act.size:
            break
        q = x + t[:, None] * w
        sigma, alb = _medium(volume, dims, tf, params, q)
        ratio = sigma / sbar
        margin[act] = np.minimum(margin[act], np.abs(u[:, 1] - ratio))
        real = u[:, 1] < ratio
        ri = np.nonzero(real)[0]
        if ri.size:
            thr[ri] *= alb[ri]
            T = _shadow(volume, dims, tf, params, q[ri], ldir, pid[act[ri]], e[ri], pp.seed, sbar, box_hi,
                        margin, act[ri])
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


def _shadow(volume, dims, tf, params, y0, l, pid, e, seed, sbar, box_hi, margin, rays):
    """Ratio-tracking transmittance from y0 along l to the box exit."""
    n = y0.shape[0]
    T = np.ones(n)
    s_exit = _exit_distance(y0, np.broadcast_to(l, y0.shape), box_hi)
    s_acc = np.zeros(n)
    y = y0.copy()
    idx = np.arange(n)
    k = 0
    while idx.size:
        u = _draw(pid[idx], e[idx], 1, np.full(idx.size, k), seed)[:, 0]
        s = -np.log(u) / sbar
        s_acc[idx] += s
        margin[rays[idx]] = np.minimum(margin[rays[idx]], sbar * np.abs(s_acc[idx] - s_exit[idx]))
        out = s_acc[idx] >= s_exit[idx]
        idx = idx[~out]
        s = s[~out]
        if not idx.size:
            break
        y[idx] = y[idx] + s[:, None] * l[None, :]
        sigma, _ = _medium(volume, dims, tf, params, y[idx])
        T[idx] *= 1.0 - sigma / sbar
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
