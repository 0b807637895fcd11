"""Independent brute-force renderer and compositor for tiny inputs (pure Python scalars).

Written separately from ``render.py``/``composite.py`` (no shared helpers) so a
slip in either shows up as a disagreement.  Instead of the running recurrence
it evaluates the emission-absorption sum in its explicit product form,

    C = sum_s c_s a_s prod_{j<s} (1 - a_j),   alpha = 1 - prod_s (1 - a_s),

with a_s = 1 - exp(-D A_s l_s) computed from exp (not expm1), which is O(S^2)
and only meant for grids of a few voxels and images of a few pixels.
Conventions C1-C12 are those listed in ``render.py``.
"""

from __future__ import annotations

import math


def _ray(cam, px, py):
    ex, ey, ez = cam.eye
    fx, fy, fz = (cam.center[0] - ex, cam.center[1] - ey, cam.center[2] - ez)
    n = math.sqrt(fx * fx + fy * fy + fz * fz)
    fx, fy, fz = fx / n, fy / n, fz / n
    ux, uy, uz = cam.up
    rx, ry, rz = fy * uz - fz * uy, fz * ux - fx * uz, fx * uy - fy * ux
    n = math.sqrt(rx * rx + ry * ry + rz * rz)
    rx, ry, rz = rx / n, ry / n, rz / n
    vx, vy, vz = ry * fz - rz * fy, rz * fx - rx * fz, rx * fy - ry * fx
    t = math.tan(math.radians(cam.fovy_deg) * 0.5)
    sx = ((px + 0.5) * 2.0 / cam.width - 1.0) * t * cam.width / cam.height
    sy = (1.0 - (py + 0.5) * 2.0 / cam.height) * t
    dx, dy, dz = fx + sx * rx + sy * vx, fy + sx * ry + sy * vy, fz + sx * rz + sy * vz
    n = math.sqrt(dx * dx + dy * dy + dz * dz)
    return (ex, ey, ez), (dx / n, dy / n, dz / n)


def _clip(o, d, lo, hi):
    tn, tf = -math.inf, math.inf
    for a in range(3):
        if d[a] == 0.0:
            if o[a] < lo[a] or o[a] > hi[a]:
                return None
            continue
        t0 = (lo[a] - o[a]) / d[a]
        t1 = (hi[a] - o[a]) / d[a]
        if t0 > t1:
            t0, t1 = t1, t0
        tn = max(tn, t0)
        tf = min(tf, t1)
    tn = max(tn, 0.0)
    return (tn, tf) if tf > tn else None


def _sample(vol, dims, stored_lo, p, h):
    """Trilinear at world point p from a nested-list or array volume vol[z][y][x]."""
    idx, frac = [], []
    for a in range(3):
        n = dims[a]
        g = min(max(p[a] / h - 0.5, 0.0), n - 1.0)
        i = min(int(math.floor(g)), n - 2)
        idx.append(i - stored_lo[a])
        frac.append(g - i)
    out = 0.0
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = ((frac[0] if dx else 1 - frac[0]) * (frac[1] if dy else 1 - frac[1])
                     * (frac[2] if dz else 1 - frac[2]))
                out += w * float(vol[idx[2] + dz][idx[1] + dy][idx[0] + dx])
    return out


def _tf(tf, v, lo, hi):
    n = len(tf)
    u = (v - lo) / (hi - lo)
    u = 0.0 if u < 0.0 else (1.0 if u > 1.0 else u)
    x = u * (n - 1)
    j = min(int(math.floor(x)), n - 2)
    w = x - j
    return [float(tf[j][c]) * (1 - w) + float(tf[j + 1][c]) * w for c in range(4)]


def render_pixel(vol, stored_lo, dims, owned_lo, owned_hi, tf, params, cam, px, py):
    """(r, g, b, alpha, depth, samples) of one pixel of one brick."""
    h = 1.0 / max(dims)
    dt = params.step_voxels * h
    o, d = _ray(cam, px, py)
    hit = _clip(o, d, [l * h for l in owned_lo], [u * h for u in owned_hi])
    if hit is None:
        return (0.0, 0.0, 0.0, 0.0, math.inf, 0)
    t_in, t_out = hit
    s = int(math.floor(t_in / dt))
    a_list, c_list = [], []
    while s * dt < t_out:
        ell = min((s + 1) * dt, t_out) - max(s * dt, t_in)
        if ell > 0:
            tm = (s + 0.5) * dt
            p = (o[0] + tm * d[0], o[1] + tm * d[1], o[2] + tm * d[2])
            rgba = _tf(tf, _sample(vol, dims, stored_lo, p, h), params.tf_lo, params.tf_hi)
            a_list.append(1.0 - math.exp(-params.density * rgba[3] * ell))
            c_list.append(rgba[:3])
            trans = 1.0
            for a in a_list:
                trans *= 1.0 - a
            if params.ert < 1.0 and 1.0 - trans >= params.ert:
                break
        s += 1
    col = [0.0, 0.0, 0.0]
    for i, (a, c) in enumerate(zip(a_list, c_list)):
        pre = 1.0
        for j in range(i):
            pre *= 1.0 - a_list[j]
        for ch in range(3):
            col[ch] += c[ch] * a * pre
    trans = 1.0
    for a in a_list:
        trans *= 1.0 - a
    return (col[0], col[1], col[2], 1.0 - trans, t_in, len(a_list))


def composite_pixel(frags):
    """frags: list of (rgba4, depth, id).  Front-to-back over after sorting by (depth, id);
    alpha as 1 - prod(1 - alpha_i), the product form of the same quantity."""
    live = sorted([f for f in frags if f[1] != math.inf], key=lambda f: (f[1], f[2]))
    col = [0.0, 0.0, 0.0]
    for i, (rgba, _, _) in enumerate(live):
        pre = 1.0
        for j in range(i):
            pre *= 1.0 - live[j][0][3]
        for ch in range(3):
            col[ch] += pre * rgba[ch]
    trans = 1.0
    for rgba, _, _ in live:
        trans *= 1.0 - rgba[3]
    depth = min([f[1] for f in frags], default=math.inf)
    return (col[0], col[1], col[2], 1.0 - trans, depth)


def _cell(dims, stored_lo, g):
    """Cell corner (stored-relative) and fractions of voxel-centre point g (clamp rule)."""
    idx, frac = [], []
    for a in range(3):
        n = dims[a]
        ga = min(max(g[a], 0.0), n - 1.0)
        i = min(int(math.floor(ga)), n - 2)
        idx.append(i - stored_lo[a])
        frac.append(ga - i)
    return idx, frac


def _patch(vol, idx, frac):
    out = 0.0
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = ((frac[0] if dx else 1 - frac[0]) * (frac[1] if dy else 1 - frac[1])
                     * (frac[2] if dz else 1 - frac[2]))
                out += w * float(vol[idx[2] + dz][idx[1] + dy][idx[0] + dx])
    return out


def render_pixel_iso(vol, stored_lo, dims, owned_lo, owned_hi, tf, params, iso_value, ambient, diffuse, cam,
                     px, py):
    """(r, g, b, alpha, depth, samples) of one pixel of one brick with an opaque
    iso-surface.  The processed samples are listed first; the surface is the first
    change of side between consecutive listed samples (or between the first one and
    the sample half a step before the brick when the first segment starts on the
    brick's entry), and enters the product form as a last layer of opacity 1.  The
    patch gradient is taken as differences of the patch at fractions 1 and 0."""
    h = 1.0 / max(dims)
    dt = params.step_voxels * h
    o, d = _ray(cam, px, py)
    hit = _clip(o, d, [l * h for l in owned_lo], [u * h for u in owned_hi])
    if hit is None:
        return (0.0, 0.0, 0.0, 0.0, math.inf, 0)
    t_in, t_out = hit

    def point(t):
        return [(o[a] + t * d[a]) / h - 0.5 for a in range(3)]

    def value(g):
        idx, frac = _cell(dims, stored_lo, g)
        return _patch(vol, idx, frac)

    samples = []  # (s, ell, v)
    s = int(math.floor(t_in / dt))
    while s * dt < t_out:
        ell = min((s + 1) * dt, t_out) - max(s * dt, t_in)
        if ell > 0:
            samples.append((s, ell, value(point((s + 0.5) * dt))))
        s += 1
    a_list, c_list = [], []
    for i, (s, ell, v) in enumerate(samples):
        if i > 0:
            prev = samples[i - 1][2]
        elif s * dt >= t_in:
            prev = value(point((s - 0.5) * dt))
        else:
            prev = None
        if prev is not None and (v >= iso_value) != (prev >= iso_value):
            f = (iso_value - prev) / (v - prev)
            g0, g1 = point((s - 0.5) * dt), point((s + 0.5) * dt)
            gh = [g0[a] + f * (g1[a] - g0[a]) for a in range(3)]
            idx, frac = _cell(dims, stored_lo, gh)
            grad = []
            for a in range(3):
                f1, f0 = list(frac), list(frac)
                f1[a], f0[a] = 1.0, 0.0
                grad.append(_patch(vol, idx, f1) - _patch(vol, idx, f0))
            norm = math.sqrt(sum(x * x for x in grad))
            cosv = abs(sum(grad[a] * d[a] for a in range(3))) / norm if norm > 0.0 else 1.0
            alb = _tf(tf, iso_value, params.tf_lo, params.tf_hi)
            a_list.append(1.0)
            c_list.append([alb[c] * (ambient + diffuse * cosv) for c in range(3)])
            break
        rgba = _tf(tf, v, params.tf_lo, params.tf_hi)
        a_list.append(1.0 - math.exp(-params.density * rgba[3] * ell))
        c_list.append(rgba[:3])
        trans = 1.0
        for a in a_list:
            trans *= 1.0 - a
        if params.ert < 1.0 and 1.0 - trans >= params.ert:
            break
    col = [0.0, 0.0, 0.0]
    for i, (a, c) in enumerate(zip(a_list, c_list)):
        pre = 1.0
        for j in range(i):
            pre *= 1.0 - a_list[j]
        for ch in range(3):
            col[ch] += c[ch] * a * pre
    trans = 1.0
    for a in a_list:
        trans *= 1.0 - a
    return (col[0], col[1], col[2], 1.0 - trans, t_in, len(a_list))
