"""CPU pins of the iso-surface oracle (reading C20/C21 in oracle/iso.py; the paper
renders iso-surfaces through the data-parallel pipeline in Fig. 1c, Fig. 3c and
Fig. 4, and section 5.1.2 asks the local render only for colour and depth)."""

import math

import numpy as np
import pytest

import oracle
from oracle import IsoParams, RenderParams
from oracle import brute
from synth import Camera, even_split, extract_brick, kd_split, orbit_camera
from tests.helpers import axis_camera, constant_tf, rand_tf, random_volume


def _ramp(dims, a=0.04, b=0.02):
    """v = b + a * x at voxel (x, y, z): trilinear reproduces it exactly."""
    nx, ny, nz = dims
    x = np.arange(nx, dtype=np.float64)
    return np.broadcast_to(b + a * x, (nz, ny, nx)).astype(np.float64).copy()


def _colour_tf(alpha=0.0, n=256):
    tf = np.empty((n, 4))
    u = np.arange(n) / (n - 1)
    tf[:, 0], tf[:, 1], tf[:, 2] = u, 1.0 - u, 0.25 + 0.5 * u * u
    tf[:, 3] = alpha
    return tf


@pytest.mark.parametrize("az", [30.0, 150.0, 250.0])
def test_linear_field_shading_closed_form(az):
    """A plane v = v_iso of a linear field, transparent volume: every hit pixel is
    albedo(v_iso) (k_a + k_d |d_x|), alpha exactly 1; misses stay empty."""
    dims = (24, 20, 16)
    vol = _ramp(dims)
    tf = _colour_tf()
    iso = IsoParams(0.02 + 0.04 * 11.3, ambient=0.3, diffuse=0.6)
    prm = RenderParams(0.5, 1.0, 20.0)
    cam = orbit_camera(dims, 40, 32, az_deg=az, el_deg=15.0, dist=1.6)
    rgba, depth, _, _ = oracle.render_image_iso(vol, dims, tf, prm, iso, cam)
    o, d = oracle.camera_rays(cam, *[a.ravel() for a in np.meshgrid(np.arange(40), np.arange(32))])
    alb = oracle.tf_lookup(tf, np.array([iso.value]), 0.0, 1.0)[0, :3]
    want = alb[None, :] * (iso.ambient + iso.diffuse * np.abs(d[:, 0]))[:, None]
    surf = rgba[:, 3] == 1.0
    assert np.all((rgba[:, 3] == 0.0) | surf)
    assert np.max(np.abs(rgba[surf, :3] - want[surf])) <= 1e-12
    assert np.all(rgba[~surf, :3] == 0.0)
    # geometry: rays meeting the plane well inside the box hit; rays missing it by a voxel do not
    h = 1.0 / max(dims)
    xp = (11.3 + 0.5) * h
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (xp - o[:, 0]) / d[:, 0]
    q = o + t[:, None] * d
    ext = np.array(dims) * h
    inner = (t > 0) & np.all((q[:, 1:] > h) & (q[:, 1:] < ext[1:] - h), axis=1)
    outer = ~((t > 0) & np.all((q[:, 1:] > -h) & (q[:, 1:] < ext[1:] + h), axis=1))
    assert inner.sum() > 40 and np.all(surf[inner]) and not np.any(surf[outer])
    assert np.all(np.isfinite(depth[surf]))


@pytest.mark.parametrize("step", [0.5, 0.37, 1.0])
def test_volume_in_front_of_the_surface_closed_form(step):
    """Constant-opacity volume in front of the plane, axis ray along +x: T is
    exp(-D A L) over the processed length L up to the hit pair's lattice point and
    C = (1 - T) rgb + T rgb (k_a + k_d), alpha = 1."""
    dims = (24, 20, 16)
    vol = _ramp(dims)
    D = 4.0
    tf = constant_tf((0.2, 0.5, 0.8), 0.3).astype(np.float64)
    rgb, A = tf[0, :3], tf[0, 3]
    v_iso = 0.02 + 0.04 * 13.7
    iso = IsoParams(v_iso, ambient=0.2, diffuse=0.7)
    prm = RenderParams(step, 1.0, D)
    cam = axis_camera(dims, axis=0, sign=1.0, size=1)
    rgba, depth, ns, _ = oracle.render_image_iso(vol, dims, tf, prm, iso, cam)
    # the lattice worked out by hand: ray x(t) = e_x + t, entry at x = 0
    h = 1.0 / max(dims)
    dt = step * h
    e_x = cam.eye[0]
    t_in = -e_x
    sa = math.floor(t_in / dt)
    if min((sa + 1) * dt, 1e9) - max(sa * dt, t_in) <= 0:
        sa += 1

    def v(s):
        g = (e_x + (s + 0.5) * dt) / h - 0.5
        return 0.02 + 0.04 * min(max(g, 0.0), dims[0] - 1.0)

    s = sa + 1
    while v(s) < v_iso:
        s += 1
    assert v(s - 1) < v_iso
    L = s * dt - t_in
    T = math.exp(-D * A * L)
    want = (1.0 - T) * rgb + T * rgb * (iso.ambient + iso.diffuse)
    assert np.max(np.abs(rgba[0, :3] - want)) <= 1e-12
    assert rgba[0, 3] == 1.0 and depth[0] == pytest.approx(t_in, abs=1e-15)
    assert ns[0] == s - sa + 1


def test_hit_point_converges_second_order():
    """v = x y / 31^2 (trilinear-exact, curved level sets): the shaded colour at the
    interpolated hit point converges to the colour at the exact root of the ray's
    quadratic at second order in the step."""
    dims = (32, 32, 8)
    nx, ny, nz = dims
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    vol = np.broadcast_to(x * y / 961.0, (nz, ny, nx)).copy()
    tf = _colour_tf()
    iso = IsoParams(0.3, ambient=0.2, diffuse=0.8)
    cam = Camera((0.2, 0.1, 0.9), (0.7, 0.75, 0.05), (0.0, 0.0, 1.0), 40.0, 24, 24)
    px, py = [a.ravel() for a in np.meshgrid(np.arange(24), np.arange(24))]
    o, d = oracle.camera_rays(cam, px, py)
    h = 1.0 / max(dims)
    # exact first crossing inside the box: a t^2 + b t + c = 0 in voxel coordinates
    g0 = o / h - 0.5
    u = d / h
    qa = u[:, 0] * u[:, 1]
    qb = g0[:, 0] * u[:, 1] + g0[:, 1] * u[:, 0]
    qc = g0[:, 0] * g0[:, 1] - 961.0 * iso.value
    t_in, t_out, hit = oracle.clip_box(o, d, np.zeros(3), np.array(dims) * h)
    root = np.full(o.shape[0], np.nan)
    for i in range(o.shape[0]):
        if not hit[i]:
            continue
        r = np.roots([qa[i], qb[i], qc[i]])
        r = np.sort(r[np.isreal(r)].real)
        r = r[(r > t_in[i] + 0.1 * h) & (r < t_out[i] - 0.1 * h)]
        if r.size:
            root[i] = r[0]
    ok = np.isfinite(root)
    gh = g0 + root[:, None] * u
    n = np.stack([gh[:, 1], gh[:, 0], np.zeros_like(root)], axis=1)
    cosv = np.abs(np.sum(n * d, axis=1)) / np.linalg.norm(n, axis=1)
    alb = oracle.tf_lookup(tf, np.array([iso.value]), 0.0, 1.0)[0, :3]
    exact = alb[None, :] * (iso.ambient + iso.diffuse * cosv)[:, None]
    errs = []
    for step in (0.4, 0.2, 0.1, 0.05):
        rgba, _, _, _ = oracle.render_brick_iso(vol, (0, 0, 0), dims, (0, 0, 0), dims, tf,
                                                RenderParams(step, 1.0, 1.0), iso, cam, px, py)
        assert np.all(rgba[ok, 3] == 1.0)
        errs.append(np.sqrt(np.mean((rgba[ok, :3] - exact[ok]) ** 2)))
    assert ok.sum() > 100
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.0 < r < 5.5 for r in ratios), (errs, ratios)


@pytest.mark.parametrize("seed,ert", [(3, 1.0), (4, 0.9), (5, 1.0)])
def test_brute_force_matches_vectorised(seed, ert):
    dims = (7, 6, 5)
    vol = random_volume(dims, seed).astype(np.float64)
    tf = rand_tf(seed + 10).astype(np.float64)
    v_iso = float(np.median(vol))
    iso = IsoParams(v_iso, 0.25, 0.75)
    prm = RenderParams(0.45, ert, 12.0)
    cam = orbit_camera(dims, 9, 8, dist=1.3)
    for lo, hi in [((0, 0, 0), dims), ((2, 0, 1), (6, 4, 5))]:
        b = extract_brick(vol, dims, lo, hi, ghost=1)
        rgba, depth, ns, _ = oracle.render_brick_iso(b.data, b.stored_lo, dims, lo, hi, tf, prm, iso, cam)
        n_surf = 0
        for py in range(cam.height):
            for px in range(cam.width):
                r = brute.render_pixel_iso(b.data, b.stored_lo, dims, lo, hi, tf, prm, v_iso, 0.25, 0.75, cam, px, py)
                i = py * cam.width + px
                assert np.max(np.abs(np.array(r[:4]) - rgba[i])) <= 1e-12, (lo, px, py)
                assert abs(r[4] - depth[i]) <= 1e-12 or (math.isinf(r[4]) and math.isinf(depth[i]))
                assert r[5] == ns[i]
                n_surf += r[3] == 1.0
        assert n_surf > 0 or ert < 1.0


def _split_image(vol, dims, boxes, tf, prm, iso, cam):
    rr, zz = [], []
    for lo, hi in boxes:
        b = extract_brick(vol, dims, lo, hi, ghost=1)
        r, z, _, _ = oracle.render_brick_iso(b.data, b.stored_lo, dims, lo, hi, tf, prm, iso, cam)
        rr.append(r)
        zz.append(z)
    return oracle.composite(np.stack(rr), np.stack(zz))


@pytest.mark.parametrize("step", [0.3, 0.5, 1.0])
def test_split_invariant_with_surface(step):
    dims = (14, 11, 9)
    vol = random_volume(dims, 21).astype(np.float64)
    tf = rand_tf(22).astype(np.float64)
    iso = IsoParams(float(np.quantile(vol, 0.7)), 0.3, 0.7)
    prm = RenderParams(step, 1.0, 25.0)
    h = 1.0 / max(dims)
    inside = Camera((7.3 * h, 5.2 * h, 4.4 * h), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 70.0, 12, 10)
    for cam in (orbit_camera(dims, 16, 14, dist=1.3), inside):
        full, fz, _, _ = oracle.render_image_iso(vol, dims, tf, prm, iso, cam)
        assert np.sum(full[:, 3] == 1.0) >= 5
        for boxes in (even_split(dims, (2, 2, 2)), even_split(dims, (1, 2, 3)), kd_split(dims, 7, seed=5, max_ratio=3.0)):
            comp, cz = _split_image(vol, dims, boxes, tf, prm, iso, cam)
            assert np.max(np.abs(comp - full)) <= 1e-12, (step, len(boxes))


def test_eye_inside_tests_the_pair_at_the_entry():
    """With the eye inside the volume t_in = 0 lies on the lattice, so the pair
    (-1, 0) is tested; a field that is above v_iso behind the eye and below it in
    front gives a hit on the first sample."""
    dims = (16, 8, 8)
    vol = _ramp(dims, a=-0.05, b=0.9)          # decreasing in x
    h = 1.0 / max(dims)
    tf = _colour_tf()
    prm = RenderParams(1.0, 1.0, 5.0)
    # eye at g_x = 8.0 looking along +x, one-voxel steps: sample -1 at g_x = 7.5 has
    # v = 0.525 >= 0.52, sample 0 at g_x = 8.5 has 0.475
    cam = Camera(((8.0 + 0.5) * h, 4.0 * h, 4.0 * h), (1.0, 4.0 * h, 4.0 * h), (0.0, 0.0, 1.0), 30.0, 1, 1)
    rgba, depth, ns, _ = oracle.render_image_iso(vol, dims, tf, prm, IsoParams(0.52), cam)
    assert rgba[0, 3] == 1.0 and depth[0] == 0.0 and ns[0] == 1
    r = brute.render_pixel_iso(vol, (0, 0, 0), dims, (0, 0, 0), dims, tf, prm, 0.52, 0.25, 0.75, cam, 0, 0)
    assert np.max(np.abs(np.array(r[:4]) - rgba[0])) <= 1e-12


def test_out_of_range_iso_is_the_volume_render():
    dims = (12, 10, 9)
    vol = random_volume(dims, 31).astype(np.float64)
    tf = rand_tf(32).astype(np.float64)
    prm = RenderParams(0.5, 0.95, 20.0)
    cam = orbit_camera(dims, 11, 9)
    px, py = [a.ravel() for a in np.meshgrid(np.arange(11), np.arange(9))]
    o, d = oracle.camera_rays(cam, px, py)
    a = oracle.march_rays(vol, (0, 0, 0), dims, (0, 0, 0), dims, tf, prm, o, d)
    b = oracle.march_rays_iso(vol, (0, 0, 0), dims, (0, 0, 0), dims, tf, prm, IsoParams(5.0), o, d)
    for x, y in zip(a, b[:3]):
        assert np.array_equal(x, y)


def _fma32(f, dlt, a):
    return (f.astype(np.float64) * dlt.astype(np.float64) + a.astype(np.float64)).astype(np.float32)


def _trilinear32(data, stored_lo, dims, g):
    """FP32 trilinear in the kernel's form fma(f, b - a, a), for the side pin."""
    R = g.shape[0]
    i0 = np.empty((R, 3), dtype=np.int64)
    fr = np.empty((R, 3), dtype=np.float32)
    for a in range(3):
        n = dims[a]
        ga = np.clip(g[:, a], 0.0, n - 1.0)
        ia = np.minimum(np.floor(ga), n - 2).astype(np.int64)
        fr[:, a] = (ga - ia).astype(np.float32)
        i0[:, a] = ia - stored_lo[a]
    x0, y0, z0 = i0[:, 0], i0[:, 1], i0[:, 2]

    def V(dz, dy, dx):
        return data[z0 + dz, y0 + dy, x0 + dx].astype(np.float32)

    def lerp(p, q, f):
        return _fma32(f, (q - p).astype(np.float32), p)

    c00 = lerp(V(0, 0, 0), V(0, 0, 1), fr[:, 0])
    c01 = lerp(V(0, 1, 0), V(0, 1, 1), fr[:, 0])
    c10 = lerp(V(1, 0, 0), V(1, 0, 1), fr[:, 0])
    c11 = lerp(V(1, 1, 0), V(1, 1, 1), fr[:, 0])
    return lerp(lerp(c00, c01, fr[:, 1]), lerp(c10, c11, fr[:, 1]), fr[:, 2])


@pytest.mark.parametrize("mc", [4, 8])
def test_iso_classes_bound_every_sample(mc):
    """A macrocell classed skippable holds only samples on its side of v_iso, for
    FP32 trilinear values; positive majorants pass through unchanged."""
    dims = (40, 36, 30)
    lo, hi = (7, 5, 0), (33, 36, 21)
    vol = random_volume(dims, 41)
    b = extract_brick(vol, dims, lo, hi, ghost=1)
    ranges = oracle.macrocell_ranges(b.data, lo, hi, b.ghost_lo, mc)
    v_iso = 0.9
    cls = oracle.iso_classes(ranges, np.zeros(ranges.shape[:-1], dtype=np.float32), v_iso)
    assert np.any(cls == 0.0) and np.any(cls == -1.0) and np.any(cls == 1.0)
    # positive majorants pass through unchanged, whatever the range
    maj = np.where(np.random.default_rng(3).random(ranges.shape[:-1]) < 0.5, np.float32(0.25), np.float32(0.0))
    cls2 = oracle.iso_classes(ranges, maj, v_iso)
    assert np.all(cls2[maj > 0] == np.float32(0.25)) and np.array_equal(cls2[maj == 0], cls[maj == 0])
    Mx, My, Mz = oracle.macrocell_grid(lo, hi, mc)
    rng = np.random.default_rng(0)
    c = np.array(lo) - 0.49 + rng.random((40000, 3)) * (np.array(hi) - np.array(lo) + 0.98)
    v = _trilinear32(b.data, b.stored_lo, dims, c - 0.5)
    m = np.clip(((np.floor(c) - np.array(lo)) // mc).astype(int), 0, np.array([Mx, My, Mz]) - 1)
    k = cls[m[:, 2], m[:, 1], m[:, 0]]
    assert np.all(v[k == 0.0] < np.float32(v_iso)) and np.all(v[k == -1.0] >= np.float32(v_iso))
    # a range touching v_iso within the margin must be sampled
    r = np.array([[0.2, v_iso], [v_iso, 0.9], [0.2, np.nextafter(np.float32(v_iso), np.float32(0))]], dtype=np.float32)
    got = oracle.iso_classes(r, np.zeros(3, dtype=np.float32), v_iso)
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0
