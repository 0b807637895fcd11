"""CPU pins of the path-tracing oracle (reading C22 in oracle/path.py; the paper's
data-parallel path tracing with ray forwarding, sections 2.2 and 5.2, Fig. 7).

The generator is pinned to the known-answer values published with Philox4x32-10
(Salmon et al., SC 2011); the estimator to closed forms: an exact white furnace,
a vacuum, the single-scattering expectation of a homogeneous cube, and the
unbiasedness of delta and ratio tracking (E[T] = exp(-integral of sigma)) in a
heterogeneous medium."""

import math

import numpy as np
import pytest

import oracle
from oracle import PathParams, RenderParams
from oracle.path import _block_of, _medium, _shadow, block_majorants, trace_paths
from oracle.rng import philox4x32, uniforms
from synth import Camera


def test_philox_known_answers():
    cases = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
              (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in cases:
        got = philox4x32(np.array(ctr), np.array(key))
        assert tuple(int(v) for v in got) == want


def test_uniforms_exact_in_fp32_and_open_interval():
    w = np.array([0, 511, 512, 0xFFFFFFFF, 0x80000000], dtype=np.uint64)
    u = uniforms(w)
    assert np.all((u > 0) & (u < 1))
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    assert u[0] == u[1] == 2.0 ** -24 and u[2] == 3 * 2.0 ** -24 and u[3] == 1.0 - 2.0 ** -24
    assert u[4] == 0.5 + 2.0 ** -24
    # many counters: mean and variance of U(0,1)
    ctr = np.stack([np.arange(1 << 16), np.zeros(1 << 16), np.zeros(1 << 16), np.zeros(1 << 16)], axis=1)
    x = uniforms(philox4x32(ctr, np.tile([7, 11], (1 << 16, 1)))).ravel()
    assert abs(x.mean() - 0.5) < 0.005 and abs(x.var() - 1 / 12) < 0.002


def _cube(n=16, value=0.5):
    dims = (n, n, n)
    return dims, np.full((n, n, n), value)


def _tf(rgb, alpha, n=256):
    tf = np.empty((n, 4))
    tf[:, :3] = rgb
    tf[:, 3] = alpha
    return tf


def _axis_paths(dims, n, y=0.5, z=0.5):
    """n paths along +x through the box from x = -1 at height (y, z) (world units of the box)."""
    h = 1.0 / max(dims)
    o = np.tile([-1.0, y * dims[1] * h, z * dims[2] * h], (n, 1))
    d = np.tile([1.0, 0.0, 0.0], (n, 1))
    return o, d, np.arange(n, dtype=np.int64)


def test_white_furnace_is_exact():
    """Albedo 1, no light, uniform environment: every path that leaves carries
    throughput 1, so every pixel is exactly L_e whatever the density."""
    dims, vol = _cube()
    vol = vol + 0.3 * np.random.default_rng(1).random(vol.shape)
    tf = _tf((1.0, 1.0, 1.0), 0.0)
    tf[:, 3] = np.linspace(0.2, 1.0, 256)
    pp = PathParams(light_rgb=(0.0, 0.0, 0.0), env_rgb=(0.3, 0.5, 0.7), max_bounces=10000, spp=4, seed=3)
    cam = Camera((1.8, 1.5, 1.2), (0.5, 0.5, 0.5), (0.0, 0.0, 1.0), 50.0, 12, 10)
    L, _ = oracle.render_path(vol, dims, tf, RenderParams(0.5, 1.0, 30.0), pp, cam)
    assert np.array_equal(L, np.tile([0.3, 0.5, 0.7], (L.shape[0], 1)))


def test_vacuum_and_zero_majorant_see_the_environment():
    dims, vol = _cube()
    pp = PathParams(env_rgb=(0.25, 0.5, 0.75), spp=2)
    cam = Camera((1.8, 1.5, 1.2), (0.5, 0.5, 0.5), (0.0, 0.0, 1.0), 50.0, 8, 6)
    for tf, D in ((_tf((0.5, 0.5, 0.5), 0.0), 30.0), (_tf((0.5, 0.5, 0.5), 0.7), 0.0)):
        with np.errstate(divide="ignore"):
            L, _ = oracle.render_path(vol, dims, tf, RenderParams(0.5, 1.0, D), pp, cam)
        assert np.array_equal(L, np.tile([0.25, 0.5, 0.75], (L.shape[0], 1)))


def test_single_scattering_expectation_of_a_homogeneous_cube():
    """Ray along +x through the unit cube at y = 1/4, z = 1/2, light travelling
    along +y, one bounce: E[L] = (1 - e^{-s}) a L_l e^{-s/4} / (4 pi) + e^{-s} L_e
    with s = sigma (the chord is 1; every shadow path runs 1/4 back towards y = 0)."""
    dims, vol = _cube()
    alb = np.array([0.9, 0.6, 0.3])
    tf = _tf(alb, 0.5)
    D = 2.4
    sigma = D * 0.5
    pp = PathParams(light_dir=(0.0, 1.0, 0.0), light_rgb=(4.0, 4.0, 4.0), env_rgb=(0.2, 0.1, 0.05),
                    max_bounces=1, seed=9)
    n = 200_000
    o, d, pid = _axis_paths(dims, n, y=0.25)
    L, _ = trace_paths(vol, dims, tf, RenderParams(0.5, 1.0, D), pp, o, d, pid)
    want = (1 - math.exp(-sigma)) * alb * 4.0 * math.exp(-sigma / 4) / (4 * math.pi) \
        + math.exp(-sigma) * np.array(pp.env_rgb)
    se = L.std(axis=0) / math.sqrt(n)
    assert np.all(np.abs(L.mean(axis=0) - want) < 4 * se), (L.mean(axis=0), want, se)


def _fibonacci_sphere(n):
    i = np.arange(n) + 0.5
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(1.0 - z * z)
    phi = math.pi * (3.0 - math.sqrt(5.0)) * i
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def test_two_bounce_escape_expectation():
    """Homogeneous cube, albedo c, no light, two bounces, ray along +x at y = 1/2,
    z = 1/4: a path sees L_e if it leaves unscattered, c L_e if it leaves after one
    real collision, nothing after two.  E[L] = L_e (e^{-s} + c P1) with
    P1 = int_0^1 s e^{-s t} <e^{-s d(x(t), w)}>_w dt, evaluated here by quadrature
    over t and a Fibonacci sphere of directions."""
    dims, vol = _cube()
    c = 0.35
    tf = _tf((c, c, c), 0.5)
    D = 3.0
    s = D * 0.5
    pp = PathParams(light_rgb=(0.0, 0.0, 0.0), env_rgb=(1.0, 1.0, 1.0), max_bounces=2, seed=13)
    n = 200_000
    o, d, pid = _axis_paths(dims, n, y=0.5, z=0.25)
    L, _ = trace_paths(vol, dims, tf, RenderParams(0.5, 1.0, D), pp, o, d, pid)
    tg, wg = np.polynomial.legendre.leggauss(48)
    tt = 0.5 * (tg + 1.0)
    w = _fibonacci_sphere(20000)
    P1 = 0.0
    for t, wt in zip(tt, 0.5 * wg):
        x = np.array([t, 0.5, 0.25])
        with np.errstate(divide="ignore"):
            dist = np.min(np.where(w > 0, (1.0 - x) / w, np.where(w < 0, -x / w, np.inf)), axis=1)
        P1 += wt * s * math.exp(-s * t) * np.mean(np.exp(-s * dist))
    want = math.exp(-s) + c * P1
    se = L[:, 0].std() / math.sqrt(n)
    assert abs(L[:, 0].mean() - want) < 4 * se, (L[:, 0].mean(), want, se)


def _ramp_medium(n=32):
    """v = x / (n - 1) at voxel x; TF opacity A(v) = v: sigma = D v, linear in x."""
    dims = (n, 8, 8)
    x = np.arange(n, dtype=np.float64) / (n - 1)
    vol = np.broadcast_to(x, (8, 8, n)).copy()
    tf = _tf((1.0, 1.0, 1.0), 0.0)
    tf[:, 3] = np.linspace(0.0, 1.0, 256)
    return dims, vol, tf


def _optical_depth_along_x(dims, D, x0_world, x1_world):
    """Integral of D v(x) over world x in [x0, x1]; v = (x/h - 1/2)/(n-1), clamped to [0, 1]."""
    h = 1.0 / max(dims)
    n = dims[0]
    xs = np.linspace(x0_world, x1_world, 200001)
    g = np.clip(xs / h - 0.5, 0.0, n - 1.0)
    v = g / (n - 1)
    return D * np.trapezoid(v, xs)


def test_delta_tracking_transmittance_is_unbiased():
    """No light, one bounce: a path sees L_e exactly when its delta-tracked flight
    leaves the box, so E[L] = L_e exp(-tau) along the camera ray."""
    dims, vol, tf = _ramp_medium()
    D = 3.0
    pp = PathParams(light_rgb=(0.0, 0.0, 0.0), env_rgb=(1.0, 1.0, 1.0), max_bounces=1, seed=21)
    n = 100_000
    o, d, pid = _axis_paths(dims, n)
    L, _ = trace_paths(vol, dims, tf, RenderParams(0.5, 1.0, D), pp, o, d, pid)
    h = 1.0 / max(dims)
    want = math.exp(-_optical_depth_along_x(dims, D, 0.0, dims[0] * h))
    p = L[:, 0].mean()
    se = math.sqrt(want * (1 - want) / n)
    assert abs(p - want) < 4 * se, (p, want, se)


def test_ratio_tracking_transmittance_is_unbiased():
    dims, vol, tf = _ramp_medium()
    D = 3.0
    h = 1.0 / max(dims)
    box_hi = np.array(dims, dtype=np.float64) * h
    n = 100_000
    x0 = 0.1 * dims[0] * h
    y0 = np.tile([x0, 4 * h, 4 * h], (n, 1))
    l = np.array([1.0, 0.0, 0.0])
    prm = RenderParams(0.5, 1.0, D)
    margin = np.full(n, np.inf)
    T = _shadow(vol, dims, tf, prm, y0, l, np.arange(n), np.zeros(n, dtype=np.int64), 5,
                block_majorants(vol, dims, tf, prm), margin, np.arange(n))
    want = math.exp(-_optical_depth_along_x(dims, D, x0, dims[0] * h))
    se = T.std() / math.sqrt(n)
    assert abs(T.mean() - want) < 4 * se, (T.mean(), want, se)
    assert np.all((T >= 0) & (T <= 1))


def test_block_majorants_bound_sigma():
    """Every point's extinction lies under its block's majorant, and a block of
    majorant 0 is exactly transparent (the apron of C13 covers the trilinear
    support of every point whose cell is in the block)."""
    dims = (40, 36, 30)
    z, y, x = np.mgrid[0:30, 0:36, 0:40]
    vol = np.exp(-((x - 8.0) ** 2 + (y - 9.0) ** 2 + (z - 7.0) ** 2) / 60.0)
    vol = vol + 0.05 * np.random.default_rng(3).random(vol.shape)
    tf = _tf((1.0, 1.0, 1.0), 0.0)
    tf[:, 3] = np.where(np.arange(256) > 150, np.linspace(0.0, 1.0, 256), 0.0)
    prm = RenderParams(0.5, 1.0, 7.0)
    grid = block_majorants(vol, dims, tf, prm)
    assert grid.shape == (2, 3, 3) and np.any(grid == 0.0) and np.any(grid > 0.0)
    h = 1.0 / max(dims)
    q = np.random.default_rng(4).random((50000, 3)) * np.array(dims) * h
    sigma, _ = _medium(vol, dims, tf, prm, q)
    b = _block_of(q, dims, h)
    sb = grid[b[:, 2], b[:, 1], b[:, 0]]
    assert np.all(sigma <= sb * (1 + 1e-12)) and np.all(sigma[sb == 0.0] == 0.0)


def test_paths_are_reproducible_and_keyed_by_pixel():
    """The same pixel gives the same paths whether rendered alone or in a full
    image (path ids are global), and another seed gives other paths."""
    dims, vol = _cube(12)
    vol = vol * np.random.default_rng(4).random(vol.shape)
    tf = _tf((0.8, 0.7, 0.6), 0.0)
    tf[:, 3] = np.linspace(0.0, 0.9, 256)
    cam = Camera((1.8, 1.5, 1.2), (0.5, 0.5, 0.5), (0.0, 0.0, 1.0), 50.0, 9, 7)
    prm = RenderParams(0.5, 1.0, 25.0)
    pp = PathParams(max_bounces=4, spp=3, seed=7)
    full, _ = oracle.render_path(vol, dims, tf, prm, pp, cam)
    sub, _ = oracle.render_path(vol, dims, tf, prm, pp, cam, np.array([4, 0, 8]), np.array([3, 6, 1]))
    assert np.array_equal(sub, full[[3 * 9 + 4, 6 * 9 + 0, 1 * 9 + 8]])
    other, _ = oracle.render_path(vol, dims, tf, prm, PathParams(max_bounces=4, spp=3, seed=8), cam)
    assert not np.array_equal(other, full)
