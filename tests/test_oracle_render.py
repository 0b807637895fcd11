"""Pins of the FP64 local-render oracle against closed forms, quadrature and brute force."""

import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import RenderParams
from oracle import brute
from synth import Camera, extract_brick, make_blobs, make_tf, make_volume_small, orbit_camera
from tests.helpers import axis_camera, constant_tf, diag_camera, linear_alpha_tf, random_volume, rand_tf


# ----------------------------------------------------------------- rays and clipping
def test_camera_basis_orthonormal_and_centre_ray():
    cam = Camera((3.0, -2.0, 1.5), (0.5, 0.4, 0.3), (0.0, 0.0, 1.0), 60.0, 9, 7)
    f, r, u = oracle.camera_basis(cam)
    M = np.stack([f, r, u])
    assert np.allclose(M @ M.T, np.eye(3), atol=1e-15)
    assert np.allclose(np.cross(r, f), u)
    o, d = oracle.camera_rays(cam, [4], [3])          # centre pixel of an odd image
    assert np.allclose(d[0], f, atol=1e-15)
    o, d = oracle.camera_rays(cam, np.arange(9), np.zeros(9))
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0)
    # row 0 is the top: its rays lean along +up; column 0 leans along -right
    assert np.all(d @ u > 0)
    assert d[0] @ r < 0 < d[-1] @ r


def test_pixel_angles_match_fov():
    cam = Camera((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0), 90.0, 4, 2)
    # fovy 90: pixel-centre tangent = (1 - 2(py+.5)/H) * 1 ; for H=2 rows at +-0.5
    o, d = oracle.camera_rays(cam, [0, 3], [0, 1])
    # x-offsets (2(px+.5)/W - 1) * aspect = (-0.75, 0.75) * 2
    assert np.allclose(d[0] / d[0][0], [1.0, 1.5, 0.5])
    assert np.allclose(d[1] / d[1][0], [1.0, -1.5, -0.5])


def test_clip_axis_aligned_and_degenerate():
    lo, hi = np.zeros(3), np.ones(3)
    o = np.array([[-1.0, 0.5, 0.5], [0.5, 0.5, 0.5], [-1.0, 2.0, 0.5], [-1.0, 1.0, 0.5], [2.0, 0.5, 0.5]])
    d = np.array([[1.0, 0, 0], [0, 0, 1.0], [1.0, 0, 0], [1.0, 0, 0], [1.0, 0, 0]])
    t_in, t_out, hit = oracle.clip_box(o, d, lo, hi)
    assert hit[0] and t_in[0] == 1.0 and t_out[0] == 2.0
    assert hit[1] and t_in[1] == 0.0 and t_out[1] == 0.5      # origin inside: t_in clamps to 0
    assert not hit[2]                                           # parallel, outside the slab
    assert hit[3] and t_out[3] - t_in[3] == 1.0                 # on the face plane: inside closed slab
    assert not hit[4]                                           # box behind the origin


def test_clip_grazing_edge_is_miss():
    # touches the cube only along the edge x = y = 0: zero-length chord is a miss
    o = np.array([[-1.0, 1.0, 0.5]])
    d = np.array([[1.0, -1.0, 0.0]]) / math.sqrt(2.0)
    _, _, hit = oracle.clip_box(o, d, np.zeros(3), np.ones(3))
    assert not hit[0]


# ----------------------------------------------------------------- trilinear and TF
def test_trilinear_reproduces_voxels_and_affine_fields():
    dims = (5, 6, 7)
    rng = np.random.default_rng(1)
    vol = rng.random((7, 6, 5))
    kk, jj, ii = np.meshgrid(range(7), range(6), range(5), indexing="ij")
    g = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(float)
    assert np.allclose(oracle.trilinear(vol, (0, 0, 0), dims, g), vol.ravel(), atol=1e-15)
    a = np.array([0.3, -1.2, 0.7])
    aff = (0.1 + a[0] * ii + a[1] * jj + a[2] * kk).astype(float)
    p = rng.random((200, 3)) * (np.array(dims) - 1)
    assert np.allclose(oracle.trilinear(aff, (0, 0, 0), dims, p), 0.1 + p @ a, atol=1e-12)
    # clamp-to-edge outside the voxel-centre range
    q = np.array([[-3.0, 2.0, 3.0], [4.0 + 9.0, 2.0, 3.0]])
    qc = np.array([[0.0, 2.0, 3.0], [4.0, 2.0, 3.0]])
    assert np.allclose(oracle.trilinear(aff, (0, 0, 0), dims, q), 0.1 + qc @ a)


def test_trilinear_asserts_outside_stored_brick():
    vol = np.zeros((4, 4, 4))
    with pytest.raises(AssertionError):
        oracle.trilinear(vol, (2, 0, 0), (8, 4, 4), np.array([[1.2, 1.0, 1.0]]))


def test_tf_lookup_exact_at_entries_and_clamped():
    tf = rand_tf(7)
    n = tf.shape[0]
    v = np.arange(n) / (n - 1)
    assert np.allclose(oracle.tf_lookup(tf, v, 0.0, 1.0), tf.astype(np.float64), atol=1e-13)
    out = oracle.tf_lookup(tf, np.array([-0.5, 1.5]), 0.0, 1.0)
    assert np.array_equal(out[0], tf[0].astype(np.float64)) and np.array_equal(out[1], tf[-1].astype(np.float64))
    # value range mapping: entry i at lo + i (hi - lo)/(N-1)
    v2 = 2.0 + 3.0 * v
    assert np.allclose(oracle.tf_lookup(tf, v2, 2.0, 5.0), tf.astype(np.float64), atol=1e-12)


# ----------------------------------------------------------------- closed forms (P-c1, P-c3)
@pytest.mark.parametrize("step", [0.5, 0.37, 1.0, 0.125])
@pytest.mark.parametrize("cam_kind", ["axis", "diag"])
def test_constant_volume_closed_form(step, cam_kind):
    """Constant field: alpha = 1 - exp(-D A L) and C = c alpha for any step and split."""
    dims = (8, 8, 8)
    vol = np.full((8, 8, 8), 0.5, dtype=np.float32)
    rgb, A, D = np.array([0.2, 0.5, 0.9]), 0.7, 3.0
    tf = constant_tf(rgb, A)
    prm = RenderParams(step_voxels=step, ert=1.0, density=D)
    cam = axis_camera(dims) if cam_kind == "axis" else diag_camera(dims)
    L = 1.0 if cam_kind == "axis" else math.sqrt(3.0)   # chord of the unit cube through its centre
    rgba, depth, _ = oracle.render_image(vol, dims, tf, prm, cam, [4], [4])
    alpha = 1.0 - math.exp(-D * float(np.float32(A)) * L)
    assert abs(rgba[0, 3] - alpha) < 1e-13
    assert np.allclose(rgba[0, :3], rgb.astype(np.float32).astype(np.float64) * alpha, atol=1e-13)
    assert abs(depth[0] - (2.5 - L / 2)) < 1e-13


def test_constant_colour_gives_c_times_alpha():
    dims = (8, 8, 8)
    vol = random_volume(dims, 3)
    tf = rand_tf(11).astype(np.float64)
    tf[:, :3] = (0.25, 0.5, 0.75)
    prm = RenderParams(step_voxels=0.5, ert=1.0, density=12.0)
    cam = orbit_camera(dims, 6, 6)
    rgba, _, _ = oracle.render_image(vol, dims, tf, prm, cam)
    assert rgba[..., 3].max() > 0.1
    assert np.allclose(rgba[..., :3], rgba[..., 3:4] * np.array([0.25, 0.5, 0.75]), atol=1e-14)


# ----------------------------------------------------------------- quadrature convergence (P-c2)
def _affine_optical_depth(o, d, t0, t1, h, n, D):
    """Integral of D * A(v) along the ray for v = x (world), A(u) = u, with clamp-to-edge."""
    def sigma(t):
        x = o[0] + t * d[0]
        return D * min(max(x, 0.5 * h), (n - 0.5) * h)
    kinks = sorted(t for t in ((0.5 * h - o[0]) / d[0], ((n - 0.5) * h - o[0]) / d[0]) if t0 < t < t1)
    pts = [t0] + kinks + [t1]
    return sum(integrate.quad(sigma, a, b, epsabs=1e-14, epsrel=1e-14)[0] for a, b in zip(pts[:-1], pts[1:]))


def _affine_setup():
    n = 16
    dims = (n, n, n)
    h = 1.0 / n
    ii = np.arange(n)
    vol = np.broadcast_to(((ii + 0.5) * h)[None, None, :], (n, n, n)).astype(np.float64)
    return n, dims, h, vol, linear_alpha_tf(), 4.0


def test_affine_field_axis_ray_is_exact():
    """Every kink of the clamped affine field and both faces sit on lattice points,
    and the midpoint rule is exact on each linear piece."""
    n, dims, h, vol, tf, D = _affine_setup()
    cam = axis_camera(dims, size=9)
    o, d = oracle.camera_rays(cam, [4], [4])
    t0, t1, _ = oracle.clip_box(o, d, np.zeros(3), np.ones(3))
    exact = math.exp(-_affine_optical_depth(o[0], d[0], t0[0], t1[0], h, n, D))
    for step in (0.5, 0.25, 0.125):
        rgba, _, _ = oracle.render_image(vol, dims, tf, RenderParams(step, 1.0, D), cam, [4], [4])
        assert abs((1.0 - rgba[0, 3]) - exact) < 1e-14


def test_affine_field_oblique_rays_converge_second_order():
    """Oblique rays: kinks fall between lattice points, so the quadrature error is
    O(dt^2); the RMS error over 49 rays shrinks ~4x per halving of the step."""
    n, dims, h, vol, tf, D = _affine_setup()
    cam = Camera((-1.3, 0.21, 0.33), (0.5, 0.5, 0.5), (0.0, 0.0, 1.0), 30.0, 7, 7)
    py, px = np.mgrid[0:7, 0:7]
    px, py = px.ravel(), py.ravel()
    o, d = oracle.camera_rays(cam, px, py)
    t0, t1, hit = oracle.clip_box(o, d, np.zeros(3), np.ones(3))
    assert hit.all()
    exact = np.array([math.exp(-_affine_optical_depth(o[i], d[i], t0[i], t1[i], h, n, D))
                      for i in range(px.size)])
    rms = []
    for step in (0.5, 0.25, 0.125, 0.0625):
        rgba, _, _ = oracle.render_image(vol, dims, tf, RenderParams(step, 1.0, D), cam, px, py)
        rms.append(float(np.sqrt(np.mean(((1.0 - rgba[:, 3]) - exact) ** 2))))
    rates = [rms[i] / rms[i + 1] for i in range(len(rms) - 1)]
    assert rms[-1] < 2e-6
    assert all(3.0 < r < 6.0 for r in rates), (rms, rates)
    assert rms[0] / rms[-1] > 40.0        # >= 2nd order over an 8x refinement (1st order: 8)


# ----------------------------------------------------------------- brute force (P-c5)
@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("ert", [1.0, 0.6])
def test_brute_force_matches_vectorised(seed, ert):
    rng = np.random.default_rng(seed)
    dims = tuple(int(v) for v in rng.integers(4, 9, size=3))
    vol = random_volume(dims, 100 + seed)
    tf = rand_tf(200 + seed)
    prm = RenderParams(step_voxels=float(rng.choice([0.5, 0.3, 1.0])), ert=ert, density=25.0)
    cam = Camera(tuple(rng.normal(size=3) * 0.3 + np.array([2.2, -1.6, 1.1])),
                 tuple(np.array(dims) / max(dims) / 2), (0.0, 0.0, 1.0), 50.0, 8, 8)
    # one brick = the whole domain, and one interior brick with ghosts
    rgba, depth, ns = oracle.render_image(vol, dims, tf, prm, cam)
    lo = (1, 0, 1)
    hi = (dims[0] - 1, dims[1], dims[2])
    sub = vol[0:dims[2], 0:dims[1], 0:dims[0]]
    rgba_b, depth_b, _ = oracle.render_brick(sub, (0, 0, 0), dims, lo, hi, tf, prm, cam)
    for py in range(8):
        for px in range(8):
            b = brute.render_pixel(vol, (0, 0, 0), dims, (0, 0, 0), dims, tf, prm, cam, px, py)
            assert np.allclose(rgba[py, px], b[:4], atol=1e-13, rtol=0)
            assert depth[py, px] == b[4] or abs(depth[py, px] - b[4]) < 1e-13
            assert ns[py, px] == b[5]
            bb = brute.render_pixel(sub, (0, 0, 0), dims, lo, hi, tf, prm, cam, px, py)
            assert np.allclose(rgba_b[py, px], bb[:4], atol=1e-13, rtol=0)


def test_ert_monotone_in_threshold():
    dims = (8, 8, 8)
    vol = random_volume(dims, 5)
    tf = rand_tf(9)
    cam = orbit_camera(dims, 8, 8)
    prev = None
    for th in (0.3, 0.6, 0.9, 0.99, 1.0):
        rgba, _, ns = oracle.render_image(vol, dims, tf, RenderParams(0.5, th, 30.0), cam)
        if prev is not None:
            assert np.all(rgba >= prev[0] - 1e-15) and np.all(ns >= prev[1])
        prev = (rgba, ns)


def test_ert_stops_once_threshold_reached():
    dims = (8, 8, 8)
    vol = np.full((8, 8, 8), 1.0, dtype=np.float32)
    tf = constant_tf((1, 1, 1), 1.0)
    prm = RenderParams(0.5, 0.9, 40.0)
    cam = axis_camera(dims)
    rgba, _, ns = oracle.render_image(vol, dims, tf, prm, cam, [4], [4])
    # per full segment a = 1 - exp(-40/16); alpha after k segments = 1 - exp(-2.5 k)
    k = math.ceil(-math.log(0.1) / 2.5)
    assert ns[0] == k
    assert abs(rgba[0, 3] - (1 - math.exp(-2.5 * k))) < 1e-14


def test_thresholds_in_one_march_equal_separate_marches():
    """render_brick_thresholds (one march, several termination thresholds) gives
    exactly what render_brick gives at each threshold alone, on a split brick."""
    dims = (40, 36, 30)
    vol = make_volume_small(dims, make_blobs(dims, 5, 6, (0.08, 0.25)), 6, 0.02)
    tf = make_tf(2001)
    cam = orbit_camera(dims, 48, 40)
    lo, hi = (0, 10, 0), (25, 36, 30)
    b = extract_brick(vol, dims, lo, hi, 1)
    py, px = np.mgrid[0:40, 0:48]
    px, py = px.ravel(), py.ravel()
    thetas = [0.99 - 1e-4, 0.99 + 1e-4, 0.5, 1.0]
    prm = oracle.RenderParams(0.5, 1.0, 30.0)
    res = oracle.render_brick_thresholds(b.data, b.stored_lo, dims, lo, hi, tf, prm, cam, px, py, thetas)
    terminated = 0
    for th, (r, z, n) in zip(thetas, res):
        p = oracle.RenderParams(0.5, th, 30.0)
        r2, z2, n2 = oracle.render_brick(b.data, b.stored_lo, dims, lo, hi, tf, p, cam, px, py)
        assert np.array_equal(r, r2) and np.array_equal(z, z2) and np.array_equal(n, n2)
        terminated += int(np.count_nonzero(r[:, 3] >= th))
    assert terminated > 0
