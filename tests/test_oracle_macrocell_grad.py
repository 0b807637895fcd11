"""Pins of the macrocell/majorant oracle and of the gradient oracle."""

import math

import numpy as np
import pytest
import torch

import oracle
from oracle import RenderParams
from oracle.macrocell import macrocell_grid
from synth import Camera, extract_brick, orbit_camera
from tests.helpers import axis_camera, constant_tf, random_volume, rand_tf


# ----------------------------------------------------------------- macrocells (P-c8)
def _brick(dims, lo, hi, seed):
    vol = random_volume(dims, seed)
    return vol, extract_brick(vol, dims, lo, hi, ghost=1)


@pytest.mark.parametrize("mc", [16, 4, 3])
def test_macrocell_range_contains_every_sample(mc):
    dims = (40, 36, 30)
    lo, hi = (7, 5, 0), (33, 36, 21)           # interior faces + global faces, partial last cells
    vol, b = _brick(dims, lo, hi, 41)
    rng_ = oracle.macrocell_ranges(b.data, lo, hi, b.ghost_lo, mc)
    Mx, My, Mz = macrocell_grid(lo, hi, mc)
    assert rng_.shape == (Mz, My, Mx, 2)
    rng = np.random.default_rng(0)
    # cell coordinates, with up to half a voxel of overshoot outside the owned box
    c = np.array(lo) - 0.49 + rng.random((20000, 3)) * (np.array(hi) - np.array(lo) + 0.98)
    v = oracle.trilinear(b.data, b.stored_lo, dims, c - 0.5)
    m = np.clip(((np.floor(c) - np.array(lo)) // mc).astype(int), 0, np.array([Mx, My, Mz]) - 1)
    r = rng_[m[:, 2], m[:, 1], m[:, 0]]
    assert np.all(v >= r[:, 0].astype(np.float64) - 1e-12) and np.all(v <= r[:, 1].astype(np.float64) + 1e-12)


def test_macrocell_window_is_one_voxel_apron():
    dims = (64, 20, 20)
    lo, hi = (0, 0, 0), (64, 20, 20)
    base = np.zeros((20, 20, 64), dtype=np.float32)
    for x, seen in ((14, {0}), (15, {0, 1}), (16, {0, 1}), (17, {1}), (47, {2, 3}), (63, {3})):
        vol = base.copy()
        vol[3, 3, x] = 1.0
        r = oracle.macrocell_ranges(vol, lo, hi, (0, 0, 0), 16)
        got = {int(m) for m in np.nonzero(r[0, 0, :, 1] == 1.0)[0]}
        assert got == seen, (x, got)


def test_majorant_zero_means_exactly_transparent():
    tf = rand_tf(51)
    n = tf.shape[0]
    rng = np.random.default_rng(1)
    ranges = np.sort(rng.random((400, 2)).astype(np.float32) * 0.6, axis=1)
    maj = oracle.majorants(ranges, tf)
    for (a, b), mj in zip(ranges, maj):
        vs = np.linspace(float(a), float(b), 257)
        A = oracle.tf_lookup(tf, vs, 0.0, 1.0)[:, 3]
        assert A.max() <= mj + 1e-7
        if mj == 0.0:
            assert np.all(A == 0.0)
    assert np.any(maj == 0.0) and np.any(maj > 0.0)
    # ranges entirely outside [lo, hi] clamp to the end entries
    assert oracle.majorants(np.array([[-5.0, -1.0]], dtype=np.float32), tf)[0] == tf[:2, 3].max()
    assert oracle.majorants(np.array([[2.0, 3.0]], dtype=np.float32), tf)[0] == tf[n - 2:, 3].max()


def _tf_alpha_max(tf, a, b, lo=0.0, hi=1.0):
    """Largest opacity of the piecewise-linear table over values [a, b], by evaluating
    it at both ends and at every table knot between them (the maximum of a
    piecewise-linear function lies at one of those)."""
    n = tf.shape[0]
    knots = lo + np.arange(n) * (hi - lo) / (n - 1)
    vs = np.concatenate([[a, b], knots[(knots > a) & (knots < b)]])
    return float(oracle.tf_lookup(tf, vs, lo, hi)[:, 3].max())


def test_majorant_entry_window_is_one_entry_wide_each_side():
    """The majorant is the largest opacity over the range widened by one table entry
    on each side, neither less nor more: a zero majorant means the table is
    transparent within one entry width of the range, and a positive one means it is
    not transparent within two entry widths."""
    n = 256
    tf = np.zeros((n, 4), dtype=np.float32)
    tf[:, :3] = 0.5
    tf[200:, 3] = np.linspace(0.1, 1.0, n - 200)        # opaque from entry 200 on
    de = 1.0 / (n - 1)
    rng = np.random.default_rng(7)
    # ranges ending at random fractional table coordinates below and around entry 200
    ends = (rng.random(2000) * 8.0 + 194.0) * de
    ranges = np.stack([ends - 5 * de, ends], axis=1).astype(np.float32)
    maj = oracle.majorants(ranges, tf)
    for (a, b), mj in zip(ranges.astype(np.float64), maj):
        if mj == 0.0:
            assert _tf_alpha_max(tf, a - de, b + de) == 0.0, (a, b)
        else:
            assert _tf_alpha_max(tf, a - 2 * de, b + 2 * de) > 0.0, (a, b)
        assert mj >= _tf_alpha_max(tf, a, b)
    assert np.any(maj == 0.0) and np.any(maj > 0.0)
    # an end exactly on entry 198 (x_max = 198): entries up to 199 are transparent
    r = np.array([[0.1, 198 * de]], dtype=np.float32)
    assert float(r[0, 1]) * (n - 1) != 198.0 or oracle.majorants(r, tf)[0] == 0.0


def test_majorant_is_the_fp64_definition():
    """Entry ranges follow the FP64 table coordinate: x_max just above an integer k
    (by 2^-40 of an entry, far below FP32 resolution) reaches entry k + 2.  A
    257-entry table on [0, 1] makes x = 256 v exact."""
    n = 257
    tf = np.zeros((n, 4), dtype=np.float32)
    tf[102, 3] = 0.5
    k = 100.0 / 256.0
    e0, e1 = oracle.entry_range(np.array([[0.0, k]]), n)
    assert e1[0] == 101
    above = np.array([[0.0, k + 2.0 ** -48]])
    e0, e1 = oracle.entry_range(above, n)
    assert e1[0] == 102
    assert oracle.entry_decision_ambiguous(above, n)[0]
    assert not oracle.entry_decision_ambiguous(np.array([[0.0, 100.4 / 256.0]]), n)[0]
    assert oracle.majorants(np.array([[0.0, 100.4 / 256.0]]), tf)[0] == 0.5
    assert oracle.majorants(np.array([[0.0, 99.4 / 256.0]]), tf)[0] == 0.0
    # the lower end: x_min = 104 reaches entry 103, x_min just below 104 reaches 102
    assert oracle.entry_range(np.array([[104.0 / 256.0, 0.5]]), n)[0][0] == 103
    assert oracle.entry_range(np.array([[104.0 / 256.0 - 2.0 ** -48, 0.5]]), n)[0][0] == 102


# ----------------------------------------------------------------- gradients (P-c9)
def _tiny_problem(seed=0):
    dims = (6, 5, 7)
    # keep values strictly inside (lo, hi): the clamp of u is a kink of the loss
    vol = 0.05 + 0.9 * random_volume(dims, 60 + seed).astype(np.float64)
    tf = rand_tf(70 + seed).astype(np.float64)
    tf[:, 3] = np.maximum(tf[:, 3], 0.05)       # keep slopes and opacity away from zero
    cams = [orbit_camera(dims, 5, 4), Camera((-1.2, 2.0, 0.9), (0.5, 0.4, 0.55), (0.0, 0.0, 1.0), 40.0, 4, 5)]
    prm = RenderParams(step_voxels=0.5, ert=1.0, density=9.0)
    tgt = [np.random.default_rng(seed).random((c.height, c.width, 4)) * 0.5 for c in cams]
    return dims, vol, tf, cams, prm, tgt


def _loss(vol, dims, tf, prm, cams, tgt):
    n_el = sum(t.size for t in tgt)
    L = 0.0
    for c, t in zip(cams, tgt):
        img = oracle.forward_image(vol, dims, tf, prm, [c])[0]
        L += np.sum((img - t) ** 2) / n_el
    return L


def _loss_grad(vol, dims, tf, prm, cams, tgt):
    n_el = sum(t.size for t in tgt)
    L, gV, gT = 0.0, np.zeros_like(vol), np.zeros_like(tf)
    for c, t in zip(cams, tgt):
        l, gv, gt, _ = oracle.loss_and_grad(vol, dims, tf, prm, [c], t[None], n_elems=n_el)
        L, gV, gT = L + l, gV + gv, gT + gt
    return L, gV, gT


def test_gradient_matches_central_differences():
    dims, vol, tf, cams, prm, tgt = _tiny_problem()
    L, gV, gT = _loss_grad(vol, dims, tf, prm, cams, tgt)
    assert abs(L - _loss(vol, dims, tf, prm, cams, tgt)) < 1e-15
    rng = np.random.default_rng(3)
    h = 1e-6
    picks = np.argsort(-np.abs(gV).ravel())[:6].tolist() + rng.integers(0, vol.size, 4).tolist()
    for f in picks:
        vp, vm = vol.copy(), vol.copy()
        vp.ravel()[f] += h
        vm.ravel()[f] -= h
        fd = (_loss(vp, dims, tf, prm, cams, tgt) - _loss(vm, dims, tf, prm, cams, tgt)) / (2 * h)
        assert abs(fd - gV.ravel()[f]) <= 1e-6 * max(abs(fd), 1e-6), (f, fd, gV.ravel()[f])
    tpicks = np.argsort(-np.abs(gT).ravel())[:8]
    for f in tpicks:
        tp, tm = tf.copy(), tf.copy()
        tp.ravel()[f] += h
        tm.ravel()[f] -= h
        fd = (_loss(vol, dims, tp, prm, cams, tgt) - _loss(vol, dims, tm, prm, cams, tgt)) / (2 * h)
        assert abs(fd - gT.ravel()[f]) <= 1e-6 * max(abs(fd), 1e-6), (f, fd, gT.ravel()[f])


def _torch_render(vol_t, tf_t, dims, prm, cam, plateau=None):
    """The same quadrature re-expressed with torch FP64 ops, for torch.autograd.  The
    trilinear value is taken as nested lerps a + f (b - a), so a sample whose eight
    corners all hold a clamp bound (0 or 1) sits exactly on it; ``plateau`` (a list)
    collects those sample values."""
    h = 1.0 / max(dims)
    dt = prm.step_voxels * h
    n = tf_t.shape[0]
    py, px = np.mgrid[0:cam.height, 0:cam.width]
    o, d = oracle.camera_rays(cam, px.ravel(), py.ravel())
    t0, t1, hit = oracle.clip_box(o, d, np.zeros(3), np.array(dims) * h)
    vol3 = vol_t.reshape(dims[2], dims[1], dims[0])
    out = []
    for r in range(o.shape[0]):
        if not hit[r]:
            out.append(torch.zeros(4, dtype=torch.float64))
            continue
        C = torch.zeros(3, dtype=torch.float64)
        T = torch.ones((), dtype=torch.float64)
        s = math.floor(t0[r] / dt)
        while s * dt < t1[r]:
            ell = min((s + 1) * dt, t1[r]) - max(s * dt, t0[r])
            p = o[r] + (s + 0.5) * dt * d[r]
            g = [min(max(p[a] / h - 0.5, 0.0), dims[a] - 1.0) for a in range(3)]
            i0 = [min(int(math.floor(g[a])), dims[a] - 2) for a in range(3)]
            f = [g[a] - i0[a] for a in range(3)]
            cell = vol3[i0[2]:i0[2] + 2, i0[1]:i0[1] + 2, i0[0]:i0[0] + 2]
            ex = cell[:, :, 0] + f[0] * (cell[:, :, 1] - cell[:, :, 0])
            ey = ex[:, 0] + f[1] * (ex[:, 1] - ex[:, 0])
            v = ey[0] + f[2] * (ey[1] - ey[0])
            if plateau is not None and float(v) in (0.0, 1.0):
                plateau.append(float(v))
            u = torch.clamp((v - prm.tf_lo) / (prm.tf_hi - prm.tf_lo), 0.0, 1.0)
            x = u * (n - 1)
            j = min(int(math.floor(float(x))), n - 2)
            w = x - j
            rgba = (1 - w) * tf_t[j] + w * tf_t[j + 1]
            tau = prm.density * rgba[3] * ell
            C = C + T * (1 - torch.exp(-tau)) * rgba[:3]
            T = T * torch.exp(-tau)
            s += 1
        out.append(torch.cat([C, (1 - T).reshape(1)]))
    return torch.stack(out).reshape(cam.height, cam.width, 4)


def test_gradient_matches_torch_autograd_fp64():
    dims, vol, tf, cams, prm, tgt = _tiny_problem(1)
    L, gV, gT = _loss_grad(vol, dims, tf, prm, cams, tgt)
    vt = torch.tensor(vol, dtype=torch.float64, requires_grad=True)
    tt = torch.tensor(tf, dtype=torch.float64, requires_grad=True)
    n_el = sum(t.size for t in tgt)
    Lt = sum(((_torch_render(vt, tt, dims, prm, c) - torch.tensor(t)) ** 2).sum() for c, t in zip(cams, tgt)) / n_el
    Lt.backward()
    assert abs(Lt.item() - L) < 1e-13
    assert np.allclose(vt.grad.numpy(), gV, atol=1e-12, rtol=1e-9)
    assert np.allclose(tt.grad.numpy(), gT, atol=1e-12, rtol=1e-9)


def test_gradient_on_clamp_plateaus_matches_torch_autograd_fp64():
    """Samples exactly on the clamped plateaus v = 0 and v = 1 (u = 0 or 1).  The
    oracle counts 0 <= u <= 1 as inside the table, so the value gradient there is
    the slope of the end segment of the table, as with torch.clamp, whose gradient
    passes at the bounds; counting them as outside would give 0 there."""
    dims = (7, 6, 5)
    base = random_volume(dims, 92).astype(np.float64)
    vol = np.clip(2.2 * base - 0.35, 0.0, 1.0)          # wide regions of exact 0 and exact 1
    assert np.count_nonzero(vol == 0.0) > 20 and np.count_nonzero(vol == 1.0) > 20
    rng = np.random.default_rng(91)
    tf = rng.random((256, 4))                            # every segment sloped, both ends included
    tf[:, 3] = 0.1 + 0.8 * tf[:, 3]
    cams = [orbit_camera(dims, 6, 5), Camera((-1.0, 1.9, 1.1), (0.5, 0.42, 0.36), (0.0, 0.0, 1.0), 45.0, 5, 6)]
    prm = RenderParams(step_voxels=0.5, ert=1.0, density=6.0)
    tgt = [np.random.default_rng(92).random((c.height, c.width, 4)) * 0.5 for c in cams]
    L, gV, gT = _loss_grad(vol, dims, tf, prm, cams, tgt)
    vt = torch.tensor(vol, dtype=torch.float64, requires_grad=True)
    tt = torch.tensor(tf, dtype=torch.float64, requires_grad=True)
    n_el = sum(t.size for t in tgt)
    on = []
    Lt = sum(((_torch_render(vt, tt, dims, prm, c, on) - torch.tensor(t)) ** 2).sum() for c, t in zip(cams, tgt)) / n_el
    assert on.count(0.0) >= 10 and on.count(1.0) >= 10, (on.count(0.0), on.count(1.0))
    Lt.backward()
    assert abs(Lt.item() - L) < 1e-13
    assert np.allclose(vt.grad.numpy(), gV, atol=1e-13, rtol=1e-9)
    assert np.allclose(tt.grad.numpy(), gT, atol=1e-13, rtol=1e-9)
    # the plateau voxels carry gradient (the end segments' slopes are not zero)
    assert np.abs(gV[vol == 1.0]).max() > 1e-4 and np.abs(gV[vol == 0.0]).max() > 1e-4


def test_gradient_constant_volume_closed_form():
    """Constant volume, constant TF: d alpha / dA = D L exp(-D A L); the TF-opacity
    gradient spreads over entries with lerp weights summing to 1."""
    dims = (8, 8, 8)
    vol = np.full((8, 8, 8), 0.5)
    D = 3.0
    tf = constant_tf((0.2, 0.5, 0.9), 0.4).astype(np.float64)
    A = float(tf[0, 3])
    cam = axis_camera(dims, size=9)
    prm = RenderParams(0.5, 1.0, D)
    img = oracle.forward_image(vol, dims, tf, prm, [cam])
    tgt = img.copy()
    tgt[0, 4, 4, 3] -= 0.1            # loss = 0.01 / n_el at the centre pixel's alpha only
    n_el = tgt.size
    L, gV, gT, _ = oracle.loss_and_grad(vol, dims, tf, prm, [cam], tgt, n_elems=n_el)
    g_alpha = 2 * 0.1 / n_el
    L_chord = 1.0
    assert abs(np.sum(gT[:, 3]) - g_alpha * D * L_chord * math.exp(-D * A * L_chord)) < 1e-14
    assert np.allclose(gT[:, :3], 0.0) and np.allclose(gV, 0.0)   # constant TF: no slope wrt v
