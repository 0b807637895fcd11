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


def _torch_render(vol_t, tf_t, dims, prm, cam):
    """The same quadrature re-expressed with torch FP64 ops, for torch.autograd."""
    h = 1.0 / max(dims)
    dt = prm.step_voxels * h
    n = tf_t.shape[0]
    py, px = np.mgrid[0:cam.height, 0:cam.width]
    o, d = oracle.camera_rays(cam, px.ravel(), py.ravel())
    t0, t1, hit = oracle.clip_box(o, d, np.zeros(3), np.array(dims) * h)
    flat = vol_t.reshape(-1)
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
            v = 0.0
            for dz in (0, 1):
                for dy in (0, 1):
                    for dx in (0, 1):
                        w = (f[0] if dx else 1 - f[0]) * (f[1] if dy else 1 - f[1]) * (f[2] if dz else 1 - f[2])
                        idx = ((i0[2] + dz) * dims[1] + i0[1] + dy) * dims[0] + i0[0] + dx
                        v = v + w * flat[idx]
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
