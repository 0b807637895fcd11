"""GPU tests of the differentiable render and its hand-written adjoint."""

import numpy as np
import pytest

import oracle
from oracle import RenderParams
from synth import Camera, fibonacci_cameras, make_blobs, make_tf, make_volume_small, perturb_blobs  # noqa: F401
from synth.volume import perturb_blobs as _perturb
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

REL_TOL = 1e-3


@pytest.fixture(scope="module")
def dpr():
    import paper_2407_00179_amd as m
    return m


def _problem(dims=(20, 18, 16), n_cams=3, size=(24, 20), seed=7):
    blobs = make_blobs(dims, seed, 5, (0.12, 0.3))
    vol = 0.03 + 0.94 * make_volume_small(dims, blobs, seed + 1, 0.02)   # away from the clamp kinks
    tgt_vol = 0.03 + 0.94 * make_volume_small(dims, _perturb(blobs, seed + 2), seed + 1, 0.02)
    tf = make_tf(2001)
    tf[:, 3] = np.maximum(tf[:, 3], 0.02)
    cams = fibonacci_cameras(dims, n_cams, *size)
    return dims, vol.astype(np.float32), tgt_vol.astype(np.float32), tf.astype(np.float32), cams


def _gpu_loss_grad(dpr, dev, vol, tf, cams, prm, target):
    import torch
    v = torch.tensor(vol, device=dev.torch_device, requires_grad=True)
    t = torch.tensor(tf, device=dev.torch_device, requires_grad=True)
    img = dpr.render_train(dev, v, t, cams, dpr.Params(prm.step_voxels, 1.0, 16, 0), 0.0, 1.0, prm.density)
    loss = ((img - torch.tensor(target, device=dev.torch_device)) ** 2).mean()
    loss.backward()
    return (img.detach().cpu().numpy().astype(np.float64), float(loss.item()),
            v.grad.cpu().numpy().astype(np.float64), t.grad.cpu().numpy().astype(np.float64))


def test_forward_matches_oracle(gpu_lib, dpr):
    dims, vol, _, tf, cams = _problem()
    prm = RenderParams(0.5, 1.0, 15.0)
    import torch
    v = torch.tensor(vol, device=gpu_lib.torch_device)
    t = torch.tensor(tf, device=gpu_lib.torch_device)
    img = dpr.render_train(gpu_lib, v, t, cams, dpr.Params(0.5, 1.0, 16, 0), 0.0, 1.0, 15.0)
    got = img.cpu().numpy().astype(np.float64)
    want = oracle.forward_image(vol, dims, tf, prm, cams)
    err = np.max(np.abs(got - want))
    log(f"train forward vs oracle: {err:.3e}")
    assert err <= 2e-5 and want[..., 3].max() > 0.3


@pytest.mark.parametrize("step", [0.5, 0.37])
def test_gradients_match_oracle_adjoint(gpu_lib, dpr, step):
    dims, vol, tgt_vol, tf, cams = _problem()
    prm = RenderParams(step, 1.0, 15.0)
    target = oracle.forward_image(tgt_vol, dims, tf, prm, cams)
    img, loss, gv, gt = _gpu_loss_grad(dpr, gpu_lib, vol, tf, cams, prm, target)
    L, wv, wt, _ = oracle.loss_and_grad(vol, dims, tf, prm, cams, target)
    log(f"loss gpu {loss:.8e} oracle {L:.8e}")
    assert abs(loss - L) <= 1e-5 * abs(L) + 1e-12
    for name, g, w in (("volume", gv, wv), ("tf", gt, wt)):
        rel = np.linalg.norm(g - w) / np.linalg.norm(w)
        big = np.abs(w) > 1e-3 * np.abs(w).max()
        per = np.max(np.abs(g[big] - w[big]) / np.abs(w[big]))
        log(f"  d/d{name}: relative L2 {rel:.2e}, max per-entry (significant) {per:.2e}")
        assert rel <= REL_TOL
        assert per <= REL_TOL


def _linear_tf(n=256):
    """A kink-free table (every channel affine in the value), so central differences
    of the loss never straddle a slope change of the transfer function."""
    u = np.arange(n) / (n - 1)
    return np.stack([0.2 + 0.7 * u, 0.9 - 0.6 * u, 0.5 + 0.0 * u, 0.05 + 0.85 * u], axis=1).astype(np.float32)


def test_gradients_match_finite_differences(gpu_lib, dpr):
    """Directional derivatives g.u against FP64 central differences of the oracle forward."""
    dims, vol, tgt_vol, _, cams = _problem(n_cams=2)
    tf = _linear_tf()
    prm = RenderParams(0.5, 1.0, 15.0)
    target = oracle.forward_image(tgt_vol, dims, tf, prm, cams)
    _, _, gv, gt = _gpu_loss_grad(dpr, gpu_lib, vol, tf, cams, prm, target)
    rng = np.random.default_rng(5004)
    h = 1e-4
    v64, t64 = vol.astype(np.float64), tf.astype(np.float64)

    def loss(v, t):
        return float(np.mean((oracle.forward_image(v, dims, t, prm, cams) - target) ** 2))

    for kind in ("volume", "tf"):
        for _ in range(3):
            if kind == "volume":
                u = rng.choice([-1.0, 1.0], size=vol.shape)
                fd = (loss(v64 + h * u, t64) - loss(v64 - h * u, t64)) / (2 * h)
                an = float(np.sum(gv * u))
            else:
                u = rng.choice([-1.0, 1.0], size=tf.shape)
                fd = (loss(v64, t64 + h * u) - loss(v64, t64 - h * u)) / (2 * h)
                an = float(np.sum(gt * u))
            log(f"  FD {kind}: fd {fd:.6e} analytic {an:.6e}")
            assert abs(fd - an) <= REL_TOL * max(abs(fd), 1e-8) + 1e-9


def test_backward_accumulates(gpu_lib, dpr):
    import ctypes as C
    import torch
    from paper_2407_00179_amd import _native as N
    dims, vol, _, tf, cams = _problem(n_cams=1)
    v = torch.tensor(vol, device=gpu_lib.torch_device)
    t = torch.tensor(tf, device=gpu_lib.torch_device)
    fn = dpr.DprRenderFn
    p = dpr.Params(0.5, 1.0, 16, 0)
    out, _ = fn.apply(v, t, gpu_lib, cams, p, 0.0, 1.0, 15.0)
    g = torch.randn_like(out)
    gv = torch.zeros_like(v)
    gt = torch.zeros_like(t)
    ca = (N.Camera * 1)(dpr.to_c_camera(cams[0]))
    nb = C.c_size_t()
    dpr.check(dpr.lib.dpr_train_workspace_size(N.I64x3(*dims), ca, 1, 0.5, C.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=gpu_lib.torch_device)
    depth = torch.empty(out.shape[:-1], device=gpu_lib.torch_device)
    cp = p.c()
    dpr.check(dpr.lib.dpr_render_train_forward(gpu_lib.h, C.c_void_p(v.data_ptr()), N.I64x3(*dims),
                                               C.c_void_p(t.data_ptr()), t.shape[0], 0.0, 1.0, 15.0, C.byref(cp), ca,
                                               1, C.c_void_p(out.data_ptr()), C.c_void_p(depth.data_ptr()),
                                               C.c_void_p(ws.data_ptr()), nb.value))
    for rep in range(2):
        dpr.check(dpr.lib.dpr_render_backward(gpu_lib.h, C.c_void_p(v.data_ptr()), N.I64x3(*dims),
                                              C.c_void_p(t.data_ptr()), t.shape[0], 0.0, 1.0, 15.0, C.byref(cp), ca,
                                              1, C.c_void_p(g.data_ptr()), C.c_void_p(ws.data_ptr()), nb.value,
                                              C.c_void_p(gv.data_ptr()), C.c_void_p(gt.data_ptr())))
        if rep == 0:
            once_v, once_t = gv.clone(), gt.clone()
    torch.cuda.synchronize()
    # atomics sum in a different order each call: compare at FP32 rounding of the largest entry
    assert torch.allclose(gv, 2 * once_v, rtol=1e-4, atol=1e-5 * float(once_v.abs().max()))
    assert torch.allclose(gt, 2 * once_t, rtol=1e-4, atol=1e-5 * float(once_t.abs().max()))
    assert float(once_v.abs().max()) > 0 and float(once_t.abs().max()) > 0
    with pytest.raises(dpr.DprError):   # workspace too small
        dpr.check(dpr.lib.dpr_render_backward(gpu_lib.h, C.c_void_p(v.data_ptr()), N.I64x3(*dims),
                                              C.c_void_p(t.data_ptr()), t.shape[0], 0.0, 1.0, 15.0, C.byref(cp), ca,
                                              1, C.c_void_p(g.data_ptr()), C.c_void_p(ws.data_ptr()), 8,
                                              C.c_void_p(gv.data_ptr()), C.c_void_p(gt.data_ptr())))


def _lattice_samples(dims, cam, px, py, step, chunk=2048):
    """Every lattice sample of the rays through pixels (px, py) across the whole
    volume (ERT off): yields per chunk of rays (ray index, flat indices of the 8
    trilinear corners (S, 8), their weights (S, 8)), by the sampling rule the
    render follows (eye-anchored segments of positive clipped length, midpoint
    sample, clamp to [0, n - 1])."""
    nx, ny, nz = dims
    h = 1.0 / max(dims)
    dt = step * h
    for c0 in range(0, px.size, chunk):
        o, d = oracle.camera_rays(cam, px[c0:c0 + chunk], py[c0:c0 + chunk])
        t_in, t_out, hit = oracle.clip_box(o, d, np.zeros(3), np.array(dims, dtype=np.float64) * h)
        rays, ts = [], []
        for r in np.flatnonzero(hit):
            s = np.arange(np.floor(t_in[r] / dt), np.ceil(t_out[r] / dt))
            ell = np.minimum((s + 1) * dt, t_out[r]) - np.maximum(s * dt, t_in[r])
            s = s[ell > 0]
            rays.append(np.full(s.size, c0 + r))
            ts.append((s + 0.5) * dt)
        if not rays:
            continue
        ray = np.concatenate(rays)
        t = np.concatenate(ts)
        loc = ray - c0
        g = (o[loc] + t[:, None] * d[loc]) / h - 0.5
        idx = np.zeros((t.size, 8), dtype=np.int64)
        w = np.ones((t.size, 8))
        for a, n in enumerate((nx, ny, nz)):
            ga = np.clip(g[:, a], 0.0, n - 1.0)
            i0 = np.minimum(np.floor(ga), n - 2).astype(np.int64)
            f = ga - i0
            for c in range(8):
                bit = (c >> a) & 1
                idx[:, c] += (i0 + bit) * (1, nx, nx * ny)[a]
                w[:, c] *= f if bit else 1.0 - f
        yield ray, idx, w


def _table_segment(v, n_tf):
    """Linear piece of the table lookup a value falls on: -1 and n - 1 for the
    clamped plateaus below 0 and above 1, else the entry interval floor(x)."""
    x = v * (n_tf - 1)
    return np.where(x < 0, -1, np.where(x >= n_tf - 1, n_tf - 1, np.floor(x))).astype(np.int64)


def _kink_free(u, v64, samples, h, n_tf):
    """Zero u on every voxel that is a trilinear corner of a sample whose value
    would change linear piece of the table between V - h u and V + h u, until no
    sample does: the loss is then smooth along u over [-h, h], so a central
    difference at h is exact to O(h^2)."""
    u = u.copy()
    vf = v64.ravel()
    for _ in range(20):
        uf = u.ravel()
        bad = []
        for _, idx, w in samples:
            v = np.sum(w * vf[idx], axis=1)
            dv = h * np.sum(w * uf[idx], axis=1)
            k = _table_segment(v + dv, n_tf) != _table_segment(v - dv, n_tf)
            if k.any():
                bad.append(idx[k][w[k] > 0])
        if not bad:
            return u
        uf[np.unique(np.concatenate(bad))] = 0.0
    raise AssertionError("no kink-free direction")


def test_cfg4_subgrid_finite_differences(gpu_lib, dpr):
    """The finite-difference protocol on the 256^3 training workload, one 512^2 camera,
    h = 1e-4: 8 seeded Rademacher directions of the density grid restricted to the
    32^3 subgrid at voxel offset (112, 112, 112), made kink-free by the exact rule
    (no sample's table coordinate crosses an entry boundary or a clamp end between
    V - h u and V + h u), and 8 directions in the 1024-dim table space (the loss is
    smooth in the table); the loss is the squared error over the pixels whose rays
    hit the subgrid, its central difference formed pixel-wise as
    sum (I+ - I-)(I+ + I- - 2 I*) / 2h; each g.u within 1e-3 of it."""
    import torch
    from synth import get_config
    cfg = get_config("cfg4")
    dims = cfg.dims
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range)
    log("cfg4: generating 256^3 volume")
    vol = make_volume_small(dims, blobs, cfg.seeds["volume"], cfg.noise_amp)
    tgt = make_volume_small(dims, _perturb(blobs, cfg.seeds["perturb"]), cfg.seeds["volume"], cfg.noise_amp)
    tf = make_tf(cfg.seeds["tf"])
    cam = fibonacci_cameras(dims, cfg.n_cams, *cfg.image)[5]
    prm = RenderParams(cfg.step_voxels, 1.0, cfg.density)
    h = 1.0 / max(dims)
    lo, hi = np.array([112.0] * 3) * h, np.array([144.0] * 3) * h
    py, px = np.mgrid[0:cam.height, 0:cam.width]
    px, py = px.ravel(), py.ravel()
    o, d = oracle.camera_rays(cam, px, py)
    _, _, hit = oracle.clip_box(o, d, lo, hi)
    px, py = px[hit], py[hit]
    assert px.size > 100
    log(f"cfg4: {px.size} pixels hit the subgrid")
    v = torch.tensor(vol, device=gpu_lib.torch_device, requires_grad=True)
    t = torch.tensor(tf, device=gpu_lib.torch_device, requires_grad=True)
    img = dpr.render_train(gpu_lib, v, t, [cam], dpr.Params(cfg.step_voxels, 1.0, 16, 0), 0.0, 1.0, cfg.density)
    tgt_img = oracle.render_image(tgt, dims, tf, prm, cam, px, py)[0]
    sel = torch.from_numpy(py * cam.width + px).to(gpu_lib.torch_device)
    pix = img.reshape(-1, 4)[sel]
    loss = ((pix - torch.tensor(tgt_img, device=gpu_lib.torch_device, dtype=torch.float32)) ** 2).sum()
    loss.backward()
    g = v.grad.cpu().numpy().astype(np.float64)
    gt = t.grad.cpu().numpy().astype(np.float64)
    v64, t64 = vol.astype(np.float64), tf.astype(np.float64)
    # against the oracle adjoint on the same pixels
    L, wv, wt, _ = oracle.loss_and_grad(v64, dims, tf, prm, [cam], [tgt_img], n_elems=1, pixels=[(px, py)])
    for name, a, b in (("volume", g, wv), ("table", gt, wt)):
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        log(f"  cfg4 subset d/d{name} vs oracle adjoint: relative L2 {rel:.2e}")
        assert rel <= REL_TOL
    rng = np.random.default_rng(cfg.seeds["fd"])
    eps = 1e-4

    def fd(vp, vm, tp, tm):
        ip = oracle.render_image(vp, dims, tp, prm, cam, px, py)[0]
        im = oracle.render_image(vm, dims, tm, prm, cam, px, py)[0]
        return float(np.sum((ip - im) * (ip + im - 2 * tgt_img))) / (2 * eps)

    samples = list(_lattice_samples(dims, cam, px, py, cfg.step_voxels))
    for r in range(8):
        u = np.zeros_like(v64)
        u[112:144, 112:144, 112:144] = rng.choice([-1.0, 1.0], size=(32, 32, 32))
        uk = _kink_free(u, v64, samples, eps, tf.shape[0])
        kept = np.count_nonzero(uk) / np.count_nonzero(u)
        f = fd(v64 + eps * uk, v64 - eps * uk, t64, t64)
        an = float(np.sum(g * uk))
        log(f"  cfg4 FD volume dir {r}: fd {f:.8e} analytic {an:.8e} (kink-free voxels kept {kept:.2f})")
        assert kept > 0.5
        assert abs(f - an) <= REL_TOL * abs(f)
    for r in range(8):
        u = rng.choice([-1.0, 1.0], size=tf.shape)
        f = fd(v64, v64, t64 + eps * u, t64 - eps * u)
        an = float(np.sum(gt * u))
        log(f"  cfg4 FD table dir {r}: fd {f:.8e} analytic {an:.8e}")
        assert abs(f - an) <= REL_TOL * abs(f)


def test_cfg4_per_voxel_finite_differences(gpu_lib, dpr):
    """Per-entry central differences (h = 1e-4) on 64 seeded voxels of the 256^3
    training workload, one camera at 128x128, against the GPU gradient entry by
    entry (1e-3 relative).  Voxels are drawn over the whole volume among those
    whose gradient is significant (above 1e-3 of the largest; the central 32^3
    subgrid holds only a few dozen voxels with any gradient from one camera) and
    whose +-h change moves no sample across a linear piece of the table."""
    import torch
    from synth import get_config
    cfg = get_config("cfg4")
    dims = cfg.dims
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range)
    vol = make_volume_small(dims, blobs, cfg.seeds["volume"], cfg.noise_amp)
    tgt = make_volume_small(dims, _perturb(blobs, cfg.seeds["perturb"]), cfg.seeds["volume"], cfg.noise_amp)
    tf = make_tf(cfg.seeds["tf"])
    cam = fibonacci_cameras(dims, cfg.n_cams, 128, 128)[5]
    prm = RenderParams(cfg.step_voxels, 1.0, cfg.density)
    p = dpr.Params(cfg.step_voxels, 1.0, 16, 0)
    t = torch.tensor(tf, device=gpu_lib.torch_device)
    with torch.no_grad():
        target = dpr.render_train(gpu_lib, torch.tensor(tgt, device=gpu_lib.torch_device), t, [cam], p, 0.0, 1.0,
                                  cfg.density)
    v = torch.tensor(vol, device=gpu_lib.torch_device, requires_grad=True)
    img = dpr.render_train(gpu_lib, v, t, [cam], p, 0.0, 1.0, cfg.density)
    ((img - target) ** 2).sum().backward()
    g = v.grad.cpu().numpy().astype(np.float64).ravel()
    tgt_img = target.cpu().numpy().astype(np.float64).reshape(-1, 4)
    v64 = vol.astype(np.float64)
    vf = v64.ravel()
    eps = 1e-4
    cand = np.flatnonzero(np.abs(g) > 1e-3 * np.abs(g).max())
    cand = np.random.default_rng(cfg.seeds["fd"] + 1).permutation(cand)[:400]
    # rays (pixels) and samples touching each candidate voxel
    py, px = np.mgrid[0:cam.height, 0:cam.width]
    px, py = px.ravel(), py.ravel()
    touch = {int(c): [] for c in cand}
    cset = np.sort(cand)
    for ray, idx, w in _lattice_samples(dims, cam, px, py, cfg.step_voxels):
        pos = np.searchsorted(cset, idx)
        pos = np.minimum(pos, cset.size - 1)
        m = (cset[pos] == idx) & (w > 0)
        for s_, c_ in zip(*np.nonzero(m)):
            touch[int(idx[s_, c_])].append((int(ray[s_]), float(np.sum(w[s_] * vf[idx[s_]])), float(w[s_, c_])))
    checked = 0
    for c in cand:
        rows = touch[int(c)]
        if not rows:
            continue
        vv = np.array([r[1] for r in rows])
        ww = np.array([r[2] for r in rows])
        if np.any(_table_segment(vv + eps * ww, tf.shape[0]) != _table_segment(vv - eps * ww, tf.shape[0])):
            continue   # a kink within +-h: not this voxel
        rays = np.unique([r[0] for r in rows])
        e = np.zeros_like(vf)
        e[c] = eps
        ip = oracle.render_image((vf + e).reshape(vol.shape), dims, tf, prm, cam, px[rays], py[rays])[0]
        im = oracle.render_image((vf - e).reshape(vol.shape), dims, tf, prm, cam, px[rays], py[rays])[0]
        f = float(np.sum((ip - im) * (ip + im - 2 * tgt_img[rays]))) / (2 * eps)
        assert abs(f - g[c]) <= REL_TOL * abs(f), (int(c), f, g[c])
        checked += 1
        if checked == 64:
            break
    log(f"  cfg4 per-voxel FD: {checked} voxels within {REL_TOL:.0e}")
    assert checked == 64
