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
        assert per <= 10 * REL_TOL


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


def test_cfg4_subgrid_finite_differences(gpu_lib, dpr):
    """256^3 density grid, 512^2 camera: directional FD restricted to the 32^3 subgrid at
    voxel offset (112,112,112), over the pixels whose rays hit that subgrid."""
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
    # pixels whose rays hit the subgrid box
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
    t = torch.tensor(tf, device=gpu_lib.torch_device)
    img = dpr.render_train(gpu_lib, v, t, [cam], dpr.Params(cfg.step_voxels, 1.0, 16, 0), 0.0, 1.0, cfg.density)
    tgt_img = oracle.render_image(tgt, dims, tf, prm, cam, px, py)[0]
    sel = torch.from_numpy(py * cam.width + px).to(gpu_lib.torch_device)
    pix = img.reshape(-1, 4)[sel]
    loss = ((pix - torch.tensor(tgt_img, device=gpu_lib.torch_device, dtype=torch.float32)) ** 2).sum()
    loss.backward()
    g = v.grad.cpu().numpy().astype(np.float64)
    v64 = vol.astype(np.float64)
    # against the oracle adjoint on the same pixels (same one-sided convention at kinks)
    L, wv, _, _ = oracle.loss_and_grad(v64, dims, tf, prm, [cam], [tgt_img], n_elems=1, pixels=[(px, py)])
    rel = np.linalg.norm(g - wv) / np.linalg.norm(wv)
    log(f"  cfg4 subset gradient vs oracle adjoint: relative L2 {rel:.2e}")
    assert rel <= REL_TOL
    rng = np.random.default_rng(cfg.seeds["fd"])
    # small step: ~700K samples, so at 1e-4 many cross a knot of the table (e.g. the
    # end of the transparent floor); FP64 central differences are still exact to ~1e-9 here
    eps = 1e-6
    # perturb only voxels off the clamped plateaus (values 0 and 1 sit on TF-clamp kinks)
    free = (v64 > 1e-3) & (v64 < 1 - 1e-3)
    def fd_at(u, e):
        ip = oracle.render_image(v64 + e * u, dims, tf, prm, cam, px, py)[0]
        im = oracle.render_image(v64 - e * u, dims, tf, prm, cam, px, py)[0]
        # pixel-wise difference of squared errors, free of cancellation
        return float(np.sum((ip - im) * (ip + im - 2 * tgt_img))) / (2 * e)

    checked = 0
    for r in range(4):
        u = np.zeros_like(v64)
        u[112:144, 112:144, 112:144] = rng.choice([-1.0, 1.0], size=(32, 32, 32))
        u *= free
        fd, fd2 = fd_at(u, eps), fd_at(u, eps / 2)
        an = float(np.sum(g * u))
        # a sample whose TF coordinate crosses a knot of the table within +-eps makes
        # the central difference depend on eps: such a direction is a kink, skipped
        kink = abs(fd - fd2) > 0.25 * REL_TOL * abs(fd2)
        log(f"  cfg4 FD dir {r}: fd {fd:.6e} (eps/2 {fd2:.6e}) analytic {an:.6e} kink={kink}")
        if kink:
            continue
        checked += 1
        assert abs(fd2 - an) <= REL_TOL * abs(fd2) + 1e-7
    assert checked >= 2
