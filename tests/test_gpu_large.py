"""GPU parity at the full sizes of the large workloads, on sampled pixels: the
27-brick FP16 volume rendered for 16 cameras by the batched renderer (the launch
the bench times), and one rank's 2048x1536x1280 FP16 brick (a 16 GB blocked
array, so voxel offsets take the 64-bit path)."""

import numpy as np
import pytest

import oracle
from oracle import RenderParams
from synth import (brick_ghosts, extract_brick, fibonacci_cameras, get_config, kd_split, make_blobs, make_tf,
                   make_volume_large, orbit_camera, pixel_subset)
from tests.gpu_util import TOL_F16, frame_np, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpr():
    import paper_2407_00179_amd as m
    return m


def test_cfg3_batched_sampled(gpu_lib, dpr):
    import torch
    cfg = get_config("cfg3")
    dims = cfg.dims
    log("cfg3: generating the 1024x1024x768 FP16 volume")
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range)
    vol = make_volume_large(dims, blobs, cfg.seeds["volume"], cfg.noise_amp, cfg.fbm_periods,
                            device=gpu_lib.torch_device)
    boxes = kd_split(dims, cfg.n_bricks, cfg.seeds["kd"], 4.0)
    tf = make_tf(cfg.seeds["tf"])
    cams = fibonacci_cameras(dims, cfg.n_cams, *cfg.image)
    vol_np = vol.cpu().numpy()
    for ert in (1.0, cfg.ert):
        log(f"cfg3 ert {ert}: building the 27-brick world")
        w = dpr.World(gpu_lib, dims)
        w.set_params(dpr.Params(cfg.step_voxels, ert, cfg.macrocell, 0))
        for lo, hi in boxes:
            glo, ghi = brick_ghosts(dims, lo, hi)
            sl = vol[lo[2] - glo[2]:hi[2] + ghi[2], lo[1] - glo[1]:hi[1] + ghi[1], lo[0] - glo[0]:hi[0] + ghi[0]]
            w.add_brick(sl.contiguous(), lo, hi, glo, ghi)
        w.commit()
        w.set_transfer_function(tf, 0.0, 1.0, cfg.density)
        frames = [dpr.Frame(gpu_lib, c.width, c.height) for c in cams]
        log("  batched render of 16 cameras at 2048x2048")
        w.render_batch(cams, frames)
        gpu_lib.sync()
        prm = RenderParams(cfg.step_voxels, ert, cfg.density)
        bricks = [extract_brick(vol_np, dims, lo, hi) for lo, hi in boxes]
        for ci in (0, 9):
            cam = cams[ci]
            px, py = pixel_subset(cam.width, cam.height, stride=128, tiles=1, tile=16, seed=ci)
            log(f"  camera {ci}: oracle on {px.size} pixels x {len(boxes)} bricks")
            orc = [oracle.render_brick(b.data, b.stored_lo, dims, b.lo, b.hi, tf, prm, cam, px, py) for b in bricks]
            want, wz = oracle.composite(np.stack([o[0] for o in orc]), np.stack([o[1] for o in orc]))
            got, gz, _ = frame_np(frames[ci])
            sel = py * cam.width + px
            err = np.max(np.abs(got[sel] - want))
            log(f"  camera {ci}: max err {err:.3e}")
            if ert >= 1.0:
                assert err <= TOL_F16
                hit = np.isfinite(wz)
                assert np.array_equal(np.isfinite(gz[sel]), hit)
                assert np.max(np.abs(gz[sel][hit] - wz[hit])) <= 1e-6 * max(1.0, np.max(np.abs(wz[hit])))
            else:
                assert err <= 2 * (1 - ert) + TOL_F16
        for f in frames:
            f.release()
        w.release()
    del vol
    torch.cuda.empty_cache()


def test_cfg5_brick_sampled(gpu_lib, dpr):
    """One rank's share of the 128-rank run: 2048x1536x1280 FP16 in one brick whose
    blocked array of voxel pairs is 16 GB (64-bit offsets), rendered at 3840x2160."""
    import torch
    cfg = get_config("cfg5")
    dims = cfg.dims
    log("cfg5: generating the 2048x1536x1280 FP16 volume")
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range, log_uniform=cfg.log_sigma)
    vol = make_volume_large(dims, blobs, cfg.seeds["volume"], cfg.noise_amp, cfg.fbm_periods,
                            device=gpu_lib.torch_device)
    tf = make_tf(cfg.seeds["tf"])
    cam = orbit_camera(dims, *cfg.image)
    log("cfg5: world with one 8 GB brick")
    w = dpr.World(gpu_lib, dims)
    w.set_params(dpr.Params(cfg.step_voxels, 1.0, cfg.macrocell, 0))
    w.add_brick(vol, (0, 0, 0), dims, (0, 0, 0), (0, 0, 0))
    vol_np = vol.cpu().numpy()
    del vol
    torch.cuda.empty_cache()
    w.commit()
    w.set_transfer_function(tf, 0.0, 1.0, cfg.density)
    w.set_camera(cam)
    out = dpr.Frame(gpu_lib, *cfg.image)
    log("cfg5: render at 3840x2160")
    w.render_partial(0, out)
    got, gz, _ = frame_np(out)
    # a grid over the middle of the screen, where the volume projects, plus one
    # dense 8x8 tile inside it
    W, H = cfg.image
    ys, xs = np.mgrid[H * 3 // 10:H * 7 // 10:36, W * 3 // 8:W * 5 // 8:40]
    rng = np.random.default_rng(5)
    tx, ty = int(rng.integers(W * 7 // 16, W * 9 // 16)), int(rng.integers(H * 7 // 16, H * 9 // 16))
    ty_, tx_ = np.mgrid[ty:ty + 8, tx:tx + 8]
    px = np.concatenate([xs.ravel(), tx_.ravel()])
    py = np.concatenate([ys.ravel(), ty_.ravel()])
    log(f"cfg5: oracle on {px.size} pixels")
    prm = RenderParams(cfg.step_voxels, 1.0, cfg.density)
    want, wz, _ = oracle.render_brick(vol_np, (0, 0, 0), dims, (0, 0, 0), dims, tf, prm, cam, px, py)
    sel = py * cfg.image[0] + px
    err = np.max(np.abs(got[sel] - want))
    log(f"cfg5: max err {err:.3e} ({np.count_nonzero(np.isfinite(wz))} hit pixels)")
    assert err <= TOL_F16
    assert np.array_equal(np.isfinite(gz[sel]), np.isfinite(wz))
    assert np.count_nonzero(np.isfinite(wz)) >= px.size // 2  # the sample lies on the volume
    out.release()
    w.release()
