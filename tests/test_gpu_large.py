"""GPU parity at the full sizes of the large workloads, at the benchmark's settings
(early termination at 0.99): the 27-brick FP16 volume rendered for 16 cameras by
the batched renderer (the launch the benchmark times), and one rank's
2048x1536x1280 FP16 brick (8 GB; stored as 2-byte voxels with 64-bit offsets)
rendered at 3840x2160 through the persistent kernel.  Checked on every 8th pixel
plus four 64x64 tiles where the volume projects: every brick's partial against the
bracketed oracle, the composited frame against the oracle's composite."""

import types

import numpy as np
import pytest

from oracle import RenderParams
from synth import (brick_ghosts, fibonacci_cameras, get_config, kd_split, make_blobs, make_tf, make_volume_large,
                   orbit_camera)
from tests.gpu_util import TOL_F16, check_partials_and_frame, frame_np, log, pc10_subset

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpr():
    import paper_2407_00179_amd as m
    return m


def _brick(data, stored_lo, lo, hi):
    return types.SimpleNamespace(data=data, stored_lo=tuple(stored_lo), lo=tuple(lo), hi=tuple(hi))


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
    prm = RenderParams(cfg.step_voxels, cfg.ert, cfg.density)
    log("cfg3: building the 27-brick world")
    w = dpr.World(gpu_lib, dims)
    w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, 0))
    bricks = []
    for lo, hi in boxes:
        glo, ghi = brick_ghosts(dims, lo, hi)
        sl = (slice(lo[2] - glo[2], hi[2] + ghi[2]), slice(lo[1] - glo[1], hi[1] + ghi[1]),
              slice(lo[0] - glo[0], hi[0] + ghi[0]))
        w.add_brick(vol[sl].contiguous(), lo, hi, glo, ghi)
        bricks.append(_brick(vol_np[sl], [lo[a] - glo[a] for a in range(3)], lo, hi))
    del vol
    torch.cuda.empty_cache()
    w.commit()
    w.set_transfer_function(tf, 0.0, 1.0, cfg.density)
    frames = [dpr.Frame(gpu_lib, c.width, c.height) for c in cams]
    log("  batched render of 16 cameras at 2048x2048")
    w.render_batch(cams, frames)
    gpu_lib.sync()
    for ci in (0, 9):
        cam = cams[ci]
        w.set_camera(cam)
        px, py = pc10_subset(cam, dims, seed=ci)
        log(f"  camera {ci}: {px.size} pixels x {len(boxes)} bricks")
        check_partials_and_frame(dpr, gpu_lib, w, bricks, dims, tf, prm, cam, px, py, TOL_F16, f"cfg3 camera {ci}",
                                 frame=frames[ci])
    for f in frames:
        f.release()
    w.release()
    torch.cuda.empty_cache()


def test_cfg5_brick_sampled(gpu_lib, dpr):
    """One rank's share of the 128-rank run: 2048x1536x1280 FP16 in one brick (8 GB,
    64-bit offsets), 3840x2160, early termination at 0.99, through dpr_render_frame;
    the frame also equals the plain per-brick launch bit for bit."""
    import torch
    cfg = get_config("cfg5")
    dims = cfg.dims
    log("cfg5: generating the 2048x1536x1280 FP16 volume")
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range, log_uniform=cfg.log_sigma)
    vol = make_volume_large(dims, blobs, cfg.seeds["volume"], cfg.noise_amp, cfg.fbm_periods,
                            device=gpu_lib.torch_device)
    tf = make_tf(cfg.seeds["tf"])
    cam = orbit_camera(dims, *cfg.image)
    prm = RenderParams(cfg.step_voxels, cfg.ert, cfg.density)
    log("cfg5: world with one 8 GB brick")
    w = dpr.World(gpu_lib, dims)
    w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, 0))
    w.add_brick(vol, (0, 0, 0), dims, (0, 0, 0), (0, 0, 0))
    vol_np = vol.cpu().numpy()
    del vol
    torch.cuda.empty_cache()
    w.commit()
    w.set_transfer_function(tf, 0.0, 1.0, cfg.density)
    w.set_camera(cam)
    out = dpr.Frame(gpu_lib, *cfg.image)
    log("cfg5: render at 3840x2160")
    w.render_frame(out)
    got, gz, _ = frame_np(out)
    plain = dpr.Frame(gpu_lib, *cfg.image)
    w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, dpr.FLAG_PLAIN))
    w.render_partial(0, plain)
    pr, pz, _ = frame_np(plain)
    assert np.array_equal(got, pr) and np.array_equal(gz, pz)
    w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, 0))
    px, py = pc10_subset(cam, dims, seed=5)
    log(f"cfg5: oracle on {px.size} pixels")
    err = check_partials_and_frame(dpr, gpu_lib, w, [_brick(vol_np, (0, 0, 0), (0, 0, 0), dims)], dims, tf, prm,
                                   cam, px, py, TOL_F16, "cfg5", frame=out)
    assert np.count_nonzero(np.isfinite(gz[py * cam.width + px])) >= 4 * 64 * 64 // 2   # the tiles lie on the volume
    log(f"cfg5: max err {err:.3e}")
    for f in (out, plain):
        f.release()
    w.release()
