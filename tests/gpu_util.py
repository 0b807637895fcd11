"""Shared helpers of the GPU parity tests: build a world through the C ABI and
compare its frames with the FP64 oracle."""

import sys

import numpy as np

import oracle
from synth import extract_brick

TOL_F32 = 2e-5     # max abs error per RGBA channel, FP32-stored volumes
TOL_F16 = 2e-3     # FP16-stored volumes
ERT_DELTA = 1e-4   # termination bracket: oracle at theta -+ delta


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_world(dpr, dev, vol, dims, boxes, tf, prm, cam, mc=16, flags=0, ghost=1, on_device=False):
    import torch
    w = dpr.World(dev, dims)
    w.set_params(dpr.Params(prm.step_voxels, prm.ert, mc, flags))
    for lo, hi in boxes:
        b = extract_brick(vol, dims, lo, hi, ghost)
        data = torch.from_numpy(b.data).to(dev.torch_device) if on_device else b.data
        w.add_brick(data, lo, hi, b.ghost_lo, b.ghost_hi)
    w.commit()
    w.set_transfer_function(tf, prm.tf_lo, prm.tf_hi, prm.density)
    w.set_camera(cam)
    return w


def frame_np(frame):
    frame.dev.sync()
    return (frame.rgba.cpu().numpy().astype(np.float64).reshape(-1, 4),
            frame.depth.cpu().numpy().astype(np.float64).reshape(-1),
            None if frame.counts is None else frame.counts.cpu().numpy().reshape(-1).astype(np.int64))


def oracle_brick(vol, dims, lo, hi, tf, prm, cam, px, py, theta=None, ghost=1):
    p = oracle.RenderParams(prm.step_voxels, prm.ert if theta is None else theta, prm.density, prm.tf_lo, prm.tf_hi)
    b = extract_brick(vol, dims, lo, hi, ghost)
    return oracle.render_brick(b.data, b.stored_lo, dims, lo, hi, tf, p, cam, px, py)


def check_bracketed(got_rgba, got_depth, got_n, oracle_at, ert, tol, what):
    """Compare with the oracle; where the ERT step is ambiguous use the bracket
    O(theta - delta) - tol <= got <= O(theta + delta) + tol per channel."""
    if ert >= 1.0:
        want, zw, nw = oracle_at(ert)
        err = np.max(np.abs(got_rgba - want)) if want.size else 0.0
        assert err <= tol, f"{what}: max err {err:.3e} > {tol:.1e}"
        bracketed = 0
        lo_rgba = hi_rgba = want
        nlo = nhi = nw
    else:
        lo_rgba, zw, nlo = oracle_at(ert - ERT_DELTA)
        hi_rgba, _, nhi = oracle_at(ert + ERT_DELTA)
        same = np.all(lo_rgba == hi_rgba, axis=1)
        err_same = np.max(np.abs(got_rgba[same] - lo_rgba[same])) if same.any() else 0.0
        assert err_same <= tol, f"{what}: max err {err_same:.3e} > {tol:.1e}"
        ok = (got_rgba >= lo_rgba - tol) & (got_rgba <= hi_rgba + tol)
        assert ok.all(), f"{what}: {np.count_nonzero(~ok)} channel values outside the ERT bracket"
        bracketed = int(np.count_nonzero(~same))
        err = err_same
    fin = np.isfinite(zw)
    assert np.array_equal(np.isfinite(got_depth), fin), f"{what}: hit/miss pattern differs"
    if fin.any():
        derr = np.max(np.abs(got_depth[fin] - zw[fin]) / np.maximum(zw[fin], 1e-30))
        assert derr <= 3e-7, f"{what}: depth rel err {derr:.2e}"
    if got_n is not None:
        assert np.all((got_n >= nlo) & (got_n <= nhi)), f"{what}: sample counts outside the oracle's"
    log(f"  {what}: max|gpu-oracle| = {err:.3e} (tol {tol:.0e}), bracketed pixels = {bracketed}")
    return err
