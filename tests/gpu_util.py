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


def pc10_subset(cam, dims, seed, stride=8, tiles=4, tile=64):
    """Pixel sample of the full-size checks: every stride-th pixel in x and y of the
    whole frame plus `tiles` full tile x tile blocks placed (seeded) where the
    volume's box projects -- found from the camera geometry by the oracle's slab
    test on a coarse pixel grid, not from any rendered frame."""
    W, H = cam.width, cam.height
    ys, xs = np.mgrid[0:H:16, 0:W:16]
    o, d = oracle.camera_rays(cam, xs.ravel(), ys.ravel())
    h = 1.0 / max(dims)
    _, _, hit = oracle.clip_box(o, d, np.zeros(3), np.array(dims, dtype=np.float64) * h)
    hx, hy = xs.ravel()[hit], ys.ravel()[hit]
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H:stride, 0:W:stride]
    px, py = [xx.ravel()], [yy.ravel()]
    for _ in range(tiles):
        k = int(rng.integers(0, hx.size))
        tx = int(np.clip(hx[k] - tile // 2, 0, W - tile))
        ty = int(np.clip(hy[k] - tile // 2, 0, H - tile))
        ty_, tx_ = np.mgrid[ty:ty + tile, tx:tx + tile]
        px.append(tx_.ravel())
        py.append(ty_.ravel())
    lin = np.unique(np.concatenate(py) * W + np.concatenate(px))
    return (lin % W).astype(np.int64), (lin // W).astype(np.int64)


def oracle_bracket(data, stored_lo, dims, lo, hi, tf, prm, cam, px, py):
    """The oracle's partial fragments at the termination thresholds theta - delta and
    theta + delta (or at theta when early termination is off), from one march per
    ray; returned as a lookup usable by check_bracketed."""
    thetas = [prm.ert] if prm.ert >= 1.0 else [prm.ert - ERT_DELTA, prm.ert + ERT_DELTA]
    p = oracle.RenderParams(prm.step_voxels, 1.0, prm.density, prm.tf_lo, prm.tf_hi)
    res = oracle.render_brick_thresholds(data, stored_lo, dims, lo, hi, tf, p, cam, px, py, thetas)
    table = dict(zip(thetas, res))
    return lambda th: table[th]


def check_partials_and_frame(dpr, dev, w, bricks, dims, tf, prm, cam, px, py, tol, what, frame=None):
    """Every brick's partial frame (dpr_render_partial, the persistent kernel)
    against the bracketed oracle on the pixel sample; then the composited frame
    (a) against the oracle's compositor applied to the GPU's own partials, on every
    sampled pixel, and (b) against the oracle's composite of the oracle's partials
    on the sampled pixels where no brick's termination step is ambiguous.
    `bricks` are synth Bricks (their stored data and boxes)."""
    sel = py * cam.width + px
    fr = dpr.Frame(dev, cam.width, cam.height)
    g_r, g_z, o_r, o_z, amb = [], [], [], [], np.zeros(px.size, dtype=bool)
    for i, b in enumerate(bricks):
        w.render_partial(i, fr)
        r, z, _ = frame_np(fr)
        at = oracle_bracket(b.data, b.stored_lo, dims, b.lo, b.hi, tf, prm, cam, px, py)
        check_bracketed(r[sel], z[sel], None, at, prm.ert, tol, f"{what} brick {i}")
        lo_r = at(prm.ert if prm.ert >= 1.0 else prm.ert - ERT_DELTA)
        hi_r = at(prm.ert if prm.ert >= 1.0 else prm.ert + ERT_DELTA)
        amb |= np.any(lo_r[0] != hi_r[0], axis=1)
        g_r.append(r[sel])
        g_z.append(z[sel])
        o_r.append(lo_r[0])
        o_z.append(lo_r[1])
    fr.release()
    got, gz, _ = frame_np(frame)
    got, gz = got[sel], gz[sel]
    mine, mz = oracle.composite(np.stack(g_r), np.stack(g_z))
    err_a = np.max(np.abs(got - mine))
    assert err_a <= tol, f"{what}: composite of the GPU partials differs by {err_a:.3e}"
    assert np.array_equal(gz, mz.astype(np.float32).astype(np.float64)), f"{what}: composite depth"
    want, wz = oracle.composite(np.stack(o_r), np.stack(o_z))
    ok = ~amb
    err_b = np.max(np.abs(got[ok] - want[ok])) if ok.any() else 0.0
    log(f"  {what}: frame vs oracle compositor on GPU partials {err_a:.3e}; vs oracle composite on "
        f"{np.count_nonzero(ok)} unambiguous of {px.size} pixels {err_b:.3e} ({np.count_nonzero(amb)} ambiguous)")
    assert err_b <= tol, f"{what}: composite vs oracle {err_b:.3e}"
    return err_b


def tf_alpha_max(tf, ranges, lo=0.0, hi=1.0, chunk=1 << 15):
    """FP64 largest table opacity over each value range [min, max] (..., 2): the
    table is piecewise linear, so the maximum lies at an end or at a knot inside."""
    tf = np.asarray(tf, dtype=np.float64)
    n = tf.shape[0]
    a = np.asarray(ranges[..., 0], dtype=np.float64).ravel()
    b = np.asarray(ranges[..., 1], dtype=np.float64).ravel()
    knots = lo + np.arange(n) * (hi - lo) / (n - 1)
    out = np.empty(a.size)
    for c0 in range(0, a.size, chunk):
        aa, bb = a[c0:c0 + chunk], b[c0:c0 + chunk]
        ends = np.maximum(oracle.tf_lookup(tf, aa, lo, hi)[:, 3], oracle.tf_lookup(tf, bb, lo, hi)[:, 3])
        inside = (knots[None, :] > aa[:, None]) & (knots[None, :] < bb[:, None])
        out[c0:c0 + chunk] = np.maximum(ends, np.max(np.where(inside, tf[None, :, 3], 0.0), axis=1))
    return out.reshape(np.shape(ranges)[:-1])


def _majorant_candidates(ranges, tf, lo, hi, eps=1e-4):
    """Majorants of the entry ranges reachable by moving each end's table
    coordinate by +-eps (the choices an FP32 decision can make)."""
    a = np.asarray(tf, dtype=np.float32)[:, 3]
    n = a.shape[0]
    xs = []
    for k in (0, 1):
        v = np.asarray(ranges[..., k], dtype=np.float64).ravel()
        xs.append((oracle.tf_coord(v, lo, hi, n), ((v > lo) & (v < hi)) * eps))
    out = []
    for s0 in (-1, 1):
        for s1 in (-1, 1):
            e0 = np.maximum(np.floor(xs[0][0] + s0 * xs[0][1]).astype(np.int64) - 1, 0)
            e1 = np.minimum(np.ceil(xs[1][0] + s1 * xs[1][1]).astype(np.int64) + 1, n - 1)
            out.append(np.array([a[i:j + 1].max() for i, j in zip(e0, e1)], dtype=np.float32))
    return np.stack(out, axis=1)


def check_majorants(got, ranges, tf, what, lo=0.0, hi=1.0):
    """GPU majorants against the FP64 definition: equal wherever a range end's entry
    decision is not within FP32 rounding of an entry boundary; there, one of the
    neighbouring choices.  Everywhere: no less than the largest opacity over the
    range, and 0 only where the table is transparent over the whole range."""
    want = oracle.majorants(ranges, tf, lo, hi)
    amb = oracle.entry_decision_ambiguous(ranges, np.shape(tf)[0], lo, hi)
    assert np.array_equal(got[~amb], want[~amb]), f"{what}: {np.count_nonzero(got[~amb] != want[~amb])} majorants differ"
    if amb.any():
        cand = _majorant_candidates(ranges[amb], tf, lo, hi)
        assert np.all(np.any(cand == got[amb][:, None], axis=1)), f"{what}: ambiguous majorant not a valid choice"
    amax = tf_alpha_max(tf, ranges, lo, hi)
    # (the FP64 lerp between two equal entries may exceed them by an ulp)
    assert np.all(got.astype(np.float64) >= amax * (1 - 1e-12)), f"{what}: a majorant below the range's opacity"
    assert np.all(amax[got == 0.0] == 0.0), f"{what}: a zero majorant over an opaque range"
    return int(np.count_nonzero(amb))


def check_iso_classes(got, ranges, tf, v_iso, what, lo=0.0, hi=1.0):
    """Majorants with iso-surface skip classes: positive entries are majorants
    (check_majorants); a zero majorant becomes 0 (range strictly below v_iso), -1
    (strictly above) or 1 (sample it), equal to the FP64 definition except where a
    range end lies within FP32 rounding of a decision boundary."""
    want_m = oracle.majorants(ranges, tf, lo, hi)
    want = oracle.iso_classes(ranges, want_m, v_iso)
    amb = oracle.entry_decision_ambiguous(ranges, np.shape(tf)[0], lo, hi) | oracle.iso_class_ambiguous(ranges, v_iso)
    assert np.array_equal(got[~amb], want[~amb]), f"{what}: {np.count_nonzero(got[~amb] != want[~amb])} classes differ"
    pos = got > 0
    amax = tf_alpha_max(tf, ranges, lo, hi)
    assert np.all(got[pos].astype(np.float64) >= amax[pos] * (1 - 1e-12)), f"{what}: a majorant below the range's opacity"
    cls = ~pos
    assert np.all(amax[cls] == 0.0), f"{what}: a skip class over an opaque range"
    r64 = ranges.astype(np.float64)
    assert np.all(r64[got == 0.0][:, 1] < v_iso), f"{what}: class 0 with a value at or above v_iso"
    assert np.all(r64[got == -1.0][:, 0] > v_iso), f"{what}: class -1 with a value below v_iso"
    assert np.all(np.isin(got[cls], np.array([0.0, -1.0, 1.0], dtype=np.float32))), f"{what}: unknown class"
    return int(np.count_nonzero(amb))
