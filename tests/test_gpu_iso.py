"""GPU parity of iso-surface fragments mixed with the emission-absorption march
(reading C20/C21 of oracle/iso.py; the paper's iso-surface figures Fig. 1c,
Fig. 3c and Fig. 4, local render per section 5.1.2).

Where floating point decides the side of a sample the GPU takes it in FP32 and
the oracle in FP64; a pixel whose oracle samples come within MARGIN of the iso
value may be decided either way, so it is left out of the elementwise
comparison, and such pixels must be rare (at most 0.5%)."""

import numpy as np
import pytest

import oracle
from oracle import IsoParams, RenderParams
from synth import even_split, kd_split, make_blobs, make_tf, make_volume_small, orbit_camera
from tests.gpu_util import TOL_F16, TOL_F32, check_iso_classes, check_majorants, frame_np, log, make_world

pytestmark = pytest.mark.gpu

MARGIN = 1e-5


@pytest.fixture(scope="module")
def dpr():
    import paper_2407_00179_amd as m
    return m


def _volume(dims, seed, dtype=np.float32):
    return make_volume_small(dims, make_blobs(dims, seed, 7, (0.06, 0.25)), seed + 1, 0.02, dtype)


def _tf(seed, cut=0.35):
    """Random TF, transparent below `cut`: large empty regions for skipping."""
    tf = make_tf(seed).astype(np.float32)
    tf[: int(cut * (tf.shape[0] - 1)), 3] = 0.0
    return tf


def _iso_world(dpr, dev, vol, dims, boxes, tf, prm, cam, iso, mc=8, flags=0):
    w = make_world(dpr, dev, vol, dims, boxes, tf, prm, cam, mc=mc, flags=flags)
    w.set_isosurface(iso.value, iso.ambient, iso.diffuse)
    return w


def _compare(got, want, margin, tol, what):
    clear = margin > MARGIN
    err = np.max(np.abs(got[clear] - want[clear])) if clear.any() else 0.0
    amb = int((~clear).sum())
    log(f"  {what}: max|gpu-oracle| = {err:.3e} on {clear.sum()} pixels, {amb} within {MARGIN:g} of the iso value")
    assert err <= tol, what
    assert amb <= max(2, 0.005 * got.shape[0]), what
    return clear


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
def test_partial_frames_match_oracle(gpu_lib, dpr, dtype):
    dims = (52, 44, 36)
    vol = _volume(dims, 41, dtype)
    tf = _tf(2001)
    prm = RenderParams(0.5, 1.0, 25.0)
    iso = IsoParams(0.55, 0.3, 0.7)
    cam = orbit_camera(dims, 72, 60, dist=1.7)
    boxes = kd_split(dims, 7, seed=4, max_ratio=4.0)
    w = _iso_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, iso)
    px, py = [a.ravel() for a in np.meshgrid(np.arange(cam.width), np.arange(cam.height))]
    tol = TOL_F16 if dtype == np.float16 else TOL_F32
    n_surf = 0
    for i, (lo, hi) in enumerate(boxes):
        f = dpr.Frame(gpu_lib, cam.width, cam.height, counts=True)
        w.render_partial(i, f)
        got, gz, gn = frame_np(f)
        from synth import extract_brick
        b = extract_brick(vol, dims, lo, hi, 1)
        want, wz, wn, mg = oracle.render_brick_iso(b.data, b.stored_lo, dims, lo, hi, tf, prm, iso, cam, px, py)
        clear = _compare(got, want, mg, tol, f"brick {i}")
        assert np.array_equal(np.isfinite(gz), np.isfinite(wz))
        assert np.array_equal(gn[clear], wn[clear])
        n_surf += int((got[:, 3] == 1.0).sum())
        f.release()
    assert n_surf > 200
    w.release()


def test_skip_batch_graph_bitwise(gpu_lib, dpr):
    """Skipping with iso classes, the batched persistent march and graph replays
    give the same bits as the plain march without skipping."""
    dims = (64, 56, 48)
    vol = _volume(dims, 51)
    tf = _tf(2002, cut=0.5)
    prm = RenderParams(0.5, 0.99, 25.0)
    iso = IsoParams(0.45)
    cam = orbit_camera(dims, 96, 80, dist=1.8)
    boxes = kd_split(dims, 9, seed=6, max_ratio=4.0)
    out = {}
    for name, flags in (("plain_noskip", dpr.FLAG_PLAIN | dpr.FLAG_NO_SKIP), ("plain", dpr.FLAG_PLAIN),
                        ("batch", 0), ("batch_direct", dpr.FLAG_NO_GRAPH), ("batch_noskip", dpr.FLAG_NO_SKIP)):
        w = _iso_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, iso, flags=flags)
        f = dpr.Frame(gpu_lib, cam.width, cam.height)
        for _ in range(3):                       # capture, then replays
            w.render_frame(f)
            out.setdefault(name, []).append(frame_np(f)[:2])
        f.release()
        w.release()
    ref = out["plain_noskip"][0]
    assert (ref[0][:, 3] == 1.0).sum() > 300
    for name, reps in out.items():
        for r in reps:
            assert np.array_equal(r[0], ref[0]) and np.array_equal(r[1], ref[1]), name


def test_split_volume_gives_the_unsplit_image(gpu_lib, dpr):
    dims = (48, 40, 36)
    vol = _volume(dims, 61)
    tf = _tf(2003)
    prm = RenderParams(0.5, 1.0, 20.0)
    iso = IsoParams(0.5, 0.25, 0.75)
    cam = orbit_camera(dims, 80, 64, dist=1.7)
    px, py = [a.ravel() for a in np.meshgrid(np.arange(cam.width), np.arange(cam.height))]
    want, wz, _, mg = oracle.render_image_iso(vol, dims, tf, prm, iso, cam, px, py)
    frames = []
    for boxes in ([((0, 0, 0), dims)], even_split(dims, (2, 2, 2)), kd_split(dims, 11, seed=9, max_ratio=3.0)):
        w = _iso_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, iso)
        f = dpr.Frame(gpu_lib, cam.width, cam.height)
        w.render_frame(f)
        got, gz, _ = frame_np(f)
        _compare(got, want, mg, TOL_F32, f"{len(boxes)} bricks")
        assert np.array_equal(np.isfinite(gz), np.isfinite(wz))
        frames.append(got)
        f.release()
        w.release()
    assert (want[:, 3] == 1.0).sum() > 300
    for g in frames[1:]:
        assert np.max(np.abs(g - frames[0])) <= TOL_F32


def test_surface_ranks_mixed_with_volume_ranks(gpu_lib, dpr):
    """Rank A renders its half of the volume with the surface, rank B its half as
    volume only; the sort-last composite of their frames is the oracle composite of
    the per-brick fragments of each kind."""
    dims = (48, 40, 32)
    vol = _volume(dims, 71)
    tf = _tf(2004)
    prm = RenderParams(0.5, 1.0, 20.0)
    iso = IsoParams(0.5)
    cam = orbit_camera(dims, 64, 56, az_deg=75.0, dist=1.7)
    half_a = [((0, 0, 0), (24, 20, 32)), ((0, 20, 0), (24, 40, 32))]
    half_b = [((24, 0, 0), (48, 40, 16)), ((24, 0, 16), (48, 40, 32))]
    wa = _iso_world(dpr, gpu_lib, vol, dims, half_a, tf, prm, cam, iso)
    wb = make_world(dpr, gpu_lib, vol, dims, half_b, tf, prm, cam, mc=8)
    fa, fb, out = (dpr.Frame(gpu_lib, cam.width, cam.height) for _ in range(3))
    wa.render_frame(fa)
    wb.render_frame(fb)
    dpr.composite(gpu_lib, [fa, fb], out, ids=[0, 1])
    got, gz, _ = frame_np(out)
    px, py = [a.ravel() for a in np.meshgrid(np.arange(cam.width), np.arange(cam.height))]
    from synth import extract_brick
    rr, zz, mgs = [], [], []
    for lo, hi in half_a:
        b = extract_brick(vol, dims, lo, hi, 1)
        r, z, _, mg = oracle.render_brick_iso(b.data, b.stored_lo, dims, lo, hi, tf, prm, iso, cam, px, py)
        rr.append(r)
        zz.append(z)
        mgs.append(mg)
    for lo, hi in half_b:
        b = extract_brick(vol, dims, lo, hi, 1)
        r, z, _ = oracle.render_brick(b.data, b.stored_lo, dims, lo, hi, tf, prm, cam, px, py)
        rr.append(r)
        zz.append(z)
    want, wz = oracle.composite(np.stack(rr), np.stack(zz))
    _compare(got, want, np.minimum(*mgs), TOL_F32, "mixed composite")
    assert (got[:, 3] == 1.0).sum() > 100 and ((got[:, 3] > 0) & (got[:, 3] < 1)).sum() > 100
    for h in (wa, wb, fa, fb, out):
        h.release()


def test_macrocell_iso_classes_bitwise(gpu_lib, dpr):
    dims = (70, 40, 33)
    vol = _volume(dims, 81)
    tf = _tf(2005, cut=0.6)
    prm = RenderParams(0.5, 0.99, 20.0)
    cam = orbit_camera(dims, 16, 16)
    boxes = kd_split(dims, 5, seed=2, max_ratio=4.0)
    seen = set()
    for mc in (4, 8, 16):
        w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, mc=mc)
        for v_iso in (0.3, 0.55):
            w.set_isosurface(v_iso)
            f = dpr.Frame(gpu_lib, cam.width, cam.height)
            w.render_frame(f)                     # builds the classes
            f.release()
            for i in range(len(boxes)):
                rng_, maj = w.macrocells(i)
                check_iso_classes(maj, rng_, tf, v_iso, f"mc {mc} iso {v_iso} brick {i}")
                seen |= set(np.unique(maj).tolist())
        w.set_isosurface(None)
        f = dpr.Frame(gpu_lib, cam.width, cam.height)
        w.render_frame(f)
        f.release()
        for i in range(len(boxes)):
            rng_, maj = w.macrocells(i)
            check_majorants(maj, rng_, tf, f"mc {mc} brick {i}, surface off")
        w.release()
    assert {0.0, -1.0, 1.0} <= seen


def test_interleaved_ranks_with_surface_deep(gpu_lib, dpr):
    """Interleaved (non-convex) ranks with the surface: deep frames merge to the
    unsplit iso image."""
    dims = (40, 40, 40)
    vol = _volume(dims, 91)
    tf = _tf(2006)
    prm = RenderParams(0.5, 1.0, 20.0)
    iso = IsoParams(0.5)
    cam = orbit_camera(dims, 64, 56, dist=1.7)
    boxes = even_split(dims, (4, 4, 4))
    owner = np.random.default_rng(8).integers(0, 3, size=len(boxes))
    deeps, worlds = [], []
    for r in range(3):
        mine = [boxes[i] for i in range(len(boxes)) if owner[i] == r]
        w = _iso_world(dpr, gpu_lib, vol, dims, mine, tf, prm, cam, iso)
        d = dpr.DeepFrame(gpu_lib, cam.width, cam.height, len(mine))
        w.render_deep(r, d)
        deeps.append(d)
        worlds.append(w)
    out = dpr.Frame(gpu_lib, cam.width, cam.height)
    dpr.composite_deep(gpu_lib, deeps, out)
    got, _, _ = frame_np(out)
    px, py = [a.ravel() for a in np.meshgrid(np.arange(cam.width), np.arange(cam.height))]
    want, _, _, mg = oracle.render_image_iso(vol, dims, tf, prm, iso, cam, px, py)
    _compare(got, want, mg, TOL_F32, "deep composite with surface")
    assert (want[:, 3] == 1.0).sum() > 200
    for h in deeps + worlds + [out]:
        h.release()


def test_set_isosurface_errors(gpu_lib, dpr):
    dims = (16, 16, 16)
    vol = _volume(dims, 3)
    w = make_world(dpr, gpu_lib, vol, dims, [((0, 0, 0), dims)], _tf(1), RenderParams(0.5, 0.99, 20.0),
                   orbit_camera(dims, 8, 8))
    with pytest.raises(dpr.DprError):
        w.set_isosurface(float("nan"))
    with pytest.raises(dpr.DprError):
        w.set_isosurface(0.5, -0.1, 0.5)
    with pytest.raises(dpr.DprError):
        w.set_isosurface(0.5, 0.1, float("inf"))
    w.set_isosurface(None)
    w.release()
