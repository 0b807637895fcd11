"""GPU tests of the persistent batched renderer (work queue + HIP graph + autotuned tiles)."""

import numpy as np
import pytest

import oracle
from oracle import RenderParams
from synth import Camera, fibonacci_cameras, kd_split, make_blobs, make_tf, make_volume_small
from tests.gpu_util import TOL_F32, frame_np, log, make_world, oracle_brick

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpr():
    import paper_2407_00179_amd as m
    return m


def _scene(dtype=np.float32, dims=(56, 48, 40), nb=7, seed=61):
    vol = make_volume_small(dims, make_blobs(dims, seed, 6, (0.06, 0.2)), seed + 1, 0.02, dtype)
    boxes = kd_split(dims, nb, seed=seed, max_ratio=4.0)
    return dims, vol, boxes, make_tf(2001)


def _cams(dims):
    cams = fibonacci_cameras(dims, 3, 96, 80)
    cams[1] = Camera(cams[1].eye, cams[1].center, cams[1].up, 50.0, 131, 67)   # ragged size
    cams.append(Camera((0.45, 0.4, 0.35), (1.5, 1.2, 0.9), (0.0, 0.0, 1.0), 80.0, 70, 70))  # eye inside
    return cams


def _reference(dpr, dev, w, cams):
    outs = []
    for c in cams:
        w.set_camera(c)
        f = dpr.Frame(dev, c.width, c.height)
        w.render_frame(f)
        outs.append(frame_np(f)[:2])
        f.release()
    return outs


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("ert", [0.99, 1.0])
def test_batch_equals_render_frame_bitwise(gpu_lib, dpr, dtype, ert):
    dims, vol, boxes, tf = _scene(dtype)
    prm = RenderParams(0.5, ert, 25.0)
    cams = _cams(dims)
    log(f"batch {dtype.__name__} ert {ert}: {len(boxes)} bricks, {len(cams)} cameras")
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cams[0], mc=8)
    ref = _reference(dpr, gpu_lib, w, cams)
    frames = [dpr.Frame(gpu_lib, c.width, c.height) for c in cams]
    for flags, what in ((0, "graph"), (dpr.FLAG_NO_GRAPH, "direct"), (dpr.FLAG_PLAIN, "plain")):
        for f in frames:
            f.rgba.fill_(-1.0)
            f.depth.fill_(-1.0)
        w.render_batch(cams, frames, flags)
        for c, f in enumerate(frames):
            got = frame_np(f)[:2]
            assert np.array_equal(got[0], ref[c][0]), (what, c, np.max(np.abs(got[0] - ref[c][0])))
            assert np.array_equal(got[1], ref[c][1]), (what, c)
    w.release()


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
def test_wide_offsets_and_f16_layouts_bitwise(gpu_lib, dpr, dtype):
    """Voxel offsets formed in 64 bits (the path of bricks of 4 GiB or more, forced
    here on small bricks) and FP16 bricks stored as 2-byte voxels instead of voxel
    pairs (automatic from 4 GiB pair copies, forced here) give the same bits as
    32-bit offsets into voxel pairs, per brick and batched."""
    dims, vol, boxes, tf = _scene(dtype)
    prm = RenderParams(0.5, 0.99, 25.0)
    cams = _cams(dims)
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cams[0], mc=8)
    frames = [dpr.Frame(gpu_lib, c.width, c.height) for c in cams]
    res = []
    variants = (0, dpr.FLAG_WIDE_OFFSETS, dpr.FLAG_F16_HALVES, dpr.FLAG_F16_HALVES | dpr.FLAG_WIDE_OFFSETS)
    for flags in variants:
        w.set_params(dpr.Params(prm.step_voxels, prm.ert, 8, flags))
        w.commit()
        w.render_batch(cams, frames)
        batch = [frame_np(f)[:2] for f in frames]
        w.render_batch(cams, frames, dpr.FLAG_PLAIN)
        plain = [frame_np(f)[:2] for f in frames]
        res.append((batch, plain))
    b0, p0 = res[0]
    for v, (b1, p1) in zip(variants[1:], res[1:]):
        for c in range(len(cams)):
            assert np.array_equal(b0[c][0], b1[c][0]) and np.array_equal(b0[c][1], b1[c][1]), (v, c)
            assert np.array_equal(p0[c][0], p1[c][0]) and np.array_equal(p0[c][1], p1[c][1]), (v, c)
    for c in range(len(cams)):
        assert np.array_equal(b0[c][0], p0[c][0]), c
    w.release()


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("iso", [None, 0.45])
def test_partial_through_persistent_kernel_equals_plain_launch(gpu_lib, dpr, dtype, iso):
    """dpr_render_partial goes through the persistent kernel (one cached item list
    per brick, graph-replayed or enqueued directly); the plain one-thread-per-pixel
    launch (DPR_FLAG_PLAIN) gives the same bits for every brick, camera and tile
    shape, including bricks off screen and a camera inside the volume."""
    dims, vol, boxes, tf = _scene(dtype)
    prm = RenderParams(0.5, 0.99, 25.0)
    cams = _cams(dims)
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cams[0], mc=8)
    if iso is not None:
        w.set_isosurface(iso)
    for ci, c in enumerate(cams):
        w.set_camera(c)
        got = dpr.Frame(gpu_lib, c.width, c.height)
        ref = dpr.Frame(gpu_lib, c.width, c.height)
        for tile, flags in (((8, 8), 0), ((16, 16), dpr.FLAG_NO_GRAPH)):
            w.set_batch_tile(*tile)
            for i in range(len(boxes)):
                got.rgba.fill_(-1.0)
                got.depth.fill_(-1.0)
                w.set_params(dpr.Params(prm.step_voxels, prm.ert, 8, flags))
                w.render_partial(i, got)
                w.set_params(dpr.Params(prm.step_voxels, prm.ert, 8, dpr.FLAG_PLAIN))
                w.render_partial(i, ref)
                g, r = frame_np(got)[:2], frame_np(ref)[:2]
                assert np.array_equal(g[0], r[0]) and np.array_equal(g[1], r[1]), (ci, tile, i)
        got.release()
        ref.release()
    w.release()


def test_graph_replays_stay_exact(gpu_lib, dpr):
    import torch
    dims, vol, boxes, tf = _scene()
    prm = RenderParams(0.5, 0.99, 25.0)
    cams = _cams(dims)
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cams[0], mc=8)
    ref = _reference(dpr, gpu_lib, w, cams)
    frames = [dpr.Frame(gpu_lib, c.width, c.height) for c in cams]
    for rep in range(5):
        for f in frames:
            f.rgba.fill_(float(rep))          # eager work between replays
        junk = torch.randn(1 << 20, device=gpu_lib.torch_device).sum().item()
        assert np.isfinite(junk)
        w.render_batch(cams, frames)
        for c, f in enumerate(frames):
            got = frame_np(f)[:2]
            assert np.array_equal(got[0], ref[c][0]) and np.array_equal(got[1], ref[c][1]), (rep, c)
    # a new transfer function invalidates the captured graph
    tf2 = make_tf(77)
    w.set_transfer_function(tf2, 0.0, 1.0, 25.0)
    ref2 = _reference(dpr, gpu_lib, w, cams)
    w.render_batch(cams, frames)
    for c, f in enumerate(frames):
        assert np.array_equal(frame_np(f)[0], ref2[c][0])
    w.release()


def test_autotune_and_tile_shapes(gpu_lib, dpr):
    dims, vol, boxes, tf = _scene(np.float16)
    prm = RenderParams(0.5, 0.99, 25.0)
    cams = _cams(dims)
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cams[0], mc=8)
    ref = _reference(dpr, gpu_lib, w, cams)
    frames = [dpr.Frame(gpu_lib, c.width, c.height) for c in cams]
    tw, th = w.autotune_batch(cams, frames)
    log(f"autotuned tile {tw}x{th}")
    assert (tw * th) % 64 == 0
    for shape in ((8, 8), (32, 16), (64, 1), (tw, th)):
        w.set_batch_tile(*shape)
        w.render_batch(cams, frames)
        for c, f in enumerate(frames):
            assert np.array_equal(frame_np(f)[0], ref[c][0]), (shape, c)
    with pytest.raises(dpr.DprError):
        w.set_batch_tile(7, 7)
    with pytest.raises(dpr.DprError):
        w.set_batch_tile(64, 32)
    w.release()


def test_batch_against_oracle(gpu_lib, dpr):
    dims, vol, boxes, tf = _scene()
    prm = RenderParams(0.5, 1.0, 25.0)
    cams = _cams(dims)[:2]
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cams[0], mc=8)
    frames = [dpr.Frame(gpu_lib, c.width, c.height) for c in cams]
    w.render_batch(cams, frames)
    for c, f in zip(cams, frames):
        py, px = np.mgrid[0:c.height, 0:c.width]
        px, py = px.ravel(), py.ravel()
        orc = [oracle_brick(vol, dims, lo, hi, tf, prm, c, px, py) for lo, hi in boxes]
        want, wz = oracle.composite(np.stack([o[0] for o in orc]), np.stack([o[1] for o in orc]))
        got, gz, _ = frame_np(f)
        err = np.max(np.abs(got - want))
        log(f"  batch vs oracle {c.width}x{c.height}: {err:.3e}")
        assert err <= TOL_F32
        fin = np.isfinite(wz)
        assert np.array_equal(np.isfinite(gz), fin)
    w.release()


def test_render_frame_paths_and_timings(gpu_lib, dpr):
    """render_frame (batched by default) equals the plain per-brick path bit for bit,
    and the in-graph HIP event timings are available afterwards."""
    dims, vol, boxes, tf = _scene(np.float16)
    prm = RenderParams(0.5, 0.99, 25.0)
    cam = _cams(dims)[1]
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, mc=8)
    with pytest.raises(dpr.DprError):
        w.batch_timings()
    a = dpr.Frame(gpu_lib, cam.width, cam.height)
    w.render_frame(a)                      # graph replay: no per-kernel timings
    with pytest.raises(dpr.DprError):
        w.batch_timings()
    w.set_params(dpr.Params(0.5, 0.99, 8, dpr.FLAG_NO_GRAPH))
    c = dpr.Frame(gpu_lib, cam.width, cam.height)
    w.render_frame(c)
    march_ms, comp_ms = w.batch_timings()
    assert march_ms > 0 and comp_ms > 0
    rc, zc, _ = frame_np(c)
    w.set_params(dpr.Params(0.5, 0.99, 8, dpr.FLAG_PLAIN))
    b = dpr.Frame(gpu_lib, cam.width, cam.height)
    w.render_frame(b)
    ra, za, _ = frame_np(a)
    rb, zb, _ = frame_np(b)
    assert np.array_equal(ra, rb) and np.array_equal(za, zb)
    assert np.array_equal(ra, rc) and np.array_equal(za, zc)
    w.release()


def test_batch_empty_views_and_tiny_frames(gpu_lib, dpr):
    """A camera that sees no brick (no items for it), next to ones that do, and a
    1x1 frame: every path gives empty fragments where nothing is hit and equals
    render_frame elsewhere."""
    dims, vol, boxes, tf = _scene()
    prm = RenderParams(0.5, 0.99, 25.0)
    cams = _cams(dims)[:2]
    # every brick behind the eye: the whole screen is queued, every ray misses
    behind = Camera((-1.0, -1.0, -1.0), (-2.0, -2.5, -3.0), (0.0, 0.0, 1.0), 40.0, 33, 21)
    # the volume in front of the eye but outside the view: no item at all
    aside = Camera((-5.0, 5.0, 0.4), (0.0, 5.0, 0.4), (0.0, 0.0, 1.0), 30.0, 29, 17)
    tiny = Camera(cams[0].eye, cams[0].center, cams[0].up, 30.0, 1, 1)
    cams = [cams[0], behind, cams[1], aside, tiny]
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cams[0], mc=8)
    ref = _reference(dpr, gpu_lib, w, cams)
    for c in (1, 3):
        assert np.all(ref[c][0] == 0.0) and np.all(np.isinf(ref[c][1]))
    frames = [dpr.Frame(gpu_lib, c.width, c.height) for c in cams]
    for flags in (0, dpr.FLAG_NO_GRAPH, dpr.FLAG_PLAIN):
        for f in frames:
            f.rgba.fill_(-1.0)
            f.depth.fill_(-1.0)
        w.render_batch(cams, frames, flags)
        for c, f in enumerate(frames):
            got = frame_np(f)[:2]
            assert np.array_equal(got[0], ref[c][0]) and np.array_equal(got[1], ref[c][1]), (flags, c)
    # only the camera whose view holds no brick: an empty item queue
    frames[3].rgba.fill_(-1.0)
    w.render_batch([aside], [frames[3]])
    got = frame_np(frames[3])[:2]
    assert np.all(got[0] == 0.0) and np.all(np.isinf(got[1]))
    w.release()


def test_batch_refresh_after_recommit(gpu_lib, dpr):
    """Same geometry, new macrocell size and a recommit: the cached batch refreshes
    its brick views (new macrocell grids) and matches a freshly built world."""
    dims, vol, boxes, tf = _scene()
    prm = RenderParams(0.5, 0.99, 25.0)
    cams = _cams(dims)[:2]
    frames = [dpr.Frame(gpu_lib, c.width, c.height) for c in cams]
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cams[0], mc=8)
    w.render_batch(cams, frames)
    w.set_params(dpr.Params(0.5, 0.99, 4, 0))
    w.commit()
    w.render_batch(cams, frames)
    got = [frame_np(f)[:2] for f in frames]
    w2 = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cams[0], mc=4)
    want = _reference(dpr, gpu_lib, w2, cams)
    for c in range(len(cams)):
        assert np.array_equal(got[c][0], want[c][0]) and np.array_equal(got[c][1], want[c][1]), c
    w.release()
    w2.release()


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
def test_queue_coverage(gpu_lib, dpr, dtype):
    """With the queue-coverage counters on, every (camera, brick, tile) item of the
    persistent queue is taken exactly once and every fragment slot written exactly
    once -- for a 4-camera batch over 7 uneven bricks (ragged frame, eye inside the
    volume), for dpr_render_frame and for one brick's dpr_render_partial -- and the
    frames are the same bits as without the counters."""
    dims, vol, boxes, tf = _scene(dtype)
    prm = RenderParams(0.5, 0.99, 20.0)
    cams = _cams(dims)
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cams[0])
    frames = [dpr.Frame(gpu_lib, c.width, c.height) for c in cams]
    w.render_batch(cams, frames)
    want = [frame_np(f)[:2] for f in frames]
    w.render_batch(cams, frames, flags=dpr.FLAG_QUEUE_COVERAGE)
    items, items_once, slots, slots_once = w.batch_coverage()
    log(f"  batch: {items} items, {slots} fragment slots")
    assert items > len(boxes) and items_once == items and slots_once == slots == items * 64
    for f, (a, b) in zip(frames, want):
        got = frame_np(f)[:2]
        assert np.array_equal(got[0], a) and np.array_equal(got[1], b)
    w.render_batch(cams, frames)   # a graph replay counts nothing
    with pytest.raises(dpr.DprError):
        w.batch_coverage()
    w.set_params(dpr.Params(prm.step_voxels, prm.ert, 16, dpr.FLAG_QUEUE_COVERAGE))
    w.set_camera(cams[2])
    w.render_frame(frames[2])
    items, items_once, slots, slots_once = w.batch_coverage()
    assert items_once == items > 0 and slots_once == slots
    assert all(np.array_equal(x, y) for x, y in zip(frame_np(frames[2])[:2], want[2]))
    part = dpr.Frame(gpu_lib, cams[2].width, cams[2].height)
    w.render_partial(3, part)
    items, items_once, slots, slots_once = w.batch_coverage()
    assert items_once == items > 0 and slots_once == slots
    for f in frames + [part]:
        f.release()
    w.release()


def test_autotune_cache(gpu_lib, dpr, tmp_path, monkeypatch):
    """With DPR_TUNE_CACHE set, the autotuner stores its choice under a key of the
    device and the shape of the work, and a later call for the same shape takes
    the stored shape without timing (shown by planting another shape)."""
    import json
    dims, vol, boxes, tf = _scene()
    prm = RenderParams(0.5, 0.99, 20.0)
    cams = _cams(dims)[:2]
    path = tmp_path / "tiles.json"
    monkeypatch.setenv("DPR_TUNE_CACHE", str(path))
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cams[0])
    frames = [dpr.Frame(gpu_lib, c.width, c.height) for c in cams]
    tw, th = w.autotune_batch(cams, frames)
    entries = json.loads(path.read_text())["entries"]
    assert list(entries.values()) == [[tw, th]]
    key = next(iter(entries))
    log(f"  cache key {key!r} -> {tw}x{th}")
    assert key.startswith("gfx950 cu") and "cameras 96x80 131x67" in key
    other = (32, 32) if (tw, th) != (32, 32) else (8, 8)
    dpr.check(dpr.lib.dpr_tune_cache_store(str(path).encode(), key.encode(), *other))
    w2 = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cams[0])
    assert w2.autotune_batch(cams, frames) == other
    ref = [frame_np(f)[:2] for f in frames]
    w.render_batch(cams, frames)
    assert all(np.array_equal(a[0], frame_np(f)[0]) for a, f in zip(ref, frames))
    for f in frames:
        f.release()
    w.release()
    w2.release()
