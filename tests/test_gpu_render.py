"""GPU parity of the per-brick ray march, macrocells and render_frame against the oracle."""

import numpy as np
import pytest

import oracle
from oracle import RenderParams
from synth import (Camera, even_split, extract_brick, get_config, kd_split, make_blobs, make_tf, make_volume_small,
                   orbit_camera)
from tests.gpu_util import (ERT_DELTA, TOL_F16, TOL_F32, check_bracketed, check_majorants, check_partials_and_frame, frame_np,
                            log, make_world, oracle_brick, pc10_subset)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpr():
    import paper_2407_00179_amd as m
    return m


def _small_case(dims=(40, 36, 28), seed=3, nb=6, dtype=np.float32):
    vol = make_volume_small(dims, make_blobs(dims, seed, nb, (0.08, 0.25)), seed + 1, 0.02, dtype)
    return vol, make_tf(2001)


@pytest.mark.parametrize("ert", [1.0, 0.99])
@pytest.mark.parametrize("size", [(64, 48), (37, 29), (1, 1), (130, 17)])
def test_single_brick_full_frame(gpu_lib, dpr, ert, size):
    dims = (40, 36, 28)
    vol, tf = _small_case(dims)
    prm = RenderParams(0.5, ert, 20.0)
    cam = orbit_camera(dims, *size)
    log(f"single brick {dims} image {size} ert {ert}")
    w = make_world(dpr, gpu_lib, vol, dims, [((0, 0, 0), dims)], tf, prm, cam)
    fr = dpr.Frame(gpu_lib, *size, counts=True)
    w.render_partial(0, fr)
    rgba, depth, n = frame_np(fr)
    py, px = np.mgrid[0:size[1], 0:size[0]]
    px, py = px.ravel(), py.ravel()
    check_bracketed(rgba, depth, n, lambda th: oracle_brick(vol, dims, (0, 0, 0), dims, tf, prm, cam, px, py, th),
                    ert, TOL_F32, f"1 brick {size}")
    w.release()


def test_cfg1_full(gpu_lib, dpr):
    cfg = get_config("cfg1")
    dims = cfg.dims
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range)
    vol = make_volume_small(dims, blobs, cfg.seeds["volume"], cfg.noise_amp)
    tf = make_tf(cfg.seeds["tf"])
    prm = RenderParams(cfg.step_voxels, cfg.ert, cfg.density)
    cam = orbit_camera(dims, *cfg.image)
    log("cfg1 64^3 256x256")
    w = make_world(dpr, gpu_lib, vol, dims, [((0, 0, 0), dims)], tf, prm, cam)
    fr = dpr.Frame(gpu_lib, *cfg.image, counts=True)
    w.render_partial(0, fr)
    rgba, depth, n = frame_np(fr)
    py, px = np.mgrid[0:cfg.image[1], 0:cfg.image[0]]
    px, py = px.ravel(), py.ravel()
    check_bracketed(rgba, depth, n, lambda th: oracle_brick(vol, dims, (0, 0, 0), dims, tf, prm, cam, px, py, th),
                    cfg.ert, TOL_F32, "cfg1")
    assert rgba[:, 3].max() > 0.9
    w.release()


@pytest.mark.parametrize("split", ["2x2x2", "kd7", "3x2x1"])
@pytest.mark.parametrize("ert", [1.0, 0.99])
def test_bricks_partials_and_frame(gpu_lib, dpr, split, ert):
    dims = (48, 40, 33)
    vol, tf = _small_case(dims, seed=11)
    prm = RenderParams(0.5, ert, 25.0)
    cam = orbit_camera(dims, 72, 61)
    boxes = (kd_split(dims, 7, seed=3, max_ratio=6.0) if split == "kd7"
             else even_split(dims, tuple(int(c) for c in split.split("x"))))
    log(f"bricks {split} ert {ert}")
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, mc=8)
    py, px = np.mgrid[0:cam.height, 0:cam.width]
    px, py = px.ravel(), py.ravel()
    parts = []
    for i, (lo, hi) in enumerate(boxes):
        fr = dpr.Frame(gpu_lib, cam.width, cam.height, counts=True)
        w.render_partial(i, fr)
        rgba, depth, n = frame_np(fr)
        check_bracketed(rgba, depth, n, lambda th: oracle_brick(vol, dims, lo, hi, tf, prm, cam, px, py, th),
                        ert, TOL_F32, f"brick {i}")
        parts.append(fr)
    out = dpr.Frame(gpu_lib, cam.width, cam.height)
    w.render_frame(out)
    got, gz, _ = frame_np(out)
    # the composite of the GPU's own partials through dpr_composite matches render_frame bitwise
    out2 = dpr.Frame(gpu_lib, cam.width, cam.height)
    dpr.composite(gpu_lib, parts[::-1], out2, ids=list(range(len(parts)))[::-1])
    got2, gz2, _ = frame_np(out2)
    assert np.array_equal(got, got2) and np.array_equal(gz, gz2)
    # versus the oracle's composite of the oracle's partials
    orc = [oracle_brick(vol, dims, lo, hi, tf, prm, cam, px, py) for lo, hi in boxes]
    want, wz = oracle.composite(np.stack([o[0] for o in orc]), np.stack([o[1] for o in orc]))
    if ert >= 1.0:
        err = np.max(np.abs(got - want))
        assert err <= TOL_F32, err
        # split invariant on the GPU: composite == unsplit render (ERT off)
        wu = make_world(dpr, gpu_lib, vol, dims, [((0, 0, 0), dims)], tf, prm, cam)
        un = dpr.Frame(gpu_lib, cam.width, cam.height)
        wu.render_partial(0, un)
        gu, guz, _ = frame_np(un)
        inv = np.max(np.abs(got - gu))
        log(f"  composite vs oracle {err:.3e}; GPU split invariant |composite - unsplit| = {inv:.3e}")
        assert inv <= TOL_F32
        fin = np.isfinite(guz)
        assert np.array_equal(np.isfinite(gz), fin) and np.allclose(gz[fin], guz[fin], rtol=3e-7, atol=0)
        wu.release()
    else:
        # per-brick ERT: every partial already matched its bracket.  Where no
        # brick's termination step is ambiguous (its partial is the same at
        # theta -+ delta) the frame matches the oracle's composite at the FP32 bar;
        # everywhere it matches the oracle compositor applied to the GPU partials.
        amb = np.zeros(px.size, dtype=bool)
        for lo, hi in boxes:
            a = oracle_brick(vol, dims, lo, hi, tf, prm, cam, px, py, ert - ERT_DELTA)[0]
            b = oracle_brick(vol, dims, lo, hi, tf, prm, cam, px, py, ert + ERT_DELTA)[0]
            amb |= np.any(a != b, axis=1)
        ok = ~amb
        err = np.max(np.abs(got[ok] - want[ok]))
        pr = [frame_np(f) for f in parts]
        mine, _ = oracle.composite(np.stack([r for r, _, _ in pr]), np.stack([z for _, z, _ in pr]))
        err_g = np.max(np.abs(got - mine))
        log(f"  composite (ERT {ert}) vs oracle composite {err:.3e} on {np.count_nonzero(ok)} unambiguous of "
            f"{px.size} pixels; vs oracle compositor on the GPU partials {err_g:.3e}")
        assert err <= TOL_F32 and err_g <= TOL_F32
        assert np.count_nonzero(ok) >= px.size // 2
    w.release()


@pytest.mark.parametrize("dtype,base", [(np.float32, 0), (np.float16, 0), (np.float16, 0x10)])
def test_skip_is_bitwise_neutral(gpu_lib, dpr, dtype, base):
    dims = (64, 56, 48)
    vol, tf = _small_case(dims, seed=21, nb=4, dtype=dtype)
    prm = RenderParams(0.5, 0.99, 20.0)
    cam = orbit_camera(dims, 96, 80)
    boxes = even_split(dims, (2, 1, 2))
    res = []
    for flags in (base, base | 1):
        w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, flags=flags)
        out = dpr.Frame(gpu_lib, cam.width, cam.height, counts=True)
        w.render_partial(1, out)
        res.append(frame_np(out))
        w.release()
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_macrocells_and_majorants_bitwise(gpu_lib, dpr):
    dims = (70, 45, 38)
    vol, tf = _small_case(dims, seed=31, nb=5)
    prm = RenderParams(0.5, 0.99, 20.0)
    cam = orbit_camera(dims, 16, 16)
    boxes = kd_split(dims, 5, seed=9, max_ratio=8.0)
    for mc in (16, 4):
        w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, mc=mc)
        for i, (lo, hi) in enumerate(boxes):
            b = extract_brick(vol, dims, lo, hi)
            want_r = oracle.macrocell_ranges(b.data, lo, hi, b.ghost_lo, mc)
            got_r, got_m = w.macrocells(i)
            assert np.array_equal(got_r, want_r), (mc, i)
            amb = check_majorants(got_m, want_r, tf, f"mc {mc} brick {i}")
            log(f"  mc {mc} brick {i}: {got_m.size} majorants, {amb} with an FP32-ambiguous entry range")
            assert np.any(got_m == 0.0) or mc == 16
        w.release()


@pytest.mark.parametrize("mc", [2, 64])
def test_commit_extreme_macrocell_edges(gpu_lib, dpr, mc):
    """The one-pass commit (blocked copy + ranges) at the smallest and largest
    macrocell edge, with ghost layers of 1 and 3 voxels (0 on volume faces): the
    ranges are the oracle's and every partial frame matches the oracle's."""
    dims = (45, 38, 29)
    vol, tf = _small_case(dims, seed=41, nb=4)
    prm = RenderParams(0.5, 1.0, 25.0)
    cam = orbit_camera(dims, 24, 20)
    boxes = kd_split(dims, 4, seed=5, max_ratio=4.0)
    py, px = np.mgrid[0:cam.height, 0:cam.width]
    px, py = px.ravel(), py.ravel()
    for ghost in (1, 3):
        log(f"mc {mc} ghost {ghost}")
        w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, mc=mc, ghost=ghost)
        for i, (lo, hi) in enumerate(boxes):
            b = extract_brick(vol, dims, lo, hi, ghost)
            got_r, _ = w.macrocells(i)
            assert np.array_equal(got_r, oracle.macrocell_ranges(b.data, lo, hi, b.ghost_lo, mc)), (ghost, i)
            fr = dpr.Frame(gpu_lib, cam.width, cam.height, counts=True)
            w.render_partial(i, fr)
            rgba, depth, n = frame_np(fr)
            check_bracketed(rgba, depth, n,
                            lambda th: oracle_brick(vol, dims, lo, hi, tf, prm, cam, px, py, th, ghost=ghost),
                            1.0, TOL_F32, f"mc {mc} ghost {ghost} brick {i}")
            fr.release()
        w.release()


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
def test_ghost_width_does_not_change_a_bit(gpu_lib, dpr, dtype):
    """Ghost layers of 1, 2 or 3 voxels give the same frames, and each its oracle
    ranges (a window clipped to the stored range sees more voxels of a wider ghost
    past a partial last macrocell)."""
    dims = (70, 45, 38)
    vol, tf = _small_case(dims, seed=33, nb=5, dtype=dtype)
    prm = RenderParams(0.5, 0.99, 20.0)
    cam = orbit_camera(dims, 48, 40)
    boxes = kd_split(dims, 6, seed=4, max_ratio=4.0)
    outs = []
    for ghost in (1, 2, 3):
        w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, mc=8, ghost=ghost)
        f = dpr.Frame(gpu_lib, cam.width, cam.height)
        w.render_frame(f)
        parts = []
        for i in range(len(boxes)):
            pf = dpr.Frame(gpu_lib, cam.width, cam.height)
            w.render_partial(i, pf)
            parts.append(frame_np(pf)[0])
            pf.release()
        ranges = [w.macrocells(i) for i in range(len(boxes))]
        outs.append((frame_np(f)[:2], parts, ranges))
        f.release()
        w.release()
    for frame, parts, _ in outs[1:]:
        assert np.array_equal(frame[0], outs[0][0][0]) and np.array_equal(frame[1], outs[0][0][1])
        for a, b in zip(parts, outs[0][1]):
            assert np.array_equal(a, b)
    for ghost, (_, _, ranges) in zip((1, 2, 3), outs):
        for i, (lo, hi) in enumerate(boxes):
            b = extract_brick(vol, dims, lo, hi, ghost)
            want = oracle.macrocell_ranges(b.data, lo, hi, b.ghost_lo, 8)
            assert np.array_equal(ranges[i][0], want), (ghost, i)
            check_majorants(ranges[i][1], want, tf, f"ghost {ghost} brick {i}")


@pytest.mark.parametrize("dims,dtype", [((150, 9, 7), np.float32), ((300, 8, 6), np.float16),
                                        ((520, 6, 5), np.float32), ((1100, 5, 4), np.float32)])
def test_macrocells_wide_bricks(gpu_lib, dpr, dims, dtype):
    """Brick widths that take each column count of the range builder, and x-chunked runs."""
    vol = make_volume_small(dims, make_blobs(dims, 5, 4, (0.1, 0.3)), 6, 0.05, dtype)
    tf = make_tf(2001)
    prm = RenderParams(0.5, 0.99, 20.0)
    cam = orbit_camera(dims, 8, 8)
    h = dims[0] // 2 + 3
    for boxes in ([((0, 0, 0), dims)], [((0, 0, 0), (h, dims[1], dims[2])), ((h, 0, 0), dims)]):
        for mc in (2, 16):
            w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, mc=mc)
            for i, (lo, hi) in enumerate(boxes):
                b = extract_brick(vol, dims, lo, hi)
                want_r = oracle.macrocell_ranges(b.data, lo, hi, b.ghost_lo, mc)
                got_r, got_m = w.macrocells(i)
                assert np.array_equal(got_r, want_r), (dims, len(boxes), mc, i)
                check_majorants(got_m, want_r, tf, f"{dims} {len(boxes)} bricks mc {mc} brick {i}")
            w.release()


@pytest.mark.parametrize("halves", [False, True])
def test_f16_volume(gpu_lib, dpr, halves):
    """FP16 bricks stored as voxel pairs and as 2-byte voxels."""
    dims = (50, 42, 36)
    vol, tf = _small_case(dims, seed=41, dtype=np.float16)
    prm = RenderParams(0.5, 0.99, 20.0)
    cam = orbit_camera(dims, 64, 64)
    boxes = even_split(dims, (2, 2, 1))
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, on_device=True,
                   flags=dpr.FLAG_F16_HALVES if halves else 0)
    py, px = np.mgrid[0:64, 0:64]
    px, py = px.ravel(), py.ravel()
    for i, (lo, hi) in enumerate(boxes):
        fr = dpr.Frame(gpu_lib, 64, 64, counts=True)
        w.render_partial(i, fr)
        rgba, depth, n = frame_np(fr)
        err = check_bracketed(rgba, depth, n,
                              lambda th: oracle_brick(vol, dims, lo, hi, tf, prm, cam, px, py, th),
                              prm.ert, TOL_F16, f"f16 brick {i}")
        assert err <= TOL_F32   # FP16 storage, FP32 arithmetic on identical bits
    w.release()


def test_step_and_camera_variants(gpu_lib, dpr):
    dims = (33, 31, 29)
    vol, tf = _small_case(dims, seed=51)
    cams = [Camera((0.5, 0.49, 3.1), (0.5, 0.47, 0.44), (0.0, 1.0, 0.0), 45.0, 41, 37),   # from +z
            Camera((0.4, 0.45, 0.42), (1.5, 1.0, 0.9), (0.0, 0.0, 1.0), 90.0, 40, 30)]    # eye inside
    for step in (1.0, 0.37, 0.25):
        for cam in cams:
            prm = RenderParams(step, 0.99, 30.0)
            boxes = even_split(dims, (2, 2, 2))
            w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, mc=4)
            py, px = np.mgrid[0:cam.height, 0:cam.width]
            px, py = px.ravel(), py.ravel()
            for i in (0, 7):
                lo, hi = boxes[i]
                fr = dpr.Frame(gpu_lib, cam.width, cam.height, counts=True)
                w.render_partial(i, fr)
                rgba, depth, n = frame_np(fr)
                check_bracketed(rgba, depth, n,
                                lambda th: oracle_brick(vol, dims, lo, hi, tf, prm, cam, px, py, th),
                                prm.ert, TOL_F32, f"step {step} brick {i}")
            w.release()


def test_cfg2_full_size_sampled(gpu_lib, dpr):
    """512^3 FP32 split 2x2x2 (257^3 stored bricks), 1024^2, early termination off
    and at 0.99: on every 8th pixel plus four 64x64 tiles, every brick's partial
    against the bracketed oracle and the composited frame against the oracle's
    composite (on pixels no brick's termination makes ambiguous); with termination
    off, the whole frame against the GPU's own unsplit render."""
    cfg = get_config("cfg2")
    dims = cfg.dims
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range)
    log("cfg2: generating 512^3 volume")
    vol = make_volume_small(dims, blobs, cfg.seeds["volume"], cfg.noise_amp)
    tf = make_tf(cfg.seeds["tf"])
    cam = orbit_camera(dims, *cfg.image)
    px, py = pc10_subset(cam, dims, seed=7)
    boxes = even_split(dims, cfg.parts)
    bricks = [extract_brick(vol, dims, lo, hi, 1) for lo, hi in boxes]
    for ert in (1.0, cfg.ert):
        prm = RenderParams(cfg.step_voxels, ert, cfg.density)
        log(f"cfg2 ert {ert}: building world")
        w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam)
        out = dpr.Frame(gpu_lib, *cfg.image)
        w.render_frame(out)
        check_partials_and_frame(dpr, gpu_lib, w, bricks, dims, tf, prm, cam, px, py, TOL_F32, f"cfg2 ert {ert}",
                                 frame=out)
        if ert >= 1.0:
            got, _, _ = frame_np(out)
            wu = make_world(dpr, gpu_lib, vol, dims, [((0, 0, 0), dims)], tf, prm, cam)
            un = dpr.Frame(gpu_lib, *cfg.image)
            wu.render_partial(0, un)
            gu, _, _ = frame_np(un)
            inv = np.max(np.abs(got - gu))
            log(f"  cfg2 GPU split invariant (full frame): {inv:.3e}")
            assert inv <= TOL_F32
            wu.release()
        w.release()


@pytest.mark.parametrize("flags", [0, 0x10])   # FP16 voxel pairs; FP16 2-byte layout
def test_release_linear_keeps_renders(gpu_lib, dpr, flags):
    """After dpr_world_release_linear the frame is the same bits, a commit with
    nothing to rebuild is a no-op, and one that must rebuild (or a path-tracer
    block-majorant build) fails with DPR_ERR_INVALID_STATE."""
    import ctypes as C
    dims = (72, 64, 56)
    vol, tf = _small_case(dims, seed=5, dtype=np.float16)
    prm = RenderParams(0.5, 0.99, 20.0)
    cam = orbit_camera(dims, 64, 48)
    boxes = even_split(dims, (2, 1, 2))
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, flags=flags)
    f = dpr.Frame(gpu_lib, 64, 48)
    w.render_frame(f)
    want = frame_np(f)[:2]

    def live():
        a, n = C.c_int64(), C.c_int64()
        dpr.check(dpr.lib.dpr_alloc_stats(C.byref(a), C.byref(n)))
        return n.value

    before = live()
    w.release_linear()
    assert live() == before - len(boxes)
    for _ in range(2):
        w.render_frame(f)
        got = frame_np(f)[:2]
        assert all(np.array_equal(a, b) for a, b in zip(want, got))
        w.commit()   # nothing to rebuild
    with pytest.raises(dpr.DprError) as e:
        w.render_path(f)
    assert e.value.status == -2
    w.set_params(dpr.Params(prm.step_voxels, prm.ert, 8, flags))
    with pytest.raises(dpr.DprError) as e:
        w.commit()
    assert e.value.status == -2
    f.release()
    w.release()


def _deblock(buf, bdim, elem_bytes, sdim):
    """Element of every stored voxel (z, y, x) of a blocked copy, from the layout's
    definition: 8^3 blocks x fastest; inside a block the index bits, from bit 0,
    are i0 i1 j0 k0 j1 k1 i2 j2 k2."""
    sx, sy, sz = sdim
    z, y, x = np.meshgrid(np.arange(sz), np.arange(sy), np.arange(sx), indexing="ij")
    i, j, k = x & 7, y & 7, z & 7
    within = ((i & 3) | ((j & 1) << 2) | ((k & 1) << 3) | ((j & 2) << 3) | ((k & 2) << 4) | ((i & 4) << 4)
              | ((j & 4) << 5) | ((k & 4) << 6))
    blk = ((z >> 3) * bdim[1] + (y >> 3)) * bdim[0] + (x >> 3)
    return buf.view(np.uint32 if elem_bytes == 4 else np.uint16)[blk * 512 + within]


@pytest.mark.parametrize("dims,dtype,flags,mc,ghost,nb", [
    ((70, 45, 38), np.float32, 0, 16, 1, 5),
    ((70, 45, 38), np.float16, 0, 2, 3, 5),      # FP16 voxel pairs
    ((70, 45, 38), np.float16, 0x10, 16, 2, 5),  # FP16 2-byte voxels
    ((301, 21, 19), np.float16, 0x10, 64, 3, 3),  # several 128-column spans, odd extents
    ((301, 21, 19), np.float32, 0, 4, 1, 2),
    ((259, 34, 33), np.float16, 0, 8, 1, 4),
])
def test_blocked_copy_bitwise(gpu_lib, dpr, dims, dtype, flags, mc, ghost, nb):
    """Every stored voxel of every brick's blocked copy, read back and de-blocked
    on the host, equals the input bit for bit (FP16 pairs: voxel x in the low
    half, voxel x + 1 -- or x again at the end of a row -- in the high half)."""
    vol, tf = _small_case(dims, seed=17, nb=4, dtype=dtype)
    prm = RenderParams(0.5, 0.99, 20.0)
    cam = orbit_camera(dims, 16, 16)
    boxes = kd_split(dims, nb, seed=11, max_ratio=6.0)
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, mc=mc, flags=flags, ghost=ghost)
    for i, (lo, hi) in enumerate(boxes):
        b = extract_brick(vol, dims, lo, hi, ghost)
        data = np.ascontiguousarray(b.data)
        sdim = (data.shape[2], data.shape[1], data.shape[0])
        buf, bdim, eb = w.blocked_copy(i)
        got = _deblock(buf, bdim, eb, sdim)
        if dtype == np.float32:
            want = data.view(np.uint32)
        elif eb == 2:
            want = data.view(np.uint16)
        else:
            h = data.view(np.uint16).astype(np.uint32)
            nxt = np.concatenate([h[:, :, 1:], h[:, :, -1:]], axis=2)
            want = h | (nxt << 16)
        assert eb == (2 if (dtype == np.float16 and flags & 0x10) else 4)
        assert np.array_equal(got, want), (i, int(np.count_nonzero(got != want)))
        # padding voxels of the last blocks stay zero
        el = buf.view(np.uint32 if eb == 4 else np.uint16)
        assert np.count_nonzero(el) == np.count_nonzero(got)
    w.release()
