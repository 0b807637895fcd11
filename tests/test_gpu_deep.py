"""GPU parity of deep (multi-fragment) frames: a rank whose bricks form a
non-convex set renders per-pixel fragment lists, and the lists of all ranks merge
to the unsplit image (paper section 5.1.1; the interleaved partition of Fig. 6)."""

import numpy as np
import pytest

import oracle
from oracle import RenderParams
from synth import even_split, kd_split, make_blobs, make_tf, make_volume_small, orbit_camera
from tests.gpu_util import TOL_F32, frame_np, log, make_world, oracle_brick

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpr():
    import paper_2407_00179_amd as m
    return m


def _volume(dims, seed, dtype=np.float32):
    return make_volume_small(dims, make_blobs(dims, seed, 7, (0.06, 0.25)), seed + 1, 0.02, dtype)


def _deep_np(deep):
    deep.dev.sync()
    P = deep.width * deep.height
    return (deep.counts.cpu().numpy().reshape(P).astype(np.int64),
            deep.rgba.cpu().numpy().reshape(deep.capacity, P, 4).astype(np.float64),
            deep.depth.cpu().numpy().reshape(deep.capacity, P).astype(np.float64),
            deep.ids.cpu().numpy().reshape(deep.capacity, P).astype(np.int64))


def _partials(dpr, dev, w, n_bricks, cam):
    rr, zz = [], []
    for i in range(n_bricks):
        f = dpr.Frame(dev, cam.width, cam.height)
        w.render_partial(i, f)
        r, z, _ = frame_np(f)
        rr.append(r)
        zz.append(z)
        f.release()
    return np.stack(rr), np.stack(zz)


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
def test_render_deep_is_the_sorted_partials(gpu_lib, dpr, dtype):
    dims = (52, 44, 36)
    vol = _volume(dims, 41, dtype)
    tf = make_tf(2001)
    prm = RenderParams(0.5, 0.99, 25.0)
    cam = orbit_camera(dims, 77, 61)
    boxes = kd_split(dims, 9, seed=4, max_ratio=4.0)
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, mc=8)
    rank = 3
    deep = dpr.DeepFrame(gpu_lib, cam.width, cam.height, len(boxes) + 2)
    for flags in (0, 0, dpr.FLAG_NO_GRAPH):        # capture, replay, direct
        w.set_params(dpr.Params(prm.step_voxels, prm.ert, 8, flags))
        deep.counts.fill_(-1)
        w.render_deep(rank, deep)
        cnt, lr, lz, lf = _deep_np(deep)
        rr, zz = _partials(dpr, gpu_lib, w, len(boxes), cam)
        want = oracle.deep_frame(rr, zz, [rank * oracle.FID_RANK + b for b in range(len(boxes))], deep.capacity)
        assert np.array_equal(cnt, want[0]), flags
        assert cnt.max() >= 2
        live = np.arange(deep.capacity)[:, None] < cnt[None, :]
        assert np.array_equal(lz[live], want[2][live]) and np.array_equal(lf[live], want[3][live])
        assert np.array_equal(lr[live], want[1][live])
    # against the oracle: each layer's fragment is its brick's oracle fragment
    px, py = np.meshgrid(np.arange(cam.width), np.arange(cam.height))
    px, py = px.ravel(), py.ravel()
    orc = [oracle_brick(vol, dims, lo, hi, tf, prm, cam, px, py) for lo, hi in boxes]
    rgba_o, z_o = np.stack([o[0] for o in orc]), np.stack([o[1] for o in orc])
    for i in range(deep.capacity):
        m = i < cnt
        b = lf[i, m] - rank * oracle.FID_RANK
        err = np.max(np.abs(lr[i, m] - rgba_o[b, np.flatnonzero(m)])) if m.any() else 0.0
        assert err <= (2e-3 if dtype == np.float16 else TOL_F32), (i, err)
    deep.release()
    w.release()


def test_interleaved_partition_deep_composite(gpu_lib, dpr):
    """4^3 boxes dealt to 4 ranks: every rank's data is non-convex.  Their deep
    frames merge to the unsplit image; the order of the parts does not matter."""
    dims = (48, 48, 48)
    vol = _volume(dims, 57)
    tf = make_tf(2001)
    prm = RenderParams(0.5, 1.0, 25.0)
    cam = orbit_camera(dims, 90, 70)
    boxes = even_split(dims, (4, 4, 4))
    owner = np.random.default_rng(5).integers(0, 4, size=len(boxes))
    deeps, worlds = [], []
    for r in range(4):
        mine = [boxes[i] for i in range(len(boxes)) if owner[i] == r]
        log(f"rank {r}: {len(mine)} bricks")
        w = make_world(dpr, gpu_lib, vol, dims, mine, tf, prm, cam, mc=8)
        d = dpr.DeepFrame(gpu_lib, cam.width, cam.height, len(mine))
        w.render_deep(10 + r, d)
        deeps.append(d)
        worlds.append(w)
    out = dpr.Frame(gpu_lib, cam.width, cam.height)
    dpr.composite_deep(gpu_lib, deeps, out)
    got, gz, _ = frame_np(out)
    px, py = np.meshgrid(np.arange(cam.width), np.arange(cam.height))
    full, fz, _ = oracle.render_image(vol, dims, tf, prm, cam, px.ravel(), py.ravel())
    err = np.max(np.abs(got - full))
    log(f"deep composite of the interleaved partition vs unsplit oracle: {err:.3e}")
    assert err <= TOL_F32
    assert np.array_equal(np.isfinite(gz), np.isfinite(fz))
    # the GPU's own unsplit render
    wu = make_world(dpr, gpu_lib, vol, dims, [((0, 0, 0), dims)], tf, prm, cam, mc=8)
    un = dpr.Frame(gpu_lib, cam.width, cam.height)
    wu.render_partial(0, un)
    gu, _, _ = frame_np(un)
    assert np.max(np.abs(got - gu)) <= TOL_F32
    # single-fragment ranks (what the flat path would emit) do not reproduce it
    flat = []
    for w in worlds:
        f = dpr.Frame(gpu_lib, cam.width, cam.height)
        w.render_frame(f)
        flat.append(f)
    fl = dpr.Frame(gpu_lib, cam.width, cam.height)
    dpr.composite(gpu_lib, flat, fl, ids=[10, 11, 12, 13])
    assert np.max(np.abs(frame_np(fl)[0] - full)) > 1e-3
    # permutation invariance, bit for bit
    for perm in ([2, 0, 3, 1], [3, 2, 1, 0]):
        o2 = dpr.Frame(gpu_lib, cam.width, cam.height)
        dpr.composite_deep(gpu_lib, [deeps[i] for i in perm], o2)
        g2, z2, _ = frame_np(o2)
        assert np.array_equal(g2, got) and np.array_equal(z2, gz)
    for h in deeps + worlds + flat + [out, un, fl, wu]:
        h.release()


def test_deep_composite_more_fragments_than_one_pass(gpu_lib, dpr):
    """12 slabs across the view direction dealt alternately to 2 ranks: pixels
    hold up to 12 fragments, so the merge takes more than one selection pass."""
    dims = (48, 20, 20)
    vol = _volume(dims, 71)
    tf = make_tf(2003)
    prm = RenderParams(0.5, 1.0, 12.0)
    cam = orbit_camera(dims, 128, 96, az_deg=8.0, el_deg=5.0)
    boxes = even_split(dims, (12, 1, 1))
    deeps, worlds = [], []
    for r in range(2):
        mine = boxes[r::2]
        w = make_world(dpr, gpu_lib, vol, dims, mine, tf, prm, cam, mc=4)
        d = dpr.DeepFrame(gpu_lib, cam.width, cam.height, len(mine))
        w.render_deep(5 - 3 * r, d)
        deeps.append(d)
        worlds.append(w)
    total = sum(_deep_np(d)[0] for d in deeps)
    log(f"fragments per pixel: max {total.max()}, pixels above 8: {(total > 8).sum()}")
    assert (total > 8).sum() >= 100
    out = dpr.Frame(gpu_lib, cam.width, cam.height)
    dpr.composite_deep(gpu_lib, deeps, out)
    got, gz, _ = frame_np(out)
    px, py = np.meshgrid(np.arange(cam.width), np.arange(cam.height))
    full, fz, _ = oracle.render_image(vol, dims, tf, prm, cam, px.ravel(), py.ravel())
    err = np.max(np.abs(got - full))
    log(f"12-slab deep composite vs unsplit oracle: {err:.3e}")
    assert err <= TOL_F32
    hit = np.isfinite(fz)
    assert np.array_equal(np.isfinite(gz), hit) and np.max(np.abs(gz[hit] - fz[hit])) <= 1e-5
    # the oracle's merge of the GPU's own deep frames, element by element
    parts = [(c, r_, z_, f_) for c, r_, z_, f_ in (_deep_np(d) for d in deeps)]
    want, wz = oracle.composite_deep(parts)
    assert np.max(np.abs(got - want)) <= TOL_F32 and np.array_equal(gz[hit], wz[hit])
    o2 = dpr.Frame(gpu_lib, cam.width, cam.height)
    dpr.composite_deep(gpu_lib, deeps[::-1], o2)
    assert np.array_equal(frame_np(o2)[0], got)
    for h in deeps + worlds + [out, o2]:
        h.release()


def test_deep_merge_ignores_bad_counts_and_depths(gpu_lib, dpr):
    """Deep frames are writable by the caller: a count above the frame's capacity
    is clamped to it, a negative count is 0, and a fragment whose depth is NaN or
    +inf is not live (as in the flat compositor).  The merge then equals the
    oracle's merge of the cleaned lists, and every pixel finishes."""
    import torch
    dims = (24, 20, 16)
    vol = _volume(dims, 13)
    tf = make_tf(2001)
    prm = RenderParams(0.5, 0.99, 20.0)
    W, H, cap = 37, 23, 4
    cam = orbit_camera(dims, W, H)
    w = make_world(dpr, gpu_lib, vol, dims, even_split(dims, (2, 1, 1)), tf, prm, cam, mc=4)
    rng = np.random.default_rng(99)
    deeps, parts = [], []
    P = W * H
    for r in range(3):
        d = dpr.DeepFrame(gpu_lib, W, H, cap)
        w.render_deep(r, d)          # marks the frame as rank r's
        cnt = rng.integers(-2, cap + 4, P)
        z = rng.uniform(1.0, 2.0, (cap, P)).astype(np.float32)
        z[rng.random((cap, P)) < 0.15] = np.nan
        z[rng.random((cap, P)) < 0.10] = np.inf
        a = rng.uniform(0.0, 0.8, (cap, P))
        rgba = np.concatenate([rng.uniform(0, 1, (cap, P, 3)) * a[..., None], a[..., None]], -1).astype(np.float32)
        d.counts.copy_(torch.from_numpy(cnt.astype(np.int32).reshape(H, W)))
        d.depth.copy_(torch.from_numpy(z.reshape(cap, H, W)))
        d.rgba.copy_(torch.from_numpy(rgba.reshape(cap, H, W, 4)))
        # the cleaned list: live layers first, in layer order, ids rank-major
        c2 = np.zeros(P, np.int64)
        r2 = np.zeros((cap, P, 4))
        z2 = np.full((cap, P), np.inf)
        f2 = np.zeros((cap, P), np.int64)
        for p in range(P):
            for l in range(min(max(int(cnt[p]), 0), cap)):
                if np.isfinite(z[l, p]):
                    k = c2[p]
                    r2[k, p], z2[k, p], f2[k, p] = rgba[l, p], z[l, p], r * 256 + l
                    c2[p] += 1
        parts.append((c2, r2, z2, f2))
        deeps.append(d)
    out = dpr.Frame(gpu_lib, W, H)
    dpr.composite_deep(gpu_lib, deeps, out)
    got, gz, _ = frame_np(out)
    want, wz = oracle.composite_deep(parts)
    err = np.max(np.abs(got - want))
    log(f"deep merge with clamped counts and NaN/inf depths: max err {err:.3e}")
    assert err <= TOL_F32
    assert np.array_equal(gz, wz.astype(np.float32).astype(np.float64))
    for h in deeps + [out, w]:
        h.release()


def test_deep_argument_errors(gpu_lib, dpr):
    dims = (24, 20, 16)
    vol = _volume(dims, 3)
    tf = make_tf(2001)
    prm = RenderParams(0.5, 0.99, 25.0)
    cam = orbit_camera(dims, 32, 24)
    boxes = even_split(dims, (2, 1, 2))
    w = make_world(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam)
    small = dpr.DeepFrame(gpu_lib, cam.width, cam.height, len(boxes) - 1)
    with pytest.raises(dpr.DprError, match="capacity"):
        w.render_deep(0, small)
    a = dpr.DeepFrame(gpu_lib, cam.width, cam.height, len(boxes))
    b = dpr.DeepFrame(gpu_lib, cam.width, cam.height, len(boxes))
    out = dpr.Frame(gpu_lib, cam.width, cam.height)
    with pytest.raises(dpr.DprError, match="rendered"):
        dpr.composite_deep(gpu_lib, [a], out)
    w.render_deep(0, a)
    w.render_deep(0, b)
    with pytest.raises(dpr.DprError, match="distinct"):
        dpr.composite_deep(gpu_lib, [a, b], out)
    with pytest.raises(dpr.DprError):
        w.render_deep(40000, a)
    wrong = dpr.DeepFrame(gpu_lib, cam.width + 1, cam.height, len(boxes))
    with pytest.raises(dpr.DprError):
        w.render_deep(1, wrong)
    for h in (small, a, b, out, wrong, w):
        h.release()
