"""GPU parity of data-parallel volumetric path tracing with ray forwarding
(reading C22 of oracle/path.py; the paper's sections 2.2 and 5.2, Fig. 7).

Both sides draw the same Philox4x32-10 numbers, so a GPU path follows the
oracle's path as long as every decision (real or null collision, leaving the box)
is taken the same way.  The GPU decides in FP32, the oracle in FP64: a pixel
whose oracle decisions come within MARGIN of flipping may go either way, so it is
left out of the elementwise comparison, and such pixels must stay rare."""

import numpy as np
import pytest

import oracle
from oracle import PathParams, RenderParams
from synth import even_split, kd_split, make_blobs, make_tf, make_volume_small, orbit_camera
from tests.gpu_util import frame_np, log, make_world

pytestmark = pytest.mark.gpu

MARGIN = 1e-4
# FP32 paths of up to a few hundred factors against FP64: 1e-4 relative
TOL = 1e-4


@pytest.fixture(scope="module")
def dpr():
    import paper_2407_00179_amd as m
    return m


def _volume(dims, seed, dtype=np.float32):
    return make_volume_small(dims, make_blobs(dims, seed, 6, (0.08, 0.25)), seed + 1, 0.02, dtype)


def _tf(seed, cut=0.2):
    tf = make_tf(seed).astype(np.float32)
    tf[: int(cut * (tf.shape[0] - 1)), 3] = 0.0
    return tf


PP = dict(light_dir=(-0.45, -0.55, -0.7), light_rgb=(3.0, 2.8, 2.5), env_rgb=(0.15, 0.2, 0.3))


def _gpu(dpr, dev, vol, dims, boxes, tf, prm, cam, bounces, spp, seed):
    w = make_world(dpr, dev, vol, dims, boxes, tf, prm, cam, mc=8)
    f = dpr.Frame(dev, cam.width, cam.height)
    st = w.render_path(f, max_bounces=bounces, spp=spp, seed=seed, **PP)
    rgba, depth, _ = frame_np(f)
    f.release()
    w.release()
    return rgba, depth, st


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
def test_paths_match_oracle(gpu_lib, dpr, dtype):
    dims = (40, 36, 32)
    vol = _volume(dims, 11, dtype)
    tf = _tf(3001)
    prm = RenderParams(0.5, 1.0, 18.0)
    cam = orbit_camera(dims, 48, 40, dist=1.6)
    pp = PathParams(max_bounces=3, spp=2, seed=5, **PP)
    want, mg = oracle.render_path(vol, dims, tf, prm, pp, cam)
    for boxes in ([((0, 0, 0), dims)], kd_split(dims, 7, seed=3, max_ratio=3.0)):
        got, depth, st = _gpu(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, 3, 2, 5)
        clear = mg > MARGIN
        err = np.abs(got[:, :3] - want) / np.maximum(1.0, np.abs(want))
        log(f"  {len(boxes)} bricks: max rel err {err[clear].max():.2e} on {clear.sum()} pixels, "
            f"{(~clear).sum()} near a flipped decision; {st}")
        assert err[clear].max() <= TOL
        assert (~clear).sum() <= 0.05 * clear.size
        assert np.all(got[:, 3] == 1.0) and np.all(np.isinf(depth))
        assert st["paths"] == cam.width * cam.height * 2 and st["events"] > 0
        if len(boxes) > 1:
            assert st["forwards"] > 0
    assert np.ptp(want) > 0.05


@pytest.mark.parametrize("bounces", [1, 12])
def test_bounce_limits_match_oracle(gpu_lib, dpr, bounces):
    """A path ends at its first real collision (1) or keeps scattering through many
    (12, each one continuing in its lane within a wave), as in the oracle."""
    dims = (28, 24, 20)
    vol = _volume(dims, 61)
    tf = _tf(3007, cut=0.1)
    prm = RenderParams(0.5, 1.0, 30.0)
    cam = orbit_camera(dims, 24, 20, dist=1.6)
    pp = PathParams(max_bounces=bounces, spp=2, seed=9, **PP)
    want, mg = oracle.render_path(vol, dims, tf, prm, pp, cam)
    got, _, st = _gpu(dpr, gpu_lib, vol, dims, kd_split(dims, 5, seed=4, max_ratio=3.0), tf, prm, cam, bounces, 2, 9)
    clear = mg > MARGIN
    err = np.abs(got[:, :3] - want) / np.maximum(1.0, np.abs(want))
    log(f"  {bounces} bounces: max rel err {err[clear].max():.2e}, {(~clear).sum()} near a flip; {st}")
    assert err[clear].max() <= TOL and (~clear).sum() <= 0.05 * clear.size
    assert st["events"] > 0


def test_bricking_does_not_change_a_bit(gpu_lib, dpr):
    """The tentative collisions come from the path's own random numbers and the
    majorants of a grid over the whole volume, so any bricking gives the same
    bits; forwarding shows in the counters only."""
    dims = (48, 44, 40)
    vol = _volume(dims, 21)
    tf = _tf(3002)
    prm = RenderParams(0.5, 1.0, 22.0)
    cam = orbit_camera(dims, 64, 56, dist=1.7)
    outs = []
    for boxes in ([((0, 0, 0), dims)], even_split(dims, (2, 2, 2)), kd_split(dims, 11, seed=8, max_ratio=4.0),
                  even_split(dims, (4, 3, 2))):
        got, _, st = _gpu(dpr, gpu_lib, vol, dims, boxes, tf, prm, cam, 4, 2, 17)
        log(f"  {len(boxes)} bricks: {st}")
        outs.append((got, st))
    assert outs[0][1]["forwards"] == 0  # one brick: nothing to hand over
    for got, st in outs[1:]:
        assert np.array_equal(got, outs[0][0])
        assert st["events"] == outs[0][1]["events"] and st["shadow_steps"] == outs[0][1]["shadow_steps"]
        assert st["forwards"] > outs[0][1]["forwards"]


def test_wide_offsets_and_f16_layouts_give_the_same_bits(gpu_lib, dpr):
    dims = (40, 36, 32)
    vol = _volume(dims, 51, np.float16)
    tf = _tf(3005)
    prm = RenderParams(0.5, 1.0, 20.0)
    cam = orbit_camera(dims, 40, 32, dist=1.7)
    outs = []
    for flags in (0, dpr.FLAG_WIDE_OFFSETS, dpr.FLAG_F16_HALVES):
        w = make_world(dpr, gpu_lib, vol, dims, kd_split(dims, 5, seed=2, max_ratio=3.0), tf, prm, cam, mc=8,
                       flags=flags)
        f = dpr.Frame(gpu_lib, cam.width, cam.height)
        st = w.render_path(f, max_bounces=3, spp=2, seed=4, **PP)
        outs.append((frame_np(f)[0], st))
        f.release()
        w.release()
    for o in outs[1:]:
        assert np.array_equal(outs[0][0], o[0]) and outs[0][1] == o[1]


def test_repeatable_and_seeded(gpu_lib, dpr):
    dims = (32, 32, 32)
    vol = _volume(dims, 31)
    tf = _tf(3003)
    prm = RenderParams(0.5, 1.0, 20.0)
    cam = orbit_camera(dims, 40, 32, dist=1.7)
    a, _, sa = _gpu(dpr, gpu_lib, vol, dims, even_split(dims, (2, 1, 2)), tf, prm, cam, 3, 3, 1)
    b, _, sb = _gpu(dpr, gpu_lib, vol, dims, even_split(dims, (2, 1, 2)), tf, prm, cam, 3, 3, 1)
    c, _, _ = _gpu(dpr, gpu_lib, vol, dims, even_split(dims, (2, 1, 2)), tf, prm, cam, 3, 3, 2)
    assert np.array_equal(a, b) and sa == sb
    assert not np.array_equal(a, c)


def test_vacuum_sees_the_environment(gpu_lib, dpr):
    dims = (24, 20, 16)
    vol = _volume(dims, 41)
    tf = _tf(3004)
    tf[:, 3] = 0.0
    cam = orbit_camera(dims, 16, 12, dist=1.5)
    got, _, st = _gpu(dpr, gpu_lib, vol, dims, even_split(dims, (2, 2, 1)), tf, RenderParams(0.5, 1.0, 20.0), cam,
                      3, 2, 1)
    assert np.array_equal(got[:, :3], np.tile(np.float32(PP["env_rgb"]), (got.shape[0], 1)).astype(np.float64))
    assert st["events"] == 0 and st["waves"] == 0


def test_path_argument_errors(gpu_lib, dpr):
    dims = (16, 16, 16)
    vol = _volume(dims, 5)
    cam = orbit_camera(dims, 8, 8)
    w = make_world(dpr, gpu_lib, vol, dims, [((0, 0, 0), dims)], _tf(1), RenderParams(0.5, 1.0, 20.0), cam)
    f = dpr.Frame(gpu_lib, 8, 8)
    for kw in (dict(max_bounces=0), dict(max_bounces=256), dict(spp=0), dict(light_dir=(0.0, 0.0, 0.0)),
               dict(light_rgb=(1.0, -1.0, 1.0)), dict(env_rgb=(float("nan"), 0.0, 0.0))):
        with pytest.raises(dpr.DprError):
            w.render_path(f, **kw)
    g = dpr.Frame(gpu_lib, 9, 8)
    with pytest.raises(dpr.DprError):
        w.render_path(g)
    for h in (f, g, w):
        h.release()
