"""The allocation-free composite (dpr_composite_noalloc) called through the C ABI
gives the bits of dpr_composite, on consecutive calls that share the library's
fixed scratch array, the second with fewer fragments and pixels than the first."""

import ctypes as C

import numpy as np
import pytest

import oracle
from tests.gpu_util import frame_np, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpr():
    import paper_2407_00179_amd as m
    return m


def _frames(dpr, dev, K, W, H, seed):
    """K frames whose per-pixel depths are independent draws, so neighbouring
    pixels disagree on the fragment order and the fix-up list fills up; about a
    quarter of the fragments are empty."""
    import torch
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 0.9, (K, H, W)).astype(np.float32)
    rgb = (rng.uniform(0.0, 1.0, (K, H, W, 3)) * a[..., None]).astype(np.float32)
    z = rng.uniform(1.0, 2.0, (K, H, W)).astype(np.float32)
    empty = rng.uniform(size=(K, H, W)) < 0.25
    a[empty] = 0.0
    rgb[empty] = 0.0
    z[empty] = np.inf
    rgba = torch.from_numpy(np.concatenate([rgb, a[..., None]], axis=-1)).to(dev.torch_device).contiguous()
    depth = torch.from_numpy(z).to(dev.torch_device).contiguous()
    frames = [dpr.Frame(dev, W, H, rgba=rgba[k], depth=depth[k]) for k in range(K)]
    return rgba, depth, frames


def _noalloc(dpr, dev, frames, out, ids):
    k = len(frames)
    fr = (C.c_void_p * k)(*[f.h.value for f in frames])
    idarr = (C.c_int32 * k)(*[int(i) for i in ids])
    dpr.check(dpr.lib.dpr_composite_noalloc(dev.h, fr, idarr, k, out.h))


@pytest.mark.parametrize("calls", [[(40, 256, 160), (24, 100, 60)], [(200, 64, 40), (5, 33, 7)]])
def test_noalloc_matches_composite_on_consecutive_calls(gpu_lib, dpr, calls):
    for n, (K, W, H) in enumerate(calls):
        log(f"no-alloc composite call {n}: K={K} {W}x{H}")
        rgba, depth, frames = _frames(dpr, gpu_lib, K, W, H, seed=700 + K)
        ids = np.random.default_rng(K).permutation(4 * K)[:K]
        ref = dpr.Frame(gpu_lib, W, H)
        got = dpr.Frame(gpu_lib, W, H)
        got.rgba.fill_(-1.0)
        got.depth.fill_(-1.0)
        dpr.composite(gpu_lib, frames, ref, ids=ids)
        _noalloc(dpr, gpu_lib, frames, got, ids)
        want_rgba, want_z, _ = frame_np(ref)
        got_rgba, got_z, _ = frame_np(got)
        assert np.array_equal(got_rgba, want_rgba), f"call {n}: RGBA differs from dpr_composite"
        assert np.array_equal(got_z, want_z), f"call {n}: depth differs from dpr_composite"
        # and both against the FP64 oracle
        r = rgba.cpu().numpy().reshape(K, -1, 4)
        z = depth.cpu().numpy().reshape(K, -1)
        o_rgba, o_z = oracle.composite(r, z, ids)
        err = float(np.max(np.abs(got_rgba - o_rgba)))
        log(f"  identical to dpr_composite; max|gpu-oracle| = {err:.3e}")
        assert err <= 2e-6 * max(1, K / 8)
        assert np.array_equal(got_z, o_z.astype(np.float32).astype(np.float64))
        for f in frames + [ref, got]:
            f.release()


def test_noalloc_rejects_frames_beyond_its_limit(gpu_lib, dpr):
    W, H = 4096, 2049   # 8,392,704 pixels > 2^23
    rgba, depth, frames = _frames(dpr, gpu_lib, 2, 8, 8, seed=1)
    import torch
    big = [dpr.Frame(gpu_lib, W, H, rgba=torch.zeros((H, W, 4), device=gpu_lib.torch_device),
                     depth=torch.full((H, W), float("inf"), device=gpu_lib.torch_device)) for _ in range(2)]
    out = dpr.Frame(gpu_lib, W, H)
    with pytest.raises(dpr.DprError) as e:
        _noalloc(dpr, gpu_lib, big, out, [0, 1])
    assert e.value.status == -5 and "allocation-free maximum" in str(e.value)
    for f in frames + big + [out]:
        f.release()
