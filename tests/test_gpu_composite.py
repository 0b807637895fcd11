"""GPU parity of the sort-last compositor on seeded synthetic fragments."""

import numpy as np
import pytest

import oracle
from synth import synthetic_frames
from tests.gpu_util import frame_np, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpr():
    import paper_2407_00179_amd as m
    return m


def _frames(dpr, dev, K, W, H, seed, t_min=2.0, t_max=3.0):
    import torch
    rgba = torch.empty((K, H, W, 4), dtype=torch.float32, device=dev.torch_device)
    depth = torch.empty((K, H, W), dtype=torch.float32, device=dev.torch_device)
    synthetic_frames(K, W, H, t_min, t_max, seed, dev.torch_device, rgba, depth)
    frames = [dpr.Frame(dev, W, H, rgba=rgba[k], depth=depth[k]) for k in range(K)]
    return rgba, depth, frames


def _oracle(rgba, depth, ids, sel=None):
    r = rgba.cpu().numpy().reshape(rgba.shape[0], -1, 4)
    z = depth.cpu().numpy().reshape(depth.shape[0], -1)
    if sel is not None:
        r, z = r[:, sel], z[:, sel]
    return oracle.composite(r, z, ids)


@pytest.mark.parametrize("K,W,H", [(8, 64, 48), (3, 1, 1), (16, 67, 5), (17, 40, 40), (64, 33, 65),
                                   (128, 50, 31), (200, 16, 16), (256, 9, 14)])
def test_composite_matches_oracle(gpu_lib, dpr, K, W, H):
    log(f"composite K={K} {W}x{H}")
    rgba, depth, frames = _frames(dpr, gpu_lib, K, W, H, seed=100 + K)
    ids = np.random.default_rng(K).permutation(1000)[:K]
    out = dpr.Frame(gpu_lib, W, H)
    dpr.composite(gpu_lib, frames, out, ids=ids)
    got, gz, _ = frame_np(out)
    want, wz = _oracle(rgba, depth, ids)
    err = np.max(np.abs(got - want))
    log(f"  max err {err:.3e}")
    assert err <= 2e-6 * max(1, K / 8)
    assert np.array_equal(gz, wz.astype(np.float32).astype(np.float64))


def test_single_fragment_identity_and_empty(gpu_lib, dpr):
    rgba, depth, frames = _frames(dpr, gpu_lib, 1, 70, 30, seed=5)
    out = dpr.Frame(gpu_lib, 70, 30)
    dpr.composite(gpu_lib, frames, out)
    got, gz, _ = frame_np(out)
    assert np.array_equal(got, rgba[0].cpu().numpy().reshape(-1, 4).astype(np.float64))
    assert np.array_equal(gz, depth[0].cpu().numpy().reshape(-1).astype(np.float64))
    # all-empty inputs give an empty frame
    import torch
    er = torch.zeros((4, 30, 70, 4), device=gpu_lib.torch_device)
    ez = torch.full((4, 30, 70), float("inf"), device=gpu_lib.torch_device)
    ef = [dpr.Frame(gpu_lib, 70, 30, rgba=er[k], depth=ez[k]) for k in range(4)]
    dpr.composite(gpu_lib, ef, out)
    got, gz, _ = frame_np(out)
    assert np.all(got == 0.0) and np.all(np.isinf(gz))


def test_permutation_invariance_and_ties(gpu_lib, dpr):
    import torch
    K, W, H = 24, 80, 40
    rgba, depth, frames = _frames(dpr, gpu_lib, K, W, H, seed=9)
    # force exact depth ties between frames; the id decides their order
    depth[1::2] = torch.where(torch.isfinite(depth[1::2]), torch.round(depth[1::2] * 4) / 4, depth[1::2])
    depth[0::2] = torch.where(torch.isfinite(depth[0::2]), torch.round(depth[0::2] * 4) / 4, depth[0::2])
    ids = np.arange(K) * 7 + 3
    out = dpr.Frame(gpu_lib, W, H)
    dpr.composite(gpu_lib, frames, out, ids=ids)
    ref, rz, _ = frame_np(out)
    want, _ = _oracle(rgba, depth, ids)
    assert np.max(np.abs(ref - want)) <= 4e-6
    for s in range(3):
        perm = np.random.default_rng(s).permutation(K)
        dpr.composite(gpu_lib, [frames[i] for i in perm], out, ids=ids[perm])
        got, gz, _ = frame_np(out)
        assert np.array_equal(got, ref) and np.array_equal(gz, rz)


@pytest.mark.parametrize("K", [1, 2, 8, 9, 16])
def test_small_k_kernel_equals_tile_order_path(gpu_lib, dpr, K):
    """Up to 16 sources are composited by sorting each pixel's keys in registers;
    the same frames padded with empty ones to 17 sources take the tile-order path.
    Both give the same bits, also with exact depth ties (the id decides) and NaN
    depths (no fragment), and match the oracle."""
    import torch
    W, H = 97, 61
    log(f"small-K composite K={K}")
    rgba, depth, frames = _frames(dpr, gpu_lib, K, W, H, seed=300 + K)
    depth.copy_(torch.where(torch.isfinite(depth), torch.round(depth * 8) / 8, depth))
    depth[0, ::7, ::5] = float("nan")
    ids = np.random.default_rng(K).permutation(500)[:K]
    out = dpr.Frame(gpu_lib, W, H)
    dpr.composite(gpu_lib, frames, out, ids=ids)
    got, gz, _ = frame_np(out)
    n_pad = 17 - K
    er = torch.zeros((n_pad, H, W, 4), dtype=torch.float32, device=gpu_lib.torch_device)
    ez = torch.full((n_pad, H, W), float("inf"), dtype=torch.float32, device=gpu_lib.torch_device)
    pads = [dpr.Frame(gpu_lib, W, H, rgba=er[i], depth=ez[i]) for i in range(n_pad)]
    out17 = dpr.Frame(gpu_lib, W, H)
    dpr.composite(gpu_lib, frames + pads, out17, ids=list(ids) + list(range(1000, 1000 + n_pad)))
    ref, rz, _ = frame_np(out17)
    assert np.array_equal(got, ref) and np.array_equal(gz, rz)
    clean = torch.where(torch.isnan(depth), torch.full_like(depth, float("inf")), depth)
    want, wz = _oracle(rgba, clean, ids)
    assert np.max(np.abs(got - want)) <= 2e-6
    assert np.array_equal(gz, wz.astype(np.float32).astype(np.float64))
    for s in range(2):
        perm = np.random.default_rng(s).permutation(K)
        dpr.composite(gpu_lib, [frames[i] for i in perm], out, ids=ids[perm])
        pg, pz, _ = frame_np(out)
        assert np.array_equal(pg, got) and np.array_equal(pz, gz)


@pytest.mark.parametrize("K", [8, 12])
def test_small_k_kernel_several_pixels_per_lane(gpu_lib, dpr, K):
    """A frame larger than one resident grid (each lane walks several pixels and
    prefetches the next one's depths): every pixel against the oracle."""
    W, H = 1100, 700
    log(f"small-K composite K={K} {W}x{H}")
    rgba, depth, frames = _frames(dpr, gpu_lib, K, W, H, seed=700 + K)
    ids = np.random.default_rng(K + 1).permutation(300)[:K]
    out = dpr.Frame(gpu_lib, W, H)
    dpr.composite(gpu_lib, frames, out, ids=ids)
    got, gz, _ = frame_np(out)
    want, wz = _oracle(rgba, depth, ids)
    assert np.max(np.abs(got - want)) <= 2e-6 * max(1, K / 8)
    assert np.array_equal(gz, wz.astype(np.float32).astype(np.float64))


def test_composite_rejects_bad_arguments(gpu_lib, dpr):
    rgba, depth, frames = _frames(dpr, gpu_lib, 3, 16, 16, seed=1)
    out = dpr.Frame(gpu_lib, 16, 16)
    with pytest.raises(dpr.DprError, match="distinct"):
        dpr.composite(gpu_lib, frames, out, ids=[1, 1, 2])
    with pytest.raises(dpr.DprError, match="alias"):
        dpr.composite(gpu_lib, frames, frames[0])
    small = dpr.Frame(gpu_lib, 8, 16)
    with pytest.raises(dpr.DprError):
        dpr.composite(gpu_lib, frames, small)
    with pytest.raises(dpr.DprError):
        dpr.composite(gpu_lib, frames * 90, out, ids=list(range(270)))


def test_composite_k128_full_hd_sampled(gpu_lib, dpr):
    """K = 128 at 3840x2160 (21 GB of fragments), checked on a pixel sample."""
    import torch
    from synth import pixel_subset
    K, W, H = 128, 3840, 2160
    log("K=128 3840x2160: generating frames")
    rgba, depth, frames = _frames(dpr, gpu_lib, K, W, H, seed=6005, t_min=2.2, t_max=3.4)
    ids = np.random.default_rng(3).permutation(K)
    out = dpr.Frame(gpu_lib, W, H)
    dpr.composite(gpu_lib, frames, out, ids=ids)
    gpu_lib.sync()
    px, py = pixel_subset(W, H, stride=64, tiles=2, tile=32, seed=1)
    sel = torch.from_numpy(py * W + px).to(gpu_lib.torch_device)
    r = rgba.reshape(K, -1, 4)[:, sel]
    z = depth.reshape(K, -1)[:, sel]
    want, wz = oracle.composite(r.cpu().numpy(), z.cpu().numpy(), ids)
    got = out.rgba.reshape(-1, 4)[sel].cpu().numpy().astype(np.float64)
    gz = out.depth.reshape(-1)[sel].cpu().numpy().astype(np.float64)
    err = np.max(np.abs(got - want))
    log(f"  K=128 sampled {sel.numel()} px: max err {err:.3e}")
    assert err <= 2e-5
    assert np.array_equal(gz, wz.astype(np.float32).astype(np.float64))
    del rgba, depth, frames
    torch.cuda.empty_cache()


@pytest.mark.parametrize("K,W,H", [(8, 200, 100), (37, 64, 64), (128, 96, 80), (256, 40, 30)])
def test_composite_out_of_tile_order(gpu_lib, dpr, K, W, H):
    """Per-pixel random depths: most pixels break their tile's order and go through
    the general per-wave sort; results must match the oracle and stay bitwise equal
    under input permutation."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(K)
    depth = (torch.rand((K, H, W), generator=g) * 5 + 0.5).to(gpu_lib.torch_device)
    empty = (torch.rand((K, H, W), generator=g) < 0.3).to(gpu_lib.torch_device)
    depth[empty] = float("inf")
    a = (torch.rand((K, H, W), generator=g) * 0.6).to(gpu_lib.torch_device)
    col = torch.rand((K, H, W, 3), generator=g).to(gpu_lib.torch_device)
    rgba = torch.cat([col * a[..., None], a[..., None]], dim=-1)
    rgba[empty] = 0.0
    rgba = rgba.contiguous()
    depth = depth.contiguous()
    # a band of rows keeps one global order (fast path) next to the shuffled rest
    depth[:, : H // 4] = torch.where(torch.isfinite(depth[:, : H // 4]),
                                     torch.arange(K, device=gpu_lib.torch_device, dtype=torch.float32)[:, None, None]
                                     + 1.0, depth[:, : H // 4])
    frames = [dpr.Frame(gpu_lib, W, H, rgba=rgba[k], depth=depth[k]) for k in range(K)]
    ids = np.random.default_rng(K).permutation(K)
    out = dpr.Frame(gpu_lib, W, H)
    dpr.composite(gpu_lib, frames, out, ids=ids)
    got, gz, _ = frame_np(out)
    want, wz = _oracle(rgba, depth, ids)
    err = np.max(np.abs(got - want))
    log(f"composite out-of-order K={K}: max err {err:.3e}")
    assert err <= 2e-6 * max(1, K / 8)
    assert np.array_equal(gz, wz.astype(np.float32).astype(np.float64))
    perm = np.random.default_rng(1).permutation(K)
    dpr.composite(gpu_lib, [frames[i] for i in perm], out, ids=ids[perm])
    got2, gz2, _ = frame_np(out)
    assert np.array_equal(got, got2) and np.array_equal(gz, gz2)
