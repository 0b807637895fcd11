#!/usr/bin/env python3
"""Benchmark of the data-parallel brick renderer + sort-last compositor on one MI355X.

Default workload (one "step" = the whole hot path once): a 512^3 FP32 blob+noise
volume split into 2x2x2 bricks of 256^3 owned cells with one ghost layer
(257^3 stored), rendered at 1024x1024 through one camera:
  commit (8^3-blocked copy of every brick + macrocell min/max ranges, one pass)
  -> transfer-function majorants
  -> 8 per-brick emission-absorption ray marches (partial RGBA+depth frames)
  -> sort-last composite of the 8 partial frames.
value = logical samples per second (lattice segments of positive length
processed before termination, skipped ones included), in Msamples/s.

Extra sections (same JSON line): the K=128 compositor at 3840x2160, the batched
persistent renderer against plain per-brick launches on the 27-brick 16-camera
workload, the backward/forward time ratio of the differentiable renderer, deep
(multi-fragment) frames of an interleaved 8-rank partition, the opaque
iso-surface mixed with the volume, and data-parallel path tracing with rays
forwarded between bricks.

The CPU baseline (the FP64 oracle, not tuned) runs first, before any GPU use,
on a bounded pixel sample of the default workload, over a fork pool of host cores.
"""

from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from synth import (even_split, extract_brick, get_config, make_blobs, make_tf,  # noqa: E402
                   make_volume_small, orbit_camera)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # CUs x lanes x clock: lane-op slots per second (non-packed)
# Algorithmic VALU lane-op slots per logical sample: 8 gathers' addressing, ~14 for
# the trilinear lerps, TF lookup + lerp, one exp, the accumulate FMAs, the advance
# and the termination compares.
OPS_PER_SAMPLE = 60

# Counters of one batch_march_kernel launch on the default workload, valid only for
# the kernel sources they were taken on (SHA-256 over march.h, k_batch.hip and
# device_common.h, in that order); after any change the bench reports null for them
# until they are measured again:
#   traffic: HBM bytes per launch, FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB; factors
#     from a plain 256 MiB device-to-device copy in the same runs);
#   valu_lane_instr_per_sample: SQ_INSTS_VALU x 64 / logical samples.
MARCH_COUNTERS = {
    "sources_sha256": "48f922c47420f72247d12cf51568fe708b51a44ee8530213a00e1298f964fbd2",
    "traffic_bytes_per_launch": 324558168,
    "fetch_kib": 149866, "write_kib": 17268, "fetch_scale": 1.9997, "write_scale": 1.0,
    "valu_lane_instr_per_sample": 68.8,
}


def march_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    base = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2407_00179_amd", "csrc")
    for f in ("march.h", "k_batch.hip", "device_common.h"):
        with open(os.path.join(base, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------- CPU baseline (oracle)
_CPU = {}


def _cpu_worker(args):
    import oracle
    bricks, vol_dims, tf, prm, cam, px, py = _CPU["data"]
    parts = []
    samples = 0
    for b in bricks:
        r, z, n = oracle.render_brick(b.data, b.stored_lo, vol_dims, b.lo, b.hi, tf, prm, cam, px[args], py[args])
        parts.append((r, z))
        samples += int(n.sum())
    oracle.composite(np.stack([p[0] for p in parts]), np.stack([p[1] for p in parts]))
    return samples


def cpu_baseline(bricks, dims, tf, prm, cam, stride, cores):
    import oracle  # noqa: F401  (imported before forking)
    py, px = np.mgrid[0:cam.height:stride, 0:cam.width:stride]
    px, py = px.ravel(), py.ravel()
    _CPU["data"] = (bricks, dims, tf, prm, cam, px, py)
    chunks = np.array_split(np.arange(px.size), cores * 4)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        samples = sum(pool.map(_cpu_worker, chunks))
    dt = time.perf_counter() - t0
    return dict(value=samples / dt / 1e6, unit="Msamples/s", cores=cores, kind="oracle",
                sample=f"every {stride}th pixel in x and y ({px.size} rays) x {len(bricks)} bricks + composite, "
                       f"{samples} logical samples in {dt:.1f} s, FP64 numpy over a fork pool")


# ---------------------------------------------------------------- GPU sections
def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def bench_main(args, dpr, torch, vol_bricks, dims, tf, cfg, cam):
    dev = dpr.Device(0)
    w = dpr.World(dev, dims)
    # batched render enqueued directly (no graph replay) so HIP events bracket each kernel
    prm = dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, dpr.FLAG_NO_GRAPH)
    w.set_params(prm)
    for b in vol_bricks:
        w.add_brick(torch.from_numpy(b.data).to(dev.torch_device), b.lo, b.hi, b.ghost_lo, b.ghost_hi)
    w.commit()
    w.set_transfer_function(tf, 0.0, 1.0, cfg.density)
    w.set_camera(cam)
    W, H = cfg.image
    K = len(vol_bricks)
    out = dpr.Frame(dev, W, H)
    total = _count_samples(dpr, dev, w, [cam], K)
    w.set_camera(cam)
    # 8x8 item tiles (the library default, and the shape the autotuner picks on this
    # workload -- see the batch section); fixed here so every timed launch, and every
    # launch a profiler sees, has the same shape
    tile = (8, 8)
    w.set_batch_tile(*tile)

    def step():
        w.commit()                                        # blocked copies + macrocell ranges
        w.set_transfer_function(tf, 0.0, 1.0, cfg.density)  # majorants follow
        w.render_frame(out)                               # batched march + tile composite

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    march_ms, comp_ms = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        a, c = w.batch_timings()          # HIP events recorded around each kernel on the device stream
        march_ms.append(a)
        comp_ms.append(c)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    # the plain per-brick path on the same frame: 8 render_partial launches + dpr_composite
    parts = [dpr.Frame(dev, W, H) for _ in range(K)]

    def plain():
        for i, f in enumerate(parts):
            w.render_partial(i, f)
        dpr.composite(dev, parts, out, ids=list(range(K)))

    plain()
    torch.cuda.synchronize()
    ms_plain = _timed(torch, plain, max(3, args.steps))
    ms_plain_march = _timed(torch, lambda: [w.render_partial(i, f) for i, f in enumerate(parts)], max(3, args.steps))
    live = sum(int(torch.isfinite(f.depth).sum().item()) for f in parts)
    comp_bytes = K * W * H * 4 + live * 16 + W * H * 20
    ms_comp8 = _timed(torch, lambda: dpr.composite(dev, parts, out, ids=list(range(K))), max(3, args.steps))
    res = dict(ms_per_step=ms_step, samples=total, tile=tile, march_ms=float(np.mean(march_ms)),
               tile_comp_ms=float(np.mean(comp_ms)), ms_plain=ms_plain, ms_plain_march=ms_plain_march,
               comp8_ms=ms_comp8, comp_bytes=comp_bytes)
    w.release()
    for f in parts + [out]:
        f.release()
    return dev, res


def bench_composite128(args, dpr, torch, dev):
    """K = 128 sort-last composite at 3840x2160 (one GPU's share of a 128-rank frame):
    the rendered frame of one rank's 2048x1536x1280 FP16 brick plus 127 synthetic
    frames whose depth slabs lie in front of and behind that brick."""
    from synth import make_volume_large, synthetic_frames
    cfg = get_config("cfg5")
    dims = cfg.dims
    K, (W, H) = 128, cfg.image
    cam = orbit_camera(dims, W, H)
    # the brick's depth range from the camera: nearest point of the box, farthest corner
    h = 1.0 / max(dims)
    hi = np.array(dims, dtype=np.float64) * h
    eye = np.array(cam.eye, dtype=np.float64)
    t_min = float(np.linalg.norm(eye - np.clip(eye, 0.0, hi)))
    t_max = float(max(np.linalg.norm(eye - np.array([x, y, z])) for x in (0.0, hi[0]) for y in (0.0, hi[1])
                      for z in (0.0, hi[2])))
    rgba = torch.empty((K, H, W, 4), dtype=torch.float32, device=dev.torch_device)
    depth = torch.empty((K, H, W), dtype=torch.float32, device=dev.torch_device)
    log("  rendering the 2048x1536x1280 FP16 brick at 3840x2160 (frame 0)")
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range, log_uniform=cfg.log_sigma)
    vol = make_volume_large(dims, blobs, cfg.seeds["volume"], cfg.noise_amp, cfg.fbm_periods,
                            device=dev.torch_device)
    w = dpr.World(dev, dims)
    w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, 0))
    w.add_brick(vol, (0, 0, 0), dims, (0, 0, 0), (0, 0, 0))
    del vol
    w.commit()
    w.set_transfer_function(make_tf(cfg.seeds["tf"]), 0.0, 1.0, cfg.density)
    w.set_camera(cam)
    real = dpr.Frame(dev, W, H, rgba=rgba[0], depth=depth[0])
    w.render_partial(0, real)
    dev.sync()
    w.release()
    torch.cuda.empty_cache()
    synthetic_frames(K - 1, W, H, t_min, t_max, cfg.seeds["frames"], dev.torch_device, rgba[1:], depth[1:])
    frames = [real] + [dpr.Frame(dev, W, H, rgba=rgba[k], depth=depth[k]) for k in range(1, K)]
    out = dpr.Frame(dev, W, H)
    ids = list(np.random.default_rng(cfg.seeds["frames"]).permutation(K))
    for _ in range(2):
        dpr.composite(dev, frames, out, ids=ids)
    torch.cuda.synchronize()
    n = max(3, args.steps)
    evs = [_events(torch) for _ in range(n)]
    for e in evs:
        e[0].record()
        dpr.composite(dev, frames, out, ids=ids)
        e[1].record()
    torch.cuda.synchronize()
    ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    live = int(torch.isfinite(depth).sum().item())
    real_live = int(torch.isfinite(depth[0]).sum().item())
    alg = K * W * H * 4 + live * 16 + W * H * 20
    dense = K * W * H * 20 + W * H * 20
    for f in frames + [out]:
        f.release()
    del rgba, depth
    torch.cuda.empty_cache()
    gbs = alg / ms / 1e6
    return dict(workload="K=128 sort-last composite, 3840x2160: the rendered frame of a 2048x1536x1280 FP16 "
                         "brick + 127 synthetic RGBA32F+depth frames (depth slabs around the brick's range)",
                ms=ms, algorithmic_bytes=alg, dense_bytes=dense, GBps=gbs, frac_hbm=gbs / HBM_PEAK_GBS,
                real_frame_fragments=real_live, brick_depth_range=[t_min, t_max])


def _timed(torch, fn, n):
    evs = [_events(torch) for _ in range(n)]
    for e in evs:
        e[0].record()
        fn()
        e[1].record()
    torch.cuda.synchronize()
    return float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))


def _count_samples(dpr, dev, w, cams, n_bricks):
    total = 0
    for c in cams:
        w.set_camera(c)
        f = dpr.Frame(dev, c.width, c.height, counts=True)
        for i in range(n_bricks):
            f.counts.zero_()
            w.render_partial(i, f)
            dev.sync()
            total += int(f.counts.sum().item())
        f.release()
    return total


def bench_batch(args, dpr, torch, dev, w, cams, n_bricks, reps):
    """Persistent batched renderer (graph) vs plain per-brick launches, same world and cameras."""
    frames = [dpr.Frame(dev, c.width, c.height) for c in cams]
    samples = _count_samples(dpr, dev, w, cams, n_bricks)
    tw, th = w.autotune_batch(cams, frames)
    w.render_batch(cams, frames)
    torch.cuda.synchronize()
    ms_batch = _timed(torch, lambda: w.render_batch(cams, frames), reps)
    w.render_batch(cams, frames, dpr.FLAG_PLAIN)
    torch.cuda.synchronize()
    ms_plain = _timed(torch, lambda: w.render_batch(cams, frames, dpr.FLAG_PLAIN), reps)
    for f in frames:
        f.release()
    return dict(samples=samples, tile=[tw, th], ms_batch=ms_batch, ms_plain=ms_plain,
                msamples_batch=samples / ms_batch / 1e3, msamples_plain=samples / ms_plain / 1e3,
                speedup=ms_plain / ms_batch)


def bench_cfg3(args, dpr, torch, dev):
    """27 uneven k-d bricks of a 1024x1024x768 FP16 volume, 16 cameras at 2048x2048."""
    from synth import fibonacci_cameras, kd_split, make_volume_large, brick_ghosts
    cfg = get_config("cfg3")
    dims = cfg.dims
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range)
    vol = make_volume_large(dims, blobs, cfg.seeds["volume"], cfg.noise_amp, cfg.fbm_periods, device=dev.torch_device)
    boxes = kd_split(dims, cfg.n_bricks, cfg.seeds["kd"], 4.0)
    w = dpr.World(dev, dims)
    w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, 0))
    for lo, hi in boxes:
        glo, ghi = brick_ghosts(dims, lo, hi)
        sl = vol[lo[2] - glo[2]:hi[2] + ghi[2], lo[1] - glo[1]:hi[1] + ghi[1], lo[0] - glo[0]:hi[0] + ghi[0]]
        w.add_brick(sl.contiguous(), lo, hi, glo, ghi)
    del vol
    torch.cuda.empty_cache()
    w.commit()
    w.set_transfer_function(make_tf(cfg.seeds["tf"]), 0.0, 1.0, cfg.density)
    cams = fibonacci_cameras(dims, cfg.n_cams, *cfg.image)
    r = bench_batch(args, dpr, torch, dev, w, cams, len(boxes), 2)
    w.release()
    torch.cuda.empty_cache()
    r["workload"] = ("1024x1024x768 FP16 blob+fBm volume, 27 k-d bricks (<=4:1), 16 cameras x 2048x2048, "
                     "step 0.5 voxel, ERT 0.99")
    return r


def bench_deep(args, dpr, torch, dev):
    """Deep frames: the default 512^3 volume cut into 4x4x4 bricks of 128^3 cells dealt
    eight to each of 8 ranks at random (every rank's data non-convex), 1024x1024.  Each
    rank renders its deep frame (batched march + per-pixel fragment lists), then the 8
    deep frames are merged; both run here one after the other on the one GPU.  The
    same 64 bricks held by one rank and composited flat give the reference image and
    time."""
    cfg = get_config("cfg2")
    dims = cfg.dims
    R = 8
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range)
    vol = make_volume_small(dims, blobs, cfg.seeds["volume"], cfg.noise_amp)
    tf = make_tf(cfg.seeds["tf"])
    cam = orbit_camera(dims, *cfg.image)
    W, H = cam.width, cam.height
    P = W * H
    boxes = even_split(dims, (4, 4, 4))
    perm = np.random.default_rng(cfg.seeds["volume"] + 17).permutation(len(boxes))
    ranks = [sorted(int(i) for i in perm[r::R]) for r in range(R)]

    def world(ids):
        w = dpr.World(dev, dims)
        w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, 0))
        for i in ids:
            b = extract_brick(vol, dims, *boxes[i], 1)
            w.add_brick(torch.from_numpy(b.data).to(dev.torch_device), b.lo, b.hi, b.ghost_lo, b.ghost_hi)
        w.commit()
        w.set_transfer_function(tf, 0.0, 1.0, cfg.density)
        w.set_camera(cam)
        return w

    worlds = [world(ids) for ids in ranks]
    deeps = [dpr.DeepFrame(dev, W, H, len(ids)) for ids in ranks]
    out = dpr.Frame(dev, W, H)

    def render_all():
        for r in range(R):
            worlds[r].render_deep(r, deeps[r])

    reps = max(3, args.steps)
    render_all()
    dpr.composite_deep(dev, deeps, out)
    torch.cuda.synchronize()
    ms_render = _timed(torch, render_all, reps)
    ms_comp = _timed(torch, lambda: dpr.composite_deep(dev, deeps, out), reps)
    live = sum(int(d.counts.sum().item()) for d in deeps)
    max_frags = max(int(d.counts.max().item()) for d in deeps)
    samples = sum(_count_samples(dpr, dev, worlds[r], [cam], len(ranks[r])) for r in range(R))
    # the same bricks held by one rank, composited flat
    flat_w = world(range(len(boxes)))
    flat = dpr.Frame(dev, W, H)
    flat_w.render_frame(flat)
    torch.cuda.synchronize()
    ms_flat = _timed(torch, lambda: flat_w.render_frame(flat), reps)
    diff = float((out.rgba - flat.rgba).abs().max().item())
    alg = R * P * 4 + live * 20 + P * 20
    for h in worlds + deeps + [out, flat, flat_w]:
        h.release()
    torch.cuda.empty_cache()
    gbs = alg / ms_comp / 1e6
    return dict(workload="512^3 FP32 volume, 4x4x4 bricks of 128^3 dealt 8 per rank to 8 ranks at random, "
                         "1024x1024, step 0.5 voxel, ERT 0.99: 8 deep renders + deep composite",
                samples=samples, ms_render_8_ranks=ms_render, ms_composite_deep=ms_comp,
                msamples_deep=samples / (ms_render + ms_comp) / 1e3, live_fragments=live,
                max_fragments_per_pixel=max_frags, composite_algorithmic_bytes=alg, composite_GBps=gbs,
                composite_frac_hbm=gbs / HBM_PEAK_GBS, ms_one_rank_flat=ms_flat,
                max_abs_diff_vs_one_rank=diff)


def bench_iso(args, dpr, torch, dev, bricks, dims, tf, cfg, cam):
    """Opaque iso-surface at value 0.5 on the default workload (8 bricks, 1024x1024):
    with the volume's TF (surface and volume mixed in each fragment) and with a fully
    transparent TF (surface alone, macrocells off the surface skipped).  Each is
    timed as a whole batched frame (march + tile composite) against the same world
    without the surface."""
    w = dpr.World(dev, dims)
    w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, 0))
    for b in bricks:
        w.add_brick(torch.from_numpy(b.data).to(dev.torch_device), b.lo, b.hi, b.ghost_lo, b.ghost_hi)
    w.commit()
    w.set_camera(cam)
    f = dpr.Frame(dev, cam.width, cam.height)
    clear = np.array(tf, dtype=np.float32, copy=True)
    clear[:, 3] = 0.0
    reps = max(3, args.steps)
    out = {}
    for name, table in (("surface_and_volume", tf), ("surface_only", clear)):
        w.set_transfer_function(table, 0.0, 1.0, cfg.density)
        res = {}
        for mode, iso in (("iso", 0.5), ("none", None)):
            w.set_isosurface(iso)
            samples = _count_samples(dpr, dev, w, [cam], len(bricks))
            w.render_frame(f)
            torch.cuda.synchronize()
            ms = _timed(torch, lambda: w.render_frame(f), reps)
            res[mode] = (samples, ms, float((f.rgba[..., 3] == 1.0).float().mean().item()))
        (si, mi, cov), (sn, mn, _) = res["iso"], res["none"]
        out[name] = dict(samples=si, ms_frame=mi, msamples=si / mi / 1e3, surface_pixel_fraction=cov,
                         without_surface=dict(samples=sn, ms_frame=mn, msamples=sn / mn / 1e3))
    f.release()
    w.release()
    out["workload"] = ("512^3 FP32 volume, 2x2x2 bricks, 1024x1024, step 0.5 voxel, ERT 0.99, iso value 0.5 "
                       "(headlight, ambient 0.25, diffuse 0.75); batched frame, graph replay")
    return out


def bench_path(args, dpr, torch, dev):
    """Data-parallel path tracing of the default 512^3 volume at 1024x1024, 1 path per
    pixel, up to 4 real collisions, one directional light: the whole volume as 1
    brick, 2x2x2 bricks and 4x4x4 bricks (rays handed between bricks in waves).
    The images must agree bit for bit."""
    cfg = get_config("cfg2")
    dims = cfg.dims
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range)
    vol = make_volume_small(dims, blobs, cfg.seeds["volume"], cfg.noise_amp)
    tf = make_tf(cfg.seeds["tf"])
    cam = orbit_camera(dims, *cfg.image)
    reps = max(3, args.steps)
    out = {}
    ref = None
    for parts in ((1, 1, 1), (2, 2, 2), (4, 4, 4)):
        w = dpr.World(dev, dims)
        w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, 0))
        for lo, hi in even_split(dims, parts):
            b = extract_brick(vol, dims, lo, hi, 1)
            w.add_brick(torch.from_numpy(b.data).to(dev.torch_device), b.lo, b.hi, b.ghost_lo, b.ghost_hi)
        w.commit()
        w.set_transfer_function(tf, 0.0, 1.0, cfg.density)
        w.set_camera(cam)
        f = dpr.Frame(dev, cam.width, cam.height)
        st = w.render_path(f, max_bounces=4, spp=1, seed=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            w.render_path(f, max_bounces=4, spp=1, seed=1)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        img = f.rgba.clone()
        same = True if ref is None else bool(torch.equal(img, ref))
        if ref is None:
            ref = img
        n = int(np.prod(parts))
        out[f"{n}_bricks"] = dict(ms_frame=ms, mpaths_per_s=st["paths"] / ms / 1e3,
                                  mevents_per_s=(st["events"] + st["shadow_steps"]) / ms / 1e3, waves=st["waves"],
                                  forwards=st["forwards"], events=st["events"], shadow_steps=st["shadow_steps"],
                                  identical_to_1_brick=same)
        f.release()
        w.release()
        torch.cuda.empty_cache()
    out["workload"] = ("512^3 FP32 volume, 1024x1024, 1 path per pixel, <= 4 real collisions, delta tracking + "
                       "ratio-tracked shadow rays; the volume as 1, 8 and 64 bricks")
    return out


def bench_train(args, dpr, torch, dev):
    """256^3 FP32 density grid + 256-entry TF as parameters, 16 cameras at 512x512:
    the differentiable forward (with checkpoint stores) and the adjoint march."""
    import ctypes as C
    from paper_2407_00179_amd import _native as N
    from synth import fibonacci_cameras, perturb_blobs
    cfg = get_config("cfg4")
    dims = cfg.dims
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range)
    vol = make_volume_small(dims, blobs, cfg.seeds["volume"], cfg.noise_amp)
    tgt = make_volume_small(dims, perturb_blobs(blobs, cfg.seeds["perturb"]), cfg.seeds["volume"], cfg.noise_amp)
    tf = make_tf(cfg.seeds["tf"])
    cams = fibonacci_cameras(dims, cfg.n_cams, *cfg.image)
    n, W, H = len(cams), cfg.image[0], cfg.image[1]
    v = torch.tensor(vol, device=dev.torch_device)
    vt = torch.tensor(tgt, device=dev.torch_device)
    t = torch.tensor(tf, device=dev.torch_device)
    ca = (N.Camera * n)(*[dpr.to_c_camera(c) for c in cams])
    cp = dpr.Params(cfg.step_voxels, 1.0, 16, 0).c()
    nb = C.c_size_t()
    dpr.check(dpr.lib.dpr_train_workspace_size(N.I64x3(*dims), ca, n, cfg.step_voxels, C.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev.torch_device)
    out = torch.empty((n, H, W, 4), device=dev.torch_device)
    target = torch.empty_like(out)
    depth = torch.empty((n, H, W), device=dev.torch_device)
    gv = torch.zeros_like(v)
    gt = torch.zeros_like(t)

    def fwd(vol_t, img):
        dpr.check(dpr.lib.dpr_render_train_forward(dev.h, C.c_void_p(vol_t.data_ptr()), N.I64x3(*dims),
                                                   C.c_void_p(t.data_ptr()), t.shape[0], 0.0, 1.0, cfg.density,
                                                   C.byref(cp), ca, n, C.c_void_p(img.data_ptr()),
                                                   C.c_void_p(depth.data_ptr()), C.c_void_p(ws.data_ptr()),
                                                   nb.value))

    fwd(vt, target)
    fwd(v, out)
    g = (2.0 / out.numel()) * (out - target)

    def bwd():
        dpr.check(dpr.lib.dpr_render_backward(dev.h, C.c_void_p(v.data_ptr()), N.I64x3(*dims),
                                              C.c_void_p(t.data_ptr()), t.shape[0], 0.0, 1.0, cfg.density,
                                              C.byref(cp), ca, n, C.c_void_p(g.data_ptr()),
                                              C.c_void_p(ws.data_ptr()), nb.value, C.c_void_p(gv.data_ptr()),
                                              C.c_void_p(gt.data_ptr())))

    bwd()
    torch.cuda.synchronize()
    reps = max(3, args.steps // 2)
    ms_f = _timed(torch, lambda: fwd(v, out), reps)
    ms_b = _timed(torch, bwd, reps)
    return dict(workload="256^3 FP32 density + 256x4 TF as parameters, 16 cameras x 512x512, step 0.5 voxel, "
                         "ERT off, checkpoint every 64 segments",
                ms_forward=ms_f, ms_backward=ms_b, bwd_fwd_ratio=ms_b / ms_f,
                workspace_bytes=nb.value)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-stride", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sections", default="batch,cfg3,train,composite128,deep,iso,path")
    ap.add_argument("--main-only", action="store_true", help="only the default workload, no extra sections")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 256 MiB device-to-device copy first (scales HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library renders on one GPU; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    cfg = get_config("cfg2")
    dims = cfg.dims
    log("generating the 512^3 volume and its 8 bricks")
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range)
    vol = make_volume_small(dims, blobs, cfg.seeds["volume"], cfg.noise_amp)
    tf = make_tf(cfg.seeds["tf"])
    cam = orbit_camera(dims, *cfg.image)
    boxes = even_split(dims, cfg.parts)
    bricks = [extract_brick(vol, dims, lo, hi, 1) for lo, hi in boxes]
    del vol

    cpu = None
    if not args.no_cpu:
        import oracle
        cores = min(16, len(os.sched_getaffinity(0)))
        log(f"CPU oracle baseline on {cores} cores")
        cpu = cpu_baseline(bricks, dims, tf, oracle.RenderParams(cfg.step_voxels, cfg.ert, cfg.density), cam,
                           args.cpu_stride, cores)
        log(f"CPU oracle: {cpu['value']:.2f} Msamples/s")

    import torch
    import paper_2407_00179_amd as dpr
    if args.copy_calibration:
        x = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 268435456 bytes read, 268435456 bytes written")
        del x, y
    log("GPU: default workload")
    dev, r = bench_main(args, dpr, torch, bricks, dims, tf, cfg, cam)
    msamples = r["samples"] / (r["ms_per_step"] / 1e3) / 1e6
    achieved = OPS_PER_SAMPLE * r["samples"] / (r["march_ms"] / 1e3) / 1e12
    counters_valid = march_sources_sha256() == MARCH_COUNTERS["sources_sha256"]
    traffic = MARCH_COUNTERS["traffic_bytes_per_launch"] if counters_valid else None
    # share of the VALU issue slots the launch used, from the measured instruction count
    valu_issue_frac = (MARCH_COUNTERS["valu_lane_instr_per_sample"] * r["samples"] / (r["march_ms"] / 1e3)
                       / 1e12 / VALU_PEAK_TOPS) if counters_valid else None
    line = {
        "metric": "Msamples/s (logical ray-march samples, render + composite)",
        "value": msamples,
        "unit": "Msamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512^3 FP32 blob+noise volume, 2x2x2 bricks (257^3 stored, 1 ghost), 1024x1024, "
                               "step 0.5 voxel, ERT 0.99, 16^3 macrocells; per step: commit (blocked copies + "
                               "macrocell ranges), majorants, batched march of the 8 bricks, tile composite",
                   "logical_samples_per_step": r["samples"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic,
                     "kernel": "batch_march_kernel", "ms_per_launch": r["march_ms"],
                     "ops_per_sample": OPS_PER_SAMPLE, "valu_issue_frac": valu_issue_frac},
        "phases_ms": {"batch_march": r["march_ms"], "tile_composite": r["tile_comp_ms"]},
        "batch_tile": r["tile"],
        "plain_per_brick": {"ms_render_and_composite": r["ms_plain"], "ms_8_marches": r["ms_plain_march"],
                            "msamples": r["samples"] / r["ms_plain"] / 1e3,
                            "batched_speedup_march": r["ms_plain_march"] / r["march_ms"]},
        "composite_k8": {"ms": r["comp8_ms"], "algorithmic_bytes": r["comp_bytes"],
                         "GBps": r["comp_bytes"] / r["comp8_ms"] / 1e6,
                         "frac_hbm": r["comp_bytes"] / r["comp8_ms"] / 1e6 / HBM_PEAK_GBS},
        "cpu_baseline": cpu,
    }
    secs = [] if args.main_only else [s for s in args.sections.split(",") if s]
    if "batch" in secs:
        log("GPU: batched renderer on the default workload")
        w = dpr.World(dev, dims)
        w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, 0))
        for b in bricks:
            w.add_brick(torch.from_numpy(b.data).to(dev.torch_device), b.lo, b.hi, b.ghost_lo, b.ghost_hi)
        w.commit()
        w.set_transfer_function(tf, 0.0, 1.0, cfg.density)
        line["batch_cfg2"] = bench_batch(args, dpr, torch, dev, w, [cam], len(bricks), max(3, args.steps))
        w.release()
    if "cfg3" in secs:
        log("GPU: 27-brick 16-camera batched workload")
        line["batch_cfg3"] = bench_cfg3(args, dpr, torch, dev)
    if "train" in secs:
        log("GPU: differentiable render forward/backward")
        line["train_cfg4"] = bench_train(args, dpr, torch, dev)
    if "iso" in secs:
        log("GPU: iso-surface on the default workload")
        line["iso_cfg2"] = bench_iso(args, dpr, torch, dev, bricks, dims, tf, cfg, cam)
    if "path" in secs:
        log("GPU: data-parallel path tracing")
        line["path_cfg2"] = bench_path(args, dpr, torch, dev)
    if "deep" in secs:
        log("GPU: deep frames of an interleaved 8-rank partition")
        line["deep_8ranks"] = bench_deep(args, dpr, torch, dev)
    if "composite128" in secs:
        log("GPU: K=128 composite at 3840x2160")
        line["composite_k128"] = bench_composite128(args, dpr, torch, dev)
    dev.release()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
