#!/usr/bin/env python3
"""Benchmark of the data-parallel brick renderer + sort-last compositor on one MI355X.

Headline workload (one "step" = the whole hot path once) -- one rank's share of
a 128-rank large-volume run: a 2048x1536x1280 FP16 blob + fBm brick (8.05 GB)
rendered at 3840x2160 through one camera, step 0.5 voxel, ERT 0.99, 16^3
macrocells, then composited with 127 synthetic RGBA32F+depth frames of the
other ranks (depth slabs in front of and behind the brick):
  commit (8^3-blocked copy + macrocell min/max ranges, one pass)
  -> transfer-function majorants
  -> batched persistent march of the brick (+ its tile composite)
  -> sort-last composite of the K = 128 frames.
value = logical samples per second of the step (lattice segments of positive
length processed before termination, skipped ones included), in Msamples/s.

Reported beside it, from the same run: per-phase HIP-event times, the commit's
and the K=128 composite's GB/s against the 8 TB/s HBM peak, the plain per-brick
march, the VALU ceiling and the measured gather ceiling of the march, the
measured copy ceiling, and the counters of the dominant kernel from the
committed rocprofv3 summary when its sources are unchanged.  Secondary keys: the
512^3 FP32 2x2x2 step, the batched renderer on the 27-brick 16-camera FP16
workload, the backward/forward ratio of the differentiable renderer, deep
frames, iso-surfaces and path tracing.

The CPU baseline (the FP64 oracle, not tuned) runs last, over a spawned pool of
host processes reading the same input bytes from shared memory: the render on a
pixel sample of the headline brick, the K=128 composite on a band of rows, the
K=8 composite of the 512^3 step's partial frames in full, and the gradient on a
pixel sample of one 512x512 camera of the 256^3 training workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import re
import shutil
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
CSRC = os.path.join(ROOT, "paper_2407_00179_amd", "csrc")
# source files whose change invalidates a kernel's stored counters
KERNEL_SOURCES = {
    "batch_march_kernel": ("march.h", "k_batch.hip", "device_common.h"),
    "commit_kernel": ("k_commit.hip", "commit_span.h", "device_common.h", "kernels.h"),
    "composite_fast_kernel": ("k_composite.hip", "composite.h", "kernels.h"),
}


def sources_sha256(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_counters(kernel, workload):
    """Counters of `kernel` on `workload` from the committed rocprofv3 summaries
    (a `counters-json:` line in a profiles/*.md file), if taken on the current
    sources; else None."""
    pdir = os.path.join(ROOT, "profiles")
    want = sources_sha256(kernel)
    for name in sorted(os.listdir(pdir)) if os.path.isdir(pdir) else []:
        if not name.endswith(".md"):
            continue
        with open(os.path.join(pdir, name)) as fh:
            for line in fh:
                m = re.match(r"\s*counters-json:\s*(\{.*\})\s*$", line)
                if not m:
                    continue
                c = json.loads(m.group(1))
                if c.get("kernel") == kernel and c.get("workload") == workload and c.get("sources_sha256") == want:
                    c["file"] = "profiles/" + name
                    return c
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


# ---------------------------------------------------------------- headline: one rank's share, K = 128
def brick_depth_range(dims, cam):
    """Nearest point and farthest corner of the brick's box from the eye."""
    h = 1.0 / max(dims)
    hi = np.array(dims, dtype=np.float64) * h
    eye = np.array(cam.eye, dtype=np.float64)
    t_min = float(np.linalg.norm(eye - np.clip(eye, 0.0, hi)))
    t_max = float(max(np.linalg.norm(eye - np.array([x, y, z])) for x in (0.0, hi[0]) for y in (0.0, hi[1])
                      for z in (0.0, hi[2])))
    return t_min, t_max


def bench_rank_share(args, dpr, torch, dev, keep_host):
    from synth import make_volume_large, synthetic_frames
    cfg = get_config("cfg5")
    dims = cfg.dims
    (W, H), K = cfg.image, 128
    cam = orbit_camera(dims, W, H)
    log("  generating the 2048x1536x1280 FP16 brick on the GPU")
    blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range, log_uniform=cfg.log_sigma)
    vol = make_volume_large(dims, blobs, cfg.seeds["volume"], cfg.noise_amp, cfg.fbm_periods,
                            device=dev.torch_device)
    host = vol.cpu().numpy() if keep_host else None
    tf = make_tf(cfg.seeds["tf"])
    w = dpr.World(dev, dims)
    # batched render enqueued directly (no graph replay) so HIP events bracket its kernels
    w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, dpr.FLAG_NO_GRAPH))
    w.add_brick(vol, (0, 0, 0), dims, (0, 0, 0), (0, 0, 0))
    voxel_bytes = vol.numel() * vol.element_size()
    del vol
    torch.cuda.empty_cache()
    w.commit()
    w.set_transfer_function(tf, 0.0, 1.0, cfg.density)
    w.set_camera(cam)
    # logical samples (per-pixel counts, written by the plain march) and the plain
    # per-brick launch itself
    cf = dpr.Frame(dev, W, H, counts=True)
    w.render_partial(0, cf)
    dev.sync()
    samples = int(cf.counts.sum().item())
    hits = int(torch.isfinite(cf.depth).sum().item())
    pf = dpr.Frame(dev, W, H)
    w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, dpr.FLAG_PLAIN))
    ms_plain = _timed(torch, lambda: w.render_partial(0, pf), 3)
    w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, dpr.FLAG_NO_GRAPH))
    # gather ceiling: the march's loads for the same samples, no dependence between samples
    sink = torch.empty((H, W), dtype=torch.float32, device=dev.torch_device)
    w.measure_gather(0, cf.counts, sink)
    ms_gather = _timed(torch, lambda: w.measure_gather(0, cf.counts, sink), 5)
    # the K = 128 frames: frame 0 is this rank's, rendered every step; 127 synthetic
    t_min, t_max = brick_depth_range(dims, cam)
    rgba = torch.empty((K, H, W, 4), dtype=torch.float32, device=dev.torch_device)
    depth = torch.empty((K, H, W), dtype=torch.float32, device=dev.torch_device)
    synthetic_frames(K - 1, W, H, t_min, t_max, cfg.seeds["frames"], dev.torch_device, rgba[1:], depth[1:])
    frames = [dpr.Frame(dev, W, H, rgba=rgba[k], depth=depth[k]) for k in range(K)]
    real = frames[0]
    out = dpr.Frame(dev, W, H)
    ids = [int(i) for i in np.random.default_rng(cfg.seeds["frames"]).permutation(K)]
    tile = (8, 8)
    w.set_batch_tile(*tile)

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        w.commit()                                            # blocked copy + macrocell ranges
        if ev is not None:
            ev[1].record()
        w.set_transfer_function(tf, 0.0, 1.0, cfg.density)   # majorants follow (at the render)
        w.render_frame(real)                                  # majorants, batched march, tile composite
        if ev is not None:
            ev[2].record()
        dpr.composite(dev, frames, out, ids=ids)              # K = 128 sort-last composite
        if ev is not None:
            ev[3].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    march_ms, tile_ms = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
        a, c = w.batch_timings()    # HIP events recorded around the march and tile kernels on the device stream
        march_ms.append(a)
        tile_ms.append(c)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    commit_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    render_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    comp_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    # the rendered frame equals the plain per-brick march bit for bit
    same = bool(torch.equal(real.rgba, cf.rgba) and torch.equal(real.depth, cf.depth))
    live = int(torch.isfinite(depth).sum().item())
    comp_alg = K * W * H * 4 + live * 16 + W * H * 20
    ncells = int(np.prod([(d + cfg.macrocell - 1) // cfg.macrocell for d in dims]))
    commit_alg = 2 * voxel_bytes + 8 * ncells          # every stored voxel read once and written once
    # FP16 bricks whose voxel-pair copy would reach 4 GiB (this one) are stored as
    # 2-byte voxels, so the commit writes exactly the algorithmic bytes
    commit_actual = commit_alg
    res = dict(ms_per_step=wall * 1e3 / args.steps, samples=samples, hit_pixels=hits, tile=tile,
               phases=dict(commit=commit_ms, render_frame=render_ms, batch_march=float(np.mean(march_ms)),
                           tile_composite=float(np.mean(tile_ms)), composite_k128=comp_ms),
               ms_plain_march=ms_plain, ms_gather_probe=ms_gather, identical_to_plain=same,
               comp_alg=comp_alg, comp_dense=K * W * H * 20 + W * H * 20, live_fragments=live,
               commit_alg=commit_alg, commit_actual=commit_actual, voxel_bytes=voxel_bytes,
               depth_range=[t_min, t_max])
    # a band of rows of the 128 frames for the oracle's composite leg
    band = None
    if keep_host:
        r0, r1 = H // 2 - 32, H // 2 + 32
        band = dict(rgba=rgba[:, r0:r1].cpu().numpy(), depth=depth[:, r0:r1].cpu().numpy(), ids=np.array(ids),
                    rows=(r0, r1))
    for f in frames + [out, cf, pf]:
        f.release()
    w.release()
    del rgba, depth, sink
    torch.cuda.empty_cache()
    return res, host, band, cam, tf


def copy_ceiling(torch, nbytes=2 << 30, reps=10):
    """Plain device-to-device copy: achievable read+write HBM GB/s."""
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    ms = _timed(torch, lambda: y.copy_(x), reps)
    del x, y
    torch.cuda.empty_cache()
    return dict(bytes_read=nbytes, bytes_written=nbytes, ms=ms, GBps=2 * nbytes / ms / 1e6)


# ---------------------------------------------------------------- secondary: 512^3 FP32, 2x2x2 bricks
def bench_cfg2_step(args, dpr, torch, dev, vol_bricks, dims, tf, cfg, cam, keep_host=False):
    w = dpr.World(dev, dims)
    w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, dpr.FLAG_NO_GRAPH))
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
    w.set_batch_tile(8, 8)

    def step():
        w.commit()
        w.set_transfer_function(tf, 0.0, 1.0, cfg.density)
        w.render_frame(out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    march_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        march_ms.append(w.batch_timings()[0])
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    parts = [dpr.Frame(dev, W, H) for _ in range(K)]
    w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, dpr.FLAG_PLAIN))
    ms_plain_march = _timed(torch, lambda: [w.render_partial(i, f) for i, f in enumerate(parts)], max(3, args.steps))
    w.set_params(dpr.Params(cfg.step_voxels, cfg.ert, cfg.macrocell, dpr.FLAG_NO_GRAPH))
    # the same 8 partial frames through the persistent kernel, one brick per launch
    ms_partials = _timed(torch, lambda: [w.render_partial(i, f) for i, f in enumerate(parts)], max(3, args.steps))
    live = sum(int(torch.isfinite(f.depth).sum().item()) for f in parts)
    comp_bytes = K * W * H * 4 + live * 16 + W * H * 20
    ms_comp8 = _timed(torch, lambda: dpr.composite(dev, parts, out, ids=list(range(K))), max(3, args.steps))
    ms_comp8_dev = _timed_back_to_back(torch, lambda: dpr.composite(dev, parts, out, ids=list(range(K))), 20)
    # the 8 partial frames on the host for the oracle's K = 8 composite leg
    k8 = None
    if keep_host:
        k8 = dict(rgba=torch.stack([f.rgba for f in parts]).cpu().numpy(),
                  depth=torch.stack([f.depth for f in parts]).cpu().numpy(), ids=np.arange(K))
    w.release()
    for f in parts + [out]:
        f.release()
    march = float(np.mean(march_ms))
    return k8, dict(workload="512^3 FP32 blob+noise volume, 2x2x2 bricks (257^3 stored, 1 ghost), 1024x1024, step 0.5 "
                         "voxel, ERT 0.99; per step: commit, majorants, batched march of the 8 bricks, tile composite",
                logical_samples=total, ms_per_step=ms_step, msamples_step=total / ms_step / 1e3,
                ms_batch_march=march, msamples_march=total / march / 1e3,
                valu_frac=OPS_PER_SAMPLE * total / (march / 1e3) / 1e12 / VALU_PEAK_TOPS,
                ms_plain_8_marches=ms_plain_march, batched_speedup_march=ms_plain_march / march,
                ms_8_partials_persistent=ms_partials,
                composite_k8=dict(ms=ms_comp8, algorithmic_bytes=comp_bytes, GBps=comp_bytes / ms_comp8 / 1e6,
                                  frac_hbm=comp_bytes / ms_comp8 / 1e6 / HBM_PEAK_GBS,
                                  how="HIP events around each call (the call's host-side marshalling included)",
                                  ms_back_to_back=ms_comp8_dev,
                                  GBps_back_to_back=None if not ms_comp8_dev else comp_bytes / ms_comp8_dev / 1e6,
                                  frac_hbm_back_to_back=None if not ms_comp8_dev else
                                  comp_bytes / ms_comp8_dev / 1e6 / HBM_PEAK_GBS))


def _timed(torch, fn, n):
    evs = [_events(torch) for _ in range(n)]
    for e in evs:
        e[0].record()
        fn()
        e[1].record()
    torch.cuda.synchronize()
    return float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))


def _timed_back_to_back(torch, fn, n):
    """Device time per call of ``fn`` with the host's per-call cost hidden: a spin
    kernel holds the stream while ``n`` calls are enqueued behind it, so the events
    bracket launches that run back to back.  None where the spin kernel is missing."""
    sleep = getattr(torch.cuda, "_sleep", None)
    if sleep is None:
        return None
    fn()
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    sleep(50_000_000)
    e0.record()
    for _ in range(n):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


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


# ---------------------------------------------------------------- CPU baseline (the oracle, not tuned)
_W = {}


def _worker_init(paths):
    for k, p in paths.items():
        _W[k] = np.load(p, mmap_mode="r")


def _leg_render(job):
    import oracle
    dims, tf, prm, cam, px, py = job
    _, _, n = oracle.render_brick(_W["volume"], (0, 0, 0), dims, (0, 0, 0), dims, tf, prm, cam, px, py)
    return int(n.sum())


def _leg_composite(job):
    import oracle
    name, c0, c1, ids = job
    rgba = np.asarray(_W[name + "_rgba"][:, :, c0:c1])
    depth = np.asarray(_W[name + "_depth"][:, :, c0:c1])
    oracle.composite(rgba, depth, ids)
    return 0


def _leg_grad(job):
    import oracle
    dims, tf, prm, cam, px, py = job
    target = [np.zeros((px.size, 4))]
    oracle.loss_and_grad(np.asarray(_W["train_volume"]), dims, tf, prm, [cam], target, pixels=[(px, py)],
                         n_elems=4 * px.size)
    return 0


def _segments(cam, dims, step_voxels, px, py):
    """Lattice segments of positive length per ray through the whole volume (ERT off)."""
    import oracle
    h = 1.0 / max(dims)
    dt = step_voxels * h
    o, d = oracle.camera_rays(cam, px, py)
    t_in, t_out, hit = oracle.clip_box(o, d, np.zeros(3), np.array(dims, dtype=np.float64) * h)
    s0, s1 = np.floor(t_in / dt), np.ceil(t_out / dt) - 1.0
    first = np.minimum((s0 + 1) * dt, t_out) - np.maximum(s0 * dt, t_in) > 0
    last = np.minimum((s1 + 1) * dt, t_out) - np.maximum(s1 * dt, t_in) > 0
    n = (s1 - s0 + 1) - (~first) - ((~last) & (s1 > s0))
    return int(np.sum(np.where(hit, np.maximum(n, 0), 0)))


def cpu_baseline(args, host_volume, band, cam5, tf5, k8=None):
    import oracle
    from synth import fibonacci_cameras
    cores = min(16, len(os.sched_getaffinity(0)))
    shm = os.path.join("/dev/shm" if os.path.isdir("/dev/shm") else "/tmp", f"dpr_bench_{os.getpid()}")
    os.makedirs(shm, exist_ok=True)
    try:
        cfg5, cfg4 = get_config("cfg5"), get_config("cfg4")
        paths = {"volume": os.path.join(shm, "volume.npy"), "band_rgba": os.path.join(shm, "band_rgba.npy"),
                 "band_depth": os.path.join(shm, "band_depth.npy"), "train_volume": os.path.join(shm, "train.npy")}
        np.save(paths["volume"], host_volume)
        np.save(paths["band_rgba"], band["rgba"])
        np.save(paths["band_depth"], band["depth"])
        if k8 is not None:
            paths.update(k8_rgba=os.path.join(shm, "k8_rgba.npy"), k8_depth=os.path.join(shm, "k8_depth.npy"))
            np.save(paths["k8_rgba"], k8["rgba"])
            np.save(paths["k8_depth"], k8["depth"])
        blobs = make_blobs(cfg4.dims, cfg4.seeds["volume"], cfg4.n_blobs, cfg4.s_range, cfg4.a_range)
        np.save(paths["train_volume"], make_volume_small(cfg4.dims, blobs, cfg4.seeds["volume"], cfg4.noise_amp))
        legs = {}
        with mp.get_context("spawn").Pool(cores, initializer=_worker_init, initargs=(paths,)) as pool:
            pool.map(abs, range(4 * cores))   # workers started and initialised before any leg is timed
            # render: every stride-th pixel in x and y of the headline frame
            s = args.cpu_stride
            py, px = np.mgrid[0:cam5.height:s, 0:cam5.width:s]
            px, py = px.ravel(), py.ravel()
            prm = oracle.RenderParams(cfg5.step_voxels, cfg5.ert, cfg5.density)
            nj = 8 * cores   # interleaved pixels, so every job gets its share of the rays that hit the brick
            jobs = [(cfg5.dims, tf5, prm, cam5, px[j::nj], py[j::nj]) for j in range(nj)]
            t0 = time.perf_counter()
            samples = sum(pool.map(_leg_render, jobs, chunksize=1))
            dt = time.perf_counter() - t0
            render = dict(value=samples / dt / 1e6, unit="Msamples/s", seconds=dt, samples=samples,
                          sample=f"every {s}th pixel in x and y of the 3840x2160 frame ({px.size} rays) through the "
                                 f"2048x1536x1280 FP16 brick, ERT 0.99: {samples} logical samples")
            # composite: the 128 frames on a band of rows
            K, R, Wd = band["depth"].shape
            live = int(np.isfinite(band["depth"]).sum())
            cols = np.array_split(np.arange(Wd), 4 * cores)
            t0 = time.perf_counter()
            pool.map(_leg_composite, [("band", int(c[0]), int(c[-1]) + 1, band["ids"]) for c in cols], chunksize=1)
            dt = time.perf_counter() - t0
            alg = K * R * Wd * 4 + live * 16 + R * Wd * 20
            legs["composite_k128"] = dict(value=alg / dt / 1e9, unit="GB/s", seconds=dt, algorithmic_bytes=alg,
                                          sample=f"rows {band['rows'][0]}..{band['rows'][1] - 1} of the 128 "
                                                 f"3840x2160 frames ({R * Wd} pixels)")
            # composite: the 8 partial frames of the 512^3 step, every pixel
            if k8 is not None:
                K8, H8, W8 = k8["depth"].shape
                live8 = int(np.isfinite(k8["depth"]).sum())
                cols8 = np.array_split(np.arange(W8), 4 * cores)
                t0 = time.perf_counter()
                pool.map(_leg_composite, [("k8", int(c[0]), int(c[-1]) + 1, k8["ids"]) for c in cols8], chunksize=1)
                dt = time.perf_counter() - t0
                alg8 = K8 * H8 * W8 * 4 + live8 * 16 + H8 * W8 * 20
                legs["composite_k8"] = dict(value=alg8 / dt / 1e9, unit="GB/s", seconds=dt, algorithmic_bytes=alg8,
                                            sample=f"all {H8 * W8} pixels of the 8 partial {W8}x{H8} frames of the "
                                                   f"512^3 FP32 step")
            # gradient: one 512x512 camera of the 256^3 training volume, every gs-th pixel
            gs = 4
            cam4 = fibonacci_cameras(cfg4.dims, cfg4.n_cams, *cfg4.image)[0]
            gy, gx = np.mgrid[0:cam4.height:gs, 0:cam4.width:gs]
            gx, gy = gx.ravel(), gy.ravel()
            prm4 = oracle.RenderParams(cfg4.step_voxels, 1.0, cfg4.density)
            tf4 = make_tf(cfg4.seeds["tf"])
            gjobs = [(cfg4.dims, tf4, prm4, cam4, gx[j::nj], gy[j::nj]) for j in range(nj)]
            t0 = time.perf_counter()
            pool.map(_leg_grad, gjobs, chunksize=1)
            dt = time.perf_counter() - t0
            gsamples = _segments(cam4, cfg4.dims, cfg4.step_voxels, gx, gy)
            legs["gradient_cfg4"] = dict(value=gsamples / dt / 1e6, unit="Msamples/s (forward + backward)",
                                         seconds=dt, samples=gsamples,
                                         sample=f"every {gs}th pixel in x and y of one 512x512 camera ({gx.size} "
                                                f"rays) of the 256^3 FP32 training volume, ERT off, L2 loss "
                                                f"against a zero target")
        return dict(value=render["value"], unit="Msamples/s", cores=cores, kind="oracle", sample=render["sample"],
                    seconds=render["seconds"], legs=legs,
                    how="FP64 numpy oracle over a spawned pool of host processes reading the inputs from shared "
                        "memory")
    finally:
        shutil.rmtree(shm, ignore_errors=True)


def roofline_of(r, copy):
    """Roofline of the step's dominant kernel (the longest of commit, march and
    K = 128 composite, by HIP-event time)."""
    ph = r["phases"]
    cands = {"batch_march_kernel": ph["batch_march"], "commit_kernel": ph["commit"],
             "composite_fast_kernel": ph["composite_k128"]}
    kern = max(cands, key=cands.get)
    ms = cands[kern]
    if kern == "batch_march_kernel":
        work = "3840x2160 march of the 2048x1536x1280 FP16 brick, ERT 0.99"
        achieved = OPS_PER_SAMPLE * r["samples"] / (ms / 1e3) / 1e12
        gather = OPS_PER_SAMPLE * r["samples"] / (r["ms_gather_probe"] / 1e3) / 1e12
        peak, bound = (VALU_PEAK_TOPS, "alu") if VALU_PEAK_TOPS <= gather else (gather, "gather")
        rf = dict(bound=bound, achieved=achieved, peak=peak, unit="Tops/s", frac=achieved / peak,
                  per_unit=f"{OPS_PER_SAMPLE} VALU lane-op slots per logical sample x {r['samples']} samples",
                  ceilings=dict(valu_Tops=VALU_PEAK_TOPS, gather_Tops=gather,
                                valu_Msamples=VALU_PEAK_TOPS * 1e6 / OPS_PER_SAMPLE,
                                gather_Msamples=r["samples"] / r["ms_gather_probe"] / 1e3,
                                gather_probe_ms=r["ms_gather_probe"]),
                  frac_of_valu_peak=achieved / VALU_PEAK_TOPS)
    elif kern == "commit_kernel":
        work = "commit of the 2048x1536x1280 FP16 brick"
        achieved = r["commit_alg"] / ms / 1e6
        rf = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                  per_unit="every stored voxel read once and written once (2 + 2 B) + 8 B per macrocell",
                  frac_of_copy_ceiling=achieved / copy["GBps"])
    else:
        work = "K=128 composite at 3840x2160"
        achieved = r["comp_alg"] / ms / 1e6
        rf = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                  per_unit="per pixel: 128 depths (4 B), RGBA of live fragments (16 B), 20 B written",
                  frac_of_copy_ceiling=achieved / copy["GBps"])
    c = stored_counters(kern, work)
    rf.update(kernel=kern, workload=work, ms_per_launch=ms,
              traffic=None if c is None else c["traffic_bytes_per_launch"],
              counters=None if c is None else {k: v for k, v in c.items() if k not in ("kernel", "workload")})
    return rf


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-stride", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sections", default="cfg2,batch,cfg3,train,iso,path,deep")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (one rank's share of the data-parallel run); "
                                   "runs on several GPUs are not supported", "n_gpus": args.gpus}))
        sys.exit(2)
    secs = [s for s in args.sections.split(",") if s and s != "none"]

    import torch
    import paper_2407_00179_amd as dpr
    dev = dpr.Device(0)
    log("GPU: copy ceiling")
    copy = copy_ceiling(torch)
    log("GPU: one rank's share of a 128-rank run (headline)")
    r, host, band, cam5, tf5 = bench_rank_share(args, dpr, torch, dev, keep_host=not args.no_cpu)
    ph = r["phases"]
    value = r["samples"] / (r["ms_per_step"] / 1e3) / 1e6
    cfg5 = get_config("cfg5")
    line = {
        "metric": "Msamples/s + composite GB/s (% HBM peak) per GPU; backward/forward time ratio",
        "value": value,
        "unit": "Msamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16 storage, f32 math",
        "data": "synthetic",
        "config": {"workload": "one rank's share of a 128-rank large-volume run: 2048x1536x1280 FP16 blob+fBm brick "
                               "(8.05 GB) -> 3840x2160 partial frame (step 0.5 voxel, ERT 0.99, 16^3 macrocells), "
                               "then K=128 sort-last composite with 127 synthetic RGBA32F+depth frames; per step: "
                               "commit (blocked copy + macrocell ranges), majorants, batched march, tile composite, "
                               "K=128 composite",
                   "logical_samples_per_step": r["samples"], "hit_pixels": r["hit_pixels"],
                   "image": list(cfg5.image), "brick": list(cfg5.dims), "batch_tile": list(r["tile"])},
        "roofline": roofline_of(r, copy),
        "phases_ms": ph,
        "render_msamples": r["samples"] / ph["batch_march"] / 1e3,
        "commit": {"ms": ph["commit"], "algorithmic_bytes": r["commit_alg"],
                   "GBps": r["commit_alg"] / ph["commit"] / 1e6,
                   "frac_hbm": r["commit_alg"] / ph["commit"] / 1e6 / HBM_PEAK_GBS,
                   "bytes_moved": r["commit_actual"], "GBps_moved": r["commit_actual"] / ph["commit"] / 1e6,
                   "frac_copy_ceiling": r["commit_alg"] / ph["commit"] / 1e6 / copy["GBps"],
                   "layout": "8^3 blocks of 2-byte FP16 voxels (the pair layout is kept for bricks below 4 GiB)"},
        "composite_k128": {"ms": ph["composite_k128"], "algorithmic_bytes": r["comp_alg"],
                           "dense_bytes": r["comp_dense"], "GBps": r["comp_alg"] / ph["composite_k128"] / 1e6,
                           "frac_hbm": r["comp_alg"] / ph["composite_k128"] / 1e6 / HBM_PEAK_GBS,
                           "frac_copy_ceiling": r["comp_alg"] / ph["composite_k128"] / 1e6 / copy["GBps"],
                           "live_fragments": r["live_fragments"], "brick_depth_range": r["depth_range"]},
        "plain_per_brick": {"ms_march": r["ms_plain_march"],
                            "msamples": r["samples"] / r["ms_plain_march"] / 1e3,
                            "batched_speedup_march": r["ms_plain_march"] / ph["batch_march"],
                            "identical_bits": r["identical_to_plain"]},
        "copy_ceiling": copy,
        "cpu_baseline": None,
    }
    cfg = get_config("cfg2")
    dims = cfg.dims
    tf = make_tf(cfg.seeds["tf"])
    cam = orbit_camera(dims, *cfg.image)
    bricks = None
    k8 = None
    if any(s in secs for s in ("cfg2", "batch", "iso")):
        log("generating the 512^3 volume and its 8 bricks")
        blobs = make_blobs(dims, cfg.seeds["volume"], cfg.n_blobs, cfg.s_range, cfg.a_range)
        vol = make_volume_small(dims, blobs, cfg.seeds["volume"], cfg.noise_amp)
        bricks = [extract_brick(vol, dims, lo, hi, 1) for lo, hi in even_split(dims, cfg.parts)]
        del vol
    if "cfg2" in secs:
        log("GPU: 512^3 FP32 2x2x2 step")
        k8, line["step_cfg2"] = bench_cfg2_step(args, dpr, torch, dev, bricks, dims, tf, cfg, cam,
                                                keep_host=not args.no_cpu)
    if "batch" in secs:
        log("GPU: batched renderer vs plain launches on the 512^3 2x2x2 workload")
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
        log("GPU: iso-surface on the 512^3 2x2x2 workload")
        line["iso_cfg2"] = bench_iso(args, dpr, torch, dev, bricks, dims, tf, cfg, cam)
    if "path" in secs:
        log("GPU: data-parallel path tracing")
        line["path_cfg2"] = bench_path(args, dpr, torch, dev)
    if "deep" in secs:
        log("GPU: deep frames of an interleaved 8-rank partition")
        line["deep_8ranks"] = bench_deep(args, dpr, torch, dev)
    dev.release()
    if not args.no_cpu:
        log("CPU oracle baseline (render, K=128 and K=8 composite and gradient legs)")
        line["cpu_baseline"] = cpu_baseline(args, host, band, cam5, tf5, k8)
        log(f"CPU oracle: {line['cpu_baseline']['value']:.2f} Msamples/s on {line['cpu_baseline']['cores']} cores")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
