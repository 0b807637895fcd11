"""MI355X-native data-parallel volume rendering and sort-last compositing.

Python face of the C ABI in ``include/dpr.h``.  Every step of rendering and
compositing runs in the HIP kernels of ``libdpr.so``; this module only passes
pointers, sizes and the current torch stream.  torch supplies device memory and
streams, nothing else.
"""

from __future__ import annotations

import atexit
import ctypes as C
import weakref
from dataclasses import dataclass

import numpy as np

from . import _native as N
from ._native import (DprError, F16, F32, FLAG_F16_HALVES, FLAG_NO_GRAPH, FLAG_NO_SKIP, FLAG_PLAIN, FLAG_QUEUE_COVERAGE,
                      FLAG_WIDE_OFFSETS,  # noqa: F401
                      check, lib)

__all__ = ["Device", "World", "Frame", "DprError", "composite", "Params", "to_c_camera", "render_train",
           "DprRenderFn"]


def _torch():
    import torch
    return torch


# objects still holding library handles; released at interpreter exit, children
# before their device, so no release runs while modules are being torn down
_live = weakref.WeakSet()


def _release_all():
    for kind in (DeepFrame, Frame, World, Device):
        for o in [o for o in list(_live) if isinstance(o, kind)]:
            try:
                o.release()
            except Exception:
                pass


atexit.register(_release_all)


@dataclass
class Params:
    step_voxels: float = 0.5
    ert_threshold: float = 0.99
    macrocell_cells: int = 16
    flags: int = 0

    def c(self):
        return N.RenderParams(self.step_voxels, self.ert_threshold, self.macrocell_cells, self.flags)


def to_c_camera(cam):
    """Any object with eye, center, up, fovy_deg, width, height -> dpr_camera."""
    return N.Camera((C.c_double * 3)(*cam.eye), (C.c_double * 3)(*cam.center), (C.c_double * 3)(*cam.up),
                    float(cam.fovy_deg), int(cam.width), int(cam.height))


class Device:
    """One GPU plus the HIP stream the library enqueues on (torch's current stream by default)."""

    def __init__(self, index=0, stream=None):
        torch = _torch()
        self.index = index
        self.torch_device = torch.device("cuda", index)
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        h = C.c_void_p()
        check(lib.dpr_device_create(index, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h
        _live.add(self)

    def set_stream(self, stream):
        self.stream = stream
        check(lib.dpr_device_set_stream(self.h, C.c_void_p(stream.cuda_stream)))

    def sync(self):
        check(lib.dpr_device_sync(self.h))

    def info(self):
        cu, ws = C.c_int32(), C.c_int32()
        check(lib.dpr_device_info(self.h, C.byref(cu), C.byref(ws)))
        return cu.value, ws.value

    def release(self):
        if self.h:
            lib.dpr_device_release(self.h)
            self.h = None


class Frame:
    """W x H premultiplied RGBA + depth held in torch tensors (borrowed by the library)."""

    def __init__(self, dev: Device, width, height, rgba=None, depth=None, counts=False):
        torch = _torch()
        self.dev = dev
        self.width, self.height = int(width), int(height)
        if rgba is None:
            rgba = torch.empty((self.height, self.width, 4), dtype=torch.float32, device=dev.torch_device)
        if depth is None:
            depth = torch.empty((self.height, self.width), dtype=torch.float32, device=dev.torch_device)
        assert rgba.is_contiguous() and depth.is_contiguous()
        assert rgba.dtype == torch.float32 and depth.dtype == torch.float32
        assert rgba.numel() == 4 * self.width * self.height and depth.numel() == self.width * self.height
        self.rgba, self.depth = rgba, depth
        h = C.c_void_p()
        check(lib.dpr_frame_wrap(dev.h, self.width, self.height, C.c_void_p(rgba.data_ptr()),
                                 C.c_void_p(depth.data_ptr()), C.byref(h)))
        self.h = h
        _live.add(self)
        self.counts = None
        if counts:
            self.attach_counts()

    def attach_counts(self, counts=None):
        torch = _torch()
        if counts is None:
            counts = torch.zeros((self.height, self.width), dtype=torch.int32, device=self.dev.torch_device)
        self.counts = counts
        check(lib.dpr_frame_attach_counts(self.h, C.c_void_p(counts.data_ptr())))
        return counts

    def release(self):
        if self.h:
            lib.dpr_frame_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class DeepFrame:
    """Deep (multi-fragment) frame in torch tensors borrowed by the library: per
    pixel a fragment count and up to ``capacity`` layers of premultiplied RGBA,
    depth and intrinsic fragment id, layer-major (shape (capacity, H, W, ...)); a
    pixel's fragments fill layers 0..count-1 front to back."""

    def __init__(self, dev: Device, width, height, capacity):
        torch = _torch()
        self.dev = dev
        self.width, self.height, self.capacity = int(width), int(height), int(capacity)
        d = dev.torch_device
        self.counts = torch.zeros((self.height, self.width), dtype=torch.int32, device=d)
        self.rgba = torch.empty((self.capacity, self.height, self.width, 4), dtype=torch.float32, device=d)
        self.depth = torch.empty((self.capacity, self.height, self.width), dtype=torch.float32, device=d)
        self.ids = torch.empty((self.capacity, self.height, self.width), dtype=torch.int32, device=d)
        h = C.c_void_p()
        check(lib.dpr_deep_frame_wrap(dev.h, self.width, self.height, self.capacity,
                                      C.c_void_p(self.counts.data_ptr()), C.c_void_p(self.rgba.data_ptr()),
                                      C.c_void_p(self.depth.data_ptr()), C.c_void_p(self.ids.data_ptr()),
                                      C.byref(h)))
        self.h = h
        _live.add(self)

    def release(self):
        if self.h:
            lib.dpr_deep_frame_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def composite_deep(dev: Device, parts, out: Frame):
    """Merge deep frames of distinct ranks per pixel and composite into ``out``."""
    k = len(parts)
    fr = (C.c_void_p * k)(*[f.h.value for f in parts])
    check(lib.dpr_composite_deep(dev.h, fr, k, out.h))


def _as_bytes_ptr(arr, dev):
    """Host numpy array or device torch tensor -> (pointer, on_device, dtype code, keepalive)."""
    torch = _torch()
    if isinstance(arr, torch.Tensor):
        assert arr.is_contiguous()
        code = {torch.float32: F32, torch.float16: F16}[arr.dtype]
        on_dev = arr.is_cuda
        return C.c_void_p(arr.data_ptr()), int(on_dev), code, arr
    a = np.ascontiguousarray(arr)
    code = {np.dtype(np.float32): F32, np.dtype(np.float16): F16}[a.dtype]
    return C.c_void_p(a.ctypes.data), 0, code, a


class World:
    """This rank's bricks, transfer function and camera (section 3.1 of the paper)."""

    def __init__(self, dev: Device, dims):
        self.dev = dev
        self.dims = tuple(int(v) for v in dims)
        h = C.c_void_p()
        check(lib.dpr_world_create(dev.h, N.I64x3(*self.dims), C.byref(h)))
        self.h = h
        _live.add(self)
        self.params = Params()

    def add_brick(self, voxels, lo, hi, ghost_lo=(0, 0, 0), ghost_hi=(0, 0, 0)):
        ptr, on_dev, code, keep = _as_bytes_ptr(voxels, self.dev)
        bid = C.c_int32()
        check(lib.dpr_world_add_brick(self.h, ptr, code, on_dev, N.I64x3(*lo), N.I64x3(*hi), N.I32x3(*ghost_lo),
                                      N.I32x3(*ghost_hi), C.byref(bid)))
        del keep
        return bid.value

    def commit(self):
        check(lib.dpr_world_commit(self.h))

    def release_linear(self):
        """Free the bricks' linear copies of a committed world (see dpr_world_release_linear)."""
        check(lib.dpr_world_release_linear(self.h))

    def set_transfer_function(self, tf, lo=0.0, hi=1.0, density=20.0):
        t = np.ascontiguousarray(tf, dtype=np.float32)
        check(lib.dpr_set_transfer_function(self.h, C.c_void_p(t.ctypes.data), t.shape[0], lo, hi, density))

    def set_isosurface(self, value=None, ambient=0.25, diffuse=0.75):
        """Opaque iso-surface at ``value`` (None: off), lit by a headlight."""
        if value is None:
            check(lib.dpr_set_isosurface(self.h, 0, 0.0, 0.0, 0.0))
        else:
            check(lib.dpr_set_isosurface(self.h, 1, float(value), float(ambient), float(diffuse)))

    def set_camera(self, cam):
        c = to_c_camera(cam)
        check(lib.dpr_set_camera(self.h, C.byref(c)))

    def set_params(self, params: Params):
        self.params = params
        c = params.c()
        check(lib.dpr_set_render_params(self.h, C.byref(c)))

    def brick_count(self):
        n = C.c_int32()
        check(lib.dpr_world_brick_count(self.h, C.byref(n)))
        return n.value

    def macrocells(self, brick_id):
        md = N.I32x3()
        check(lib.dpr_world_brick_macrocells(self.h, brick_id, md, None, None, 0))
        cnt = md[0] * md[1] * md[2]
        ranges = np.empty((md[2], md[1], md[0], 2), dtype=np.float32)
        maj = np.empty((md[2], md[1], md[0]), dtype=np.float32)
        check(lib.dpr_world_brick_macrocells(self.h, brick_id, md, C.c_void_p(ranges.ctypes.data),
                                             C.c_void_p(maj.ctypes.data), cnt))
        return ranges, maj

    def blocked_copy(self, brick_id):
        """(raw bytes of a brick's 8^3-blocked copy as uint8, blocks per axis, element bytes); see dpr_world_brick_blocked."""
        bd = N.I32x3()
        eb = C.c_int32()
        check(lib.dpr_world_brick_blocked(self.h, int(brick_id), bd, C.byref(eb), None, 0))
        n = bd[0] * bd[1] * bd[2] * 512 * eb.value
        buf = np.empty(n, dtype=np.uint8)
        check(lib.dpr_world_brick_blocked(self.h, int(brick_id), bd, C.byref(eb), C.c_void_p(buf.ctypes.data), n))
        return buf, (bd[0], bd[1], bd[2]), eb.value

    def render_partial(self, brick_id, frame: Frame):
        check(lib.dpr_render_partial(self.h, brick_id, frame.h))

    def render_frame(self, frame: Frame):
        check(lib.dpr_render_frame(self.h, frame.h))

    def measure_gather(self, brick_id, counts, sink):
        """Gather-ceiling probe: the march's loads for the first counts[p] logical
        samples of every pixel (device int32 / float tensors of the camera's size)."""
        check(lib.dpr_measure_gather(self.h, int(brick_id), C.c_void_p(counts.data_ptr()),
                                     C.c_void_p(sink.data_ptr())))

    def render_deep(self, rank, deep: "DeepFrame"):
        """Every brick of this world into ``deep`` (fragment ids rank * 65536 + brick)."""
        check(lib.dpr_render_deep(self.h, int(rank), deep.h))

    def render_path(self, frame: Frame, light_dir=(-0.45, -0.55, -0.7), light_rgb=(3.0, 2.8, 2.5),
                    env_rgb=(0.15, 0.2, 0.3), max_bounces=3, spp=1, seed=1):
        """Path-traced image of the world's camera into ``frame`` (RGB radiance, A = 1);
        returns the tracer's counters."""
        prm = N.PathParams((C.c_float * 3)(*light_dir), (C.c_float * 3)(*light_rgb), (C.c_float * 3)(*env_rgb),
                           int(max_bounces), int(spp), int(seed) & 0xFFFFFFFF)
        st = N.PathStats()
        check(lib.dpr_render_path(self.h, C.byref(prm), frame.h, C.byref(st)))
        return dict(paths=st.paths, events=st.events, shadow_steps=st.shadow_steps, forwards=st.forwards,
                    waves=st.waves)

    def render_batch(self, cams, frames, flags=0):
        arr = (N.Camera * len(cams))(*[to_c_camera(c) for c in cams])
        fr = (C.c_void_p * len(frames))(*[f.h.value for f in frames])
        check(lib.dpr_render_batch(self.h, arr, len(cams), fr, flags))

    def autotune_batch(self, cams, frames):
        arr = (N.Camera * len(cams))(*[to_c_camera(c) for c in cams])
        fr = (C.c_void_p * len(frames))(*[f.h.value for f in frames])
        tw, th = C.c_int32(), C.c_int32()
        check(lib.dpr_autotune_batch(self.h, arr, len(cams), fr, C.byref(tw), C.byref(th)))
        return tw.value, th.value

    def set_batch_tile(self, tw, th):
        check(lib.dpr_set_batch_tile(self.h, tw, th))

    def batch_coverage(self):
        """(items, items taken once, fragment slots, slots written once) of the last
        batched render, which must have run with FLAG_QUEUE_COVERAGE."""
        out = (C.c_int64 * 4)()
        check(lib.dpr_batch_coverage(self.h, out))
        return tuple(out)

    def batch_timings(self):
        """(march_ms, composite_ms) of the last batched render, from HIP events."""
        a, c = C.c_float(), C.c_float()
        check(lib.dpr_batch_timings(self.h, C.byref(a), C.byref(c)))
        return a.value, c.value

    def release(self):
        if self.h:
            lib.dpr_world_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def composite(dev: Device, parts, out: Frame, ids=None):
    """Sort-last composite of ``parts`` (Frames) into ``out``; ids are intrinsic fragment ids."""
    k = len(parts)
    fr = (C.c_void_p * k)(*[f.h.value for f in parts])
    idarr = None if ids is None else (C.c_int32 * k)(*[int(i) for i in ids])
    check(lib.dpr_composite(dev.h, fr, idarr, k, out.h))


def composite_noalloc(dev: Device, parts, out: Frame, ids=None):
    """``composite`` through the entry point that allocates nothing (its scratch is
    the library's fixed per-GPU array; frames up to 8,388,608 pixels)."""
    k = len(parts)
    fr = (C.c_void_p * k)(*[f.h.value for f in parts])
    idarr = None if ids is None else (C.c_int32 * k)(*[int(i) for i in ids])
    check(lib.dpr_composite_noalloc(dev.h, fr, idarr, k, out.h))


# ---------------------------------------------------------------- differentiable render
def _follow_current_stream(dev, device):
    """Point the library's device at torch's current stream (where the call's
    buffers were just allocated and filled) and return that stream."""
    torch = _torch()
    stream = torch.cuda.current_stream(device)
    if dev.stream is None or dev.stream.cuda_stream != stream.cuda_stream:
        dev.set_stream(stream)
    return stream


def _cam_array(cams):
    return (N.Camera * len(cams))(*[to_c_camera(c) for c in cams])


def _train_args(volume, tf):
    torch = _torch()
    assert volume.is_cuda and volume.dtype == torch.float32 and volume.is_contiguous()
    assert tf.is_cuda and tf.dtype == torch.float32 and tf.is_contiguous() and tf.shape[-1] == 4
    nz, ny, nx = volume.shape
    return N.I64x3(nx, ny, nz)


def _make_fn():
    torch = _torch()

    class DprRenderFn(torch.autograd.Function):
        """Differentiable render of a whole FP32 volume with a TF table (ERT off, no skipping).

        forward(volume (nz,ny,nx), tf (N,4), dev, cams, params, lo, hi, density) -> images (n,H,W,4).
        backward runs the hand-written adjoint ray march (dpr_render_backward).
        """

        @staticmethod
        def forward(ctx, volume, tf, dev, cams, params, lo, hi, density):
            dims = _train_args(volume, tf)
            # the library enqueues on the stream torch allocates and zero-fills on
            _follow_current_stream(dev, volume.device)
            ca = _cam_array(cams)
            n, W, H = len(cams), int(cams[0].width), int(cams[0].height)
            nbytes = C.c_size_t()
            check(lib.dpr_train_workspace_size(dims, ca, n, float(params.step_voxels), C.byref(nbytes)))
            ws = torch.empty(nbytes.value, dtype=torch.uint8, device=volume.device)
            out = torch.empty((n, H, W, 4), dtype=torch.float32, device=volume.device)
            depth = torch.empty((n, H, W), dtype=torch.float32, device=volume.device)
            cp = params.c()
            check(lib.dpr_render_train_forward(dev.h, C.c_void_p(volume.data_ptr()), dims, C.c_void_p(tf.data_ptr()),
                                               tf.shape[0], lo, hi, density, C.byref(cp), ca, n,
                                               C.c_void_p(out.data_ptr()), C.c_void_p(depth.data_ptr()),
                                               C.c_void_p(ws.data_ptr()), nbytes.value))
            ctx.save_for_backward(volume, tf)
            ctx.ws, ctx.dev, ctx.cams, ctx.params, ctx.rng = ws, dev, cams, params, (lo, hi, density)
            ctx.mark_non_differentiable(depth)
            return out, depth

        @staticmethod
        def backward(ctx, g_out, g_depth):
            volume, tf = ctx.saved_tensors
            dims = _train_args(volume, tf)
            stream = _follow_current_stream(ctx.dev, volume.device)
            # the forward's workspace is read here, possibly on another stream
            ctx.ws.record_stream(stream)
            ca = _cam_array(ctx.cams)
            g = g_out.contiguous()
            gv = torch.zeros_like(volume)
            gt = torch.zeros_like(tf)
            lo, hi, density = ctx.rng
            cp = ctx.params.c()
            check(lib.dpr_render_backward(ctx.dev.h, C.c_void_p(volume.data_ptr()), dims, C.c_void_p(tf.data_ptr()),
                                          tf.shape[0], lo, hi, density, C.byref(cp), ca, len(ctx.cams),
                                          C.c_void_p(g.data_ptr()), C.c_void_p(ctx.ws.data_ptr()), ctx.ws.numel(),
                                          C.c_void_p(gv.data_ptr()), C.c_void_p(gt.data_ptr())))
            return gv, gt, None, None, None, None, None, None

    return DprRenderFn


_FN = None


def render_train(dev, volume, tf, cams, params=None, lo=0.0, hi=1.0, density=20.0):
    """Images (n, H, W, 4) of ``volume`` seen by ``cams``, differentiable in volume and tf."""
    global _FN
    if _FN is None:
        _FN = _make_fn()
    params = params or Params(0.5, 1.0, 16, 0)
    out, _ = _FN.apply(volume, tf, dev, cams, params, lo, hi, density)
    return out


def __getattr__(name):
    if name == "DprRenderFn":
        global _FN
        if _FN is None:
            _FN = _make_fn()
        return _FN
    raise AttributeError(name)
