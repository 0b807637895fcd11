"""Allocation failures: with DPR_FAULT_INJECT=alloc:N the N-th device or pinned
host allocation of the process fails.  Injected at every allocation a small but
complete scenario makes (world, commit, transfer function, batched frame, plain
partials through the persistent kernel, sort-last composite), each failure must
surface as DPR_ERR_OUT_OF_MEMORY and leave no allocation behind once the objects
are released, and the library must render the same bits afterwards."""

import os

import numpy as np
import pytest

from synth import even_split, make_blobs, make_tf, make_volume_small, orbit_camera
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpr():
    import paper_2407_00179_amd as m
    return m


def _stats(dpr):
    import ctypes as C
    a, live = C.c_int64(), C.c_int64()
    dpr.check(dpr.lib.dpr_alloc_stats(C.byref(a), C.byref(live)))
    return a.value, live.value


def _scenario(dpr, vol, dims, boxes, tf, cam):
    import torch
    objs = []
    try:
        dev = dpr.Device(0)
        objs.append(dev)
        w = dpr.World(dev, dims)
        objs.append(w)
        w.set_params(dpr.Params(0.5, 0.99, 8, 0))
        v = torch.tensor(vol, device=dev.torch_device)
        for lo, hi in boxes:
            glo = tuple(1 if lo[a] > 0 else 0 for a in range(3))
            ghi = tuple(1 if hi[a] < dims[a] else 0 for a in range(3))
            sl = tuple(slice(lo[a] - glo[a], hi[a] + ghi[a]) for a in (2, 1, 0))
            w.add_brick(v[sl].contiguous(), lo, hi, glo, ghi)
        w.commit()
        w.set_transfer_function(tf, 0.0, 1.0, 20.0)
        w.set_camera(cam)
        frame = dpr.Frame(dev, cam.width, cam.height)
        objs.append(frame)
        w.render_frame(frame)
        parts = []
        for i in range(len(boxes)):
            parts.append(dpr.Frame(dev, cam.width, cam.height))
            objs.append(parts[-1])
            w.render_partial(i, parts[-1])
        out = dpr.Frame(dev, cam.width, cam.height)
        objs.append(out)
        dpr.composite(dev, parts, out, ids=list(range(len(parts))))
        dev.sync()
        return frame.rgba.cpu().numpy(), out.rgba.cpu().numpy()
    finally:
        for o in reversed(objs):
            o.release()


def test_injected_allocation_failures_report_oom_and_leak_nothing(gpu_lib, dpr):
    dims = (40, 36, 30)
    vol = make_volume_small(dims, make_blobs(dims, 31, 6, (0.1, 0.25)), 32, 0.02)
    tf = make_tf(2001)
    cam = orbit_camera(dims, 48, 40)
    boxes = even_split(dims, (2, 1, 2))
    os.environ.pop("DPR_FAULT_INJECT", None)
    want = _scenario(dpr, vol, dims, boxes, tf, cam)   # warm: the process's own one-time set-up
    t0, live0 = _stats(dpr)
    again = _scenario(dpr, vol, dims, boxes, tf, cam)
    t1, live1 = _stats(dpr)
    n = t1 - t0
    log(f"  scenario: {n} allocations, {live0} live before and {live1} after")
    assert live1 == live0 and n >= 10
    assert all(np.array_equal(a, b) for a, b in zip(want, again))
    failed = 0
    try:
        for k in range(1, n + 1):
            total, _ = _stats(dpr)
            os.environ["DPR_FAULT_INJECT"] = f"alloc:{total + k}"
            try:
                got = _scenario(dpr, vol, dims, boxes, tf, cam)
            except dpr.DprError as e:
                assert e.status == -3, f"allocation {k}: {e}"   # DPR_ERR_OUT_OF_MEMORY
                failed += 1
            else:
                # the failed allocation was one the library can do without
                assert all(np.array_equal(a, b) for a, b in zip(want, got)), f"allocation {k}"
            os.environ.pop("DPR_FAULT_INJECT", None)
            _, live = _stats(dpr)
            assert live == live0, f"allocation {k} failing leaves {live - live0} allocations behind"
    finally:
        os.environ.pop("DPR_FAULT_INJECT", None)
    log(f"  {failed} of {n} injected failures reported DPR_ERR_OUT_OF_MEMORY")
    assert failed >= n // 2
    after = _scenario(dpr, vol, dims, boxes, tf, cam)
    assert all(np.array_equal(a, b) for a, b in zip(want, after))
    assert _stats(dpr)[1] == live0
