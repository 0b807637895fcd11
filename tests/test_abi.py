"""C-ABI tests that need no GPU: the library loads, exports every declared entry
point, and its host-side validation answers without touching a device."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpr.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dpr_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def N():
    from paper_2407_00179_amd import _native
    return _native


def test_header_declares_the_paper_entry_points():
    names = _declared()
    for n in ("dpr_world_add_brick", "dpr_set_transfer_function", "dpr_set_camera", "dpr_render_partial",
              "dpr_composite", "dpr_render_frame"):
        assert n in names


def test_library_exports_every_declared_symbol(N):
    for name in _declared():
        assert hasattr(N.lib, name), name
    assert set(N.EXPORTED) == set(_declared())


def test_version_and_error_strings(N):
    assert b"gfx950" in N.lib.dpr_version()
    assert isinstance(N.lib.dpr_last_error(), bytes)


def test_allocation_counters_answer_without_gpu(N):
    a, live = C.c_int64(-1), C.c_int64(-1)
    assert N.lib.dpr_alloc_stats(C.byref(a), C.byref(live)) == 0
    assert a.value >= 0 and 0 <= live.value <= a.value
    assert N.lib.dpr_alloc_stats(None, None) == 0


def test_device_create_without_gpu_reports_device_error(N):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = C.c_void_p()
    st = N.lib.dpr_device_create(0, None, C.byref(h))
    assert st == -4  # DPR_ERR_DEVICE
    assert b"device" in N.lib.dpr_last_error()
    assert not h.value


def test_null_handles_are_invalid_arguments(N):
    assert N.lib.dpr_device_create(0, None, None) == -1
    assert N.lib.dpr_world_create(None, N.I64x3(4, 4, 4), C.byref(C.c_void_p())) == -1
    assert N.lib.dpr_world_commit(None) == -1
    assert N.lib.dpr_render_partial(None, 0, None) == -1
    assert N.lib.dpr_render_frame(None, None) == -1
    assert N.lib.dpr_composite(None, None, None, 1, None) == -1
    assert N.lib.dpr_device_sync(None) == -1
    assert N.lib.dpr_frame_map(None, None, None) == -1
    assert N.lib.dpr_set_camera(None, None) == -1
    assert N.lib.dpr_render_deep(None, 0, None) == -1
    assert N.lib.dpr_render_path(None, None, None, None) == -1
    assert N.lib.dpr_set_isosurface(None, 1, 0.5, 0.2, 0.8) == -1
    assert N.lib.dpr_composite_deep(None, None, 1, None) == -1
    assert N.lib.dpr_deep_frame_create(None, 4, 4, 2, C.byref(C.c_void_p())) == -1
    assert N.lib.dpr_deep_frame_wrap(None, 4, 4, 2, None, None, None, None, C.byref(C.c_void_p())) == -1
    N.lib.dpr_deep_frame_release(None)
    N.lib.dpr_world_release(None)
    N.lib.dpr_frame_release(None)
    N.lib.dpr_device_release(None)


def _part(N, dims, boxes, ghosts):
    n = len(boxes)
    lo = (C.c_int64 * (3 * n))(*[v for b in boxes for v in b[0]])
    hi = (C.c_int64 * (3 * n))(*[v for b in boxes for v in b[1]])
    glo = (C.c_int32 * (3 * n))(*[v for g in ghosts for v in g[0]])
    ghi = (C.c_int32 * (3 * n))(*[v for g in ghosts for v in g[1]])
    return N.lib.dpr_check_partition(N.I64x3(*dims), n, lo, hi, glo, ghi)


def test_partition_validation(N):
    from synth import brick_ghosts, even_split, kd_split
    dims = (32, 24, 16)
    boxes = even_split(dims, (2, 2, 2))
    ghosts = [brick_ghosts(dims, lo, hi) for lo, hi in boxes]
    assert _part(N, dims, boxes, ghosts) == 0
    kd = kd_split(dims, 7, seed=5, max_ratio=8)
    assert _part(N, dims, kd, [brick_ghosts(dims, lo, hi) for lo, hi in kd]) == 0
    # overlapping owned boxes
    bad = list(boxes)
    bad[1] = ((15, 0, 0), (32, 12, 8))
    assert _part(N, dims, bad, ghosts) == -1
    assert b"overlap" in N.lib.dpr_last_error()
    # missing ghost layer on an interior face
    g2 = list(ghosts)
    g2[0] = ((0, 0, 0), (0, 1, 1))
    assert _part(N, dims, boxes, g2) == -1
    assert b"ghost" in N.lib.dpr_last_error()
    # ghost layer reaching outside the domain
    g3 = list(ghosts)
    g3[0] = ((1, 0, 0), (1, 1, 1))
    assert _part(N, dims, boxes, g3) == -1
    # owned box outside the domain / empty box
    assert _part(N, dims, [((0, 0, 0), (33, 24, 16))], [((0, 0, 0), (0, 0, 0))]) == -1
    assert _part(N, dims, [((4, 0, 0), (4, 24, 16))], [((1, 0, 0), (1, 0, 0))]) == -1
    # a gap is allowed unless tiling is required
    gap = boxes[:-1]
    assert _part(N, dims, gap, ghosts[:-1]) == 0
    assert _part(N, dims, [], []) == -2


def test_partition_tiling_requirement(monkeypatch):
    import subprocess
    import sys
    code = ("import ctypes as C, sys; sys.path.insert(0, %r)\n"
            "from paper_2407_00179_amd import _native as N\n"
            "lo=(C.c_int64*3)(0,0,0); hi=(C.c_int64*3)(8,8,4); g=(C.c_int32*3)(0,0,0); gh=(C.c_int32*3)(0,0,1)\n"
            "print(N.lib.dpr_check_partition(N.I64x3(8,8,8),1,lo,hi,g,gh))\n") % ROOT
    env = dict(os.environ, DPR_REQUIRE_TILING="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    assert out.stdout.strip() == "-1"
    env["DPR_REQUIRE_TILING"] = "0"
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    assert out.stdout.strip() == "0"


def test_camera_validation(N):
    from paper_2407_00179_amd import to_c_camera
    from synth import Camera
    good = Camera((2.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, 64, 48)
    assert N.lib.dpr_check_camera(C.byref(to_c_camera(good))) == 0
    for bad in (Camera((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, 64, 48),
                Camera((2.0, 0.0, 0.0), (0.0, 0.0, 0.0), (1.0, 0.0, 0.0), 60.0, 64, 48),
                Camera((2.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 180.0, 64, 48),
                Camera((2.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, 0, 48)):
        assert N.lib.dpr_check_camera(C.byref(to_c_camera(bad))) == -1
    assert N.lib.dpr_check_camera(None) == -1


def test_missing_library_fails_loudly(tmp_path):
    """The package has no CPU fallback: without libdpr.so the import raises."""
    import shutil
    import subprocess
    import sys
    pkg = os.path.join(ROOT, "paper_2407_00179_amd")
    dst = tmp_path / "paper_2407_00179_amd"
    shutil.copytree(pkg, dst, ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__"))
    code = "import sys; sys.path.insert(0, %r); import paper_2407_00179_amd" % str(tmp_path)
    env = {k: v for k, v in os.environ.items() if k != "DPR_LIBRARY"}
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env)
    assert r.returncode != 0 and "libdpr.so" in r.stderr
