"""The C ABI from a plain C program.  tests/native/abi_client.c is compiled as
strict C99 (-pedantic -Werror) against include/dpr.h and linked against the
in-tree library; its process holds no Python and no PyTorch.  On the CPU it
exercises the host-side calls; on a GPU it renders a split volume through
dpr_world_add_brick (host buffers), dpr_world_commit, dpr_set_transfer_function,
dpr_set_camera, dpr_render_partial, dpr_composite and dpr_render_frame, and the
frames it writes are compared with the oracle here."""

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "abi_client.c")
LIB_DIR = os.path.join(ROOT, "paper_2407_00179_amd")


def _build(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    if not os.path.exists(os.path.join(LIB_DIR, "libdpr.so")):
        pytest.fail("libdpr.so is not built")
    exe = str(tmp_path / "abi_client")
    cmd = [cc, "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-O1", "-I", os.path.join(ROOT, "include"),
           SRC, "-L", LIB_DIR, "-ldpr", f"-Wl,-rpath,{LIB_DIR}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    return exe


def _env():
    # the program must find the in-tree library by its run path, nothing else
    return {k: v for k, v in os.environ.items() if k != "DPR_LIBRARY"}


def test_c_client_host_calls(tmp_path):
    exe = _build(tmp_path)
    r = subprocess.run([exe, "check"], capture_output=True, text=True, timeout=300, env=_env())
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr
    assert "gfx950" in r.stdout


def _read_frame(path, w, h):
    a = np.fromfile(path, dtype=np.float32)
    assert a.size == w * h * 5, path
    return a[:w * h * 4].reshape(-1, 4).astype(np.float64), a[w * h * 4:].astype(np.float64)


@pytest.mark.gpu
@pytest.mark.parametrize("dtype,flags", [("f32", 0), ("f16", 0), ("f16", 0x10)])
def test_c_client_renders_like_the_oracle(tmp_path, gpu_lib, dtype, flags):
    """FP32 bricks, FP16 bricks as voxel pairs, and FP16 bricks in the 2-byte
    layout (DPR_FLAG_F16_HALVES), all from host buffers of a C program."""
    import oracle
    from synth import even_split, extract_brick, make_blobs, make_tf, make_volume_small, orbit_camera
    from tests.gpu_util import TOL_F16, TOL_F32, log, oracle_brick

    dims = (40, 36, 30)
    vol = make_volume_small(dims, make_blobs(dims, 41, 6, (0.08, 0.25)), 42, 0.02)
    np_dtype = np.float16 if dtype == "f16" else np.float32
    vol = vol.astype(np_dtype)
    tol = TOL_F16 if dtype == "f16" else TOL_F32
    tf = make_tf(2001)
    cam = orbit_camera(dims, 48, 40)
    boxes = even_split(dims, (2, 1, 2))
    prm = oracle.RenderParams(0.5, 1.0, 20.0)  # ERT off: plain parity, no bracket
    lines = [f"dims {dims[0]} {dims[1]} {dims[2]}",
             "camera " + " ".join(repr(float(v)) for v in (*cam.eye, *cam.center, *cam.up, cam.fovy_deg))
             + f" {cam.width} {cam.height}",
             f"params {prm.step_voxels} {prm.ert} 8 {flags}",
             f"tf {len(tf)} {prm.tf_lo} {prm.tf_hi} {prm.density}",
             f"dtype {dtype}",
             f"bricks {len(boxes)}"]
    for i, (lo, hi) in enumerate(boxes):
        b = extract_brick(vol, dims, lo, hi)
        np.ascontiguousarray(b.data, dtype=np_dtype).tofile(str(tmp_path / f"brick{i}.{dtype}"))
        lines.append(" ".join(str(int(v)) for v in (*lo, *hi, *b.ghost_lo, *b.ghost_hi)))
    np.ascontiguousarray(tf, dtype=np.float32).tofile(str(tmp_path / "tf.f32"))
    (tmp_path / "scene.txt").write_text("\n".join(lines) + "\n")

    exe = _build(tmp_path)
    log(f"C client: {len(boxes)} {dtype} bricks of {dims} (flags {flags:#x}) at {cam.width}x{cam.height}")
    r = subprocess.run([exe, "render", str(tmp_path)], capture_output=True, text=True, timeout=300, env=_env())
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr

    W, H = cam.width, cam.height
    py, px = np.mgrid[0:H, 0:W]
    px, py = px.ravel(), py.ravel()
    parts, zs = [], []
    for i, (lo, hi) in enumerate(boxes):
        got, gz = _read_frame(str(tmp_path / f"partial{i}.f32"), W, H)
        want, wz, _ = oracle_brick(vol, dims, lo, hi, tf, prm, cam, px, py)
        err = np.max(np.abs(got - want))
        assert err <= tol, f"brick {i}: {err:.3e}"
        fin = np.isfinite(wz)
        assert np.array_equal(np.isfinite(gz), fin)
        assert np.max(np.abs(gz[fin] - wz[fin]) / wz[fin], initial=0.0) <= 3e-7
        parts.append(want)
        zs.append(wz)
    want_c, want_z = oracle.composite(np.stack(parts), np.stack(zs), np.arange(len(boxes)))
    comp, cz = _read_frame(str(tmp_path / "composite.f32"), W, H)
    whole, fz = _read_frame(str(tmp_path / "frame.f32"), W, H)
    err = np.max(np.abs(comp - want_c))
    log(f"  composite max|c-oracle| = {err:.3e}")
    assert err <= tol
    assert np.array_equal(np.isfinite(cz), np.isfinite(want_z))
    # the batched whole-frame render gives the same bits as partials + composite
    assert np.array_equal(whole, comp) and np.array_equal(fz, cz)
