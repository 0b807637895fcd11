"""The autotuner's tile-shape cache (host only, no GPU): round trips, several keys,
replacement, and files that are missing or unreadable."""

import ctypes as C
import json

import pytest


@pytest.fixture(scope="module")
def N():
    from paper_2407_00179_amd import _native
    return _native


def _lookup(N, path, key):
    found, w, h = C.c_int32(-1), C.c_int32(0), C.c_int32(0)
    assert N.lib.dpr_tune_cache_lookup(str(path).encode(), key.encode(), C.byref(found), C.byref(w), C.byref(h)) == 0
    return (w.value, h.value) if found.value else None


def test_round_trip_and_replacement(N, tmp_path):
    path = tmp_path / "tiles.json"
    assert _lookup(N, path, "gfx950 cu256 f32 bricks 257x257x257") is None      # no file yet
    assert N.lib.dpr_tune_cache_store(str(path).encode(), b"gfx950 cu256 f32 bricks 257x257x257", 8, 8) == 0
    assert N.lib.dpr_tune_cache_store(str(path).encode(), b"gfx950 cu256 f16-2byte cameras 3840x2160", 16, 8) == 0
    assert _lookup(N, path, "gfx950 cu256 f32 bricks 257x257x257") == (8, 8)
    assert _lookup(N, path, "gfx950 cu256 f16-2byte cameras 3840x2160") == (16, 8)
    assert _lookup(N, path, "gfx950 cu256 f32") is None
    assert N.lib.dpr_tune_cache_store(str(path).encode(), b"gfx950 cu256 f32 bricks 257x257x257", 32, 16) == 0
    assert _lookup(N, path, "gfx950 cu256 f32 bricks 257x257x257") == (32, 16)
    doc = json.loads(path.read_text())    # the file is plain JSON
    assert doc["version"] == 1 and doc["entries"] == {"gfx950 cu256 f32 bricks 257x257x257": [32, 16],
                                                       "gfx950 cu256 f16-2byte cameras 3840x2160": [16, 8]}
    assert not list(tmp_path.glob("*.tmp*"))


def test_unreadable_file_is_replaced(N, tmp_path):
    path = tmp_path / "tiles.json"
    path.write_text('{"version": 1, "entries": {"a": [8, ')
    assert _lookup(N, path, "a") is None
    assert N.lib.dpr_tune_cache_store(str(path).encode(), b"b", 16, 16) == 0
    assert json.loads(path.read_text())["entries"] == {"b": [16, 16]}


def test_bad_keys_are_invalid_arguments(N, tmp_path):
    path = str(tmp_path / "tiles.json").encode()
    f, w, h = C.c_int32(), C.c_int32(), C.c_int32()
    assert N.lib.dpr_tune_cache_store(path, b'a"b', 8, 8) == -1
    assert N.lib.dpr_tune_cache_store(path, b"a\\b", 8, 8) == -1
    assert N.lib.dpr_tune_cache_store(path, b"", 8, 8) == -1
    assert N.lib.dpr_tune_cache_lookup(path, b'"', C.byref(f), C.byref(w), C.byref(h)) == -1
    assert N.lib.dpr_tune_cache_lookup(None, b"a", C.byref(f), C.byref(w), C.byref(h)) == -1
