"""Pins of the composite oracle and of the data-parallel split invariant (FP64)."""

import math

import numpy as np
import pytest

import oracle
from oracle import RenderParams
from oracle import brute
from synth import extract_brick, even_split, kd_split, orbit_camera
from tests.helpers import random_volume, rand_tf


def _rand_frags(K, P, seed, empty_frac=0.3, ties=False):
    rng = np.random.default_rng(seed)
    a = rng.random((K, P))
    rgba = np.concatenate([rng.random((K, P, 3)) * a[..., None], a[..., None]], axis=-1)
    depth = rng.random((K, P)) * 10 + 0.1
    if ties:
        depth = np.round(depth)
    empty = rng.random((K, P)) < empty_frac
    rgba[empty] = 0.0
    depth[empty] = np.inf
    return rgba, depth


def test_single_fragment_is_identity_bitwise():
    rgba, depth = _rand_frags(1, 500, 1)
    out, z = oracle.composite(rgba, depth)
    assert np.array_equal(out, rgba[0]) and np.array_equal(z, depth[0])


def test_empty_fragments_are_identities():
    rgba, depth = _rand_frags(3, 400, 2)
    e_rgba = np.zeros((4, 400, 4))
    e_depth = np.full((4, 400), np.inf)
    out, z = oracle.composite(rgba, depth)
    out2, z2 = oracle.composite(np.concatenate([e_rgba[:2], rgba, e_rgba[2:]]),
                                np.concatenate([e_depth[:2], depth, e_depth[2:]]),
                                ids=[10, 11, 0, 1, 2, 12, 13])
    assert np.array_equal(out, out2) and np.array_equal(z, z2)
    all_empty, ze = oracle.composite(e_rgba, e_depth)
    assert np.all(all_empty == 0.0) and np.all(np.isinf(ze))


def test_two_fragments_closed_form_and_order():
    rgba, depth = _rand_frags(2, 300, 3, empty_frac=0.0)
    out, z = oracle.composite(rgba, depth)
    near = np.where(depth[0] <= depth[1], 0, 1)
    far = 1 - near
    cols = np.arange(300)
    n, f = rgba[near, cols], rgba[far, cols]
    assert np.allclose(out[:, :3], n[:, :3] + (1 - n[:, 3:4]) * f[:, :3], atol=1e-15)
    assert np.allclose(out[:, 3], 1 - (1 - n[:, 3]) * (1 - f[:, 3]), atol=1e-15)
    assert np.array_equal(z, np.minimum(depth[0], depth[1]))


def test_opaque_nearest_wins_exactly():
    rgba, depth = _rand_frags(5, 300, 4, empty_frac=0.0)
    k = np.argmin(depth, axis=0)
    cols = np.arange(300)
    rgba[k, cols, 3] = 1.0
    out, _ = oracle.composite(rgba, depth)
    assert np.array_equal(out, rgba[k, cols])


def test_permutation_invariance_bitwise():
    K = 9
    rgba, depth = _rand_frags(K, 1000, 5)
    ids = np.arange(K)
    out, z = oracle.composite(rgba, depth, ids)
    for s in range(4):
        perm = np.random.default_rng(s).permutation(K)
        o2, z2 = oracle.composite(rgba[perm], depth[perm], ids[perm])
        assert np.array_equal(out, o2) and np.array_equal(z, z2)


def test_ties_broken_by_intrinsic_id():
    K = 6
    rgba, depth = _rand_frags(K, 800, 6, ties=True)
    ids = np.arange(K) * 3 + 1
    out, _ = oracle.composite(rgba, depth, ids)
    perm = np.random.default_rng(9).permutation(K)
    o2, _ = oracle.composite(rgba[perm], depth[perm], ids[perm])
    assert np.array_equal(out, o2)
    for p in range(0, 800, 37):
        frags = [(rgba[k, p], depth[k, p], ids[k]) for k in range(K)]
        b = brute.composite_pixel(frags)
        assert np.allclose(out[p], b[:4], atol=1e-15)


def test_associativity():
    K = 8
    rgba, depth = _rand_frags(K, 600, 7)
    order = np.argsort(depth, axis=0, kind="stable")
    out, _ = oracle.composite(rgba, depth)
    # split each pixel's sorted list into a front half and a back half, composite each, then over
    P = depth.shape[1]
    cols = np.arange(P)
    front = order[: K // 2]
    back = order[K // 2:]
    fr, fz = oracle.composite(rgba[front, cols], depth[front, cols])
    br, bz = oracle.composite(rgba[back, cols], depth[back, cols])
    over_rgb = fr[:, :3] + (1 - fr[:, 3:4]) * br[:, :3]
    over_a = 1 - (1 - fr[:, 3]) * (1 - br[:, 3])
    assert np.allclose(out[:, :3], over_rgb, atol=1e-14)
    assert np.allclose(out[:, 3], over_a, atol=1e-14)


def test_brute_composite_matches():
    K = 7
    rgba, depth = _rand_frags(K, 200, 8)
    ids = np.random.default_rng(1).permutation(K)
    out, z = oracle.composite(rgba, depth, ids)
    for p in range(200):
        b = brute.composite_pixel([(rgba[k, p], depth[k, p], ids[k]) for k in range(K)])
        assert np.allclose(out[p], b[:4], atol=1e-15) and z[p] == b[4]


# ----------------------------------------------------------------- split invariant (P-c6)
def _split_render(vol, dims, boxes, tf, prm, cam, shuffle_seed=None):
    parts_rgba, parts_z = [], []
    for lo, hi in boxes:
        b = extract_brick(vol, dims, lo, hi, ghost=1)
        r, z, _ = oracle.render_brick(b.data, b.stored_lo, dims, lo, hi, tf, prm, cam)
        parts_rgba.append(r)
        parts_z.append(z)
    ids = np.arange(len(boxes))
    if shuffle_seed is not None:
        perm = np.random.default_rng(shuffle_seed).permutation(len(boxes))
        parts_rgba = [parts_rgba[i] for i in perm]
        parts_z = [parts_z[i] for i in perm]
        ids = ids[perm]
    return oracle.composite(np.stack(parts_rgba), np.stack(parts_z), ids)


@pytest.mark.parametrize("split", ["2x2x2", "kd5", "3x3x3", "1x2x3"])
def test_split_invariant_exact_without_ert(split):
    dims = (12, 10, 14)
    vol = random_volume(dims, 21)
    tf = rand_tf(31)
    prm = RenderParams(step_voxels=0.5, ert=1.0, density=30.0)
    cam = orbit_camera(dims, 12, 10)
    full, zf, _ = oracle.render_image(vol, dims, tf, prm, cam)
    if split == "kd5":
        boxes = kd_split(dims, 5, seed=3, max_ratio=8.0)
    else:
        boxes = even_split(dims, tuple(int(c) for c in split.split("x")))
    comp, zc = _split_render(vol, dims, boxes, tf, prm, cam, shuffle_seed=1)
    assert full[..., 3].max() > 0.2
    assert np.max(np.abs(comp - full)) <= 1e-12
    assert np.allclose(zc, zf, atol=1e-13, rtol=0) and np.array_equal(np.isinf(zc), np.isinf(zf))


@pytest.mark.parametrize("step", [0.5, 1.0, 0.3])
def test_split_invariant_other_steps(step):
    dims = (9, 9, 9)
    vol = random_volume(dims, 22)
    tf = rand_tf(32)
    prm = RenderParams(step_voxels=step, ert=1.0, density=25.0)
    cam = orbit_camera(dims, 9, 9)
    full, _, _ = oracle.render_image(vol, dims, tf, prm, cam)
    comp, _ = _split_render(vol, dims, even_split(dims, (2, 3, 2)), tf, prm, cam)
    assert np.max(np.abs(comp - full)) <= 1e-12


def test_split_with_ert_within_bound():
    """Per-brick ERT: |unsplit - composite| <= 2 (1 - theta) per channel."""
    dims = (12, 12, 12)
    vol = random_volume(dims, 23)
    tf = rand_tf(33)
    theta = 0.9
    prm = RenderParams(step_voxels=0.5, ert=theta, density=80.0)
    cam = orbit_camera(dims, 12, 12)
    full, _, ns = oracle.render_image(vol, dims, tf, prm, cam)
    comp, _ = _split_render(vol, dims, even_split(dims, (2, 2, 2)), tf, prm, cam)
    noert, _, ns_off = oracle.render_image(vol, dims, tf, RenderParams(0.5, 1.0, 80.0), cam)
    assert np.any(ns < ns_off)                      # ERT actually fired somewhere
    assert np.max(np.abs(comp - full)) <= 2 * (1 - theta) + 1e-12
    assert np.all(noert - full >= -1e-12) and np.all(noert - full <= (1 - theta) + 1e-12)


def test_interleaved_nonconvex_partition_breaks_single_fragment_compositing():
    """4^3 sub-boxes dealt to 4 pseudo-ranks: each rank's set is non-convex, so one
    fragment per pixel per rank cannot composite to the unsplit image (paper Fig. 6
    setup; section 2.1 on convex partitions)."""
    dims = (16, 16, 16)
    vol = random_volume(dims, 24)
    tf = rand_tf(34)
    prm = RenderParams(step_voxels=0.5, ert=1.0, density=30.0)
    cam = orbit_camera(dims, 12, 12)
    full, _, _ = oracle.render_image(vol, dims, tf, prm, cam)
    boxes = even_split(dims, (4, 4, 4))
    owner = np.random.default_rng(5).integers(0, 4, size=len(boxes))
    rank_rgba, rank_z = [], []
    for r in range(4):
        # each rank renders its own boxes and merges them locally front to back
        # into ONE fragment with the nearest entry depth (what a single-fragment rank emits)
        mine = [boxes[i] for i in range(len(boxes)) if owner[i] == r]
        rr, zz = _split_render(vol, dims, mine, tf, prm, cam)
        rank_rgba.append(rr)
        rank_z.append(zz)
    comp, _ = oracle.composite(np.stack(rank_rgba), np.stack(rank_z))
    assert np.max(np.abs(comp - full)) > 1e-3
