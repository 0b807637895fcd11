"""CPU pins of the deep-frame oracle (paper section 5.1.1: possibly several
fragments per pixel; section 2.1 and Fig. 6: interleaved boxes dealt to ranks)."""

import numpy as np

import oracle
from oracle import RenderParams
from synth import even_split, extract_brick, kd_split, orbit_camera
from tests.helpers import rand_tf, random_volume


def _brick_frags(vol, dims, boxes, tf, prm, cam):
    rr, zz = [], []
    for lo, hi in boxes:
        b = extract_brick(vol, dims, lo, hi, ghost=1)
        r, z, _ = oracle.render_brick(b.data, b.stored_lo, dims, lo, hi, tf, prm, cam)
        rr.append(r.reshape(-1, 4))
        zz.append(z.reshape(-1))
    return np.stack(rr), np.stack(zz)


def _deal(n_boxes, n_ranks, seed):
    owner = np.random.default_rng(seed).integers(0, n_ranks, size=n_boxes)
    return [[i for i in range(n_boxes) if owner[i] == r] for r in range(n_ranks)]


def _rank_parts(rr, zz, ranks, capacity=None):
    parts = []
    for r, mine in enumerate(ranks):
        fids = [r * oracle.FID_RANK + j for j in range(len(mine))]
        parts.append(oracle.deep_frame(rr[mine], zz[mine], fids, capacity))
    return parts


def test_interleaved_partition_composites_to_unsplit_image():
    """The negative pin's setup (4^3 boxes dealt to 4 ranks, every rank's data
    non-convex) composites to the unsplit image once ranks emit deep frames."""
    dims = (16, 16, 16)
    vol = random_volume(dims, 24)
    tf = rand_tf(34)
    prm = RenderParams(step_voxels=0.5, ert=1.0, density=30.0)
    cam = orbit_camera(dims, 12, 12)
    full, fz, _ = oracle.render_image(vol, dims, tf, prm, cam)
    boxes = even_split(dims, (4, 4, 4))
    rr, zz = _brick_frags(vol, dims, boxes, tf, prm, cam)
    parts = _rank_parts(rr, zz, _deal(len(boxes), 4, 5))
    assert max(int(p[0].max()) for p in parts) >= 2          # some pixel really holds several fragments
    comp, cz = oracle.composite_deep(parts)
    assert np.max(np.abs(comp - full.reshape(-1, 4))) <= 1e-12
    hit = np.isfinite(fz.reshape(-1))
    assert np.array_equal(np.isfinite(cz), hit)
    assert np.max(np.abs(cz[hit] - fz.reshape(-1)[hit])) <= 1e-12


def test_kd_partition_dealt_to_three_ranks():
    dims = (14, 11, 9)
    vol = random_volume(dims, 7)
    tf = rand_tf(8)
    prm = RenderParams(step_voxels=0.37, ert=1.0, density=25.0)
    cam = orbit_camera(dims, 10, 9)
    full, _, _ = oracle.render_image(vol, dims, tf, prm, cam)
    boxes = kd_split(dims, 9, seed=3, max_ratio=3.0)
    rr, zz = _brick_frags(vol, dims, boxes, tf, prm, cam)
    comp, _ = oracle.composite_deep(_rank_parts(rr, zz, _deal(len(boxes), 3, 11), capacity=12))
    assert np.max(np.abs(comp - full.reshape(-1, 4))) <= 1e-12


def test_deep_frame_layout():
    rng = np.random.default_rng(2)
    B, P = 5, 300
    depth = np.round(rng.random((B, P)) * 4, 1) + 1.0      # many exact ties
    depth[rng.random((B, P)) < 0.4] = np.inf
    rgba = rng.random((B, P, 4)) * np.isfinite(depth)[..., None]
    fids = rng.permutation(1000)[:B]
    count, lr, lz, lf = oracle.deep_frame(rgba, depth, fids, capacity=7)
    assert lr.shape == (7, P, 4) and lz.shape == (7, P) and lf.shape == (7, P)
    assert np.array_equal(count, np.isfinite(depth).sum(axis=0))
    for p in range(P):
        n = count[p]
        keys = [(lz[i, p], lf[i, p]) for i in range(n)]
        assert keys == sorted(keys) and len(set(lf[:n, p])) == n
        assert np.all(np.isinf(lz[n:, p])) and np.all(lf[n:, p] == -1) and np.all(lr[n:, p] == 0.0)
        # every live fragment appears once, with its own RGBA
        for i in range(n):
            b = int(np.flatnonzero(fids == lf[i, p])[0])
            assert lz[i, p] == depth[b, p] and np.array_equal(lr[i, p], rgba[b, p])
    # the packing does not depend on the order the bricks are given in
    perm = rng.permutation(B)
    again = oracle.deep_frame(rgba[perm], depth[perm], fids[perm], capacity=7)
    for a, b in zip((count, lr, lz, lf), again):
        assert np.array_equal(a, b)


def test_deep_composite_laws():
    rng = np.random.default_rng(9)
    B, P = 6, 200
    depth = rng.random((B, P)) * 3 + 1
    depth[rng.random((B, P)) < 0.3] = np.inf
    a = rng.random((B, P)) * 0.7
    rgba = np.concatenate([rng.random((B, P, 3)) * a[..., None], a[..., None]], axis=-1) * np.isfinite(depth)[..., None]
    ranks = [[0, 3], [1], [2, 4, 5]]
    parts = _rank_parts(rgba, depth, ranks)
    comp, cz = oracle.composite_deep(parts)
    # merging deep frames == compositing every fragment with its intrinsic id
    ids = np.concatenate([[r * oracle.FID_RANK + j for j in range(len(m))] for r, m in enumerate(ranks)])
    order = np.concatenate(ranks)
    flat, fz = oracle.composite(rgba[order], depth[order], ids)
    assert np.array_equal(comp, flat) and np.array_equal(cz, fz)
    # the order of the deep frames is irrelevant, bit for bit
    again, az = oracle.composite_deep([parts[2], parts[0], parts[1]])
    assert np.array_equal(comp, again) and np.array_equal(cz, az)
    # one fragment composites to itself
    one = oracle.deep_frame(rgba[:1], depth[:1], [0])
    c1, z1 = oracle.composite_deep([one])
    live = np.isfinite(depth[0])
    assert np.array_equal(c1[live], rgba[0][live]) and np.all(c1[~live] == 0.0)
    assert np.array_equal(z1, depth[0])
