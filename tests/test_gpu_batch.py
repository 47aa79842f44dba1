"""GPU parity of the batched form: every set of a batch equals the oracle's
build of that set alone (and the plain GPU build), eagerly and through HIP
graph replays with other work in between."""
import os

import numpy as np
import pytest

import parity
from paper_1301_1704_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1301_1704_amd as F
    if not os.path.exists(F.LIB_PATH):
        from paper_1301_1704_amd import _compile
        _compile.build()
    F._lib()
    return F


def _compare_set(g, o):
    parity.compare_tables(g, o, 64)
    parity.compare_lists(g, o)


def _small_batch(seed, n_sets, lo=4, hi=13):
    xyz, off, lev = I.batch_sets(n_sets, seed, lo, hi)
    return xyz, off, lev


@pytest.mark.parametrize("seed,n_sets", [(1, 1), (2, 7), (3, 40)])
def test_batch_sets_match_oracle(F, oracle_lib, seed, n_sets):
    import torch
    xyz, off, lev = _small_batch(seed, n_sets)
    b = F.Batch(off, lev)
    x = parity.to_gpu(xyz)
    b.launch(x)
    b.wait()
    for i in range(n_sets):
        pts = xyz[int(off[i]):int(off[i + 1])]
        o = oracle_lib.OracleTree(pts, None, key_bits=64, max_level=int(lev[i]))
        t = b.tree(i)
        assert t.depth == int(lev[i]) and t.n_src == pts.shape[0]
        _compare_set(t, o)
    b.free()
    torch.cuda.synchronize()


def test_build_batch_one_call(F, oracle_lib):
    """fmmds_build_batch (create, launch, wait in one call) gives every set
    the oracle's build, and the returned batch launches again like any other."""
    import torch
    xyz, off, lev = _small_batch(21, 9)
    x = parity.to_gpu(xyz)
    b = F.build_batch(x, off, lev)
    for i in range(9):
        pts = xyz[int(off[i]):int(off[i + 1])]
        o = oracle_lib.OracleTree(pts, None, key_bits=64, max_level=int(lev[i]))
        _compare_set(b.tree(i), o)
    first = b.tree(3).host_list(4, int(lev[3]))
    b.launch(x)
    b.wait()
    again = b.tree(3).host_list(4, int(lev[3]))
    assert all(np.array_equal(u, v) for u, v in zip(first, again))
    b.free()
    with pytest.raises(F.FmmdsError) as e:
        F.build_batch(x, off, np.full(9, 30, np.uint8))
    assert e.value.status == F.ERR_ARG
    torch.cuda.synchronize()


def test_batch_mixed_levels_and_tiny_sets(F, oracle_lib):
    """Sets of 1, 2 and a few points, and levels 2..7 in one batch."""
    parts = [I.uniform_points(5, 1), I.uniform_points(6, 2), I.uniform_points(7, 9),
             I.cluster_points(8, 3000, I.cluster_centres(9, 4), 0.02),
             I.uniform_points(10, 5000), np.full((100, 3), 0.7, np.float32)]
    lev = np.asarray([2, 3, 7, 6, 4, 5], dtype=np.uint8)
    off = np.zeros(len(parts) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([p.shape[0] for p in parts])
    xyz = np.ascontiguousarray(np.concatenate(parts, axis=0))
    b = F.Batch(off, lev)
    b.launch(parity.to_gpu(xyz))
    b.wait()
    for i, pts in enumerate(parts):
        o = oracle_lib.OracleTree(pts, None, key_bits=64, max_level=int(lev[i]))
        _compare_set(b.tree(i), o)
    b.free()


def test_batch_graph_replay(F):
    """The captured graph replays give the eager result every time, with
    eager work and synchronizations between replays, and new coordinates
    written into the same input buffer are picked up."""
    import torch
    xyz, off, lev = _small_batch(11, 24)
    xyz2, _, _ = _small_batch(11, 24)
    xyz2 = np.clip(xyz2 + 1e-3 * I.normal(12, xyz2.size).reshape(xyz2.shape), 0,
                   1 - 2 ** -24).astype(np.float32)
    x = parity.to_gpu(xyz)
    eager = F.Batch(off, lev)
    eager.launch(x)
    eager.wait()
    ref = {i: [eager.tree(i).host_list(k, int(lev[i])) for k in (2, 4)] + [eager.tree(i).host_perm(0)]
           for i in range(0, 24, 5)}
    g = F.Batch(off, lev)
    assert g.sort_items in (8, 12, 16, 32)
    for rep in range(4):
        g.launch(x, capture=True)
        g.wait()
        assert g.sort_items in (8, 12, 16, 32)
        for i, r in ref.items():
            t = g.tree(i)
            got = [t.host_list(k, int(lev[i])) for k in (2, 4)] + [t.host_perm(0)]
            for (a, bb), (c, d) in zip(got[:2], r[:2]):
                assert np.array_equal(a, c) and np.array_equal(bb, d), (rep, i)
            assert np.array_equal(got[2], r[2])
        y = torch.randn(1000, device="cuda").sum()  # eager work in between
        torch.cuda.synchronize()
        del y
    # new coordinates in the same buffer: the replay rebuilds them
    x.copy_(torch.from_numpy(xyz2).cuda())
    torch.cuda.synchronize()
    g.launch(x, capture=True)
    g.wait()
    e2 = F.Batch(off, lev)
    x2 = parity.to_gpu(xyz2)
    e2.launch(x2)
    e2.wait()
    for i in range(24):
        for k in (2, 4):
            a = g.tree(i).host_list(k, int(lev[i]))
            c = e2.tree(i).host_list(k, int(lev[i]))
            assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    for bb in (eager, g, e2):
        bb.free()


def test_batch_equals_plain_builds(F):
    import torch
    xyz, off, lev = _small_batch(21, 12, 8, 15)
    b = F.Batch(off, lev)
    b.launch(parity.to_gpu(xyz))
    b.wait()
    for i in range(12):
        pts = parity.to_gpu(xyz[int(off[i]):int(off[i + 1])])
        p = F.build(pts, None, max_level=int(lev[i]), key_bits=64)
        torch.cuda.synchronize()
        t = b.tree(i)
        assert np.array_equal(p.host_perm(0), t.host_perm(0))
        for l in range(int(lev[i]) + 1):
            assert np.array_equal(p.host_keys(0, l), t.host_keys(0, l))
            assert np.array_equal(p.host_begin(0, l), t.host_begin(0, l))
        for l in range(2, int(lev[i]) + 1):
            for k in (2, 4):
                x1, y1 = p.host_list(k, l)
                x2, y2 = t.host_list(k, l)
                assert np.array_equal(x1, x2) and np.array_equal(y1, y2)
        p.free()
    b.free()


def test_batch_range_error(F):
    xyz, off, lev = _small_batch(31, 5)
    xyz[int(off[3]) + 1, 2] = 1.0
    b = F.Batch(off, lev)
    b.launch(parity.to_gpu(xyz))
    with pytest.raises(F.FmmdsError) as e:
        b.wait()
    assert e.value.status == F.ERR_RANGE
    b.free()


def test_batch_bad_plans(F):
    with pytest.raises(F.FmmdsError):
        F.Batch(np.asarray([0, 5, 5], np.uint64), np.asarray([3, 3], np.uint8))  # empty set
    with pytest.raises(F.FmmdsError):
        F.Batch(np.asarray([0, 5], np.uint64), np.asarray([1], np.uint8))  # level < 2
    with pytest.raises(F.FmmdsError):
        F.Batch(np.asarray([1, 5], np.uint64), np.asarray([3], np.uint8))  # offsets[0] != 0


@pytest.mark.timeout(900)
def test_batch_full_512_sets_sampled(F, oracle_lib):
    """The full batched workload (512 sets, 2^10..2^20 points): sampled sets
    against the oracle, through a graph replay."""
    xyz, off, lev = I.batch_sets()
    b = F.Batch(off, lev)
    x = parity.to_gpu(xyz)
    b.launch(x, capture=True)
    b.wait()
    b.launch(x, capture=True)
    b.wait()
    rng = np.random.default_rng(5)
    for i in sorted(set(rng.integers(0, 512, 6).tolist()) | {0, 511}):
        pts = xyz[int(off[i]):int(off[i + 1])]
        o = oracle_lib.OracleTree(pts, None, key_bits=64, max_level=int(lev[i]))
        _compare_set(b.tree(i), o)
    b.free()


def _tile_edge_batch(sizes, levels, seed):
    parts = [I.uniform_points(seed + i, n) if i % 2 == 0 else
             I.cluster_points(seed + i, n, I.cluster_centres(seed + i, 4), 0.02)
             for i, n in enumerate(sizes)]
    off = np.zeros(len(parts) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    return (parts, np.ascontiguousarray(np.concatenate(parts, axis=0)), off,
            np.asarray(levels, dtype=np.uint8))


@pytest.mark.parametrize("items", [8, 12, 16, 32])
def test_batch_every_sort_tile_size(F, oracle_lib, monkeypatch, items):
    """Each sort tile size, fixed through FMMDS_BATCH_SORT_ITEMS, on sets
    that fill one partial tile, exactly one or two tiles, or several tiles
    and a ragged tail (the sort's tiles never straddle two sets): every set
    against the oracle, eagerly and through a graph replay."""
    sizes = [1, 7, 2047, 2048, 2049, 3072, 4096, 8192, 8197, 20001, 3, 16384]
    levels = [2, 3, 4, 4, 5, 3, 4, 5, 5, 6, 2, 4]
    parts, xyz, off, lev = _tile_edge_batch(sizes, levels, 40)
    monkeypatch.setenv("FMMDS_BATCH_SORT_ITEMS", str(items))
    b = F.Batch(off, lev)
    assert b.sort_items == items
    x = parity.to_gpu(xyz)
    for capture in (False, True):
        b.launch(x, capture=capture)
        b.wait()
        assert b.sort_items == items
        for i, pts in enumerate(parts):
            o = oracle_lib.OracleTree(pts, None, key_bits=64, max_level=int(lev[i]))
            _compare_set(b.tree(i), o)
    b.free()


@pytest.mark.parametrize("items", [8, 16])
def test_batch_keys_over_32_bits(F, oracle_lib, monkeypatch, items):
    """600 sets, one of them at level 8: composite keys of 10 + 24 bits, so
    keys and point indices sort as separate arrays."""
    rng = np.random.default_rng(9)
    sizes = [int(v) for v in rng.integers(1, 40, 600)]
    sizes[3] = 6000
    sizes[599] = 2500
    levels = [2 + (i % 3) for i in range(600)]
    levels[3] = 8
    parts, xyz, off, lev = _tile_edge_batch(sizes, levels, 70)
    monkeypatch.setenv("FMMDS_BATCH_SORT_ITEMS", str(items))
    b = F.Batch(off, lev)
    assert b.sort_items == items
    b.launch(parity.to_gpu(xyz))
    b.wait()
    for i in sorted({0, 1, 2, 3, 4, 300, 598, 599} | set(rng.integers(0, 600, 12).tolist())):
        o = oracle_lib.OracleTree(parts[i], None, key_bits=64, max_level=int(lev[i]))
        _compare_set(b.tree(i), o)
    b.free()
