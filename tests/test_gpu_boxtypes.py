"""GPU parity of the simulated partition and the source box types (Section
3.1, Algorithm 6; Section 3.2): fmmds_partition and fmmds_box_types through
the C ABI against the oracle, element by element (integer outputs,
tolerance 0). Small builds compare every level for several ranks; the full
2 x 2^24 level-8 build compares sampled boxes against the oracle's per-box
definition and checks properties that hold at any size."""
import os
import sys

import numpy as np
import pytest

import parity
from paper_1301_1704_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


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


def _gpu_types(g, l_par, owner, rank):
    import torch
    out, sizes = g.box_types(l_par, owner, rank)
    torch.cuda.synchronize()
    flat = out.cpu().numpy()[:sum(sizes)]
    return np.split(flat, np.cumsum(sizes)[:-1])


CASES = [
    ("shared-uniform", lambda: (I.uniform_points(91, 30000), None), 6, 64),
    ("separate-mixed", lambda: (I.uniform_points(92, 20000),
                                I.sphere_cluster_points(93, 94, 25000)), 6, 64),
    ("clustered-u32", lambda: (I.sphere_cluster_points(95, 96, 40000), None), 7, 32),
]


@pytest.mark.parametrize("name,make,L,kb", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("n_ranks", [1, 2, 7, 64])
def test_partition_and_types_match_oracle(F, oracle_lib, name, make, L, kb, n_ranks):
    import torch
    src, recv = make()
    _say(f"case {name} L={L} kb={kb} ranks={n_ranks}")
    g = F.build(parity.to_gpu(src), None if recv is None else parity.to_gpu(recv),
                max_level=L, key_bits=kb)
    torch.cuda.synchronize()
    o = oracle_lib.OracleTree(src, recv, key_bits=kb, max_level=L)
    for l_par in sorted({3, 4, L}):
        owner = g.partition(l_par, n_ranks)
        torch.cuda.synchronize()
        o_owner = o.partition(l_par, n_ranks)
        assert np.array_equal(owner.cpu().numpy().view(np.uint32), o_owner), l_par
        ranks = range(n_ranks) if n_ranks <= 7 else (0, 1, n_ranks // 2, n_ranks - 1)
        for rank in ranks:
            got = _gpu_types(g, l_par, owner, rank)
            exp = o.box_types(l_par, o_owner, rank)
            for l, (a, b) in enumerate(zip(got, exp), start=2):
                assert np.array_equal(a, b), (l_par, rank, l)
    g.free()
    o.close()


def test_full_grid_closed_form(F):
    import golden_io
    import torch
    rows = golden_io.read_table("box_types_full_grid.txt")
    g = F.build(parity.to_gpu(I.full_grid_points(5)), None, max_level=5, key_bits=64)
    torch.cuda.synchronize()
    owner = g.partition(3, 2)
    torch.cuda.synchronize()
    assert owner.cpu().numpy().tolist() == [0] * 256 + [1] * 256
    for rank in (0, 1):
        types = _gpu_types(g, 3, owner, rank)
        for row in rows:
            assert np.bincount(types[row[0] - 2], minlength=5).tolist() == row[1:], (rank, row)
    g.free()


def test_batch_view_equals_plain_build(F):
    """Box types of a set inside a batch equal those of the same set built
    alone (set-local ranks and lists)."""
    import torch
    sizes = [5000, 12000, 3000]
    pts = [I.sphere_cluster_points(97 + i, 98, n) for i, n in enumerate(sizes)]
    lev = np.asarray([5, 6, 4], np.uint8)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    b = F.Batch(off, lev)
    b.launch(parity.to_gpu(np.concatenate(pts)))
    b.wait()
    for i in range(3):
        t = b.tree(i)
        alone = F.build(parity.to_gpu(pts[i]), None, max_level=int(lev[i]), key_bits=64)
        torch.cuda.synchronize()
        for l_par in range(3, int(lev[i]) + 1):
            ow_b = t.partition(l_par, 5)
            ow_a = alone.partition(l_par, 5)
            torch.cuda.synchronize()
            assert torch.equal(ow_b, ow_a)
            for rank in (0, 2, 4):
                for x, y in zip(_gpu_types(t, l_par, ow_b, rank),
                                _gpu_types(alone, l_par, ow_a, rank)):
                    assert np.array_equal(x, y), (i, l_par, rank)
        alone.free()
    b.free()


def test_argument_errors(F):
    import torch
    g = F.build(parity.to_gpu(I.uniform_points(99, 5000)), None, max_level=5)
    torch.cuda.synchronize()
    for bad in (2, 6):
        with pytest.raises(F.FmmdsError) as e:
            g.partition(bad, 4)
        assert e.value.status == F.ERR_LEVEL
    with pytest.raises(F.FmmdsError) as e:
        g.partition(3, 0)
    assert e.value.status == F.ERR_ARG
    owner = g.partition(3, 4)
    with pytest.raises(F.FmmdsError) as e:
        g.box_types(6, owner, 0)
    assert e.value.status == F.ERR_LEVEL
    g.free()


@pytest.mark.slow
def test_full_uniform_2x2p24_L8_sampled(F, oracle_lib):
    """The benchmark build with 64 ranks at partition level 4: sampled boxes
    of every level against the oracle's per-box definition, and at full size:
    each box of level >= l_par is DOMESTIC or EXPORT on its owner and IMPORT
    or OTHER elsewhere, and ROOT occurs only at the critical level."""
    import torch
    c = I.config_plain_uniform()
    _say("case full uniform 2x2^24 L8, 64 ranks, l_par 4")
    g = F.build(parity.to_gpu(c["src"]), parity.to_gpu(c["recv"]), max_level=8, key_bits=64)
    torch.cuda.synchronize()
    o = oracle_lib.OracleTree(c["src"], c["recv"], key_bits=64, max_level=8, with_lists=False)
    R, l_par = 64, 4
    owner = g.partition(l_par, R)
    torch.cuda.synchronize()
    ow = owner.cpu().numpy().view(np.uint32)
    assert np.array_equal(ow, o.partition(l_par, R))
    rng = np.random.default_rng(5)
    for rank in (0, 31, 63):
        types = _gpu_types(g, l_par, owner, rank)
        for l in range(2, 9):
            ty = types[l - 2]
            if l < l_par - 1:
                assert not ty.any()
            if l != l_par - 1:
                assert not (ty == 3).any()
            if l >= l_par:
                keys = g.host_keys(0, l)
                here = ow[keys >> np.uint64(3 * (l - l_par))] == rank
                assert np.isin(ty[here], (0, 1)).all() and np.isin(ty[~here], (2, 4)).all()
            for k in rng.choice(ty.size, size=min(ty.size, 300), replace=False):
                assert ty[k] == o.box_type_one(l_par, ow, rank, l, int(k)), (rank, l, k)
    g.free()
    o.close()
