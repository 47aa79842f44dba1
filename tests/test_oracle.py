"""Pins for the CPU oracle, against what the paper and the mathematics fix.

None of these tests re-runs the oracle's own formulas: expected values come
from exact rational arithmetic and pair enumeration (tests/brute.py), closed
forms on the full grid, a hand-worked example, and invariants that any correct
build satisfies (arXiv 1301.1704, Section 1.4 and Section 2).
"""
import numpy as np
import pytest

import brute
import golden_io
from paper_1301_1704_amd import inputs as I

pytestmark = pytest.mark.timeout(300) if hasattr(pytest.mark, "timeout") else []


def _tiny_sets():
    """(name, src, recv or None, max_level) cases of a few hundred points."""
    rng_u = I.uniform_points(11, 300)
    cl = I.cluster_points(12, 240, I.cluster_centres(13, 4), 0.03)
    # points on box faces of level 3 and their FP32 neighbours
    faces = []
    for k in (0, 1, 3, 4, 7):
        v = np.float32(k / 8.0)
        for w in (v, np.nextafter(v, np.float32(1)), np.nextafter(v, np.float32(0))):
            if 0 <= w < 1:
                faces.append(w)
    faces = np.asarray(faces, dtype=np.float32)
    fpts = np.stack(np.meshgrid(faces, faces[::2], faces[1::3], indexing="ij"), -1).reshape(-1, 3)
    dup = np.concatenate([rng_u[:40], rng_u[:40], rng_u[10:30]], axis=0)
    return [
        ("uniform-shared-L3", rng_u, None, 3),
        ("uniform-separate-L4", rng_u[:150], I.uniform_points(14, 170), 4),
        ("clusters-separate-L4", cl, rng_u[:90], 4),
        ("faces-shared-L3", np.ascontiguousarray(fpts, dtype=np.float32), None, 3),
        ("duplicates-separate-L3", dup, cl[:60], 3),
        ("single-point-L2", rng_u[:1], rng_u[5:6], 2),
    ]


CASES = _tiny_sets()


# ----------------------------------------------------------------- keys

@pytest.mark.parametrize("L", [1, 2, 3, 5, 8, 10, 13, 21])
def test_keys_match_exact_digits(oracle_lib, L):
    """Quantization and interleave: every 3-bit digit of the key is the
    octant of the point's box inside its parent, with box coordinates from
    exact rational arithmetic at each level."""
    pts = [I.uniform_points(21, 40)]
    # box faces at this level and their FP32 neighbours
    f = []
    for k in (0, 1, (1 << L) - 1, 1 << (L - 1), 3):
        v = np.float32(min(k, (1 << L) - 1) / float(1 << L))
        f += [v, np.nextafter(v, np.float32(1)), np.nextafter(v, np.float32(0))]
    f = np.asarray([w for w in f if 0 <= w < 1], dtype=np.float32)
    pts.append(np.stack([f, f[::-1], np.roll(f, 1)], axis=1))
    pts.append(np.asarray([[0.0, -0.0, 1e-40], [np.float32(1 - 2 ** -24)] * 3], dtype=np.float32))
    p = np.concatenate(pts, axis=0).astype(np.float32)
    keys = oracle_lib.point_keys(p, L)
    for i in range(p.shape[0]):
        assert int(keys[i]) == brute.morton_by_digits(p[i], L), (L, p[i])


def test_key_bit_convention(oracle_lib):
    """The library's bit order reading: x to bit 0, y to bit 1, z to bit 2
    of each 3-bit digit (the paper fixes none; parity unpinned by the
    paper, pinned here as the stated convention)."""
    q = np.float32(0.5)
    p = np.asarray([[q, 0, 0], [0, q, 0], [0, 0, q]], dtype=np.float32)
    assert oracle_lib.point_keys(p, 1).tolist() == [1, 2, 4]
    assert oracle_lib.point_keys(p, 2).tolist() == [8, 16, 32]


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf, 1.0, 1.5, -1e-30, -0.5])
def test_range_errors(oracle_lib, bad):
    p = np.asarray([[0.25, 0.25, 0.25], [0.5, bad, 0.5]], dtype=np.float32)
    with pytest.raises(oracle_lib.OracleError) as e:
        oracle_lib.point_keys(p, 4)
    assert e.value.status == oracle_lib.ERR_RANGE
    with pytest.raises(oracle_lib.OracleError) as e:
        oracle_lib.OracleTree(p, key_bits=64, max_level=4)
    assert e.value.status == oracle_lib.ERR_RANGE


def test_negative_zero_and_subnormal_accepted(oracle_lib):
    p = np.asarray([[-0.0, 1e-45, 1e-38]], dtype=np.float32)
    assert oracle_lib.point_keys(p, 10).tolist() == [0]


@pytest.mark.parametrize("kb,L,ok", [(32, 10, True), (32, 11, False), (64, 21, True),
                                     (64, 22, False), (64, 1, False), (16, 4, False)])
def test_argument_checks(oracle_lib, kb, L, ok):
    p = I.uniform_points(3, 10)
    if ok:
        t = oracle_lib.OracleTree(p, key_bits=kb, max_level=L, with_lists=False)
        assert t.depth == L
    else:
        with pytest.raises(oracle_lib.OracleError) as e:
            oracle_lib.OracleTree(p, key_bits=kb, max_level=L)
        assert e.value.status == oracle_lib.ERR_ARG


# ----------------------------------------------------------- hand example

def test_worked_example(oracle_lib):
    g = golden_io.read_kv("worked_example_level2.txt")
    t = oracle_lib.OracleTree(np.asarray(g["src"], np.float32), np.asarray(g["recv"], np.float32),
                              key_bits=32, max_level=g["max_level"])
    assert t.depth == 2
    for s, name in ((0, "src"), (1, "recv")):
        assert t.perm(s).tolist() == g[f"{name}_perm"]
        for l in range(3):
            assert t.keys(s, l).tolist() == g[f"{name}_keys_{l}"]
            assert t.begin(s, l).tolist() == g[f"{name}_begin_{l}"]
            if l >= 1:
                assert t.parent(s, l).tolist() == g[f"{name}_parent_{l}"]
            if l < 2:
                assert t.child(s, l).tolist() == g[f"{name}_child_{l}"]
    for kind in (2, 4):
        off, ent = t.list(kind, 2)
        assert off.tolist() == g[f"e{kind}_offsets_2"]
        assert ent.tolist() == g[f"e{kind}_entries_2"]


# ------------------------------------------------------------ brute force

@pytest.mark.parametrize("name,src,recv,L", CASES, ids=[c[0] for c in CASES])
def test_tables_and_order_by_brute_force(oracle_lib, name, src, recv, L):
    t = oracle_lib.OracleTree(src, recv, key_bits=64, max_level=L)
    for s, pts in ((0, src), (1, src if recv is None else recv)):
        perm, tab = brute.tables([tuple(p) for p in pts], L, L)
        assert t.perm(s).tolist() == perm
        assert t.sorted_xyz(s).tobytes() == np.ascontiguousarray(pts[perm]).tobytes()
        for l in range(L + 1):
            assert t.keys(s, l).tolist() == tab[l]["keys"], (s, l)
            assert t.begin(s, l).tolist() == tab[l]["begin"], (s, l)
            if l >= 1:
                assert t.parent(s, l).tolist() == tab[l]["parent"], (s, l)
            if l < L:
                assert t.child(s, l).tolist() == tab[l]["child"], (s, l)


@pytest.mark.parametrize("name,src,recv,L", CASES, ids=[c[0] for c in CASES])
def test_lists_by_pair_enumeration(oracle_lib, name, src, recv, L):
    t = oracle_lib.OracleTree(src, recv, key_bits=64, max_level=L)
    sp = [tuple(p) for p in src]
    rp = sp if recv is None else [tuple(p) for p in recv]
    exp = brute.lists_by_pairs(sp, rp, L, L)
    for l in range(2, L + 1):
        for kind, lists in ((2, exp[l][0]), (4, exp[l][1])):
            off, ent = t.list(kind, l)
            eo, ee = brute.csr(lists)
            assert off.tolist() == eo.tolist(), (kind, l)
            assert ent.tolist() == ee.tolist(), (kind, l)
            for r in range(len(lists)):
                assert t.box_list(kind, l, r).tolist() == lists[r]


@pytest.mark.parametrize("s", [1, 3, 8, 40, 1000])
def test_depth_rule_by_brute_force(oracle_lib, s):
    src = I.cluster_points(31, 300, I.cluster_centres(32, 3), 0.02)
    recv = I.uniform_points(33, 200)
    L = 5
    exp = L
    for l in range(2, L + 1):
        if (brute.max_occupancy([tuple(p) for p in src], l) <= s and
                brute.max_occupancy([tuple(p) for p in recv], l) <= s):
            exp = l
            break
    t = oracle_lib.OracleTree(src, recv, key_bits=64, cluster_s=s, max_level=L)
    assert t.depth == exp
    for l in range(2, exp + 1):
        assert t.max_occupancy(0, l) == brute.max_occupancy([tuple(p) for p in src], l)
    with pytest.raises(oracle_lib.OracleError):
        t.child(0, exp)  # the finest kept level has no children


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("L,m", [(3, 2), (4, 6), (5, 8), (5, 32)])
def test_slab_closed_forms(oracle_lib, L, m):
    """The oracle's finest-level list totals on a slab of box centres equal
    the slab closed form (which reduces to the full-grid one at m = 2^L)."""
    e2, e4 = brute.slab_list_totals(L, m)
    t = oracle_lib.OracleTree(brute.slab_points(L, m), key_bits=64, max_level=L)
    assert t.n_boxes(0, L) == (1 << L) ** 2 * m
    o2, _ = t.list(2, L)
    o4, _ = t.list(4, L)
    assert (int(o2[-1]), int(o4[-1])) == (e2, e4)


def test_slab_closed_form_is_the_full_grid_one():
    for L, e2, e4 in golden_io.read_table("closed_forms.txt"):
        assert brute.slab_list_totals(L, 1 << L) == (e2, e4)


@pytest.mark.parametrize("row", golden_io.read_table("closed_forms.txt")[:5])
def test_full_grid_closed_forms(oracle_lib, row):
    L, e2_total, e4_total = row
    t = oracle_lib.OracleTree(I.full_grid_points(L), key_bits=64, max_level=L)
    assert t.n_boxes(0, L) == 8 ** L
    for l in range(L + 1):
        b = t.begin(0, l)
        assert np.all(np.diff(b.astype(np.int64)) == 8 ** (L - l))
    o2, _ = t.list(2, L)
    o4, _ = t.list(4, L)
    assert int(o2[-1]) == e2_total and int(o4[-1]) == e4_total
    # per box: |E2| = prod b, |E4| = prod a - prod b
    m = 1 << L
    c = np.arange(m)
    bx = 3 - (c == 0) - (c == m - 1)
    p = c >> 1
    ax = 2 * (3 - (p == 0) - (p == (m >> 1) - 1))
    keys = t.keys(0, L)
    co = np.zeros((keys.size, 3), dtype=np.int64)
    for bit in range(L):
        for d in range(3):
            co[:, d] |= ((keys >> np.uint64(3 * bit + d)) & np.uint64(1)).astype(np.int64) << bit
    B = bx[co[:, 0]] * bx[co[:, 1]] * bx[co[:, 2]]
    A = ax[co[:, 0]] * ax[co[:, 1]] * ax[co[:, 2]]
    assert np.array_equal(np.diff(o2.astype(np.int64)), B)
    assert np.array_equal(np.diff(o4.astype(np.int64)), A - B)
    if L >= 3:
        assert B.max() == 27 and (A - B).max() == 189


# -------------------------------------------------------------- invariants

def _inv_cases():
    return [
        ("uniform", I.uniform_points(41, 3000), I.uniform_points(42, 2500), 5),
        ("sphere+clusters", I.sphere_cluster_points(43, 44, 4000),
         I.sphere_cluster_points(45, 44, 3000), 6),
    ]


@pytest.mark.parametrize("name,src,recv,L", _inv_cases(), ids=[c[0] for c in _inv_cases()])
def test_partition_of_sources(oracle_lib, name, src, recv, L):
    """For every receiver leaf b, the near list E2(b) at the finest level and
    the interaction lists E4 of b's ancestors at levels 2..D cover every
    source point exactly once (the near/far split of Eq. (2) done
    hierarchically, Section 1.4)."""
    t = oracle_lib.OracleTree(src, recv, key_bits=64, max_level=L)
    D = t.depth
    N = src.shape[0]
    sb = {l: t.begin(0, l).astype(np.int64) for l in range(D + 1)}
    lists = {(k, l): t.list(k, l) for k in (2, 4) for l in range(2, D + 1)}
    rpar = {l: t.parent(1, l) for l in range(1, D + 1)}
    # first sorted source point of each source box, and the leaf range it spans
    n_leaf = t.n_boxes(1, D)
    for b in range(n_leaf):
        covered = np.zeros(N, dtype=np.int32)
        anc = b
        for l in range(D, 1, -1):
            kinds = (2, 4) if l == D else (4,)
            for k in kinds:
                off, ent = lists[(k, l)]
                for s in ent[off[anc]:off[anc + 1]]:
                    covered[sb[l][s]:sb[l][s + 1]] += 1
            anc = int(rpar[l][anc])
        assert covered.min() == 1 and covered.max() == 1, b
        if b > 60:
            break


def test_invariants_and_symmetry_shared(oracle_lib):
    p = I.sphere_cluster_points(51, 52, 5000)
    t = oracle_lib.OracleTree(p, key_bits=64, max_level=6)
    n = p.shape[0]
    perm = t.perm(0)
    assert np.array_equal(np.sort(perm), np.arange(n, dtype=np.uint32))
    keys6 = oracle_lib.point_keys(p, 6)[perm]
    assert np.all(np.diff(keys6.astype(np.int64)) >= 0)
    ties = np.diff(keys6.astype(np.int64)) == 0
    assert np.all(np.diff(perm.astype(np.int64))[ties] > 0)
    for l in range(7):
        k = t.keys(0, l)
        b = t.begin(0, l)
        assert np.all(np.diff(k.astype(np.int64)) > 0)
        assert b[0] == 0 and b[-1] == n and np.all(np.diff(b.astype(np.int64)) > 0)
        if l < 6:
            c = t.child(0, l)
            assert c[0] == 0 and c[-1] == t.n_boxes(0, l + 1)
            par = t.parent(0, l + 1)
            assert np.array_equal(np.repeat(np.arange(k.size), np.diff(c.astype(np.int64))), par)
    for l in range(2, 7):
        for kind in (2, 4):
            off, ent = t.list(kind, l)
            pairs = set()
            for r in range(off.size - 1):
                row = ent[off[r]:off[r + 1]]
                assert np.all(np.diff(row.astype(np.int64)) > 0)
                pairs.update((r, int(s)) for s in row)
            assert pairs == {(s, r) for (r, s) in pairs}, (kind, l)
            assert np.diff(off.astype(np.int64)).max() <= (27 if kind == 2 else 189)


# ------------------------------------------- simulated partition, box types

TYPE_CASES = [
    ("uniform", I.uniform_points(71, 150), None, 4),
    ("separate", I.uniform_points(72, 120), I.sphere_cluster_points(73, 74, 140), 4),
    ("clustered", I.sphere_cluster_points(75, 76, 160), None, 5),
]


@pytest.mark.parametrize("name,src,recv,L", TYPE_CASES, ids=[c[0] for c in TYPE_CASES])
@pytest.mark.parametrize("n_ranks", [1, 2, 3, 5])
def test_partition_and_box_types_by_brute_force(oracle_lib, name, src, recv, L, n_ranks):
    """Section 3.2 partition and Section 3.1 box types against pair
    enumeration on exact box coordinates, for every rank."""
    t = oracle_lib.OracleTree(src, recv, key_bits=64, max_level=L)
    sp = [tuple(p) for p in src]
    rp = sp if recv is None else [tuple(p) for p in recv]
    for l_par in range(3, L + 1):
        owner = t.partition(l_par, n_ranks)
        assert owner.tolist() == brute.partition(rp, l_par, n_ranks), l_par
        for rank in range(n_ranks):
            exp = brute.box_types(sp, rp, L, L, l_par, owner.tolist(), rank)
            got = t.box_types(l_par, owner, rank)
            assert [g.tolist() for g in got] == exp, (l_par, rank)


def test_single_rank_is_all_domestic(oracle_lib):
    p = I.sphere_cluster_points(77, 78, 3000)
    t = oracle_lib.OracleTree(p, key_bits=64, max_level=6)
    for l_par in (3, 4, 6):
        owner = t.partition(l_par, 1)
        assert not owner.any()
        for ty in t.box_types(l_par, owner, 0):
            assert not ty.any()


def test_box_types_full_grid_closed_form(oracle_lib):
    """Counts per type on the full grid split by the plane z = 1/2 (the
    derivation is in the fixture)."""
    rows = golden_io.read_table("box_types_full_grid.txt")
    t = oracle_lib.OracleTree(I.full_grid_points(5), key_bits=64, max_level=5)
    owner = t.partition(3, 2)
    assert owner.tolist() == [0] * 256 + [1] * 256
    for rank in (0, 1):
        types = t.box_types(3, owner, rank)
        for row in rows:
            l, counts = row[0], row[1:]
            assert np.bincount(types[l - 2], minlength=5).tolist() == counts, (rank, l)


def test_root_boxes_where_the_split_cuts_a_critical_box(oracle_lib):
    """Three ranks over the 512 equal level-3 boxes of the full grid: the
    splits at Morton indices 171 and 342 fall inside the level-2 boxes 21 and
    42, which are the only ROOT boxes (Algorithm 6: a critical-level box with
    children on this rank and on another)."""
    t = oracle_lib.OracleTree(I.full_grid_points(4), key_bits=64, max_level=4)
    owner = t.partition(3, 3)
    assert owner.tolist() == [0] * 171 + [1] * 171 + [2] * 170
    keys2 = t.keys(0, 2)
    for rank, roots in ((0, [21]), (1, [21, 42]), (2, [42])):
        ty = t.box_types(3, owner, rank)
        assert keys2[ty[0] == 3].tolist() == roots
        for deeper in ty[1:]:
            assert not (deeper == 3).any()


def test_box_types_exchange_symmetry_shared(oracle_lib):
    """Shared sources and receivers (E4 symmetric): from l_par down, a box is
    EXPORT on its owner exactly when it is IMPORT on some other rank."""
    p = I.sphere_cluster_points(79, 80, 4000)
    t = oracle_lib.OracleTree(p, key_bits=64, max_level=6)
    R, l_par = 4, 3
    owner = t.partition(l_par, R)
    types = [t.box_types(l_par, owner, r) for r in range(R)]
    for l in range(l_par, 7):
        keys = t.keys(0, l)
        own = owner[keys >> np.uint64(3 * (l - l_par))]
        for i in range(keys.size):
            on_owner = types[own[i]][l - 2][i]
            elsewhere = [types[r][l - 2][i] for r in range(R) if r != own[i]]
            assert on_owner in (0, 1) and all(v in (2, 4) for v in elsewhere)
            assert (on_owner == 1) == any(v == 2 for v in elsewhere)


def test_one_box_type_agrees_with_whole_levels(oracle_lib):
    """The per-box evaluation (no lists) used for sampled checks of large
    builds gives the pinned whole-level result."""
    src = I.sphere_cluster_points(81, 82, 3000)
    recv = I.uniform_points(83, 2500)
    t = oracle_lib.OracleTree(src, recv, key_bits=64, max_level=6)
    for l_par, R in ((3, 3), (4, 5)):
        owner = t.partition(l_par, R)
        for rank in (0, R - 1):
            types = t.box_types(l_par, owner, rank)
            for l in range(2, 7):
                for k in range(0, types[l - 2].size, 7):
                    assert t.box_type_one(l_par, owner, rank, l, k) == types[l - 2][k], (l, k)


# ------------------------------------------------------------- near field

NEAR_CASES = [
    ("shared", I.uniform_points(101, 300), None, 3),
    ("separate", I.sphere_cluster_points(102, 103, 250), I.uniform_points(104, 200), 4),
]


@pytest.mark.parametrize("name,src,recv,L", NEAR_CASES, ids=[c[0] for c in NEAR_CASES])
@pytest.mark.parametrize("charged", [False, True])
def test_near_field_by_brute_force(oracle_lib, name, src, recv, L, charged):
    """Algorithm 2's gather plus the Laplace kernel, against the sum over
    every source point in the receiver's E2 neighborhood found from exact
    box coordinates (FP64 both; only the summation order differs)."""
    q = I.uniform_points(105, src.shape[0])[:, 0] - 0.5 if charged else None
    t = oracle_lib.OracleTree(src, recv, key_bits=64, max_level=L)
    phi, a = t.near_field(q)
    rp = src if recv is None else recv
    exp = brute.near_field([tuple(p) for p in src], [tuple(p) for p in rp], L, q)
    assert np.allclose(phi, exp, rtol=1e-12, atol=1e-12 * a.max())
    assert np.all(a >= np.abs(phi) * (1 - 1e-12))


def test_near_field_special_cases(oracle_lib):
    """One source point: each receiver in a neighboring box sees exactly
    q / r, the others 0; duplicated points do not see themselves."""
    src = np.asarray([[0.30, 0.30, 0.30]], dtype=np.float32)
    recv = np.asarray([[0.31, 0.29, 0.30], [0.55, 0.30, 0.30], [0.30, 0.30, 0.30],
                       [0.45, 0.45, 0.45]], dtype=np.float32)
    t = oracle_lib.OracleTree(src, recv, key_bits=64, max_level=3)
    phi, _ = t.near_field(np.asarray([2.0], dtype=np.float32))
    d0 = np.sqrt(np.sum((recv[0].astype(np.float64) - src[0]) ** 2))
    d3 = np.sqrt(np.sum((recv[3].astype(np.float64) - src[0]) ** 2))
    # boxes at level 3 have side 1/8: 0.30 -> 2, 0.55 -> 4 (two boxes away), 0.45 -> 3
    assert phi[0] == pytest.approx(2.0 / d0, rel=1e-15)
    assert phi[1] == 0.0
    assert phi[2] == 0.0  # same position as the source
    assert phi[3] == pytest.approx(2.0 / d3, rel=1e-15)


def test_near_field_pair_symmetry_shared(oracle_lib):
    """Shared sets: E2 is symmetric, so with unit charges the total over all
    receivers counts every near pair twice: equal to twice the pair sum."""
    p = I.sphere_cluster_points(106, 107, 800)
    t = oracle_lib.OracleTree(p, key_bits=64, max_level=4)
    phi, _ = t.near_field()
    keys = oracle_lib.point_keys(p, 4)
    c = np.stack([np.floor(p[:, d].astype(np.float64) * 16) for d in range(3)], axis=1)
    total = 0.0
    for i in range(len(p)):
        near = np.max(np.abs(c[i + 1:] - c[i]), axis=1) <= 1
        d = np.sqrt(np.sum((p[i + 1:][near].astype(np.float64) - p[i]) ** 2, axis=1))
        total += np.sum(1.0 / d[d > 0])
    assert keys.size == len(p)
    assert phi.sum() == pytest.approx(2.0 * total, rel=1e-12)


def test_near_field_one_point_agrees(oracle_lib):
    """The per-point evaluation (no lists) used for sampled checks of large
    builds gives the pinned whole-array result."""
    src = I.sphere_cluster_points(108, 109, 4000)
    recv = I.uniform_points(110, 3000)
    q = I.uniform_points(111, 4000)[:, 1] - 0.3
    t = oracle_lib.OracleTree(src, recv, key_bits=64, max_level=5)
    phi, a = t.near_field(q)
    for j in range(0, 3000, 37):
        f1, a1 = t.near_field_one(j, q)
        assert f1 == pytest.approx(phi[j], rel=1e-12, abs=1e-12 * a[j])
        assert a1 == pytest.approx(a[j], rel=1e-12)


def test_order_after_a_move_is_a_merge(oracle_lib):
    """The premise of the incremental rebuild, on the oracle alone: after the
    points move, the points that stayed in their finest box keep their
    relative order, so the new order is the merge of that old subsequence
    with the movers sorted by (key, index)."""
    from paper_1301_1704_amd import inputs as I
    L = 6
    p = I.sphere_cluster_points(501, 502, 20000)
    q = I.moved_points(p, 503, 2e-3)
    a = oracle_lib.OracleTree(p, None, key_bits=64, max_level=L, with_lists=False)
    b = oracle_lib.OracleTree(q, None, key_bits=64, max_level=L, with_lists=False)
    old_perm, new_perm = a.perm(0).astype(np.int64), b.perm(0).astype(np.int64)
    old_key = np.empty(p.shape[0], np.uint64)
    new_key = np.empty(p.shape[0], np.uint64)
    # every point's finest key, from each tree's boxes and bookmarks
    for tree, perm, out in ((a, old_perm, old_key), (b, new_perm, new_key)):
        keys, begin = tree.keys(0, L), tree.begin(0, L).astype(np.int64)
        out[perm] = np.repeat(keys, np.diff(begin))
    stay = old_key == new_key
    assert 0 < stay.sum() < p.shape[0]
    # stayers: same relative order in both
    assert np.array_equal(old_perm[stay[old_perm]], new_perm[stay[new_perm]])
    # the whole new order is (key, index) ascending, so it is the merge
    k = new_key[new_perm]
    assert np.all((k[1:] > k[:-1]) | ((k[1:] == k[:-1]) & (new_perm[1:] > new_perm[:-1])))
    a.close()
    b.close()


def test_dense_histogram_scans_give_the_tables(oracle_lib):
    """Algorithm 3 written out with numpy on the dense occupancy histogram of
    every level (reading c6: bookmark = exclusive scan of Bin, rank =
    inclusive scan of the nonempty flags minus one) equals the oracle's
    compacted tables, and the parent rank is ScannedRank of the key >> 3."""
    from paper_1301_1704_amd import inputs as I
    L = 6
    p = I.sphere_cluster_points(511, 512, 30000)
    o = oracle_lib.OracleTree(p, None, key_bits=64, max_level=L, with_lists=False)
    perm = o.perm(0).astype(np.int64)
    keys_L, begin_L = o.keys(0, L), o.begin(0, L).astype(np.int64)
    point_key = np.empty(p.shape[0], np.uint64)
    point_key[perm] = np.repeat(keys_L, np.diff(begin_L))
    for l in range(L + 1):
        k = (point_key >> np.uint64(3 * (L - l))).astype(np.int64)
        bins = np.bincount(k, minlength=8 ** l)
        scanned_bin = np.concatenate([[0], np.cumsum(bins)])
        flags = bins > 0
        scanned_rank = np.cumsum(flags) - 1
        nonempty = np.nonzero(flags)[0]
        assert np.array_equal(o.keys(0, l).astype(np.int64), nonempty)
        assert np.array_equal(o.begin(0, l).astype(np.int64),
                              np.concatenate([scanned_bin[nonempty], [p.shape[0]]]))
        if l >= 1:
            assert np.array_equal(o.parent(0, l).astype(np.int64),
                                  prev_rank[nonempty >> 3])
        prev_rank = scanned_rank
    o.close()


def test_list_ranges_equal_whole_lists(oracle_lib):
    """The range queries that check full-size builds return, for any range of
    receiver boxes, exactly the slice of the whole lists (both built from the
    definition of Section 1.4), also under concurrent queries."""
    import concurrent.futures as cf
    from paper_1301_1704_amd import inputs as I
    src = I.sphere_cluster_points(601, 602, 20000)
    recv = I.uniform_points(603, 15000)
    o = oracle_lib.OracleTree(src, recv, key_bits=64, max_level=6, with_lists=True)
    for l in range(2, 7):
        lk = o.lookup(l)
        for kind in (2, 4):
            off, ent = o.list(kind, l)
            n = off.size - 1
            cuts = sorted({0, 1, n // 7, n // 3, n // 2, n - 1, n})
            ranges = [(a, b) for a, b in zip(cuts[:-1], cuts[1:])] + [(0, n), (n, n)]
            with cf.ThreadPoolExecutor(4) as ex:
                got = list(ex.map(lambda r: lk.range(kind, *r), ranges))
            for (a, b), (ro, re) in zip(ranges, got):
                assert np.array_equal(ro, off[a:b + 1] - off[a])
                assert np.array_equal(re, ent[off[a]:off[b]])
        lk.close()
    with pytest.raises(oracle_lib.OracleError):
        o.lookup(7)
    o.close()


class _HostTree:
    """A stand-in for a GPU tree holding given host lists (for the checker's
    own test on the CPU)."""

    def __init__(self, o, lists):
        self.depth = o.depth
        self._o = o
        self._lists = lists

    def n_boxes(self, s, l):
        return self._o.n_boxes(s, l)

    def host_list(self, kind, l):
        off, ent = self._lists[(kind, l)]
        return off.copy(), ent.copy()


def test_chunked_list_check_finds_a_planted_difference(oracle_lib):
    """The complete full-size list check accepts the oracle's own lists and
    rejects one changed entry, one changed offset and one dropped entry."""
    import parity
    from paper_1301_1704_amd import inputs as I
    src, recv = I.uniform_points(611, 30000), I.uniform_points(612, 25000)
    o = oracle_lib.OracleTree(src, recv, key_bits=64, max_level=6, with_lists=True)
    lists = {(k, l): o.list(k, l) for l in range(2, 7) for k in (2, 4)}
    plain = oracle_lib.OracleTree(src, recv, key_bits=64, max_level=6, with_lists=False)
    parity.compare_lists_chunked(_HostTree(o, lists), plain, chunk=1000, threads=3)

    def planted(change):
        bad = {k: (v[0].copy(), v[1].copy()) for k, v in lists.items()}
        change(bad)
        with pytest.raises(AssertionError):
            parity.compare_lists_chunked(_HostTree(o, bad), plain, chunk=1000, threads=3)

    def entry(b):
        b[(4, 6)][1][12345] ^= 1

    def offset(b):
        b[(2, 5)][0][777] += 1

    def dropped(b):
        off, ent = b[(4, 4)]
        b[(4, 4)] = (np.concatenate([off[:10], off[10:] - 1]).astype(np.uint32),
                     np.delete(ent, int(off[9])))

    for change in (entry, offset, dropped):
        planted(change)
    o.close()
    plain.close()
