"""Element-by-element comparison of a GPU tree with the CPU oracle."""
from __future__ import annotations

import numpy as np

SRC, RECV = 0, 1


def to_gpu(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _eq(name, got, exp):
    got = np.asarray(got)
    exp = np.asarray(exp)
    assert got.shape == exp.shape, f"{name}: shape {got.shape} vs {exp.shape}"
    if not np.array_equal(got, exp):
        bad = np.argwhere(got != exp)
        i = tuple(bad[0])
        raise AssertionError(f"{name}: {len(bad)} mismatches; first at {list(i)}: "
                             f"got {got[i]} expected {exp[i]}")


def compare_tables(g, o, key_bits):
    """Every table of every level, both sets, bit for bit."""
    assert g.depth == o.depth, (g.depth, o.depth)
    for s in (SRC, RECV):
        _eq(f"perm[{s}]", g.host_perm(s), o.perm(s))
        gx, ox = g.host_sorted_xyz(s), o.sorted_xyz(s)
        assert gx.tobytes() == ox.tobytes(), f"sorted_xyz[{s}] differs"
        for l in range(g.depth + 1):
            assert g.n_boxes(s, l) == o.n_boxes(s, l), (s, l)
            ok = o.keys(s, l)
            if key_bits == 32:
                ok = ok.astype(np.uint32)
            _eq(f"keys[{s}][{l}]", g.host_keys(s, l), ok)
            _eq(f"begin[{s}][{l}]", g.host_begin(s, l), o.begin(s, l))
            if l >= 1:
                _eq(f"parent[{s}][{l}]", g.host_parent(s, l), o.parent(s, l))
            if l < g.depth:
                _eq(f"child[{s}][{l}]", g.host_child(s, l), o.child(s, l))


def compare_lists(g, o):
    for l in range(2, g.depth + 1):
        for kind in (2, 4):
            go, ge = g.host_list(kind, l)
            oo, oe = o.list(kind, l)
            _eq(f"E{kind} offsets L{l}", go, oo)
            _eq(f"E{kind} entries L{l}", ge, oe)


def compare_lists_sampled(g, o, n_rows=1500, seed=0):
    """Lists of sampled receiver boxes against the oracle's per-box
    definition, plus structure checks of the whole CSR on the GPU copy."""
    rng = np.random.default_rng(seed)
    for l in range(2, g.depth + 1):
        nr = g.n_boxes(RECV, l)
        rows = np.unique(np.concatenate([[0, nr - 1], rng.integers(0, nr, size=min(n_rows, nr))]))
        for kind in (2, 4):
            got = g.host_list_rows(kind, l, rows)
            for r, row in zip(rows, got):
                _eq(f"E{kind} L{l} box {r}", row, o.box_list(kind, l, int(r)))
            off, ent = g.host_list(kind, l)
            assert off[0] == 0 and off[-1] == ent.size
            d = np.diff(off.astype(np.int64))
            assert d.min() >= 0 and d.max() <= (27 if kind == 2 else 189)
            assert ent.size == 0 or int(ent.max()) < g.n_boxes(SRC, l)
