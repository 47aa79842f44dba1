"""Element-by-element comparison of a GPU tree with the CPU oracle."""
from __future__ import annotations

import concurrent.futures as cf
import os
import sys

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


def _progress(msg):
    """Progress of long comparisons, past pytest's capture."""
    print(msg, file=sys.__stderr__, flush=True)


def compare_lists_chunked(g, o, chunk=1 << 17, threads=None):
    """Every offset and every entry of every E2 / E4 list of every level
    2..depth against the oracle's lists of the same receiver boxes, computed
    from the definition (Section 1.4) a range of boxes at a time, so that
    full-size builds are compared completely with bounded host memory. The
    ranges run on several host threads (the oracle call releases the GIL);
    each thread compares its own range."""
    threads = threads or max(1, min(16, os.cpu_count() or 1))
    for l in range(2, g.depth + 1):
        nr = g.n_boxes(RECV, l)
        assert nr == o.n_boxes(RECV, l), (l, nr, o.n_boxes(RECV, l))
        lk = o.lookup(l)
        try:
            for kind in (2, 4):
                goff, gent = g.host_list(kind, l)
                assert goff.size == nr + 1 and goff[0] == 0 and int(goff[-1]) == gent.size

                def job(r0, kind=kind, goff=goff, gent=gent):
                    r1 = min(nr, r0 + chunk)
                    ooff, oent = lk.range(kind, r0, r1)
                    rel = goff[r0:r1 + 1] - goff[r0]
                    if not np.array_equal(rel, ooff):
                        j = int(np.argmax(rel != ooff))
                        return f"E{kind} L{l}: offset of box {r0 + j}: {rel[j]} vs {ooff[j]} (from box {r0})"
                    got = gent[int(goff[r0]):int(goff[r1])]
                    if not np.array_equal(got, oent):
                        j = int(np.argmax(got != oent))
                        return f"E{kind} L{l}: entry {int(goff[r0]) + j}: {got[j]} vs {oent[j]}"
                    return int(ooff[-1])

                starts = list(range(0, nr, chunk))
                with cf.ThreadPoolExecutor(threads) as ex:
                    res = list(ex.map(job, starts))
                total = 0
                for r0, v in zip(starts, res):
                    if isinstance(v, str):
                        raise AssertionError(v)
                    assert int(goff[r0]) == total, (kind, l, r0)
                    total += v
                assert total == gent.size
                _progress(f"  E{kind} level {l}: {nr} receiver boxes, {gent.size} entries equal")
                del goff, gent
        finally:
            lk.close()
