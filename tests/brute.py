"""Brute-force checker for tiny inputs, independent of the oracle's code.

Everything here is derived from the paper's definitions by a different route
than the oracle takes:
  - box coordinates come from exact rational arithmetic,
    floor(Fraction(x) * 2^l), computed separately at every level;
  - the Morton index is assembled from per-level octant digits (the octant of
    a box inside its parent is its coordinates mod 2), most significant digit
    first, rather than by interleaving the bits of the finest coordinates;
  - lists come from enumerating every (receiver box, source box) pair and
    testing the distance conditions on coordinates (Section 1.4 E2, E4).
Only for inputs of a few hundred points.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def exact_coords(p, level: int):
    s = 1 << level
    return tuple(int((Fraction(float(v)) * s).__floor__()) for v in p)


def octant(c) -> int:
    return (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2)


def morton_by_digits(p, level: int) -> int:
    """Key at `level`: the sequence of octants of the point's box at levels
    1..level, the coarsest in the most significant 3-bit digit."""
    key = 0
    for m in range(1, level + 1):
        key = (key << 3) | octant(exact_coords(p, m))
    return key


def order(points, L: int):
    """Points ordered by (level-L key, original index)."""
    keys = [morton_by_digits(p, L) for p in points]
    return sorted(range(len(points)), key=lambda i: (keys[i], i)), keys


def tables(points, L: int, depth: int):
    """Per level 0..depth: (keys, begin, parent, child) by counting."""
    perm, _ = order(points, L)
    out = []
    for l in range(depth + 1):
        ks = [morton_by_digits(points[i], l) for i in perm]
        keys, begin = [], []
        for k, v in enumerate(ks):
            if k == 0 or v != ks[k - 1]:
                keys.append(v)
                begin.append(k)
        begin.append(len(points))
        out.append({"keys": keys, "begin": begin})
    for l in range(1, depth + 1):
        up = out[l - 1]["keys"]
        # parent: the level-(l-1) box that contains the box's first point
        out[l]["parent"] = [up.index(morton_by_digits(points[perm[b]], l - 1))
                            for b in out[l]["begin"][:-1]]
    for l in range(depth):
        n_up = len(out[l]["keys"])
        par = out[l + 1]["parent"]
        out[l]["child"] = [min(k for k, q in enumerate(par) if q == j) for j in range(n_up)] + [len(par)]
    return perm, out


def box_coords(points, perm, tab, level: int):
    """Exact coordinates of each nonempty box (from its first point)."""
    return [exact_coords(points[perm[b]], level) for b in tab[level]["begin"][:-1]]


def lists_by_pairs(src, recv, L: int, depth: int):
    """{level: (E2 per receiver box, E4 per receiver box)}, levels 2..depth,
    by testing every pair of nonempty boxes."""
    sp, st = tables(src, L, depth)
    rp, rt = tables(recv, L, depth)
    res = {}
    for l in range(2, depth + 1):
        sc = box_coords(src, sp, st, l)
        rc = box_coords(recv, rp, rt, l)
        e2, e4 = [], []
        for c in rc:
            a, b = [], []
            for j, d in enumerate(sc):
                cheb = max(abs(d[i] - c[i]) for i in range(3))
                pcheb = max(abs((d[i] >> 1) - (c[i] >> 1)) for i in range(3))
                if cheb <= 1:
                    a.append(j)
                elif pcheb <= 1:
                    b.append(j)
            e2.append(a)
            e4.append(b)
        res[l] = (e2, e4)
    return res


def csr(lists):
    off = np.zeros(len(lists) + 1, dtype=np.uint32)
    off[1:] = np.cumsum([len(x) for x in lists])
    ent = np.asarray([v for x in lists for v in x], dtype=np.uint32)
    return off, ent


def max_occupancy(points, level: int) -> int:
    counts = {}
    for p in points:
        k = morton_by_digits(p, level)
        counts[k] = counts.get(k, 0) + 1
    return max(counts.values())
