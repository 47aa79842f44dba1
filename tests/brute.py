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
Only for inputs of a few hundred points. At the end: the list totals of a
slab of box centres in closed form, for sizes no enumeration reaches.
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


# ------------------------------------------------------- partition, box types

def partition(recv, l_par: int, n_ranks: int):
    """Rank of every Morton index at l_par (Section 3.2 reading): a nonempty
    receiver box whose first point is the p-th of M in Morton order goes to
    rank min(R - 1, R * p // M); other indices take the rank of the nearest
    nonempty box before them (0 if none). Counted from exact coordinates."""
    counts = {}
    for p in recv:
        k = morton_by_digits(p, l_par)
        counts[k] = counts.get(k, 0) + 1
    M = len(recv)
    owner, before, cur = [], 0, 0
    for m in range(8 ** l_par):
        if m in counts:
            cur = min(n_ranks - 1, n_ranks * before // M)
            before += counts[m]
        owner.append(cur)
    return owner


def box_types(src, recv, L: int, depth: int, l_par: int, owner, rank: int):
    """Source box types of `rank` per level 2..depth (DOMESTIC 0, EXPORT 1,
    IMPORT 2, ROOT 3, OTHER 4), from box coordinates and pair tests."""
    sp, st = tables(src, L, depth)
    rp, rt = tables(recv, L, depth)
    l_crit = l_par - 1

    def own_of(c, l):  # owner of the level-l box with coordinates c
        a = [v >> (l - l_par) for v in c]
        key = 0
        for m in range(l_par - 1, -1, -1):  # digits from the coarsest level
            key = (key << 3) | (((a[0] >> m) & 1) | (((a[1] >> m) & 1) << 1) |
                                (((a[2] >> m) & 1) << 2))
        return owner[key]

    def m2l(r, k):  # k in E4(r)
        cheb = max(abs(r[i] - k[i]) for i in range(3))
        pcheb = max(abs((r[i] >> 1) - (k[i] >> 1)) for i in range(3))
        return cheb >= 2 and pcheb <= 1

    out = []
    for l in range(2, depth + 1):
        sc = box_coords(src, sp, st, l)
        rc = box_coords(recv, rp, rt, l)
        if l < l_crit:
            out.append([0] * len(sc))
            continue
        types = []
        if l == l_crit:
            sch = box_coords(src, sp, st, l_par)
            rch = box_coords(recv, rp, rt, l_par)
            remote = [any(tuple(v >> 1 for v in c) == tuple(r) and own_of(c, l_par) != rank
                          for c in rch) for r in rc]
            for k in sc:
                kids = [c for c in sch if tuple(v >> 1 for v in c) == tuple(k)]
                on = any(own_of(c, l_par) == rank for c in kids)
                off = any(own_of(c, l_par) != rank for c in kids)
                if not on:
                    types.append(2)
                elif off:
                    types.append(3)
                else:
                    need = any(remote[i] and m2l(r, k) for i, r in enumerate(rc))
                    types.append(1 if need else 0)
        else:
            for k in sc:
                here = own_of(k, l) == rank
                if here:
                    need = any(own_of(r, l) != rank and m2l(r, k) for r in rc)
                    types.append(1 if need else 0)
                else:
                    need = any(own_of(r, l) == rank and m2l(r, k) for r in rc)
                    types.append(2 if need else 4)
        out.append(types)
    return out


# ------------------------------------------------------------- near field

def near_field(src, recv, depth: int, charges=None):
    """For every receiver point, in input order: the sum of q / |x - y| over
    the source points whose finest-level box is within Chebyshev distance 1
    of the receiver point's box (the E2 neighborhood), distance-0 pairs left
    out; FP64. No tables or lists: boxes from exact coordinates."""
    sc = [exact_coords(p, depth) for p in src]
    out = []
    for y in recv:
        cy = exact_coords(y, depth)
        f = 0.0
        for i, x in enumerate(src):
            if max(abs(sc[i][d] - cy[d]) for d in range(3)) > 1:
                continue
            r = float(np.sqrt(sum((float(x[d]) - float(y[d])) ** 2 for d in range(3))))
            if r == 0.0:
                continue
            f += (1.0 if charges is None else float(charges[i])) / r
        out.append(f)
    return np.asarray(out)


def slab_points(level: int, m: int) -> np.ndarray:
    """One point at the centre of every level-``level`` box whose z-coordinate
    is below m (the slab 2^level x 2^level x m), x fastest."""
    side = 1 << level
    ax = ((np.arange(side, dtype=np.float64) + 0.5) / side).astype(np.float32)
    z, y, x = np.meshgrid(ax[:m], ax, ax, indexing="ij")
    return np.ascontiguousarray(np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1))


def slab_list_totals(level: int, m: int):
    """E2 / E4 totals at ``level`` of slab_points(level, m) (m even, every
    box of the slab nonempty, sources = receivers), from Section 1.4's
    definitions. Both lists are products over the axes: a box at coordinate
    c has b(c) axis neighbours within one box (3, 2 at an end of the axis)
    and a(c) children of its parent's axis neighbours (6, 4 when the parent is
    at an end). A full axis of 2^level boxes gives sum b = 3 * 2^level - 2 and
    sum a = 6 * 2^level - 8; the z axis, m boxes from 0 with m / 2 parents,
    sum b = 3m - 2 and sum a = 6m - 8. So E2 = prod sum b and
    E4 = prod sum a - E2 (m = 2^level gives the full-grid closed forms)."""
    bx, ax = 3 * (1 << level) - 2, 6 * (1 << level) - 8
    bz, az = 3 * m - 2, 6 * m - 8
    e2 = bx * bx * bz
    return e2, ax * ax * az - e2
