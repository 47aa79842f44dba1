"""CPU oracle for the FMM data-structure build: TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. It loads ``liboracle_fmmds.so``, a plain single-threaded
C++ build written from the paper's definitions (see fmmds_oracle.cpp), and
returns numpy arrays. It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_fmmds.so")
SOURCES = [os.path.join(HERE, "fmmds_oracle.cpp")]

OK, ERR_ARG, ERR_RANGE, ERR_NOMEM, ERR_LEVEL, ERR_OVERFLOW = 0, 1, 2, 3, 5, 6
SRC, RECV = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (host only)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp] + SOURCES
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        u32, u64, i32 = C.c_uint32, C.c_uint64, C.c_int
        vp = C.c_void_p
        L.oref_point_keys.argtypes = [vp, u32, u32, vp]
        L.oref_build.argtypes = [vp, u32, vp, u32, u32, u32, u32, i32, C.POINTER(vp)]
        L.oref_free.argtypes = [vp]
        L.oref_free.restype = None
        for f in ("oref_depth",):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = u32
        L.oref_n_points.argtypes = [vp, i32]
        L.oref_n_points.restype = u32
        L.oref_n_boxes.argtypes = [vp, i32, u32]
        L.oref_n_boxes.restype = u32
        L.oref_max_occupancy.argtypes = [vp, i32, u32]
        L.oref_max_occupancy.restype = u32
        L.oref_perm.argtypes = [vp, i32, vp]
        L.oref_sorted_xyz.argtypes = [vp, i32, vp]
        for f in ("oref_keys", "oref_begin", "oref_parent", "oref_child"):
            getattr(L, f).argtypes = [vp, i32, u32, vp]
        L.oref_list_sizes.argtypes = [vp, i32, u32, C.POINTER(u32), C.POINTER(u64)]
        L.oref_list.argtypes = [vp, i32, u32, vp, vp]
        L.oref_box_list.argtypes = [vp, i32, u32, u32, vp]
        L.oref_lookup_open.argtypes = [vp, u32]
        L.oref_lookup_open.restype = vp
        L.oref_lookup_close.argtypes = [vp]
        L.oref_lookup_close.restype = None
        L.oref_list_range.argtypes = [vp, i32, u32, u32, vp, vp]
        L.oref_partition.argtypes = [vp, u32, u32, vp]
        L.oref_box_types.argtypes = [vp, u32, vp, u32, vp]
        L.oref_box_type_one.argtypes = [vp, u32, vp, u32, u32, u32]
        L.oref_near_field.argtypes = [vp, vp, vp, vp]
        L.oref_near_field_one.argtypes = [vp, vp, u32, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double)]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(-1, 3))


def point_keys(xyz, level: int) -> np.ndarray:
    x = _f32(xyz)
    out = np.empty(x.shape[0], dtype=np.uint64)
    st = lib().oref_point_keys(_ptr(x), x.shape[0], level, _ptr(out))
    if st != OK:
        raise OracleError(st, "oref_point_keys")
    return out


class OracleTree:
    """Tables (and optionally lists) of one build, fetched as numpy arrays."""

    def __init__(self, src, recv=None, *, key_bits=64, cluster_s=0, max_level=5,
                 with_lists=True):
        self._h = None
        s = _f32(src)
        r = None if recv is None else _f32(recv)
        h = C.c_void_p()
        st = lib().oref_build(_ptr(s), s.shape[0], None if r is None else _ptr(r),
                              0 if r is None else r.shape[0], key_bits, cluster_s,
                              max_level, 1 if with_lists else 0, C.byref(h))
        if st != OK:
            raise OracleError(st, "oref_build")
        self._h = h
        self.shared = r is None
        self.key_bits = key_bits
        self.with_lists = with_lists
        self.depth = int(lib().oref_depth(h))

    def close(self):
        if self._h is not None:
            lib().oref_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def n_points(self, s: int) -> int:
        return int(lib().oref_n_points(self._h, s))

    def n_boxes(self, s: int, level: int) -> int:
        return int(lib().oref_n_boxes(self._h, s, level))

    def max_occupancy(self, s: int, level: int) -> int:
        return int(lib().oref_max_occupancy(self._h, s, level))

    def perm(self, s: int) -> np.ndarray:
        out = np.empty(self.n_points(s), dtype=np.uint32)
        lib().oref_perm(self._h, s, _ptr(out))
        return out

    def sorted_xyz(self, s: int) -> np.ndarray:
        out = np.empty((self.n_points(s), 3), dtype=np.float32)
        lib().oref_sorted_xyz(self._h, s, _ptr(out))
        return out

    def _get(self, fn, s, level, n, dtype):
        out = np.empty(n, dtype=dtype)
        st = getattr(lib(), fn)(self._h, s, level, _ptr(out))
        if st != OK:
            raise OracleError(st, fn)
        return out

    def keys(self, s: int, level: int) -> np.ndarray:
        return self._get("oref_keys", s, level, self.n_boxes(s, level), np.uint64)

    def begin(self, s: int, level: int) -> np.ndarray:
        return self._get("oref_begin", s, level, self.n_boxes(s, level) + 1, np.uint32)

    def parent(self, s: int, level: int) -> np.ndarray:
        return self._get("oref_parent", s, level, self.n_boxes(s, level), np.uint32)

    def child(self, s: int, level: int) -> np.ndarray:
        return self._get("oref_child", s, level, self.n_boxes(s, level) + 1, np.uint32)

    def list(self, kind: int, level: int):
        """(offsets, entries) of E2 (kind 2) or E4 (kind 4) at a level."""
        nb, ne = C.c_uint32(), C.c_uint64()
        st = lib().oref_list_sizes(self._h, kind, level, C.byref(nb), C.byref(ne))
        if st != OK:
            raise OracleError(st, "oref_list_sizes")
        off = np.empty(nb.value + 1, dtype=np.uint32)
        ent = np.empty(ne.value, dtype=np.uint32)
        st = lib().oref_list(self._h, kind, level, _ptr(off), _ptr(ent))
        if st != OK:
            raise OracleError(st, "oref_list")
        return off, ent

    def box_list(self, kind: int, level: int, recv_box: int) -> np.ndarray:
        buf = np.empty(189, dtype=np.uint32)
        n = lib().oref_box_list(self._h, kind, level, recv_box, _ptr(buf))
        if n < 0:
            raise OracleError(-n, "oref_box_list")
        return buf[:n].copy()

    def lookup(self, level: int) -> "ListLookup":
        """Range queries of the lists of one level (oref_list_range)."""
        return ListLookup(self, level)

    def partition(self, l_par: int, n_ranks: int) -> np.ndarray:
        """Rank of every Morton index at level l_par (Section 3.2)."""
        out = np.empty(1 << (3 * l_par), dtype=np.uint32)
        st = lib().oref_partition(self._h, l_par, n_ranks, _ptr(out))
        if st != OK:
            raise OracleError(st, "oref_partition")
        return out

    def box_types(self, l_par: int, owner: np.ndarray, rank: int) -> list:
        """Source box types of `rank` per level 2..depth (list of uint8
        arrays; index 0 is level 2): DOMESTIC 0, EXPORT 1, IMPORT 2, ROOT 3,
        OTHER 4 (Section 3.1, Algorithm 6)."""
        ow = np.ascontiguousarray(owner, dtype=np.uint32)
        sizes = [self.n_boxes(SRC, l) for l in range(2, self.depth + 1)]
        out = np.empty(sum(sizes), dtype=np.uint8)
        st = lib().oref_box_types(self._h, l_par, _ptr(ow), rank, _ptr(out))
        if st != OK:
            raise OracleError(st, "oref_box_types")
        return np.split(out, np.cumsum(sizes)[:-1])

    def box_type_one(self, l_par: int, owner: np.ndarray, rank: int, level: int,
                     box: int) -> int:
        """Type of one source box, from the definition without lists."""
        ow = np.ascontiguousarray(owner, dtype=np.uint32)
        v = lib().oref_box_type_one(self._h, l_par, _ptr(ow), rank, level, box)
        if v < 0:
            raise OracleError(-v, "oref_box_type_one")
        return int(v)

    def near_field(self, charges=None):
        """(phi, abs_sum) per receiver point in original order, FP64: the
        Laplace sum over the source points of the E2 boxes of each receiver
        point's finest-level box (Algorithm 2)."""
        m = self.n_points(RECV)
        phi = np.empty(m, dtype=np.float64)
        a = np.empty(m, dtype=np.float64)
        q = None if charges is None else np.ascontiguousarray(charges, dtype=np.float32)
        st = lib().oref_near_field(self._h, None if q is None else _ptr(q), _ptr(phi), _ptr(a))
        if st != OK:
            raise OracleError(st, "oref_near_field")
        return phi, a

    def near_field_one(self, j: int, charges=None):
        """(phi, abs_sum) of receiver point j (original index), FP64, from
        the definition without lists."""
        q = None if charges is None else np.ascontiguousarray(charges, dtype=np.float32)
        f, a = C.c_double(), C.c_double()
        st = lib().oref_near_field_one(self._h, None if q is None else _ptr(q), j,
                                       C.byref(f), C.byref(a))
        if st != OK:
            raise OracleError(st, "oref_near_field_one")
        return f.value, a.value


class ListLookup:
    """E2 / E4 lists of ranges of receiver boxes of one level, computed from
    the definition on demand. The oracle call releases the GIL, so several
    Python threads can query one lookup at once."""

    def __init__(self, tree: OracleTree, level: int):
        self._tree = tree  # the lookup reads the tree's tables
        self.level = level
        self._h = lib().oref_lookup_open(tree._h, level)
        if not self._h:
            raise OracleError(ERR_LEVEL, "oref_lookup_open")

    def range(self, kind: int, r0: int, r1: int):
        """(offsets relative to box r0, entries) of receiver boxes [r0, r1)."""
        off = np.empty(r1 - r0 + 1, dtype=np.uint32)
        ent = np.empty((r1 - r0) * (27 if kind == 2 else 189), dtype=np.uint32)
        st = lib().oref_list_range(self._h, kind, r0, r1, _ptr(off), _ptr(ent))
        if st != OK:
            raise OracleError(st, "oref_list_range")
        return off, ent[:int(off[-1])]

    def close(self):
        if getattr(self, "_h", None):
            lib().oref_lookup_close(self._h)
            self._h = None

    def __del__(self):
        self.close()
