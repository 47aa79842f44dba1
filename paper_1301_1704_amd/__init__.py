"""Python binding of libfmmds (include/fmmds.h): argument marshalling only.

Every step of the build runs in the library's HIP kernels on the GPU. This
module passes device pointers of torch tensors and torch's current stream to
the C ABI, and copies results back when asked. There is no CPU path: if the
library is missing or no GPU is present the calls raise.

The HIP runtime: torch ships its own libamdhip64.so.7. torch is imported
before libfmmds.so is loaded, so the library binds to that same runtime
instance (one HIP runtime per process) and can use torch's memory and streams.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmmds.so")
MAX_LEVEL = 21

OK, ERR_ARG, ERR_RANGE, ERR_NOMEM, ERR_DEVICE, ERR_LEVEL, ERR_OVERFLOW, ERR_TOO_LARGE = range(8)
SRC, RECV = 0, 1

_u32, _u64, _vp = C.c_uint32, C.c_uint64, C.c_void_p
ALLOC_FN = C.CFUNCTYPE(_vp, _vp, C.c_size_t, _vp)
RELEASE_FN = C.CFUNCTYPE(None, _vp, _vp, C.c_size_t, _vp)


class Options(C.Structure):
    _fields_ = [("key_bits", _u32), ("cluster_s", _u32), ("max_level", _u32),
                ("reserved", _u32), ("stream", _vp), ("alloc", ALLOC_FN),
                ("release", RELEASE_FN), ("alloc_ctx", _vp)]


class Level(C.Structure):
    _fields_ = [("n", _u32), ("key", _vp), ("begin", _vp), ("parent", _vp), ("child", _vp)]


class TreeStruct(C.Structure):
    _fields_ = [("depth", _u32), ("key_bits", _u32), ("max_level", _u32), ("shared", _u32),
                ("n_src", _u32), ("n_recv", _u32),
                ("src_perm", _vp), ("recv_perm", _vp),
                ("src_sorted_xyz", _vp), ("recv_sorted_xyz", _vp),
                ("src", Level * (MAX_LEVEL + 1)), ("recv", Level * (MAX_LEVEL + 1)),
                ("impl", _vp)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", _u64), ("total_ms", C.c_double),
                ("bytes", C.c_double)]


class FmmdsError(RuntimeError):
    def __init__(self, status: int, what: str = "fmmds"):
        name = _lib().fmmds_status_string(status).decode() if _LIB is not None else str(status)
        super().__init__(f"{what}: {name} (status {status})")
        self.status = status


_LIB = None
_HIP = None


def _lib():
    global _LIB, _HIP
    if _LIB is None:
        import torch  # binds the HIP runtime first (see module docstring)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1301_1704_amd/_compile.py "
                               "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        L.fmmds_build.argtypes = [_vp, _u32, _vp, _u32, C.POINTER(Options),
                                  C.POINTER(C.POINTER(TreeStruct))]
        L.fmmds_build.restype = C.c_int
        L.fmmds_build_dense.argtypes = [_vp, _u32, _vp, _u32, C.POINTER(Options),
                                        C.POINTER(C.POINTER(TreeStruct))]
        L.fmmds_build_dense.restype = C.c_int
        L.fmmds_rebuild.argtypes = [C.POINTER(TreeStruct), _vp, _vp, _u32, C.POINTER(Options),
                                    C.POINTER(C.POINTER(TreeStruct))]
        L.fmmds_rebuild.restype = C.c_int
        for f in ("fmmds_neighbors", "fmmds_interactions"):
            getattr(L, f).argtypes = [C.POINTER(TreeStruct), _u32, C.POINTER(_vp), C.POINTER(_vp),
                                      C.POINTER(_u32), C.POINTER(_u64)]
            getattr(L, f).restype = C.c_int
        L.fmmds_free.argtypes = [C.POINTER(TreeStruct)]
        L.fmmds_free.restype = None
        L.fmmds_trim.restype = None
        L.fmmds_cache_info.argtypes = [C.POINTER(_u64)] * 4
        L.fmmds_cache_info.restype = None
        L.fmmds_batch_create.argtypes = [_vp, _vp, _u32, C.POINTER(Options), C.POINTER(_vp)]
        L.fmmds_batch_create.restype = C.c_int
        L.fmmds_batch_launch.argtypes = [_vp, _vp, C.c_int]
        L.fmmds_batch_launch.restype = C.c_int
        L.fmmds_batch_wait.argtypes = [_vp]
        L.fmmds_batch_wait.restype = C.c_int
        L.fmmds_batch_tree.argtypes = [_vp, _u32]
        L.fmmds_batch_tree.restype = C.POINTER(TreeStruct)
        L.fmmds_batch_footprint.argtypes = [_vp, _vp, _u32, C.POINTER(_u64)]
        L.fmmds_batch_footprint.restype = C.c_int
        L.fmmds_batch_bytes.argtypes = [_vp]
        L.fmmds_batch_bytes.restype = _u64
        L.fmmds_batch_sort_items.argtypes = [_vp]
        L.fmmds_batch_sort_items.restype = _u32
        L.fmmds_batch_free.argtypes = [_vp]
        L.fmmds_batch_free.restype = None
        L.fmmds_build_batch.argtypes = [_vp, _vp, _vp, _u32, C.POINTER(Options), C.POINTER(_vp)]
        L.fmmds_build_batch.restype = C.c_int
        L.fmmds_free_batch.argtypes = [_vp]
        L.fmmds_free_batch.restype = None
        L.fmmds_partition.argtypes = [C.POINTER(TreeStruct), _u32, _u32, _vp, _vp]
        L.fmmds_partition.restype = C.c_int
        L.fmmds_box_types.argtypes = [C.POINTER(TreeStruct), _u32, _vp, _u32, _vp, _vp]
        L.fmmds_box_types.restype = C.c_int
        L.fmmds_near_field.argtypes = [C.POINTER(TreeStruct), _vp, _vp, _vp, _vp]
        L.fmmds_near_field.restype = C.c_int
        L.fmmds_near_field_static.argtypes = [C.POINTER(TreeStruct), _vp, _vp, _vp, _vp]
        L.fmmds_near_field_static.restype = C.c_int
        L.fmmds_displace.argtypes = [C.POINTER(DisplaceSet), _u32, C.c_float, _vp, _vp]
        L.fmmds_displace.restype = C.c_int
        L.fmmds_profile_enable.argtypes = [C.c_int, C.c_char_p]
        L.fmmds_profile_enable.restype = None
        L.fmmds_profile_reset.restype = None
        L.fmmds_profile_read.argtypes = [C.POINTER(KernelStat), _u32]
        L.fmmds_profile_read.restype = _u32
        L.fmmds_status_string.argtypes = [C.c_int]
        L.fmmds_status_string.restype = C.c_char_p
        H = C.CDLL("libamdhip64.so.7")  # the instance torch already loaded
        H.hipMemcpy.argtypes = [_vp, _vp, C.c_size_t, C.c_int]
        H.hipMemcpy.restype = C.c_int
        H.hipDeviceSynchronize.restype = C.c_int
        _LIB, _HIP = L, H
        del torch
    return _LIB


def exported_symbols():
    return ["fmmds_build", "fmmds_neighbors", "fmmds_interactions", "fmmds_free",
            "fmmds_trim", "fmmds_cache_info", "fmmds_profile_enable", "fmmds_profile_reset",
            "fmmds_profile_read", "fmmds_status_string", "fmmds_batch_create",
            "fmmds_batch_launch", "fmmds_batch_wait", "fmmds_batch_tree",
            "fmmds_batch_footprint", "fmmds_batch_bytes", "fmmds_batch_sort_items",
            "fmmds_batch_free", "fmmds_displace", "fmmds_partition", "fmmds_box_types",
            "fmmds_near_field", "fmmds_near_field_static", "fmmds_rebuild", "fmmds_build_dense",
            "fmmds_build_batch", "fmmds_free_batch"]


class DisplaceSet(C.Structure):
    _fields_ = [("xyz", _vp), ("n", _u64), ("seed", _u64), ("out_first", _u64)]


def displace(items, sigma: float, out=None, stream=None):
    """One time step of moving systems on the GPU (fmmds_displace): `items` is
    a list of (xyz tensor (n, 3) float32 CUDA, seed, out_first); each tensor is
    updated in place and, when `out` is given, also copied to rows
    out_first.. of `out`. Ordered on `stream` (default: the current stream)."""
    import torch
    arr = (DisplaceSet * len(items))()
    for k, (x, seed, first) in enumerate(items):
        if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("xyz must be a contiguous float32 CUDA tensor")
        arr[k].xyz, arr[k].n = x.data_ptr(), x.shape[0]
        arr[k].seed, arr[k].out_first = int(seed) & 0xFFFFFFFFFFFFFFFF, int(first)
    s = stream if stream is not None else torch.cuda.current_stream()
    st = _lib().fmmds_displace(arr, len(items), float(sigma),
                               None if out is None else out.data_ptr(), s.cuda_stream)
    if st != OK:
        raise FmmdsError(st, "fmmds_displace")


def batch_footprint(set_offsets, levels) -> int:
    """Device bytes a batch of this shape would allocate (host only)."""
    off = np.ascontiguousarray(set_offsets, dtype=np.uint64)
    lev = np.ascontiguousarray(levels, dtype=np.uint8)
    out = _u64()
    st = _lib().fmmds_batch_footprint(off.ctypes.data_as(_vp), lev.ctypes.data_as(_vp),
                                      int(lev.size), C.byref(out))
    if st != OK:
        raise FmmdsError(st, "fmmds_batch_footprint")
    return int(out.value)


def cache_info() -> dict:
    """Counters of the library's device-memory cache."""
    v = [_u64() for _ in range(4)]
    _lib().fmmds_cache_info(*[C.byref(x) for x in v])
    return {"hits": v[0].value, "misses": v[1].value, "miss_bytes": v[2].value,
            "cached_bytes": v[3].value}


def trim():
    """Return the library's cached device memory to HIP."""
    _lib().fmmds_trim()


def profile_enable(on: bool = True, only: str | None = None, serial: bool = False):
    """Time kernels of later builds with HIP events on the build stream: every
    kernel, or only the one named `only`. `serial`: the receivers' chain runs
    on the build stream too, so that each kernel is timed alone."""
    mode = (2 if serial else 1) if on else 0
    _lib().fmmds_profile_enable(mode, None if only is None else only.encode())


def profile_reset():
    _lib().fmmds_profile_reset()


def profile_read() -> dict:
    """{kernel: {"launches", "total_ms", "bytes"}} accumulated since the reset."""
    buf = (KernelStat * 32)()
    n = _lib().fmmds_profile_read(buf, 32)
    return {buf[i].name.decode(): {"launches": int(buf[i].launches),
                                   "total_ms": float(buf[i].total_ms),
                                   "bytes": float(buf[i].bytes)} for i in range(min(n, 32))}


def _device_to_host(ptr: int, count: int, dtype) -> np.ndarray:
    out = np.empty(count, dtype=dtype)
    if count:
        st = _HIP.hipMemcpy(out.ctypes.data_as(_vp), _vp(ptr), out.nbytes, 2)
        if st != 0:
            raise FmmdsError(ERR_DEVICE, f"hipMemcpy (hip error {st})")
    return out


class _TorchAllocator:
    """Routes the library's allocations through torch's caching allocator."""

    def __init__(self):
        import torch
        self._torch = torch
        self.alloc = ALLOC_FN(self._alloc)
        self.release = RELEASE_FN(self._release)

    def _alloc(self, ctx, nbytes, stream):
        try:
            return self._torch.cuda.caching_allocator_alloc(int(nbytes), stream=stream or 0)
        except Exception:
            return None

    def _release(self, ctx, ptr, nbytes, stream):
        self._torch.cuda.caching_allocator_delete(ptr)


_TORCH_ALLOC = None


class Tree:
    """A built tree: device tables and lists owned by libfmmds."""

    def __init__(self, handle, allocator=None, owner=None):
        self._h = handle
        self._alloc = allocator  # keeps callbacks alive as long as the tree
        self._owner = owner      # a Batch: this tree is a view into it
        t = handle.contents
        self.depth = int(t.depth)
        self.key_bits = int(t.key_bits)
        self.max_level = int(t.max_level)
        self.shared = bool(t.shared)
        self.n_src = int(t.n_src)
        self.n_recv = int(t.n_recv)

    # -- lifetime
    def free(self):
        if self._h is not None:
            if self._owner is None:
                _lib().fmmds_free(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.free()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # -- raw views (device pointers)
    def _t(self):
        if self._h is None:
            raise RuntimeError("tree already freed")
        return self._h.contents

    def level(self, s: int, l: int) -> Level:
        if not 0 <= l <= self.depth:
            raise IndexError(l)
        return (self._t().src if s == SRC else self._t().recv)[l]

    def n_boxes(self, s: int, l: int) -> int:
        return int(self.level(s, l).n)

    def _list(self, kind: int, l: int):
        off, ent, nb, ne = _vp(), _vp(), _u32(), _u64()
        f = _lib().fmmds_neighbors if kind == 2 else _lib().fmmds_interactions
        st = f(self._h, l, C.byref(off), C.byref(ent), C.byref(nb), C.byref(ne))
        if st != OK:
            raise FmmdsError(st, "fmmds_neighbors" if kind == 2 else "fmmds_interactions")
        return off.value, ent.value, nb.value, ne.value

    def neighbors(self, l: int):
        """(offsets_ptr, entries_ptr, n_recv_boxes, n_entries) of E2 at level l."""
        return self._list(2, l)

    def interactions(self, l: int):
        """(offsets_ptr, entries_ptr, n_recv_boxes, n_entries) of E4 at level l."""
        return self._list(4, l)

    # -- simulated partition and source box types (Section 3)
    def partition(self, l_par: int, n_ranks: int, stream=None):
        """Rank of every Morton index of level l_par (fmmds_partition): an
        int32 CUDA tensor of 8^l_par entries (ranks are nonnegative)."""
        import torch
        out = torch.empty(1 << (3 * l_par), dtype=torch.int32, device="cuda")
        s = stream if stream is not None else torch.cuda.current_stream()
        st = _lib().fmmds_partition(self._h, l_par, n_ranks, out.data_ptr(), s.cuda_stream)
        if st != OK:
            raise FmmdsError(st, "fmmds_partition")
        return out

    def box_types(self, l_par: int, owner, rank: int, stream=None):
        """Source box types of `rank` (fmmds_box_types): a uint8 CUDA tensor
        with levels 2..depth concatenated, and the per-level sizes."""
        import torch
        sizes = [self.n_boxes(SRC, l) for l in range(2, self.depth + 1)]
        out = torch.empty(max(sum(sizes), 1), dtype=torch.uint8, device="cuda")
        s = stream if stream is not None else torch.cuda.current_stream()
        st = _lib().fmmds_box_types(self._h, l_par, owner.data_ptr(), rank, out.data_ptr(),
                                    s.cuda_stream)
        if st != OK:
            raise FmmdsError(st, "fmmds_box_types")
        return out, sizes

    # -- near-field sum over E2 (Algorithm 2 with a Laplace kernel)
    def near_field(self, charges=None, count_pairs: bool = False, stream=None,
                   phi=None, no_alloc: bool = False):
        """phi per receiver point (original order) as a float32 CUDA tensor,
        and the number of pairs visited (if count_pairs, else None). `phi`:
        an output tensor to fill (float32, n_recv values) instead of a new
        one. `no_alloc`: fmmds_near_field_static (the library's fixed
        scratch instead of its cache)."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        if phi is None:
            phi = torch.empty(self.n_recv, dtype=torch.float32, device="cuda")
        elif phi.dtype != torch.float32 or not phi.is_cuda or phi.numel() != self.n_recv or \
                not phi.is_contiguous():
            raise ValueError("phi: contiguous float32 CUDA tensor of n_recv values")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda") if count_pairs else None
        if charges is not None:
            if charges.dtype != torch.float32 or not charges.is_cuda or \
                    charges.numel() != self.n_src:
                raise ValueError("charges: float32 CUDA tensor of n_src values")
            charges = charges.contiguous()
        fn = _lib().fmmds_near_field_static if no_alloc else _lib().fmmds_near_field
        st = fn(self._h, None if charges is None else charges.data_ptr(), phi.data_ptr(),
                None if cnt is None else cnt.data_ptr(), s.cuda_stream)
        if st != OK:
            raise FmmdsError(st, "fmmds_near_field_static" if no_alloc else "fmmds_near_field")
        return phi, (None if cnt is None else cnt)

    # -- host copies (for checks and small consumers)
    def host_perm(self, s: int) -> np.ndarray:
        _lib()
        t = self._t()
        return _device_to_host(t.src_perm if s == SRC else t.recv_perm,
                               self.n_src if s == SRC else self.n_recv, np.uint32)

    def host_sorted_xyz(self, s: int) -> np.ndarray:
        _lib()
        t = self._t()
        n = self.n_src if s == SRC else self.n_recv
        return _device_to_host(t.src_sorted_xyz if s == SRC else t.recv_sorted_xyz,
                               3 * n, np.float32).reshape(n, 3)

    def host_keys(self, s: int, l: int) -> np.ndarray:
        lv = self.level(s, l)
        return _device_to_host(lv.key, lv.n, np.uint64 if self.key_bits == 64 else np.uint32)

    def host_begin(self, s: int, l: int) -> np.ndarray:
        lv = self.level(s, l)
        return _device_to_host(lv.begin, lv.n + 1, np.uint32)

    def host_parent(self, s: int, l: int) -> np.ndarray:
        lv = self.level(s, l)
        if not lv.parent:
            raise ValueError("no parent array at level 0")
        return _device_to_host(lv.parent, lv.n, np.uint32)

    def host_child(self, s: int, l: int) -> np.ndarray:
        lv = self.level(s, l)
        if not lv.child:
            raise ValueError("no child array at the finest level")
        return _device_to_host(lv.child, lv.n + 1, np.uint32)

    def host_list(self, kind: int, l: int):
        off, ent, nb, ne = self._list(kind, l)
        return _device_to_host(off, nb + 1, np.uint32), _device_to_host(ent, ne, np.uint32)

    def host_list_rows(self, kind: int, l: int, rows) -> list:
        """Entries of selected receiver boxes only (sampled checks at full size)."""
        off_p, ent_p, nb, ne = self._list(kind, l)
        off = _device_to_host(off_p, nb + 1, np.uint32)
        out = []
        for r in rows:
            a, b = int(off[r]), int(off[r + 1])
            out.append(_device_to_host(ent_p + 4 * a, b - a, np.uint32))
        return out


def _build_options(src, recv, max_level, key_bits, cluster_s, stream, allocator):
    import torch
    for name, x in (("src", src), ("recv", recv)):
        if x is None:
            continue
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32
                and x.dim() == 2 and x.shape[1] == 3 and x.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous float32 CUDA tensor of shape (n, 3)")
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    opt = Options()
    opt.key_bits, opt.cluster_s, opt.max_level, opt.reserved = key_bits, cluster_s, max_level, 0
    opt.stream = s.cuda_stream
    keep = None
    if allocator == "torch":
        global _TORCH_ALLOC
        if _TORCH_ALLOC is None:
            _TORCH_ALLOC = _TorchAllocator()
        keep = _TORCH_ALLOC
        opt.alloc, opt.release = keep.alloc, keep.release
    elif allocator != "pool":
        raise ValueError(allocator)
    return opt, keep


def build(src, recv=None, *, max_level: int, key_bits: int = 64, cluster_s: int = 0,
          stream=None, allocator: str = "pool") -> Tree:
    """Build the FMM data structures on the GPU.

    src, recv: torch float32 CUDA tensors of shape (n, 3), contiguous; recv
    None means receivers are the sources. stream: a torch.cuda.Stream (default:
    the current stream). allocator: "pool" (the library's stream-ordered pool)
    or "torch" (torch's caching allocator)."""
    L = _lib()
    opt, keep = _build_options(src, recv, max_level, key_bits, cluster_s, stream, allocator)
    out = C.POINTER(TreeStruct)()
    st = L.fmmds_build(src.data_ptr(), src.shape[0],
                       None if recv is None else recv.data_ptr(),
                       0 if recv is None else recv.shape[0], C.byref(opt), C.byref(out))
    if st != OK:
        raise FmmdsError(st, "fmmds_build")
    return Tree(out, keep)


def build_dense(src, recv=None, *, max_level: int, key_bits: int = 64, cluster_s: int = 0,
                stream=None, allocator: str = "pool") -> Tree:
    """The same build through the dense-histogram construction
    (fmmds_build_dense, max_level <= 8); returns the tree build() returns."""
    L = _lib()
    opt, keep = _build_options(src, recv, max_level, key_bits, cluster_s, stream, allocator)
    out = C.POINTER(TreeStruct)()
    st = L.fmmds_build_dense(src.data_ptr(), src.shape[0],
                             None if recv is None else recv.data_ptr(),
                             0 if recv is None else recv.shape[0], C.byref(opt), C.byref(out))
    if st != OK:
        raise FmmdsError(st, "fmmds_build_dense")
    return Tree(out, keep)


def rebuild(prev: Tree, src, recv=None, *, in_prev_order: bool = False, key_bits: int = None,
            cluster_s: int = 0, stream=None, allocator: str = "pool") -> Tree:
    """Rebuild for moved points (fmmds_rebuild): the result equals
    build(src, recv, max_level=prev.max_level, ...) on the same positions,
    computed from prev's order (only points that changed finest box are
    sorted). in_prev_order: src / recv hold the positions in prev's sorted
    order (row k is original point prev's perm[k]) instead of original order."""
    L = _lib()
    if prev._h is None:
        raise ValueError("prev is freed")
    kb = prev.key_bits if key_bits is None else key_bits
    opt, keep = _build_options(src, recv, prev.max_level, kb, cluster_s, stream, allocator)
    if src.shape[0] != prev.n_src or (recv is None) != prev.shared or (
            recv is not None and recv.shape[0] != prev.n_recv):
        raise ValueError("point counts (or shared receivers) differ from prev")
    out = C.POINTER(TreeStruct)()
    st = L.fmmds_rebuild(prev._h, src.data_ptr(), None if recv is None else recv.data_ptr(),
                         1 if in_prev_order else 0, C.byref(opt), C.byref(out))
    if st != OK:
        raise FmmdsError(st, "fmmds_rebuild")
    return Tree(out, keep)


class Batch:
    """Batched build of many point sets (fmmds_batch_*): plan once, launch
    many times (optionally as a replayed HIP graph), read per-set trees."""

    def __init__(self, set_offsets, levels, *, stream=None, allocator: str = "pool",
                 build_from=None):
        import torch
        L = _lib()
        self._off = np.ascontiguousarray(set_offsets, dtype=np.uint64)
        self._lev = np.ascontiguousarray(levels, dtype=np.uint8)
        self.n_sets = int(self._lev.size)
        opt = Options()
        opt.key_bits, opt.cluster_s, opt.max_level, opt.reserved = 64, 0, 21, 0
        self._stream = stream
        opt.stream = stream.cuda_stream if stream is not None else None
        self._keep = None
        if allocator == "torch":
            global _TORCH_ALLOC
            if _TORCH_ALLOC is None:
                _TORCH_ALLOC = _TorchAllocator()
            self._keep = _TORCH_ALLOC
            opt.alloc, opt.release = self._keep.alloc, self._keep.release
        h = _vp()
        if build_from is None:
            st = L.fmmds_batch_create(self._off.ctypes.data_as(_vp),
                                      self._lev.ctypes.data_as(_vp), self.n_sets, C.byref(opt),
                                      C.byref(h))
            what = "fmmds_batch_create"
        else:
            if self._stream is None:
                torch.cuda.current_stream().synchronize()
            st = L.fmmds_build_batch(build_from.data_ptr(), self._off.ctypes.data_as(_vp),
                                     self._lev.ctypes.data_as(_vp), self.n_sets, C.byref(opt),
                                     C.byref(h))
            what = "fmmds_build_batch"
        if st != OK:
            raise FmmdsError(st, what)
        self._h = h
        self._torch = torch

    def launch(self, xyz, capture: bool = False):
        """Enqueue a build of the concatenated coordinates (float32 CUDA
        tensor (total, 3)). Work queued on the current stream before this call
        is complete before the batch reads xyz."""
        if self._stream is None:
            self._torch.cuda.current_stream().synchronize()
        st = _lib().fmmds_batch_launch(self._h, xyz.data_ptr(), 1 if capture else 0)
        if st != OK:
            raise FmmdsError(st, "fmmds_batch_launch")

    def wait(self):
        st = _lib().fmmds_batch_wait(self._h)
        if st != OK:
            raise FmmdsError(st, "fmmds_batch_wait")

    def tree(self, i: int) -> Tree:
        t = _lib().fmmds_batch_tree(self._h, i)
        if not t:
            raise RuntimeError("no tree: launch and wait first")
        return Tree(t, owner=self)

    @property
    def nbytes(self) -> int:
        return int(_lib().fmmds_batch_bytes(self._h))

    @property
    def sort_items(self) -> int:
        return int(_lib().fmmds_batch_sort_items(self._h))

    def free(self):
        if getattr(self, "_h", None) is not None:
            _lib().fmmds_free_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_batch(xyz, set_offsets, levels, *, stream=None, allocator: str = "pool") -> Batch:
    """The batched form in one call (fmmds_build_batch): every set of the
    concatenated coordinates `xyz` (float32 CUDA tensor (total, 3)) built and
    waited for; per-set trees from .tree(i)."""
    return Batch(set_offsets, levels, stream=stream, allocator=allocator, build_from=xyz)
