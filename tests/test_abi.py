"""Host-side checks of the C ABI: the library builds, loads, exports every
function include/fmmds.h declares, and rejects bad arguments before any
device work (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmmds.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fmmds_[a-z_]+)\s*\(", text)) -
                  {"fmmds_alloc_fn", "fmmds_release_fn"})


@pytest.fixture(scope="module")
def lib():
    import paper_1301_1704_amd as F
    if not os.path.exists(F.LIB_PATH):
        from paper_1301_1704_amd import _compile
        _compile.build()
    return F._lib()


def test_header_declares_the_four_calls():
    fns = declared_functions()
    for f in ("fmmds_build", "fmmds_neighbors", "fmmds_interactions", "fmmds_free"):
        assert f in fns


def test_every_declared_symbol_is_exported(lib):
    for f in declared_functions():
        assert hasattr(lib, f), f


def test_binding_names_match_header():
    import paper_1301_1704_amd as F
    assert sorted(F.exported_symbols()) == declared_functions()


def test_status_strings(lib):
    for s in range(8):
        assert lib.fmmds_status_string(s)
    assert lib.fmmds_status_string(2) == b"coordinate outside [0, 1)"


def _opt(F, key_bits=64, max_level=5, cluster_s=0, reserved=0):
    o = F.Options()
    o.key_bits, o.max_level, o.cluster_s, o.reserved = key_bits, max_level, cluster_s, reserved
    return o


@pytest.mark.parametrize("kw", [dict(key_bits=16), dict(key_bits=32, max_level=11),
                                dict(max_level=1), dict(max_level=22), dict(reserved=1)])
def test_bad_options_rejected_on_host(lib, kw):
    import paper_1301_1704_amd as F
    out = C.POINTER(F.TreeStruct)()
    fake = C.c_void_p(0x1000)  # never dereferenced: options are checked first
    st = lib.fmmds_build(fake, 10, None, 0, C.byref(_opt(F, **kw)), C.byref(out))
    assert st == F.ERR_ARG and not out


def test_null_and_empty_inputs_rejected(lib):
    import paper_1301_1704_amd as F
    out = C.POINTER(F.TreeStruct)()
    assert lib.fmmds_build(None, 10, None, 0, C.byref(_opt(F)), C.byref(out)) == F.ERR_ARG
    assert lib.fmmds_build(C.c_void_p(0x1000), 0, None, 0, C.byref(_opt(F)),
                           C.byref(out)) == F.ERR_ARG
    assert lib.fmmds_build(C.c_void_p(0x1000), 0xFFFFFFFF, None, 0, C.byref(_opt(F)),
                           C.byref(out)) == F.ERR_ARG
    assert lib.fmmds_build(C.c_void_p(0x1000), 10, C.c_void_p(0x2000), 0, C.byref(_opt(F)),
                           C.byref(out)) == F.ERR_ARG
    assert lib.fmmds_build(C.c_void_p(0x1000), 10, None, 0, None, C.byref(out)) == F.ERR_ARG


def test_queries_on_null_tree(lib):
    import paper_1301_1704_amd as F
    off, ent, nb, ne = C.c_void_p(), C.c_void_p(), C.c_uint32(), C.c_uint64()
    assert lib.fmmds_neighbors(None, 2, C.byref(off), C.byref(ent), C.byref(nb),
                               C.byref(ne)) == F.ERR_ARG
    assert lib.fmmds_interactions(None, 2, C.byref(off), C.byref(ent), C.byref(nb),
                                  C.byref(ne)) == F.ERR_ARG
    lib.fmmds_free(None)


def test_rebuild_arguments_rejected_on_host(lib):
    """fmmds_rebuild checks its arguments against the previous tree before
    any device work (the tree here is a host struct with fake pointers)."""
    import paper_1301_1704_amd as F
    t = F.TreeStruct()
    t.depth, t.key_bits, t.max_level, t.shared, t.n_src, t.n_recv = 5, 64, 5, 1, 10, 10
    fake = C.c_void_p(0x1000)
    t.src_perm = t.recv_perm = t.src_sorted_xyz = t.recv_sorted_xyz = 0x1000
    out = C.POINTER(F.TreeStruct)()
    ok = _opt(F, max_level=5)
    assert lib.fmmds_rebuild(None, fake, None, 0, C.byref(ok), C.byref(out)) == F.ERR_ARG
    assert lib.fmmds_rebuild(C.byref(t), fake, None, 0, None, C.byref(out)) == F.ERR_ARG
    assert lib.fmmds_rebuild(C.byref(t), fake, None, 2, C.byref(ok), C.byref(out)) == F.ERR_ARG
    assert lib.fmmds_rebuild(C.byref(t), fake, fake, 0, C.byref(ok), C.byref(out)) == F.ERR_ARG
    assert lib.fmmds_rebuild(C.byref(t), fake, None, 0, C.byref(_opt(F, max_level=6)),
                             C.byref(out)) == F.ERR_ARG
    t.src_perm = None
    assert lib.fmmds_rebuild(C.byref(t), fake, None, 0, C.byref(ok), C.byref(out)) == F.ERR_ARG
    assert not out


def test_batch_footprint_plans_on_host(lib):
    """fmmds_batch_footprint runs the batch plan and layout on the host: it
    grows with the points and the levels, and rejects bad shapes, among them
    2^31 sets or more (set ids are 31 bits in the sort's tile tables; checked
    before the offsets are read)."""
    import numpy as np
    import paper_1301_1704_amd as F

    def footprint(off, lev, n_sets=None):
        off = np.ascontiguousarray(off, dtype=np.uint64)
        lev = np.ascontiguousarray(lev, dtype=np.uint8)
        b = C.c_uint64(0)
        st = lib.fmmds_batch_footprint(off.ctypes.data_as(C.c_void_p),
                                       lev.ctypes.data_as(C.c_void_p),
                                       len(lev) if n_sets is None else n_sets, C.byref(b))
        return st, b.value

    st1, b1 = footprint([0, 1000, 3000], [3, 4])
    st2, b2 = footprint([0, 1000, 300000], [3, 6])
    assert st1 == F.OK and st2 == F.OK and 0 < b1 < b2
    assert footprint([0, 1000, 1000], [3, 4])[0] == F.ERR_ARG    # an empty set
    assert footprint([0, 1000], [1])[0] == F.ERR_ARG             # level below 2
    assert footprint([0, 1000], [3], n_sets=2 ** 31)[0] == F.ERR_ARG
    assert footprint([0, 1000], [3], n_sets=0)[0] == F.ERR_ARG
