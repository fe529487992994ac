"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/ht.h declares, builds the same tree as the oracle, and
rejects bad arguments before enqueuing anything."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1708_03340_amd as H
from oracle import ht_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ht.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ht_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(H.LIB_PATH):
        pytest.fail("libht.so is not built (run __graft_entry__.build())")
    return H.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(H.EXPORTS)


def test_version_and_status_strings(L):
    assert L.ht_version() == 1
    for s in range(6):
        assert L.ht_status_string(s)


@pytest.mark.parametrize("d", [2, 3, 4, 5, 7, 8, 13, 16, 33, 64, 100, 128])
def test_tree_matches_oracle(L, d):
    t = H.ht_tree(d)
    tr = O.Tree(d)
    for node in range(2 * d - 1):
        assert t["lo"][node] == tr.lo[node] - 1 and t["hi"][node] == tr.hi[node] - 1
        assert t["depth"][node] == tr.depth[node]
        assert t["height"][node] == tr.height[node]
        assert t["parent"][node] == tr.parent[node]
        sons = tr.sons[node]
        if sons is None:
            assert t["son1"][node] == -1 and t["son2"][node] == -1
        else:
            assert (t["son1"][node], t["son2"][node]) == sons


def _host_desc(d, n, k, fdt=H.HT_F32):
    nn = 2 * d - 1
    ns = (ctypes.c_int64 * d)(*([n] * d))
    rk = (ctypes.c_int32 * nn)(*([1] + [k] * (nn - 1)))
    desc = H.HtDesc(d, ctypes.cast(ns, ctypes.POINTER(ctypes.c_int64)),
                    ctypes.cast(rk, ctypes.POINTER(ctypes.c_int32)), fdt, fdt, None, None, None, 0)
    desc._keep = (ns, rk)
    return desc


def _opts(mode, d, r=0, eps=0.0, prec=H.HT_PREC_MIXED):
    nn = 2 * d - 1
    rk = (ctypes.c_int32 * nn)(*([1] + [r] * (nn - 1)))
    o = H.HtTruncOpts(mode, ctypes.cast(rk, ctypes.POINTER(ctypes.c_int32)), eps, 1, 0, prec)
    o._keep = rk
    return o


def test_workspace_queries_host_only(L):
    X = (H.HtDesc * 2)(_host_desc(64, 10000, 64), _host_desc(64, 10000, 64))
    keep = [X[0], X[1]]
    o = _opts(H.HT_RANK_TOL, 64, eps=1e-6)
    nb = ctypes.c_size_t(0)
    assert L.ht_truncate_workspace(None, X, 2, ctypes.byref(o), ctypes.byref(nb)) == 0
    assert 1 << 30 < nb.value < 16 << 30          # a few GiB at d=64, n=1e4, K=128
    x1 = _host_desc(16, 1000, 32, H.HT_F64)
    assert L.ht_orthogonalize_workspace(None, ctypes.byref(x1), 0, ctypes.byref(nb)) == 0 and nb.value > 0
    assert L.ht_gramians_workspace(None, ctypes.byref(x1), ctypes.byref(nb)) == 0 and nb.value > 0
    assert L.ht_entries_workspace(None, ctypes.byref(x1), 1000, ctypes.byref(nb)) == 0 and nb.value > 0
    del keep


def test_bad_arguments_rejected(L):
    nb = ctypes.c_size_t(0)
    o = _opts(H.HT_RANK_FIXED, 4, r=2)
    x = _host_desc(4, 16, 4)
    # d < 2
    bad = _host_desc(1, 16, 4)
    assert L.ht_truncate_workspace(None, ctypes.byref(bad), 1, ctypes.byref(o), ctypes.byref(nb)) == 1
    # sum rank above 128
    big = (H.HtDesc * 2)(_host_desc(4, 1000, 65), _host_desc(4, 1000, 65))
    assert L.ht_truncate_workspace(None, big, 2, ctypes.byref(o), ctypes.byref(nb)) == 5
    # too many summands / none
    assert L.ht_truncate_workspace(None, ctypes.byref(x), 0, ctypes.byref(o), ctypes.byref(nb)) == 1
    # mismatched n between summands
    mm = (H.HtDesc * 2)(_host_desc(4, 16, 4), _host_desc(4, 17, 4))
    assert L.ht_truncate_workspace(None, mm, 2, ctypes.byref(o), ctypes.byref(nb)) == 2
    # bad mode / precision / negative eps
    for oo in (H.HtTruncOpts(7, None, 0.0, 1, 0, 0), H.HtTruncOpts(0, None, 0.0, 1, 0, 0),
               H.HtTruncOpts(1, None, -1.0, 1, 0, 0), H.HtTruncOpts(1, None, 0.1, 1, 0, 9)):
        assert L.ht_truncate_workspace(None, ctypes.byref(x), 1, ctypes.byref(oo), ctypes.byref(nb)) == 1
    assert b"eps" in L.ht_last_error() or b"precision" in L.ht_last_error()
    # a missing context is an error for the enqueueing calls
    assert L.ht_truncate(None, ctypes.byref(x), None, 1, ctypes.byref(o), None, None, None, None, None,
                         None, 0, None) == 1
    assert L.ht_tree(1, None, None, None, None, None, None, None) == 1


def test_null_and_negative_summand_counts_rejected(L):
    """X == NULL with n_in > 0, and n_in < 0, are argument errors (no
    dereference, no exception across the C boundary)."""
    nb = ctypes.c_size_t(0)
    o = _opts(H.HT_RANK_FIXED, 4, r=2)
    assert L.ht_truncate_workspace(None, None, 2, ctypes.byref(o), ctypes.byref(nb)) == 1
    assert b"X is NULL" in L.ht_last_error()
    x = _host_desc(4, 16, 4)
    assert L.ht_truncate_workspace(None, ctypes.byref(x), -3, ctypes.byref(o), ctypes.byref(nb)) == 1
    assert L.ht_truncate_workspace(None, ctypes.byref(x), 9, ctypes.byref(o), ctypes.byref(nb)) == 1


@pytest.mark.parametrize("d,n,k,mode,prec", [(4, 16, 4, 0, 0), (13, 300, 20, 1, 1), (64, 10000, 64, 1, 1),
                                             (64, 10000, 64, 0, 0)])
def test_plan_cache_key_repeats(L, d, n, k, mode, prec):
    """Two builds of the same ht_truncate call give byte-identical plan-cache
    keys, so a repeated call reuses its launch tables (no upload, no host
    synchronisation); a different call gives a different key."""
    L.ht_debug_plan_key_repeats.argtypes = [ctypes.POINTER(H.HtDesc), ctypes.c_int32,
                                            ctypes.POINTER(H.HtTruncOpts), ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_uint64)]
    L.ht_debug_plan_key_repeats.restype = ctypes.c_int
    X = (H.HtDesc * 2)(_host_desc(d, n, k), _host_desc(d, n, k))
    o = _opts(mode, d, r=k, eps=1e-6, prec=prec)
    eq, h1 = ctypes.c_int32(0), ctypes.c_uint64(0)
    assert L.ht_debug_plan_key_repeats(X, 2, ctypes.byref(o), ctypes.byref(eq), ctypes.byref(h1)) == 0
    assert eq.value == 1
    o2 = _opts(mode, d, r=max(1, k - 1), eps=1e-5, prec=prec)
    h2 = ctypes.c_uint64(0)
    assert L.ht_debug_plan_key_repeats(X, 2, ctypes.byref(o2), ctypes.byref(eq), ctypes.byref(h2)) == 0
    assert eq.value == 1 and h2.value != h1.value
