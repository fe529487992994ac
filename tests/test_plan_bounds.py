"""Host-only proof that every launch of every plan stays inside its buffers
(include/ht_debug.h), for every shape the GPU tests and the benchmark use and
for edge cases (odd d, n < K, ragged sizes, non-uniform ranks, 1-3 summands)."""
import ctypes
import os

import pytest

import paper_1708_03340_amd as H
from oracle import ht_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    L = H.lib()
    P = ctypes.POINTER
    L.ht_debug_validate_truncate.argtypes = [P(H.HtDesc), ctypes.c_int32, P(H.HtTruncOpts)]
    L.ht_debug_validate_orthogonalize.argtypes = [P(H.HtDesc), ctypes.c_int32]
    L.ht_debug_validate_gramians.argtypes = [P(H.HtDesc)]
    L.ht_debug_validate_entries.argtypes = [P(H.HtDesc), ctypes.c_int64]
    for f in ("truncate", "orthogonalize", "gramians", "entries"):
        getattr(L, "ht_debug_validate_" + f).restype = ctypes.c_int
    return L


def desc(d, n, ranks, fdt=H.HT_F32, tdt=None):
    nn = 2 * d - 1
    ns = (ctypes.c_int64 * d)(*([n] * d if isinstance(n, int) else n))
    rk = (ctypes.c_int32 * nn)(*ranks)
    dd = H.HtDesc(d, ctypes.cast(ns, ctypes.POINTER(ctypes.c_int64)), ctypes.cast(rk, ctypes.POINTER(ctypes.c_int32)),
                  fdt, fdt if tdt is None else tdt, None, None, None, 0)
    dd._keep = (ns, rk)
    return dd


def uniform(d, k):
    return [1] + [k] * (2 * d - 2)


def opts(d, mode, r=None, eps=1e-6, max_rank=0, prec=H.HT_PREC_MIXED):
    nn = 2 * d - 1
    rk = (ctypes.c_int32 * nn)(*(r if r is not None else [1] * nn))
    o = H.HtTruncOpts(mode, ctypes.cast(rk, ctypes.POINTER(ctypes.c_int32)), eps, 1, max_rank, prec)
    o._keep = rk
    return o


def check(L, status):
    assert status == 0, L.ht_last_error().decode()


CASES = [
    # d, n, k (per summand), n_in, mode, r (fixed), prec
    (4, 16, 4, 2, 0, 4, 0), (4, 16, 4, 2, 0, 4, 1),
    (16, 1000, 32, 2, 0, 32, 0), (16, 1000, 32, 2, 0, 32, 1),
    (64, 10000, 64, 2, 1, 0, 1), (64, 10000, 64, 2, 0, 64, 1), (64, 10000, 64, 2, 0, 64, 0),
    (128, 100000, 64, 2, 0, 64, 1),
    (2, 9, 5, 2, 0, 3, 0), (3, 7, 3, 2, 0, 2, 1), (5, 3, 4, 2, 0, 3, 0), (7, 65, 37, 2, 1, 0, 1),
    (6, 129, 1, 3, 0, 2, 0), (9, 100, 48, 1, 0, 17, 1), (33, 4096, 48, 2, 1, 0, 1), (17, 100, 8, 2, 0, 8, 0),
]


@pytest.mark.parametrize("case", CASES)
def test_truncate_plans_in_bounds(L, case):
    d, n, k, n_in, mode, r, prec = case
    X = (H.HtDesc * n_in)(*[desc(d, n, uniform(d, k)) for _ in range(n_in)])
    o = opts(d, mode, [1] + [r] * (2 * d - 2) if mode == 0 else None, prec=prec)
    check(L, L.ht_debug_validate_truncate(X, n_in, ctypes.byref(o)))


def test_truncate_plans_nonuniform_ranks(L):
    import numpy as np
    rng = np.random.default_rng(3)
    for trial in range(40):
        d = int(rng.integers(2, 18))
        nn = 2 * d - 1
        ns = [int(x) for x in rng.integers(1, 300, size=d)]
        xs = []
        n_in = int(rng.integers(1, 4))
        for c in range(n_in):
            xs.append(desc(d, ns, [1] + [int(x) for x in rng.integers(1, 128 // n_in + 1, size=nn - 1)],
                           fdt=int(rng.integers(0, 2)), tdt=int(rng.integers(0, 2))))
        for x in xs[1:]:
            x.frame_dtype, x.transfer_dtype = xs[0].frame_dtype, xs[0].transfer_dtype
        X = (H.HtDesc * n_in)(*xs)
        mode = int(rng.integers(0, 2))
        r = [1] + [int(x) for x in rng.integers(1, 130, size=nn - 1)]
        o = opts(d, mode, r, max_rank=int(rng.integers(0, 40)), prec=int(rng.integers(0, 2)))
        check(L, L.ht_debug_validate_truncate(X, n_in, ctypes.byref(o)))


@pytest.mark.parametrize("d,n,k,prec", [(4, 16, 8, 0), (5, 70, 9, 1), (16, 1000, 64, 0), (64, 10000, 128, 1),
                                        (3, 129, 128, 0)])
def test_orthogonalize_plans_in_bounds(L, d, n, k, prec):
    check(L, L.ht_debug_validate_orthogonalize(ctypes.byref(desc(d, n, uniform(d, k), H.HT_F64)), prec))


@pytest.mark.parametrize("d,k", [(2, 3), (6, 6), (16, 64), (64, 128), (7, 1)])
def test_gramians_plans_in_bounds(L, d, k):
    check(L, L.ht_debug_validate_gramians(ctypes.byref(desc(d, 50, uniform(d, k), H.HT_F64))))


@pytest.mark.parametrize("d,n,k,m", [(7, 33, 5, 3000), (4, 16, 8, 1), (128, 100000, 64, 10000),
                                     (2, 5, 3, 17), (9, 100, 64, 70000)])
def test_entries_plans_in_bounds(L, d, n, k, m):
    check(L, L.ht_debug_validate_entries(ctypes.byref(desc(d, n, uniform(d, k))), m))


def test_validator_catches_overrun(L):
    """A descriptor whose out ranks exceed what the buffers hold must fail:
    rank 65 frames with n = 10 cannot be truncated to rank 200 in bounds,
    and the validator must refuse oversized fixed ranks instead (clamped)."""
    d = 4
    X = (H.HtDesc * 1)(desc(d, 10, uniform(d, 65)))
    o = opts(d, 0, [1] + [200] * (2 * d - 2))
    check(L, L.ht_debug_validate_truncate(X, 1, ctypes.byref(o)))   # ranks clamp to K
