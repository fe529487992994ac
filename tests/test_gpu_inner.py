"""Inner product by Definition (phi) / Lemma (phi) and norms of lazy sums
(Section 3.2; the norm through the orthogonalised sum of Section 3.4) on the
GPU, called through the C ABI, against the oracle.

Gates: an inner product <X, Y> may cancel, so its error is measured against
||X|| ||Y|| (float64 path: 1e-12 for N(0,1) data, 1e-10 at the full-size
workloads); <X, X> and norms have no cancellation (relative 1e-12); a
difference norm ||A - B|| is relative to itself (1e-10).
"""
import sys

import numpy as np
import pytest

import htsynth as S
from oracle import ht_oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1708_03340_amd as H
    H.lib()
    return H


def rand_ht(rng, d, n, k, dtype=np.float64):
    tr = O.Tree(d)
    ns = [int(n)] * d if np.isscalar(n) else list(n)
    U = [rng.standard_normal((ns[mu], k)).astype(dtype) for mu in range(d)]
    B = {}
    for t in range(tr.n_nodes):
        if not tr.is_leaf(t):
            B[t] = rng.standard_normal((k, k) if t == 0 else (k, k, k)).astype(dtype)
            if t == 0:
                B[t] = B[t].astype(np.float64)
    return O.HT(tr, U, B, 0)


def dev_of(H, X, fdt, tdt):
    return H.DeviceHT.from_arrays(X.d, X.U, [X.B.get(t) for t in range(X.tree.n_nodes)], X.log2_scale,
                                  frame_dtype=fdt, transfer_dtype=tdt)


def nrm(X):
    m, e = O.norm_log2(X)
    return float(np.ldexp(m, e))


def check_inner(H, X, Y, fdt, tdt, tol, label):
    import torch
    g = H.ht_inner(dev_of(H, X, fdt, tdt), dev_of(H, Y, fdt, tdt))
    torch.cuda.synchronize()
    got = g.value()
    ref = O.inner(X, Y)
    scale = nrm(X) * nrm(Y)
    err = abs(got - ref) / scale
    say(f"  {label}: <X,Y> gpu {got:.6e} oracle {ref:.6e}, |diff| / (||X|| ||Y||) = {err:.3e}, "
        f"flags {int(g.flags_dev.item())}")
    assert err <= tol
    return got


def test_inner_small_uneven_ranks(H):
    import torch
    say("case inner d=4 n=16, ranks 4 and 3")
    rng = np.random.default_rng(11)
    X, Y = rand_ht(rng, 4, 16, 4), rand_ht(rng, 4, 16, 3)
    check_inner(H, X, Y, torch.float64, torch.float64, 1e-13, "d=4")
    gx = H.ht_inner(dev_of(H, X, torch.float64, torch.float64), dev_of(H, X, torch.float64, torch.float64))
    torch.cuda.synchronize()
    rel = abs(gx.value() - O.inner(X, X)) / O.inner(X, X)
    say(f"  <X,X> relative error {rel:.3e}")
    assert rel <= 1e-13


@pytest.mark.parametrize("d", [2, 3, 7])
def test_inner_ragged_modes_and_dtypes(H, d):
    """Modes of different sizes, float32 X against float64 Y (the oracle sees
    the same float32-rounded values)."""
    import torch
    say(f"case inner d={d} ragged n, float32 x float64")
    rng = np.random.default_rng(100 + d)
    ns = [int(v) for v in rng.integers(3, 90, size=d)]
    X = rand_ht(rng, d, ns, 6, np.float32)
    Y = rand_ht(rng, d, ns, 9)
    import paper_1708_03340_amd as HH
    gx = HH.DeviceHT.from_arrays(d, X.U, [X.B.get(t) for t in range(X.tree.n_nodes)], 0,
                                 frame_dtype=torch.float32, transfer_dtype=torch.float32)
    gy = HH.DeviceHT.from_arrays(d, Y.U, [Y.B.get(t) for t in range(Y.tree.n_nodes)], 0,
                                 frame_dtype=torch.float64, transfer_dtype=torch.float64)
    g = H.ht_inner(gx, gy)
    torch.cuda.synchronize()
    ref = O.inner(X, Y)
    err = abs(g.value() - ref) / (nrm(X) * nrm(Y))
    say(f"  |diff| / (||X|| ||Y||) = {err:.3e}")
    assert err <= 1e-13


def test_inner_and_norms_d16_workload(H):
    """The d=16, n=1000, k=32 pair: <A, C>, ||A + C||, and the difference
    norm between A + C and its rank-32 truncation (a three-summand lazy sum)."""
    import torch
    say("case inner / norms d16_n1000_k32")
    a, c = S.workload_pair("d16_n1000_k32")
    A, C = O.from_input(a), O.from_input(c)
    f64 = torch.float64
    check_inner(H, A, C, f64, f64, 1e-12, "<A, C>")
    da, dc = H.DeviceHT.from_input(a), H.DeviceHT.from_input(c)
    X = O.add(A, C)
    n_gpu = H.ht_norm([da, dc]).value()
    n_ref = nrm(X)
    say(f"  ||A + C|| gpu {n_gpu:.12e} oracle {n_ref:.12e}")
    assert abs(n_gpu - n_ref) / n_ref <= 1e-12
    T, _ = O.truncate(X, mode="fixed", ranks=[32] * 31)
    dt = dev_of(H, T, f64, f64)
    dn_gpu = H.ht_norm([da, dc, dt], [1.0, 1.0, -1.0]).value()
    m, e = O.diff_norm_log2(X, T)
    dn_ref = float(np.ldexp(m, e))
    rel = abs(dn_gpu - dn_ref) / dn_ref
    say(f"  ||A + C - T(A + C)|| gpu {dn_gpu:.12e} oracle {dn_ref:.12e} (relative {dn_ref / n_ref:.2e}), "
        f"rel err {rel:.3e}")
    assert rel <= 1e-10
    z = H.ht_norm([da, da], [1.0, -1.0]).value()
    mz, ez = O.diff_norm_log2(A, A)
    say(f"  ||A - A|| gpu {z:.3e}, oracle {np.ldexp(mz, ez):.3e} (||A|| = {nrm(A):.3e})")
    assert z <= 1e-12 * nrm(A)


def test_inner_d64_full_size(H):
    """<A, C> and <A, A> of the d=64, n=1e4, k=64 pair (float32 frames)."""
    import torch
    say("case inner d64_n1e4_k64")
    a, c = S.workload_pair("d64_n1e4_k64")
    A, C = O.from_input(a), O.from_input(c)
    da, dc = H.DeviceHT.from_input(a), H.DeviceHT.from_input(c)
    g = H.ht_inner(da, dc)
    gaa = H.ht_inner(da, da)
    torch.cuda.synchronize()
    ref = O.inner(A, C)
    na, nc = nrm(A), nrm(C)
    err = abs(g.value() - ref) / (na * nc)
    raa = abs(gaa.value() - na * na) / (na * na)
    say(f"  <A,C> gpu {g.value():.6e} oracle {ref:.6e}, |diff| / (||A|| ||C||) = {err:.3e}; "
        f"<A,A> vs ||A||^2 {raa:.3e}")
    assert err <= 1e-10
    assert raa <= 1e-12


def test_inner_beyond_float64_range(H):
    """d=128 with N(0,1) data: <A, A> is far outside the float64 range; the
    mantissa/exponent result must equal ||A||^2 from the oracle's scaled norm."""
    import torch
    say("case inner d=128, n=300, k=6 (beyond the float64 range)")
    rng = np.random.default_rng(7)
    A = rand_ht(rng, 128, 300, 6)
    A.log2_scale = 900
    da = dev_of(H, A, torch.float64, torch.float64)
    g = H.ht_inner(da, da)
    nm = H.ht_norm([da])
    torch.cuda.synchronize()
    m_i, e_i = g.mantissa_exponent()
    m_n, e_n = O.norm_log2(A)
    ratio = np.ldexp(m_i / (m_n * m_n), e_i - 2 * e_n)
    gm, ge = nm.mantissa_exponent()
    rn = np.ldexp(gm / m_n, ge - e_n)
    say(f"  log2 <A,A> = {np.log2(m_i) + e_i:.6f}, <A,A> / ||A||^2 = {ratio:.15f}, "
        f"gpu norm / oracle norm = {rn:.15f}")
    assert abs(ratio - 1.0) <= 1e-12
    assert abs(rn - 1.0) <= 1e-12
