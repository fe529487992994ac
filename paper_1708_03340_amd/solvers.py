"""Truncated iterative solvers in HT arithmetic (Section 5): Algorithm (CG)
and Algorithm (richardson), driven from the host.

Every arithmetic step is one call of the C ABI: ht_apply for the operator
(Lemma (operator)), ht_truncate for every truncated sum (the sum is lazy:
the summands and coefficients go to the truncation, nothing is
materialised), ht_inner for the inner products (Definition (phi)).  The
host only keeps the scalars alpha, beta and <R, R> of the iteration.

A truncation T is given as ``Trunc(mode="fixed", rank=k)`` (every node cut
to at most k) or ``Trunc(mode="tol", eps=e)`` (relative accuracy e); the
float64 path is used throughout.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

from . import (HT_FLAG_NONFINITE, HT_PREC_FP64, HT_RANK_FIXED, HT_RANK_TOL, DeviceHT, HTError, Truncator, ht_apply,
               ht_inner)


@dataclass
class Trunc:
    mode: str = "fixed"          # "fixed" or "tol"
    rank: int = 0                # fixed: the rank every node is cut to (at most)
    eps: float = 0.0             # tol: relative accuracy
    max_rank: int = 0            # tol: optional cap


def kron_sum_operator(mats, dtype=None) -> DeviceHT:
    """The H-operator of sum_mu I (x) .. (x) M_mu (x) .. (x) I on the device
    (hierarchical ranks 2): leaf frame mu holds vec(I) and vec(M_mu) (entry
    (j, i) of column r at row j n_mu + i); at every inner node column 0 of
    the frame is the identity on the node's modes and column 1 the sum of
    the terms with one M_mu among them, so H_t[0,0,0] = H_t[1,1,0] =
    H_t[1,0,1] = 1, and the root adds the two sons' sums,
    B_D[1,0] = B_D[0,1] = 1.  ``mats`` are square torch tensors on the
    device."""
    import torch
    from . import ht_tree
    d = len(mats)
    dtype = dtype or torch.float64
    tr = ht_tree(d)
    nn = 2 * d - 1
    leaves = [None] * d
    transfer = [None] * nn
    for mu, M in enumerate(mats):
        n = int(M.shape[0])
        eye = torch.eye(n, dtype=dtype, device=M.device)
        leaves[mu] = torch.stack([eye.reshape(-1), M.to(dtype).reshape(-1)]).contiguous()
    dev = mats[0].device
    for t in range(nn):
        if int(tr["son1"][t]) < 0:
            continue
        if t == 0:
            h = torch.zeros(2, 2, dtype=torch.float64, device=dev)
            h[1, 0] = h[0, 1] = 1.0
        else:
            h = torch.zeros(2, 2, 2, dtype=dtype, device=dev)
            h[0, 0, 0] = h[1, 1, 0] = h[1, 0, 1] = 1.0
        transfer[t] = h
    return DeviceHT(d, [int(M.shape[0]) ** 2 for M in mats], [1] + [2] * (nn - 1), leaves, transfer, 0)


def compact(X: DeviceHT, ranks: Sequence[int]) -> DeviceHT:
    """X restricted to its leading ranks (the truncation writes its result at
    the rank cap, zero beyond the chosen ranks): contiguous copies of the
    leading rows of the frames and sub-blocks of the transfer tensors."""
    import torch
    from . import ht_tree
    tr = ht_tree(X.d)
    nn = 2 * X.d - 1
    r = [1] + [int(v) for v in ranks[1:]]
    leaves = [None] * X.d
    transfer = [None] * nn
    for t in range(nn):
        s1, s2 = int(tr["son1"][t]), int(tr["son2"][t])
        if s1 < 0:
            mu = int(tr["lo"][t])
            leaves[mu] = X.leaves[mu][:r[t]].contiguous()
        elif t == 0:
            transfer[t] = X.transfer[t][:r[s1], :r[s2]].contiguous()
        else:
            transfer[t] = X.transfer[t][:r[t], :r[s1], :r[s2]].contiguous()
    del torch
    return DeviceHT(X.d, X.n, r, leaves, transfer, X.scale_value())


def truncate(Xs: List[DeviceHT], coef: Sequence[float], T: Trunc) -> DeviceHT:
    """T(sum_c coef[c] Xs[c]) on the GPU, compacted to the chosen ranks;
    raises HTError when the truncation reports a NaN or Inf."""
    import torch
    nn = 2 * Xs[0].d - 1
    if T.mode == "fixed":
        tr = Truncator(Xs, list(coef), mode=HT_RANK_FIXED, ranks=[T.rank] * nn, precision=HT_PREC_FP64,
                       out_frame_dtype=torch.float64, out_transfer_dtype=torch.float64)
    else:
        tr = Truncator(Xs, list(coef), mode=HT_RANK_TOL, eps=T.eps, relative=True, max_rank=T.max_rank,
                       precision=HT_PREC_FP64, out_frame_dtype=torch.float64, out_transfer_dtype=torch.float64)
    res = tr()
    ranks = res.ranks                 # waits for the truncation
    if res.flags & HT_FLAG_NONFINITE:
        raise HTError("truncation met a NaN or Inf")
    return compact(res.out, ranks)


def inner(X: DeviceHT, Y: DeviceHT) -> float:
    return ht_inner(X, Y).value()


def _inner_me(X: DeviceHT, Y: DeviceHT):
    """<X, Y> as (m, e), the value m 2^e: the inner products of tensors
    with many modes leave the float64 range long before their ratios do."""
    return ht_inner(X, Y).mantissa_exponent()


def _ratio(a, b) -> float:
    (ma, ea), (mb, eb) = a, b
    return math.ldexp(ma / mb, ea - eb)


def _log2(a) -> float:
    m, e = a
    return math.log2(abs(m)) + e if m != 0.0 else float("-inf")


def cg(Aop: DeviceHT, B: DeviceHT, T: Trunc, eps: float, max_steps: int, history: Optional[list] = None):
    """Algorithm (CG): X_0 = B, R_0 = T(B - A X_0), D_0 = R_0; while
    sqrt(<R_j, R_j>) > eps and j < max_steps: Z = T(A D_j),
    alpha = <R_j, R_j> / <D_j, Z>, X_j+1 = T(X_j + alpha D_j),
    R_j+1 = T(R_j - alpha Z), beta = <R_j+1, R_j+1> / <R_j, R_j>,
    D_j+1 = T(beta D_j + R_j+1).  The inner products stay as m 2^e on the
    host, so alpha, beta and the stopping test are exact in range.
    Returns (X, steps)."""
    X = B
    R = truncate([B, ht_apply(Aop, X)], [1.0, -1.0], T)
    D = R
    rr = _inner_me(R, R)
    j = 0
    log2_eps = math.log2(eps) if eps > 0.0 else float("-inf")
    while rr[0] > 0.0 and 0.5 * _log2(rr) > log2_eps and j < max_steps:
        Z = truncate([ht_apply(Aop, D)], [1.0], T)
        alpha = _ratio(rr, _inner_me(D, Z))
        X = truncate([X, D], [1.0, alpha], T)
        R = truncate([R, Z], [1.0, -alpha], T)
        rr_new = _inner_me(R, R)
        beta = _ratio(rr_new, rr)
        D = truncate([D, R], [beta, 1.0], T)
        rr = rr_new
        j += 1
        if history is not None:
            history.append(dict(X=X, R=R, D=D, rr=math.ldexp(rr[0], int(min(max(rr[1], -20000), 20000))),
                                rr_log2=_log2(rr), alpha=alpha, beta=beta))
    return X, j


def richardson_step(Aop: DeviceHT, X: DeviceHT, B: DeviceHT, omega: float, T: Trunc) -> DeviceHT:
    """Algorithm (richardson): Z = T(A X); Z = T(Z - B); X <- T(X - omega Z)."""
    Z = truncate([ht_apply(Aop, X)], [1.0], T)
    Z = truncate([Z, B], [1.0, -1.0], T)
    return truncate([X, Z], [1.0, -omega], T)


def richardson(Aop: DeviceHT, X: DeviceHT, B: DeviceHT, omega: float, T: Trunc, steps: int) -> DeviceHT:
    for _ in range(steps):
        X = richardson_step(Aop, X, B, omega, T)
    return X
