"""Seeded synthetic inputs for hierarchical-SVD truncation of HT sums.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic.  Both the CPU oracle and the HIP path consume exactly the
arrays produced here, so every comparison between them starts from identical
inputs.

An HT tensor (Section 2.1 of the paper: leaf frames U_mu, transfer tensors
B_t of shape k_t x k_s1 x k_s2 and a k_t1 x k_t2 root matrix) with uniform
rank k is returned as an :class:`HTInput`:

* ``leaves[mu]``  -- n_mu x k array for mode mu (0-based), row index = i_mu;
* ``inner[j]``    -- k x k x k array for the j-th non-root inner node of the
  balanced dimension tree, nodes counted in preorder (root first, then the
  left subtree, then the right subtree);
* ``root``        -- k x k array (always float64).

The runs of the paper use "random H-tensors" (Section 4: n = 10 000,
k = 100, d up to 64); the configurations below stand in for them.  Recipes:

* i.i.d. N(0,1) entries, or
* "spectrum g": M_1(B_t) = P diag(g) W^T with P (k x k) and W (k^2 x k, k x k
  for the root) the Q factors of N(0,1) matrices, and
* orthonormal leaves: the Q factor of an N(0,1) n x k matrix.

Tensor A of configuration s uses seed 2s, its partner C uses 2s+1;
configuration 4 uses s = 1000 + b for tensor b.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "HTInput", "WORKLOADS", "make_tensor", "make_pair", "workload_pair",
    "batched_meta", "entry_indices",
]


@dataclass
class HTInput:
    d: int
    n: List[int]
    k: int
    leaves: List[np.ndarray]
    inner: List[np.ndarray]
    root: np.ndarray
    log2_scale: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def dtype(self):
        return self.leaves[0].dtype


def _orth(rng, rows, cols):
    q, _ = np.linalg.qr(rng.standard_normal((rows, cols)))
    return q


def _spectrum_tensor(rng, k, g, root=False):
    p = _orth(rng, k, k)
    w = _orth(rng, k if root else k * k, k)
    m1 = (p * g[None, :]) @ w.T
    return m1 if root else m1.reshape(k, k, k)


def make_tensor(seed, d, n, k, *, leaf="normal", spectrum=None, dtype=np.float64):
    """One HT tensor with uniform rank k on the balanced tree of dimension d.

    leaf: "normal" (i.i.d. N(0,1)) or "orth" (Q factor of N(0,1)).
    spectrum: None for i.i.d. N(0,1) transfer tensors, else the array g of
    singular values of M_1(B_t) (length k).
    Draw order: leaves by mode, inner nodes in preorder, root.
    """
    rng = np.random.default_rng(seed)
    ns = [int(n)] * d if np.isscalar(n) else [int(x) for x in n]
    leaves = []
    for mu in range(d):
        if leaf == "orth":
            u = _orth(rng, ns[mu], k)
        else:
            u = rng.standard_normal((ns[mu], k))
        leaves.append(u.astype(dtype))
    inner = []
    for _ in range(d - 2):
        if spectrum is None:
            b = rng.standard_normal((k, k, k))
        else:
            b = _spectrum_tensor(rng, k, np.asarray(spectrum, dtype=np.float64))
        inner.append(b.astype(dtype))
    if spectrum is None:
        root = rng.standard_normal((k, k))
    else:
        root = _spectrum_tensor(rng, k, np.asarray(spectrum, dtype=np.float64), root=True)
    return HTInput(d=d, n=ns, k=k, leaves=leaves, inner=inner, root=root.astype(np.float64))


def _cfg(s, d, n, k, leaf, spectrum, dtype, **trunc):
    return dict(seed_base=s, d=d, n=n, k=k, leaf=leaf, spectrum=spectrum, dtype=dtype, trunc=trunc)


# Workloads by shape: sizes, value distributions, truncation and the seed base
# (seeds 2s and 2s+1 for the two summands).
WORKLOADS = {
    "d4_n16_k4": _cfg(1, 4, 16, 4, "normal", None, np.float64, mode="fixed", rank=4),
    "d16_n1000_k32": _cfg(2, 16, 1000, 32, "orth", ("pow", 10.0, -1.0 / 8.0), np.float64, mode="fixed", rank=32),
    "d64_n1e4_k64": _cfg(3, 64, 10000, 64, "normal", ("geo", 0.9), np.float32, mode="tol", eps=1e-6, rank=64),
    "d128_n1e5_k64": _cfg(5, 128, 100000, 64, "normal", ("pow", 10.0, -1.0 / 16.0), np.float32, mode="fixed", rank=64),
}


def _spectrum(spec, k):
    if spec is None:
        return None
    i = np.arange(k, dtype=np.float64)
    if spec[0] == "geo":
        return spec[1] ** i
    if spec[0] == "pow":
        return spec[1] ** (spec[2] * i)
    raise ValueError(spec)


def make_pair(s, d, n, k, *, leaf="normal", spectrum=None, dtype=np.float64):
    """(A, C) for seed base s: seeds 2s and 2s+1."""
    g = _spectrum(spectrum, k) if isinstance(spectrum, tuple) else spectrum
    a = make_tensor(2 * s, d, n, k, leaf=leaf, spectrum=g, dtype=dtype)
    c = make_tensor(2 * s + 1, d, n, k, leaf=leaf, spectrum=g, dtype=dtype)
    return a, c


def workload_pair(name, **override):
    """Inputs of a named workload; keyword overrides (e.g. n=..., d=...)
    shrink it for quick tests while keeping the recipe."""
    c = dict(WORKLOADS[name])
    c.update(override)
    a, b = make_pair(c["seed_base"], c["d"], c["n"], c["k"], leaf=c["leaf"],
                     spectrum=c["spectrum"], dtype=c["dtype"])
    a.meta = b.meta = dict(workload=name, trunc=c["trunc"])
    return a, b


def batched_meta(count=256, seed=4):
    """Shapes of the batched workload: d ~ U{4..32}, n ~ U[100, 4096],
    k ~ U{8..48}, drawn by a meta generator."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        d = int(rng.integers(4, 33))
        n = int(rng.integers(100, 4097))
        k = int(rng.integers(8, 49))
        out.append(dict(index=b, d=d, n=n, k=k, seed_base=1000 + b))
    return out


def entry_indices(m, d, n, seed=5005):
    """m x d int32 multi-indices, each i_mu ~ U{0..n_mu-1}."""
    rng = np.random.default_rng(seed)
    ns = [int(n)] * d if np.isscalar(n) else [int(x) for x in n]
    cols = [rng.integers(0, ns[mu], size=m, dtype=np.int64) for mu in range(d)]
    return np.stack(cols, axis=1).astype(np.int32)
