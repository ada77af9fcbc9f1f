"""Samplet-compressed kernel matrix (Section 3.3).

K^Sigma = [(k, sigma_b (x) sigma_b')] = T K T^T, where T holds the samplet
coefficient vectors as rows (Remark on coefficient vectors, Section 3.2) and
K = [k(x_i, x_j)] with the points in tree order.  K^eta keeps the entries of
K^Sigma on the compression pattern and sets the rest to zero (Theorem
(S-compression)).

Every experiment of the paper scales the kernel by 1/N (eq. (expKernel2) and
the sentence after it), which bounds the largest eigenvalue of K by its trace,
tr K = k(0) = 1.  ``scale`` carries that factor.

The paper assembles K^eta in O(N log N) with an H^2 / fast multipole method
that it only cites; here the entries are the exact definition evaluated with
O(N^2) kernel evaluations.
"""
from __future__ import annotations

import numpy as np

from .kernels import dmatern_dl, matern, pairwise_dist
from .samplets import SampletBasis


def kernel_fn(p: int, ell: float, deriv: bool):
    if deriv:
        return lambda r: dmatern_dl(r, p, ell)
    return lambda r: matern(r, p, ell)


def kernel_matrix(basis: SampletBasis, p: int, ell: float, scale: float, deriv: bool = False) -> np.ndarray:
    """K (points in tree order) times ``scale``."""
    t = basis.tree
    x = t.points[t.perm]
    return kernel_fn(p, ell, deriv)(pairwise_dist(x, x)) * scale


def compress_dense(basis: SampletBasis, p: int, ell: float, scale: float, deriv: bool = False) -> np.ndarray:
    """Dense K^Sigma = T K T^T (small N only)."""
    T = basis.dense_T()
    K = kernel_matrix(basis, p, ell, scale, deriv)
    return T @ K @ T.T


def compress_rows(basis: SampletBasis, rows: np.ndarray, p: int, ell: float, scale: float,
                  deriv: bool = False, T=None, chunk: int = 1 << 24, use_c: bool = False) -> np.ndarray:
    """Rows ``rows`` of K^Sigma (dense, len(rows) x N) without forming K.

    Row b of K^Sigma is T (K omega_b): first the kernel is applied to the
    coefficient vector omega_b (only the points of b's cluster contribute),
    then the samplet transform T maps the result to samplet coordinates.
    ``use_c`` evaluates the kernel sums with the oracle's plain C helper, the rows
    owned by one cluster together (the same sums, each in the same order).
    """
    t = basis.tree
    n = int(t.size[0])
    x = t.points[t.perm]
    if T is None:
        T = basis.sparse_T()
    owner = basis.support_cluster_of()
    f = kernel_fn(p, ell, deriv)
    out = np.zeros((len(rows), n))
    if use_c:
        from . import native
        rows = np.asarray(rows)
        for c in np.unique(owner[rows]):
            ks = np.nonzero(owner[rows] == c)[0]
            s, sz = int(t.start[c]), int(t.size[c])
            W = np.asarray(basis.coef[c])[rows[ks] - basis.cluster_start[c]].T      # sz x len(ks)
            acc = native.kernel_apply_multi(x, x[s:s + sz], W, p, ell, scale, deriv)
            for q, k in enumerate(ks):
                out[k] = T @ acc[:, q]
        return out
    for k, b in enumerate(rows):
        c = owner[b]
        s, sz = int(t.start[c]), int(t.size[c])
        w = np.asarray(basis.coef[c])[b - basis.cluster_start[c]]
        if use_c:
            from . import native
            acc = native.kernel_apply(x, x[s:s + sz], w, p, ell, scale, deriv)
        else:
            acc = np.zeros(n)
            step = max(1, chunk // max(sz, 1))
            for j0 in range(0, n, step):
                j1 = min(n, j0 + step)
                kk = f(pairwise_dist(x[j0:j1], x[s:s + sz])) * scale   # (j1-j0, sz)
                acc[j0:j1] = kk @ w
        out[k] = T @ acc
    return out
