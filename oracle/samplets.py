"""Samplet basis by the two-scale construction (Section 3.2).

For every cluster, from the leaves up:

* its input functions are the Dirac measures at its points (leaf) or the
  scaling distributions handed up by its two sons (eq. (refinementRelation));
* the moment matrix M has entries (x^alpha, phi_k) for all monomials of total
  degree <= q (m_q of them) and all input functions phi_k;
* M^T = Q R is a QR decomposition (eq. (QR)); the first m_q columns of Q define
  the cluster's scaling distributions, the remaining ones its samplets, which
  then have vanishing moments up to degree q (eq. (vanishingMomentsQR));
* the basis is the root's scaling distributions followed by every cluster's
  samplets (eq. (Wbasis)).

Readings where the paper is silent:

* monomials are taken in graded order (degree 0, 1, ..., q; within a degree
  the exponent tuples in descending lexicographic order) and evaluated at
  (x - c)/s, with c the centre of the cluster's bounding box and s half the
  longest side of the box (s = 1 for a degenerate box).  In exact arithmetic
  this only rescales R: centring and scaling map the monomial columns by an
  upper triangular matrix with positive diagonal.
* the QR decomposition is the Householder one: for column k the reflector maps
  x = R[k:, k] to alpha e_1 with alpha = -sign(x_0) ||x|| (sign(0) = +1); a zero
  column is left alone.  Q = H_1 H_2 ... H_m.
* a cluster with at most m_q input functions has no samplets; all its input
  functions are passed up unchanged.
* basis order: level by level, clusters left to right, the root first with its
  scaling distributions before its samplets; inside a cluster in column order
  of Q.
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import product as iproduct

import numpy as np

from .tree import ClusterTree


def monomial_exponents(d: int, q: int) -> list[tuple[int, ...]]:
    """Exponent tuples of all monomials of total degree <= q, graded order."""
    out = []
    for deg in range(q + 1):
        same = [a for a in iproduct(range(deg + 1), repeat=d) if sum(a) == deg]
        same.sort(reverse=True)
        out.extend(same)
    return out


def householder_qr(a: np.ndarray):
    """Full Householder QR a = Q R of an (n, m) matrix, n > m."""
    n, m = a.shape
    r = np.array(a, dtype=np.float64, copy=True)
    qm = np.eye(n)
    for k in range(m):
        x = r[k:, k].copy()
        nrm = np.sqrt(np.dot(x, x))
        if nrm == 0.0:
            continue
        alpha = -nrm if x[0] >= 0.0 else nrm
        v = x
        v[0] -= alpha
        vv = np.dot(v, v)
        r[k:, :] -= np.outer((2.0 / vv) * v, v @ r[k:, :])
        qm[:, k:] -= np.outer(qm[:, k:] @ v, (2.0 / vv) * v)
    return qm, r


@dataclass
class SampletBasis:
    tree: ClusterTree
    q: int
    m: int                      # number of monomials m_q
    cluster_start: np.ndarray   # (nc+1,) basis index ranges per cluster
    coef: list                  # per cluster: (n_c, size_c) coefficients over the cluster's points
    moments_r: list             # per cluster: R factor (diagnostics)

    @property
    def n(self) -> int:
        return int(self.cluster_start[-1])

    def nfun(self, c: int) -> int:
        return int(self.cluster_start[c + 1] - self.cluster_start[c])

    def dense_T(self) -> np.ndarray:
        """Dense N x N transform: row b = coefficient vector of basis function b
        over the points in tree order (the paper's omega vectors)."""
        t = self.tree
        n = int(t.size[0])
        T = np.zeros((n, n))
        for c in range(t.n_clusters):
            b0, b1 = self.cluster_start[c], self.cluster_start[c + 1]
            s = t.start[c]
            T[b0:b1, s:s + t.size[c]] = self.coef[c]
        return T

    def sparse_T(self):
        import scipy.sparse as sp
        t = self.tree
        n = int(t.size[0])
        rows, cols, vals = [], [], []
        for c in range(t.n_clusters):
            b0, b1 = self.cluster_start[c], self.cluster_start[c + 1]
            if b1 == b0:
                continue
            s, sz = t.start[c], t.size[c]
            rr, cc = np.meshgrid(np.arange(b0, b1), np.arange(s, s + sz), indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(np.asarray(self.coef[c]).ravel())
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(n, n))

    def support_cluster_of(self) -> np.ndarray:
        """Cluster owning each basis index."""
        nc = self.tree.n_clusters
        return np.repeat(np.arange(nc), np.diff(self.cluster_start))


def monomials_at(p: np.ndarray, lo: np.ndarray, hi: np.ndarray, exps) -> np.ndarray:
    """(npts, m) values of the centred, scaled monomials."""
    c = 0.5 * (lo + hi)
    s = 0.5 * np.max(hi - lo)
    if s == 0.0:
        s = 1.0
    y = (p - c) / s
    v = np.ones((p.shape[0], len(exps)))
    for k, a in enumerate(exps):
        for ax, e in enumerate(a):
            for _ in range(e):
                v[:, k] *= y[:, ax]
    return v


def build_samplets(tree: ClusterTree, q: int) -> SampletBasis:
    d = tree.points.shape[1]
    exps = monomial_exponents(d, q)
    m = len(exps)
    nc = tree.n_clusters
    scal = [None] * nc      # scaling distributions handed up: (k, size) over cluster points
    sam = [None] * nc       # samplets: (k, size)
    rs = [None] * nc
    for c in range(nc - 1, -1, -1):            # sons have larger numbers than fathers
        sz = int(tree.size[c])
        if tree.is_leaf(c):
            phi = np.eye(sz)
        else:
            a, b = tree.sons[c]
            na, nb = int(tree.size[a]), int(tree.size[b])
            fa, fb = scal[a], scal[b]
            phi = np.zeros((fa.shape[0] + fb.shape[0], sz))
            phi[:fa.shape[0], :na] = fa
            phi[fa.shape[0]:, na:na + nb] = fb
        nin = phi.shape[0]
        if nin <= m:
            scal[c] = phi
            sam[c] = np.zeros((0, sz))
            continue
        v = monomials_at(tree.cluster_points(c), tree.lo[c], tree.hi[c], exps)
        mt = phi @ v                                # M^T, (nin, m)
        qm, r = householder_qr(mt)
        newf = qm.T @ phi                           # rows: new functions over the cluster points
        scal[c] = newf[:m]
        sam[c] = newf[m:]
        rs[c] = r
    coef = []
    counts = np.zeros(nc, dtype=np.int64)
    for c in range(nc):
        if c == 0:
            blk = np.vstack([scal[0], sam[0]])
        else:
            blk = sam[c]
        coef.append(blk)
        counts[c] = blk.shape[0]
    cs = np.zeros(nc + 1, dtype=np.int64)
    cs[1:] = np.cumsum(counts)
    assert cs[-1] == tree.size[0]
    return SampletBasis(tree, q, m, cs, coef, rs)
