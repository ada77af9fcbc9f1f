"""Compression pattern (Section 3.3, Theorem (S-compression), eq. (cutoff); Section 5 a-posteriori pattern).

A block (nu, nu') of K^Sigma is dropped when the clusters are eta-admissible,
dist(nu, nu') >= eta * max(diam(nu), diam(nu')).  Clusters of different
levels are paired too (the block cluster tree is T x T).  The pattern S is the
set of all basis pairs whose supporting clusters are not admissible.

Reading: diam and dist are those of the clusters' bounding boxes (the Lemma on
bounding boxes in Section 3.2); diam = Euclidean length of the box diagonal,
dist = Euclidean norm of the componentwise gap max(0, lo' - hi, lo - hi').
Both are evaluated in this order: squares summed over axes 0, 1, ..., then one
square root; the bound is eta times the larger diameter; the pair is kept iff
dist < bound.

The a-posteriori pattern (numerical results, Section 5) additionally drops the
entries below a threshold tau in modulus.  Reading: the decision for (i, j) and
(j, i) is taken once on the entry with i <= j, and the diagonal is always kept.
"""
from __future__ import annotations

import numpy as np

from .samplets import SampletBasis
from .tree import ClusterTree


def _norm_rows(v: np.ndarray) -> np.ndarray:
    acc = v[..., 0] * v[..., 0]
    for a in range(1, v.shape[-1]):
        acc = acc + v[..., a] * v[..., a]
    return np.sqrt(acc)


def diameters(tree: ClusterTree) -> np.ndarray:
    return _norm_rows(tree.hi - tree.lo)


def block_row(tree: ClusterTree, eta: float, c: int, diam: np.ndarray | None = None) -> np.ndarray:
    """The sorted clusters nu' with (c, nu') kept: eq. (cutoff) against every cluster."""
    if diam is None:
        diam = diameters(tree)
    gap = np.maximum(0.0, np.maximum(tree.lo - tree.hi[c], tree.lo[c] - tree.hi))
    dist = _norm_rows(gap)
    bound = eta * np.maximum(diam[c], diam)
    return np.nonzero(dist < bound)[0].astype(np.int64)


def block_rows(tree: ClusterTree, eta: float, clusters, diam: np.ndarray | None = None,
               chunk: int = 256) -> dict:
    """block_row for each listed cluster, evaluated for `chunk` clusters at a time with
    the same operations in the same order (an (chunk x n_clusters) array per step)."""
    if diam is None:
        diam = diameters(tree)
    cl = np.unique(np.asarray(clusters, dtype=np.int64))
    out = {}
    for s in range(0, len(cl), chunk):
        c = cl[s:s + chunk]
        gap = np.maximum(0.0, np.maximum(tree.lo[None, :, :] - tree.hi[c][:, None, :],
                                         tree.lo[c][:, None, :] - tree.hi[None, :, :]))
        dist = _norm_rows(gap)
        bound = eta * np.maximum(diam[c][:, None], diam[None, :])
        keep = dist < bound
        for t, cc in enumerate(c):
            out[int(cc)] = np.nonzero(keep[t])[0].astype(np.int64)
    return out


def block_pattern(tree: ClusterTree, eta: float) -> list[np.ndarray]:
    """For each cluster nu, the sorted array of clusters nu' with (nu, nu') kept.

    Brute force over all cluster pairs (the definition, no tree traversal).
    """
    diam = diameters(tree)
    return [block_row(tree, eta, c, diam) for c in range(tree.n_clusters)]


def block_csr(blocks: list[np.ndarray]):
    """Cluster-level CSR (row_ptr int64, col int32) of a block pattern."""
    rp = np.zeros(len(blocks) + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(b) for b in blocks])
    col = np.concatenate(blocks).astype(np.int32) if blocks else np.zeros(0, np.int32)
    return rp, col


def entry_csr(basis: SampletBasis, blocks: list[np.ndarray]):
    """Entry-level CSR (row_ptr int64, col int32) of the pattern of basis pairs."""
    cs = basis.cluster_start
    nc = len(blocks)
    n = basis.n
    row_cols = []
    for c in range(nc):
        cols = np.concatenate([np.arange(cs[b], cs[b + 1]) for b in blocks[c]]) if len(blocks[c]) else np.zeros(0, np.int64)
        for _ in range(cs[c], cs[c + 1]):
            row_cols.append(cols)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in row_cols])
    col = np.concatenate(row_cols).astype(np.int32) if n else np.zeros(0, np.int32)
    return rp, col


def dense_mask(rp: np.ndarray, col: np.ndarray, n: int) -> np.ndarray:
    mask = np.zeros((n, n), dtype=bool)
    rows = np.repeat(np.arange(n), np.diff(rp))
    mask[rows, col] = True
    return mask


def threshold_mask(mask: np.ndarray, values: np.ndarray, tau: float) -> np.ndarray:
    """A-posteriori pattern: drop |v_ij| < tau, decided on the upper triangle, keep the diagonal."""
    n = mask.shape[0]
    upper = np.triu(np.abs(values), 1)
    drop_u = np.triu(upper < tau, 1)
    drop = drop_u | drop_u.T
    out = mask & ~drop
    out[np.arange(n), np.arange(n)] = mask[np.arange(n), np.arange(n)]
    return out


def csr_from_mask(mask: np.ndarray):
    n = mask.shape[0]
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum(mask.sum(axis=1))
    col = np.nonzero(mask)[1].astype(np.int32)
    return rp, col
