"""Binary cluster tree (Section 3.2, Definition of a cluster tree; Lemma on bounding boxes).

The paper requires a binary tree whose non-leaf clusters are disjoint unions of
their two sons, preferably balanced, and measures clusters by their smallest
axis-parallel bounding boxes.  It does not fix a splitting rule.  Reading used
here: a cluster with more than ``leaf_size`` points is split at the median
along the longest side of its bounding box (ties between sides go to the lowest
axis); the first son receives the floor(n/2) points with the smallest
coordinates along that axis, ties broken by the original point index.

Clusters are numbered level by level (root = 0, then level 1 left to right,
...).  Points are permuted so that every cluster is a contiguous range of the
permutation (leaves left to right).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class ClusterTree:
    points: np.ndarray      # (N, d) original points
    perm: np.ndarray        # perm[k] = original index of the k-th point in tree order
    start: np.ndarray       # (nc,) first position in perm
    size: np.ndarray        # (nc,) number of points
    level: np.ndarray       # (nc,)
    parent: np.ndarray      # (nc,) -1 for the root
    sons: np.ndarray        # (nc, 2) -1 for leaves
    lo: np.ndarray          # (nc, d) bounding box
    hi: np.ndarray          # (nc, d)

    @property
    def n_clusters(self) -> int:
        return int(self.start.shape[0])

    @property
    def depth(self) -> int:
        return int(self.level.max())

    def is_leaf(self, c: int) -> bool:
        return self.sons[c, 0] < 0

    def cluster_points(self, c: int) -> np.ndarray:
        """Coordinates of cluster c's points in tree order."""
        idx = self.perm[self.start[c]:self.start[c] + self.size[c]]
        return self.points[idx]


def build_tree(points: np.ndarray, leaf_size: int) -> ClusterTree:
    pts = np.asarray(points, dtype=np.float64)
    n, d = pts.shape
    perm = np.arange(n, dtype=np.int64)
    start, size, level, parent, sons, lo, hi = [], [], [], [], [], [], []

    def add(s, m, lev, par):
        idx = perm[s:s + m]
        p = pts[idx]
        start.append(s)
        size.append(m)
        level.append(lev)
        parent.append(par)
        sons.append([-1, -1])
        lo.append(p.min(axis=0))
        hi.append(p.max(axis=0))
        return len(start) - 1

    add(0, n, 0, -1)
    c = 0
    while c < len(start):          # breadth-first: sons are appended after all clusters of a level
        s, m = start[c], size[c]
        if m > leaf_size:
            ext = hi[c] - lo[c]
            axis = int(np.argmax(ext))          # first maximum = lowest axis on ties
            idx = perm[s:s + m]
            order = np.lexsort((idx, pts[idx, axis]))   # by coordinate, then original index
            perm[s:s + m] = idx[order]
            h = m // 2
            a = add(s, h, level[c] + 1, c)
            b = add(s + h, m - h, level[c] + 1, c)
            sons[c] = [a, b]
        c += 1

    return ClusterTree(pts, perm, np.array(start, dtype=np.int64), np.array(size, dtype=np.int64),
                       np.array(level, dtype=np.int64), np.array(parent, dtype=np.int64),
                       np.array(sons, dtype=np.int64), np.array(lo), np.array(hi))
