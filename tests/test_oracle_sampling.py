"""Pins of the oracle helpers the CPU baseline samples with.

- block_rows (batched eq. (cutoff)) equals block_row cluster by cluster, bit for bit;
- compress_rows with the C helper (the rows of one cluster summed together) equals
  the single-row sums bit for bit;
- masked_product_entries equals the full formatted product at the listed positions
  bit for bit (same merge, same order) and counts sum |S_i cap S_j| multiply-adds,
  checked against the dense 0/1 pattern matrix: (M M)_ij.
"""
import numpy as np

import synth
from oracle import native, pattern, samplets, tree


def test_block_rows_equal_block_row():
    pts = synth.points_cube(3000, 2, 9)
    ot = tree.build_tree(pts, 16)
    d = pattern.diameters(ot)
    br = pattern.block_rows(ot, 1.3, np.arange(ot.n_clusters)[::-1], d, chunk=29)
    assert sorted(br) == list(range(ot.n_clusters))
    for c in range(ot.n_clusters):
        assert np.array_equal(br[c], pattern.block_row(ot, 1.3, c, d))


def test_masked_product_entries_match_full_product():
    n = 1500
    pts = synth.points_cube(n, 3, 12)
    ot = tree.build_tree(pts, 32)
    ob = samplets.build_samplets(ot, 1)
    rp, col = pattern.entry_csr(ob, pattern.block_pattern(ot, 1.0))
    rows = np.repeat(np.arange(n), np.diff(rp))
    a = synth.pair_uniform(31, rows, col, n) - 0.5
    b = synth.pair_uniform(32, rows, col, n) - 0.5
    full = native.masked_product_csr(rp, col, a, b)
    tpos = native.transpose_positions(rp, col)
    pick = (synth.uniform(33, np.arange(700)) * rp[-1]).astype(np.int64)
    c = np.zeros(rp[-1])
    macs = native.masked_product_entries(rows[pick], col[pick], pick, rp, col, a, b[tpos], c)
    assert np.array_equal(c[pick], full[pick])
    m = pattern.dense_mask(rp, col, n).astype(np.float64)
    mm = m @ m
    assert macs == int(mm[rows[pick], col[pick]].sum())


def test_compress_rows_batched_equals_single_rows():
    from oracle import compress
    n = 3000
    pts = synth.points_cube(n, 3, 4)
    ot = tree.build_tree(pts, 32)
    ob = samplets.build_samplets(ot, 1)
    rows = np.array([0, 3, 7, 100, 101, 2999, 1500])
    got = compress.compress_rows(ob, rows, 1, 0.3, 1.0 / n, use_c=True)
    T = ob.sparse_T()
    owner = ob.support_cluster_of()
    x = ot.points[ot.perm]
    for k, b in enumerate(rows):
        c = owner[b]
        s, sz = int(ot.start[c]), int(ot.size[c])
        w = np.asarray(ob.coef[c])[b - ob.cluster_start[c]]
        assert np.array_equal(got[k], T @ native.kernel_apply(x, x[s:s + sz], w, 1, 0.3, 1.0 / n)), k
    # and the numpy evaluation of the same rows agrees to rounding
    ref = compress.compress_rows(ob, rows, 1, 0.3, 1.0 / n)
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
