"""Host-only planning of the tiled layout and product schedule (no device memory).

The exact multiply-add count of one product P_S(A B) is the numerator of every
algorithmic rate the benchmark reports.  It is pinned here against two counts that
share nothing with the library:
  - entry level, from the definition of the formatted product (eq. (product)):
    sum over (i, j) in S of |{k : (i, k) in S and (k, j) in S}|, i.e. the sum of
    (M M) over the positions of M for the 0/1 pattern matrix M (dense, small N);
  - cluster level, the cost in the proof of Theorem (product):
    sum over kept blocks (nu, nu') of n_nu n_nu' sum_{mu in S_nu cap S_nu'} n_mu,
    from the oracle's brute-force block pattern.
For block patterns the two agree exactly.  The per-class sums of the schedule must
add up to the same total.  Calls that need the device tables fail with EINVAL on a
pattern that is only planned.
"""
import ctypes

import numpy as np
import pytest

import synth
from oracle import pattern, samplets, tree

CASES = [("cube2", 2048, 16, 1, 1.6, 1), ("cube3", 4096, 32, 1, 1.0, 2), ("cube2", 4096, 32, 2, 1.6, 3),
         ("sphere", 3000, 32, 1, 1.0, 5), ("cube2", 777, 16, 1, 0.7, 8)]


@pytest.fixture(scope="module")
def S():
    from paper_2211_11681_amd import spm
    spm._lib.load()
    return spm


def oracle_blocks(kind, n, leaf, q, eta, seed):
    pts = synth.workload_points(kind, n, seed)
    ot = tree.build_tree(pts, leaf)
    ob = samplets.build_samplets(ot, q)
    return ob, pattern.block_pattern(ot, eta)


def block_macs(cs, blocks):
    nf = np.diff(cs)
    total = 0
    for nu, row in enumerate(blocks):
        for nu2 in row:
            mid = np.intersect1d(row, blocks[nu2], assume_unique=True)
            total += int(nf[nu]) * int(nf[nu2]) * int(nf[mid].sum())
    return total


def entry_macs(rp, col, n):
    m = pattern.dense_mask(rp, col, n).astype(np.float64)
    return int(round(float(((m @ m) * m).sum())))


@pytest.mark.parametrize("kind,n,leaf,q,eta,seed", CASES)
def test_plan_macs_match_definition(S, kind, n, leaf, q, eta, seed):
    ob, blocks = oracle_blocks(kind, n, leaf, q, eta, seed)
    cs = ob.cluster_start
    brp, bcol = pattern.block_csr(blocks)
    pat = S.Pattern.plan_blocks(n, cs, brp, bcol)
    ref_blocks = block_macs(cs, blocks)
    assert pat.macs == float(ref_blocks)
    if n <= 2048:
        rp, col = pattern.entry_csr(ob, blocks)
        assert entry_macs(rp, col, n) == ref_blocks
    cls = pat.classes()
    assert sum(c["exact_macs"] for c in cls) == pat.macs
    assert sum(c["out_tiles"] for c in cls) == pat.n_tiles
    assert all(c["padded_macs"] >= c["exact_macs"] > 0 for c in cls)
    assert pat.workspace_bytes() > 0


def test_plan_macs_masked_pattern_tile_level(S, cfg1_setup):
    """A-posteriori pattern (N = 2048, tau = 1e-6): the count runs over the tile
    structure, the cluster pairs holding at least one entry."""
    s = cfg1_setup
    rp, col = pattern.csr_from_mask(s["mask_post"])
    cs = s["basis"].cluster_start
    pat = S.Pattern.plan_csr(s["n"], rp, col, cs)
    clus = np.searchsorted(cs, np.arange(s["n"]), side="right") - 1
    rows = np.repeat(np.arange(s["n"]), np.diff(rp))
    nc = len(cs) - 1
    tiles = np.zeros((nc, nc), bool)
    tiles[clus[rows], clus[col]] = True
    blocks = [np.nonzero(tiles[c])[0] for c in range(nc)]
    assert pat.macs == float(block_macs(cs, blocks))
    assert pat.nnz == rp[-1]


def test_planned_pattern_rejects_compute(S):
    from paper_2211_11681_amd import _lib
    ob, blocks = oracle_blocks("cube2", 777, 16, 1, 0.7, 8)
    brp, bcol = pattern.block_csr(blocks)
    pat = S.Pattern.plan_blocks(777, ob.cluster_start, brp, bcol)
    lib = _lib.load()
    dummy = ctypes.c_void_p(4096)             # never dereferenced: the call fails first
    st = lib.spm_axpy(pat._h, 0, 1.0, None, 1.0, dummy, None)
    assert st == -1 and b"not uploaded" in lib.spm_last_error()
    st = lib.spm_masked_gemm(pat._h, 0, dummy, 0, dummy, 0, ctypes.c_void_p(8192), None)
    assert st == -1 and b"not uploaded" in lib.spm_last_error()
    # the host queries work without device tables
    rp, col = pat.download_csr()
    orp, ocol = pattern.entry_csr(ob, blocks)
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)


def test_split_parity_cases_cover_both_paths(S):
    """The split-precision product runs on the matrix cores when the pattern carries
    cluster levels, every cluster size is even and no unit class exceeds 7 x 7 blocks,
    else on the per-tile compensated kernel.  The GPU parity cases of the product
    (tests/test_gpu_parity.py, PRODUCT_CASES) must exercise both."""
    from test_gpu_parity import PRODUCT_CASES
    on_cores = []
    for kind, n, leaf, q, eta, seed in PRODUCT_CASES:
        t = S.Tree(synth.workload_points(kind, n, seed), leaf, q)
        arr = t.arrays()
        rp, col = t.block_pattern(eta)
        pat = S.Pattern.plan_blocks(n, arr["cluster_start"], rp, col, levels=arr["level"])
        even = bool(np.all(np.diff(arr["cluster_start"]) % 2 == 0))
        small = all(c["row_blocks"] <= 7 and c["col_blocks"] <= 7 for c in pat.classes())
        on_cores.append(even and small)
    assert any(on_cores) and not all(on_cores), on_cores
