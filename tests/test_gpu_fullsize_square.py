"""Parity on the million-point square at full size, in the launch configuration
``bench.py`` times by default.

Workload: N = 1048576 points uniform in [0,1]^2 (seed 3), Matern nu = 3/2,
l = 0.1, scaled by 1/N, degree 2 (m = 6), leaf 32, eta = 1.6: 3.8e7 tiles and
4.59e9 stored entries, so element offsets run past 2^32.  The library builds tree, pattern and K^eta and computes
C = P_S(K K) in FP64 exactly as the benchmark does.  The oracle computes, from
the paper's definitions, the rows of K^Sigma = T K T^T for a sample of basis
functions (four leaves and their ancestors on levels 13 and 11, the first and
last function of each) and their block rows of the pattern (eq. (cutoff)), and
from them every sampled entry c_ij = sum_{k in S_i cap S_j} K_ik K_jk with
(i, j) in S.  The last leaf is one of the four: its tiles lie beyond element 2^32.

Tolerance: relative Frobenius error <= 1e-12 over the sampled entries of C and
of K^eta, and per entry <= 1e-12 * k_max^2 for C and 1e-12 * k_max for K, with
k_max the largest sampled row norm of K^eta.  Entries of K^Sigma in the rows of
fine samplets (three vanishing moments) are cancellations of kernel values of
size 1/N, so their absolute rounding error is set by that size, not by their
own row norm: measured 1e-21 to 4e-20 in every sampled row while the row norms
fall from 5e-7 (level 11) to 2e-10 (leaves).  A bound relative to each row's
own norm would test the conditioning of the exact construction, not the
arithmetic of either side.

The same sampled entries check the two FP32 forms of the product (the FP32-split
product on the matrix cores, relative Frobenius error over the sample <= 1e-8; F32ACC
<= 1e-6).

The construction of the million-point problem takes about two minutes on the GPU
host (tree, pattern, schedule and the O(N^2) compression).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import compress, pattern, samplets, tree

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]

N, D, SEED, LEAF, Q, ETA, P, ELL = 1048576, 2, 3, 32, 2, 1.6, 1, 0.1


def test_square_full_size_sampled_entries():
    print("case: full-size product N=1048576 square leaf32 q2 eta1.6 matern3/2 l0.1", flush=True)
    from paper_2211_11681_amd import spm
    spm._lib.load()
    assert torch.cuda.is_available()
    pts = synth.points_cube(N, D, SEED)
    t = spm.Tree(pts, LEAF, Q)
    pat = spm.Pattern.from_tree(t, ETA)
    print(f"library: {pat.n_tiles} tiles, {pat.nnz} entries; compressing", flush=True)
    K = spm.kernel_compress(pat, t, P, ELL, 1.0 / N)
    C = spm.masked_gemm(pat, K, K)
    torch.cuda.synchronize()
    cs_lib = t.arrays()["cluster_start"]
    print("library: product done", flush=True)

    # oracle construction
    ot = tree.build_tree(pts, LEAF)
    ob = samplets.build_samplets(ot, Q)
    cs = ob.cluster_start
    assert np.array_equal(cs, cs_lib)
    nf = np.diff(cs)
    leaves = np.nonzero(ot.sons[:, 0] < 0)[0]
    chosen = []
    for li in (len(leaves) // 7, len(leaves) // 2, 5 * len(leaves) // 6, len(leaves) - 1):
        c = int(leaves[li])
        while c >= 0:
            if c == leaves[li] or int(ot.level[c]) in (13, 11):
                chosen.append(c)
            c = ot.parent[c]
    rows = np.array(sorted({int(cs[c]) + k for c in set(chosen) for k in (0, int(nf[c]) - 1)}), np.int64)
    clus_of = np.searchsorted(cs, rows, side="right") - 1
    print(f"oracle rows: {len(rows)} from clusters {sorted(set(chosen))}", flush=True)
    kr = compress.compress_rows(ob, rows, P, ELL, 1.0 / N, use_c=True)
    diam = pattern.diameters(ot)
    masks = np.zeros((len(rows), N), bool)
    for a, c in enumerate(clus_of):
        for b in pattern.block_row(ot, ETA, int(c), diam):
            masks[a, cs[b]:cs[b + 1]] = True
    keta = np.where(masks, kr, 0.0)
    norms = np.linalg.norm(keta, axis=1)

    # positions of (i, j) in the tile layout
    tr, tc, to = pat.tiles()
    nc = len(cs) - 1
    tkey = tr.astype(np.int64) * nc + tc

    def position(i, j):
        ci = np.searchsorted(cs, i, side="right") - 1
        cj = np.searchsorted(cs, j, side="right") - 1
        t_ = np.searchsorted(tkey, ci * nc + cj)
        assert tkey[t_] == ci * nc + cj
        return to[t_] + (j - cs[cj]) * nf[ci] + (i - cs[ci])

    pairs = [(a, b) for a in range(len(rows)) for b in range(len(rows)) if masks[a, rows[b]]]
    assert len(pairs) > 50
    pos = np.array([position(rows[a], rows[b]) for a, b in pairs], np.int64)
    print(f"sampled positions up to {pos.max()} (2^32 = {2 ** 32})", flush=True)
    assert pos.max() >= 2 ** 32
    got = C[torch.from_numpy(pos).cuda()].cpu().numpy()
    ref = np.array([keta[a] @ keta[b] for a, b in pairs])
    kmax = norms.max()
    cfro = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    cent = np.abs(got - ref).max() / kmax ** 2
    print(f"C: {len(pairs)} sampled entries, rel Frobenius {cfro:.3e}, max error / k_max^2 {cent:.3e}, "
          f"max error / (|K_i||K_j|) {(np.abs(got - ref) / np.outer(norms, norms)[tuple(np.array(pairs).T)]).max():.3e}",
          flush=True)
    assert cfro < 1e-12 and cent < 1e-12

    # K entries: 64 seeded columns of each sampled row
    kpos, kref, kscale = [], [], []
    for a, i in enumerate(rows):
        cols = np.nonzero(masks[a])[0]
        pick = cols[(synth.uniform(900 + a, np.arange(64)) * len(cols)).astype(np.int64)]
        for j in pick:
            kpos.append(position(i, j))
            kref.append(keta[a, j])
            kscale.append(norms[a])
    gk = K[torch.tensor(kpos, dtype=torch.int64, device="cuda")].cpu().numpy()
    kref = np.array(kref)
    kfro = np.linalg.norm(gk - kref) / np.linalg.norm(kref)
    kent = np.abs(gk - kref).max() / kmax
    print(f"K: {len(kpos)} sampled entries, rel Frobenius {kfro:.3e}, max error / k_max {kent:.3e}, "
          f"max error / |K_i| {(np.abs(gk - kref) / np.array(kscale)).max():.3e}, largest position {max(kpos)}",
          flush=True)
    assert max(kpos) >= 2 ** 32
    assert kfro < 1e-12 and kent < 1e-12

    # the FP32 forms of the same product at the same sampled entries (the FP32-split
    # product runs on the matrix cores here: levels in the plan, even cluster sizes),
    # against the oracle: relative Frobenius error over the sample <= 1e-8 (F32SPLIT)
    # and <= 1e-6 (F32ACC), the bounds of the small parity cases
    del C
    torch.cuda.empty_cache()
    pos_t = torch.from_numpy(pos).cuda()
    Kcur, cur = K, "f64"
    del K
    for prec, tol in (("f32split", 1e-8), ("f32acc", 1e-6)):
        print(f"case: full-size product in {prec}", flush=True)
        Ks = spm.convert(pat, Kcur, cur, prec)
        del Kcur
        torch.cuda.empty_cache()
        Kcur, cur = Ks, prec
        Cs = spm.masked_gemm(pat, Ks, Ks, prec=prec)
        g = Cs[pos_t].double()
        if prec == "f32split":
            g = g + Cs[pat.n_stored + pos_t].double()
        err = np.linalg.norm(g.cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"{prec}: {len(pairs)} sampled entries, rel Frobenius {err:.3e}", flush=True)
        assert err <= tol, (prec, err)
        del Cs, Ks
        torch.cuda.empty_cache()
