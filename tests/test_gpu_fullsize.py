"""Parity at the benchmark's full size, in the launch configuration bench.py times.

Workload: N = 131072 points uniform in [0,1]^3 (seed 2), exponential kernel
(Matern nu = 1/2) l = 0.3 scaled by 1/N, degree 1 (m = 4), leaf 32, eta = 1.0.
The library builds tree, pattern and K^eta and computes C = P_S(K K) exactly as
bench.py does.  The oracle computes, from the paper's definitions, the rows of
K^Sigma = T K T^T for a sample of basis functions (three leaves and their
ancestors on levels 10, 8, 6, 4, 3, 2 and 1, two functions each, and the first
root function) and from them every sampled entry c_ij = sum_{k in S_i cap S_j}
K_ik K_jk with (i, j) in S.  The coarse rows are full rows of the pattern, whose
output tiles have the longest middle lists and the most stages.
Sampled entries of K^eta and of C are compared one by one.

Tolerance per entry: 1e-12 * ||K_i|| ||K_j|| for C (the Cauchy-Schwarz scale of
the sum) and 1e-12 * ||K_i|| for K.  The FP32 forms of the product are held at the
same entries to a relative Frobenius error of 1e-8 (FP32-split) and 1e-6 (F32ACC).

The same run checks the two operations that the error measure e_F uses, as the
benchmark runs them at this size: rows of Y = K^eta X for a uniform block X of 10
vectors against the oracle rows (tolerance 1e-12 * ||K_i|| ||X||), and the fast
samplet transform of X against the oracle's sparse T at every entry (1e-12 * ||X||).

It also certifies the masked Newton-Schulz inverse of A = K^eta + 1e-2 I at this
size, 20 iterations all in FP64 and in the recipes of the inverse benchmark (the
first 17 in F32ACC or in the FP32-split product on matrix cores, the last 3 in
FP64): for the sampled pairs (i, j) in S the
residual entry delta_ij - sum_{k in S_i cap S_j} A_ik X_kj, with the oracle's rows
of A and the library's X, must vanish to 1e-10 of sum_k |A_ik X_kj| (the converged
iteration has P_S(A X) = I on S; a wrong iterate leaves residuals of order 1).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import compress, pattern, samplets, tree

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

N, D, SEED, LEAF, Q, ETA, P, ELL = 131072, 3, 2, 32, 1, 1.0, 0, 0.3


def test_product_full_size_sampled_entries():
    print("case: full-size product N=131072 cube3 leaf32 eta1.0 exponential l0.3", flush=True)
    from paper_2211_11681_amd import spm
    spm._lib.load()
    assert torch.cuda.is_available()
    pts = synth.points_cube(N, D, SEED)
    t = spm.Tree(pts, LEAF, Q)
    pat = spm.Pattern.from_tree(t, ETA)
    K = spm.kernel_compress(pat, t, P, ELL, 1.0 / N)
    C = spm.masked_gemm(pat, K, K)
    torch.cuda.synchronize()
    cs_lib = t.arrays()["cluster_start"]

    # oracle construction
    ot = tree.build_tree(pts, LEAF)
    ob = samplets.build_samplets(ot, Q)
    blocks = pattern.block_pattern(ot, ETA)
    cs = ob.cluster_start
    assert np.array_equal(cs, cs_lib)
    nf = np.diff(cs)
    leaves = np.nonzero(ot.sons[:, 0] < 0)[0]
    parent = ot.parent
    chosen = []
    for li in (len(leaves) // 7, len(leaves) // 2, 5 * len(leaves) // 6):
        c = int(leaves[li])
        while c >= 0:
            if c == leaves[li] or int(ot.level[c]) in (10, 8, 6, 4, 3, 2, 1):
                chosen.append(c)
            c = parent[c]
    rows = {int(cs[c]) + k for c in set(chosen) for k in (0, int(nf[c]) - 1)}
    rows.add(0)                                                     # first root function (level 0)
    rows = np.array(sorted(rows), np.int64)
    clus_of = np.searchsorted(cs, rows, side="right") - 1
    print(f"oracle rows: {len(rows)} from clusters {sorted(set(chosen))}", flush=True)
    kr = compress.compress_rows(ob, rows, P, ELL, 1.0 / N, use_c=True)
    masks = np.zeros((len(rows), N), bool)
    for a, c in enumerate(clus_of):
        for b in blocks[c]:
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

    # C entries: every sampled pair inside S
    pairs = [(a, b) for a in range(len(rows)) for b in range(len(rows)) if masks[a, rows[b]]]
    assert len(pairs) > 100
    idx = torch.tensor([position(rows[a], rows[b]) for a, b in pairs], dtype=torch.int64, device="cuda")
    got = C[idx].cpu().numpy()
    ref = np.array([keta[a] @ keta[b] for a, b in pairs])
    scale = np.array([norms[a] * norms[b] for a, b in pairs])
    err = np.abs(got - ref) / scale
    print(f"C: {len(pairs)} sampled entries, max error / (|K_i||K_j|) = {err.max():.3e}", flush=True)
    assert err.max() < 1e-12

    # the FP32 forms of the product at the same entries (relative Frobenius error over
    # the sample: FP32-split on the matrix cores <= 1e-8, F32ACC <= 1e-6)
    for prec, tol in (("f32split", 1e-8), ("f32acc", 1e-6)):
        Ks = spm.convert(pat, K, "f64", prec)
        Cs = spm.masked_gemm(pat, Ks, Ks, prec=prec)
        g = Cs[idx].double()
        if prec == "f32split":
            g = g + Cs[pat.n_stored + idx].double()
        e32 = np.linalg.norm(g.cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"{prec}: {len(pairs)} sampled entries, rel Frobenius {e32:.3e}", flush=True)
        assert e32 <= tol, (prec, e32)
        del Ks, Cs

    # K entries: 64 seeded columns of each sampled row
    kpos, kref, kscale = [], [], []
    for a, i in enumerate(rows):
        cols = np.nonzero(masks[a])[0]
        pick = cols[(synth.uniform(700 + a, np.arange(64)) * len(cols)).astype(np.int64)]
        for j in pick:
            kpos.append(position(i, j))
            kref.append(keta[a, j])
            kscale.append(norms[a])
    gk = K[torch.tensor(kpos, dtype=torch.int64, device="cuda")].cpu().numpy()
    kerr = np.abs(gk - np.array(kref)) / np.array(kscale)
    print(f"K: {len(kpos)} sampled entries, max error / |K_i| = {kerr.max():.3e}", flush=True)
    assert kerr.max() < 1e-12

    # S x dense and the fast samplet transform at full size
    from oracle import ops
    x = synth.uniform(91, np.arange(10 * N)).reshape(10, N)
    X = torch.from_numpy(x).cuda()
    Y = spm.spmm(pat, K, X).cpu().numpy()
    yref = keta @ x.T                                               # sampled rows, 10 columns
    nx = np.linalg.norm(x)
    yerr = np.abs(Y[:, rows].T - yref).max(axis=1) / (norms * nx)
    print(f"S x dense: {len(rows)} sampled rows, max error / (|K_i||X|) = {yerr.max():.3e}", flush=True)
    assert yerr.max() < 1e-12
    W = spm.fst(t, X).cpu().numpy()
    wref = ops.fst(ob, x.T).T
    ferr = np.abs(W - wref).max() / nx
    print(f"FST: all {W.size} entries, max error / |X| = {ferr:.3e}", flush=True)
    assert ferr < 1e-12

    # masked Newton-Schulz inverse: sampled entries of I - P_S(A X)
    mu = 1e-2
    A = K.clone()
    spm.axpy(pat, mu, None, 1.0, A)
    arow = keta.copy()
    arow[np.arange(len(rows)), rows] += mu

    def positions(ii, j):                                          # position() over an array of rows
        ci = np.searchsorted(cs, ii, side="right") - 1
        cj = np.searchsorted(cs, j, side="right") - 1
        t_ = np.searchsorted(tkey, ci * nc + cj)
        assert np.all(tkey[t_] == ci * nc + cj)
        return to[t_] + (j - cs[cj]) * nf[ci] + (ii - cs[ci])

    for bulk, nfin in (("f64", 20), ("f32acc", 3), ("f32split", 3)):
        print(f"case: Newton-Schulz 20 iterations, bulk {bulk}, last {nfin} in FP64", flush=True)
        Xns, res, _ = spm.newton_schulz(pat, A, 20, nfin, bulk, 2.0 / (1.0 + 2.0 * mu))
        worst = 0.0
        for a, b in pairs:
            ks = np.nonzero(masks[a] & masks[b])[0]
            pos = positions(ks, rows[b]).astype(np.int64)
            xk = Xns[torch.from_numpy(pos).cuda()].cpu().numpy()
            terms = arow[a, ks] * xk
            r = (1.0 if rows[a] == rows[b] else 0.0) - terms.sum()
            worst = max(worst, abs(r) / max(np.abs(terms).sum(), 1e-300))
        print(f"NS ({bulk} bulk): final residual {float(res[-1]):.3e}; {len(pairs)} sampled residual entries, "
              f"max |r_ij| / sum|A_ik X_kj| = {worst:.3e}", flush=True)
        assert float(res[-1]) < 1e-8
        assert worst < 1e-10
        del Xns
