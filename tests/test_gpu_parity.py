"""GPU parity: libspm through its C ABI against the FP64 oracle.

Tolerance for FP64 paths: 1e-12 relative Frobenius error (the stated bound for
FP64 values); pattern and index data bit-exact.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import compress, native, ops, pattern, samplets, tree

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def relerr(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


@pytest.fixture(scope="module")
def S():
    from paper_2211_11681_amd import spm
    spm._lib.load()
    assert torch.cuda.is_available()
    return spm


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def oracle_problem(kind, n, leaf, q, eta, seed, p, ell, tau=None):
    pts = synth.workload_points(kind, n, seed)
    ot = tree.build_tree(pts, leaf)
    ob = samplets.build_samplets(ot, q)
    blocks = pattern.block_pattern(ot, eta)
    rp, col = pattern.entry_csr(ob, blocks)
    ks = compress.compress_dense(ob, p, ell, 1.0 / n)
    mask = pattern.dense_mask(rp, col, n)
    if tau is not None:
        mask = pattern.threshold_mask(mask, ks, tau)
        rp, col = pattern.csr_from_mask(mask)
    return dict(pts=pts, tree=ot, basis=ob, rp=rp, col=col, mask=mask, ks=ks, n=n)


@pytest.fixture(scope="module")
def cfg1(S):
    """N=2048 unit square, Matern-3/2 l=0.5, m=3, leaf 16, eta=1.6, tau=1e-6 a-posteriori."""
    pr = oracle_problem("cube2", 2048, 16, 1, 1.6, 1, 1, 0.5, tau=1e-6)
    pat = S.Pattern.from_csr(2048, pr["rp"], pr["col"], pr["basis"].cluster_start)
    pr["pat"] = pat
    return pr


def test_csr_pattern_roundtrip(S, cfg1):
    print("case: cfg1 a-posteriori pattern upload", flush=True)
    pat = cfg1["pat"]
    rp, col = pat.download_csr()
    assert np.array_equal(rp, cfg1["rp"]) and np.array_equal(col, cfg1["col"])
    assert pat.nnz == cfg1["rp"][-1] and pat.n_stored > pat.nnz
    vals = np.where(cfg1["mask"], cfg1["ks"], 0.0)[cfg1["mask"]]
    t = pat.values_from_csr(to_dev(vals))
    back = pat.values_to_csr(t).cpu().numpy()
    assert np.array_equal(back, vals)
    # masked positions inside tiles hold 0
    assert int((t != 0).sum()) <= pat.nnz


def _dense_from_tiles(pat, vals, n, cs):
    """Dense matrix from tile-layout values (host-side test helper)."""
    tr, tc, to = pat.tiles()
    nf = np.diff(cs)
    out = np.zeros((n, n))
    v = vals.cpu().numpy() if isinstance(vals, torch.Tensor) else vals
    for t in range(len(tr)):
        r, c = tr[t], tc[t]
        blk = v[to[t]:to[t] + nf[r] * nf[c]].reshape(nf[c], nf[r]).T
        out[cs[r]:cs[r + 1], cs[c]:cs[c + 1]] = blk
    return out


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_product_cfg1_vs_oracle(S, cfg1, ta, tb):
    print(f"case: cfg1 product transA={ta} transB={tb}", flush=True)
    pat, mask, ks = cfg1["pat"], cfg1["mask"], cfg1["ks"]
    n = 2048
    a = np.where(mask, ks, 0.0)
    i, j = np.nonzero(mask)
    kt = np.zeros_like(a)
    kt[i, j] = a[i, j] * (1.0 + 0.1 * synth.pair_uniform(205, i, j, n))   # perturbed, not symmetric
    A = pat.values_from_csr(to_dev(a[mask]))
    B = pat.values_from_csr(to_dev(kt[mask]))
    C = S.masked_gemm(pat, A, B, transA=bool(ta), transB=bool(tb))
    got = pat.values_to_csr(C).cpu().numpy()
    ref = ops.masked_product(a.T if ta else a, kt.T if tb else kt, mask)[mask]
    assert relerr(got, ref) < TOL64
    if ta == 0 and tb == 0:
        ref2 = native.masked_product_csr(cfg1["rp"], cfg1["col"], a[mask], kt[mask])
        assert relerr(got, ref2) < TOL64
    # outputs at masked tile positions are exactly zero
    assert np.array_equal(_dense_from_tiles(pat, C, n, cfg1["basis"].cluster_start)[~mask], np.zeros((~mask).sum()))


PRODUCT_CASES = [("cube3", 4096, 32, 1, 1.0, 2), ("cube2", 4096, 32, 2, 1.6, 3), ("sphere", 4096, 32, 1, 1.0, 5),
                 ("cube3", 3000, 32, 1, 1.0, 4), ("cube2", 2048, 16, 1, 0.5, 7)]


@pytest.mark.parametrize("kind,n,leaf,q,eta,seed", PRODUCT_CASES)
def test_product_patterns_vs_oracle(S, kind, n, leaf, q, eta, seed):
    # block patterns of several shapes (tile sizes 4..28, root of 2m, unbalanced trees)
    # with non-symmetric random operands, all four transpose variants
    print(f"case: product {kind} n={n} leaf={leaf} q={q} eta={eta}", flush=True)
    pts = synth.workload_points(kind, n, seed)
    t = S.Tree(pts, leaf, q)
    pat = S.Pattern.from_tree(t, eta)
    rp, col = pat.download_csr()
    mask = pattern.dense_mask(rp, col, n)
    i, j = np.nonzero(mask)
    a = np.zeros((n, n)); b = np.zeros((n, n))
    a[i, j] = 2 * synth.pair_uniform(31, i, j, n) - 1
    b[i, j] = 2 * synth.pair_uniform(32, i, j, n) - 1
    A, B = pat.values_from_csr(to_dev(a[mask])), pat.values_from_csr(to_dev(b[mask]))
    A32 = {prec: S.convert(pat, A, "f64", prec) for prec in ("f32split", "f32acc")}
    B32 = {prec: S.convert(pat, B, "f64", prec) for prec in ("f32split", "f32acc")}
    for ta, tb in [(0, 0), (0, 1), (1, 0), (1, 1)]:
        C = S.masked_gemm(pat, A, B, transA=bool(ta), transB=bool(tb))
        ref = ops.masked_product(a.T if ta else a, b.T if tb else b, mask)[mask]
        assert relerr(pat.values_to_csr(C).cpu().numpy(), ref) < TOL64, (ta, tb)
        # FP32 modes on the same unit classes: F32SPLIT within 1e-8, F32ACC within 1e-6
        for prec, tol in (("f32split", 1e-8), ("f32acc", 1e-6)):
            C32 = S.masked_gemm(pat, A32[prec], B32[prec], transA=bool(ta), transB=bool(tb), prec=prec)
            err = relerr(pat.values_to_csr(S.convert(pat, C32, prec, "f64")).cpu().numpy(), ref)
            assert err <= tol, (prec, ta, tb, err)


def test_product_identity_exact(S, cfg1):
    pat, mask = cfg1["pat"], cfg1["mask"]
    a = np.where(mask, cfg1["ks"], 0.0)
    A = pat.values_from_csr(to_dev(a[mask]))
    eye = pat.values_from_csr(to_dev(np.eye(2048)[mask]))
    assert torch.equal(S.masked_gemm(pat, eye, A), A)
    assert torch.equal(S.masked_gemm(pat, A, eye), A)


COMPRESS_CASES = [("cube2", 2048, 16, 1, 1.6, 1, 1, 0.5), ("cube3", 4096, 32, 1, 1.0, 2, 0, 0.3),
                  ("cube2", 4096, 32, 2, 1.6, 3, 1, 0.1), ("sphere", 2048, 32, 1, 1.0, 5, 1, 0.3),
                  ("cube3", 3000, 32, 1, 1.0, 4, 2, 0.2)]


@pytest.mark.parametrize("kind,n,leaf,q,eta,seed,p,ell", COMPRESS_CASES)
def test_compression_vs_oracle_dense(S, kind, n, leaf, q, eta, seed, p, ell):
    print(f"case: compression {kind} n={n} leaf={leaf} q={q} p={p}", flush=True)
    pr = oracle_problem(kind, n, leaf, q, eta, seed, p, ell)
    t = S.Tree(pr["pts"], leaf, q)
    pat = S.Pattern.from_tree(t, eta)
    rp, col = pat.download_csr()
    assert np.array_equal(rp, pr["rp"]) and np.array_equal(col, pr["col"])
    k = S.kernel_compress(pat, t, p, ell, 1.0 / n)
    got = pat.values_to_csr(k).cpu().numpy()
    ref = pr["ks"][pr["mask"]]
    assert relerr(got, ref) < TOL64
    kd = S.kernel_compress(pat, t, p, ell, 1.0 / n, deriv=True)
    refd = compress.compress_dense(pr["basis"], p, ell, 1.0 / n, deriv=True)[pr["mask"]]
    assert relerr(pat.values_to_csr(kd).cpu().numpy(), refd) < TOL64


def test_compression_multi_panel_sampled_rows(S):
    # N = 16384 needs several panels (2 GiB panel budget); check sampled rows of
    # K^Sigma on the pattern against the oracle's row-wise construction.
    print("case: compression n=16384 cube3 sampled rows", flush=True)
    n, leaf, q, eta, p, ell = 16384, 32, 1, 1.0, 2, 0.2
    pts = synth.points_cube(n, 3, 4)
    t = S.Tree(pts, leaf, q)
    pat = S.Pattern.from_tree(t, eta)
    k = S.kernel_compress(pat, t, p, ell, 1.0 / n)
    csr = pat.values_to_csr(k).cpu().numpy()
    rp, col = pat.download_csr()
    ot = tree.build_tree(pts, leaf)
    ob = samplets.build_samplets(ot, q)
    rng = np.random.default_rng(0)
    rows = np.concatenate([[0, 1, 5, 9], rng.integers(0, n, 12)])
    ref = compress.compress_rows(ob, rows, p, ell, 1.0 / n, use_c=True)
    for kk, r in enumerate(rows):
        cols = col[rp[r]:rp[r + 1]]
        assert relerr(csr[rp[r]:rp[r + 1]], ref[kk, cols]) < TOL64, r


def test_axpy_convert_reductions(S, cfg1):
    pat, mask = cfg1["pat"], cfg1["mask"]
    n = 2048
    a = np.where(mask, cfg1["ks"], 0.0)
    A = pat.values_from_csr(to_dev(a[mask]))
    Y = A.clone()
    S.axpy(pat, 0.1, None, 1.0, Y)
    ref = ops.axpy(0.1, None, 1.0, a, mask)[mask]
    assert np.array_equal(pat.values_to_csr(Y).cpu().numpy(), ref)
    Z = A.clone()
    S.axpy(pat, 2.0, A, -0.5, Z)
    assert np.array_equal(pat.values_to_csr(Z).cpu().numpy(), (2.0 * a - 0.5 * a)[mask])
    # conversions
    sp = S.convert(pat, A, "f64", "f32split")
    back = S.convert(pat, sp, "f32split", "f64")
    assert relerr(back.cpu().numpy(), A.cpu().numpy()) < 1e-14
    hi = S.convert(pat, A, "f64", "f32acc")
    assert torch.equal(hi, A.float())
    # reductions
    y = synth.normals(n, 105)
    yd = to_dev(y)
    assert abs(S.sqdist(pat, A).item() - np.sum(a * a)) < 1e-13 * np.sum(a * a)
    d2 = np.sum(np.where(mask, np.eye(n) - a, 0.0) ** 2)
    assert abs(S.sqdist_eye(pat, A).item() - d2) < 1e-13 * d2
    assert abs(S.dot(pat, A, Z).item() - np.sum(a * 1.5 * a)) < 1e-13 * np.sum(1.5 * a * a)
    qf = y @ a @ y
    assert abs(S.quadform(pat, A, yd).item() - qf) < 1e-12 * abs(qf)
    F = S.fill_outer(pat, yd, 2.0)
    assert np.array_equal(pat.values_to_csr(F).cpu().numpy(), np.where(mask, 2.0 * np.outer(y, y), 0.0)[mask])
    # deterministic: bitwise equal on repeat
    assert S.sqdist(pat, A).item() == S.sqdist(pat, A).item()


def test_split_precision_errors(S, cfg1):
    pat, mask = cfg1["pat"], cfg1["mask"]
    a = np.where(mask, cfg1["ks"], 0.0)
    ref = native.masked_product_csr(cfg1["rp"], cfg1["col"], a[mask], a[mask])
    A = pat.values_from_csr(to_dev(a[mask]))
    As = S.convert(pat, A, "f64", "f32split")
    Cs = S.masked_gemm(pat, As, As, prec="f32split")
    e_split = relerr(pat.values_to_csr(S.convert(pat, Cs, "f32split", "f64")).cpu().numpy(), ref)
    Aa = S.convert(pat, A, "f64", "f32acc")
    Ca = S.masked_gemm(pat, Aa, Aa, prec="f32acc")
    e_acc = relerr(pat.values_to_csr(S.convert(pat, Ca, "f32acc", "f64")).cpu().numpy(), ref)
    print(f"split-precision relative Frobenius errors: f32split {e_split:.3e}  f32acc {e_acc:.3e}")
    assert e_split <= 1e-8
    assert e_acc <= 1e-6


def test_backward_vs_oracle(S, cfg1):
    pat, mask = cfg1["pat"], cfg1["mask"]
    n = 2048
    i, j = np.nonzero(mask)
    a = np.zeros((n, n)); b = np.zeros((n, n)); dc = np.zeros((n, n))
    a[i, j] = 2 * synth.pair_uniform(1, i, j, n) - 1
    b[i, j] = 2 * synth.pair_uniform(2, i, j, n) - 1
    dc[i, j] = 2 * synth.pair_uniform(3, i, j, n) - 1
    A, B, dC = (pat.values_from_csr(to_dev(x[mask])) for x in (a, b, dc))
    dA, dB = S.masked_gemm_backward(pat, dC, A, B)
    assert relerr(pat.values_to_csr(dA).cpu().numpy(), ops.masked_product(dc, b.T, mask)[mask]) < TOL64
    assert relerr(pat.values_to_csr(dB).cpu().numpy(), ops.masked_product(a.T, dc, mask)[mask]) < TOL64


def test_newton_schulz_vs_oracle(S):
    print("case: NS n=1024 cube2 leaf16 eta1 matern52", flush=True)
    n = 1024
    pts = synth.points_cube(n, 2, 4)
    ot = tree.build_tree(pts, 16)
    ob = samplets.build_samplets(ot, 1)
    rp, col = pattern.entry_csr(ob, pattern.block_pattern(ot, 1.0))
    mask = pattern.dense_mask(rp, col, n)
    a = np.where(mask, compress.compress_dense(ob, 2, 0.2, 1.0 / n), 0.0) + 1e-2 * np.eye(n)
    alpha0 = 2.0 / (1.0 + 2e-2)
    xo, reso, xs = ops.newton_schulz(a, mask, 20, alpha0)
    pat = S.Pattern.from_csr(n, rp, col, ob.cluster_start)
    A = pat.values_from_csr(to_dev(a[mask]))
    X, res, ck = S.newton_schulz(pat, A, 20, 3, "f64", alpha0, checkpoints=True)
    res = res.cpu().numpy()
    assert np.allclose(res, reso, rtol=1e-9, atol=1e-15)
    assert relerr(pat.values_to_csr(X).cpu().numpy(), xo[mask]) < TOL64
    for k in (0, 5, 20):
        assert relerr(pat.values_to_csr(ck[k]).cpu().numpy(), xs[k][mask]) < TOL64
    # FP32 bulk + 3 FP64 iterations reach the same final residual scale
    for bulk in ("f32split", "f32acc"):
        Xb, resb, _ = S.newton_schulz(pat, A, 20, 3, bulk, alpha0)
        rb = resb.cpu().numpy()
        print(f"NS bulk={bulk}: final residual {rb[-1]:.3e} (fp64 {res[-1]:.3e})")
        assert rb[-1] < 1e-8


@pytest.mark.parametrize("kind,n,leaf,q,eta,seed,p,ell", [("cube3", 4096, 32, 1, 1.0, 2, 0, 0.3),
                                                          ("cube2", 2048, 16, 1, 1.6, 1, 1, 0.5)])
def test_expm_taylor_vs_oracle(S, kind, n, leaf, q, eta, seed, p, ell):
    # truncated exponential series on S (Horner, formatted products), 10 terms, on the
    # oracle's K^eta uploaded to the tile layout
    print(f"case: expm_taylor {kind} n={n} leaf={leaf} q={q} eta={eta} matern p={p} l={ell}", flush=True)
    pr = oracle_problem(kind, n, leaf, q, eta, seed, p, ell)
    pat = S.Pattern.from_csr(n, pr["rp"], pr["col"], pr["basis"].cluster_start)
    mask = pr["mask"]
    a = np.where(mask, pr["ks"], 0.0)
    K = pat.values_from_csr(to_dev(a[mask]))
    E = S.expm_taylor(pat, K, 10)
    ref = ops.expm_taylor(a, mask, 10)[mask]
    err = relerr(pat.values_to_csr(E).cpu().numpy(), ref)
    print(f"expm_taylor: relative Frobenius error vs oracle {err:.3e}")
    assert err < TOL64
    # no terms: the identity, exactly
    E0 = S.expm_taylor(pat, K, 0)
    assert np.array_equal(pat.values_to_csr(E0).cpu().numpy(), np.eye(n)[mask])


@pytest.mark.parametrize("kind,n,leaf,q,eta,seed,p,ell", [("cube3", 4096, 32, 1, 1.0, 2, 2, 0.2),
                                                          ("cube2", 2048, 16, 1, 1.6, 1, 1, 0.5)])
def test_ns_sqrt_vs_oracle(S, kind, n, leaf, q, eta, seed, p, ell):
    # coupled masked Newton-Schulz square root of A = K^eta + 1e-2 I, 12 iterations
    print(f"case: ns_sqrt {kind} n={n} leaf={leaf} q={q} eta={eta} matern p={p} l={ell}", flush=True)
    pr = oracle_problem(kind, n, leaf, q, eta, seed, p, ell)
    pat = S.Pattern.from_csr(n, pr["rp"], pr["col"], pr["basis"].cluster_start)
    mask = pr["mask"]
    a = np.where(mask, pr["ks"], 0.0) + 1e-2 * np.eye(n)
    A = pat.values_from_csr(to_dev(a[mask]))
    Y, Z, res = S.ns_sqrt(pat, A, 12)
    y_ref, z_ref, res_ref = ops.ns_sqrt(a, mask, 12)
    ey = relerr(pat.values_to_csr(Y).cpu().numpy(), y_ref[mask])
    ez = relerr(pat.values_to_csr(Z).cpu().numpy(), z_ref[mask])
    print(f"ns_sqrt: Y error {ey:.3e}, Z error {ez:.3e}, residual {float(res[-1]):.3e} (oracle {res_ref[-1]:.3e})")
    assert ey < TOL64 and ez < TOL64
    r = res.cpu().numpy()
    assert np.all(np.abs(r - np.array(res_ref)) <= 1e-12 * np.maximum(np.array(res_ref), 1e-3))


@pytest.mark.parametrize("kind,n,leaf,q,eta,seed,p,ell,nodes,iters", [("cube2", 1024, 16, 1, 1.6, 1, 1, 0.5, 5, 16),
                                                                      ("cube3", 1500, 32, 1, 1.0, 3, 2, 0.2, 3, 12)])
def test_contour_invsqrt_vs_oracle(S, kind, n, leaf, q, eta, seed, p, ell, nodes, iters):
    # contour quadrature for A^{-1/2}, A = K^eta / lambda_max + 1e-2 I, spectrum in [1e-2, 1.01]
    print(f"case: contour_invsqrt {kind} n={n} leaf={leaf} eta={eta} nodes={nodes} iters={iters}", flush=True)
    pr = oracle_problem(kind, n, leaf, q, eta, seed, p, ell)
    pat = S.Pattern.from_csr(n, pr["rp"], pr["col"], pr["basis"].cluster_start)
    mask = pr["mask"]
    k = np.where(mask, pr["ks"], 0.0)
    a = k / np.linalg.eigvalsh(k)[-1] + 1e-2 * np.eye(n)
    A = pat.values_from_csr(to_dev(a[mask]))
    out, res = S.contour_invsqrt(pat, A, 1e-2, 1.01, nodes, iters)
    ref = ops.contour_invsqrt(a, mask, 1e-2, 1.01, nodes, iters)
    err = relerr(pat.values_to_csr(out).cpu().numpy(), ref[mask])
    r = res.cpu().numpy()
    print(f"contour_invsqrt: error vs oracle {err:.3e}, node residuals {r}")
    assert err < TOL64
    assert np.all(np.isfinite(r)) and r.shape == (nodes,)


def test_spmm_vs_oracle(S, cfg1):
    # S-matrix times a dense block of 10 columns (uniform entries, as in the paper's e_F)
    print("case: spmm cfg1 r=10", flush=True)
    pat, mask, n = cfg1["pat"], cfg1["mask"], cfg1["n"]
    a = np.where(mask, cfg1["ks"], 0.0)
    A = pat.values_from_csr(to_dev(a[mask]))
    x = synth.uniform(77, np.arange(10 * n)).reshape(10, n)
    Y = S.spmm(pat, A, to_dev(x))
    ref = ops.spmm(a, x.T).T
    err = relerr(Y.cpu().numpy(), ref)
    print(f"spmm: relative Frobenius error vs oracle {err:.3e}")
    assert err < TOL64


@pytest.mark.parametrize("kind,n,leaf,q,eta,seed,p,ell,r", [("cube3", 3000, 32, 1, 1.0, 4, 2, 0.2, 17),
                                                             ("cube2", 2048, 16, 1, 1.6, 1, 1, 0.5, 3),
                                                             ("sphere", 2048, 32, 1, 1.0, 5, 1, 0.3, 1)])
def test_spmm_patterns_vs_oracle(S, kind, n, leaf, q, eta, seed, p, ell, r):
    # S x dense on ragged cluster sizes; r = 17 takes two passes of 16 columns
    print(f"case: spmm {kind} n={n} leaf={leaf} eta={eta} r={r}", flush=True)
    pr = oracle_problem(kind, n, leaf, q, eta, seed, p, ell)
    pat = S.Pattern.from_csr(n, pr["rp"], pr["col"], pr["basis"].cluster_start)
    a = np.where(pr["mask"], pr["ks"], 0.0)
    A = pat.values_from_csr(to_dev(a[pr["mask"]]))
    x = 2 * synth.uniform(79, np.arange(r * n)).reshape(r, n) - 1
    Y = S.spmm(pat, A, to_dev(x))
    err = relerr(Y.cpu().numpy(), ops.spmm(a, x.T).T)
    print(f"spmm: relative Frobenius error vs oracle {err:.3e}")
    assert err < TOL64


def test_matrix_function_argument_errors(S, cfg1):
    # the drivers added for Section 4.4 reject bad arguments before any device work
    from paper_2211_11681_amd._lib import SpmError
    pat, n = cfg1["pat"], cfg1["n"]
    A = pat.empty("f64").zero_()
    S.axpy(pat, 1.0, None, 1.0, A)                                 # A = I
    for lo, hi, nodes in [(0.0, 1.0, 3), (1.0, 0.5, 3), (0.5, 1.0, 0), (float("nan"), 1.0, 3)]:
        with pytest.raises(SpmError):
            S.contour_invsqrt(pat, A, lo, hi, nodes, 4)
    with pytest.raises(SpmError):
        S.contour_invsqrt(pat, A, 0.5, 2.0, 3, -1)
    # a single node on the identity with bounds [1, 1] gives c_1 (1 + w_1^2)^{-1} I
    Z, res = S.contour_invsqrt(pat, A, 1.0, 1.0, 1, 30)
    w2, c = S.contour_rule(1.0, 1.0, 1)
    z = pat.values_to_csr(Z).cpu().numpy()
    d = np.eye(n)[cfg1["mask"]]
    assert np.max(np.abs(z - c[0] / (1.0 + w2[0]) * d)) < 1e-14
    assert float(res[0]) < 1e-15
    # zero vectors: S x dense and the transform do nothing (empty tensors may hold no storage)
    X0 = torch.zeros(0, n, dtype=torch.float64, device="cuda")
    assert S.spmm(pat, A, X0).shape == (0, n)


def test_fst_vs_oracle(S):
    # fast samplet transform of 3 vectors (original point order -> basis order) and back
    print("case: fst cube3 n=3000 leaf 32 q 1", flush=True)
    n = 3000
    pts = synth.workload_points("cube3", n, 4)
    t = S.Tree(pts, 32, 1)
    ot = tree.build_tree(pts, 32)
    ob = samplets.build_samplets(ot, 1)
    x = 2 * synth.uniform(78, np.arange(3 * n)).reshape(3, n) - 1
    W = S.fst(t, to_dev(x))
    ref = ops.fst(ob, x.T).T
    err = relerr(W.cpu().numpy(), ref)
    back = S.fst(t, W, inverse=True).cpu().numpy()
    print(f"fst: relative error vs oracle {err:.3e}, round trip {relerr(back, x):.3e}")
    assert err < TOL64 and relerr(back, x) < TOL64


def test_caller_workspace_paths(S, cfg1):
    """The pattern uploaded into caller memory and the products with a caller workspace
    give the results of the allocating entry points bit for bit."""
    print("case: caller-workspace upload and products (cfg1)", flush=True)
    import ctypes
    from paper_2211_11681_amd import _lib
    pat, mask = cfg1["pat"], cfg1["mask"]
    a = np.where(mask, cfg1["ks"], 0.0)
    i, j = np.nonzero(mask)
    b = np.zeros_like(a)
    b[i, j] = a[i, j] * (1.0 + 0.1 * synth.pair_uniform(206, i, j, 2048))
    A, B = pat.values_from_csr(to_dev(a[mask])), pat.values_from_csr(to_dev(b[mask]))
    p2 = S.Pattern.plan_csr(2048, cfg1["rp"], cfg1["col"], cfg1["basis"].cluster_start)
    assert p2.workspace_bytes() > 0
    p2.upload_workspace()
    assert (p2.nnz, p2.n_stored, p2.n_tiles, p2.macs) == (pat.nnz, pat.n_stored, pat.n_tiles, pat.macs)
    lib = _lib.load()
    st = lib.spm_pattern_upload_workspace(p2._h, ctypes.c_void_p(p2._ws.data_ptr()), p2._ws.numel() * 8, None)
    assert st == -1                                     # already uploaded
    for prec in ("f64", "f32acc", "f32split"):
        Ap, Bp = (A, B) if prec == "f64" else (S.convert(pat, A, "f64", prec), S.convert(pat, B, "f64", prec))
        for ta, tb in [(0, 0), (1, 0), (0, 1), (1, 1)]:
            C1 = pat.empty(prec)
            S.call("spm_masked_gemm", pat._h, S.prec_code(prec), S._ptr(Ap), ta, S._ptr(Bp), tb, S._ptr(C1),
                   S._stream())
            C2 = S.masked_gemm(p2, Ap, Bp, transA=bool(ta), transB=bool(tb), prec=prec)
            assert torch.equal(C1, C2), (prec, ta, tb)
        dA1, dB1 = S.masked_gemm_backward(pat, Ap, Bp, Ap, prec=prec)
        dA2 = pat.empty(prec)
        dB2 = pat.empty(prec)
        S.call("spm_masked_gemm_backward", pat._h, S.prec_code(prec), S._ptr(Ap), S._ptr(Bp), S._ptr(Ap),
               S._ptr(dA2), S._ptr(dB2), S._stream())
        assert torch.equal(dA1, dA2) and torch.equal(dB1, dB2), prec
    # a short workspace is refused before any work
    need = S.gemm_workspace_bytes(pat, "f64", False, False)
    C = pat.empty("f64")
    st = lib.spm_masked_gemm_ws(pat._h, 0, ctypes.c_void_p(A.data_ptr()), 0, ctypes.c_void_p(B.data_ptr()), 0,
                                ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(C.data_ptr()), need - 8, None)
    assert st == -1 and b"workspace" in lib.spm_last_error()


def test_newton_schulz_diverging_reports_enotconv(S, cfg1):
    """An initial scale far above 2 / lambda_max makes the iteration diverge; three
    iterations keep every value finite, so the growing residual is what is reported."""
    print("case: Newton-Schulz diverging from alpha0 = 60 (cfg1)", flush=True)
    from paper_2211_11681_amd import _lib
    pat, mask = cfg1["pat"], cfg1["mask"]
    a = np.where(mask, cfg1["ks"], 0.0)
    a[np.arange(2048), np.arange(2048)] += 1e-2
    A = pat.values_from_csr(to_dev(a[mask]))
    with pytest.raises(_lib.SpmError) as ei:
        S.newton_schulz(pat, A, 3, 3, "f64", 60.0)
    assert ei.value.status == -5 and "exceeds the initial residual" in str(ei.value)
    X, res, _ = S.newton_schulz(pat, A, 3, 3, "f64", 2.0 / 1.02)   # the converging start still passes
    r = res.cpu().numpy()
    assert np.all(np.isfinite(r)) and r[-1] < r[0]
