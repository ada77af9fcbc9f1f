"""Pins of the oracle's operations: formatted product, addition, Newton-Schulz,
adjoints and the Gaussian-process lengthscale gradient."""
import numpy as np
import pytest

import synth
from oracle import compress, native, ops, pattern, samplets, tree


def _small(n=256, d=2, leaf=16, q=1, eta=1.0, seed=21):
    t = tree.build_tree(synth.points_cube(n, d, seed), leaf)
    b = samplets.build_samplets(t, q)
    rp, col = pattern.entry_csr(b, pattern.block_pattern(t, eta))
    return t, b, rp, col, pattern.dense_mask(rp, col, n)


def _rand_on(mask, seed):
    n = mask.shape[0]
    i, j = np.nonzero(mask)
    v = np.zeros(mask.shape)
    v[i, j] = 2.0 * synth.pair_uniform(seed, i, j, n) - 1.0
    return v


def test_product_brute_force_tiny():
    # triple loop over (i, j) in S and k in S_i cap S_j, pure Python
    t, b, rp, col, mask = _small(n=64, leaf=8, eta=0.8)
    a, bb = _rand_on(mask, 1), _rand_on(mask, 2)
    rows = [set(col[rp[i]:rp[i + 1]].tolist()) for i in range(64)]
    ref = np.zeros_like(a)
    for i in range(64):
        for j in rows[i]:
            s = 0.0
            for k in sorted(rows[i] & rows[j]):
                s += a[i, k] * bb[k, j]
            ref[i, j] = s
    assert np.abs(ops.masked_product(a, bb, mask) - ref).max() < 1e-14
    got = native.masked_product_csr(rp, col, a[mask], bb[mask])
    assert np.array_equal(got, ref[mask])          # same summation order: bit-exact


def test_product_c_merge_equals_dense(cfg1_setup):
    ks, mask, rp, col = cfg1_setup["ks"], cfg1_setup["mask_prior"], cfg1_setup["rp"], cfg1_setup["col"]
    a = np.where(mask, ks, 0.0)
    kt = a * (1.0 + 0.1 * _rand_on(mask, 205).clip(0))   # perturbed, non-symmetric operand
    dense = ops.masked_product(a, kt, mask)
    got = native.masked_product_csr(rp, col, a[mask], kt[mask])
    ref = dense[mask]
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_product_identities(cfg1_setup):
    mask, rp, col = cfg1_setup["mask_prior"], cfg1_setup["rp"], cfg1_setup["col"]
    a = np.where(mask, cfg1_setup["ks"], 0.0)
    eye = np.eye(2048)
    # exact: one nonzero term per entry
    assert np.array_equal(native.masked_product_csr(rp, col, eye[mask], a[mask]), a[mask])
    assert np.array_equal(native.masked_product_csr(rp, col, a[mask], eye[mask]), a[mask])
    d1, d2 = np.diag(np.arange(1.0, 2049.0)), np.diag(np.linspace(-1, 1, 2048))
    assert np.array_equal(native.masked_product_csr(rp, col, d1[mask], d2[mask]), (d1 @ d2)[mask])
    # symmetric operands in the same summation order give an exactly symmetric product
    s = np.triu(a) + np.triu(a, 1).T
    c = np.zeros_like(s)
    c[mask] = native.masked_product_csr(rp, col, s[mask], s[mask])
    assert np.array_equal(c, c.T)


def test_product_bilinear_and_full_pattern():
    t, b, rp, col, mask = _small(n=256)
    a, bb, cc = _rand_on(mask, 3), _rand_on(mask, 4), _rand_on(mask, 5)
    lhs = ops.masked_product(2.0 * a + 3.0 * cc, bb, mask)
    rhs = 2.0 * ops.masked_product(a, bb, mask) + 3.0 * ops.masked_product(cc, bb, mask)
    assert np.abs(lhs - rhs).max() < 1e-12
    # eta -> infinity keeps everything: the product is the plain matrix product
    t, b, rp, col, full = _small(n=256, eta=1e9)
    assert full.all()
    a, bb = _rand_on(full, 6), _rand_on(full, 7)
    got = native.masked_product_csr(rp, col, a[full], bb[full])
    assert np.allclose(got, (a @ bb)[full], rtol=1e-12, atol=1e-13)


def test_axpy_and_identity(cfg1_setup):
    mask = cfg1_setup["mask_post"]
    y = np.where(mask, cfg1_setup["ks"], 0.0)
    out = ops.axpy(0.1, None, 1.0, y, mask)
    off = ~np.eye(2048, dtype=bool)
    assert np.array_equal(out[off], y[off])
    assert np.array_equal(np.diag(out), 0.1 + np.diag(y))
    z = ops.axpy(2.0, y, -1.0, y, mask)
    assert np.array_equal(z, np.where(mask, 2.0 * y - y, 0.0))


def _spd_problem(n=256, eta=1.0, mu=1e-2, p=2, ell=0.2, d=3, seed=4, leaf=32):
    t = tree.build_tree(synth.points_cube(n, d, seed), leaf)
    b = samplets.build_samplets(t, 1)
    rp, col = pattern.entry_csr(b, pattern.block_pattern(t, eta))
    mask = pattern.dense_mask(rp, col, n)
    ks = compress.compress_dense(b, p, ell, 1.0 / n)
    a = np.where(mask, ks, 0.0) + mu * np.eye(n)
    return b, mask, a


def test_newton_schulz_full_pattern_is_textbook_inverse():
    b, mask, a = _spd_problem(eta=1e9)
    assert mask.all()
    x, res, _ = ops.newton_schulz(a, mask, 20, 2.0 / (1.0 + 2 * 1e-2))
    assert res[-1] < 1e-12
    assert np.allclose(x, np.linalg.inv(a), rtol=1e-9, atol=1e-9)
    assert all(res[k + 1] <= res[k] for k in range(len(res) - 1) if res[k] > 1e-13)


def test_newton_schulz_masked_fixed_point():
    # The fixed point with P_S(A X) = I is given column by column by the local
    # solves A[S_j, S_j] x = e_j (independent computation via LAPACK).
    b, mask, a = _spd_problem(n=1024, d=2, leaf=16, eta=1.0)
    assert mask.mean() < 0.5
    x, res, _ = ops.newton_schulz(a, mask, 40, 2.0 / (1.0 + 2 * 1e-2))
    xstar = ops.column_local_inverse(a, mask)
    assert res[-1] < 1e-10
    assert np.abs(x - xstar).max() < 1e-8 * np.abs(xstar).max()


def test_adjoint_dot_product_identity():
    t, b, rp, col, mask = _small(n=256)
    a, bb, dc = _rand_on(mask, 8), _rand_on(mask, 9), _rand_on(mask, 10)
    da = ops.masked_product(dc, bb.T, mask)      # P_S(dC B^T)
    db = ops.masked_product(a.T, dc, mask)       # P_S(A^T dC)
    d_a, d_b = _rand_on(mask, 11), _rand_on(mask, 12)
    lhs_a = np.sum(dc * ops.masked_product(d_a, bb, mask))
    lhs_b = np.sum(dc * ops.masked_product(a, d_b, mask))
    assert abs(lhs_a - np.sum(da * d_a)) < 1e-12 * abs(lhs_a)
    assert abs(lhs_b - np.sum(db * d_b)) < 1e-12 * abs(lhs_b)


def _gp(n, eta, ell, iters=15, mu=1e-2):
    t = tree.build_tree(synth.points_sphere(n, 5), 32)
    b = samplets.build_samplets(t, 1)
    rp, col = pattern.entry_csr(b, pattern.block_pattern(t, eta))
    mask = pattern.dense_mask(rp, col, n)
    y = synth.normals(n, 105)

    def amat(l):
        return np.where(mask, compress.compress_dense(b, 1, l, 1.0 / n), 0.0) + mu * np.eye(n)

    da = np.where(mask, compress.compress_dense(b, 1, ell, 1.0 / n, deriv=True), 0.0)
    return b, mask, y, amat, da


@pytest.mark.parametrize("eta", [1.0, 1e9])
def test_gp_gradient_matches_central_fd(eta):
    b, mask, y, amat, da = _gp(256, eta, 0.3)
    alpha0 = 2.0 / (1.0 + 2e-2)
    f, g, _ = ops.gp_objective_and_grad(amat(0.3), da, mask, y, 15, alpha0)
    h = 1e-4
    fp = ops.quadform(ops.newton_schulz(amat(0.3 + h), mask, 15, alpha0)[0], y)
    fm = ops.quadform(ops.newton_schulz(amat(0.3 - h), mask, 15, alpha0)[0], y)
    fd = (fp - fm) / (2 * h)
    assert abs(g - fd) < 1e-6 * abs(fd)


def test_gp_gradient_closed_form_full_pattern():
    # converged, unmasked: d/dl y^T A^{-1} y = -y^T A^{-1} A' A^{-1} y
    b, mask, y, amat, da = _gp(256, 1e9, 0.3)
    a = amat(0.3)
    f, g, res = ops.gp_objective_and_grad(a, da, mask, y, 30, 2.0 / (1.0 + 2e-2))
    ai = np.linalg.inv(a)
    assert res[-1] < 1e-12
    assert abs(f - y @ ai @ y) < 1e-10 * abs(f)
    assert abs(g - (-(y @ ai @ da @ ai @ y))) < 1e-9 * abs(g)


def test_sampled_rows_product_matches_full(cfg1_setup):
    mask, rp, col = cfg1_setup["mask_prior"], cfg1_setup["rp"], cfg1_setup["col"]
    a = np.where(mask, cfg1_setup["ks"], 0.0)
    full = native.masked_product_csr(rp, col, a[mask], a[mask])
    rows = np.array([0, 5, 64, 900, 2047])
    part, cnt = native.masked_product_rows(rows, rp, col, a[mask], a[mask])
    assert cnt == sum(rp[r + 1] - rp[r] for r in rows)
    for r in rows:
        assert np.array_equal(part[rp[r]:rp[r + 1]], full[rp[r]:rp[r + 1]])


def test_expm_taylor_full_pattern_is_library_expm():
    # With S = everything the formatted series is the plain truncated Taylor series of
    # exp(A); 20 terms at ||A||_2 <= 0.6 leave a remainder below 1e-20.
    import scipy.linalg
    rng = np.random.default_rng(3)
    n = 40
    a = rng.standard_normal((n, n))
    a *= 0.6 / np.linalg.norm(a, 2)
    full = np.ones((n, n), bool)
    e = ops.expm_taylor(a, full, 20)
    ref = scipy.linalg.expm(a)
    assert np.linalg.norm(e - ref) <= 1e-13 * np.linalg.norm(ref)
    # the series applied to a block agrees with the same library routine
    x = rng.uniform(size=(n, 10))
    assert np.linalg.norm(ops.expm_series_apply(a, x, 30) - ref @ x) <= 1e-13 * np.linalg.norm(ref @ x)
    # the error estimator of a scaled identity is the scale
    assert abs(ops.error_estimator(-2.5 * np.eye(n), x) - 2.5) < 1e-14


def test_expm_taylor_diagonal_and_block_patterns():
    import math

    import scipy.linalg
    rng = np.random.default_rng(4)
    n = 24
    # diagonal pattern: each entry is the scalar series of its own exponential
    d = rng.uniform(-0.5, 0.5, n)
    e = ops.expm_taylor(np.diag(d), np.eye(n, dtype=bool), 12)
    ref = np.array([sum(v ** j / math.factorial(j) for j in range(13)) for v in d])
    assert np.allclose(np.diag(e), ref, rtol=0, atol=1e-15) and np.count_nonzero(e - np.diag(np.diag(e))) == 0
    # block-diagonal pattern: blocks do not interact, each is its own exponential
    mask = np.zeros((n, n), bool)
    for b0, b1 in [(0, 5), (5, 14), (14, 24)]:
        mask[b0:b1, b0:b1] = True
    a = np.where(mask, rng.standard_normal((n, n)) * 0.1, 0.0)
    e = ops.expm_taylor(a, mask, 20)
    for b0, b1 in [(0, 5), (5, 14), (14, 24)]:
        blk = scipy.linalg.expm(a[b0:b1, b0:b1])
        assert np.linalg.norm(e[b0:b1, b0:b1] - blk) <= 1e-14 * np.linalg.norm(blk)
    assert np.count_nonzero(e[~mask]) == 0


def test_expm_taylor_error_on_compressed_kernel(cfg1_setup):
    # The paper's measure (Section 5): e_F(exp(K) X - E X) with exp(K) X from 30 terms
    # of the series applied to X.  K^eta (scaled by 1/N, so ||K||_2 <= 1) is
    # compressible: the truncation error falls with the terms until the compression
    # error is reached.
    pr = cfg1_setup
    mask = pr["mask_prior"]
    a = np.where(mask, pr["ks"], 0.0)
    x = np.random.default_rng(5).uniform(size=(a.shape[0], 10))
    ref = ops.expm_series_apply(a, x, 30)
    err = {t: np.linalg.norm(ref - ops.expm_taylor(a, mask, t) @ x) / np.linalg.norm(x) for t in (1, 3, 12)}
    print("e_F by terms:", {t: f"{v:.2e}" for t, v in err.items()})
    assert err[12] < err[3] < err[1]
    assert err[12] < 1e-6


def test_ns_sqrt_full_pattern_is_library_sqrtm():
    # S = everything: the coupled iteration converges to the principal square root and
    # its inverse (spectrum of A in (0, 2)); 30 iterations reach rounding level.
    import scipy.linalg
    rng = np.random.default_rng(6)
    n = 30
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = rng.uniform(0.05, 1.5, n)
    a = (q * lam) @ q.T
    y, z, res = ops.ns_sqrt(a, np.ones((n, n), bool), 30)
    r = scipy.linalg.sqrtm(a).real
    assert np.linalg.norm(y - r) <= 1e-12 * np.linalg.norm(r)
    assert np.linalg.norm(z - np.linalg.inv(r)) <= 1e-12 * np.linalg.norm(np.linalg.inv(r))
    assert res[-1] < 1e-13 and res[0] > res[5] > res[10]


def test_ns_sqrt_diagonal_and_block_patterns():
    import scipy.linalg
    rng = np.random.default_rng(7)
    n = 20
    d = rng.uniform(0.1, 1.8, n)
    y, z, _ = ops.ns_sqrt(np.diag(d), np.eye(n, dtype=bool), 40)
    assert np.allclose(np.diag(y), np.sqrt(d), rtol=1e-14, atol=0)
    assert np.allclose(np.diag(z), 1.0 / np.sqrt(d), rtol=1e-14, atol=0)
    mask = np.zeros((n, n), bool)
    blocks = [(0, 7), (7, 12), (12, 20)]
    a = np.zeros((n, n))
    for b0, b1 in blocks:
        mask[b0:b1, b0:b1] = True
        g = rng.standard_normal((b1 - b0, b1 - b0))
        a[b0:b1, b0:b1] = np.eye(b1 - b0) + 0.3 * (g + g.T) / np.sqrt(b1 - b0)
    assert np.linalg.norm(np.eye(n) - a, 2) < 1
    y, z, _ = ops.ns_sqrt(a, mask, 40)
    for b0, b1 in blocks:
        r = scipy.linalg.sqrtm(a[b0:b1, b0:b1]).real
        assert np.linalg.norm(y[b0:b1, b0:b1] - r) <= 1e-12 * np.linalg.norm(r)
    assert np.count_nonzero(y[~mask]) == 0 and np.count_nonzero(z[~mask]) == 0


def test_ns_sqrt_on_compressed_kernel(cfg1_setup):
    # A = K^eta + 1e-2 I (K scaled by 1/N): the masked iteration settles, and the
    # paper's measure e_F(Y Y - A) is small (the square root is compressible on S).
    pr = cfg1_setup
    mask = pr["mask_prior"]
    n = pr["n"]
    a = np.where(mask, pr["ks"], 0.0) + 1e-2 * np.eye(n)
    y, z, res = ops.ns_sqrt(a, mask, 16)
    x = np.random.default_rng(8).uniform(size=(n, 10))
    e_sq = ops.error_estimator(y @ y - a, x)
    print(f"residuals {res[0]:.2e} -> {res[-1]:.2e}; e_F(YY - A) = {e_sq:.2e}")
    assert res[-1] < 1e-3 * res[0]
    assert e_sq < 1e-4


def test_spmm_brute_force_tiny():
    # the oracle's S-matrix times block against an explicit triple loop over the pattern
    rng = np.random.default_rng(9)
    n, r = 9, 3
    mask = rng.uniform(size=(n, n)) < 0.4
    a = np.where(mask, rng.standard_normal((n, n)), 0.0)
    x = rng.standard_normal((n, r))
    y = np.zeros((n, r))
    for i in range(n):
        for k in range(n):
            if mask[i, k]:
                for c in range(r):
                    y[i, c] += a[i, k] * x[k, c]
    assert np.allclose(ops.spmm(a, x), y, rtol=1e-14, atol=1e-14)


def test_fst_orthogonal_and_vanishing_moments():
    # T is orthogonal (norms kept, T^T inverts it) and samplets have vanishing moments:
    # a polynomial of degree <= q has coefficients only on the root's scaling functions.
    import synth
    from oracle import samplets, tree
    pts = synth.points_cube(700, 2, 21)
    ot = tree.build_tree(pts, 12)
    ob = samplets.build_samplets(ot, 1)
    rng = np.random.default_rng(10)
    x = rng.standard_normal((700, 3))
    w = ops.fst(ob, x)
    assert np.allclose(np.linalg.norm(w, axis=0), np.linalg.norm(x, axis=0), rtol=1e-13)
    assert np.allclose(ops.ifst(ob, w), x, rtol=0, atol=1e-13)
    poly = 0.3 + 1.7 * pts[:, 0] - 0.9 * pts[:, 1]
    wp = ops.fst(ob, poly)
    assert int(ob.cluster_start[1]) >= ob.m  # the root's scaling functions come first
    assert np.max(np.abs(wp[ob.m:])) <= 1e-11 * np.linalg.norm(poly)
    assert np.linalg.norm(wp[:ob.m]) == pytest.approx(np.linalg.norm(poly), rel=1e-12)


def test_contour_rule_scalar_convergence():
    # The rule integrates lambda^{-1/2} = (2/pi) int_0^inf dw / (lambda + w^2) for every
    # lambda in [m, M], with an error falling exponentially in the number of nodes.
    m, M = 1e-2, 1.0
    lam = np.geomspace(m, M, 200)
    errs = []
    for nodes in (4, 8, 16):
        w2, c = ops.contour_invsqrt_rule(m, M, nodes)
        approx = (c[None, :] / (lam[:, None] + w2[None, :])).sum(axis=1)
        errs.append(np.max(np.abs(approx * np.sqrt(lam) - 1.0)))
    assert errs[0] > 10 * errs[1] > 100 * errs[2] and errs[2] < 1e-8
    # the printed "second kind" in place of the quarter period does not converge
    from scipy.special import ellipe, ellipj
    k2 = 1 - m / M
    t = ellipe(k2) * (np.arange(1, 17) - 0.5) / 16
    sn, cn, dn, _ = ellipj(t, k2)
    c2 = 2 * ellipe(k2) * np.sqrt(m) / (np.pi * 16) * dn / cn ** 2
    bad = (c2[None, :] / (lam[:, None] + (m * sn ** 2 / cn ** 2)[None, :])).sum(axis=1)
    assert np.max(np.abs(bad * np.sqrt(lam) - 1.0)) > 1e-2


def test_contour_invsqrt_full_pattern_is_library():
    # S = everything and converged shifted inverses: the library inverse square root,
    # up to the rule's error (16 nodes on [0.05, 1.5])
    import scipy.linalg
    rng = np.random.default_rng(11)
    n = 30
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = rng.uniform(0.05, 1.5, n)
    a = (q * lam) @ q.T
    x = ops.contour_invsqrt(a, np.ones((n, n), bool), 0.05, 1.5, 16, 40)
    ref = np.linalg.inv(scipy.linalg.sqrtm(a).real)
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)


@pytest.mark.parametrize("lam,nodes", [(0.3, 1), (2.0, 3), (1e-3, 7)])
def test_contour_rule_exact_at_unit_ratio(lam, nodes):
    # With lam_min = lam_max the parameter is 0, sn = sin, cn = cos, dn = 1 and the
    # quarter period is pi/2: c_k / (lam + w_k^2) = 1 / (nodes sqrt(lam)) for every
    # node, so the rule reproduces lam^{-1/2} exactly whatever the node count.
    w2, c = ops.contour_invsqrt_rule(lam, lam, nodes)
    assert np.sum(c / (lam + w2)) == pytest.approx(lam ** -0.5, rel=1e-14)
    t = (np.pi / 2) * (np.arange(nodes) + 0.5) / nodes
    np.testing.assert_allclose(w2, lam * np.tan(t) ** 2, rtol=1e-13)
