"""Pins of the oracle's construction side: synthetic inputs, kernels, tree,
samplets, pattern and compression, against facts the paper and mathematics fix."""
import numpy as np
import pytest
import scipy.linalg
import scipy.special

import synth
from oracle import compress, kernels, native, pattern, samplets, tree


# ---------------------------------------------------------------- synth
def test_splitmix64_reference_values():
    # splitmix64 seeded with state 0: the first outputs of the published generator
    # (state += 0x9E3779B97F4A7C15, then the mix function) are fixed numbers.
    state = np.uint64(0)
    outs = []
    for k in range(3):
        with np.errstate(over="ignore"):
            state = state + synth.GAMMA
        outs.append(int(synth._mix(np.array([state]))[0]))
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_synth_reproducible_and_in_range():
    a = synth.points_cube(1000, 3, 7)
    b = synth.points_cube(1000, 3, 7)
    assert np.array_equal(a, b)
    assert a.min() >= 0.0 and a.max() < 1.0
    s = synth.points_sphere(500, 3)
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-15)
    z = synth.normals(20000, 105)
    assert abs(z.mean()) < 0.03 and abs(z.std() - 1.0) < 0.03


def test_pair_uniform_torch_matches_numpy():
    import torch
    i = np.array([0, 1, 5, 77, 2047, 123456], dtype=np.int64)
    j = np.array([0, 3, 5, 1000, 2047, 99], dtype=np.int64)
    ref = synth.pair_uniform(205, i, j, 131072)
    got = synth.pair_uniform_torch(205, torch.from_numpy(i), torch.from_numpy(j), 131072).numpy()
    assert np.array_equal(ref, got)


# ---------------------------------------------------------------- kernels
@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_matern_half_integer_equals_bessel_form(p):
    # eq. (matern) with the modified Bessel function K_nu, evaluated by scipy
    nu, ell = p + 0.5, 0.37
    r = np.linspace(1e-3, 4.0, 50)
    z = np.sqrt(2 * nu) * r / ell
    ref = 2 ** (1 - nu) / scipy.special.gamma(nu) * z ** nu * scipy.special.kv(nu, z)
    assert np.allclose(kernels.matern(r, p, ell), ref, rtol=1e-12, atol=1e-15)
    assert kernels.matern(np.array([0.0]), p, ell)[0] == 1.0


def test_matern_closed_forms():
    r, ell = np.linspace(0, 2, 9), 0.3
    s3, s5 = np.sqrt(3) * r / ell, np.sqrt(5) * r / ell
    assert np.allclose(kernels.matern(r, 0, ell), np.exp(-r / ell), rtol=1e-14)
    assert np.allclose(kernels.matern(r, 1, ell), (1 + s3) * np.exp(-s3), rtol=1e-14)
    assert np.allclose(kernels.matern(r, 2, ell), (1 + s5 + s5 ** 2 / 3) * np.exp(-s5), rtol=1e-14)


@pytest.mark.parametrize("p", [0, 1, 2])
def test_matern_lengthscale_derivative_fd(p):
    r, ell, h = np.linspace(0.01, 2, 30), 0.45, 1e-5
    fd = (kernels.matern(r, p, ell + h) - kernels.matern(r, p, ell - h)) / (2 * h)
    assert np.allclose(kernels.dmatern_dl(r, p, ell), fd, rtol=1e-8, atol=1e-10)


def test_c_kernel_apply_matches_numpy():
    rng = np.random.default_rng(0)
    x, y, w = rng.random((300, 3)), rng.random((17, 3)), rng.standard_normal(17)
    for p in (0, 1, 2):
        for deriv in (False, True):
            f = kernels.dmatern_dl if deriv else kernels.matern
            ref = (f(kernels.pairwise_dist(x, y), p, 0.3) @ w) * 0.5
            got = native.kernel_apply(x, y, w, p, 0.3, 0.5, deriv)
            assert np.allclose(got, ref, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------- tree
@pytest.mark.parametrize("n,d,leaf", [(2048, 2, 16), (1000, 3, 32), (513, 2, 8)])
def test_cluster_tree_invariants(n, d, leaf):
    pts = synth.points_cube(n, d, 3)
    t = tree.build_tree(pts, leaf)
    assert np.array_equal(np.sort(t.perm), np.arange(n))
    assert t.start[0] == 0 and t.size[0] == n and t.parent[0] == -1
    for c in range(t.n_clusters):
        p = t.cluster_points(c)
        assert np.array_equal(p.min(axis=0), t.lo[c]) and np.array_equal(p.max(axis=0), t.hi[c])
        if t.is_leaf(c):
            assert t.size[c] <= leaf
            continue
        a, b = t.sons[c]
        # disjoint union, contiguous
        assert t.start[a] == t.start[c] and t.start[b] == t.start[a] + t.size[a]
        assert t.size[a] + t.size[b] == t.size[c] and t.size[a] == t.size[c] // 2
        assert t.level[a] == t.level[c] + 1 and t.parent[a] == c and t.parent[b] == c
        # median split along the longest box side
        ax = int(np.argmax(t.hi[c] - t.lo[c]))
        assert t.cluster_points(a)[:, ax].max() <= t.cluster_points(b)[:, ax].min()
    # level-major numbering
    assert np.all(np.diff(t.level) >= 0)
    if n == 2048:
        assert t.depth == 7 and np.all(t.size[t.sons[:, 0] < 0] == 16)


# ---------------------------------------------------------------- samplets
def test_householder_qr_equals_lapack():
    # LAPACK's dgeqrf/dorgqr use the same reflector convention (beta = -sign(alpha) ||x||),
    # so the full Q and R agree with scipy's up to rounding.
    rng = np.random.default_rng(1)
    for n, m in [(16, 3), (8, 4), (32, 6), (20, 10)]:
        a = rng.standard_normal((n, m))
        q, r = samplets.householder_qr(a)
        q2, r2 = scipy.linalg.qr(a, mode="full")
        assert np.allclose(q, q2, atol=1e-13) and np.allclose(r, r2, atol=1e-12)
        assert np.allclose(q @ r, a, atol=1e-13)
        assert np.allclose(np.tril(r, -1), 0.0, atol=1e-14)


@pytest.mark.parametrize("kind,n,leaf,q", [("cube2", 2048, 16, 1), ("cube3", 1024, 32, 1),
                                           ("cube2", 1024, 32, 2), ("sphere", 1024, 32, 1),
                                           ("cube2", 700, 16, 1)])
def test_samplet_basis_properties(kind, n, leaf, q):
    pts = synth.workload_points(kind, n, 5)
    t = tree.build_tree(pts, leaf)
    b = samplets.build_samplets(t, q)
    T = b.dense_T()
    # orthonormal basis (Theorem on samplet properties)
    assert np.abs(T @ T.T - np.eye(n)).max() < 1e-12
    # vanishing moments up to degree q, with raw (uncentred) monomials
    x = t.points[t.perm]
    exps = samplets.monomial_exponents(x.shape[1], q)
    mono = np.stack([np.prod(x ** np.array(a), axis=1) for a in exps], axis=1)
    m = len(exps)
    for c in range(t.n_clusters):
        rows = T[b.cluster_start[c]:b.cluster_start[c + 1]]
        if c == 0:
            rows = rows[m:]          # the root's scaling distributions have no vanishing moments
        if rows.shape[0] == 0:
            continue
        mom = rows @ mono
        scale = np.abs(rows).sum(axis=1)[:, None] * np.abs(mono).max(axis=0)[None, :]
        assert np.all(np.abs(mom) <= 1e-11 * scale)
        # ||omega||_1 <= sqrt(|nu|) (Theorem on samplet properties, item 4)
        assert np.all(np.abs(rows).sum(axis=1) <= np.sqrt(t.size[c]) * (1 + 1e-12))
    # samplet counts: m per internal cluster, |leaf| - m per leaf, 2m at the root
    nf = np.diff(b.cluster_start)
    leaves = t.sons[:, 0] < 0
    if np.all(t.size[leaves] > m):
        assert nf[0] == 2 * m
        assert np.all(nf[1:][~leaves[1:]] == m)
        assert np.all(nf[leaves] == t.size[leaves] - m)


def test_samplet_subspaces_match_lapack_qr():
    # The scaling/samplet split of each cluster is fixed by the moment matrix:
    # the samplet span is the orthogonal complement of range(M^T).  Rebuild it
    # cluster by cluster with LAPACK QR and compare orthogonal projectors.
    pts = synth.points_cube(512, 2, 9)
    t = tree.build_tree(pts, 16)
    b = samplets.build_samplets(t, 1)
    T = b.dense_T()
    x = t.points[t.perm]
    # level-J+1 functions for each cluster: scaling functions of the sons
    for c in range(1, t.n_clusters):
        rows = T[b.cluster_start[c]:b.cluster_start[c + 1]]
        s, sz = t.start[c], t.size[c]
        if rows.shape[0] == 0:
            continue
        sub = rows[:, s:s + sz]
        # samplets of c are orthogonal to all degree<=1 polynomials on c
        v = np.column_stack([np.ones(sz), x[s:s + sz]])
        qv, _ = scipy.linalg.qr(v, mode="economic")
        assert np.abs(sub @ qv).max() < 1e-12
        # and supported on c only
        assert np.abs(rows[:, :s]).max(initial=0) == 0 and np.abs(rows[:, s + sz:]).max(initial=0) == 0


# ---------------------------------------------------------------- pattern
def test_pattern_against_pointwise_definition(cfg1_setup):
    # Recompute the admissibility for every cluster pair from the point sets
    # themselves (boxes re-derived from points, pure Python loops).
    t, blocks = cfg1_setup["tree"], cfg1_setup["blocks"]
    nc = t.n_clusters
    boxes = [(t.cluster_points(c).min(0), t.cluster_points(c).max(0)) for c in range(nc)]
    import math
    for c in range(0, nc, 7):
        kept = set(blocks[c].tolist())
        for c2 in range(nc):
            (l1, h1), (l2, h2) = boxes[c], boxes[c2]
            g = [max(0.0, l2[a] - h1[a], l1[a] - h2[a]) for a in range(2)]
            dist = math.sqrt(g[0] * g[0] + g[1] * g[1])
            d1 = math.sqrt(sum((h1[a] - l1[a]) ** 2 for a in range(2)))
            d2 = math.sqrt(sum((h2[a] - l2[a]) ** 2 for a in range(2)))
            assert (dist < 1.6 * max(d1, d2)) == (c2 in kept)


def test_pattern_structure(cfg1_setup):
    t, blocks, rp, col = cfg1_setup["tree"], cfg1_setup["blocks"], cfg1_setup["rp"], cfg1_setup["col"]
    nc = t.n_clusters
    sets = [set(b.tolist()) for b in blocks]
    for c in range(nc):
        assert c in sets[c]
        for c2 in blocks[c]:
            assert c in sets[c2]                    # symmetric
        # ancestors have distance 0 and are always kept
        a = t.parent[c]
        while a >= 0:
            assert a in sets[c]
            a = t.parent[a]
    # admissibility is inherited by sons (what a pruned traversal relies on)
    for c in range(nc):
        for c2 in range(nc):
            if c2 not in sets[c] and not t.is_leaf(c2):
                for s in t.sons[c2]:
                    assert s not in sets[c]
    mask = pattern.dense_mask(rp, col, 2048)
    assert np.array_equal(mask, mask.T) and mask.diagonal().all()
    assert np.all(np.diff(col[rp[5]:rp[6]]) > 0)


def test_pattern_nnz_grows_like_n_log_n():
    # O(N log N) nonzeros (Corollary after Theorem (S-compression)): nnz/N grows
    # at most logarithmically as N doubles at fixed leaf size.
    ratios = []
    for n in (1024, 2048, 4096, 8192):
        t = tree.build_tree(synth.points_cube(n, 2, 11), 16)
        b = samplets.build_samplets(t, 1)
        blocks = pattern.block_pattern(t, 1.0)
        nf = np.diff(b.cluster_start)
        nnz = sum(nf[c] * nf[bl].sum() for c, bl in enumerate(blocks))
        ratios.append(nnz / n)
    inc = np.diff(ratios)
    assert np.all(inc > 0) and np.all(inc < 0.6 * np.array(ratios[:-1]))


# ---------------------------------------------------------------- compression
def test_compression_invariants(cfg1_setup):
    ks, b = cfg1_setup["ks"], cfg1_setup["basis"]
    K = compress.kernel_matrix(b, 1, 0.5, 1.0 / 2048)
    # orthogonal change of basis: trace and Frobenius norm are kept; tr K = k(0) = 1 with the 1/N scaling
    assert abs(np.trace(ks) - 1.0) < 1e-12
    assert abs(np.linalg.norm(ks) - np.linalg.norm(K)) < 1e-12 * np.linalg.norm(K)
    assert np.abs(ks - ks.T).max() < 1e-15
    # eigenvalues in [0, 1]
    ev = np.linalg.eigvalsh(K)
    assert ev.min() > -1e-12 and ev.max() <= 1.0 + 1e-12


def test_compression_error_decays_with_eta():
    t = tree.build_tree(synth.points_cube(1024, 2, 4), 16)
    b = samplets.build_samplets(t, 1)
    ks = compress.compress_dense(b, 0, 1.0, 1.0 / 1024)
    errs = []
    for eta in (0.5, 1.0, 2.0):
        rp, col = pattern.entry_csr(b, pattern.block_pattern(t, eta))
        m = pattern.dense_mask(rp, col, 1024)
        errs.append(np.linalg.norm(np.where(m, 0, ks)) / np.linalg.norm(ks))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-4


def test_compress_rows_matches_dense(cfg1_setup):
    b, ks = cfg1_setup["basis"], cfg1_setup["ks"]
    rows = np.array([0, 3, 7, 100, 500, 2047])
    got = compress.compress_rows(b, rows, 1, 0.5, 1.0 / 2048)
    assert np.abs(got - ks[rows]).max() < 1e-16 + 1e-12 * np.abs(ks).max()


def test_derivative_compression_fd():
    t = tree.build_tree(synth.points_cube(256, 2, 6), 16)
    b = samplets.build_samplets(t, 1)
    h = 1e-5
    d = compress.compress_dense(b, 1, 0.4, 1 / 256, deriv=True)
    fd = (compress.compress_dense(b, 1, 0.4 + h, 1 / 256) - compress.compress_dense(b, 1, 0.4 - h, 1 / 256)) / (2 * h)
    assert np.abs(d - fd).max() < 1e-8 * np.abs(d).max()
