"""GPU parity of the reverse-mode path: torch.autograd over libspm's adjoints.

The masked-product adjoint, the Newton-Schulz reverse sweep and the GP
lengthscale gradient df/dl of f(l) = y^T X_K(K^eta(l) + mu I) y are compared
with the FP64 oracle (dense, on the pattern) and, for df/dl, with a central
difference of the GPU forward pass.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import compress, ops, pattern, samplets, tree

pytestmark = pytest.mark.gpu


def relerr(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


@pytest.fixture(scope="module")
def lib():
    from paper_2211_11681_amd import autograd, spm
    spm._lib.load()
    assert torch.cuda.is_available()
    return spm, autograd


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def problem(kind, n, leaf, q, eta, seed):
    pts = synth.workload_points(kind, n, seed)
    ot = tree.build_tree(pts, leaf)
    ob = samplets.build_samplets(ot, q)
    rp, col = pattern.entry_csr(ob, pattern.block_pattern(ot, eta))
    return pts, ob, rp, col, pattern.dense_mask(rp, col, n)


def test_masked_gemm_autograd(lib):
    print("case: autograd masked product n=1024 cube2 leaf16 eta1.0", flush=True)
    spm, ag = lib
    n = 1024
    _, ob, rp, col, mask = problem("cube2", n, 16, 1, 1.0, 11)
    pat = spm.Pattern.from_csr(n, rp, col, ob.cluster_start)
    i, j = np.nonzero(mask)
    a, b, g = (np.zeros((n, n)) for _ in range(3))
    a[i, j] = 2 * synth.pair_uniform(21, i, j, n) - 1
    b[i, j] = 2 * synth.pair_uniform(22, i, j, n) - 1
    g[i, j] = 2 * synth.pair_uniform(23, i, j, n) - 1
    A = pat.values_from_csr(to_dev(a[mask])).requires_grad_()
    B = pat.values_from_csr(to_dev(b[mask])).requires_grad_()
    G = pat.values_from_csr(to_dev(g[mask]))
    C = ag.MaskedGemm.apply(pat, A, B)
    C.backward(G)
    assert relerr(pat.values_to_csr(C.detach()).cpu().numpy(), ops.masked_product(a, b, mask)[mask]) < 1e-12
    assert relerr(pat.values_to_csr(A.grad).cpu().numpy(), ops.masked_product(g, b.T, mask)[mask]) < 1e-12
    assert relerr(pat.values_to_csr(B.grad).cpu().numpy(), ops.masked_product(a.T, g, mask)[mask]) < 1e-12


def test_newton_schulz_backward_vs_oracle(lib):
    print("case: NS reverse sweep n=1024 cube2 leaf16 eta1.0 matern32 l0.3 mu1e-2 K=10", flush=True)
    spm, ag = lib
    n, iters, mu = 1024, 10, 1e-2
    _, ob, rp, col, mask = problem("cube2", n, 16, 1, 1.0, 12)
    a = np.where(mask, compress.compress_dense(ob, 1, 0.3, 1.0 / n), 0.0) + mu * np.eye(n)
    alpha0 = 2.0 / (1.0 + 2.0 * mu)
    y = synth.normals(n, 112)
    seed = np.where(mask, np.outer(y, y), 0.0)
    _, _, xs = ops.newton_schulz(a, mask, iters, alpha0)
    abar_ref = ops.ns_backward(a, mask, xs, seed)
    pat = spm.Pattern.from_csr(n, rp, col, ob.cluster_start)
    A = pat.values_from_csr(to_dev(a[mask])).requires_grad_()
    X, res = ag.NewtonSchulz.apply(pat, A, iters, alpha0)
    assert relerr(pat.values_to_csr(X.detach()).cpu().numpy(), xs[-1][mask]) < 1e-12
    X.backward(pat.values_from_csr(to_dev(seed[mask])))
    err = relerr(pat.values_to_csr(A.grad).cpu().numpy(), abar_ref[mask])
    print(f"NS reverse sweep: relative error of A-bar {err:.3e}")
    assert err < 1e-11


@pytest.mark.parametrize("kind,n,leaf,seed", [("sphere", 2048, 32, 5), ("cube3", 1024, 16, 13)])
def test_gp_gradient_vs_oracle_and_fd(lib, kind, n, leaf, seed):
    print(f"case: GP gradient {kind} n={n} leaf{leaf} eta1.0 matern32 l0.3 mu1e-2 K=15", flush=True)
    spm, ag = lib
    p, ell, mu, iters, eta = 1, 0.3, 1e-2, 15, 1.0
    alpha0 = 2.0 / (1.0 + 2.0 * mu)
    pts, ob, rp, col, mask = problem(kind, n, leaf, 1, eta, seed)
    y = synth.normals(n, 100 + seed)
    # oracle: dense on the pattern
    a = np.where(mask, compress.compress_dense(ob, p, ell, 1.0 / n), 0.0) + mu * np.eye(n)
    da = np.where(mask, compress.compress_dense(ob, p, ell, 1.0 / n, deriv=True), 0.0)
    f_ref, g_ref, _ = ops.gp_objective_and_grad(a, da, mask, y, iters, alpha0)
    # library: tree, pattern and K^eta built on the GPU path
    t = spm.Tree(pts, leaf, 1)
    pat = spm.Pattern.from_tree(t, eta)
    yd = to_dev(y)
    f, g, res = ag.gp_quadform_and_grad(pat, t, p, ell, mu, yd, iters, alpha0, 1.0 / n)

    def forward(l):
        K = spm.kernel_compress(pat, t, p, l, 1.0 / n)
        spm.axpy(pat, mu, None, 1.0, K)
        X, _, _ = spm.newton_schulz(pat, K, iters, iters, "f64", alpha0)
        return float(spm.quadform(pat, X, yd))

    h = 1e-4
    g_fd = (forward(ell + h) - forward(ell - h)) / (2 * h)
    print(f"f {f:.15e} (oracle {f_ref:.15e}); df/dl {g:.12e} oracle {g_ref:.12e} FD {g_fd:.12e}; "
          f"final residual {float(res[-1]):.3e}")
    assert abs(f - f_ref) <= 1e-11 * abs(f_ref)
    assert abs(g - g_ref) <= 1e-10 * abs(g_ref)
    assert abs(g - g_fd) <= 1e-6 * abs(g)
