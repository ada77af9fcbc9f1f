"""S-format operations on dense arrays (zero outside the pattern).

* ``masked_product``: the formatted product (Section 4.1, Theorem (product),
  eq. (product)).  The paper stresses that it is exact on the compression
  pattern: c_ij = sum_k a_ik b_kj for (i, j) in S, where only k with
  (i, k) and (k, j) in S contribute because A and B vanish elsewhere.  The sum
  in eq. (product) runs over the samplets of all levels; it is read as running
  over all N basis indices, the root's scaling distributions included.
* ``axpy``: formatted addition (Section 4.1).
* ``newton_schulz``: X_0 = alpha I, Y = P_S(A X), Z = 2I - Y, X <- P_S(X Z).
  The paper inverts A = K + mu I by selected inversion (Section 4.2); its
  regularised-inverse lemma (eq. (perturbation)) shows the inverse is
  compressible on the pattern of K.  The iteration here keeps every iterate
  and every intermediate product on that pattern.
* ``ns_backward``: reverse mode of the iteration for f = y^T X_K y.
* ``error_estimator``: e_F(A) = ||A X||_F / ||X||_F with X in U[0,1]^{N x 10}
  (Section 5.1).
* ``expm_taylor``: the power series of the exponential (end of Section 4.4) cut
  after ``terms`` terms and evaluated in the S-format by Horner's rule, every
  product formatted: E = I, then E <- I + P_S(A E) / k for k = terms .. 1.  The
  paper does not fix the evaluation order of the series; Horner's rule is the
  reading taken here.
* ``expm_series_apply``: exp(A) X by the series applied to a block X without
  any pattern (the paper's reference for its exponential errors, Section 5.3,
  30 terms).
* ``fst`` / ``ifst``: the samplet transform of vectors, omega = T x with x in
  the points' original order (Section 3.2: the rows of T are the samplets'
  coefficient vectors over the points), and its inverse T^T (T is orthogonal).
* ``contour_invsqrt_rule`` / ``contour_invsqrt``: A^{-1/2} by the quadrature of
  Section 4.4 (eq. ContInt): A^{-1/2} ~ sum_k c_k (A + w_k^2 I)^{-1} with
  w_k = sqrt(m) sn(t_k)/cn(t_k), c_k = 2 Kq sqrt(m) dn(t_k) / (pi n cn(t_k)^2),
  t_k = Kq (k - 1/2) / n, Jacobi functions of parameter 1 - m/M, [m, M] the
  spectral bounds.  It is the midpoint rule for
  A^{-1/2} = (2/pi) int_0^inf (A + w^2 I)^{-1} dw after w = sqrt(m) sn/cn, which
  maps t in (0, Kq) onto w in (0, inf); so Kq is the quarter period, the complete
  elliptic integral of the first kind (the printed "second kind" is read as a
  garble).  Each shifted inverse is the masked Newton-Schulz iteration.
* ``spmm``: an S-matrix (zero outside the pattern) times a dense block, the
  product inside the error estimator e_F (Section 5.1).
* ``ns_sqrt``: coupled Newton-Schulz iteration for A^{1/2} and A^{-1/2} with
  every product formatted: Y_0 = A, Z_0 = I, T_k = (3I - P_S(Z_k Y_k)) / 2,
  Y_{k+1} = P_S(Y_k T_k), Z_{k+1} = P_S(T_k Z_k).  The paper computes the
  square root of a kernel matrix on the pattern by a contour integral, with its
  inverse square root lemma for compressibility (Section 4.4), and measures it
  by e_F(A^{1/2} A^{1/2} - A) (Section 5.3); this iteration, which converges for
  ||I - A|| < 1, stands in for the contour integral.
"""
from __future__ import annotations

import numpy as np


def masked_product(a: np.ndarray, b: np.ndarray, mask: np.ndarray) -> np.ndarray:
    return np.where(mask, a @ b, 0.0)


def axpy(alpha: float, x, beta: float, y: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """alpha X + beta Y on the pattern; X = None means the identity."""
    if x is None:
        x = np.eye(y.shape[0])
    return np.where(mask, alpha * x + beta * y, 0.0)


def residual(a: np.ndarray, x: np.ndarray, mask: np.ndarray) -> float:
    n = a.shape[0]
    e = np.eye(n) - masked_product(a, x, mask)
    return float(np.sqrt(np.sum(e * e)) / np.sqrt(n))


def newton_schulz(a: np.ndarray, mask: np.ndarray, iters: int, alpha0: float):
    """Returns (X_iters, residuals r_0..r_iters, iterates X_0..X_iters)."""
    n = a.shape[0]
    eye = np.eye(n)
    x = np.where(mask, alpha0 * eye, 0.0)
    xs = [x]
    res = []
    for _ in range(iters):
        y = masked_product(a, x, mask)
        e = eye - y
        res.append(float(np.sqrt(np.sum(e * e)) / np.sqrt(n)))
        z = np.where(mask, 2.0 * eye - y, 0.0)
        x = masked_product(x, z, mask)
        xs.append(x)
    res.append(residual(a, x, mask))
    return x, res, xs


def quadform(x: np.ndarray, y: np.ndarray) -> float:
    return float(y @ x @ y)


def ns_backward(a: np.ndarray, mask: np.ndarray, xs: list, xbar_final: np.ndarray) -> np.ndarray:
    """Adjoint of X_K(A) for the loss seed X_K-bar; returns A-bar on the pattern.

    Forward step k: Y_k = P(A X_k), Z_k = 2I - Y_k, X_{k+1} = P(X_k Z_k).
    The adjoint of C = P(U V) with respect to U is P(C-bar V^T) and with respect
    to V is P(U^T C-bar) (mask applied since only pattern entries are free).
    """
    n = a.shape[0]
    eye = np.eye(n)
    abar = np.zeros_like(a)
    xbar = xbar_final
    for k in range(len(xs) - 2, -1, -1):
        xk = xs[k]
        yk = masked_product(a, xk, mask)
        zk = np.where(mask, 2.0 * eye - yk, 0.0)
        xbar_k = masked_product(xbar, zk.T, mask)
        zbar = masked_product(xk.T, xbar, mask)
        ybar = -zbar
        abar += masked_product(ybar, xk.T, mask)
        xbar_k += masked_product(a.T, ybar, mask)
        xbar = xbar_k
    return abar


def gp_objective_and_grad(a: np.ndarray, da: np.ndarray, mask: np.ndarray, y: np.ndarray,
                          iters: int, alpha0: float):
    """f = y^T X_K(A) y and df/dl = <A-bar, dA/dl>_S."""
    xk, res, xs = newton_schulz(a, mask, iters, alpha0)
    f = quadform(xk, y)
    seed = np.where(mask, np.outer(y, y), 0.0)
    abar = ns_backward(a, mask, xs, seed)
    return f, float(np.sum(abar * da)), res


def column_local_inverse(a: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """The X with support S and P_S(A X) = I: column j solves A[S_j, S_j] x = e_j on S_j."""
    n = a.shape[0]
    x = np.zeros_like(a)
    for j in range(n):
        s = np.nonzero(mask[:, j])[0]
        rhs = (s == j).astype(np.float64)
        x[s, j] = np.linalg.solve(a[np.ix_(s, s)], rhs)
    return x


def error_estimator(a: np.ndarray, xprobe: np.ndarray) -> float:
    return float(np.linalg.norm(a @ xprobe) / np.linalg.norm(xprobe))


def expm_taylor(a: np.ndarray, mask: np.ndarray, terms: int) -> np.ndarray:
    """sum_{j <= terms} A^j / j! in the S-format (Horner, formatted products)."""
    n = a.shape[0]
    eye = np.eye(n)
    e = np.where(mask, eye, 0.0)
    for k in range(terms, 0, -1):
        e = np.where(mask, eye + masked_product(a, e, mask) / k, 0.0)
    return e


def expm_series_apply(a: np.ndarray, x: np.ndarray, terms: int = 30) -> np.ndarray:
    """sum_{j <= terms} A^j X / j!, the powers applied to X one at a time."""
    out = x.copy()
    t = x.copy()
    for j in range(1, terms + 1):
        t = a @ t / j
        out = out + t
    return out


def ns_sqrt(a: np.ndarray, mask: np.ndarray, iters: int):
    """Returns (Y, Z, residuals ||I - P_S(Z_k Y_k)||_F / sqrt(N) for k = 0..iters-1)."""
    n = a.shape[0]
    eye = np.eye(n)
    y = np.where(mask, a, 0.0)
    z = np.where(mask, eye, 0.0)
    res = []
    for _ in range(iters):
        w = masked_product(z, y, mask)
        res.append(float(np.linalg.norm(eye - w) / np.sqrt(n)))
        t = np.where(mask, 0.5 * (3.0 * eye - w), 0.0)
        y, z = masked_product(y, t, mask), masked_product(t, z, mask)
    return y, z, res


def spmm(a: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A X for an S-matrix A held dense (zero outside S) and a dense block X."""
    return a @ x


def fst(basis, x: np.ndarray) -> np.ndarray:
    """T x for x of shape (n,) or (n, r) in the points' original order."""
    return basis.sparse_T() @ x[basis.tree.perm]


def ifst(basis, w: np.ndarray) -> np.ndarray:
    """T^T w for w in basis order, returned in the points' original order."""
    out = np.empty_like(w)
    out[basis.tree.perm] = basis.sparse_T().T @ w
    return out


def contour_invsqrt_rule(m_lo: float, m_hi: float, nodes: int):
    """Shifts w_k^2 and weights c_k of the quadrature for A^{-1/2} on [m_lo, m_hi]."""
    from scipy.special import ellipj, ellipk
    k2 = 1.0 - m_lo / m_hi
    kq = ellipk(k2)
    t = kq * (np.arange(1, nodes + 1) - 0.5) / nodes
    sn, cn, dn, _ = ellipj(t, k2)
    w = np.sqrt(m_lo) * sn / cn
    c = 2.0 * kq * np.sqrt(m_lo) / (np.pi * nodes) * dn / cn ** 2
    return w ** 2, c


def contour_invsqrt(a: np.ndarray, mask: np.ndarray, m_lo: float, m_hi: float, nodes: int, ns_iters: int):
    """sum_k c_k X_k with X_k the masked Newton-Schulz inverse of A + w_k^2 I
    (X_0 = 2 / (m_lo + m_hi + 2 w_k^2) I, the inverse of the shifted bounds' midpoint)."""
    n = a.shape[0]
    eye = np.eye(n)
    out = np.zeros_like(a)
    for w2, c in zip(*contour_invsqrt_rule(m_lo, m_hi, nodes)):
        x, _, _ = newton_schulz(np.where(mask, a + w2 * eye, 0.0), mask, ns_iters, 2.0 / (m_lo + m_hi + 2.0 * w2))
        out = out + c * x
    return out
