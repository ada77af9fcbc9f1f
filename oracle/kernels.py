"""Matern kernels (Section 2, eq. (matern) and the explicit half-integer form).

For nu = p + 1/2 the paper gives

    k(r) = exp(-sqrt(2 nu) r / l) * p!/(2p)! * sum_{q=0}^{p} (p+q)!/(q! (p-q)!)
           * (sqrt(8 nu) r / l)^(p-q).

``matern(r, p, l)`` evaluates exactly that sum.  ``dmatern_dl`` is its
derivative with respect to the lengthscale l, obtained by differentiating the
same sum term by term (no closed form is assumed): with s = sqrt(2 nu) r / l
the sum is a polynomial P(s) in s, k = exp(-s) P(s), and
dk/dl = (ds/dl) (P'(s) - P(s)) exp(-s) with ds/dl = -s / l.
"""
from __future__ import annotations

from math import factorial

import numpy as np


def _poly_coeffs(p: int) -> np.ndarray:
    """Coefficients c_k of P(s) = sum_k c_k s^k with s = sqrt(2 nu) r / l.

    (sqrt(8 nu) r / l) = 2 s, so the term q contributes
    p!/(2p)! (p+q)!/(q!(p-q)!) 2^(p-q) s^(p-q).
    """
    c = np.zeros(p + 1)
    pref = factorial(p) / factorial(2 * p)
    for q in range(p + 1):
        k = p - q
        c[k] += pref * factorial(p + q) / (factorial(q) * factorial(p - q)) * 2.0 ** k
    return c


def matern(r: np.ndarray, p: int, ell: float) -> np.ndarray:
    """Matern kernel with nu = p + 1/2 at distances r (paper's half-integer form)."""
    nu = p + 0.5
    s = np.sqrt(2.0 * nu) * np.asarray(r, dtype=np.float64) / ell
    c = _poly_coeffs(p)
    poly = np.zeros_like(s)
    for k in range(p, -1, -1):
        poly = poly * s + c[k]
    return np.exp(-s) * poly


def dmatern_dl(r: np.ndarray, p: int, ell: float) -> np.ndarray:
    """d/dl of :func:`matern` at fixed r."""
    nu = p + 0.5
    s = np.sqrt(2.0 * nu) * np.asarray(r, dtype=np.float64) / ell
    c = _poly_coeffs(p)
    poly = np.zeros_like(s)
    dpoly = np.zeros_like(s)
    for k in range(p, -1, -1):
        poly = poly * s + c[k]
    for k in range(p, 0, -1):
        dpoly = dpoly * s + k * c[k]
    return (-s / ell) * (dpoly - poly) * np.exp(-s)


def pairwise_dist(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Euclidean distances between rows of x (n,d) and y (m,d)."""
    diff = x[:, None, :] - y[None, :, :]
    return np.sqrt(np.sum(diff * diff, axis=2))
