"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds random-number generation only: no cluster tree, no samplet,
no kernel function and no matrix arithmetic of the method lives here.

Generator: splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) used as a counter-based generator.  Stream ``s``
starts from the state ``mix(s)`` and draw ``k`` of the stream is
``mix(mix(s) + (k + 1) * GAMMA)`` with ``GAMMA = 0x9E3779B97F4A7C15`` and the
splitmix64 output function ``mix``.  A draw becomes a double in [0, 1) as
``(x >> 11) * 2**-53``.

Workloads (the paper's experiments in its numerical-results section use
i.i.d. uniform points in the unit cube; a surface-like cloud stands in for the
scanned head, which is not available):

* ``points_cube(n, d, seed)``: point i, coordinate a takes draw ``i*d + a``.
* ``points_sphere(n, seed)``: three standard normals per point from the
  Box-Muller transform of draws ``4i .. 4i+3`` (the fourth normal is unused),
  normalised to unit length.
* ``normals(n, seed)``: Box-Muller normals, entry i from draws ``2i, 2i+1``.
* ``pair_uniform(seed, i, j, n)``: one uniform per matrix position (i, j) of an
  n x n matrix, draw ``i*n + j``.  Used for perturbations and for random
  operands on a pattern; it is evaluated elementwise, so any subset of entries
  can be produced without the rest.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_S30, _S27, _S31, _S11 = (np.uint64(s) for s in (30, 27, 31, 11))
_TWO_M53 = float(2.0 ** -53)


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> _S30)) * _M1
        z = (z ^ (z >> _S27)) * _M2
    return z ^ (z >> _S31)


def stream_key(seed: int) -> np.uint64:
    return _mix(np.array([seed], dtype=np.uint64))[0]


def draws_u64(seed: int, counters: np.ndarray) -> np.ndarray:
    """Raw 64-bit draws at the given counters of stream ``seed``."""
    key = stream_key(seed)
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = key + (c + np.uint64(1)) * GAMMA
    return _mix(state)


def uniform(seed: int, counters: np.ndarray) -> np.ndarray:
    """Doubles in [0, 1) at the given counters."""
    return (draws_u64(seed, counters) >> _S11).astype(np.float64) * _TWO_M53


def points_cube(n: int, d: int, seed: int) -> np.ndarray:
    """n points i.i.d. uniform in [0,1)^d, row-major (n, d) float64."""
    u = uniform(seed, np.arange(n * d, dtype=np.uint64))
    pts = u.reshape(n, d)
    _assert_distinct(pts)
    return pts


def _box_muller(u1: np.ndarray, u2: np.ndarray):
    r = np.sqrt(-2.0 * np.log(1.0 - u1))  # 1-u1 lies in (0, 1]
    t = 2.0 * np.pi * u2
    return r * np.cos(t), r * np.sin(t)


def normals(n: int, seed: int) -> np.ndarray:
    """n standard normal deviates (Box-Muller, first output of each pair)."""
    u = uniform(seed, np.arange(2 * n, dtype=np.uint64)).reshape(n, 2)
    z, _ = _box_muller(u[:, 0], u[:, 1])
    return z


def points_sphere(n: int, seed: int) -> np.ndarray:
    """n points uniform on the unit sphere S^2 in R^3 (normalised Gaussians)."""
    u = uniform(seed, np.arange(4 * n, dtype=np.uint64)).reshape(n, 4)
    z0, z1 = _box_muller(u[:, 0], u[:, 1])
    z2, _ = _box_muller(u[:, 2], u[:, 3])
    g = np.stack([z0, z1, z2], axis=1)
    nrm = np.sqrt(g[:, 0] * g[:, 0] + g[:, 1] * g[:, 1] + g[:, 2] * g[:, 2])
    pts = g / nrm[:, None]
    _assert_distinct(pts)
    return pts


def pair_uniform(seed: int, i: np.ndarray, j: np.ndarray, n: int) -> np.ndarray:
    """Uniform [0,1) value attached to matrix position (i, j) of an n x n matrix."""
    i = np.asarray(i, dtype=np.uint64)
    j = np.asarray(j, dtype=np.uint64)
    with np.errstate(over="ignore"):
        c = i * np.uint64(n) + j
    return uniform(seed, c)


def pair_uniform_torch(seed: int, i, j, n: int):
    """Same values as :func:`pair_uniform` computed with torch int64 tensors.

    Works on any torch device.  Unsigned 64-bit arithmetic is emulated on
    int64: products and sums wrap modulo 2**64, and logical right shifts mask
    off the sign-extended bits.
    """
    import torch

    def s64(v: int) -> int:
        v &= (1 << 64) - 1
        return v - (1 << 64) if v >= (1 << 63) else v

    def shr(x, s):
        return (x >> s) & ((1 << (64 - s)) - 1)

    def mix(z):
        z = (z ^ shr(z, 30)) * s64(0xBF58476D1CE4E5B9)
        z = (z ^ shr(z, 27)) * s64(0x94D049BB133111EB)
        return z ^ shr(z, 31)

    key = s64(int(stream_key(seed)))
    c = i.to(torch.int64) * n + j.to(torch.int64)
    state = key + (c + 1) * s64(int(GAMMA))
    x = mix(state)
    return shr(x, 11).to(torch.float64) * _TWO_M53


def _assert_distinct(pts: np.ndarray) -> None:
    """The method assumes mutually distinct points."""
    u = np.unique(pts, axis=0)
    if u.shape[0] != pts.shape[0]:
        raise ValueError("synthetic point set has coincident points")


# Workload recipes (point cloud, seed) used by tests and the benchmark.
def workload_points(kind: str, n: int, seed: int) -> np.ndarray:
    if kind == "cube2":
        return points_cube(n, 2, seed)
    if kind == "cube3":
        return points_cube(n, 3, seed)
    if kind == "sphere":
        return points_sphere(n, seed)
    raise ValueError(f"unknown point cloud {kind!r}")
