"""Pins of the a-posteriori pattern (Section 5.1: entries of the compressed matrix
below a threshold tau in modulus are dropped) and of its CSR form.

The oracle's reading: the decision for (i, j) and (j, i) is taken once, on the
entry with i < j, by the strict test |v_ij| < tau; the diagonal is always kept;
only entries of the a-priori pattern can survive.  The checks below are written
as plain loops over every position (brute force) on small inputs built so that
each plausible slip changes the answer:
  - values exactly equal to tau (a non-strict test would drop them);
  - values that differ above and below the diagonal (a decision taken on the
    lower triangle, or per entry, would differ or break symmetry);
  - tiny diagonal values (dropping them loses the identity of the format).
On the smallest workload (N = 2048 unit square, Matern-3/2, tau = 1e-6) the
thresholded pattern is checked against the same definition entry by entry.
"""
import numpy as np

import synth
from oracle import pattern


def _brute_threshold(mask, values, tau):
    n = mask.shape[0]
    out = np.zeros_like(mask)
    for i in range(n):
        for j in range(n):
            if not mask[i, j]:
                continue
            if i == j:
                out[i, j] = True
                continue
            a, b = (i, j) if i < j else (j, i)
            out[i, j] = not (abs(values[a, b]) < tau)
    return out


def _brute_csr(mask):
    n = mask.shape[0]
    rp = [0]
    col = []
    for i in range(n):
        for j in range(n):
            if mask[i, j]:
                col.append(j)
        rp.append(len(col))
    return np.array(rp, np.int64), np.array(col, np.int32)


def _small_case(n, seed):
    """Symmetric a-priori mask with full diagonal; values that differ above and below
    the diagonal, a few exactly at tau, tiny diagonal values."""
    u = synth.uniform(seed, np.arange(n * n)).reshape(n, n)
    mask = (u + u.T) < 1.2
    mask[np.arange(n), np.arange(n)] = True
    tau = 0.25
    v = synth.uniform(seed + 1, np.arange(n * n)).reshape(n, n) - 0.5      # |v| < 0.5, not symmetric
    iu = np.triu_indices(n, 1)
    pick = synth.uniform(seed + 2, np.arange(len(iu[0]))) < 0.1
    v[iu[0][pick], iu[1][pick]] = tau * np.where(synth.uniform(seed + 3, np.arange(pick.sum())) < 0.5, 1.0, -1.0)
    v[np.arange(n), np.arange(n)] = 1e-9
    return mask, v, tau


def test_threshold_mask_matches_brute_force():
    for n, seed in ((7, 11), (24, 21), (57, 31)):
        mask, v, tau = _small_case(n, seed)
        got = pattern.threshold_mask(mask, v, tau)
        ref = _brute_threshold(mask, v, tau)
        assert np.array_equal(got, ref), (n, seed)
        # the construction exercises every branch of the definition
        iu = np.triu_indices(n, 1)
        assert np.any(mask[iu] & (np.abs(v[iu]) == tau))                     # kept at equality
        assert np.any(mask[iu] & (np.abs(v[iu]) < tau))                      # dropped
        assert np.any((np.abs(v) < tau) != (np.abs(v.T) < tau))             # triangle matters
        assert np.array_equal(got, got.T)
        assert np.all(got[np.arange(n), np.arange(n)])
        assert not np.any(got & ~mask)


def test_threshold_mask_decides_on_upper_triangle():
    n = 5
    mask = np.ones((n, n), bool)
    v = np.full((n, n), 1.0)
    v[3, 1] = 0.0            # below the diagonal only: must not drop (1, 3) or (3, 1)
    v[0, 4] = 0.0            # above the diagonal: drops (0, 4) and (4, 0)
    got = pattern.threshold_mask(mask, v, 0.5)
    assert got[1, 3] and got[3, 1]
    assert not got[0, 4] and not got[4, 0]
    assert got.sum() == n * n - 2


def test_csr_from_mask_matches_brute_force():
    for n, seed in ((1, 5), (9, 41), (40, 51)):
        mask, v, tau = _small_case(n, seed)
        m = pattern.threshold_mask(mask, v, tau)
        rp, col = pattern.csr_from_mask(m)
        rp_b, col_b = _brute_csr(m)
        assert rp.dtype == np.int64 and col.dtype == np.int32
        assert np.array_equal(rp, rp_b) and np.array_equal(col, col_b)
        assert np.array_equal(pattern.dense_mask(rp, col, n), m)


def test_cfg1_a_posteriori_pattern_definition(cfg1_setup):
    """N = 2048: subset of the a-priori pattern, symmetric, diagonal kept; every
    dropped off-diagonal pair has |K_ij| < tau (i < j) and every kept one |K_ij| >= tau."""
    s = cfg1_setup
    prior, post, ks, n = s["mask_prior"], s["mask_post"], s["ks"], s["n"]
    tau = 1e-6
    assert not np.any(post & ~prior)
    assert np.array_equal(post, post.T)
    assert np.all(post[np.arange(n), np.arange(n)])
    iu = np.triu_indices(n, 1)
    p_up, q_up, k_up = prior[iu], post[iu], np.abs(ks[iu])
    dropped = p_up & ~q_up
    kept = q_up
    assert dropped.sum() > 1000 and kept.sum() > 1000
    assert np.all(k_up[dropped] < tau)
    assert np.all(k_up[kept] >= tau)
    rp, col = pattern.csr_from_mask(post)
    assert rp[-1] == post.sum()
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(post[rows, col])
    for i in (0, 1, n // 2, n - 1):
        assert np.array_equal(col[rp[i]:rp[i + 1]], np.nonzero(post[i])[0])
