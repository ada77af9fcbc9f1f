"""FP64 CPU oracle for samplet (S-format) kernel matrix arithmetic.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or run anything in this package.
It shares no code with the GPU library (``paper_2211_11681_amd``); the only
code both sides use is the seeded input generator in ``synth``.

Everything here is written from the paper (Harbrecht, Multerer, Schenk,
Schwab, "Multiresolution kernel matrix algebra"): plain, slow, obviously
correct, float64 throughout.  Each function names the passage it follows.

Modules
  kernels   Matern kernels (Section 2, eq. (matern) and its half-integer form)
  tree      binary cluster tree (Section 3.2, Definition of a cluster tree)
  samplets  two-scale samplet construction (Section 3.2, eqs. (refinementRelation),
            (QR), (vanishingMomentsQR), (Wbasis))
  pattern   eta-admissibility compression pattern (Section 3.3, Theorem
            (S-compression), eq. (cutoff))
  compress  K^Sigma = T K T^T restricted to the pattern (Section 3.3)
  ops       formatted product exact on the pattern (Section 4.1, eq. (product)),
            formatted addition, Newton-Schulz on the pattern, adjoints, the
            Gaussian-process lengthscale gradient
  native    plain C helpers (entrywise sorted-merge product, kernel row sums)

Parity unpinned: none of the functions here lacks a pin; see
``tests/test_oracle_*.py`` for what pins each one.
"""
