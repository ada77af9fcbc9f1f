"""Benchmark of the S-format masked product on one MI355X.

Workload (the product benchmark of the paper's numerical results, Section 5.1,
at the sizes of this build's headline configuration): N = 131072 points i.i.d.
uniform in the unit cube [0,1]^3 (seed 2), exponential kernel (Matern nu = 1/2)
with lengthscale 0.3 scaled by 1/N, samplets with vanishing moments up to
degree 1 (m = 4), leaf size 32, eta = 1.0.  K = P_S(T K T^T) is built on the
device before timing.

One step = the whole hot path on one batch of input:
    C = P_S(K K)            (spm_masked_gemm, FP64)
    Y = K + 0.1 I           (spm_axpy: copy of K, then the identity on the diagonal)

Output: one JSON line.  value = pattern entries of C per second (whole job,
inputs resident in HBM).  roofline: the product's algorithmic FP64 flops
(2 x the exact multiply-adds over the tile structure, F in the roofline model)
per call divided by its average duration from HIP events on the launch stream,
against the dense FP64 MFMA peak; traffic = HBM bytes per call from the
committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (null once the device code
differs from the one the counters were taken on).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = dict(workload="samplet_masked_product_cube3", n=131072, dim=3, kernel="matern_nu0.5", lengthscale=0.3,
                vanishing_moments_degree=1, leaf=32, eta=1.0, seed=2)

PEAK_FP64 = 78.6      # TFLOP/s, MI355X dense FP64 matrix (and vector) peak
PEAK_HBM = 8000.0     # GB/s
TRAFFIC_SUMMARY = "masked_product_cube3_n131072_traffic.md"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=WORKLOAD["n"], help="override N (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy K once (n_stored doubles read and written) so that "
                         "HBM counters can be scaled by a plain copy of known size")
    ap.add_argument("--workload", default="product",
                    choices=["product", "newton_schulz", "gp_gradient", "expm", "ns_sqrt", "contour", "product_2d",
                             "matfun_tables"],
                    help="product (default): the masked product benchmark; newton_schulz: 20 masked Newton-Schulz "
                         "iterations for (K + 1e-2 I)^-1 at N = 262144; gp_gradient: the GP objective and its "
                         "lengthscale gradient through 15 iterations (reverse mode), N from --n (default 524288); "
                         "expm: the truncated exponential series of K (10 terms) on the product workload; "
                         "ns_sqrt: 12 coupled Newton-Schulz iterations for (K + 1e-2 I)^{+-1/2} on it; "
                         "contour: (K + 1e-2 I)^{-1/2} on it by a 6-node contour quadrature with 12 masked "
                         "Newton-Schulz iterations per shifted inverse; product_2d: one product P_S(K K) at "
                         "N = 1048576 in the unit square (Matern-3/2, l = 0.1, q = 2, eta = 1.6) in FP64, F32ACC "
                         "and F32SPLIT, with the split modes' errors against FP64; matfun_tables: the protocol of "
                         "the paper's square-root and exponential tables on a synthetic surface cloud")
    return ap.parse_args()


def cpu_baseline(points, leaf, q, eta, threads):
    """Oracle's sorted-merge product timed on the host over a bounded row sample.

    Sample: all basis rows of 48 leaves spread evenly over the leaf order and of
    the middle cluster of every internal level from level 4 down (the rows of
    levels 0-3 are full and would dominate); their output entries
    c_ij = sum_{k in S_i cap S_j} a_ik b_kj are computed by the oracle's plain C
    merge with synthetic operand values (the pattern, not the values, sets the
    work)."""
    import numpy as np

    import synth
    from oracle import native, pattern, samplets, tree

    ot = tree.build_tree(points, leaf)
    ob = samplets.build_samplets(ot, q)
    blocks = pattern.block_pattern(ot, eta)
    cs = ob.cluster_start
    n = int(cs[-1])
    leaves = np.nonzero(ot.sons[:, 0] < 0)[0]
    lv = ot.level
    sample = [int(leaves[(2 * k + 1) * len(leaves) // 96]) for k in range(48)]
    for level in range(4, int(lv[leaves].min())):
        inner = np.nonzero((lv == level) & (ot.sons[:, 0] >= 0))[0]
        sample.append(int(inner[len(inner) // 2]))
    need = sorted(set(np.concatenate([blocks[c] for c in sample]).tolist()) | set(sample))
    rowlen = np.zeros(n, np.int64)
    cols_of = {}
    for c in need:
        cc = np.concatenate([np.arange(cs[b], cs[b + 1]) for b in blocks[c]]).astype(np.int32)
        cols_of[c] = cc
        rowlen[cs[c]:cs[c + 1]] = len(cc)
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum(rowlen)
    col = np.empty(rp[-1], np.int32)
    rows_i = np.repeat(np.arange(n), rowlen)
    for c in need:
        for i in range(cs[c], cs[c + 1]):
            col[rp[i]:rp[i + 1]] = cols_of[c]
    a = 2.0 * synth.pair_uniform(11, rows_i, col, n) - 1.0
    bt = 2.0 * synth.pair_uniform(12, col, rows_i, n) - 1.0      # bt[pos(j,k)] = b_kj
    rows = np.concatenate([np.arange(cs[c], cs[c + 1]) for c in sample])
    used = native.set_threads(threads)
    t0 = time.perf_counter()
    _, cnt = native.masked_product_rows_bt(rows, rp, col, a, bt)
    dt = time.perf_counter() - t0
    return {"value": cnt / dt, "unit": "entries/s", "cores": used, "kind": "oracle",
            "sample": f"all {len(rows)} basis rows of {len(sample)} clusters (48 leaves spread over the leaf "
                      f"order, the middle cluster of internal levels {[int(lv[c]) for c in sample[48:]]}): {cnt} output "
                      f"entries of P_S(A B) by the oracle's C sorted-merge product, synthetic operand values, "
                      f"{dt:.2f} s wall on {used} threads"}


def recorded_traffic():
    """HBM bytes per product call from the committed rocprofv3 counter summary, or
    None when the kernels or the schedule builder have changed since the counters
    were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    h = hashlib.sha256()
    for name in ("spm_device.hip", "spm_host.cpp"):     # kernels and the schedule they run
        with open(os.path.join(ROOT, "paper_2211_11681_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if fields.get("source_sha256") != h.hexdigest():
        return None
    return float(fields["hbm_bytes_per_product"])


NS_WORKLOAD = dict(workload="newton_schulz_cube3", n=262144, dim=3, kernel="matern_nu2.5", lengthscale=0.2,
                   vanishing_moments_degree=1, leaf=32, eta=1.0, seed=4, mu=1e-2, iterations=20, final_f64=3)
GP_WORKLOAD = dict(workload="gp_lengthscale_gradient_sphere", n=524288, kernel="matern_nu1.5", lengthscale=0.3,
                   vanishing_moments_degree=1, leaf=32, eta=1.0, seed=5, mu=1e-2, iterations=15, fd_step=1e-4)


def _timed(fn):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    out = fn()
    e1.record()
    torch.cuda.synchronize()
    return out, e0.elapsed_time(e1)


def newton_schulz_main(args):
    """Masked Newton-Schulz inverse of A = K + mu I: N = 262144 points in the unit cube
    (seed 4), Matern nu = 5/2, l = 0.2, scaled by 1/N, degree 1, leaf 32, eta = 1.0.
    20 iterations (40 products and the residual product), once all in FP64 and once
    with the bulk in F32ACC and the last 3 iterations in FP64."""
    import torch

    import synth
    from paper_2211_11681_amd import spm as S

    w = dict(NS_WORKLOAD)
    n = args.n if args.n != WORKLOAD["n"] else w["n"]
    w["n"] = n
    print(f"[bench] newton_schulz: building tree, pattern and K for n={n}", file=sys.stderr, flush=True)
    pts = synth.points_cube(n, w["dim"], w["seed"])
    t0 = time.perf_counter()
    tree = S.Tree(pts, w["leaf"], w["vanishing_moments_degree"])
    pat = S.Pattern.from_tree(tree, w["eta"])
    A = S.kernel_compress(pat, tree, 2, w["lengthscale"], 1.0 / n)
    S.axpy(pat, w["mu"], None, 1.0, A)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    alpha0 = 2.0 / (1.0 + 2.0 * w["mu"])
    runs = {}
    for bulk in ("f64", "f32acc"):
        S.newton_schulz(pat, A, 1, 1, bulk, alpha0)                    # warm-up (scratch, kernels)
        (X, res, _), ms = _timed(lambda: S.newton_schulz(pat, A, w["iterations"], w["final_f64"], bulk, alpha0))
        r = res.cpu().tolist()
        runs[bulk] = {"ms": ms, "ms_per_product": ms / (2 * w["iterations"] + 1), "residual_final": r[-1],
                      "residuals": r}
        print(f"[bench] NS bulk {bulk}: {ms:.1f} ms, final residual {r[-1]:.3e}", file=sys.stderr, flush=True)
        del X
    out = {"metric": "masked Newton-Schulz inverse, 20 iterations (41 products), final residual ||I - P_S(A X)||_F/sqrt(N)",
           "value": 1e3 / runs["f64"]["ms"], "unit": "inverses/s (all FP64)", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f64", "data": "synthetic",
           "config": dict(w, n_tiles=pat.n_tiles, nnz=pat.nnz, macs_per_product=pat.macs, setup_s=t_setup),
           "runs": runs, "speedup_f32acc_bulk_vs_f64": runs["f64"]["ms"] / runs["f32acc"]["ms"]}
    print(json.dumps(out), flush=True)


def gp_gradient_main(args):
    """f(l) = y^T X_15(K^eta(l) + mu I) y and df/dl by reverse mode through the 15
    Newton-Schulz iterations (per-iteration checkpoints), checked against a central
    difference of two further forward passes.  Points on the unit sphere (seed 5),
    Matern nu = 3/2, l = 0.3, scaled by 1/N, y ~ N(0, I) in samplet coordinates."""
    import torch

    import synth
    from paper_2211_11681_amd import autograd as AG
    from paper_2211_11681_amd import spm as S

    w = dict(GP_WORKLOAD)
    n = args.n if args.n != WORKLOAD["n"] else w["n"]
    w["n"] = n
    print(f"[bench] gp_gradient: building tree and pattern for n={n}", file=sys.stderr, flush=True)
    pts = synth.points_sphere(n, w["seed"])
    t0 = time.perf_counter()
    tree = S.Tree(pts, w["leaf"], w["vanishing_moments_degree"])
    pat = S.Pattern.from_tree(tree, w["eta"])
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    y = torch.from_numpy(synth.normals(n, 100 + w["seed"])).cuda()
    alpha0 = 2.0 / (1.0 + 2.0 * w["mu"])
    iters, ell, mu = w["iterations"], w["lengthscale"], w["mu"]
    (f, g, res), ms = _timed(lambda: AG.gp_quadform_and_grad(pat, tree, 1, ell, mu, y, iters, alpha0, 1.0 / n))

    def forward(l):
        K = S.kernel_compress(pat, tree, 1, l, 1.0 / n)
        S.axpy(pat, mu, None, 1.0, K)
        X, _, _ = S.newton_schulz(pat, K, iters, iters, "f64", alpha0)
        return float(S.quadform(pat, X, y))

    h = w["fd_step"]
    (fp, fm), ms_fd = _timed(lambda: (forward(ell + h), forward(ell - h)))
    g_fd = (fp - fm) / (2 * h)
    print(f"[bench] GP: f {f:.12e} df/dl {g:.12e} FD {g_fd:.12e}, {ms:.1f} ms", file=sys.stderr, flush=True)
    out = {"metric": "GP objective and lengthscale gradient through 15 Newton-Schulz iterations (reverse mode)",
           "value": 1e3 / ms, "unit": "gradients/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
           "data": "synthetic",
           "config": dict(w, n_tiles=pat.n_tiles, nnz=pat.nnz, macs_per_product=pat.macs, setup_s=t_setup),
           "ms_forward_and_backward": ms, "products": 2 * iters + 5 * iters,
           "f": f, "df_dl": g, "df_dl_central_difference": g_fd, "rel_diff_vs_fd": abs(g - g_fd) / abs(g),
           "residual_final": float(res[-1]), "ms_two_forward_passes_for_fd": ms_fd}
    print(json.dumps(out), flush=True)


def expm_main(args):
    """exp(K) by its power series cut after 10 terms, Horner's rule with formatted
    products, on the product benchmark's K (N = 131072 cube, exponential kernel)."""
    import numpy as np
    import torch

    import synth
    from paper_2211_11681_amd import spm as S

    w = dict(WORKLOAD, workload="expm_taylor_cube3", terms=10)
    n = args.n
    w["n"] = n
    print(f"[bench] expm: building tree, pattern and K for n={n}", file=sys.stderr, flush=True)
    pts = synth.points_cube(n, w["dim"], w["seed"])
    tree = S.Tree(pts, w["leaf"], w["vanishing_moments_degree"])
    pat = S.Pattern.from_tree(tree, w["eta"])
    K = S.kernel_compress(pat, tree, 0, w["lengthscale"], 1.0 / n)
    E = pat.empty("f64")
    S.expm_taylor(pat, K, 1, out=E)                                     # warm-up
    reps = max(1, args.steps // 2)
    _, ms = _timed(lambda: [S.expm_taylor(pat, K, w["terms"], out=E) for _ in range(reps)])
    ms /= reps
    print(f"[bench] expm: {ms:.1f} ms for {w['terms']} terms", file=sys.stderr, flush=True)
    # the paper's error measure (Section 5.3): e_F(exp(K) - E) with exp(K) X from 30 terms
    # of the series applied to a uniform block X of 10 columns
    X = torch.from_numpy(synth.uniform(91, np.arange(10 * n)).reshape(10, n)).cuda()
    ref, t = X.clone(), X
    for j in range(1, 31):
        t = S.spmm(pat, K, t) / j
        ref += t
    (approx,), ms_spmm = _timed(lambda: (S.spmm(pat, E, X),))
    e_f = float(torch.linalg.norm(ref - approx) / torch.linalg.norm(X))
    print(f"[bench] expm: e_F(exp(K) - E) = {e_f:.3e}", file=sys.stderr, flush=True)
    # fast samplet transform of the 10 probe vectors and back (point order <-> basis order);
    # the first call on a tree uploads its transform tables, so it is not timed
    S.fst(tree, X)
    (Wt,), ms_fst = _timed(lambda: (S.fst(tree, X),))
    (Xb,), ms_ifst = _timed(lambda: (S.fst(tree, Wt, inverse=True),))
    fst_rt = float(torch.linalg.norm(Xb - X) / torch.linalg.norm(X))
    out = {"metric": "truncated exponential series exp(K) on S, 10 terms (10 masked products)",
           "value": 1e3 / ms, "unit": "exponentials/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
           "data": "synthetic", "config": dict(w, n_tiles=pat.n_tiles, nnz=pat.nnz, macs_per_product=pat.macs),
           "ms": ms, "ms_per_product": ms / w["terms"], "e_F_vs_30_term_series": e_f, "ms_spmm_10_columns": ms_spmm,
           "ms_fst_10_vectors": ms_fst, "ms_inverse_fst_10_vectors": ms_ifst, "fst_round_trip_rel_err": fst_rt}
    print(json.dumps(out), flush=True)


def ns_sqrt_main(args):
    """(K + 1e-2 I)^{1/2} and its inverse by 12 coupled masked Newton-Schulz iterations
    (36 products) on the product benchmark's K (N = 131072 cube, exponential kernel)."""
    import numpy as np
    import torch

    import synth
    from paper_2211_11681_amd import spm as S

    w = dict(WORKLOAD, workload="ns_sqrt_cube3", mu=1e-2, iterations=12)
    n = args.n
    w["n"] = n
    print(f"[bench] ns_sqrt: building tree, pattern and K for n={n}", file=sys.stderr, flush=True)
    pts = synth.points_cube(n, w["dim"], w["seed"])
    tree = S.Tree(pts, w["leaf"], w["vanishing_moments_degree"])
    pat = S.Pattern.from_tree(tree, w["eta"])
    A = S.kernel_compress(pat, tree, 0, w["lengthscale"], 1.0 / n)
    S.axpy(pat, w["mu"], None, 1.0, A)
    S.ns_sqrt(pat, A, 1)                                              # warm-up
    (Y, Z, res), ms = _timed(lambda: S.ns_sqrt(pat, A, w["iterations"]))
    r = res.cpu().tolist()
    print(f"[bench] ns_sqrt: {ms:.1f} ms, residuals {r[0]:.3e} -> {r[-1]:.3e}", file=sys.stderr, flush=True)
    # the paper's measure (Section 5.3): e_F(Y Y - A), and e_F(Z Y - I) for the inverse
    X = torch.from_numpy(synth.uniform(92, np.arange(10 * n)).reshape(10, n)).cuda()
    YX = S.spmm(pat, Y, X)
    nx = torch.linalg.norm(X)
    e_sq = float(torch.linalg.norm(S.spmm(pat, Y, YX) - S.spmm(pat, A, X)) / nx)
    e_inv = float(torch.linalg.norm(S.spmm(pat, Z, YX) - X) / nx)
    print(f"[bench] ns_sqrt: e_F(YY - A) = {e_sq:.3e}, e_F(ZY - I) = {e_inv:.3e}", file=sys.stderr, flush=True)
    out = {"metric": "coupled Newton-Schulz square root and inverse square root on S, 12 iterations (36 products)",
           "value": 1e3 / ms, "unit": "square roots/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
           "data": "synthetic", "config": dict(w, n_tiles=pat.n_tiles, nnz=pat.nnz, macs_per_product=pat.macs),
           "ms": ms, "ms_per_product": ms / (3 * w["iterations"]), "residuals": r,
           "e_F_YY_minus_A": e_sq, "e_F_ZY_minus_I": e_inv}
    print(json.dumps(out), flush=True)


def contour_main(args):
    """(K + 1e-2 I)^{-1/2} by the contour quadrature of Section 4.4: 6 nodes, each a shifted
    inverse by 12 masked Newton-Schulz iterations (25 products per node), on the product
    benchmark's K (N = 131072 cube, exponential kernel)."""
    import numpy as np
    import torch

    import synth
    from paper_2211_11681_amd import spm as S

    w = dict(WORKLOAD, workload="contour_invsqrt_cube3", mu=1e-2, nodes=6, ns_iterations=12)
    n = args.n
    w["n"] = n
    print(f"[bench] contour: building tree, pattern and K for n={n}", file=sys.stderr, flush=True)
    pts = synth.points_cube(n, w["dim"], w["seed"])
    tree = S.Tree(pts, w["leaf"], w["vanishing_moments_degree"])
    pat = S.Pattern.from_tree(tree, w["eta"])
    A = S.kernel_compress(pat, tree, 0, w["lengthscale"], 1.0 / n)
    S.axpy(pat, w["mu"], None, 1.0, A)
    # spectral bounds: mu below (K is positive semi-definite), 1.05 x a power-iteration estimate above
    v = torch.from_numpy(synth.uniform(93, np.arange(n)).reshape(1, n)).cuda()
    for _ in range(40):
        v = S.spmm(pat, A, v)
        lam = float(torch.linalg.norm(v))
        v = v / lam
    lo, hi = w["mu"], 1.05 * lam
    w.update(lam_min=lo, lam_max=hi)
    S.contour_invsqrt(pat, A, lo, hi, 1, 1)                           # warm-up
    (Z, res), ms = _timed(lambda: S.contour_invsqrt(pat, A, lo, hi, w["nodes"], w["ns_iterations"]))
    r = res.cpu().tolist()
    print(f"[bench] contour: {ms:.1f} ms, node residuals {r}", file=sys.stderr, flush=True)
    # accuracy on a uniform probe block X of 10 columns: e_F(Z A Z - I)
    X = torch.from_numpy(synth.uniform(94, np.arange(10 * n)).reshape(10, n)).cuda()
    e_inv = float(torch.linalg.norm(S.spmm(pat, Z, S.spmm(pat, A, S.spmm(pat, Z, X))) - X) / torch.linalg.norm(X))
    print(f"[bench] contour: e_F(ZAZ - I) = {e_inv:.3e}", file=sys.stderr, flush=True)
    products = w["nodes"] * (2 * w["ns_iterations"] + 1)
    out = {"metric": "inverse square root on S by the contour quadrature (6 nodes x 12 Newton-Schulz iterations)",
           "value": 1e3 / ms, "unit": "inverse square roots/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f64", "data": "synthetic",
           "config": dict(w, n_tiles=pat.n_tiles, nnz=pat.nnz, macs_per_product=pat.macs),
           "ms": ms, "products": products, "ms_per_product": ms / products, "node_residuals": r,
           "e_F_ZAZ_minus_I": e_inv}
    print(json.dumps(out), flush=True)


PRODUCT_2D = dict(workload="samplet_masked_product_square2d", n=1048576, dim=2, kernel="matern_nu1.5",
                  lengthscale=0.1, vanishing_moments_degree=2, leaf=32, eta=1.6, seed=3)


def product_2d_main(args):
    """One product P_S(K K) on a million points in the unit square, in FP64 and in the
    two FP32 modes, with the relative Frobenius error of each mode against FP64."""
    import numpy as np
    import torch

    import synth
    from paper_2211_11681_amd import spm as S

    os.environ.setdefault("SPM_PROGRESS", "1")       # the O(N^2) construction reports its panels
    w = dict(PRODUCT_2D)
    n = args.n if args.n != WORKLOAD["n"] else w["n"]
    w["n"] = n
    print(f"[bench] product_2d: tree for n={n}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    pts = synth.points_cube(n, w["dim"], w["seed"])
    tree = S.Tree(pts, w["leaf"], w["vanishing_moments_degree"])
    print(f"[bench] product_2d: pattern and schedule ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    pat = S.Pattern.from_tree(tree, w["eta"])
    print(f"[bench] product_2d: {pat.n_tiles} tiles, {pat.nnz} entries ({time.perf_counter() - t0:.1f} s); "
          f"compressing K", file=sys.stderr, flush=True)
    K = S.kernel_compress(pat, tree, 1, w["lengthscale"], 1.0 / n)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    print(f"[bench] product_2d: setup {t_setup:.1f} s, {pat.macs:.3e} MACs per product", file=sys.stderr, flush=True)
    C = pat.empty("f64")
    S.masked_gemm(pat, K, K, out=C)                                   # warm-up
    reps = max(1, min(args.steps, 3))
    _, ms = _timed(lambda: [S.masked_gemm(pat, K, K, out=C) for _ in range(reps)])
    ms /= reps
    print(f"[bench] product_2d: FP64 {ms:.1f} ms", file=sys.stderr, flush=True)
    ref_norm = S.sqdist(pat, C).item() ** 0.5
    out = {"metric": "pattern entries/s of P_S(A*B) (FP64), with FP32 modes at stated relative error",
           "value": pat.nnz / (ms * 1e-3), "unit": "entries/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f64", "data": "synthetic",
           "config": dict(w, n_tiles=pat.n_tiles, nnz=pat.nnz, macs_per_product=pat.macs, setup_s=t_setup),
           "product_ms": ms, "algorithmic_TFLOPs": 2.0 * pat.macs / (ms * 1e-3) / 1e12}
    for prec in ("f32acc", "f32split"):
        Ks = S.convert(pat, K, "f64", prec)
        Cs = S.masked_gemm(pat, Ks, Ks, prec=prec)                    # warm-up (and the result)
        (_,), ms_p = _timed(lambda: (S.masked_gemm(pat, Ks, Ks, prec=prec, out=Cs),))
        del Ks
        C64 = S.convert(pat, Cs, prec, "f64")
        del Cs
        err = S.sqdist(pat, C64, C).item() ** 0.5 / ref_norm
        del C64
        torch.cuda.synchronize()
        out[prec] = {"product_ms": ms_p, "entries_per_s": pat.nnz / (ms_p * 1e-3), "speedup_vs_f64": ms / ms_p,
                     "rel_frobenius_err_vs_f64": err}
        print(f"[bench] product_2d: {prec} {ms_p:.1f} ms, rel err {err:.3e}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


MATFUN = dict(workload="matfun_tables_sphere", sizes=[5000, 10000, 50000, 100000], radius=0.5,
              kernel="matern_nu0.5", lengthscale=0.5, vanishing_moments_degree=2, leaf=32, eta=1.25, seed=21,
              mu=1e-4, lam_min=1e-4, lam_max=1.0, nodes=7, ns_iterations=24, exp_terms=8, exp_reference_terms=30,
              coupled_ns_iterations=30)


def matfun_tables_main(args):
    """The protocol of the paper's tables for the square root and the exponential
    (Section 5.3), on a synthetic stand-in for the scanned head: points on a sphere
    of radius 1/2 (a closed surface about one unit across), kernel exp(-2r)/N,
    mu = 1e-4, spectral bounds [mu, 1], seven quadrature nodes; the exponential by
    8 terms against 30 terms of the series applied to a uniform block X (N x 10).
    Degree q = 2 (three vanishing moments): the paper's q = 3 gives the root 40
    functions in 3D, more than a cluster may own here."""
    import numpy as np
    import torch

    import synth
    from paper_2211_11681_amd import spm as S

    os.environ.setdefault("SPM_PROGRESS", "1")       # the quadrature reports its nodes
    w = dict(MATFUN)
    rows = []
    t_all = time.perf_counter()
    for n in w["sizes"]:
        pts = w["radius"] * synth.points_sphere(n, w["seed"])
        tree = S.Tree(pts, w["leaf"], w["vanishing_moments_degree"])
        pat = S.Pattern.from_tree(tree, w["eta"])
        K = S.kernel_compress(pat, tree, 0, w["lengthscale"], 1.0 / n)
        A = K.clone()
        S.axpy(pat, w["mu"], None, 1.0, A)
        X = torch.from_numpy(synth.uniform(95, np.arange(10 * n)).reshape(10, n)).cuda()
        nx = float(torch.linalg.norm(X))
        # square root: A^{1/2} = P_S(A A^{-1/2}) with A^{-1/2} by the contour quadrature
        (Z, res), ms_c = _timed(lambda: S.contour_invsqrt(pat, A, w["lam_min"], w["lam_max"], w["nodes"],
                                                            w["ns_iterations"]))
        Y = S.masked_gemm(pat, A, Z)
        e_sqrt = float(torch.linalg.norm(S.spmm(pat, Y, S.spmm(pat, Y, X)) - S.spmm(pat, A, X))) / nx
        del Z, Y
        # the coupled Newton-Schulz square root on the same A
        (Yc, Zc, rc), ms_ns = _timed(lambda: S.ns_sqrt(pat, A, w["coupled_ns_iterations"]))
        e_ns = float(torch.linalg.norm(S.spmm(pat, Yc, S.spmm(pat, Yc, X)) - S.spmm(pat, A, X))) / nx
        del Yc, Zc
        # exponential: 8 terms in the S-format against 30 terms applied to X
        E, ms_e = _timed(lambda: S.expm_taylor(pat, K, w["exp_terms"]))
        ref, t = X.clone(), X
        for j in range(1, w["exp_reference_terms"] + 1):
            t = S.spmm(pat, K, t) / j
            ref += t
        e_exp = float(torch.linalg.norm(ref - S.spmm(pat, E, X))) / nx
        del E
        row = {"n": n, "nnz": pat.nnz, "e_F_sqrt_contour": e_sqrt, "ms_contour": ms_c,
               "node_residuals_max": float(res.max()), "e_F_sqrt_coupled_ns": e_ns, "ms_coupled_ns": ms_ns,
               "coupled_ns_final_residual": float(rc[-1]), "e_F_exp": e_exp, "ms_exp": ms_e}
        rows.append(row)
        print(f"[bench] matfun N={n}: e_F sqrt contour {e_sqrt:.3e} ({ms_c:.0f} ms), coupled NS {e_ns:.3e} "
              f"({ms_ns:.0f} ms), exp {e_exp:.3e} ({ms_e:.0f} ms)", file=sys.stderr, flush=True)
        del K, A, X, ref, t
        torch.cuda.empty_cache()
    out = {"metric": "errors e_F of the S-format square root (contour quadrature) and exponential, by N",
           "value": rows[-1]["e_F_sqrt_contour"], "unit": "e_F", "n_gpus": 1, "higher_is_better": False,
           "dtype": "f64", "data": "synthetic", "config": w, "rows": rows,
           "total_s": time.perf_counter() - t_all}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the product is not sharded "
              f"across GPUs.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_2211_11681_amd import spm as S

    S._lib.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "newton_schulz":
        return newton_schulz_main(args)
    if args.workload == "gp_gradient":
        return gp_gradient_main(args)
    if args.workload == "expm":
        return expm_main(args)
    if args.workload == "ns_sqrt":
        return ns_sqrt_main(args)
    if args.workload == "contour":
        return contour_main(args)
    if args.workload == "product_2d":
        return product_2d_main(args)
    if args.workload == "matfun_tables":
        return matfun_tables_main(args)
    n = args.n
    w = WORKLOAD
    print(f"[bench] building tree, pattern and K for n={n}", file=sys.stderr, flush=True)
    pts = synth.points_cube(n, w["dim"], w["seed"])
    t0 = time.perf_counter()
    tree = S.Tree(pts, w["leaf"], w["vanishing_moments_degree"])
    pat = S.Pattern.from_tree(tree, w["eta"])
    K = S.kernel_compress(pat, tree, 0, w["lengthscale"], 1.0 / n)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    print(f"[bench] setup {t_setup:.1f} s: tiles {pat.n_tiles} nnz {pat.nnz} macs {pat.macs:.3e}",
          file=sys.stderr, flush=True)
    C = pat.empty("f64")
    Y = pat.empty("f64")

    def step():
        S.masked_gemm(pat, K, K, out=C)
        S.axpy(pat, 1.0, K, 0.0, Y)
        S.axpy(pat, 0.1, None, 1.0, Y)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for k in range(args.steps):
        ev[k][0].record()
        S.masked_gemm(pat, K, K, out=C)
        ev[k][1].record()
        S.axpy(pat, 1.0, K, 0.0, Y)
        S.axpy(pat, 0.1, None, 1.0, Y)
    end.record()
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(end)
    ms_step = ms_total / args.steps
    ms_gemm = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    if args.copy_calibration:
        Kc = K.clone()
        torch.cuda.synchronize()
        del Kc
    print(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step, product {ms_gemm:.3f} ms", file=sys.stderr, flush=True)

    flops = 2.0 * pat.macs
    tflops = flops / (ms_gemm * 1e-3) / 1e12
    compulsory = 3 * pat.n_stored * 8          # A, B (here the same array, counted twice as operands) and C
    traffic = recorded_traffic() if n == WORKLOAD["n"] else None
    out = {
        "metric": "pattern entries/s of P_S(A*B) (FP64), with HBM GB/s and FP32-split at stated relative error",
        "value": pat.nnz / (ms_step * 1e-3),
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": dict(w, n=n, n_tiles=pat.n_tiles, nnz=pat.nnz, macs_per_product=pat.macs),
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": PEAK_FP64, "unit": "TFLOP/s",
                     "frac": tflops / PEAK_FP64, "traffic": traffic},
        "product_ms": ms_gemm,
        "product_compulsory_GBps": compulsory / (ms_gemm * 1e-3) / 1e9,
        "product_hbm_GBps": None if traffic is None else traffic / (ms_gemm * 1e-3) / 1e9,
        "setup_s": t_setup,
    }
    if not args.no_split:
        ref_norm = S.sqdist(pat, C).item() ** 0.5
        for prec in ("f32split", "f32acc"):
            Ks = S.convert(pat, K, "f64", prec)
            Cs = S.masked_gemm(pat, Ks, Ks, prec=prec)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = max(1, args.steps // 2)
            e0.record()
            for _ in range(reps):
                S.masked_gemm(pat, Ks, Ks, prec=prec, out=Cs)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            C64 = S.convert(pat, Cs, prec, "f64")
            err = S.sqdist(pat, C64, C).item() ** 0.5 / ref_norm
            out[prec] = {"product_ms": ms, "entries_per_s": pat.nnz / (ms * 1e-3), "speedup_vs_f64": ms_gemm / ms,
                         "rel_frobenius_err_vs_f64": err}
            del Ks, Cs, C64
            print(f"[bench] {prec}: {ms:.3f} ms, rel err {err:.3e}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("SPM_CPU_THREADS", min(16, os.cpu_count() or 1)))
        out["cpu_baseline"] = cpu_baseline(pts, w["leaf"], w["vanishing_moments_degree"], w["eta"], threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
