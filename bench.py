"""Benchmark of the S-format masked product on one MI355X.

Workload (the product benchmark of the paper's numerical results, Section 5.1, at
the million-point size the headline metric is quoted on): N = 1048576 points
i.i.d. uniform in the unit square [0,1]^2 (seed 3), Matern nu = 3/2 kernel with
lengthscale 0.1 scaled by 1/N, samplets with vanishing moments up to degree 2
(m = 6), leaf size 32, eta = 1.6.  K = P_S(T K T^T) is built on the device before
timing (O(N^2) construction, about a minute).

One step = the FP64 product C = P_S(K K) (spm_masked_gemm_ws, operands resident
in HBM).  After the timed FP64 steps the same product is timed in the two FP32
forms (F32SPLIT: hi/lo operands; F32ACC: hi-only operands), each with the same
number of warm-up and timed repetitions (F32SPLIT capped to about a minute of
work), and their relative Frobenius error is measured against the FP64 result
over every stored entry and against the FP64 oracle over sampled entries.

Output: one JSON line.  value = pattern entries of C per second of the FP64 step.
roofline: the product's algorithmic FP64 flops (2 x the exact multiply-adds over
the tile structure) per call divided by its average duration from HIP events on
the launch stream, against the dense FP64 MFMA peak; traffic = HBM bytes per call
from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (null once the
device code or schedule differs from the one the counters were taken on).
CPU leg (the only part of this file that runs the oracle, skipped with
--no-cpu-baseline): on the host cores, the FP64 oracle computes reference entries
of P_S(K K) for a sample of output positions (oracle_sample, the error of every form
against them), and its sorted-merge product is timed over a level-stratified sample
of output tiles and extrapolated to the whole product by exact multiply-adds
(cpu_baseline).

--workload product_cube3 runs the same measurement on N = 131072 points in the
unit cube (exponential kernel, l = 0.3, degree 1, leaf 32, eta = 1.0, seed 2),
one step being the FP64 product plus spm_axpy K + 0.1 I.
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

WORKLOAD = dict(workload="samplet_masked_product_square2d", n=1048576, dim=2, kernel="matern_nu1.5", matern_p=1,
                lengthscale=0.1, vanishing_moments_degree=2, leaf=32, eta=1.6, seed=3)
CUBE3 = dict(workload="samplet_masked_product_cube3", n=131072, dim=3, kernel="matern_nu0.5", matern_p=0,
             lengthscale=0.3, vanishing_moments_degree=1, leaf=32, eta=1.0, seed=2)

PEAK_FP64 = 78.6      # TFLOP/s, MI355X dense FP64 matrix (and vector) peak
PEAK_HBM = 8000.0     # GB/s
TRAFFIC_SUMMARIES = {"samplet_masked_product_square2d": "masked_product_square2d_n1048576_traffic.md",
                     "samplet_masked_product_cube3": "masked_product_cube3_n131072_traffic.md"}
SPLIT_BUDGET_S = 60.0  # timed work of one FP32 form is capped at about this long


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None, help="override N (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU leg (the oracle's reference entries and the CPU baseline)")
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--no-oracle-sample", action="store_true",
                    help="skip only the oracle's reference entries of the CPU leg")
    ap.add_argument("--split-modes", default="f32split,f32acc", help="comma-separated FP32 forms to time")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy K once (n_stored doubles read and written) so that "
                         "HBM counters can be scaled by a plain copy of known size")
    ap.add_argument("--workload", default="product",
                    choices=["product", "product_cube3", "newton_schulz", "gp_gradient", "expm", "ns_sqrt",
                             "contour", "matfun_tables"],
                    help="product (default): the masked product on the million-point square in FP64, F32SPLIT "
                         "and F32ACC; product_cube3: the same on N = 131072 in the unit cube; newton_schulz: 20 "
                         "masked Newton-Schulz iterations for (K + 1e-2 I)^-1 at N = 262144; gp_gradient: the GP "
                         "objective and its lengthscale gradient through 15 iterations (reverse mode), N from --n "
                         "(default 524288); expm: the truncated exponential series of K (10 terms) on the cube "
                         "workload; ns_sqrt: 12 coupled Newton-Schulz iterations for (K + 1e-2 I)^{+-1/2} on it; "
                         "contour: (K + 1e-2 I)^{-1/2} on it by a 6-node contour quadrature with 12 masked "
                         "Newton-Schulz iterations per shifted inverse; matfun_tables: the protocol of the paper's "
                         "square-root and exponential tables on a synthetic surface cloud")
    return ap.parse_args()


def host_cpu():
    """CPU model and logical CPU count of the host (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(ot, ob, eta, total_macs, nnz, threads, seed=77, clusters_per_level=6, tiles_per_cluster=256,
                 tile_cap=None):
    """The oracle's sorted-merge product timed on the host over a level-stratified
    sample of output tiles, extrapolated to the whole product by exact multiply-adds.

    Sample: for every tree level, `clusters_per_level` seeded clusters nu of that level,
    and for each `tiles_per_cluster` seeded tiles (nu, nu') of its block row (all of
    them when the row is shorter); every entry of the sampled tiles is computed by the
    oracle's C merge (c_ij = sum over k in S_i cap S_j of a_ik b_kj) on the rows of
    those clusters, with synthetic operand values (the pattern, not the values, sets
    the work).  The timed region is the merge alone.  The merge counts its own multiply-adds; the full product's time is
    extrapolated as total_macs / (sample multiply-adds per second), so the rate is
    that of a mix covering every level, the dense coarse rows included."""
    import numpy as np

    import synth
    from oracle import native, pattern

    cs = ob.cluster_start
    nf = np.diff(cs)
    lv = ot.level
    diam = pattern.diameters(ot)
    rng_u = lambda k, m: synth.uniform(seed * 1000 + k, np.arange(m))
    picked = []
    for L in range(int(lv.max()) + 1):
        at = np.nonzero((lv == L) & (nf > 0))[0]
        if len(at) == 0:
            continue
        sel = np.unique((rng_u(L, clusters_per_level) * len(at)).astype(np.int64))
        picked.extend(int(at[i]) for i in sel)
    rows_of = pattern.block_rows(ot, eta, picked, diam)
    tiles = []
    for k, nu in enumerate(picked):
        br = rows_of[nu]
        br = br[nf[br] > 0]
        if len(br) > tiles_per_cluster:
            br = br[np.unique((rng_u(100 + k, tiles_per_cluster) * len(br)).astype(np.int64))]
        tiles.extend((nu, int(c)) for c in br)
    if tile_cap is not None:
        tiles = tiles[:tile_cap]
    cols = sorted({c for _, c in tiles} - set(rows_of))
    # the block rows of the column clusters, in parallel slices (numpy releases the GIL)
    from concurrent.futures import ThreadPoolExecutor
    parts = [cols[k::threads] for k in range(threads) if cols[k::threads]]
    with ThreadPoolExecutor(max_workers=max(1, len(parts))) as ex:
        for r in ex.map(lambda part: pattern.block_rows(ot, eta, part, diam), parts):
            rows_of.update(r)
    # entry-level CSR of the rows the sample reads: rows of nu (A) and of nu' (B^T)
    need = sorted({nu for nu, _ in tiles} | {c for _, c in tiles})
    n = int(cs[-1])
    rowlen = np.zeros(n, np.int64)
    colsof = {}
    def basis_of(br):                       # basis indices of the clusters br, in order
        lens = nf[br]
        first = np.repeat(cs[br] - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
        return (first + np.arange(int(lens.sum()))).astype(np.int32)

    for c in need:
        cc = basis_of(rows_of[c])
        colsof[c] = cc
        rowlen[cs[c]:cs[c + 1]] = len(cc)
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum(rowlen)
    col = np.empty(rp[-1], np.int32)
    for c in need:                          # the rows of cluster c share one column list
        col[rp[cs[c]]:rp[cs[c + 1]]] = np.tile(colsof[c], int(nf[c]))
    # synthetic operand values in [-1, 1) (a fixed arithmetic sequence: the pattern, not
    # the values, sets the work of the merge)
    period_a, period_b = np.arange(65521, dtype=np.int64), np.arange(65519, dtype=np.int64)
    a = np.resize((period_a * 40503 % 65521) / 32760.5 - 1.0, int(rp[-1]))      # a_e = f(e mod 65521)
    bt = np.resize((period_b * 30011 % 65519) / 32759.5 - 1.0, int(rp[-1]))
    ii, jj, pos = [], [], []
    for nu, c in tiles:
        off = int(np.searchsorted(colsof[nu], cs[c]))           # first column of c in row nu's list
        i = np.repeat(np.arange(cs[nu], cs[nu + 1]), nf[c])
        j = np.tile(np.arange(cs[c], cs[c + 1]), int(nf[nu]))
        ii.append(i)
        jj.append(j)
        pos.append(rp[i] + off + (j - cs[c]))
    ii, jj, pos = np.concatenate(ii), np.concatenate(jj), np.concatenate(pos)
    out = np.zeros(rp[-1])
    used = native.set_threads(threads)
    t0 = time.perf_counter()
    macs = native.masked_product_entries(ii, jj, pos, rp, col, a, bt, out)
    dt = time.perf_counter() - t0
    rate = macs / dt
    t_full = total_macs / rate
    model, ncpu = host_cpu()
    levels = sorted({int(lv[nu]) for nu, _ in tiles})
    return {"value": nnz / t_full, "unit": "entries/s", "cores": used, "kind": "oracle", "extrapolated": True,
            "extrapolated_product_s": t_full, "macs_per_s": rate, "host_cpu": model, "host_logical_cpus": ncpu,
            "sample": f"{len(tiles)} output tiles ({len(ii)} entries, {macs} multiply-adds) of P_S(A B): "
                      f"{clusters_per_level} seeded clusters on each tree level {levels[0]}..{levels[-1]} and up to "
                      f"{tiles_per_cluster} seeded tiles of each one's block row, computed by the oracle's C "
                      f"sorted-merge product in {dt:.2f} s on {used} threads ({rate / 1e9:.3f} GMAC/s); the whole "
                      f"product ({total_macs:.4e} multiply-adds) extrapolated by exact multiply-adds to "
                      f"{t_full:.1f} s"}


def cpu_leg_sampled_entries(pts, w, leaves_at=(7, 2), levels=(13, 11)):
    """Oracle rows of K^eta = P_S(T K T^T) for a small sample of basis functions (the
    first and last function of two leaves and of their ancestors on the given levels),
    and the sampled pairs (i, j) of S with the reference entries
    c_ij = sum_{k in S_i cap S_j} K_ik K_jk of P_S(K K)."""
    import numpy as np

    from oracle import compress, pattern, samplets, tree

    ot = tree.build_tree(pts, w["leaf"])
    ob = samplets.build_samplets(ot, w["vanishing_moments_degree"])
    cs = ob.cluster_start
    n = int(cs[-1])
    nf = np.diff(cs)
    leaves = np.nonzero(ot.sons[:, 0] < 0)[0]
    chosen = []
    for k in leaves_at:
        c = int(leaves[len(leaves) // k])
        leaf = c
        while c >= 0:
            if c == leaf or int(ot.level[c]) in levels:
                chosen.append(c)
            c = int(ot.parent[c])
    rows = np.array(sorted({int(cs[c]) + k for c in set(chosen) for k in (0, int(nf[c]) - 1)}), np.int64)
    clus_of = np.searchsorted(cs, rows, side="right") - 1
    kr = compress.compress_rows(ob, rows, w["matern_p"], w["lengthscale"], 1.0 / n, use_c=True)
    diam = pattern.diameters(ot)
    masks = np.zeros((len(rows), n), bool)
    for a_, c in enumerate(clus_of):
        for b in pattern.block_row(ot, w["eta"], int(c), diam):
            masks[a_, cs[b]:cs[b + 1]] = True
    keta = np.where(masks, kr, 0.0)
    pairs = [(a_, b) for a_ in range(len(rows)) for b in range(len(rows)) if masks[a_, rows[b]]]
    ref = np.array([keta[a_] @ keta[b] for a_, b in pairs])
    ij = np.array([(rows[a_], rows[b]) for a_, b in pairs], np.int64)
    return ot, ob, ij, ref


def tile_positions(pat, cs, ij):
    """Element offsets of the basis pairs ij (m x 2) in the tile layout."""
    import numpy as np

    tr, tc, to = pat.tiles()
    nc = len(cs) - 1
    nf = np.diff(cs)
    tkey = tr.astype(np.int64) * nc + tc
    ci = np.searchsorted(cs, ij[:, 0], side="right") - 1
    cj = np.searchsorted(cs, ij[:, 1], side="right") - 1
    t = np.searchsorted(tkey, ci * nc + cj)
    assert np.all(tkey[t] == ci * nc + cj)
    return to[t] + (ij[:, 1] - cs[cj]) * nf[ci] + (ij[:, 0] - cs[ci])


def recorded_traffic(workload):
    """HBM bytes per product call from the committed rocprofv3 counter summary of the
    workload, or None when there is none or the kernels or the schedule builder have
    changed since the counters were taken."""
    import hashlib

    name = TRAFFIC_SUMMARIES.get(workload)
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
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
    each with the bulk in the FP32-split product or in F32ACC and the last 3 iterations
    in FP64."""
    import torch

    import synth
    from paper_2211_11681_amd import spm as S

    w = dict(NS_WORKLOAD)
    n = args.n or w["n"]
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
    for bulk in ("f64", "f32split", "f32acc"):
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
           "runs": runs, "speedup_f32split_bulk_vs_f64": runs["f64"]["ms"] / runs["f32split"]["ms"],
           "speedup_f32acc_bulk_vs_f64": runs["f64"]["ms"] / runs["f32acc"]["ms"]}
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
    n = args.n or w["n"]
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

    w = dict(CUBE3, workload="expm_taylor_cube3", terms=10)
    n = args.n or w["n"]
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

    w = dict(CUBE3, workload="ns_sqrt_cube3", mu=1e-2, iterations=12)
    n = args.n or w["n"]
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

    w = dict(CUBE3, workload="contour_invsqrt_cube3", mu=1e-2, nodes=6, ns_iterations=12)
    n = args.n or w["n"]
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
    if args.workload == "matfun_tables":
        return matfun_tables_main(args)
    if args.workload == "product_cube3":
        return product_main(args, dict(CUBE3), with_axpy=True)
    return product_main(args, dict(WORKLOAD), with_axpy=False)


def product_main(args, w, with_axpy):
    """The masked product P_S(K K) in FP64 (timed steps), then in the FP32 forms."""
    import numpy as np
    import torch

    import synth
    from paper_2211_11681_amd import spm as S

    n = args.n or w["n"]
    full = n == w["n"]
    w["n"] = n
    os.environ.setdefault("SPM_PROGRESS", "1")       # the O(N^2) construction reports its panels
    print(f"[bench] {w['workload']}: building tree, pattern and K for n={n}", file=sys.stderr, flush=True)
    pts = synth.points_cube(n, w["dim"], w["seed"])
    t0 = time.perf_counter()
    tree = S.Tree(pts, w["leaf"], w["vanishing_moments_degree"])
    pat = S.Pattern.from_tree(tree, w["eta"])
    t_plan = time.perf_counter() - t0
    print(f"[bench] tree, pattern and schedule {t_plan:.1f} s: tiles {pat.n_tiles} nnz {pat.nnz} "
          f"macs {pat.macs:.4e}", file=sys.stderr, flush=True)
    K = S.kernel_compress(pat, tree, w["matern_p"], w["lengthscale"], 1.0 / n)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    print(f"[bench] setup {t_setup:.1f} s", file=sys.stderr, flush=True)
    C = pat.empty("f64")
    Y = pat.empty("f64") if with_axpy else None
    ws = S.gemm_workspace(pat, "f64")
    stream = torch.cuda.current_stream()

    def product():
        S.masked_gemm(pat, K, K, out=C, workspace=ws)

    def step():
        product()
        if with_axpy:
            S.axpy(pat, 1.0, K, 0.0, Y)
            S.axpy(pat, 0.1, None, 1.0, Y)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for k in range(args.steps):
        ev[k][0].record(stream)
        product()
        ev[k][1].record(stream)
        if with_axpy:
            S.axpy(pat, 1.0, K, 0.0, Y)
            S.axpy(pat, 0.1, None, 1.0, Y)
    end.record(stream)
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(end)
    ms_step = ms_total / args.steps
    ms_gemm = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    if args.copy_calibration:
        Kc = K.clone()
        torch.cuda.synchronize()
        del Kc
    print(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step, product {ms_gemm:.3f} ms", file=sys.stderr, flush=True)
    del Y, ws

    flops = 2.0 * pat.macs
    tflops = flops / (ms_gemm * 1e-3) / 1e12
    # compulsory HBM bytes of one call: A and B (one array here, counted once) and C
    compulsory = 2 * pat.n_stored * 8
    traffic = recorded_traffic(w["workload"]) if full else None
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
        "config": dict(w, n_tiles=pat.n_tiles, nnz=pat.nnz, n_stored=pat.n_stored, macs_per_product=pat.macs,
                       step="FP64 product" + (" + axpy K + 0.1 I" if with_axpy else "")),
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": PEAK_FP64, "unit": "TFLOP/s",
                     "frac": tflops / PEAK_FP64, "traffic": traffic},
        "product_ms": ms_gemm,
        "product_compulsory_GBps": compulsory / (ms_gemm * 1e-3) / 1e9,
        "product_hbm_GBps": None if traffic is None else traffic / (ms_gemm * 1e-3) / 1e9,
        "setup_s": t_setup,
        "plan_s": t_plan,
        "classes": pat.classes(),
    }
    ref_norm = S.sqdist(pat, C).item() ** 0.5

    # CPU leg, first part: oracle rows for sampled entries (FP64 oracle on the host,
    # independent of the library)
    sample = None
    if full and not args.no_cpu_baseline and not args.no_oracle_sample:
        t1 = time.perf_counter()
        ot, ob, ij, ref = cpu_leg_sampled_entries(pts, w)
        pos = torch.from_numpy(tile_positions(pat, ob.cluster_start, ij)).cuda()
        got = C[pos].cpu().numpy()
        e64 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        sample = dict(ot=ot, ob=ob, ij=ij, ref=ref, pos=pos)
        out["oracle_sample"] = {"entries": len(ref), "largest_position": int(pos.max()),
                                "f64_rel_frobenius_err": e64, "s": time.perf_counter() - t1}
        print(f"[bench] oracle sample: {len(ref)} entries, FP64 rel err {e64:.3e} "
              f"({time.perf_counter() - t1:.1f} s)", file=sys.stderr, flush=True)

    if not args.no_split:
        # the FP32 operands are made from K once: hi/lo first, hi-only from the hi/lo copy
        # (fl32(hi + lo) = hi), so that K itself can be released before the split runs
        modes = [m for m in ("f32split", "f32acc") if m in args.split_modes.split(",")]
        Kcur, cur = K, "f64"
        del K
        for prec in modes:
            Ks = S.convert(pat, Kcur, cur, prec)
            del Kcur
            torch.cuda.empty_cache()
            Kcur, cur = Ks, prec
            Cs = pat.empty(prec)
            wsp = S.gemm_workspace(pat, prec)

            def prod_s():
                S.masked_gemm(pat, Ks, Ks, prec=prec, out=Cs, workspace=wsp)

            t_first = time.perf_counter()
            prod_s()                                                # first warm-up, sizes the repetitions
            torch.cuda.synchronize()
            t_first = time.perf_counter() - t_first
            reps = max(1, min(args.steps, int(SPLIT_BUDGET_S / max(t_first, 1e-3))))
            warm = max(0, min(args.warmup - 1, reps))
            for _ in range(warm):
                prod_s()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                prod_s()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            del wsp
            # error against the FP64 result over every stored entry, in the split format's
            # precision (FP64 -> hi/lo loses about 2^-48) or after widening FP32 to FP64
            if prec == "f32split":
                Cref = S.convert(pat, C, "f64", "f32split")
                err = S.sqdist(pat, Cs, Cref, prec="f32split").item() ** 0.5 / ref_norm
                del Cref
            else:
                C64 = S.convert(pat, Cs, prec, "f64")
                err = S.sqdist(pat, C64, C).item() ** 0.5 / ref_norm
                del C64
            res = {"product_ms": ms, "reps": reps, "entries_per_s": pat.nnz / (ms * 1e-3),
                   "speedup_vs_f64": ms_gemm / ms, "rel_frobenius_err_vs_f64": err}
            if sample is not None:
                hi = Cs[sample["pos"]].double()
                if prec == "f32split":
                    hi = hi + Cs[pat.n_stored + sample["pos"]].double()
                got = hi.cpu().numpy()
                res["rel_frobenius_err_vs_oracle_sample"] = float(np.linalg.norm(got - sample["ref"]) /
                                                                 np.linalg.norm(sample["ref"]))
            out[prec] = res
            del Ks, Cs
            torch.cuda.empty_cache()
            print(f"[bench] {prec}: {ms:.3f} ms x {reps}, rel err vs FP64 {err:.3e}", file=sys.stderr, flush=True)
        del Kcur
    # CPU leg, second part: the oracle's product timed on the host cores
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("SPM_CPU_THREADS", os.cpu_count() or 1))
        if sample is not None:
            ot, ob = sample["ot"], sample["ob"]
        else:
            from oracle import samplets, tree as otree
            ot = otree.build_tree(pts, w["leaf"])
            ob = samplets.build_samplets(ot, w["vanishing_moments_degree"])
        print(f"[bench] CPU baseline on {threads} threads", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(ot, ob, w["eta"], pat.macs, pat.nnz, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
