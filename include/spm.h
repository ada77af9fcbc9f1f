/*
 * spm.h -- samplet (S-format) kernel matrix arithmetic on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libspm.  Plain pointers and sizes only.  "host" arguments are read
 * (or written) before the call returns; "device" arguments are device memory
 * allocated by the caller (for instance torch tensors) and are accessed
 * asynchronously on the HIP stream passed as `stream` (NULL = the null stream).
 * Every function returns an spm_status; nothing aborts and no exception crosses
 * the boundary.  spm_last_error() gives a message for the last failure on the
 * calling thread.  Asynchronous kernel faults surface at the caller's next
 * synchronising call.
 *
 * Terms (Harbrecht, Multerer, Schenk, Schwab, "Multiresolution kernel matrix
 * algebra", Sections 3 and 4):
 *   cluster tree  binary tree of point clusters (Section 3.2, Definition of a
 *                 cluster tree); clusters are numbered level by level.
 *   basis         samplet basis (Section 3.2, eq. (Wbasis)): the root's scaling
 *                 distributions followed by every cluster's samplets.  Cluster c
 *                 owns the basis indices [cluster_start[c], cluster_start[c+1]).
 *   pattern S     compression pattern: the basis pairs whose clusters are not
 *                 eta-admissible (Section 3.3, eq. (cutoff)), optionally thinned
 *                 entry by entry (a-posteriori pattern, Section 5).  S must be
 *                 structurally symmetric and contain the diagonal.
 *   S-matrix      values on S stored in the library's tile layout: for every
 *                 block-row (cluster) c, the tiles (c, c') for c' in S_c in
 *                 ascending c', each a dense n_c x n_c' block stored
 *                 column-major (element (i, j) at j*n_c + i).  Length n_stored.
 *                 Positions that are inside a tile but outside S hold 0.
 *
 * Precision modes for value arrays:
 *   SPM_F64       double[n_stored]
 *   SPM_F32SPLIT  float hi[n_stored] followed by float lo[n_stored]
 *                 (x = hi + lo, hi = fl32(x), lo = fl32(x - hi)); arithmetic in
 *                 FP32 with error-free products and compensated sums.  The masked
 *                 product on a pattern planned with cluster levels (every cluster
 *                 size even, unit classes of at most 7 x 7 blocks of 16) runs on
 *                 the bf16 matrix cores instead: every row of op(A) and column of
 *                 op(B) is scaled, per tree level of the summation cluster, by a
 *                 power of two and cut into four 8-bit slices that bf16 holds
 *                 exactly; the products of slice pairs whose orders add up to at
 *                 most 5 are summed exactly in FP32 (integers below 2^24) and
 *                 added in FP64.  The dropped pairs and the last slice bound the
 *                 error by about 2^-32 of the product of the row and column
 *                 scales per term (measured relative Frobenius error against
 *                 FP64: 5e-10 to 8e-10).
 *   SPM_F32ACC    float hi[n_stored]; FP32 products.  The masked product sums
 *                 them in FP32 over a stage (at most 32 summation indices)
 *                 and adds the stage sums in FP64; tile classes the FP32
 *                 matrix-core kernel does not cover (more than 7 blocks of
 *                 16 rows on a side) use compensated FP32 sums instead.
 *                 Results are rounded to FP32.
 */
#ifndef SPM_H
#define SPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPM_OK = 0,
    SPM_EINVAL = -1,        /* bad argument: null pointer, size, aliasing, flag */
    SPM_EPATTERN = -2,      /* pattern fails validation */
    SPM_ENOMEM = -3,        /* host or device allocation failed */
    SPM_EHIP = -4,          /* a HIP runtime call or kernel launch failed */
    SPM_ENOTCONV = -5,      /* Newton-Schulz final residual non-finite or above the initial one */
    SPM_EUNSUPPORTED = -6   /* valid input outside what the kernels support */
} spm_status;

typedef enum { SPM_F64 = 0, SPM_F32SPLIT = 1, SPM_F32ACC = 2 } spm_prec;

typedef struct spm_tree_s *spm_tree;        /* host-side cluster tree + samplet basis */
typedef struct spm_pattern_s *spm_pattern;  /* device-side tiled pattern; immutable */

const char *spm_status_string(int status);
const char *spm_last_error(void);

/* ------------------------------------------------------------------------
 * Construction (host).  Section 3.2: cluster tree and two-scale samplet
 * construction; Section 3.3: eta-admissibility pattern.
 * ---------------------------------------------------------------------- */

/* Cluster tree of n points (host, row-major n x d, 1 <= d <= 3, mutually
 * distinct) by median splits along the longest bounding-box side until a
 * cluster has at most leaf_size points; samplets with vanishing moments up to
 * total degree q (Section 3.2, eqs. (QR), (vanishingMomentsQR)).  The handle
 * owns copies of everything it needs.  EINVAL for bad sizes; EUNSUPPORTED if a
 * cluster would own more than 32 basis functions (the kernels' tile limit). */
int spm_tree_build(const double *points, int64_t n, int32_t d, int32_t leaf_size, int32_t q,
                   spm_tree *out);
int spm_tree_destroy(spm_tree t);

/* n_clusters, depth (max level), m = number of monomials of degree <= q. */
int spm_tree_info(spm_tree t, int32_t *n_clusters, int32_t *depth, int32_t *m);

/* Host output arrays (any may be NULL): perm[n] (original index of the k-th
 * point in tree order), cluster_start[nc+1] (basis ranges), level[nc],
 * pt_start[nc], pt_size[nc] (point ranges in tree order). */
int spm_tree_arrays(spm_tree t, int64_t *perm, int64_t *cluster_start, int32_t *level,
                    int64_t *pt_start, int64_t *pt_size);

/* Block pattern of the eta-admissibility condition (Section 3.3, eq. (cutoff)):
 * cluster pairs (c, c') with dist(B_c, B_c') < eta * max(diam B_c, diam B_c'),
 * bounding boxes B, Euclidean diameter and gap distance.  Host outputs:
 * blk_row_ptr[nc+1]; blk_col[n_blocks] sorted per row (pass blk_col = NULL to
 * get n_blocks first). */
int spm_tree_block_pattern(spm_tree t, double eta, int64_t *blk_row_ptr, int32_t *blk_col,
                           int64_t *n_blocks);

/* ------------------------------------------------------------------------
 * Pattern upload: validation, tile layout, transpose map, schedule.
 * ---------------------------------------------------------------------- */

/* Entry-level pattern (host CSR, row_ptr[n+1] int64, col_idx sorted unique per
 * row) with cluster ranges cluster_start[n_clusters+1] (host, level order).
 * Tiles are the cluster pairs holding at least one entry; positions of a tile
 * outside S are masked.  EPATTERN if unsorted, duplicate, out of range,
 * unsymmetric, missing a diagonal entry, or cluster ranges do not tile [0, n). */
int spm_compress_pattern_upload(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                                int32_t n_clusters, const int64_t *cluster_start, void *stream,
                                spm_pattern *out);

/* Block pattern (host cluster-level CSR as from spm_tree_block_pattern); every
 * tile is full.  Same validation at cluster level. */
int spm_block_pattern_upload(int64_t n, int32_t n_clusters, const int64_t *cluster_start,
                             const int64_t *blk_row_ptr, const int32_t *blk_col, void *stream,
                             spm_pattern *out);

/* Planning without device memory, for callers that own the device memory (the upload
 * above is plan + spm_pattern_upload_workspace into a block the library allocates).
 * spm_block_pattern_plan / spm_compress_pattern_plan: the same validation, tile
 * layout, transpose map and schedule as the uploads, on the host only (EPATTERN,
 * EINVAL, EUNSUPPORTED as above).  cluster_level (host, n_clusters values in
 * [0, 64), or NULL): the tree level of every cluster.  With levels the plan also
 * holds a second copy of every unit's middle clusters, ordered level by level, with
 * stages of one level each: the split-precision product (SPM_F32SPLIT) scales its
 * operands per row and level and runs on that copy (the FP64 and F32ACC products
 * keep the first order); without levels SPM_F32SPLIT runs on the per-tile
 * compensated kernel.  The handle answers spm_pattern_info, spm_pattern_tiles,
 * spm_pattern_download_csr, spm_pattern_classes and spm_pattern_workspace_bytes;
 * every compute call on it returns EINVAL until it is uploaded.
 * spm_pattern_upload: device tables in a block the library allocates (freed by
 * spm_pattern_destroy).
 * spm_pattern_workspace_bytes: device bytes of the pattern's tables.
 * spm_pattern_upload_workspace: copies the tables into the caller's device memory ws
 * (at least that many bytes, 256-byte aligned); the pattern keeps pointers into ws,
 * which the caller keeps alive and unmodified until spm_pattern_destroy (which does
 * not free it).  Synchronous (blocking copies).  EINVAL on a short or misaligned
 * workspace or a pattern already uploaded. */
int spm_block_pattern_plan(int64_t n, int32_t n_clusters, const int64_t *cluster_start,
                           const int64_t *blk_row_ptr, const int32_t *blk_col, const int32_t *cluster_level,
                           spm_pattern *out);
int spm_compress_pattern_plan(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, int32_t n_clusters,
                              const int64_t *cluster_start, const int32_t *cluster_level, spm_pattern *out);
int spm_pattern_upload(spm_pattern p, void *stream);
int spm_pattern_workspace_bytes(spm_pattern p, size_t *bytes);
int spm_pattern_upload_workspace(spm_pattern p, void *ws, size_t bytes, void *stream);

/* Frees the host tables and, for patterns uploaded by spm_block_pattern_upload or
 * spm_compress_pattern_upload, the device tables. */
int spm_pattern_destroy(spm_pattern p);

/* nnz = |S|, n_stored = value-array length, n_tiles, macs = exact multiply-adds
 * of one product P_S(A B) over the tile structure (sum over output tiles (c,c')
 * of n_c n_c' sum_{mu in S_c cap S_c'} n_mu). */
int spm_pattern_info(spm_pattern p, int64_t *nnz, int64_t *n_stored, int64_t *n_tiles, double *macs);

/* Launch classes of the product schedule: units (pairs of groups of clusters) binned
 * by their size in 16-row blocks (row_blocks x col_blocks).  Per class: units,
 * output tiles, exact multiply-adds (the sum over its output tiles (c, c') of
 * n_c n_c' sum_{mu in S_c cap S_c'} n_mu, the cost in the proof of Theorem (product);
 * over all classes it is the macs of spm_pattern_info) and the multiply-adds the
 * FP64 kernels issue for it including padding, before skipping empty blocks.  Call
 * with all arrays NULL to get the count in *n_classes; otherwise *n_classes is the
 * capacity of the arrays (any may be NULL) and receives the count. */
int spm_pattern_classes(spm_pattern p, int32_t *n_classes, int32_t *row_blocks, int32_t *col_blocks,
                        int64_t *units, int64_t *out_tiles, double *exact_macs, double *padded_macs);

/* Host copies of the tile structure (any may be NULL): tile_row[n_tiles],
 * tile_col[n_tiles], tile_off[n_tiles] (element offset of each tile). */
int spm_pattern_tiles(spm_pattern p, int32_t *tile_row, int32_t *tile_col, int64_t *tile_off);

/* Entry-level CSR of S (host outputs, row_ptr[n+1], col_idx[nnz]). */
int spm_pattern_download_csr(spm_pattern p, int64_t *row_ptr, int32_t *col_idx);

/* Device conversions between CSR order (values of S row by row, nnz doubles)
 * and the tile layout (n_stored doubles; masked positions set to 0). */
int spm_values_from_csr(spm_pattern p, const double *csr_vals, double *vals, void *stream);
int spm_values_to_csr(spm_pattern p, const double *vals, double *csr_vals, void *stream);

/* ------------------------------------------------------------------------
 * Compression on the device (Section 3.3): vals = P_S(T K T^T) with
 * K = scale * [k(|x_i - x_j|)] the Matern kernel nu = matern_p + 1/2 of
 * lengthscale ell (deriv = 1: its derivative in ell) at the tree's points.
 * The pattern must have been built on the same tree's cluster ranges.
 * Exact O(N^2) evaluation by a two-sided fast samplet transform in panels;
 * temporary device memory is allocated and freed inside: one panel of rows of
 * at most 16 GB, plus the scaling rows of the panel roots kept for the levels
 * above them, at the tree level where the two together are smallest (42 GB at
 * N = 2^20 in 2D).  Synchronises the stream before returning.  With the
 * environment variable SPM_PROGRESS set, reports every tenth of its panels on
 * stderr.  ENOMEM when the temporaries cannot be allocated.
 * ---------------------------------------------------------------------- */
int spm_kernel_compress(spm_pattern p, spm_tree t, int32_t matern_p, double ell, double scale,
                        int32_t deriv, double *vals, void *stream);

/* ------------------------------------------------------------------------
 * Arithmetic on S-matrices (device value arrays of one pattern).
 * ---------------------------------------------------------------------- */

/* C = P_S(op(A) op(B)), op(X) = X or X^T (Section 4.1, Theorem (product),
 * eq. (product)): for every (i,j) in S, c_ij = sum_k op(A)_ik op(B)_kj, the sum
 * over the k with (i,k) and (k,j) in S, exact on the pattern.  A, B, C in
 * precision `prec`; C must not alias A or B (EINVAL).  Takes its workspace
 * (transposed operand copies) from the stream-ordered allocator (hipMallocAsync). */
int spm_masked_gemm(spm_pattern p, int prec, const void *A, int transA, const void *B, int transB,
                    void *C, void *stream);

/* The same product with the workspace supplied by the caller: ws (device, 256-byte
 * aligned, not overlapping A, B or C) of at least spm_masked_gemm_workspace() bytes
 * for the same precision and transpose flags (0 bytes: ws may be NULL).  Nothing is
 * allocated; ws may be reused once the call's work on the stream has completed.
 * EINVAL on a short, misaligned or overlapping workspace. */
int spm_masked_gemm_workspace(spm_pattern p, int prec, int transA, int transB, size_t *bytes);
int spm_masked_gemm_ws(spm_pattern p, int prec, const void *A, int transA, const void *B, int transB,
                       void *C, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same product with its
 * workspace in a fixed device array of the library, spm_masked_gemm_noalloc_max_bytes()
 * bytes (64 MiB) on every device it runs on, held until the process ends.  Nothing
 * is allocated.  EINVAL when the product needs more workspace than that (the value
 * arrays of the pattern are then too large: use spm_masked_gemm_ws).  Every call on
 * one device shares that device's array, so calls that overlap on one GPU (on
 * different streams, or from several threads) race; calls ordered on one stream are
 * safe.  The array's contents are left from the last call; each call overwrites the
 * part it uses before reading it. */
int spm_masked_gemm_noalloc_max_bytes(size_t *bytes);
int spm_masked_gemm_noalloc(spm_pattern p, int prec, const void *A, int transA, const void *B, int transB,
                            void *C, void *stream);

/* Adjoint of C = P_S(A B) (one pattern for all operands):
 * dA = P_S(dC B^T), dB = P_S(A^T dC).  dA or dB may be NULL to skip it.
 * spm_masked_gemm_backward allocates its workspace like spm_masked_gemm;
 * spm_masked_gemm_backward_ws takes it from the caller (at least
 * spm_masked_gemm_backward_workspace() bytes, rules as for spm_masked_gemm_ws). */
int spm_masked_gemm_backward(spm_pattern p, int prec, const void *dC, const void *A, const void *B,
                             void *dA, void *dB, void *stream);
int spm_masked_gemm_backward_workspace(spm_pattern p, int prec, size_t *bytes);
int spm_masked_gemm_backward_ws(spm_pattern p, int prec, const void *dC, const void *A, const void *B,
                                void *dA, void *dB, void *ws, size_t ws_bytes, void *stream);

/* Y = alpha X + beta Y on the stored values (formatted addition, Section 4.1);
 * X = NULL stands for the identity (only the diagonal of Y changes). */
int spm_axpy(spm_pattern p, int prec, double alpha, const void *X, double beta, void *Y, void *stream);

/* Precision conversion between value arrays (F64 -> split rounds to nearest;
 * split -> F64 is exact). */
int spm_convert(spm_pattern p, int prec_from, const void *X, int prec_to, void *Y, void *stream);

/* Deterministic FP64 reductions (fixed order, no atomics); result written to
 * the device double *out.
 *   spm_sqdist      sum_e (x_e - y_e)^2 over stored values (Y = NULL: sum x_e^2)
 *   spm_sqdist_eye  || alpha I - X ||_F^2 over S
 *   spm_dot         <X, Y>_S = sum_e x_e y_e
 *   spm_quadform    y^T X y, y a device vector of length n in basis order  */
int spm_sqdist(spm_pattern p, int prec, const void *X, const void *Y, double *out, void *stream);
int spm_sqdist_eye(spm_pattern p, int prec, double alpha, const void *X, double *out, void *stream);
int spm_dot(spm_pattern p, const double *X, const double *Y, double *out, void *stream);
int spm_quadform(spm_pattern p, const double *X, const double *y, double *out, void *stream);

/* X = alpha P_S(y y^T) (the seed of the quadratic-form adjoint). */
int spm_fill_outer(spm_pattern p, double alpha, const double *y, double *X, void *stream);

/* Truncated power series of exp(A) on S (the exponential's series at the end of
 * Section 4.4; its errors are reported in Section 5.3), FP64, by Horner's rule with
 * formatted products:
 *   E = I;  for k = terms, ..., 1:  E <- I + P_S(A E) / k,
 * so that on the full pattern E = sum_{j <= terms} A^j / j!.  A and E are device
 * F64 value arrays (distinct); terms >= 0 (0 gives E = I).  scratch: device
 * workspace of at least spm_expm_taylor_scratch() bytes (one value array), unused
 * when terms = 0; 256-byte aligned; it includes the products' workspace, so nothing
 * is allocated.  Asynchronous on the stream; EINVAL on null or overlapping
 * buffers, a negative term count or a short or misaligned scratch. */
int spm_expm_taylor_scratch(spm_pattern p, size_t *bytes);
int spm_expm_taylor(spm_pattern p, const double *A, double *E, int32_t terms, void *scratch,
                    size_t scratch_bytes, void *stream);

/* Fast samplet transform of r vectors (Section 3.2, the transform T of
 * K^Sigma = T K T^T): inverse = 0 gives Y = T X with X in the points' original
 * order and Y in basis order; inverse = 1 gives Y = T^T X (T is orthogonal) with X
 * in basis order and Y in the original order (r = 0 does nothing; X and Y may then
 * be null).  X, Y: distinct device F64 arrays,
 * r x n row-major (vector j at offset j n).  Uses a stream-ordered temporary of
 * r n doubles and the tree's transform tables, which the first call on a tree
 * uploads (synchronously) and the tree keeps until spm_tree_destroy; later calls
 * are asynchronous on the stream.  EINVAL on null or overlapping buffers or r < 0;
 * ENOMEM when the tables or the temporary cannot be allocated. */
int spm_fst(spm_tree t, const double *X, int32_t r, double *Y, int32_t inverse, void *stream);

/* Y = A X: an S-matrix A (device F64 value array) times a dense block X of r
 * columns, the product of the paper's error estimator e_F(A) = ||A X||_F / ||X||_F
 * (Section 5.1).  X and Y: device F64, column-major n x r (column j at offset
 * j n), rows in basis order; Y must not overlap A or X.  Each block row of Y is
 * summed by one workgroup in a fixed order (deterministic run to run); X is read
 * in passes of 16 columns.  r = 0 does nothing (X and Y may then be null).
 * Asynchronous on the stream;
 * EINVAL on null or overlapping buffers, r < 0, or n >= 2^25 (32-bit offsets). */
int spm_spmm(spm_pattern p, const double *A, const double *X, int32_t r, double *Y, void *stream);

/* Coupled Newton-Schulz iteration for the square root and the inverse square root
 * of A on S (the matrix square root of Section 4.4, whose errors Section 5.3
 * reports), FP64, every product formatted:
 *   Y_0 = A,  Z_0 = I;  for k = 0..iters-1:  W_k = P_S(Z_k Y_k),
 *   r_k = ||I - W_k||_F / sqrt(n),  T_k = (3I - W_k) / 2,
 *   Y_{k+1} = P_S(Y_k T_k),  Z_{k+1} = P_S(T_k Z_k).
 * On the full pattern Y -> A^{1/2} and Z -> A^{-1/2} when ||I - A|| < 1 (for
 * K + mu I with K scaled by 1/N, any 0 < mu < 1).  A, Y, Z: distinct device F64
 * value arrays; Y and Z receive Y_iters and Z_iters.  residuals: device array of
 * iters doubles, or NULL.  scratch: device workspace of at least
 * spm_ns_sqrt_scratch() bytes (three value arrays and the products' workspace),
 * 256-byte aligned; nothing is allocated.  Asynchronous on the stream; EINVAL on
 * null or overlapping buffers, a negative iteration count or a short or misaligned
 * scratch. */
int spm_ns_sqrt_scratch(spm_pattern p, size_t *bytes);
int spm_ns_sqrt(spm_pattern p, const double *A, double *Y, double *Z, int32_t iters, double *residuals,
                void *scratch, size_t scratch_bytes, void *stream);

/* Masked Newton-Schulz inverse of A (FP64 on S):
 *   X_0 = alpha0 I;  for k = 0..iters-1:  Y_k = P_S(A X_k),  r_k = ||I - Y_k||_F / sqrt(n),
 *   Z_k = 2I - Y_k,  X_{k+1} = P_S(X_k Z_k);  finally r_iters = ||I - P_S(A X_iters)||_F / sqrt(n).
 * Iterations 0 .. iters-n_final_f64-1 run in precision `bulk`, the rest in FP64.
 * Every residual is summed in FP64; those of the bulk iterations are taken of the
 * bulk-precision product P_S(A X_k) (rounded to that precision), the others and the
 * final one of FP64 products.  X (device, F64) receives X_iters.  residuals (device,
 * iters+1 doubles).  checkpoints (host array of iters+1 device F64 pointers, or
 * NULL) receives X_0 .. X_iters.  scratch: device workspace of at least
 * spm_newton_schulz_scratch() bytes, 256-byte aligned; nothing else is allocated.
 * Returns ENOTCONV when the final residual is not finite or exceeds the initial
 * one r_0 (a diverging iteration; X is still written); this call synchronises the
 * stream (to read the two residuals). */
int spm_newton_schulz_scratch(spm_pattern p, int bulk, size_t *bytes);
int spm_newton_schulz(spm_pattern p, const double *A, double *X, int32_t iters, int32_t n_final_f64,
                      int bulk, double alpha0, double *residuals, double *const *checkpoints,
                      void *scratch, size_t scratch_bytes, void *stream);

/* Quadrature rule of the contour integral for the inverse square root (Section 4.4,
 * eq. ContInt): A^{-1/2} ~ sum_k c[k] (A + w2[k] I)^{-1} for a spectrum in
 * [lam_min, lam_max], k = 0..nodes-1, with w_k = sqrt(lam_min) sn(t_k)/cn(t_k),
 * c_k = 2 Kq sqrt(lam_min) dn(t_k) / (pi nodes cn(t_k)^2), t_k = Kq (k + 1/2) / nodes,
 * Jacobi functions of parameter 1 - lam_min/lam_max and Kq their quarter period
 * (the complete elliptic integral of the first kind).  Host arrays w2[nodes],
 * c[nodes]; host only (no device work).  EINVAL unless 0 < lam_min <= lam_max
 * (finite) and nodes >= 1. */
int spm_contour_rule(double lam_min, double lam_max, int32_t nodes, double *w2, double *c);

/* out = sum_k c_k X_k ~ A^{-1/2} (FP64 on S), X_k the masked Newton-Schulz inverse
 * (spm_newton_schulz, all FP64, ns_iters iterations, X_0 = 2/(lam_min + lam_max +
 * 2 w_k^2) I) of A + w_k^2 I, with the rule of spm_contour_rule on [lam_min, lam_max].
 * A^{1/2} follows as P_S(A out).  out: device F64 value array distinct from A.
 * residuals: device array of `nodes` doubles (the final Newton-Schulz residual of
 * each shifted inverse), or NULL.  scratch: device workspace of at least
 * spm_contour_invsqrt_scratch() bytes, 256-byte aligned; nothing is allocated.
 * Synchronises the stream once per node (as
 * spm_newton_schulz does); with the environment variable SPM_PROGRESS set, reports
 * each node on stderr.  ENOTCONV when a shifted inverse's residual is not finite,
 * EINVAL on bad arguments. */
int spm_contour_invsqrt_scratch(spm_pattern p, int32_t ns_iters, size_t *bytes);
int spm_contour_invsqrt(spm_pattern p, const double *A, double lam_min, double lam_max, int32_t nodes,
                        int32_t ns_iters, double *out, double *residuals, void *scratch, size_t scratch_bytes,
                        void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SPM_H */
