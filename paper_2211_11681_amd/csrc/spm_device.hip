// Device side of libspm for gfx950: pattern upload, elementwise ops, deterministic
// reductions, the masked product and the Newton-Schulz driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "spm_internal.h"

using spm::fail;

namespace spm {

template <typename T>
static int to_device(DevBuf<T> &b, const std::vector<T> &v, hipStream_t s)
{
    b.n = v.size();
    if (v.empty()) { b.ptr = nullptr; return SPM_OK; }
    if (hipMalloc(&b.ptr, v.size() * sizeof(T)) != hipSuccess) {
        b.ptr = nullptr;
        return fail(SPM_ENOMEM, "device allocation for pattern layout");
    }
    // blocking copy: several sources are temporaries of the caller
    (void)s;
    SPM_HIP(hipMemcpy(b.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return SPM_OK;
}

template <typename T>
static void release(DevBuf<T> &b)
{
    if (b.ptr) (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.n = 0;
}

static constexpr int kRedTiles = 64;      // tiles per reduction block
static constexpr int kRedThreads = 256;

int upload_pattern_device(spm_pattern_s *p, hipStream_t s)
{
    int st;
    if ((st = to_device(p->d_cstart, p->cstart, s))) return st;
    if ((st = to_device(p->d_blk_rp, p->blk_rp, s))) return st;
    if ((st = to_device(p->d_tile_off, p->tile_off, s))) return st;
    if ((st = to_device(p->d_colprefix, p->colprefix, s))) return st;
    if ((st = to_device(p->d_rowbase, p->rowbase, s))) return st;
    if ((st = to_device(p->d_rowlen, p->rowlen, s))) return st;
    if ((st = to_device(p->d_nfun, p->nfun, s))) return st;
    if ((st = to_device(p->d_tile_row, p->tile_row, s))) return st;
    if ((st = to_device(p->d_tile_col, p->tile_col, s))) return st;
    if ((st = to_device(p->d_trans, p->trans, s))) return st;
    if ((st = to_device(p->d_diag_tile, p->diag_tile, s))) return st;
    if ((st = to_device(p->d_order, p->order, s))) return st;
    if ((st = to_device(p->d_grp_mem, p->grp_mem, s))) return st;
    if ((st = to_device(p->d_grp_s, p->grp_s, s))) return st;
    if ((st = to_device(p->d_grp_g, p->grp_g, s))) return st;
    if ((st = to_device(p->d_grp_R, p->grp_R, s))) return st;
    if ((st = to_device(p->d_gl_rp, p->gl_rp, s))) return st;
    if ((st = to_device(p->d_gl_mu, p->gl_mu, s))) return st;
    if ((st = to_device(p->d_gl_tile, p->gl_tile, s))) return st;
    if ((st = to_device(p->d_unit_gr, p->unit_gr, s))) return st;
    if ((st = to_device(p->d_unit_gc, p->unit_gc, s))) return st;
    if ((st = to_device(p->d_unit_out, p->unit_out, s))) return st;
    if ((st = to_device(p->d_unit_order, p->unit_order, s))) return st;
    if ((st = to_device(p->d_pair_off, p->pair_off, s))) return st;
    if ((st = to_device(p->d_pair_a, p->pair_a, s))) return st;
    if ((st = to_device(p->d_pair_b, p->pair_b, s))) return st;
    if ((st = to_device(p->d_gl_nm, p->gl_nm, s))) return st;
    if ((st = to_device(p->d_gl_offd, p->gl_offd, s))) return st;
    if ((st = to_device(p->d_gl_offt, p->gl_offt, s))) return st;
    if ((st = to_device(p->d_stage_off, p->stage_off, s))) return st;
    if ((st = to_device(p->d_stage_first, p->stage_first, s))) return st;
    if (!p->csr_pos.empty()) {
        if ((st = to_device(p->d_csr_pos, p->csr_pos, s))) return st;
        std::vector<uint8_t> keep(p->n_stored);
        for (int64_t e = 0; e < p->n_stored; ++e) keep[e] = p->csr_pos[e] >= 0;
        if (p->masked && (st = to_device(p->d_keep, keep, s))) return st;
    }
    int64_t nblk = (p->n_tiles + kRedTiles - 1) / kRedTiles + 1;
    std::vector<double> zeros(nblk, 0.0);
    if ((st = to_device(p->d_partial, zeros, s))) return st;
    SPM_HIP(hipStreamSynchronize(s));
    return SPM_OK;
}

void free_pattern_device(spm_pattern_s *p)
{
    release(p->d_cstart); release(p->d_blk_rp); release(p->d_tile_off); release(p->d_colprefix);
    release(p->d_rowbase); release(p->d_rowlen); release(p->d_csr_pos);
    release(p->d_nfun); release(p->d_tile_row); release(p->d_tile_col); release(p->d_trans);
    release(p->d_diag_tile); release(p->d_order); release(p->d_keep); release(p->d_partial);
    release(p->d_grp_mem); release(p->d_grp_s); release(p->d_grp_g); release(p->d_grp_R); release(p->d_gl_rp);
    release(p->d_gl_mu); release(p->d_gl_tile); release(p->d_unit_gr); release(p->d_unit_gc); release(p->d_unit_out);
    release(p->d_unit_order); release(p->d_pair_off); release(p->d_pair_a); release(p->d_pair_b);
    release(p->d_gl_nm); release(p->d_gl_offd); release(p->d_gl_offt); release(p->d_stage_off); release(p->d_stage_first);
}

}  // namespace spm

namespace {

constexpr int kMax = spm::kMaxFun;
constexpr int kRedTilesK = 64;   // tiles per reduction block (matches spm::kRedTiles)

inline unsigned grid1d(int64_t n, int threads, int64_t cap = 1 << 20)
{
    int64_t g = (n + threads - 1) / threads;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// ------------------------------------------------------------------ values <-> CSR
// CSR position of element e (tile t, local (i, j)) of an unmasked block pattern:
// rowbase[r] + i * rowlen[r] + colprefix[t] + j.
__global__ void k_from_csr(int64_t n_tiles, const int64_t *tile_off, const int32_t *tile_row,
                           const int32_t *tile_col, const int32_t *nfun, const int64_t *rowbase,
                           const int64_t *rowlen, const int64_t *colprefix, const int64_t *csr_pos,
                           const double *csr, double *vals, int to_csr)
{
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int r = tile_row[t], c = tile_col[t];
        const int nr = nfun[r], ncl = nfun[c];
        const int64_t off = tile_off[t];
        for (int e = threadIdx.x; e < nr * ncl; e += blockDim.x) {
            int i = e % nr, j = e / nr;
            int64_t pos = csr_pos ? csr_pos[off + e] : rowbase[r] + (int64_t)i * rowlen[r] + colprefix[t] + j;
            if (to_csr) {
                if (pos >= 0) vals[pos] = csr[off + e];   // here csr = tile values, vals = CSR output
            } else {
                vals[off + e] = pos >= 0 ? csr[pos] : 0.0;
            }
        }
    }
}

// ------------------------------------------------------------------ precision helpers
struct SplitVal {
    float hi, lo;
};

__device__ inline double load_val(int prec, const void *x, int64_t e, int64_t ns)
{
    if (prec == SPM_F64) return static_cast<const double *>(x)[e];
    const float *f = static_cast<const float *>(x);
    if (prec == SPM_F32SPLIT) return (double)f[e] + (double)f[ns + e];
    return (double)f[e];
}

__device__ inline void store_val(int prec, void *x, int64_t e, int64_t ns, double v)
{
    if (prec == SPM_F64) { static_cast<double *>(x)[e] = v; return; }
    float *f = static_cast<float *>(x);
    float hi = (float)v;
    f[e] = hi;
    if (prec == SPM_F32SPLIT) f[ns + e] = (float)(v - (double)hi);
}

__global__ void k_convert(int64_t ns, int pf, const void *x, int pt, void *y)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ns; e += (int64_t)gridDim.x * blockDim.x)
        store_val(pt, y, e, ns, load_val(pf, x, e, ns));
}

// Y = alpha X + beta Y elementwise (X non-null)
__global__ void k_axpy(int64_t ns, int prec, double alpha, const void *x, double beta, void *y)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ns; e += (int64_t)gridDim.x * blockDim.x) {
        double xv = load_val(prec, x, e, ns), yv = load_val(prec, y, e, ns);
        store_val(prec, y, e, ns, alpha * xv + beta * yv);
    }
}

__global__ void k_scale(int64_t ns, int prec, double beta, void *y)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ns; e += (int64_t)gridDim.x * blockDim.x)
        store_val(prec, y, e, ns, 0.0 + beta * load_val(prec, y, e, ns));
}

// diagonal entries: y_ii = alpha + y_ii (after scaling by beta)
__global__ void k_diag_add(int nc, const int32_t *diag_tile, const int64_t *tile_off, const int32_t *nfun,
                           int prec, int64_t ns, double alpha, void *y)
{
    for (int c = blockIdx.x; c < nc; c += gridDim.x) {
        int t = diag_tile[c];
        if (t < 0) continue;
        int n = nfun[c];
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            int64_t e = tile_off[t] + (int64_t)i * n + i;
            store_val(prec, y, e, ns, alpha + load_val(prec, y, e, ns));
        }
    }
}

// ------------------------------------------------------------------ deterministic reductions
enum RedOp { RED_SQDIST = 0, RED_SQDIST_EYE = 1, RED_DOT = 2, RED_QUAD = 3 };

// One partial per block of kRedTiles tiles, in a fixed order.
__global__ __launch_bounds__(256) void k_reduce_tiles(int op, int64_t n_tiles, const int64_t *tile_off,
                                                      const int32_t *tile_row, const int32_t *tile_col,
                                                      const int32_t *nfun, const int64_t *cstart, int prec,
                                                      int64_t ns, const void *x, const void *y, const double *vec,
                                                      double alpha, double *partial)
{
    __shared__ double red[256];
    const int64_t t0 = (int64_t)blockIdx.x * kRedTilesK, t1 = min(n_tiles, t0 + kRedTilesK);
    double acc = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        const int r = tile_row[t], c = tile_col[t];
        const int nr = nfun[r], ncl = nfun[c];
        const int64_t off = tile_off[t];
        for (int e = threadIdx.x; e < nr * ncl; e += blockDim.x) {
            const int i = e % nr, j = e / nr;
            double xv = load_val(prec, x, off + e, ns), v;
            switch (op) {
            case RED_SQDIST: {
                double d = y ? xv - load_val(prec, y, off + e, ns) : xv;
                v = d * d;
                break;
            }
            case RED_SQDIST_EYE: {
                double d = (r == c && i == j) ? alpha - xv : xv;
                v = d * d;
                break;
            }
            case RED_DOT: v = xv * load_val(prec, y, off + e, ns); break;
            default: v = vec[cstart[r] + i] * xv * vec[cstart[c] + j]; break;
            }
            acc += v;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out = post(sum of partials); post: 0 = identity, 1 = sqrt(s) * scale
__global__ __launch_bounds__(1024) void k_reduce_final(int64_t np, const double *partial, int post, double scale,
                                                       double *out)
{
    __shared__ double red[1024];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += 1024) acc += partial[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = post == 1 ? sqrt(red[0]) * scale : red[0];
}

__global__ void k_fill_outer(int64_t n_tiles, const int64_t *tile_off, const int32_t *tile_row,
                             const int32_t *tile_col, const int32_t *nfun, const int64_t *cstart,
                             const uint8_t *keep, double alpha, const double *y, double *x)
{
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int r = tile_row[t], c = tile_col[t];
        const int nr = nfun[r], ncl = nfun[c];
        const int64_t off = tile_off[t];
        for (int e = threadIdx.x; e < nr * ncl; e += blockDim.x) {
            const int i = e % nr, j = e / nr;
            double v = alpha * (y[cstart[r] + i] * y[cstart[c] + j]);
            x[off + e] = (keep && !keep[off + e]) ? 0.0 : v;
        }
    }
}

// ------------------------------------------------------------------ masked product
// One wavefront per output tile (r, c).  The intersection S_r cap S_c of the two
// sorted block rows (the pattern is symmetric, so block row c is block column c)
// is found 64 entries at a time: every lane binary-searches one entry of the
// shorter row in the longer one, and a ballot compacts the hits.  For every hit mu
// the tiles op(A)_{r,mu} and op(B)_{mu,c} are staged in LDS and accumulated into
// the output tile held in registers (column-major element e = lane + 64 s).
struct GemmArgs {
    const int64_t *blk_rp, *tile_off;
    const int32_t *tile_col, *tile_row, *trans, *nfun, *order;
    const uint8_t *keep;
    int64_t n_tiles, ns;
};

// FP32 forms.  F32SPLIT: operands hi + lo; every product hi_a hi_b is made exact
// with an FMA (p = a b, e = fma(a, b, -p)), the cross terms hi_a lo_b + lo_a hi_b
// are added to the error term, and the running sum is a (s, c) pair updated by
// TwoSum (Knuth).  F32ACC: hi operands only, same compensated sum.
template <int TA, int TB, bool SPLIT>
__global__ __launch_bounds__(64) void k_mgemm_f32(GemmArgs g, const float *__restrict__ A,
                                                 const float *__restrict__ B, float *__restrict__ C)
{
    __shared__ float sAh[kMax * kMax], sAl[kMax * kMax];
    __shared__ float sBh[kMax * kMax], sBl[kMax * kMax];
    __shared__ int32_t sPa[64], sPb[64];
    const int lane = threadIdx.x;
    const int64_t ns = g.ns;
    const int64_t t = g.order[blockIdx.x];
    const int r = g.tile_row[t], c = g.tile_col[t];
    const int nr = g.nfun[r], ncl = g.nfun[c];
    const int64_t ra = g.blk_rp[r], la = g.blk_rp[r + 1] - ra;
    const int64_t rb = g.blk_rp[c], lb = g.blk_rp[c + 1] - rb;
    const bool a_short = la <= lb;
    const int64_t rs = a_short ? ra : rb, ls = a_short ? la : lb;
    const int64_t rl = a_short ? rb : ra, ll = a_short ? lb : la;
    const int nout = nr * ncl;
    float sh[kMax * kMax / 64], sl[kMax * kMax / 64];
#pragma unroll
    for (int s = 0; s < kMax * kMax / 64; ++s) { sh[s] = 0.f; sl[s] = 0.f; }

    for (int64_t base = 0; base < ls; base += 64) {
        const int64_t idx = base + lane;
        bool found = false;
        int64_t pl = 0;
        if (idx < ls) {
            const int32_t mu = g.tile_col[rs + idx];
            int64_t lo = 0, hi = ll;
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (g.tile_col[rl + mid] < mu) lo = mid + 1; else hi = mid;
            }
            found = lo < ll && g.tile_col[rl + lo] == mu;
            pl = lo;
        }
        const uint64_t bal = __ballot(found);
        const int cnt = __popcll(bal);
        if (found) {
            const int rank = __popcll(bal & ((1ull << lane) - 1ull));
            sPa[rank] = (int32_t)(a_short ? idx : pl);
            sPb[rank] = (int32_t)(a_short ? pl : idx);
        }
        __syncthreads();
        for (int f = 0; f < cnt; ++f) {
            const int64_t ta = ra + sPa[f];
            const int64_t tb = rb + sPb[f];
            const int mu = g.tile_col[ta];
            const int nm = g.nfun[mu];
            if (TA == 0) {
                const int64_t o = g.tile_off[ta];
                for (int e = lane; e < nr * nm; e += 64) {
                    int i = e % nr, k = e / nr;
                    sAh[k * kMax + i] = A[o + e];
                    if (SPLIT) sAl[k * kMax + i] = A[ns + o + e];
                }
            } else {
                const int64_t o = g.tile_off[g.trans[ta]];
                for (int e = lane; e < nr * nm; e += 64) {
                    int k = e % nm, i = e / nm;
                    sAh[k * kMax + i] = A[o + e];
                    if (SPLIT) sAl[k * kMax + i] = A[ns + o + e];
                }
            }
            if (TB == 0) {
                const int64_t o = g.tile_off[g.trans[tb]];
                for (int e = lane; e < nm * ncl; e += 64) {
                    int k = e % nm, j = e / nm;
                    sBh[k * kMax + j] = B[o + e];
                    if (SPLIT) sBl[k * kMax + j] = B[ns + o + e];
                }
            } else {
                const int64_t o = g.tile_off[tb];
                for (int e = lane; e < nm * ncl; e += 64) {
                    int j = e % ncl, k = e / ncl;
                    sBh[k * kMax + j] = B[o + e];
                    if (SPLIT) sBl[k * kMax + j] = B[ns + o + e];
                }
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < kMax * kMax / 64; ++s) {
                const int e = lane + 64 * s;
                if (e < nout) {
                    const int i = e % nr, j = e / nr;
                    float hs = sh[s], ls2 = sl[s];
                    for (int k = 0; k < nm; ++k) {
                        const float ah = sAh[k * kMax + i], bh = sBh[k * kMax + j];
                        const float p = ah * bh;
                        float err = fmaf(ah, bh, -p);
                        if (SPLIT) err = fmaf(ah, sBl[k * kMax + j], fmaf(sAl[k * kMax + i], bh, err));
                        const float s2 = hs + p;
                        const float bv = s2 - hs;
                        const float ts = (hs - (s2 - bv)) + (p - bv);
                        hs = s2;
                        ls2 += ts + err;
                    }
                    sh[s] = hs;
                    sl[s] = ls2;
                }
            }
            __syncthreads();
        }
    }
    const int64_t off = g.tile_off[t];
#pragma unroll
    for (int s = 0; s < kMax * kMax / 64; ++s) {
        const int e = lane + 64 * s;
        if (e < nout) {
            const float hi = sh[s] + sl[s];
            const float lo = (sh[s] - hi) + sl[s];
            C[off + e] = hi;
            if (SPLIT) C[ns + off + e] = lo;
        }
    }
}

// Positions inside a tile but outside S are set to zero after a product (patterns
// uploaded entry by entry only).
__global__ void k_apply_keep(int64_t ns, int prec, const uint8_t *__restrict__ keep, void *c)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ns; e += (int64_t)gridDim.x * blockDim.x) {
        if (keep[e]) continue;
        if (prec == SPM_F64) {
            static_cast<double *>(c)[e] = 0.0;
        } else {
            static_cast<float *>(c)[e] = 0.f;
            if (prec == SPM_F32SPLIT) static_cast<float *>(c)[ns + e] = 0.f;
        }
    }
}


// ------------------------------------------------------------------ grouped MFMA product (FP64)
// One unit (G_r, G_c) = the output tiles between the (up to 4) row clusters of G_r
// and the column clusters of G_c, held as 16x16 blocks of MFMA accumulators.  The
// unit's middle clusters mu (U(G_r) cap U(G_c), listed by the schedule builder) come
// in stages of consecutive clusters with at most 32 padded k rows.  Per stage the
// panels op(A)_{G_r,mu} (R x k) and op(B)_{mu,G_c} (k x C) of all its clusters are
// gathered into LDS by direct global-to-LDS loads (one dword per lane, 32 doubles per
// wave instruction; absent tiles and padding read a zero word) and multiplied with
// v_mfma_f64_16x16x4f64 (lane l: A row l%16 and k l/16, B column l%16 and k l/16;
// accumulator register r holds row 4r + l/16, column l%16).
// Panel layouts follow the source tiles so that the gathers read contiguous memory:
//   row-fast  [k][x], stride Xp = x rounded up to 32: one instruction = 32 x of one k
//             (tiles whose element order runs along x: op(A) = A, op(B) = B^T)
//   k-fast    [x][k], stride 33: one instruction = 32 k of one x
//             (tiles whose element order runs along k: op(A) = A^T, op(B) = B, and
//             every panel of clusters with at most 8 functions)
// The panels are double-buffered: the gathers of stage s+1 and the stage table of
// stage s+2 are in flight while the MFMAs of stage s run.
// WAVES = 8: one workgroup per unit.  WAVES = 1: one wavefront per unit, four units
// per workgroup, each with its own LDS; no workgroup barriers.
typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ double g_zero_word[2];   // zero-initialised source of padding

struct GroupArgs {
    const int32_t *grp_mem, *grp_s, *grp_g;
    const int32_t *unit_gr, *unit_gc, *unit_out, *unit_order;
    const int64_t *pair_off;
    const int32_t *pair_a, *pair_b;
    const int32_t *gl_nm;
    const int64_t *gl_offd, *gl_offt;
    const int64_t *stage_off;
    const int32_t *stage_first;
    const int64_t *tile_off;
    const int32_t *nfun;
    int64_t first, count;
    int32_t RB, CB;
    int32_t akf, bkf;        // k-fast layout of the A / B panels for the whole launch
    int32_t panel_doubles;   // LDS doubles of one operand buffer (A panel + B panel)
};

constexpr int kKS = 32;   // k rows per stage
constexpr int kSP = 8;    // middle clusters per stage
constexpr int kKF = 33;   // stride of k-fast panels

struct StageTab {
    int64_t off[kSP][8];  // element offsets: slots 0..3 op(A) tiles of the row members, 4..7 op(B) tiles of the column members
    int32_t nm[kSP];      // functions of each middle cluster
    int32_t kb[kSP];      // first k row of each middle cluster in the stage
    int32_t kmap[kKS];    // k row -> middle cluster of the stage, -1 past the end
    int32_t ks;           // padded k rows of the stage
    int32_t pad;
};

// Per k row records of a stage (row-fast gathers, 8-wave units only): offsets of the
// row's middle cluster and the row inside it.
struct KTab {
    int64_t koff[kKS][8];
    int32_t knm[kKS];     // functions of the row's cluster (0 past the end)
    int32_t kkm[kKS];     // k row inside the cluster
};

template <int WAVES>
constexpr size_t unit_tab_bytes()
{
    return 2 * (sizeof(StageTab) + (WAVES == 8 ? sizeof(KTab) : 0));
}

template <int WAVES>
__device__ inline void unit_sync()
{
    __builtin_amdgcn_s_waitcnt(0);
    if (WAVES > 1) __syncthreads();
    else __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

__device__ inline void lds_gather(const double *src, int half, double *dst)
{
    __builtin_amdgcn_global_load_lds((const void *)(reinterpret_cast<const uint32_t *>(src) + half),
                                     (__attribute__((address_space(3))) void *)dst, 4, 0, 0);
}

template <int TA, int TB, int WAVES>
__global__ __launch_bounds__(WAVES == 8 ? 512 : 256) void k_mgemm_grp(GroupArgs g, const double *__restrict__ A,
                                                                     const double *__restrict__ B,
                                                                     double *__restrict__ C)
{
    extern __shared__ double lds_all[];
    constexpr int NT = WAVES * 64;                 // threads per unit
    constexpr int UPW = WAVES == 8 ? 1 : 4;        // units per workgroup
    constexpr int MAXB = WAVES == 8 ? 8 : 1;       // accumulator blocks per wave
    const int tid = threadIdx.x % NT, lane = tid & 63, wave = tid >> 6;
    const int uslot = threadIdx.x / NT;
    const int64_t uidx = (int64_t)blockIdx.x * UPW + uslot;
    if (uidx >= g.count) return;                    // whole unit slot idle (tail)
    const int R = g.RB * 16, Cc = g.CB * 16;
    const int pd = g.panel_doubles;
    double *lds = lds_all + (size_t)uslot * (2 * pd + unit_tab_bytes<WAVES>() / sizeof(double));
    StageTab *tab = reinterpret_cast<StageTab *>(lds + 2 * pd);
    KTab *ktab = reinterpret_cast<KTab *>(tab + 2);     // used when WAVES == 8

    const int u = g.unit_order[g.first + uidx];
    const int gr = g.unit_gr[u], gc = g.unit_gc[u];
    const int sr = g.grp_s[gr], sc = g.grp_s[gc];
    const int ngr = g.grp_g[gr], ngc = g.grp_g[gc];
    int nrk[4], nck[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        nrk[k] = k < ngr ? g.nfun[g.grp_mem[gr * 4 + k]] : 0;
        nck[k] = k < ngc ? g.nfun[g.grp_mem[gc * 4 + k]] : 0;
    }
    // panel layouts (fixed per launch)
    const bool akf = g.akf != 0, bkf = g.bkf != 0;
    const int Rp = (R + 31) & ~31, Cp = (Cc + 31) & ~31;
    const int asz = akf ? R * kKF : kKS * Rp;       // doubles of the A panel
    const int a_rs = akf ? kKF : 1, a_ks = akf ? 1 : Rp;   // address = row * a_rs + k * a_ks
    const int b_cs = bkf ? kKF : 1, b_ks = bkf ? 1 : Cp;   // address = col * b_cs + k * b_ks
    const int nblk = g.RB * g.CB;
    const int nsplit = (WAVES == 1 || nblk >= WAVES) ? 1 : WAVES / nblk;
    const int kslice = nsplit == 1 ? 0 : wave / nblk;
    const bool active = WAVES == 1 || nblk >= WAVES || wave < nblk * nsplit;
    const int b0 = (WAVES == 1 || nblk >= WAVES) ? wave : wave % nblk;
    const int bstep = (WAVES == 8 && nblk >= WAVES) ? WAVES : 1 << 20;
    const int64_t s0 = g.stage_off[u], nst = g.stage_off[u + 1] - s0;
    const int64_t p0 = g.pair_off[u], npairs = g.pair_off[u + 1] - p0;
    const int half = lane & 1, l2 = lane >> 1;

    // row-fast rows of this lane: row = 32 * blk + l2 -> (member, index), for up to 4 blocks
    int rkr[4], ri[4], ckc[4], cj[4];
#pragma unroll
    for (int bl = 0; bl < 4; ++bl) {
        const int row = 32 * bl + l2, col = 32 * bl + l2;
        rkr[bl] = row / sr; ri[bl] = row - rkr[bl] * sr;
        ckc[bl] = col / sc; cj[bl] = col - ckc[bl] * sc;
    }

    // ---- stage tables, fetched by wave 0 in three steps spread over three stages so that
    // no load waits for another one inside a stage: bounds -> union entries -> offsets.
    // Lane (p, slot): middle cluster p of the stage, slot 0..3 row members (op(A)),
    // 4..7 column members (op(B)); slot 0 also carries the cluster size.
    const int tp = lane >> 3, tslot = lane & 7, tk = tslot & 3;
    auto bounds = [&](int64_t st, int64_t &fb, int &np) {
        fb = 0;
        np = 0;
        if (wave != 0 || st >= nst) return;
        fb = g.stage_first[s0 + st];
        const int64_t fe = st + 1 < nst ? g.stage_first[s0 + st + 1] : npairs;
        np = (int)(fe - fb);
    };
    auto entry = [&](int64_t fb, int np) -> int {
        if (wave != 0 || tp >= np) return -1;
        return tslot < 4 ? g.pair_a[p0 + fb + tp] : g.pair_b[p0 + fb + tp];
    };
    auto offsets = [&](int e, int64_t &off, int &nm) {
        off = -1;
        nm = 0;
        if (e < 0) return;
        if (tslot < 4 ? tk < ngr : tk < ngc) {
            const int64_t *src = tslot < 4 ? (TA == 0 ? g.gl_offd : g.gl_offt) : (TB == 0 ? g.gl_offt : g.gl_offd);
            off = src[(int64_t)e * 4 + tk];
        }
        if (tslot == 0) nm = g.gl_nm[e];
    };
    auto write_tab = [&](StageTab *T, KTab *KT, int64_t t_off, int t_nm, int t_np) {
        if (wave != 0) return;
        int nmv[kSP], kbv[kSP];
        int acc = 0;
#pragma unroll
        for (int q = 0; q < kSP; ++q) {
            nmv[q] = __shfl(t_nm, q * 8);
            kbv[q] = acc;
            acc += q < t_np ? (nmv[q] + 3) & ~3 : 0;
        }
        T->off[tp][tslot] = tp < t_np ? t_off : -1;
        if (lane < kSP) { T->nm[lane] = lane < t_np ? nmv[lane] : 0; T->kb[lane] = kbv[lane]; }
        int m = -1;
#pragma unroll
        for (int q = 0; q < kSP; ++q)
            if (q < t_np && (lane & 31) >= kbv[q] && (lane & 31) < kbv[q] + ((nmv[q] + 3) & ~3)) m = q;
        if (lane < kKS) T->kmap[lane] = m;
        if (lane == 0) T->ks = acc;
        if (WAVES == 8) {
            // per k row records: lane kk (and kk + 32 for slots 4..7) gathers the offsets of its cluster
            const int kk = lane & 31, sb = lane < 32 ? 0 : 4;
            const int mm = m;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t v = __shfl(t_off, (mm < 0 ? 0 : mm) * 8 + sb + q);
                KT->koff[kk][sb + q] = (mm >= 0) ? v : -1;
            }
            if (lane < 32) {
                KT->knm[kk] = mm >= 0 ? nmv[mm < 0 ? 0 : mm] : 0;
                KT->kkm[kk] = mm >= 0 ? kk - kbv[mm < 0 ? 0 : mm] : 0;
            }
        }
    };

    // ---- gathers of one stage into an operand buffer.  Rows (columns) outside the
    // members' functions are not gathered: they only feed outputs that are dropped.
    const double *const zero = g_zero_word;
    auto gather = [&](const StageTab *T, const KTab *KT, double *buf) {
        const int ks = T->ks;
        double *pA = buf, *pB = buf + asz;
        // k-fast panels: this lane's k row is l2 for every instruction
        const int pi = l2 < ks ? T->kmap[l2] : -1;
        const int nm_l = pi >= 0 ? T->nm[pi] : 0;
        const int kkm_l = pi >= 0 ? l2 - T->kb[pi] : 0;
        const bool kval = pi >= 0 && kkm_l < nm_l;
        if (akf) {
#pragma unroll
            for (int kr = 0; kr < 4; ++kr) {
                if (kr >= ngr) break;
                const int n = nrk[kr];
                const int64_t oo = kval ? T->off[pi][kr] : -1;
                const bool ok = oo >= 0;
                const double *base = A + (ok ? oo : 0);
                double *dst = pA + kr * sr * kKF;
                for (int i = wave; i < n; i += WAVES) {
                    const double *src = ok ? base + (TA == 1 ? i * nm_l + kkm_l : kkm_l * n + i) : zero;
                    lds_gather(src, half, dst + i * kKF);
                }
            }
        } else if (WAVES == 8) {
            const int nb = Rp >> 5;
#pragma unroll
            for (int bl = 0; bl < 4; ++bl) {
                if (bl >= nb) break;
                const int kr = rkr[bl], i = ri[bl];
                const int n = kr == 0 ? nrk[0] : kr == 1 ? nrk[1] : kr == 2 ? nrk[2] : nrk[3];
                const bool rv = kr < ngr && i < n;
                for (int kk = wave; kk < ks; kk += WAVES) {
                    const int nm = KT->knm[kk], kkm = KT->kkm[kk];
                    const int64_t oo = KT->koff[kk][kr & 3];
                    const double *src = (rv && oo >= 0 && kkm < nm) ? A + oo + kkm * n + i : zero;   // TA = 0 here
                    lds_gather(src, half, pA + kk * Rp + bl * 32);
                }
            }
        }
        if (bkf) {
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
                if (kc >= ngc) break;
                const int n = nck[kc];
                const int64_t oo = kval ? T->off[pi][4 + kc] : -1;
                const bool ok = oo >= 0;
                const double *base = B + (ok ? oo : 0);
                double *dst = pB + kc * sc * kKF;
                for (int j = wave; j < n; j += WAVES) {
                    const double *src = ok ? base + (TB == 0 ? j * nm_l + kkm_l : kkm_l * n + j) : zero;
                    lds_gather(src, half, dst + j * kKF);
                }
            }
        } else if (WAVES == 8) {
            const int nb = Cp >> 5;
#pragma unroll
            for (int bl = 0; bl < 4; ++bl) {
                if (bl >= nb) break;
                const int kc = ckc[bl], j = cj[bl];
                const int n = kc == 0 ? nck[0] : kc == 1 ? nck[1] : kc == 2 ? nck[2] : nck[3];
                const bool cv = kc < ngc && j < n;
                for (int kk = wave; kk < ks; kk += WAVES) {
                    const int nm = KT->knm[kk], kkm = KT->kkm[kk];
                    const int64_t oo = KT->koff[kk][4 + (kc & 3)];
                    const double *src = (cv && oo >= 0 && kkm < nm) ? B + oo + kkm * n + j : zero;   // TB = 1 here
                    lds_gather(src, half, pB + kk * Cp + bl * 32);
                }
            }
        }
    };

    dbl4 acc[MAXB];
#pragma unroll
    for (int j = 0; j < MAXB; ++j) acc[j] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int lr = lane & 15, lk = lane >> 4;
    // owned output blocks of this wave and their operand offsets in the panels
    int nown = 0, aoffs[MAXB], boffs[MAXB];
#pragma unroll
    for (int j = 0; j < MAXB; ++j) {
        const int b = b0 + j * bstep;
        const int rb = b / g.CB, cb = b - rb * g.CB;
        aoffs[j] = 16 * rb * a_rs;
        boffs[j] = 16 * cb * b_cs;
        if (b < nblk) nown = j + 1;
    }

    // prologue: tables 0 and 1 written; registers: offsets of stage 2, entries of stage 3,
    // bounds of stage 4
    int64_t fb;
    int np;
    int64_t r_off;
    int r_nm, r_np, r_e, r_enp;
    int64_t r_fb;
    int r_bnp;
    for (int st = 0; st < 2; ++st) {
        bounds(st, fb, np);
        offsets(entry(fb, np), r_off, r_nm);
        write_tab(&tab[st], &ktab[st], r_off, r_nm, np);
    }
    bounds(2, fb, np);
    offsets(entry(fb, np), r_off, r_nm);
    r_np = np;
    bounds(3, fb, np);
    r_e = entry(fb, np);
    r_enp = np;
    bounds(4, r_fb, r_bnp);
    unit_sync<WAVES>();
    if (nst > 0) gather(&tab[0], &ktab[0], lds);
    for (int64_t s = 0; s < nst; ++s) {
        const int ks_s = tab[s & 1].ks;             // read before table s is replaced below
        unit_sync<WAVES>();                         // gathers of stage s done; MFMAs of stage s-1 done
        write_tab(&tab[s & 1], &ktab[s & 1], r_off, r_nm, r_np);  // table s+2 replaces table s
        if (s + 1 < nst) gather(&tab[(s + 1) & 1], &ktab[(s + 1) & 1], lds + ((s + 1) & 1) * pd);
        // advance the fetch pipeline: offsets of s+3, entries of s+4, bounds of s+5
        offsets(r_e, r_off, r_nm);
        r_np = r_enp;
        r_e = entry(r_fb, r_bnp);
        r_enp = r_bnp;
        bounds(s + 5, r_fb, r_bnp);
        if (active) {
            const double *sA = lds + (s & 1) * pd, *sB = sA + asz;
            for (int k0 = 4 * kslice; k0 < ks_s; k0 += 4 * nsplit) {
                const double *pa = sA + lr * a_rs + (k0 + lk) * a_ks;
                const double *pb = sB + lr * b_cs + (k0 + lk) * b_ks;
#pragma unroll
                for (int j = 0; j < MAXB; ++j)
                    if (j < nown) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[aoffs[j]], pb[boffs[j]], acc[j], 0, 0, 0);
            }
        }
    }
    if (nsplit > 1) {                               // add the k slices in a fixed order
        unit_sync<WAVES>();
        // waves nblk.. hold the partial sums of k slices 1..nsplit-1: slot (wave - nblk)
        if (active && kslice > 0)
            for (int r = 0; r < 4; ++r) lds[(((wave - nblk) * 4) + r) * 64 + lane] = acc[0][r];
        unit_sync<WAVES>();
        if (active && kslice == 0)
            for (int sl = 1; sl < nsplit; ++sl) {
                const int w2 = sl * nblk + wave;
                for (int r = 0; r < 4; ++r) acc[0][r] += lds[(((w2 - nblk) * 4) + r) * 64 + lane];
            }
    }
    if (!active || kslice != 0) return;
    // store the output tiles that belong to S
#pragma unroll
    for (int j = 0; j < MAXB; ++j) {
        const int b = b0 + j * bstep;
        if (b >= nblk) continue;
        const int rb = b / g.CB, cb = b - rb * g.CB;
        const int col = 16 * cb + lr;
        const int kc = col / sc, jj = col - kc * sc;
        if (kc >= ngc) continue;
        const int ncl = nck[kc];
        if (jj >= ncl) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * rb + 4 * r + lk;
            const int kr = row / sr, i = row - kr * sr;
            if (kr >= ngr) continue;
            const int t = g.unit_out[u * 16 + kr * 4 + kc];
            const int nr = nrk[kr];
            if (t >= 0 && i < nr) C[g.tile_off[t] + (int64_t)jj * nr + i] = acc[j][r];
        }
    }
}

GemmArgs gemm_args(spm_pattern p)
{
    GemmArgs g;
    g.blk_rp = p->d_blk_rp.ptr; g.tile_off = p->d_tile_off.ptr;
    g.tile_col = p->d_tile_col.ptr; g.tile_row = p->d_tile_row.ptr; g.trans = p->d_trans.ptr;
    g.nfun = p->d_nfun.ptr; g.order = p->d_order.ptr; g.keep = p->d_keep.ptr;
    g.n_tiles = p->n_tiles; g.ns = p->n_stored;
    return g;
}

bool valid_prec(int prec) { return prec == SPM_F64 || prec == SPM_F32SPLIT || prec == SPM_F32ACC; }

size_t value_bytes(spm_pattern p, int prec)
{
    return (size_t)p->n_stored * (prec == SPM_F64 ? 8 : prec == SPM_F32SPLIT ? 8 : 4);
}

bool overlap2(const void *a, size_t na, const void *b, size_t nb)
{
    if (!a || !b) return false;
    const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
    return x < y + nb && y < x + na;
}

bool overlap(const void *a, const void *b, size_t bytes)
{
    if (!a || !b) return false;
    const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
    return x < y + bytes && y < x + bytes;
}

}  // namespace

namespace spm {

int launch_gemm_grouped(spm_pattern p, const double *A, int ta, const double *B, int tb, double *C, hipStream_t s)
{
    GroupArgs g;
    g.grp_mem = p->d_grp_mem.ptr; g.grp_s = p->d_grp_s.ptr; g.grp_g = p->d_grp_g.ptr;
    g.unit_gr = p->d_unit_gr.ptr; g.unit_gc = p->d_unit_gc.ptr; g.unit_out = p->d_unit_out.ptr;
    g.unit_order = p->d_unit_order.ptr; g.pair_off = p->d_pair_off.ptr; g.pair_a = p->d_pair_a.ptr;
    g.pair_b = p->d_pair_b.ptr; g.gl_nm = p->d_gl_nm.ptr; g.gl_offd = p->d_gl_offd.ptr; g.gl_offt = p->d_gl_offt.ptr;
    g.stage_off = p->d_stage_off.ptr; g.stage_first = p->d_stage_first.ptr; g.tile_off = p->d_tile_off.ptr;
    g.nfun = p->d_nfun.ptr;
    const int sel = (ta ? 2 : 0) + (tb ? 1 : 0);
    static bool attr_set = false;
    if (!attr_set) {
        const int mx = 160 * 1024;
#define SPM_ATTR(W)                                                                                                       \
    SPM_HIP(hipFuncSetAttribute((const void *)k_mgemm_grp<0, 0, W>, hipFuncAttributeMaxDynamicSharedMemorySize, mx));     \
    SPM_HIP(hipFuncSetAttribute((const void *)k_mgemm_grp<0, 1, W>, hipFuncAttributeMaxDynamicSharedMemorySize, mx));     \
    SPM_HIP(hipFuncSetAttribute((const void *)k_mgemm_grp<1, 0, W>, hipFuncAttributeMaxDynamicSharedMemorySize, mx));     \
    SPM_HIP(hipFuncSetAttribute((const void *)k_mgemm_grp<1, 1, W>, hipFuncAttributeMaxDynamicSharedMemorySize, mx));
        SPM_ATTR(1) SPM_ATTR(8)
#undef SPM_ATTR
        attr_set = true;
    }
    for (const auto &L : p->launches) {
        g.first = L.first;
        g.count = L.count;
        g.RB = L.rb;
        g.CB = L.cb;
        const int R = 16 * L.rb, Cc = 16 * L.cb, Rp = (R + 31) & ~31, Cp = (Cc + 31) & ~31;
        // row-fast panels need the per k row records, which only 8-wave units build
        g.akf = (ta == 1 || L.smax_r <= 8 || L.waves == 1) ? 1 : 0;
        g.bkf = (tb == 0 || L.smax_c <= 8 || L.waves == 1) ? 1 : 0;
        // the k-slice reduction (at most 7 x 4 x 64 doubles) fits in two buffers
        g.panel_doubles = (g.akf ? R * kKF : kKS * Rp) + (g.bkf ? Cc * kKF : kKS * Cp);
        const int waves = L.waves == 1 ? 1 : 8;
        const int upw = waves == 1 ? 4 : 1;
        const size_t lds = upw * (2 * (size_t)g.panel_doubles * sizeof(double) +
                                  (waves == 8 ? unit_tab_bytes<8>() : unit_tab_bytes<1>()));
        if (lds > 160 * 1024) return fail(SPM_EUNSUPPORTED, "grouped product: LDS budget exceeded");
        dim3 grid((unsigned)((L.count + upw - 1) / upw));
#define SPM_LAUNCH_GRP(W)                                                                                   \
    switch (sel) {                                                                                          \
    case 0: hipLaunchKernelGGL((k_mgemm_grp<0, 0, W>), grid, dim3(W == 8 ? 512 : 256), lds, s, g, A, B, C); break;   \
    case 1: hipLaunchKernelGGL((k_mgemm_grp<0, 1, W>), grid, dim3(W == 8 ? 512 : 256), lds, s, g, A, B, C); break;   \
    case 2: hipLaunchKernelGGL((k_mgemm_grp<1, 0, W>), grid, dim3(W == 8 ? 512 : 256), lds, s, g, A, B, C); break;   \
    default: hipLaunchKernelGGL((k_mgemm_grp<1, 1, W>), grid, dim3(W == 8 ? 512 : 256), lds, s, g, A, B, C); break;  \
    }
        if (waves == 1) { SPM_LAUNCH_GRP(1) } else { SPM_LAUNCH_GRP(8) }
#undef SPM_LAUNCH_GRP
    }
    SPM_HIP(hipGetLastError());
    return SPM_OK;
}

int launch_gemm(spm_pattern p, int prec, const void *A, int ta, const void *B, int tb, void *C, hipStream_t s)
{
    if (p->n_tiles == 0) return SPM_OK;
    if (prec == SPM_F64) {
        int st = launch_gemm_grouped(p, static_cast<const double *>(A), ta, static_cast<const double *>(B), tb,
                                     static_cast<double *>(C), s);
        if (st) return st;
        if (p->d_keep.ptr)
            hipLaunchKernelGGL(k_apply_keep, dim3(grid1d(p->n_stored, 256)), dim3(256), 0, s, p->n_stored, prec,
                               p->d_keep.ptr, C);
        SPM_HIP(hipGetLastError());
        return SPM_OK;
    }
    GemmArgs g = gemm_args(p);
    dim3 grid((unsigned)p->n_tiles), block(64);
    const int sel = (ta ? 2 : 0) + (tb ? 1 : 0);
    {
        auto a = static_cast<const float *>(A);
        auto b = static_cast<const float *>(B);
        auto c = static_cast<float *>(C);
        const bool sp = prec == SPM_F32SPLIT;
        switch (sel + (sp ? 4 : 0)) {
        case 0: hipLaunchKernelGGL((k_mgemm_f32<0, 0, false>), grid, block, 0, s, g, a, b, c); break;
        case 1: hipLaunchKernelGGL((k_mgemm_f32<0, 1, false>), grid, block, 0, s, g, a, b, c); break;
        case 2: hipLaunchKernelGGL((k_mgemm_f32<1, 0, false>), grid, block, 0, s, g, a, b, c); break;
        case 3: hipLaunchKernelGGL((k_mgemm_f32<1, 1, false>), grid, block, 0, s, g, a, b, c); break;
        case 4: hipLaunchKernelGGL((k_mgemm_f32<0, 0, true>), grid, block, 0, s, g, a, b, c); break;
        case 5: hipLaunchKernelGGL((k_mgemm_f32<0, 1, true>), grid, block, 0, s, g, a, b, c); break;
        case 6: hipLaunchKernelGGL((k_mgemm_f32<1, 0, true>), grid, block, 0, s, g, a, b, c); break;
        default: hipLaunchKernelGGL((k_mgemm_f32<1, 1, true>), grid, block, 0, s, g, a, b, c); break;
        }
    }
    if (p->d_keep.ptr)
        hipLaunchKernelGGL(k_apply_keep, dim3(grid1d(p->n_stored, 256)), dim3(256), 0, s, p->n_stored, prec,
                           p->d_keep.ptr, C);
    SPM_HIP(hipGetLastError());
    return SPM_OK;
}

int launch_reduce(spm_pattern p, int op, int prec, const void *x, const void *y, const double *vec, double alpha,
                  int post, double scale, double *out, hipStream_t s)
{
    const int64_t nb = std::max<int64_t>(1, (p->n_tiles + kRedTiles - 1) / kRedTiles);
    hipLaunchKernelGGL(k_reduce_tiles, dim3((unsigned)nb), dim3(kRedThreads), 0, s, op, p->n_tiles,
                       p->d_tile_off.ptr, p->d_tile_row.ptr, p->d_tile_col.ptr, p->d_nfun.ptr, p->d_cstart.ptr,
                       prec, p->n_stored, x, y, vec, alpha, p->d_partial.ptr);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, s, nb, p->d_partial.ptr, post, scale, out);
    SPM_HIP(hipGetLastError());
    return SPM_OK;
}

int launch_axpy(spm_pattern p, int prec, double alpha, const void *X, double beta, void *Y, hipStream_t s)
{
    const int64_t ns = p->n_stored;
    if (X) {
        hipLaunchKernelGGL(k_axpy, dim3(grid1d(ns, 256)), dim3(256), 0, s, ns, prec, alpha, X, beta, Y);
    } else {
        if (beta != 1.0) hipLaunchKernelGGL(k_scale, dim3(grid1d(ns, 256)), dim3(256), 0, s, ns, prec, beta, Y);
        hipLaunchKernelGGL(k_diag_add, dim3(grid1d(p->nc, 1, 65536)), dim3(64), 0, s, p->nc, p->d_diag_tile.ptr,
                           p->d_tile_off.ptr, p->d_nfun.ptr, prec, ns, alpha, Y);
    }
    SPM_HIP(hipGetLastError());
    return SPM_OK;
}

int launch_convert(spm_pattern p, int pf, const void *X, int pt, void *Y, hipStream_t s)
{
    const int64_t ns = p->n_stored;
    hipLaunchKernelGGL(k_convert, dim3(grid1d(ns, 256)), dim3(256), 0, s, ns, pf, X, pt, Y);
    SPM_HIP(hipGetLastError());
    return SPM_OK;
}

}  // namespace spm

// ============================================================================ C ABI
extern "C" int spm_values_from_csr(spm_pattern p, const double *csr, double *vals, void *stream)
{
    if (!p || !csr || !vals) return fail(SPM_EINVAL, "spm_values_from_csr: null pointer");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_from_csr, dim3(grid1d(p->n_tiles, 1, 1 << 20)), dim3(64), 0, s, p->n_tiles,
                       p->d_tile_off.ptr, p->d_tile_row.ptr, p->d_tile_col.ptr, p->d_nfun.ptr, p->d_rowbase.ptr,
                       p->d_rowlen.ptr, p->d_colprefix.ptr, p->d_csr_pos.ptr, csr, vals, 0);
    SPM_HIP(hipGetLastError());
    return SPM_OK;
}

extern "C" int spm_values_to_csr(spm_pattern p, const double *vals, double *csr, void *stream)
{
    if (!p || !csr || !vals) return fail(SPM_EINVAL, "spm_values_to_csr: null pointer");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_from_csr, dim3(grid1d(p->n_tiles, 1, 1 << 20)), dim3(64), 0, s, p->n_tiles,
                       p->d_tile_off.ptr, p->d_tile_row.ptr, p->d_tile_col.ptr, p->d_nfun.ptr, p->d_rowbase.ptr,
                       p->d_rowlen.ptr, p->d_colprefix.ptr, p->d_csr_pos.ptr, vals, csr, 1);
    SPM_HIP(hipGetLastError());
    return SPM_OK;
}

extern "C" int spm_masked_gemm(spm_pattern p, int prec, const void *A, int ta, const void *B, int tb, void *C,
                               void *stream)
{
    if (!p || !A || !B || !C) return fail(SPM_EINVAL, "spm_masked_gemm: null pointer");
    if (!valid_prec(prec)) return fail(SPM_EINVAL, "spm_masked_gemm: bad precision");
    if ((ta != 0 && ta != 1) || (tb != 0 && tb != 1)) return fail(SPM_EINVAL, "spm_masked_gemm: bad transpose flag");
    const size_t vb = value_bytes(p, prec);
    if (overlap(A, C, vb) || overlap(B, C, vb)) return fail(SPM_EINVAL, "spm_masked_gemm: C aliases an operand");
    return spm::launch_gemm(p, prec, A, ta, B, tb, C, (hipStream_t)stream);
}

extern "C" int spm_masked_gemm_backward(spm_pattern p, int prec, const void *dC, const void *A, const void *B,
                                        void *dA, void *dB, void *stream)
{
    if (!p || !dC || !A || !B) return fail(SPM_EINVAL, "spm_masked_gemm_backward: null pointer");
    if (!valid_prec(prec)) return fail(SPM_EINVAL, "spm_masked_gemm_backward: bad precision");
    const size_t vb = value_bytes(p, prec);
    for (void *o : {dA, dB})
        if (o && (overlap(o, dC, vb) || overlap(o, A, vb) || overlap(o, B, vb)))
            return fail(SPM_EINVAL, "spm_masked_gemm_backward: output aliases an input");
    if (dA && dB && overlap(dA, dB, vb)) return fail(SPM_EINVAL, "spm_masked_gemm_backward: dA aliases dB");
    int st;
    if (dA && (st = spm::launch_gemm(p, prec, dC, 0, B, 1, dA, (hipStream_t)stream))) return st;   // P_S(dC B^T)
    if (dB && (st = spm::launch_gemm(p, prec, A, 1, dC, 0, dB, (hipStream_t)stream))) return st;   // P_S(A^T dC)
    return SPM_OK;
}

extern "C" int spm_axpy(spm_pattern p, int prec, double alpha, const void *X, double beta, void *Y, void *stream)
{
    if (!p || !Y) return fail(SPM_EINVAL, "spm_axpy: null pointer");
    if (!valid_prec(prec)) return fail(SPM_EINVAL, "spm_axpy: bad precision");
    return spm::launch_axpy(p, prec, alpha, X, beta, Y, (hipStream_t)stream);
}

extern "C" int spm_convert(spm_pattern p, int pf, const void *X, int pt, void *Y, void *stream)
{
    if (!p || !X || !Y) return fail(SPM_EINVAL, "spm_convert: null pointer");
    if (!valid_prec(pf) || !valid_prec(pt)) return fail(SPM_EINVAL, "spm_convert: bad precision");
    if (overlap2(X, value_bytes(p, pf), Y, value_bytes(p, pt)))
        return fail(SPM_EINVAL, "spm_convert: X and Y overlap");
    return spm::launch_convert(p, pf, X, pt, Y, (hipStream_t)stream);
}

extern "C" int spm_sqdist(spm_pattern p, int prec, const void *X, const void *Y, double *out, void *stream)
{
    if (!p || !X || !out) return fail(SPM_EINVAL, "spm_sqdist: null pointer");
    if (!valid_prec(prec)) return fail(SPM_EINVAL, "spm_sqdist: bad precision");
    return spm::launch_reduce(p, RED_SQDIST, prec, X, Y, nullptr, 0.0, 0, 1.0, out, (hipStream_t)stream);
}

extern "C" int spm_sqdist_eye(spm_pattern p, int prec, double alpha, const void *X, double *out, void *stream)
{
    if (!p || !X || !out) return fail(SPM_EINVAL, "spm_sqdist_eye: null pointer");
    if (!valid_prec(prec)) return fail(SPM_EINVAL, "spm_sqdist_eye: bad precision");
    return spm::launch_reduce(p, RED_SQDIST_EYE, prec, X, nullptr, nullptr, alpha, 0, 1.0, out, (hipStream_t)stream);
}

extern "C" int spm_dot(spm_pattern p, const double *X, const double *Y, double *out, void *stream)
{
    if (!p || !X || !Y || !out) return fail(SPM_EINVAL, "spm_dot: null pointer");
    return spm::launch_reduce(p, RED_DOT, SPM_F64, X, Y, nullptr, 0.0, 0, 1.0, out, (hipStream_t)stream);
}

extern "C" int spm_quadform(spm_pattern p, const double *X, const double *y, double *out, void *stream)
{
    if (!p || !X || !y || !out) return fail(SPM_EINVAL, "spm_quadform: null pointer");
    return spm::launch_reduce(p, RED_QUAD, SPM_F64, X, nullptr, y, 0.0, 0, 1.0, out, (hipStream_t)stream);
}

extern "C" int spm_fill_outer(spm_pattern p, double alpha, const double *y, double *X, void *stream)
{
    if (!p || !y || !X) return fail(SPM_EINVAL, "spm_fill_outer: null pointer");
    hipLaunchKernelGGL(k_fill_outer, dim3(grid1d(p->n_tiles, 1, 1 << 20)), dim3(64), 0, (hipStream_t)stream,
                       p->n_tiles, p->d_tile_off.ptr, p->d_tile_row.ptr, p->d_tile_col.ptr, p->d_nfun.ptr,
                       p->d_cstart.ptr, p->d_keep.ptr, alpha, y, X);
    SPM_HIP(hipGetLastError());
    return SPM_OK;
}

// ---------------------------------------------------------------- Newton-Schulz
namespace {

__global__ void k_fill(int64_t ns, int prec, double v, void *x)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ns; e += (int64_t)gridDim.x * blockDim.x)
        store_val(prec, x, e, ns, v);
}

size_t ns_scratch(spm_pattern p, int bulk, int32_t nbulk)
{
    size_t b = 2 * (size_t)p->n_stored * sizeof(double);
    if (bulk != SPM_F64 && nbulk > 0) b += 4 * value_bytes(p, bulk);
    return b;
}

}  // namespace

extern "C" int spm_newton_schulz_scratch(spm_pattern p, int bulk, size_t *bytes)
{
    if (!p || !bytes) return fail(SPM_EINVAL, "spm_newton_schulz_scratch: null pointer");
    if (!valid_prec(bulk)) return fail(SPM_EINVAL, "spm_newton_schulz_scratch: bad precision");
    *bytes = ns_scratch(p, bulk, 1);
    return SPM_OK;
}

extern "C" int spm_newton_schulz(spm_pattern p, const double *A, double *X, int32_t iters, int32_t nfin, int bulk,
                                 double alpha0, double *res, double *const *ckpt, void *scratch,
                                 size_t scratch_bytes, void *stream)
{
    if (!p || !A || !X || !res) return fail(SPM_EINVAL, "spm_newton_schulz: null pointer");
    if (iters < 0 || nfin < 0) return fail(SPM_EINVAL, "spm_newton_schulz: negative iteration count");
    if (!valid_prec(bulk)) return fail(SPM_EINVAL, "spm_newton_schulz: bad precision");
    const int32_t nbulk = bulk == SPM_F64 ? 0 : std::max(0, iters - nfin);
    const size_t need = ns_scratch(p, bulk, nbulk);
    if (!scratch || scratch_bytes < need) return fail(SPM_EINVAL, "spm_newton_schulz: scratch too small");
    const size_t vb8 = (size_t)p->n_stored * sizeof(double);
    if (overlap(A, X, vb8) || overlap2(X, vb8, scratch, need) || overlap2(A, vb8, scratch, need))
        return fail(SPM_EINVAL, "spm_newton_schulz: buffers overlap");
    hipStream_t s = (hipStream_t)stream;
    const int64_t ns = p->n_stored;
    const double rs = 1.0 / std::sqrt((double)p->n);
    double *Y = static_cast<double *>(scratch);
    double *T = Y + ns;
    char *sp = reinterpret_cast<char *>(T + ns);
    const size_t vb = value_bytes(p, bulk);
    void *As = sp, *Xs = sp + vb, *Ys = sp + 2 * vb, *Ts = sp + 3 * vb;
    double *cur = X, *oth = T;
    int st;
    hipLaunchKernelGGL(k_fill, dim3(grid1d(ns, 256)), dim3(256), 0, s, ns, (int)SPM_F64, 0.0, (void *)cur);
    if ((st = spm::launch_axpy(p, SPM_F64, alpha0, nullptr, 1.0, cur, s))) return st;
    if (nbulk > 0) {
        if ((st = spm::launch_convert(p, SPM_F64, A, bulk, As, s))) return st;
        if ((st = spm::launch_convert(p, SPM_F64, cur, bulk, Xs, s))) return st;
    }
    for (int32_t k = 0; k < iters; ++k) {
        const bool low = k < nbulk;
        if (ckpt && ckpt[k]) {
            if (low) { if ((st = spm::launch_convert(p, bulk, Xs, SPM_F64, ckpt[k], s))) return st; }
            else SPM_HIP(hipMemcpyAsync(ckpt[k], cur, vb8, hipMemcpyDeviceToDevice, s));
        }
        if (low) {
            if ((st = spm::launch_gemm(p, bulk, As, 0, Xs, 0, Ys, s))) return st;
            if ((st = spm::launch_reduce(p, 1, bulk, Ys, nullptr, nullptr, 1.0, 1, rs, res + k, s))) return st;
            if ((st = spm::launch_axpy(p, bulk, 2.0, nullptr, -1.0, Ys, s))) return st;
            if ((st = spm::launch_gemm(p, bulk, Xs, 0, Ys, 0, Ts, s))) return st;
            std::swap(Xs, Ts);
            if (k == nbulk - 1 && (st = spm::launch_convert(p, bulk, Xs, SPM_F64, cur, s))) return st;
        } else {
            if ((st = spm::launch_gemm(p, SPM_F64, A, 0, cur, 0, Y, s))) return st;
            if ((st = spm::launch_reduce(p, 1, SPM_F64, Y, nullptr, nullptr, 1.0, 1, rs, res + k, s))) return st;
            if ((st = spm::launch_axpy(p, SPM_F64, 2.0, nullptr, -1.0, Y, s))) return st;
            if ((st = spm::launch_gemm(p, SPM_F64, cur, 0, Y, 0, oth, s))) return st;
            std::swap(cur, oth);
        }
    }
    if (ckpt && ckpt[iters]) SPM_HIP(hipMemcpyAsync(ckpt[iters], cur, vb8, hipMemcpyDeviceToDevice, s));
    if ((st = spm::launch_gemm(p, SPM_F64, A, 0, cur, 0, Y, s))) return st;
    if ((st = spm::launch_reduce(p, 1, SPM_F64, Y, nullptr, nullptr, 1.0, 1, rs, res + iters, s))) return st;
    if (cur != X) SPM_HIP(hipMemcpyAsync(X, cur, vb8, hipMemcpyDeviceToDevice, s));
    double last = 0.0;
    SPM_HIP(hipMemcpyAsync(&last, res + iters, sizeof(double), hipMemcpyDeviceToHost, s));
    SPM_HIP(hipStreamSynchronize(s));
    if (!std::isfinite(last)) return fail(SPM_ENOTCONV, "spm_newton_schulz: residual is not finite");
    return SPM_OK;
}
