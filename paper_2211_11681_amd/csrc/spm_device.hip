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

template <int TA, int TB>
__global__ __launch_bounds__(64) void k_mgemm_f64(GemmArgs g, const double *__restrict__ A,
                                                 const double *__restrict__ B, double *__restrict__ C)
{
    __shared__ double sA[kMax * kMax];   // sA[k * kMax + i] = op(A)_{r,mu}(i, k)
    __shared__ double sB[kMax * kMax];   // sB[k * kMax + j] = op(B)_{mu,c}(k, j)
    __shared__ int32_t sPa[64], sPb[64];
    const int lane = threadIdx.x;
    const int64_t t = g.order[blockIdx.x];
    const int r = g.tile_row[t], c = g.tile_col[t];
    const int nr = g.nfun[r], ncl = g.nfun[c];
    const int64_t ra = g.blk_rp[r], la = g.blk_rp[r + 1] - ra;
    const int64_t rb = g.blk_rp[c], lb = g.blk_rp[c + 1] - rb;
    const bool a_short = la <= lb;
    const int64_t rs = a_short ? ra : rb, ls = a_short ? la : lb;
    const int64_t rl = a_short ? rb : ra, ll = a_short ? lb : la;
    const int nout = nr * ncl;
    double acc[kMax * kMax / 64];
#pragma unroll
    for (int s = 0; s < kMax * kMax / 64; ++s) acc[s] = 0.0;

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
            const int64_t ta = ra + sPa[f];      // tile (r, mu)
            const int64_t tb = rb + sPb[f];      // tile (c, mu)
            const int mu = g.tile_col[ta];
            const int nm = g.nfun[mu];
            // op(A)_{r,mu}
            if (TA == 0) {
                const double *src = A + g.tile_off[ta];          // (i, k) at k * nr + i
                for (int e = lane; e < nr * nm; e += 64) { int i = e % nr, k = e / nr; sA[k * kMax + i] = src[e]; }
            } else {
                const double *src = A + g.tile_off[g.trans[ta]]; // tile (mu, r): (k, i) at i * nm + k
                for (int e = lane; e < nr * nm; e += 64) { int k = e % nm, i = e / nm; sA[k * kMax + i] = src[e]; }
            }
            // op(B)_{mu,c}
            if (TB == 0) {
                const double *src = B + g.tile_off[g.trans[tb]]; // tile (mu, c): (k, j) at j * nm + k
                for (int e = lane; e < nm * ncl; e += 64) { int k = e % nm, j = e / nm; sB[k * kMax + j] = src[e]; }
            } else {
                const double *src = B + g.tile_off[tb];          // tile (c, mu): (j, k) at k * ncl + j
                for (int e = lane; e < nm * ncl; e += 64) { int j = e % ncl, k = e / ncl; sB[k * kMax + j] = src[e]; }
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < kMax * kMax / 64; ++s) {
                const int e = lane + 64 * s;
                if (e < nout) {
                    const int i = e % nr, j = e / nr;
                    double a = acc[s];
                    for (int k = 0; k < nm; ++k) a = fma(sA[k * kMax + i], sB[k * kMax + j], a);
                    acc[s] = a;
                }
            }
            __syncthreads();
        }
    }
    const int64_t off = g.tile_off[t];
#pragma unroll
    for (int s = 0; s < kMax * kMax / 64; ++s) {
        const int e = lane + 64 * s;
        if (e < nout) C[off + e] = acc[s];
    }
}

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

int launch_gemm(spm_pattern p, int prec, const void *A, int ta, const void *B, int tb, void *C, hipStream_t s)
{
    if (p->n_tiles == 0) return SPM_OK;
    GemmArgs g = gemm_args(p);
    dim3 grid((unsigned)p->n_tiles), block(64);
    const int sel = (ta ? 2 : 0) + (tb ? 1 : 0);
    if (prec == SPM_F64) {
        auto a = static_cast<const double *>(A);
        auto b = static_cast<const double *>(B);
        auto c = static_cast<double *>(C);
        switch (sel) {
        case 0: hipLaunchKernelGGL((k_mgemm_f64<0, 0>), grid, block, 0, s, g, a, b, c); break;
        case 1: hipLaunchKernelGGL((k_mgemm_f64<0, 1>), grid, block, 0, s, g, a, b, c); break;
        case 2: hipLaunchKernelGGL((k_mgemm_f64<1, 0>), grid, block, 0, s, g, a, b, c); break;
        default: hipLaunchKernelGGL((k_mgemm_f64<1, 1>), grid, block, 0, s, g, a, b, c); break;
        }
    } else {
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
