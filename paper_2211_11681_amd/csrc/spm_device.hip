// Device side of libspm for gfx950: pattern upload, elementwise ops, deterministic
// reductions, the masked product and the Newton-Schulz driver.
#include <hip/hip_runtime.h>
#include <mutex>
#include <set>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "spm_internal.h"

using spm::fail;

namespace spm {

static constexpr int kRedTiles = 64;      // tiles per reduction block
static constexpr int kRedThreads = 256;
static constexpr size_t kTableAlign = 256;

namespace {

inline size_t align_up(size_t x) { return (x + kTableAlign - 1) & ~(kTableAlign - 1); }

// Visits every device table of the pattern with its host source: f(device buffer, host
// vector).  The keep mask and the reduction partials have no host vector; they are
// handled by the callers.
template <class F>
void for_each_table(spm_pattern_s *p, F &&f)
{
    f(p->d_cstart, p->cstart); f(p->d_blk_rp, p->blk_rp); f(p->d_tile_off, p->tile_off);
    f(p->d_colprefix, p->colprefix); f(p->d_rowbase, p->rowbase); f(p->d_rowlen, p->rowlen);
    f(p->d_pc_rp, p->pc_rp); f(p->d_pc_off, p->pc_off); f(p->d_pc_g, p->pc_g); f(p->d_pc_w, p->pc_w);
    f(p->d_nfun, p->nfun); f(p->d_tile_row, p->tile_row); f(p->d_tile_col, p->tile_col);
    f(p->d_trans, p->trans); f(p->d_diag_tile, p->diag_tile); f(p->d_order, p->order);
    f(p->d_grp_mem, p->grp_mem); f(p->d_grp_s, p->grp_s); f(p->d_grp_g, p->grp_g); f(p->d_grp_R, p->grp_R);
    f(p->d_gl_rp, p->gl_rp); f(p->d_gl_mu, p->gl_mu); f(p->d_gl_tile, p->gl_tile);
    f(p->d_unit_gr, p->unit_gr); f(p->d_unit_gc, p->unit_gc); f(p->d_unit_out, p->unit_out);
    f(p->d_unit_order, p->unit_order); f(p->d_pair_off, p->pair_off); f(p->d_pair_a, p->pair_a);
    f(p->d_pair_b, p->pair_b); f(p->d_gl_nm, p->gl_nm); f(p->d_gl_offd, p->gl_offd);
    f(p->d_stage_off, p->stage_off); f(p->d_stage_first, p->stage_first); f(p->d_csr_pos, p->csr_pos);
    f(p->d_clevel, p->clevel); f(p->d_gl_nml, p->gl_nml); f(p->d_gl_offT, p->gl_offT);
    f(p->d_stage_off_lv, p->stage_off_lv); f(p->d_stage_first_lv, p->stage_first_lv);
    f(p->d_pair_a_lv, p->pair_a_lv); f(p->d_pair_b_lv, p->pair_b_lv); f(p->d_diag_pos, p->diag_pos);
}

static constexpr int kFlatBlocks = 2048;  // fixed grid of the flat reductions (so a fixed summation order)
int64_t partial_count(const spm_pattern_s *p)
{
    return std::max<int64_t>((p->n_tiles + kRedTiles - 1) / kRedTiles + 1, kFlatBlocks);
}

}  // namespace

size_t pattern_device_bytes(const spm_pattern_s *pc)
{
    spm_pattern_s *p = const_cast<spm_pattern_s *>(pc);
    size_t b = 0;
    for_each_table(p, [&](auto &, const auto &v) { b += align_up(v.size() * sizeof(v[0])); });
    if (p->masked) b += align_up((size_t)p->n_stored);
    b += align_up((size_t)partial_count(p) * sizeof(double));
    return b;
}

int upload_pattern_device(spm_pattern_s *p, void *ws, size_t bytes, hipStream_t s)
{
    (void)s;
    const size_t need = pattern_device_bytes(p);
    if (ws) {
        if (bytes < need) return fail(SPM_EINVAL, "pattern upload: workspace too small");
        if (reinterpret_cast<uintptr_t>(ws) % kTableAlign)
            return fail(SPM_EINVAL, "pattern upload: workspace not aligned to 256 bytes");
        p->dev_block = ws;
        p->owns_block = false;
    } else {
        if (hipMalloc(&p->dev_block, need) != hipSuccess) {
            p->dev_block = nullptr;
            return fail(SPM_ENOMEM, "device allocation for the pattern layout");
        }
        p->owns_block = true;
    }
    char *base = static_cast<char *>(p->dev_block);
    size_t off = 0;
    int st = SPM_OK;
    // blocking copies: the host tables may be modified or freed by the caller afterwards
    for_each_table(p, [&](auto &d, const auto &v) {
        using T = std::remove_reference_t<decltype(v[0])>;
        d.n = v.size();
        d.ptr = v.empty() ? nullptr : reinterpret_cast<std::remove_const_t<T> *>(base + off);
        if (!st && !v.empty() && hipMemcpy(d.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
            st = fail(SPM_EHIP, "pattern upload: hipMemcpy failed");
        off += align_up(v.size() * sizeof(T));
    });
    if (st) return st;
    if (p->masked) {
        std::vector<uint8_t> keep(p->n_stored);
        for (int64_t e = 0; e < p->n_stored; ++e) keep[e] = p->csr_pos[e] >= 0;
        p->d_keep.ptr = reinterpret_cast<uint8_t *>(base + off);
        p->d_keep.n = keep.size();
        SPM_HIP(hipMemcpy(p->d_keep.ptr, keep.data(), keep.size(), hipMemcpyHostToDevice));
        off += align_up((size_t)p->n_stored);
    }
    std::vector<double> zeros(partial_count(p), 0.0);
    p->d_partial.ptr = reinterpret_cast<double *>(base + off);
    p->d_partial.n = zeros.size();
    SPM_HIP(hipMemcpy(p->d_partial.ptr, zeros.data(), zeros.size() * sizeof(double), hipMemcpyHostToDevice));
    p->uploaded = true;
    return SPM_OK;
}

void free_pattern_device(spm_pattern_s *p)
{
    if (p->owns_block && p->dev_block) (void)hipFree(p->dev_block);
    p->dev_block = nullptr;
    p->owns_block = false;
    p->uploaded = false;
    for_each_table(p, [&](auto &d, const auto &) { d.ptr = nullptr; d.n = 0; });
    p->d_keep = {};
    p->d_partial = {};
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

// Sum of squares, squared distance and dot product over the stored entries in storage
// order, as one coalesced pass: workgroup b owns a fixed contiguous range of 4096-entry
// segments, and each thread sums entries tid + 256 k of each segment.  For
// sum (alpha I - X)^2 the diagonal entries of the segment are marked in an LDS bitmap
// from the ascending list of diagonal positions (the list pointer only moves forward).
constexpr int kFlatSeg = 4096;
template <int PREC, int OP>
__global__ __launch_bounds__(256) void k_reduce_flat(int64_t ns, const void *x, const void *y,
                                                     const int64_t *__restrict__ diag, int64_t ndiag,
                                                     double alpha, double *partial)
{
    __shared__ double red[256];
    __shared__ uint32_t mark[kFlatSeg / 32];
    const int tid = threadIdx.x;
    const int64_t nseg = (ns + kFlatSeg - 1) / kFlatSeg;
    const int64_t per = (nseg + gridDim.x - 1) / gridDim.x;
    const int64_t g0 = (int64_t)blockIdx.x * per, g1 = min(nseg, g0 + per);
    double acc = 0.0;
    int64_t q = 0;
    if (OP == RED_SQDIST_EYE && g0 < g1) {
        int64_t lo = 0, hi = ndiag;                       // first diagonal position >= segment g0
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (diag[mid] < g0 * kFlatSeg) lo = mid + 1;
            else hi = mid;
        }
        q = lo;
    }
    for (int64_t g = g0; g < g1; ++g) {
        const int64_t a = g * kFlatSeg;
        if (OP == RED_SQDIST_EYE) {
            for (int w = tid; w < kFlatSeg / 32; w += 256) mark[w] = 0;
            __syncthreads();
            for (;;) {
                const int64_t qq = q + tid;
                const bool in = qq < ndiag && diag[qq] < a + kFlatSeg;
                if (in) {
                    const int o = (int)(diag[qq] - a);
                    atomicOr(&mark[o >> 5], 1u << (o & 31));
                }
                const int cnt = __syncthreads_count(in);
                q += cnt;
                if (cnt < 256) break;
            }
        }
        double xv[16], yv[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int64_t e = a + tid + 256 * k;
            xv[k] = e < ns ? load_val(PREC, x, e, ns) : 0.0;
            yv[k] = ((OP == RED_SQDIST && y) || OP == RED_DOT) && e < ns ? load_val(PREC, y, e, ns) : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int o = tid + 256 * k;
            if (OP == RED_DOT) {
                acc += xv[k] * yv[k];
            } else {
                double d = xv[k] - yv[k];
                if (OP == RED_SQDIST_EYE && (mark[o >> 5] >> (o & 31) & 1u)) d = alpha - xv[k];
                acc += d * d;
            }
        }
        if (OP == RED_SQDIST_EYE) __syncthreads();     // the bitmap is cleared for the next segment
    }
    red[tid] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) partial[blockIdx.x] = red[0];
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
// Computes C = P_S(A B^T) for A and B in the tile layout (the callers transpose
// operands beforehand so that every product has this form).
//
// One unit (G_r, G_c) = the output tiles between the (up to 4) row clusters of G_r
// and the column clusters of G_c, held as 16x16 blocks of MFMA accumulators.  The
// unit's middle clusters mu (U(G_r) cap U(G_c), listed by the schedule builder) come
// in stages of consecutive clusters with at most 32 padded k rows.  Per stage the
// panels A_{G_r,mu} (R x k) and (B_{G_c,mu})^T (k x C) are gathered into LDS, k-major
// with row stride Xa (Xb), a power of two, by direct global-to-LDS loads: every tile
// of the layout is column-major, so consecutive panel rows of one k are consecutive
// source elements.  WIDTH = 16: two doubles per lane, 128 per wave instruction (all
// cluster sizes even); WIDTH = 4: one dword per lane, 32 doubles per instruction.
// Absent tiles and padding read a zero word.  The panels feed v_mfma_f64_16x16x4f64
// (lane l: A row l%16 and k l/16, B column l%16 and k l/16; accumulator register r
// holds row 4r + l/16, column l%16).  Panels are double-buffered: the gathers of
// stage s+1 and the stage records of stage s+2 are in flight while the MFMAs of
// stage s run; the records are fetched in three dependent steps spread over three
// stages.  WAVES = 8: big units; WAVES = 1: 16 x 16 units.
typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ double g_zero_word[2];   // zero-initialised source of padding (16 bytes)

struct GroupArgs {
    const int32_t *grp_mem, *grp_s, *grp_g;
    const int32_t *unit_gr, *unit_gc, *unit_out, *unit_order;
    const int64_t *pair_off;
    const int32_t *pair_a, *pair_b;
    const int32_t *gl_nm;
    const int64_t *gl_offd;
    const int64_t *stage_off;
    const int32_t *stage_first;
    const int64_t *tile_off;
    const int32_t *nfun;
    int64_t first, count;
    int32_t RB, CB;
    int32_t lxa, lxb;        // log2 of the panel row strides
    int32_t WR, WC, nsplit;  // wave grid over the blocks and number of k slices
};

constexpr int kKS = 32;   // k rows per stage
constexpr int kSP = 8;    // middle clusters per stage

// Stage records, one per k row: for each of the 8 member slots (0..3 row members, 4..7
// column members) the element offset of column k of the member's tile, i.e. tile offset
// plus (k row inside the middle cluster) x (member size); -1 where the tile is absent
// or the row is padding.
struct KTab {
    int64_t kofs[kKS][8];
    int32_t ks;           // k rows of the stage (its clusters packed without padding)
    int32_t act;          // bit q (row member q), 4 + q (column member q): the member has a
                          // tile in some middle cluster of the stage (grouped kernel only)
    int32_t pad[2];
};

template <int WAVES>
__device__ inline void unit_sync()
{
    __builtin_amdgcn_s_waitcnt(0);
    if (WAVES > 1) __syncthreads();
    else __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <int WIDTH>
__device__ inline void lds_gather(const double *src, int half, double *dst)
{
    if constexpr (WIDTH == 16)
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
    else
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint32_t *>(src) + half,
                                         (__attribute__((address_space(3))) void *)dst, 4, 0, 0);
}

__device__ inline int sel4(int k, int a0, int a1, int a2, int a3)
{
    return k == 0 ? a0 : k == 1 ? a1 : k == 2 ? a2 : a3;
}

// Lane constants of one gather variant: the panel row x this lane fills, as member slot
// and row inside the member.
struct GatherLane {
    int slot, i;
    bool ok;
};

__device__ inline GatherLane gather_lane(int x, int s, int ng, int n0, int n1, int n2, int n3)
{
    GatherLane r;
    r.slot = x / s;
    r.i = x - r.slot * s;
    r.ok = r.slot < ng && r.i < sel4(r.slot & 3, n0, n1, n2, n3);
    r.slot &= 3;
    return r;
}

// Gathers one operand panel of a stage: instruction `ins` covers the doubles
// [D*ins, D*ins + D) of the k-major panel with row stride 2^lx; nv = max(1, 2^lx / D)
// lane variants.  Every load of the stage goes to LDS directly; nothing waits here.
template <int WAVES, int WIDTH>
__device__ inline void gather_panel(const KTab *T, int slot_base, const double *__restrict__ M,
                                    double *panel, int ks, int lx, int wave, int dl, int half,
                                    const GatherLane (&gl)[4], const double *zero)
{
    constexpr int D = WIDTH * 8;
    constexpr int LD = WIDTH == 16 ? 7 : 5;   // log2 D
    const int X = 1 << lx;
    // whole k steps: the MFMAs read rows up to the next multiple of 4, and rows past the
    // stage's last cluster have offset -1 in the record (zero words)
    const int nins = (((ks + 3) & ~3) * X + D - 1) >> LD;
    // with 16-byte lanes D = 128 >= X always (rows are at most 128 wide)
    if (WIDTH == 16 || lx <= LD) {
        // D >= X: lane row x is fixed, k = ins * (D / X) + (dl >> lx)
        const GatherLane g = gl[0];
        const int kstep = 1 << (LD - lx);
        const char *trow = reinterpret_cast<const char *>(&T->kofs[dl >> lx][slot_base + g.slot]);
        const int rstride = kstep * 64 * WAVES;   // bytes between the records of consecutive instructions
        for (int ins = wave; ins < nins; ins += 4 * WAVES) {
            // four record reads in flight before the gathers that use them
            int64_t o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int iq = ins + q * WAVES < nins ? ins + q * WAVES : ins;
                o[q] = *reinterpret_cast<const int64_t *>(trow + (size_t)iq * kstep * 64);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (ins + q * WAVES >= nins) break;
                const double *src = (g.ok && o[q] >= 0) ? M + o[q] + g.i : zero;
                lds_gather<WIDTH>(src, half, panel + (ins + q * WAVES) * D);
            }
        }
        (void)rstride;
    } else if constexpr (WIDTH != 16) {
        // D < X: variant v = ins % nv covers rows [v*D, v*D + D), k = ins / nv
        const int lnv = lx - LD, nv = 1 << lnv;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (v >= nv) break;
            if (WAVES > 1 && WAVES >= nv && v != (wave & (nv - 1))) continue;
            const GatherLane g = gl[v];
            const int step = WAVES > nv ? WAVES : nv;
            const int first = WAVES >= nv ? wave : v + wave * nv;
            const int ins_step = WAVES >= nv ? step : WAVES * nv;
            for (int ins = first; ins < nins; ins += ins_step) {
                const int kk = ins >> lnv;
                const int64_t o = T->kofs[kk][slot_base + g.slot];
                const double *src = (g.ok && o >= 0) ? M + o + g.i : zero;
                lds_gather<WIDTH>(src, half, panel + ins * D);
            }
        }
    }
}

template <int WAVES, int WIDTH, int MR, int MC>
__global__ __launch_bounds__(WAVES * 64) void k_mgemm_grp(GroupArgs g, const double *__restrict__ A,
                                                         const double *__restrict__ B, double *__restrict__ C)
{
    extern __shared__ double lds[];
    constexpr int D = WIDTH * 8;                   // doubles per gather instruction
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = WAVES == 1 ? 0 : __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t uidx = blockIdx.x;
    if (uidx >= g.count) return;
    const int Xa = 1 << g.lxa, Xb = 1 << g.lxb;
    const int pd = kKS * (Xa + Xb);                // doubles of one operand buffer
    KTab *ktab = reinterpret_cast<KTab *>(lds + 2 * pd);

    const int u = g.unit_order[g.first + uidx];
    const int gr = g.unit_gr[u], gc = g.unit_gc[u];
    const int sr = g.grp_s[gr], sc = g.grp_s[gc];
    const int ngr = g.grp_g[gr], ngc = g.grp_g[gc];
    const int nr0 = g.nfun[g.grp_mem[gr * 4]];
    const int nr1 = ngr > 1 ? g.nfun[g.grp_mem[gr * 4 + 1]] : 0;
    const int nr2 = ngr > 2 ? g.nfun[g.grp_mem[gr * 4 + 2]] : 0;
    const int nr3 = ngr > 3 ? g.nfun[g.grp_mem[gr * 4 + 3]] : 0;
    const int nc0 = g.nfun[g.grp_mem[gc * 4]];
    const int nc1 = ngc > 1 ? g.nfun[g.grp_mem[gc * 4 + 1]] : 0;
    const int nc2 = ngc > 2 ? g.nfun[g.grp_mem[gc * 4 + 2]] : 0;
    const int nc3 = ngc > 3 ? g.nfun[g.grp_mem[gc * 4 + 3]] : 0;
    // wave (wr, wc, kslice) owns the blocks (wr + i WR, wc + j WC), i < MR, j < MC, over
    // the k rows of its slice
    const int nw = g.WR * g.WC, nsplit = g.nsplit;
    const bool active = wave < nw * nsplit;
    const int wr = wave % g.WR, wc = (wave / g.WR) % g.WC, kslice = wave / nw;
    // per-unit bases, so that the stage loop keeps few uniform values live
    const int64_t s0 = g.stage_off[u], p0 = g.pair_off[u];
    const int nst = (int)(g.stage_off[u + 1] - s0), npairs = (int)(g.pair_off[u + 1] - p0);
    const int32_t *const stf = g.stage_first + s0;
    const int32_t *const ptab = (lane & 7) < 4 ? g.pair_a + p0 : g.pair_b + p0;   // this lane's list

    // per lane gather constants (variant v covers panel rows v*D .. v*D + D - 1 when D < X)
    const int dl = WIDTH == 16 ? 2 * lane : lane >> 1;
    const int half = lane & 1;
    GatherLane gla[4], glb[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int xa = D >= Xa ? (dl & (Xa - 1)) : v * D + dl;
        const int xb = D >= Xb ? (dl & (Xb - 1)) : v * D + dl;
        gla[v] = gather_lane(xa, sr, ngr, nr0, nr1, nr2, nr3);
        glb[v] = gather_lane(xb, sc, ngc, nc0, nc1, nc2, nc3);
    }
    const double *const zero = g_zero_word;
    // member sizes of the record writer's slots (lanes 0..31 row members, 32..63 column)
    int nslot[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) nslot[q] = lane < 32 ? sel4(q, nr0, nr1, nr2, nr3) : sel4(q, nc0, nc1, nc2, nc3);

    // ---- stage records, fetched by one wave in three steps (bounds -> union entries ->
    // offsets), one step per stage; each step only consumes loads of earlier stages, so
    // no stage waits for its own loads.  Lane (p, slot): middle cluster p of the stage,
    // slot 0..3 row members, 4..7 column members; slot 0 also carries the cluster size.
    // the stage records are kept by a wave without MFMA blocks when there is one
    const int twave = nw * nsplit < WAVES ? WAVES - 1 : 0;
    const int tp = lane >> 3, tslot = lane & 7, tk = tslot & 3;
    const bool tvalid = tslot < 4 ? tk < ngr : tk < ngc;
    // bounds of a stage: lane 0 loads its first union entry, lane 1 the end (per lane, so
    // that the value stays in a vector register and is only waited for at the next sync)
    auto load_bounds = [&](int st, int32_t &fbe) {
        fbe = 0;
        if (wave != twave || st >= nst || lane > 1) return;
        fbe = lane == 0 || st + 1 < nst ? stf[st + lane] : npairs;
    };
    auto load_entry = [&](int32_t fb, int np, int32_t &e) {
        e = -1;
        if (wave != twave || tp >= np) return;
        e = ptab[fb + tp];
    };
    auto load_offsets = [&](int32_t e, int64_t &off, int32_t &nm) {
        off = -1;
        nm = 0;
        if (e < 0) return;
        if (tvalid) off = g.gl_offd[(int64_t)e * 4 + tk];
        if (tslot == 0) nm = g.gl_nm[e];
    };
    auto write_tab = [&](KTab *T, int64_t t_off, int t_nm, int t_np) {
        if (wave != twave) return;
        int nmv[kSP], kbv[kSP];
        int kacc = 0;
#pragma unroll
        for (int q = 0; q < kSP; ++q) {
            nmv[q] = __shfl(t_nm, q * 8);
            kbv[q] = kacc;
            kacc += q < t_np ? nmv[q] : 0;
        }
        const int kk = lane & 31;
        const bool rows = lane < 32;
        int m = -1;
#pragma unroll
        for (int q = 0; q < kSP; ++q)
            if (q < t_np && kk >= kbv[q] && kk < kbv[q] + nmv[q]) m = q;
        const int mm = m < 0 ? 0 : m;
        int nmm = 0, kbm = 0;
#pragma unroll
        for (int q = 0; q < kSP; ++q)
            if (q == mm) { nmm = nmv[q]; kbm = kbv[q]; }
        const int kkm = kk - kbm;
        const bool live = m >= 0 && kkm < nmm;
        int act = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t o = __shfl(t_off, mm * 8 + (rows ? 0 : 4) + q);
            const int n = nslot[q];
            const bool on = live && o >= 0;
            T->kofs[kk][(rows ? 0 : 4) + q] = on ? o + (int64_t)kkm * n : -1;
            const uint64_t b = __builtin_amdgcn_ballot_w64(on);
            act |= ((uint32_t)b != 0 ? 1 << q : 0) | ((b >> 32) != 0 ? 16 << q : 0);
        }
        if (lane == 0) {
            T->ks = kacc;
            T->act = act;
        }
    };

    dbl4 acc[MR][MC];
#pragma unroll
    for (int i = 0; i < MR; ++i)
#pragma unroll
        for (int j = 0; j < MC; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int lr = lane & 15, lk = lane >> 4;
    int arow[MR], bcol[MC];                         // panel row offsets of the owned blocks (clamped)
#pragma unroll
    for (int i = 0; i < MR; ++i) arow[i] = 16 * min(wr + i * g.WR, g.RB - 1) + lr;
#pragma unroll
    for (int j = 0; j < MC; ++j) bcol[j] = 16 * min(wc + j * g.WC, g.CB - 1) + lr;
    // members covering each owned block (bits of KTab::act): a block none of whose row (or
    // column) members has a tile in the stage's middle clusters adds only zeros
    int amask[MR], bmask[MC];
#pragma unroll
    for (int i = 0; i < MR; ++i) {
        const int r0 = 16 * min(wr + i * g.WR, g.RB - 1), m0 = r0 / sr, m1 = min((r0 + 15) / sr, 3);
        amask[i] = ((2 << m1) - 1) & ~((1 << m0) - 1);
    }
#pragma unroll
    for (int j = 0; j < MC; ++j) {
        const int c0 = 16 * min(wc + j * g.WC, g.CB - 1), m0 = c0 / sc, m1 = min((c0 + 15) / sc, 3);
        bmask[j] = (((2 << m1) - 1) & ~((1 << m0) - 1)) << 4;
    }

    // prologue: records of stages 0 and 1 written; in registers: offsets of stage 2,
    // entries of stage 3, bounds of stage 4 (all loads complete at the first sync)
    int32_t fbe, e;
    int64_t off;
    int32_t nm;
    auto fb_of = [&](int32_t v) { return __builtin_amdgcn_readlane(v, 0); };
    auto np_of = [&](int32_t v) { return __builtin_amdgcn_readlane(v, 1) - __builtin_amdgcn_readlane(v, 0); };
    for (int st = 0; st < 2; ++st) {
        load_bounds(st, fbe);
        load_entry(fb_of(fbe), np_of(fbe), e);
        load_offsets(e, off, nm);
        write_tab(&ktab[st], off, nm, np_of(fbe));
    }
    load_bounds(2, fbe);
    int np2 = np_of(fbe);
    load_entry(fb_of(fbe), np2, e);
    load_offsets(e, off, nm);                      // stage 2
    load_bounds(3, fbe);
    int np3 = np_of(fbe);
    load_entry(fb_of(fbe), np3, e);                // stage 3
    load_bounds(4, fbe);                           // stage 4
    unit_sync<WAVES>();
    int ks_next = ktab[0].ks, act_next = ktab[0].act;
    if (nst > 0) {
        gather_panel<WAVES, WIDTH>(&ktab[0], 0, A, lds, ks_next, g.lxa, wave, dl, half, gla, zero);
        gather_panel<WAVES, WIDTH>(&ktab[0], 4, B, lds + kKS * Xa, ks_next, g.lxb, wave, dl, half, glb, zero);
    }
    // Iteration s: records s+2 are written into the slot of stage s (whose gathers were
    // issued one iteration earlier), the record loads advance by one stage, the gathers
    // of stage s+1 are issued, then the MFMAs of stage s run.  Nothing issued in an
    // iteration is consumed before the sync that opens the next one.
    for (int s = 0; s < nst; ++s) {
        unit_sync<WAVES>();                         // gathers of stage s landed; MFMAs of s-1 done
        const int ks_s = ks_next, act_s = act_next;
        const int np4 = np_of(fbe);
        const int32_t fb4 = fb_of(fbe);
        write_tab(&ktab[s & 1], off, nm, np2);      // stage s+2
        load_offsets(e, off, nm);                   // stage s+3
        load_entry(fb4, np4, e);                    // stage s+4
        load_bounds(s + 5, fbe);                    // stage s+5
        np2 = np3;
        np3 = np4;
        if (s + 1 < nst) {
            const KTab *T1 = &ktab[(s + 1) & 1];
            double *buf = lds + ((s + 1) & 1) * pd;
            ks_next = T1->ks;
            act_next = T1->act;
            gather_panel<WAVES, WIDTH>(T1, 0, A, buf, ks_next, g.lxa, wave, dl, half, gla, zero);
            gather_panel<WAVES, WIDTH>(T1, 4, B, buf + kKS * Xa, ks_next, g.lxb, wave, dl, half, glb, zero);
        }
        if (active) {
            const double *sA = lds + (s & 1) * pd, *sB = sA + kKS * Xa;
            if constexpr (WAVES <= 2 || MR * MC <= 2 || MR + MC >= 8) {
                // the fragments of all (up to 8) k steps of the stage are read first, then
                // the MFMAs issue back to back (patches of 16 or fewer fragment registers
                // per k step; the wide 1 x 7 patches run at one workgroup per CU and have
                // the registers)
                double fa[8][MR], fb[8][MC];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int kr = min(4 * (kslice + t * nsplit), kKS - 4) + lk;
#pragma unroll
                    for (int i = 0; i < MR; ++i) fa[t][i] = sA[kr * Xa + arow[i]];
#pragma unroll
                    for (int j = 0; j < MC; ++j) fb[t][j] = sB[kr * Xb + bcol[j]];
                }
                bool on[MR][MC];
#pragma unroll
                for (int i = 0; i < MR; ++i)
#pragma unroll
                    for (int j = 0; j < MC; ++j) on[i][j] = (act_s & amask[i]) != 0 && (act_s & bmask[j]) != 0;
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (4 * (kslice + t * nsplit) < ks_s)
#pragma unroll
                        for (int i = 0; i < MR; ++i)
#pragma unroll
                            for (int j = 0; j < MC; ++j)
                                if (on[i][j])
                                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[t][i], fb[t][j], acc[i][j], 0, 0, 0);
            } else {
                // fragments of the next k step are read while the MFMAs of this one run
                int k0 = 4 * kslice;
                double fa[MR], fb[MC];
#pragma unroll
                for (int i = 0; i < MR; ++i) fa[i] = sA[(k0 + lk) * Xa + arow[i]];
#pragma unroll
                for (int j = 0; j < MC; ++j) fb[j] = sB[(k0 + lk) * Xb + bcol[j]];
                for (; k0 < ks_s; k0 += 4 * nsplit) {
                    const int kn = min(k0 + 4 * nsplit, kKS - 4) + lk;
                    double na[MR], nb[MC];
#pragma unroll
                    for (int i = 0; i < MR; ++i) na[i] = sA[kn * Xa + arow[i]];
#pragma unroll
                    for (int j = 0; j < MC; ++j) nb[j] = sB[kn * Xb + bcol[j]];
#pragma unroll
                    for (int i = 0; i < MR; ++i)
#pragma unroll
                        for (int j = 0; j < MC; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
#pragma unroll
                    for (int i = 0; i < MR; ++i) fa[i] = na[i];
#pragma unroll
                    for (int j = 0; j < MC; ++j) fb[j] = nb[j];
                }
            }
        }
    }
    if (nsplit > 1) {                               // add the k slices in a fixed order
        unit_sync<WAVES>();
        // waves nw.. hold the partial sums of k slices 1..nsplit-1: slot (wave - nw)
        if (active && kslice > 0)
#pragma unroll
            for (int i = 0; i < MR; ++i)
#pragma unroll
                for (int j = 0; j < MC; ++j)
                    for (int r = 0; r < 4; ++r)
                        lds[((((wave - nw) * MR + i) * MC + j) * 4 + r) * 64 + lane] = acc[i][j][r];
        unit_sync<WAVES>();
        if (active && kslice == 0)
            for (int sl = 1; sl < nsplit; ++sl) {
                const int w2 = sl * nw + wave;
#pragma unroll
                for (int i = 0; i < MR; ++i)
#pragma unroll
                    for (int j = 0; j < MC; ++j)
                        for (int r = 0; r < 4; ++r)
                            acc[i][j][r] += lds[((((w2 - nw) * MR + i) * MC + j) * 4 + r) * 64 + lane];
            }
    }
    if (!active || kslice != 0) return;
    // store the output tiles that belong to S (member sizes re-read here rather than
    // kept live through the stage loop)
    const int gr2 = g.unit_gr[u], gc2 = g.unit_gc[u];
    const int sr2 = g.grp_s[gr2], sc2 = g.grp_s[gc2], ngr2 = g.grp_g[gr2], ngc2 = g.grp_g[gc2];
#pragma unroll
    for (int i = 0; i < MR; ++i) {
        const int rb = wr + i * g.WR;
        if (rb >= g.RB) continue;
#pragma unroll
        for (int j = 0; j < MC; ++j) {
            const int cb = wc + j * g.WC;
            if (cb >= g.CB) continue;
            const int col = 16 * cb + lr;
            const int kc = col / sc2, jj = col - kc * sc2;
            if (kc >= ngc2) continue;
            const int ncl = g.nfun[g.grp_mem[gc2 * 4 + kc]];
            if (jj >= ncl) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * rb + 4 * r + lk;
                const int kr = row / sr2, ii = row - kr * sr2;
                if (kr >= ngr2) continue;
                const int nr = g.nfun[g.grp_mem[gr2 * 4 + kr]];
                const int t = g.unit_out[u * 16 + kr * 4 + kc];
                if (t >= 0 && ii < nr) C[g.tile_off[t] + (int64_t)jj * nr + ii] = acc[i][j][r];
            }
        }
    }
}

// Thin units (one side a single 16-row block, at most 7 blocks): no LDS panels.
// Wave b < nblk owns output block b and loads its MFMA fragments straight from the tile
// layout into registers, one stage ahead (two register sets, the loop unrolled by two
// so that the sets are static); the last wave keeps the stage records in a ring of
// three LDS slots, two stages ahead.  Each stage ends with one barrier that waits for
// LDS only, so fragment loads stay in flight across it.
__device__ inline void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vector memory may stay outstanding
    __builtin_amdgcn_s_barrier();
}

// Exchange of one double between adjacent lanes (2m <-> 2m + 1).
__device__ inline double swap_adjacent(double x)
{
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, true);           // quad_perm 1,0,3,2
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0xB1, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Record producer of the register-direct kernels (one wave, lane = this lane): keeps the
// stage records of the unit in the ring `ring` of LEAD + 1 slots, LEAD stages ahead of
// the consumers, with one LDS barrier per stage plus one after the prologue: before the
// first barrier it writes records 0 .. LEAD - 1, and between barriers s and s + 1 record
// s + LEAD, into the slot of record s - 1, which consumers no longer read once they may
// read records up to s + LEAD - 1 in that interval.  The four staging sets of its record
// loads follow the ring in LDS (ring_bytes<LEAD>() in all).
struct UnitInfo {
    int64_t s0, p0;
    int nst, npairs, ngr, ngc;
    int nr0, nr1, nr2, nr3, nc0, nc1, nc2, nc3;
};

// Stage record of the split-precision product (its operands are stored k-contiguous,
// in the layout of the transposed tiles): per k pair p (k rows 2p, 2p + 1, always in one
// cluster since every cluster size is even) and member slot, the element offset of
// (member row 0, k row 2p) in the tile (mu, member), -1 where the tile is absent or the
// rows are padding; the lane adds (its member row) x nmu[p].
struct OzTab {
    int64_t kofs[16][8];
    int32_t nmu[16];      // functions of the k pair's cluster (row stride of its tiles)
    int32_t ks;           // k rows of the stage
    int32_t level;        // tree level of the stage's clusters, -1 for an empty stage
    int32_t pad[2];
};

template <int LEAD, typename Rec = KTab>
constexpr size_t ring_bytes()
{
    return (((LEAD + 1) * sizeof(Rec) + 15) & ~(size_t)15) + 4 * (128 * 8 + 3 * 64 * 4);
}

// The fragment that every consumer wave of a unit needs (the unit's single 16-row side),
// which the record wave copies into LDS once instead: per stage four quarters of 64 lanes
// x 16 bytes, lane L holding what consumer lane L would load itself (the rows 2m, 2m + 1
// of one k column, at k step 2q for even and 2q + 1 for odd lanes).  The copy of stage t
// goes into slot t of a ring of as many slots as the record ring.
struct SharedSide {
    const double *X;     // operand of the shared side
    double *dst;         // LDS ring, 512 doubles per slot
    int slot;            // record column of the lane's member
    int ipair;           // offset of the lane's row pair inside a tile column (split-precision
                         // records: the lane's row inside its member)
    int kodd;            // 1 on odd lanes
    bool ok;             // the lane's row exists
};

template <int LEAD, bool SHARE, typename Rec = KTab>
__device__ void record_producer(const GroupArgs &g, const UnitInfo &ui, double *lds, Rec *ring, int lane,
                                const SharedSide &sh)
{
    // OzTab records: g.gl_offd holds the offsets of the transposed tiles (mu, member) and
    // g.gl_nm the cluster size | level << 8 (the caller passes those tables)
    constexpr bool OZ = std::is_same<Rec, OzTab>::value;
    const int64_t s0 = ui.s0, p0 = ui.p0;
    const int nst = ui.nst, npairs = ui.npairs, ngr = ui.ngr, ngc = ui.ngc;
    const int nr0 = ui.nr0, nr1 = ui.nr1, nr2 = ui.nr2, nr3 = ui.nr3;
    const int nc0 = ui.nc0, nc1 = ui.nc1, nc2 = ui.nc2, nc3 = ui.nc3;
    // ---- stage records.  Record t (written LEAD stages ahead, in iteration t - LEAD) needs
    // three dependent loads: the stage bounds, the union entries of its middle clusters
    // and their tile offsets.  Each step is issued kLag iterations before the next one
    // uses it, so a load has kLag stages to arrive; every load is unconditional (clamped
    // indices, results masked), which keeps the loop straight-line.  Lane (p, slot):
    // middle cluster p of the stage, slot 0..3 row members, 4..7 column members.
    constexpr int kLag = 4;
    const int32_t *const stf = g.stage_first + s0;
    const int32_t *const ptab = (lane & 7) < 4 ? g.pair_a + p0 : g.pair_b + p0;
    const int tp = lane >> 3, tslot = lane & 7, tk = tslot & 3;
    const bool tvalid = tslot < 4 ? tk < ngr : tk < ngc;
    int nslot[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) nslot[q] = lane < 32 ? sel4(q, nr0, nr1, nr2, nr3) : sel4(q, nc0, nc1, nc2, nc3);
    // The loads of the loop go straight to LDS (one staging set per phase), so the
    // wave waits for them explicitly: each phase issues exactly four load instructions
    // (offsets 16 B and cluster size of the entries, entries, bounds), after the four
    // shared-fragment copies with SHARE, and at the start of a phase vmcnt <= 4 (kLag - 1)
    // (8 (kLag - 1) with SHARE) means the set loaded kLag phases ago has landed.  A copy
    // for stage t is issued in phase t - LEAD, so it has landed at the start of phase
    // t - LEAD + kLag and is visible to the consumers from barrier t - LEAD + kLag + 1 on,
    // no later than barrier t when LEAD >= kLag + 1.
    struct Staging {
        int64_t off[128];                          // 16 bytes per lane, the first 8 used
        int32_t nm[64], ent[64], bnd[64];
    };
    constexpr int kSlots = LEAD + 1;
    Staging *stg = reinterpret_cast<Staging *>(reinterpret_cast<char *>(lds) + ((kSlots * sizeof(Rec) + 15) & ~(size_t)15));
    auto dma4 = [&](const void *src, void *dst) {
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)dst, 4, 0, 0);
    };
    auto dma16 = [&](const void *src, void *dst) {
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
    };
    auto bound_ptr = [&](int t) { return stf + min(t + (lane & 1), nst - 1); };
    auto fb_of = [&](int32_t raw) { return __builtin_amdgcn_readlane(raw, 0); };
    auto np_of = [&](int32_t raw, int t) {
        if (t >= nst) return 0;
        const int end = t + 1 < nst ? __builtin_amdgcn_readlane(raw, 1) : npairs;
        return end - __builtin_amdgcn_readlane(raw, 0);
    };
    auto entry_ptr = [&](int fb) { return ptab + max(0, min(fb + tp, npairs - 1)); };
    auto issue_offsets = [&](int32_t e_raw, bool ok, Staging *P) {
        const int32_t ec = ok ? e_raw : 0;
        dma16(g.gl_offd + (int64_t)ec * 4 + tk, P->off);
        dma4(g.gl_nm + ec, P->nm);
    };
    // OzTab writer shared by both paths: the stage's cluster sizes nmv (uniform), the
    // lane's k pair kp = lane % 16 and slot group sg = lane / 16 (slots sg and sg + 4);
    // off_of(m, sl) is the tile offset of pair m's cluster for slot sl
    auto write_oz = [&](OzTab *T, uint32_t Bw, uint32_t Lw, int kb, int lev0, auto &&off_of, auto &&nm_of) {
        const int kp = lane & 15, sg = lane >> 4, k = 2 * kp;
        const bool live = ((Lw >> k) & 1u) != 0;
        const uint32_t prefix = Bw & ((2u << k) - 1u);
        const int m = __builtin_popcount(prefix) - 1;
        const int kkm = k - (prefix ? 31 - __builtin_clz(prefix) : 0);
        const int mm = m < 0 ? 0 : m;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int sl = sg + 4 * h;
            const int64_t o = off_of(mm, sl);
            T->kofs[kp][sl] = (live && o >= 0) ? o + kkm : -1;
        }
        const int nmm = nm_of(mm);
        if (sg == 0) T->nmu[kp] = live ? nmm : 0;
        if (lane == 0) {
            T->ks = kb;
            T->level = kb > 0 ? lev0 : -1;
        }
    };
    auto write_tab = [&](Rec *T, int64_t o_raw, int32_t m_raw, bool ok, int t_np) {
        if constexpr (OZ) {
            const int64_t t_off = (ok && tvalid) ? o_raw : -1;
            const int t_nml = (ok && tslot == 0) ? m_raw : 0;
            uint32_t Bm = 0, Lm = 0;
            int kb = 0;
            const int lev0 = __builtin_amdgcn_readlane(t_nml, 0) >> 8;
#pragma unroll
            for (int q = 0; q < kSP; ++q) {
                const int nmq = __builtin_amdgcn_readlane(t_nml, q * 8) & 0xFF;
                if (q < t_np) {
                    Bm |= 1u << kb;
                    Lm |= (nmq >= 32 ? 0xFFFFFFFFu : ((1u << nmq) - 1u)) << kb;
                    kb += nmq;
                }
            }
            write_oz(T, Bm, Lm, kb, lev0, [&](int m, int sl) { return __shfl(t_off, m * 8 + sl); },
                     [&](int m) { return __shfl(t_nml, m * 8) & 0xFF; });
            return;
        } else {
        const int64_t t_off = (ok && tvalid) ? o_raw : -1;
        const int t_nm = (ok && tslot == 0) ? m_raw : 0;
        int nmv[kSP], kbv[kSP];
        int kacc = 0;
#pragma unroll
        for (int q = 0; q < kSP; ++q) {
            nmv[q] = __shfl(t_nm, q * 8);
            kbv[q] = kacc;
            kacc += q < t_np ? nmv[q] : 0;
        }
        const int kk = lane & 31;
        const bool rows = lane < 32;
        int m = -1;
#pragma unroll
        for (int q = 0; q < kSP; ++q)
            if (q < t_np && kk >= kbv[q] && kk < kbv[q] + nmv[q]) m = q;
        const int mm = m < 0 ? 0 : m;
        int nmm = 0, kbm = 0;
#pragma unroll
        for (int q = 0; q < kSP; ++q)
            if (q == mm) { nmm = nmv[q]; kbm = kbv[q]; }
        const int kkm = kk - kbm;
        const bool live = m >= 0 && kkm < nmm;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t o = __shfl(t_off, mm * 8 + (rows ? 0 : 4) + q);
            T->kofs[kk][(rows ? 0 : 4) + q] = (live && o >= 0) ? o + (int64_t)kkm * nslot[q] : -1;
        }
        if (lane == 0) T->ks = kacc;
        }
    };
    // The same record built from the staging set of the loop: the stage's cluster sizes go
    // to scalar registers, whose bit masks of cluster starts (B) and of live rows (L) give
    // each lane kk its cluster (the set bits of B up to kk) and whether row kk exists; the
    // tile offsets are read from the staged copy of the union entries.
    auto write_tab_stg = [&](Rec *T, const Staging *P, int32_t m_raw, bool ok, int t_np) {
        const int t_nm = (ok && tslot == 0) ? m_raw : 0;
        uint64_t Bm = 0, Lm = 0;
        int kb = 0;
#pragma unroll
        for (int q = 0; q < kSP; ++q) {
            const int nmq = __builtin_amdgcn_readlane(t_nm, q * 8) & (OZ ? 0xFF : ~0);
            if (q < t_np) {
                Bm |= 1ull << kb;
                Lm |= ((1ull << nmq) - 1) << kb;
                kb += nmq;
            }
        }
        if constexpr (OZ) {
            const int lev0 = __builtin_amdgcn_readlane(t_nm, 0) >> 8;
            write_oz(T, (uint32_t)Bm, (uint32_t)Lm, kb, lev0, [&](int m, int sl) { return P->off[2 * (m * 8 + sl)]; },
                     [&](int m) { return __shfl(t_nm, m * 8) & 0xFF; });
            return;
        } else {
        const int kk = lane & 31;
        const bool rows = lane < 32;
        const uint32_t Bw = (uint32_t)Bm, Lw = (uint32_t)Lm;
        const bool live = ((Lw >> kk) & 1u) != 0;
        const uint32_t prefix = Bw & ((2u << kk) - 1u);
        const int m = __builtin_popcount(prefix) - 1;
        const int kkm = kk - (prefix ? 31 - __builtin_clz(prefix) : 0);
        const int mm = m < 0 ? 0 : m;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int sl = (rows ? 0 : 4) + q;
            const int64_t o = P->off[2 * (mm * 8 + sl)];
            T->kofs[kk][sl] = (live && o >= 0) ? o + (int64_t)kkm * nslot[q] : -1;
        }
        if (lane == 0) T->ks = kb;
        }
    };
    // copy of the shared fragment of the record just written to ring slot t_slot (the
    // record is re-read from LDS: this wave wrote it, and LDS accesses of a wave are ordered)
    auto share = [&](const Rec *T, int t_slot) {
        if constexpr (SHARE && !OZ) {
            double *d = sh.dst + t_slot * 512;
            const int lk = lane >> 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t o = T->kofs[4 * (2 * q + sh.kodd) + lk][sh.slot];
                dma16((sh.ok && o >= 0) ? sh.X + o + sh.ipair : g_zero_word, d + q * 128);
            }
        } else if constexpr (SHARE && OZ) {
            // the split-precision slices: lane L copies what consumer lane L loads, the k pair
            // 4 (L / 16) + q of its row (sh.ipair = the row inside the member), 16 bytes
            double *d = sh.dst + t_slot * 512;
            const int lk = lane >> 4;
            const uint4 *const X4 = reinterpret_cast<const uint4 *>(sh.X);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int pp = 4 * lk + q;
                const int64_t o = T->kofs[pp][sh.slot];
                const int nmu = T->nmu[pp];
                const void *src = (sh.ok && o >= 0) ? (const void *)(X4 + ((o + (int64_t)sh.ipair * nmu) >> 1))
                                                    : (const void *)g_zero_word;
                dma16(src, d + q * 128);
            }
        }
    };
    // Staging set p serves the iterations s with s % kLag == p: it holds the offsets of
    // stage s + LEAD, the entries of stage s + LEAD + kLag and the bounds of stage
    // s + LEAD + 2 kLag; registers keep np(s + LEAD) (npw), np(s + LEAD + kLag) (npo) and the
    // validity of the lane's entry for both.
    int32_t npw[kLag], npo[kLag];
    bool oko[kLag], oke[kLag];
    {
        // prologue (waits allowed): records 0 .. LEAD - 1, then the loads of the four sets
        int32_t bt[LEAD + 2 * kLag], et[LEAD + kLag];
#pragma unroll
        for (int t = 0; t < LEAD + 2 * kLag; ++t) bt[t] = *bound_ptr(t);
#pragma unroll
        for (int t = 0; t < LEAD + kLag; ++t) et[t] = *entry_ptr(fb_of(bt[t]));
#pragma unroll
        for (int t = 0; t < LEAD; ++t) {
            const bool ok = tp < np_of(bt[t], t);
            const int32_t ec = ok ? et[t] : 0;
            write_tab(&ring[t], g.gl_offd[(int64_t)ec * 4 + tk], g.gl_nm[ec], ok, np_of(bt[t], t));
            share(&ring[t], t);
        }
        __builtin_amdgcn_s_waitcnt(0);             // nothing of the prologue left in flight
#pragma unroll
        for (int q = 0; q < kLag; ++q) {
            npw[q] = np_of(bt[q + LEAD], q + LEAD);
            oko[q] = tp < npw[q];
            issue_offsets(et[q + LEAD], oko[q], &stg[q]);
            const int t2 = q + LEAD + kLag;
            npo[q] = np_of(bt[t2], t2);
            oke[q] = tp < npo[q];
            dma4(entry_ptr(fb_of(bt[t2])), stg[q].ent);
            dma4(bound_ptr(q + LEAD + 2 * kLag), stg[q].bnd);
        }
    }
    lds_barrier();
    int slot = LEAD;                               // ring slot of stage s + LEAD
    auto phase = [&](int s, Staging *P, int32_t &nw, int32_t &no, bool &ko, bool &ke) {
        // this set's loads have landed: vmcnt(12).  With SHARE a phase issues four copies
        // before its four loads while the prologue issued the four sets alone, so phase
        // q < kLag finds 12 + 4q loads issued after its set (vmcnt(12 + 4q)), every later
        // phase 24 (vmcnt(24), which also covers the copies of phase s - kLag)
        if constexpr (SHARE) {
            if (s >= 3) __builtin_amdgcn_s_waitcnt(0x4F78);          // vmcnt(24)
            else if (s == 2) __builtin_amdgcn_s_waitcnt(0x4F74);     // vmcnt(20)
            else if (s == 1) __builtin_amdgcn_s_waitcnt(0x4F70);     // vmcnt(16)
            else __builtin_amdgcn_s_waitcnt(0x0F7C);                 // vmcnt(12)
        } else {
            __builtin_amdgcn_s_waitcnt(0x0F7C);
        }
        const int32_t m = P->nm[lane];
        const int32_t er = P->ent[lane];
        const int32_t br = P->bnd[lane];
        write_tab_stg(&ring[slot], P, m, ko, nw);  // stage s + LEAD
        share(&ring[slot], slot);
        slot = slot == kSlots - 1 ? 0 : slot + 1;
        issue_offsets(er, ke, P);                  // stage s + LEAD + kLag
        nw = no;
        ko = ke;
        const int t3 = s + LEAD + 2 * kLag;
        const int np3 = np_of(br, t3);
        dma4(entry_ptr(fb_of(br)), P->ent);        // stage s + LEAD + 2 kLag
        no = np3;
        ke = tp < np3;
        dma4(bound_ptr(s + LEAD + 3 * kLag), P->bnd); // stage s + LEAD + 3 kLag
        lds_barrier();
    };
    for (int s = 0; s < nst; s += kLag) {
        phase(s, &stg[0], npw[0], npo[0], oko[0], oke[0]);
        if (s + 1 >= nst) break;
        phase(s + 1, &stg[1], npw[1], npo[1], oko[1], oke[1]);
        if (s + 2 >= nst) break;
        phase(s + 2, &stg[2], npw[2], npo[2], oko[2], oke[2]);
        if (s + 3 >= nst) break;
        phase(s + 3, &stg[3], npw[3], npo[3], oko[3], oke[3]);
    }
    __builtin_amdgcn_s_waitcnt(0);                 // let the last loads land before the wave ends
}

template <int WAVES, bool PAIRED>
__global__ __launch_bounds__(WAVES * 64) void k_mgemm_thin(GroupArgs g, const double *__restrict__ A,
                                                          const double *__restrict__ B, double *__restrict__ C)
{
    extern __shared__ double lds[];
    KTab *ring = reinterpret_cast<KTab *>(lds);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t uidx = blockIdx.x;
    if (uidx >= g.count) return;
    const int u = g.unit_order[g.first + uidx];
    const int gr = g.unit_gr[u], gc = g.unit_gc[u];
    const int sr = g.grp_s[gr], sc = g.grp_s[gc];
    const int ngr = g.grp_g[gr], ngc = g.grp_g[gc];
    const int nr0 = g.nfun[g.grp_mem[gr * 4]];
    const int nr1 = ngr > 1 ? g.nfun[g.grp_mem[gr * 4 + 1]] : 0;
    const int nr2 = ngr > 2 ? g.nfun[g.grp_mem[gr * 4 + 2]] : 0;
    const int nr3 = ngr > 3 ? g.nfun[g.grp_mem[gr * 4 + 3]] : 0;
    const int nc0 = g.nfun[g.grp_mem[gc * 4]];
    const int nc1 = ngc > 1 ? g.nfun[g.grp_mem[gc * 4 + 1]] : 0;
    const int nc2 = ngc > 2 ? g.nfun[g.grp_mem[gc * 4 + 2]] : 0;
    const int nc3 = ngc > 3 ? g.nfun[g.grp_mem[gc * 4 + 3]] : 0;
    const int nblk = g.RB * g.CB;
    const int producer = WAVES - 1;
    const int64_t s0 = g.stage_off[u], p0 = g.pair_off[u];
    const int nst = (int)(g.stage_off[u + 1] - s0), npairs = (int)(g.pair_off[u + 1] - p0);
    const int lr = lane & 15, lk = lane >> 4;

    // SHARE (several consumer waves, every cluster size even): the record wave copies the
    // shared 16-row side into LDS five stages ahead and the consumers load only their own
    // block from global memory
    constexpr bool SHARE = WAVES > 2 && PAIRED;
    constexpr int LEAD = SHARE ? 5 : 3;
    constexpr int kSlots = LEAD + 1;
    double *const shr = lds + ring_bytes<LEAD>() / sizeof(double);
    const bool shA = g.RB == 1;                        // the shared side: rows (else columns)
    const bool odd = (lr & 1) != 0;
    if (wave == producer) {
        const UnitInfo ui{s0, p0, nst, npairs, ngr, ngc, nr0, nr1, nr2, nr3, nc0, nc1, nc2, nc3};
        SharedSide sh{};
        if constexpr (SHARE) {
            const int ssz = shA ? sr : sc, sng = shA ? ngr : ngc;
            const int kx = lr / ssz, ix = lr - kx * ssz;
            sh.X = shA ? A : B;
            sh.dst = shr;
            sh.slot = (shA ? 0 : 4) + (kx & 3);
            sh.ipair = odd ? ix - 1 : ix;
            sh.kodd = odd ? 1 : 0;
            sh.ok = kx < sng && ix < (shA ? sel4(kx & 3, nr0, nr1, nr2, nr3) : sel4(kx & 3, nc0, nc1, nc2, nc3));
        }
        record_producer<LEAD, SHARE>(g, ui, lds, ring, lane, sh);
        return;
    }
    if (wave >= nblk) {                                // no block: take part in the barriers only
        lds_barrier();
        for (int s = 0; s < nst; ++s) lds_barrier();
        return;
    }
    // ---- consumer: block (rb, cb)
    const int rb = g.RB == 1 ? 0 : wave, cb = g.RB == 1 ? wave : 0;
    const int ra = 16 * rb + lr, kra = ra / sr, ia = ra - kra * sr;
    const bool oka = kra < ngr && ia < sel4(kra & 3, nr0, nr1, nr2, nr3);
    const int slota = kra & 3;
    const int cbb = 16 * cb + lr, kcb = cbb / sc, jb = cbb - kcb * sc;
    const bool okb = kcb < ngc && jb < sel4(kcb & 3, nc0, nc1, nc2, nc3);
    const int slotb = 4 + (kcb & 3);
    const double *const zero = g_zero_word;
    // A stage's 8 k steps are loaded in quarters of two steps, into a ring of eight
    // register sets (two stages): a quarter is computed while the seven loaded after it
    // are in flight, and its set is then refilled with the same quarter two stages on.
    // PAIRED (every cluster size even): lanes 2m and 2m + 1 load the two rows (2m, 2m + 1)
    // of one k column with one 16-byte load each, the even lane at k step j, the odd lane
    // at k step j + 1; one value is swapped between them when the quarter is computed.
    // Without PAIRED a lane loads its own row at both steps.
    typedef double dbl2 __attribute__((ext_vector_type(2)));
    const int iap = PAIRED && odd ? ia - 1 : ia, jbp = PAIRED && odd ? jb - 1 : jb;
    auto load_q = [&](const KTab *T, int q, dbl2 &va, dbl2 &vb) {
        if constexpr (PAIRED) {
            const int k = 4 * (2 * q + (odd ? 1 : 0)) + lk;
            const int64_t oa = T->kofs[k][slota], ob = T->kofs[k][slotb];
            va = *reinterpret_cast<const dbl2 *>((oka && oa >= 0) ? A + oa + iap : zero);
            vb = *reinterpret_cast<const dbl2 *>((okb && ob >= 0) ? B + ob + jbp : zero);
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = 4 * (2 * q + h) + lk;
                const int64_t oa = T->kofs[k][slota], ob = T->kofs[k][slotb];
                va[h] = *((oka && oa >= 0) ? A + oa + ia : zero);
                vb[h] = *((okb && ob >= 0) ? B + ob + jb : zero);
            }
        }
    };
    // SHARE: the wave's own side only (the block of the wide side it computes)
    const double *const own = shA ? B : A;
    const bool ook = shA ? okb : oka;
    const int oslot = shA ? slotb : slota, oip = shA ? jbp : iap;
    auto load_own = [&](const KTab *T, int q, dbl2 &v) {
        const int64_t o = T->kofs[4 * (2 * q + (odd ? 1 : 0)) + lk][oslot];
        const bool live = ook && o >= 0;
        v = *reinterpret_cast<const dbl2 *>(live ? own + o + oip : zero);
        return live;
    };
    // two accumulators (even and odd k steps), so that consecutive MFMAs of a wave do not
    // wait for each other; they are added once at the end
    dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0}, acc1 = dbl4{0.0, 0.0, 0.0, 0.0};
    // rows at and past the stage's k count have no record (offset -1) and load zeros, so
    // every k step runs unconditionally: straight-line code lets each MFMA wait for its
    // own loads only
    // even lane: (x, partner's x), odd lane: (partner's y, y); each moved value has one
    // use, so the compiler folds the lane move into the select
    auto unpair = [&](const dbl2 &v, double &f0, double &f1) {
        const double px = swap_adjacent(v.x), py = swap_adjacent(v.y);
        f0 = odd ? py : v.x;
        f1 = odd ? v.y : px;
    };
    auto comp_q = [&](const dbl2 &va, const dbl2 &vb) {
        double a0 = va.x, a1 = va.y, b0 = vb.x, b1 = vb.y;
        if constexpr (PAIRED) {
            unpair(va, a0, a1);
            unpair(vb, b0, b1);
        }
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc1, 0, 0, 0);
    };
    // stage s is in sets 4 (s & 1) .. 4 (s & 1) + 3; past the last stage the records have
    // no rows, so the refills are unconditional and load zeros.  Units have an even
    // number of stages, so the loop body (two stages) has no exit in its middle, which
    // would make the compiler wait for loads at the loop head that are still in flight.
    // Loads are issued in ring order (the loop's waits count on set 0 being the oldest).
    if constexpr (SHARE) {
        // A stage in which no function of the wave's own block meets a middle cluster of
        // the stage adds only zeros: its MFMAs are skipped (a wave-uniform branch; the
        // flag is taken from the lanes' record entries when the stage's loads are issued).
        dbl2 qo[8];
        bool act[2];
        lds_barrier();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bool live = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                live |= load_own(&ring[h], q, qo[4 * h + q]);
                __builtin_amdgcn_sched_barrier(0);
            }
            act[h] = __builtin_amdgcn_ballot_w64(live) != 0;
        }
        int slot = 2, shs = 0;                         // ring slots of stages s + 2 and s
        auto half = [&](int h) {
            const int base = 4 * h;
            const dbl2 *sp = reinterpret_cast<const dbl2 *>(shr + shs * 512) + lane;
            dbl2 sv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) sv[q] = sp[q * 64];
            const bool run = act[h];
            bool live = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (run) {
                    const dbl2 va = shA ? sv[q] : qo[base + q], vb = shA ? qo[base + q] : sv[q];
                    comp_q(va, vb);
                }
                live |= load_own(&ring[slot], q, qo[base + q]);
                __builtin_amdgcn_sched_barrier(0);
            }
            act[h] = __builtin_amdgcn_ballot_w64(live) != 0;
            slot = slot == kSlots - 1 ? 0 : slot + 1;
            shs = shs == kSlots - 1 ? 0 : shs + 1;
            lds_barrier();
        };
        for (int s = 0; s < nst; s += 2) {
            half(0);
            half(1);
        }
    } else {
        dbl2 qa[8], qb[8];
        lds_barrier();
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            load_q(&ring[q >> 2], q & 3, qa[q], qb[q]);
            __builtin_amdgcn_sched_barrier(0);
        }
        int slot = 2;                                  // ring slot of stage s + 2
        for (int s = 0; s < nst; s += 2) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                comp_q(qa[q], qb[q]);
                load_q(&ring[slot], q, qa[q], qb[q]);
                __builtin_amdgcn_sched_barrier(0);     // a quarter's swaps must not move ahead
            }
            slot = slot == kSlots - 1 ? 0 : slot + 1;
            lds_barrier();
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                comp_q(qa[4 + q], qb[4 + q]);
                load_q(&ring[slot], q, qa[4 + q], qb[4 + q]);
                __builtin_amdgcn_sched_barrier(0);
            }
            slot = slot == kSlots - 1 ? 0 : slot + 1;
            lds_barrier();
        }
    }
    acc += acc1;
    // store the block where it belongs to S
    const int col = 16 * cb + lr;
    const int kc = col / sc, jj = col - kc * sc;
    if (kc >= ngc) return;
    const int ncl = sel4(kc & 3, nc0, nc1, nc2, nc3);
    if (jj >= ncl) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * rb + 4 * r + lk;
        const int kr = row / sr, ii = row - kr * sr;
        if (kr >= ngr) continue;
        const int nr = sel4(kr & 3, nr0, nr1, nr2, nr3);
        const int t = g.unit_out[u * 16 + kr * 4 + kc];
        if (t >= 0 && ii < nr) C[g.tile_off[t] + (int64_t)jj * nr + ii] = acc[r];
    }
}

// ---------------------------------------------------------------- FP32-accumulate product
// F32ACC: the same unit schedule with FP32 operands and v_mfma_f32_16x16x4f32.  Each
// stage's MFMA sums (FP32, 32 k rows) are added into FP64 accumulators; the result is
// rounded to FP32 once.  Register-direct for every unit class: consumer wave w owns
// block row w (all column blocks, MC >= CB) when the unit has several block rows, else
// column block w; the last wave keeps the records.  QUAD (every cluster size a multiple
// of 4): a 16-byte load gives rows 4m .. 4m+3 of one k column; lane 4m + q loads it at
// k step j + q and a 4 x 4 transpose inside the lane quad gives each lane its own row
// at the four k steps.
__device__ inline float dpp_xor1(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, true));   // 1,0,3,2
}

__device__ inline float dpp_xor2(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, true));   // 2,3,0,1
}

// lane q of a quad holds v = M[q][0..3]; afterwards it holds M[0..3][q] (2 x 2 block
// transposes at lane distance 1, then the exchange of the off-diagonal blocks at distance 2)
__device__ inline void quad_transpose(float (&v)[4], int q)
{
    const bool b0 = (q & 1) != 0, b1 = (q & 2) != 0;
    const float r0 = dpp_xor1(b0 ? v[0] : v[1]);
    const float r1 = dpp_xor1(b0 ? v[2] : v[3]);
    const float t0 = b0 ? r0 : v[0], t1 = b0 ? v[1] : r0;
    const float t2 = b0 ? r1 : v[2], t3 = b0 ? v[3] : r1;
    const float p0 = dpp_xor2(b1 ? t0 : t2);
    const float p1 = dpp_xor2(b1 ? t1 : t3);
    v[0] = b1 ? p0 : t0;
    v[1] = b1 ? p1 : t1;
    v[2] = b1 ? t2 : p0;
    v[3] = b1 ? t3 : p1;
}

// lane 2m + p holds v = {row 2m at k step p, row 2m+1 at k step p, row 2m at step p + 2,
// row 2m+1 at step p + 2}; afterwards it holds row 2m + p at k steps 0, 1, 2, 3
// (each lane sends its partner the row the partner owns, one exchange per load)
__device__ inline void pair_exchange(float (&v)[4], int p)
{
    const float r0 = dpp_xor1(p ? v[0] : v[1]);
    const float r1 = dpp_xor1(p ? v[2] : v[3]);
    const float a0 = p ? r0 : v[0], a1 = p ? v[1] : r0;
    const float a2 = p ? r1 : v[2], a3 = p ? v[3] : r1;
    v[0] = a0; v[1] = a1; v[2] = a2; v[3] = a3;
}

template <int WAVES, int MC, int LW>
__global__ __launch_bounds__(WAVES * 64) void k_mgemm_f32acc(GroupArgs g, const float *__restrict__ A,
                                                            const float *__restrict__ B, float *__restrict__ C)
{
    typedef float flt4 __attribute__((ext_vector_type(4)));
    extern __shared__ double lds[];
    KTab *ring = reinterpret_cast<KTab *>(lds);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t uidx = blockIdx.x;
    if (uidx >= g.count) return;
    const int u = g.unit_order[g.first + uidx];
    const int gr = g.unit_gr[u], gc = g.unit_gc[u];
    const int sr = g.grp_s[gr], sc = g.grp_s[gc];
    const int ngr = g.grp_g[gr], ngc = g.grp_g[gc];
    const int nr0 = g.nfun[g.grp_mem[gr * 4]];
    const int nr1 = ngr > 1 ? g.nfun[g.grp_mem[gr * 4 + 1]] : 0;
    const int nr2 = ngr > 2 ? g.nfun[g.grp_mem[gr * 4 + 2]] : 0;
    const int nr3 = ngr > 3 ? g.nfun[g.grp_mem[gr * 4 + 3]] : 0;
    const int nc0 = g.nfun[g.grp_mem[gc * 4]];
    const int nc1 = ngc > 1 ? g.nfun[g.grp_mem[gc * 4 + 1]] : 0;
    const int nc2 = ngc > 2 ? g.nfun[g.grp_mem[gc * 4 + 2]] : 0;
    const int nc3 = ngc > 3 ? g.nfun[g.grp_mem[gc * 4 + 3]] : 0;
    const bool rows_split = g.RB > 1;
    const int nconsumer = rows_split ? g.RB : g.CB;
    const int producer = WAVES - 1;
    const int64_t s0 = g.stage_off[u], p0 = g.pair_off[u];
    const int nst = (int)(g.stage_off[u + 1] - s0), npairs = (int)(g.pair_off[u + 1] - p0);
    const int lr = lane & 15, lk = lane >> 4;

    if (wave == producer) {
        const UnitInfo ui{s0, p0, nst, npairs, ngr, ngc, nr0, nr1, nr2, nr3, nc0, nc1, nc2, nc3};
        record_producer<2, false>(g, ui, lds, ring, lane, SharedSide{});
        return;
    }
    if (wave >= nconsumer) {
        lds_barrier();
        for (int s = 0; s < nst; ++s) lds_barrier();
        return;
    }
    const int ncb = rows_split ? g.CB : 1;           // column blocks of this wave
    const int rb = rows_split ? wave : 0;
    const int ra = 16 * rb + lr, kra = ra / sr, ia = ra - kra * sr;
    const bool oka = kra < ngr && ia < sel4(kra & 3, nr0, nr1, nr2, nr3);
    const int slota = kra & 3;
    int jb[MC], slotb[MC], cbv[MC];
    bool okb[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) {
        cbv[c] = rows_split ? min(c, g.CB - 1) : wave;
        const int col = 16 * cbv[c] + lr, kcb = col / sc;
        jb[c] = col - kcb * sc;
        okb[c] = kcb < ngc && jb[c] < sel4(kcb & 3, nc0, nc1, nc2, nc3);
        slotb[c] = 4 + (kcb & 3);
    }
    const float *const zero = reinterpret_cast<const float *>(g_zero_word);
    const int q = lr & 3;
    // Fragments of half h (k steps 4h .. 4h + 3) of the stage whose record is T, kept as
    // loaded (LW = 4: rows 4m .. 4m + 3 at k step 4h + q; LW = 2: rows 2m, 2m + 1 at k
    // steps 4h + p and 4h + p + 2, p = l % 2) and put in MFMA order (the quad transpose,
    // or one pair exchange per load) only when the half is computed, so no load is
    // waited for when issued.  LW = 2 needs every cluster size even: a row pair then
    // never straddles two clusters or the end of one, and its 8 bytes are aligned.
    auto load_half = [&](const KTab *T, int h, flt4 &fa, flt4 (&fb)[MC]) {
        if constexpr (LW == 2) {
            const int pp = lr & 1;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int k = 4 * (4 * h + 2 * j + pp) + lk;
                const int64_t oa = T->kofs[k][slota];
                const float2 va = *reinterpret_cast<const float2 *>((oka && oa >= 0) ? A + oa + (ia - pp) : zero);
                fa[2 * j] = va.x;
                fa[2 * j + 1] = va.y;
#pragma unroll
                for (int c = 0; c < MC; ++c) {
                    const int64_t ob = T->kofs[k][slotb[c]];
                    const float2 vb =
                        *reinterpret_cast<const float2 *>((okb[c] && ob >= 0) ? B + ob + (jb[c] - pp) : zero);
                    fb[c][2 * j] = vb.x;
                    fb[c][2 * j + 1] = vb.y;
                }
            }
        } else if constexpr (LW == 4) {
            const int k = 4 * (4 * h + q) + lk;
            const int64_t oa = T->kofs[k][slota];
            fa = *reinterpret_cast<const flt4 *>((oka && oa >= 0) ? A + oa + (ia - q) : zero);
#pragma unroll
            for (int c = 0; c < MC; ++c) {
                const int64_t ob = T->kofs[k][slotb[c]];
                fb[c] = *reinterpret_cast<const flt4 *>((okb[c] && ob >= 0) ? B + ob + (jb[c] - q) : zero);
            }
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = 4 * (4 * h + t) + lk;
                const int64_t oa = T->kofs[k][slota];
                fa[t] = *((oka && oa >= 0) ? A + oa + ia : zero);
#pragma unroll
                for (int c = 0; c < MC; ++c) {
                    const int64_t ob = T->kofs[k][slotb[c]];
                    fb[c][t] = *((okb[c] && ob >= 0) ? B + ob + jb[c] : zero);
                }
            }
        }
    };
    dbl4 acc[MC];
    flt4 a32[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) acc[c] = dbl4{0.0, 0.0, 0.0, 0.0};
    // rows at and past ks load zeros, so all k steps run unconditionally
    auto compute_half = [&](const flt4 &fa_raw, const flt4 (&fb_raw)[MC]) {
        float fa[4] = {fa_raw.x, fa_raw.y, fa_raw.z, fa_raw.w};
        if constexpr (LW == 4) quad_transpose(fa, q);
        if constexpr (LW == 2) pair_exchange(fa, lr & 1);
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            float fb[4] = {fb_raw[c].x, fb_raw[c].y, fb_raw[c].z, fb_raw[c].w};
            if constexpr (LW == 4) quad_transpose(fb, q);
            if constexpr (LW == 2) pair_exchange(fb, lr & 1);
#pragma unroll
            for (int t = 0; t < 4; ++t) a32[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[t], fb[t], a32[c], 0, 0, 0);
        }
    };
    // Stage s: half 1 of s is loaded while half 0 runs, half 0 of s + 1 while half 1 runs;
    // the stage's FP32 sums then go into the FP64 accumulators.
    flt4 fax, fbx[MC], fay, fby[MC];
    lds_barrier();
    if (nst > 0) load_half(&ring[0], 0, fax, fbx);
    int slot = 0;                                      // ring slot of stage s
    for (int s = 0; s < nst; ++s) {
        const int next = slot == 2 ? 0 : slot + 1;
        load_half(&ring[slot], 1, fay, fby);
        __builtin_amdgcn_sched_barrier(0);             // keep the loads ahead of the other half's compute
#pragma unroll
        for (int c = 0; c < MC; ++c) a32[c] = flt4{0.f, 0.f, 0.f, 0.f};
        compute_half(fax, fbx);
        __builtin_amdgcn_sched_barrier(0);
        // unconditional: past the last stage the record has no rows and the loads read zeros
        load_half(&ring[next], 0, fax, fbx);
        __builtin_amdgcn_sched_barrier(0);
        compute_half(fay, fby);
#pragma unroll
        for (int c = 0; c < MC; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[c][r] += (double)a32[c][r];
        slot = next;
        lds_barrier();
    }
    // store the blocks where they belong to S
#pragma unroll
    for (int c = 0; c < MC; ++c) {
        if (c >= ncb) continue;
        const int col = 16 * cbv[c] + lr;
        const int kc = col / sc, jj = col - kc * sc;
        if (kc >= ngc) continue;
        const int ncl = sel4(kc & 3, nc0, nc1, nc2, nc3);
        if (jj >= ncl) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * rb + 4 * lk + r;    // FP32 MFMA: register r of lane l is row 4 (l / 16) + r
            const int kr = row / sr, ii = row - kr * sr;
            if (kr >= ngr) continue;
            const int nr = sel4(kr & 3, nr0, nr1, nr2, nr3);
            const int t = g.unit_out[u * 16 + kr * 4 + kc];
            if (t >= 0 && ii < nr) C[g.tile_off[t] + (int64_t)jj * nr + ii] = (float)acc[c][r];
        }
    }
}

// ---------------------------------------------------------------- split-precision product on matrix cores
// F32SPLIT: operands hi + lo (FP32 pairs, exact in FP64).  Every value x of row i of an
// operand whose column cluster lies on tree level L is scaled by 2^-e, e = e(i, L) the
// exponent of the largest |x| over that row and level (so |x 2^-e| < 1), and cut into
// four 8-bit slices, x 2^-e = sum_s sigma_s 2^-8s up to 2^-33 (round to nearest at each
// step: |sigma_1| <= 256, |sigma_s| <= 128 after; integers of at most 8 significant bits,
// exact in bf16).  That is the error-free splitting of Ozaki, Ogita, Oishi and Rump
// (2012) with one exponent per row and level.  Products of slices are exact in FP32 (at
// most 16 bits), and a stage's sums over its 32 k rows (one level) stay below 2^24, so the
// matrix core's FP32 accumulation is exact; the slice pairs (s, t) with s + t <= 5 of one
// weight 2^-8(s+t) share an accumulator.  The stage sums are combined in FP64 with the
// row and column exponents of their level, which keeps the error near 2^-32 of each
// row-and-level maximum.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kOzSlices = 4;
constexpr int kOzNoExp = -100000;      // a row and level without a nonzero value

// One workgroup per block row r of the operand view V (rows of op(A), or columns of op(B)
// as rows of op(B)^T).  The descriptors of the row's tiles are loaded kSliceBatch at a time,
// one per thread, into LDS; the waves then take the batch's tiles in turn, the lanes of a
// wave the elements of a tile.  Element (i, k) of view tile t = (r, mu) is read from the
// source tile t, column-major (i, k) at k n_r + i (rowsrc = 0), or from the source tile
// trans[t] = (mu, r), column-major (k, i) at i n_mu + k (rowsrc = 1).  Pass 1 reads every
// source tile in storage order and forms e(i, L) in LDS (integer maxima: the result does
// not depend on the order); pass 2 writes the slices of element (i, k) at position
// d = tile_off[trans t] + i n_mu + k (the transposed tile, rows k-contiguous): the k pair
// (d, d + 1), d even, is 16 bytes holding (sigma_s(d), sigma_s(d + 1)) for s = 1..4.
// Every cluster size is even.  Quotients by a cluster size (at most 32) of an index below
// 1024 are taken as (e + 1/2) / n in float, which is at least 1/(2 n) away from an integer.
constexpr int kSliceWaves = 8;
constexpr int kSliceBatch = 64 * kSliceWaves;

__device__ inline int small_quot(int e, float rcp) { return (int)(((float)e + 0.5f) * rcp); }

__global__ __launch_bounds__(64 * kSliceWaves) void k_oz_slice(int32_t nc, int32_t nlev, int rowsrc, int64_t ns,
                                                  const int64_t *__restrict__ blk_rp, const int32_t *__restrict__ tile_col,
                                                  const int64_t *__restrict__ tile_off, const int32_t *__restrict__ trans,
                                                  const int32_t *__restrict__ nfun, const int64_t *__restrict__ cstart,
                                                  const int32_t *__restrict__ clevel, const float *__restrict__ X,
                                                  uint4 *__restrict__ S, int32_t *__restrict__ expo)
{
    extern __shared__ int emax[];            // kMax x nlev
    __shared__ int64_t b_src[kSliceBatch], b_dst[kSliceBatch];
    __shared__ int32_t b_nm[kSliceBatch], b_lev[kSliceBatch];
    const int r = blockIdx.x;
    if (r >= nc) return;
    const int nr = nfun[r];
    if (nr == 0) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const float rnr = 1.0f / (float)nr;
    for (int x = threadIdx.x; x < nr * nlev; x += blockDim.x) emax[x] = kOzNoExp;
    const int64_t t0 = blk_rp[r], t1 = blk_rp[r + 1];
    auto load_batch = [&](int64_t tb) {
        __syncthreads();                      // the previous batch is consumed
        const int64_t t = tb + threadIdx.x;
        if (t < t1) {
            const int mu = tile_col[t];
            const int64_t d0 = tile_off[trans[t]];
            b_nm[threadIdx.x] = nfun[mu];
            b_lev[threadIdx.x] = clevel[mu];
            b_dst[threadIdx.x] = d0;
            b_src[threadIdx.x] = rowsrc ? d0 : tile_off[t];
        }
        __syncthreads();
        return (int)min((int64_t)kSliceBatch, t1 - tb);
    };
    for (int64_t tb = t0; tb < t1; tb += kSliceBatch) {
        const int nb = load_batch(tb);
        for (int b = wave; b < nb; b += kSliceWaves) {
            const int nm = b_nm[b], L = b_lev[b];
            const float rnm = 1.0f / (float)max(nm, 1);
            const float *xs = X + b_src[b];
            for (int e = lane; e < nr * nm; e += 64) {
                const int i = rowsrc ? small_quot(e, rnm) : e - small_quot(e, rnr) * nr;
                const double x = (double)xs[e] + (double)xs[ns + e];
                if (x != 0.0) {
                    const int ex = ilogb(fabs(x)) + 1;
                    int *slot = &emax[i * nlev + L];
                    if (ex > *slot) atomicMax(slot, ex);
                }
            }
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < nr * nlev; x += blockDim.x) expo[(cstart[r] + x / nlev) * nlev + x % nlev] = emax[x];
    for (int64_t tb = t0; tb < t1; tb += kSliceBatch) {
        const int nb = load_batch(tb);
        for (int b = wave; b < nb; b += kSliceWaves) {
            const int nm = b_nm[b], L = b_lev[b];
            const int np = nm >> 1;
            const float rnp = 1.0f / (float)max(np, 1);
            const int64_t d0 = b_dst[b], base = b_src[b];
            for (int e = lane; e < nr * np; e += 64) {
                const int i = small_quot(e, rnp), k = 2 * (e - i * np);
                const int ex = emax[i * nlev + L];
                const int sh = ex == kOzNoExp ? 0 : -ex;
                uint32_t w[kOzSlices];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int64_t q = base + (rowsrc ? (int64_t)i * nm + k + h : (int64_t)(k + h) * nr + i);
                    double y = ldexp((double)X[q] + (double)X[ns + q], sh);
#pragma unroll
                    for (int sl = 0; sl < kOzSlices; ++sl) {
                        y = y * 256.0;
                        const double sg = rint(y);
                        y = y - sg;
                        const uint32_t bits = __float_as_uint((float)sg) >> 16;     // exact in bf16
                        w[sl] = h == 0 ? bits : (w[sl] | bits << 16);
                    }
                }
                S[(d0 + (int64_t)i * nm + k) >> 1] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
    }
}

struct OzArgs {
    const int32_t *exp_a, *exp_b;     // e(i, L) of the two views, n x nlev
    const int64_t *cstart;
    int32_t nlev;
};

// Register-direct split-precision product on the unit schedule.  Workgroup = one unit, or
// one block row of a unit with several block rows and columns; every consumer wave owns
// one 16 x 16 output block (a block row of a unit with one column block, else a column
// block), and the last wave keeps the stage records.  Per stage a lane needs, for its row
// and its 8 k rows (4 k pairs), the four slices of both operands (16 bytes per k pair and
// operand).  SHARE (several consumers): the side all consumers share (the unit's single
// 16-row block row, else its single column block) is copied to LDS by the record wave
// LEAD = 5 stages ahead, and each consumer loads only its own side; otherwise both sides
// are loaded.  The loads of a consumer run two stages ahead in a ring of three register
// sets (the level-homogeneous stage lists have a multiple of three stages per unit).  The
// slice pairs go to v_mfma_f32_16x16x32_bf16; accumulators of one weight hold exact
// integer sums for at most four stages of one level, then are added in FP64 scaled by
// 2^(e_row + e_col - 8 (s + t)).
// register sets of the consumer ring: three without SHARE (both sides loaded), two with it
// (fewer registers, so that two 8-wave workgroups fit a CU); the level-homogeneous stage
// lists have a multiple of six stages per unit

template <int WAVES, bool SHARE>
__global__ __launch_bounds__(WAVES * 64, SHARE ? 4 : 1) void k_mgemm_oz(GroupArgs g, OzArgs z, int rows_split, int sub_rows,
                                                        const uint4 *__restrict__ SA, const uint4 *__restrict__ SB,
                                                        float *__restrict__ C, int64_t ns)
{
    constexpr int LEAD = SHARE ? 5 : 3;
    constexpr int kSlots = LEAD + 1;
    extern __shared__ double lds[];
    OzTab *ring = reinterpret_cast<OzTab *>(lds);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // workgroup -> (unit, fixed block row): the sub_rows block rows of one unit go to
    // workgroups 8 apart, which the round-robin dispatch puts on one XCD (one L2)
    int64_t uidx = blockIdx.x;
    int rbf = 0;
    if (sub_rows > 1) {
        const int64_t grp = uidx / (8 * sub_rows), within = uidx % (8 * sub_rows);
        rbf = (int)(within / 8);
        uidx = grp * 8 + within % 8;
    }
    if (uidx >= g.count) return;
    const int u = g.unit_order[g.first + uidx];
    const int gr = g.unit_gr[u], gc = g.unit_gc[u];
    const int sr = g.grp_s[gr], sc = g.grp_s[gc];
    const int ngr = g.grp_g[gr], ngc = g.grp_g[gc];
    const int nr0 = g.nfun[g.grp_mem[gr * 4]];
    const int nr1 = ngr > 1 ? g.nfun[g.grp_mem[gr * 4 + 1]] : 0;
    const int nr2 = ngr > 2 ? g.nfun[g.grp_mem[gr * 4 + 2]] : 0;
    const int nr3 = ngr > 3 ? g.nfun[g.grp_mem[gr * 4 + 3]] : 0;
    const int nc0 = g.nfun[g.grp_mem[gc * 4]];
    const int nc1 = ngc > 1 ? g.nfun[g.grp_mem[gc * 4 + 1]] : 0;
    const int nc2 = ngc > 2 ? g.nfun[g.grp_mem[gc * 4 + 2]] : 0;
    const int nc3 = ngc > 3 ? g.nfun[g.grp_mem[gc * 4 + 3]] : 0;
    const int nconsumer = rows_split ? g.RB : g.CB;
    const int producer = WAVES - 1;
    const int64_t s0 = g.stage_off[u], p0 = g.pair_off[u];
    const int nst = (int)(g.stage_off[u + 1] - s0), npairs = (int)(g.pair_off[u + 1] - p0);
    const int lr = lane & 15, lk = lane >> 4;
    const int nlev = z.nlev;
    // LDS after the record ring and staging: the shared-side slots (SHARE), then the
    // exponent tables of the workgroup's rows and columns
    double *const shr = lds + ring_bytes<LEAD, OzTab>() / sizeof(double);
    const int erows = rows_split ? 16 * g.RB : 16, ecols = rows_split ? 16 : 16 * g.CB;
    const int erow0 = rows_split ? 0 : 16 * rbf;
    int *const ea = reinterpret_cast<int *>(reinterpret_cast<char *>(shr) + (SHARE ? kSlots * 4096 : 0));
    int *const eb = ea + erows * nlev;
    // the shared side: the rows (block row rb, all consumers own column blocks) unless the
    // consumers own block rows
    const bool shA = !rows_split;
    const int rb_sh = rbf;                            // block row of the shared rows

    if (wave == producer) {
        const UnitInfo ui{s0, p0, nst, npairs, ngr, ngc, nr0, nr1, nr2, nr3, nc0, nc1, nc2, nc3};
        SharedSide sh{};
        if constexpr (SHARE) {
            const int ssz = shA ? sr : sc, sng = shA ? ngr : ngc;
            const int x = shA ? 16 * rb_sh + lr : lr;        // rows of block rb_sh, or of column block 0
            const int kx = x / ssz, ix = x - kx * ssz;
            sh.X = reinterpret_cast<const double *>(shA ? SA : SB);
            sh.dst = shr;
            sh.slot = (shA ? 0 : 4) + (kx & 3);
            sh.ipair = ix;
            sh.ok = kx < sng && ix < (shA ? sel4(kx & 3, nr0, nr1, nr2, nr3) : sel4(kx & 3, nc0, nc1, nc2, nc3));
        }
        record_producer<LEAD, SHARE, OzTab>(g, ui, lds, ring, lane, sh);
        return;
    }
    // consumers fill the exponent tables (visible after the first barrier)
    for (int x = tid; wave < nconsumer && x < (erows + ecols) * nlev; x += 64 * nconsumer) {
        const bool isr = x < erows * nlev;
        const int y = isr ? x : x - erows * nlev;
        const int rc = y / nlev, L = y - rc * nlev;
        const int pos = isr ? erow0 + rc : rc;
        const int ss = isr ? sr : sc, ngg = isr ? ngr : ngc;
        const int km = pos / ss, ii = pos - km * ss;
        int v = kOzNoExp;
        if (km < ngg) {
            const int cl = g.grp_mem[(isr ? gr : gc) * 4 + km];
            if (ii < g.nfun[cl]) v = (isr ? z.exp_a : z.exp_b)[(z.cstart[cl] + ii) * nlev + L];
        }
        (isr ? ea : eb)[y] = v;
    }
    if (wave >= nconsumer) {
        lds_barrier();
        for (int s = 0; s < nst; ++s) lds_barrier();
        return;
    }
    const int rb = rows_split ? wave : rbf, cb = rows_split ? 0 : wave;
    const int ra = 16 * rb + lr, kra = ra / sr, ia = ra - kra * sr;
    const bool oka = kra < ngr && ia < sel4(kra & 3, nr0, nr1, nr2, nr3);
    const int slota = kra & 3;
    const int cbb = 16 * cb + lr, kcb = cbb / sc, jb = cbb - kcb * sc;
    const bool okb = kcb < ngc && jb < sel4(kcb & 3, nc0, nc1, nc2, nc3);
    const int slotb = 4 + (kcb & 3);
    // absent k pairs load 16 zero bytes from a global word (a pointer select, so that every
    // load is a global load issued unconditionally)
    const u32x4 *const zero4 = reinterpret_cast<const u32x4 *>(g_zero_word);
    const u32x4 *const A4 = reinterpret_cast<const u32x4 *>(SA), *const B4 = reinterpret_cast<const u32x4 *>(SB);
    // a lane's four k pairs of one operand: member q holds the k pair 4 lk + q, word s of
    // it the two bf16 values of slice s
    struct Frag {
        u32x4 q0, q1, q2, q3;
    };
    auto load_side = [&](const OzTab *T, int slot, bool ok, int row, const u32x4 *base, Frag &f) {
        auto one = [&](int pp) {
            const int64_t o = T->kofs[pp][slot];
            const int nmu = T->nmu[pp];
            return *((ok && o >= 0) ? base + ((o + (int64_t)row * nmu) >> 1) : zero4);
        };
        const int p0 = 4 * lk;
        f.q0 = one(p0);
        f.q1 = one(p0 + 1);
        f.q2 = one(p0 + 2);
        f.q3 = one(p0 + 3);
    };
    // own side (the block the wave owns) and, without SHARE, the other side too
    auto load_stage = [&](const OzTab *T, Frag &fo, Frag &fx) {
        if (SHARE) {
            if (shA) load_side(T, slotb, okb, jb, B4, fo);
            else load_side(T, slota, oka, ia, A4, fo);
        } else {
            load_side(T, slota, oka, ia, A4, fx);
            load_side(T, slotb, okb, jb, B4, fo);
        }
    };
    flt4 P0 = flt4{0.f, 0.f, 0.f, 0.f}, P1 = P0, P2 = P0, P3 = P0;
    dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
    // this lane's output rows (16 rb + 4 lk + r) and column in the exponent tables
    const int erl = 16 * rb - erow0 + 4 * lk, ecl = 16 * cb + lr;
    auto flush = [&](int L) {
        const int ecv = eb[ecl * nlev + L];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int erv = ea[(erl + r) * nlev + L];
            // exact: four integers below 2^24 at weights 2^-16 .. 2^-40 span 48 bits
            double t = (double)P0[r] * 0x1p-16;
            t += (double)P1[r] * 0x1p-24;
            t += (double)P2[r] * 0x1p-32;
            t += (double)P3[r] * 0x1p-40;
            if (erv != kOzNoExp && ecv != kOzNoExp) acc[r] += ldexp(t, erv + ecv);
        }
        P0 = flt4{0.f, 0.f, 0.f, 0.f};
        P1 = P0;
        P2 = P0;
        P3 = P0;
    };
    auto mfmas = [&](const Frag &fa, const Frag &fb) {
        const bf16x8 a0 = (bf16x8)(u32x4){fa.q0.x, fa.q1.x, fa.q2.x, fa.q3.x};
        const bf16x8 a1 = (bf16x8)(u32x4){fa.q0.y, fa.q1.y, fa.q2.y, fa.q3.y};
        const bf16x8 a2 = (bf16x8)(u32x4){fa.q0.z, fa.q1.z, fa.q2.z, fa.q3.z};
        const bf16x8 a3 = (bf16x8)(u32x4){fa.q0.w, fa.q1.w, fa.q2.w, fa.q3.w};
        const bf16x8 b0 = (bf16x8)(u32x4){fb.q0.x, fb.q1.x, fb.q2.x, fb.q3.x};
        const bf16x8 b1 = (bf16x8)(u32x4){fb.q0.y, fb.q1.y, fb.q2.y, fb.q3.y};
        const bf16x8 b2 = (bf16x8)(u32x4){fb.q0.z, fb.q1.z, fb.q2.z, fb.q3.z};
        const bf16x8 b3 = (bf16x8)(u32x4){fb.q0.w, fb.q1.w, fb.q2.w, fb.q3.w};
        // weight classes w = s + t (0-based slice indices)
        P0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, P0, 0, 0, 0);
        P1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, P1, 0, 0, 0);
        P2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b2, P2, 0, 0, 0);
        P3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b3, P3, 0, 0, 0);
        P1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, P1, 0, 0, 0);
        P2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, P2, 0, 0, 0);
        P3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b2, P3, 0, 0, 0);
        P2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b0, P2, 0, 0, 0);
        P3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b1, P3, 0, 0, 0);
        P3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, b0, P3, 0, 0, 0);
    };
    int cur = -1, cnt = 0;
    // stage in ring slot `slot`: the own side in fo (and fx without SHARE), the shared side
    // from its LDS slot (the same index: both rings have kSlots slots)
    auto stage = [&](int slot, const Frag &fo, const Frag &fx) {
        const OzTab *T = &ring[slot];
        const int lv = T->level;                                 // wave-uniform
        if (lv < 0) return;                                      // empty stage
        if (cur >= 0 && (lv != cur || cnt == 4)) {
            flush(cur);
            cnt = 0;
        }
        cur = lv;
        if (SHARE) {
            // the shared side straight from LDS into operand order: word s of k pair q of this
            // lane sits at ((q * 64 + lane) * 4 + s) words
            const uint32_t *sp = reinterpret_cast<const uint32_t *>(shr + slot * 512) + 4 * lane;
            Frag fs;
            fs.q0 = (u32x4){sp[0], sp[1], sp[2], sp[3]};
            fs.q1 = (u32x4){sp[256], sp[257], sp[258], sp[259]};
            fs.q2 = (u32x4){sp[512], sp[513], sp[514], sp[515]};
            fs.q3 = (u32x4){sp[768], sp[769], sp[770], sp[771]};
            if (shA) mfmas(fs, fo);
            else mfmas(fo, fs);
        } else {
            mfmas(fx, fo);
        }
        ++cnt;
    };
    auto nxt = [&](int x) { return x == kSlots - 1 ? 0 : x + 1; };
    lds_barrier();
    // records 0 .. LEAD - 1 are in the ring when the loop starts; past the last stage the
    // records have no rows and the loads read zeros
    int sl0 = 0;                                                 // ring slot of stage s
    if constexpr (SHARE) {
        // two sets: stage s + 1 is loaded while stage s runs
        Frag o0, o1, x0;
        load_stage(&ring[0], o0, x0);
        for (int s = 0; s < nst; s += 2) {
            const int sl1 = nxt(sl0);
            load_stage(&ring[sl1], o1, x0);
            __builtin_amdgcn_sched_barrier(0);
            stage(sl0, o0, x0);
            lds_barrier();
            const int sl2 = nxt(sl1);
            load_stage(&ring[sl2], o0, x0);
            __builtin_amdgcn_sched_barrier(0);
            stage(sl1, o1, x0);
            lds_barrier();
            sl0 = sl2;
        }
    } else {
        // three sets: stage s + 2 is loaded while stage s runs
        Frag o0, o1, o2, x0, x1, x2;
        load_stage(&ring[0], o0, x0);
        load_stage(&ring[1], o1, x1);
        for (int s = 0; s < nst; s += 3) {
            const int sl1 = nxt(sl0), sl2 = nxt(sl1);
            load_stage(&ring[sl2], o2, x2);
            __builtin_amdgcn_sched_barrier(0);
            stage(sl0, o0, x0);
            lds_barrier();
            const int sl3 = nxt(sl2);
            load_stage(&ring[sl3], o0, x0);
            __builtin_amdgcn_sched_barrier(0);
            stage(sl1, o1, x1);
            lds_barrier();
            const int sl4 = nxt(sl3);
            load_stage(&ring[sl4], o1, x1);
            __builtin_amdgcn_sched_barrier(0);
            stage(sl2, o2, x2);
            lds_barrier();
            sl0 = sl3;
        }
    }
    if (cur >= 0 && cnt > 0) flush(cur);
    // store the block where it belongs to S (hi and lo of each FP64 sum)
    const int col = 16 * cb + lr;
    const int kc = col / sc, jj = col - kc * sc;
    if (kc >= ngc) return;
    const int ncl = sel4(kc & 3, nc0, nc1, nc2, nc3);
    if (jj >= ncl) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * rb + 4 * lk + r;
        const int kr = row / sr, ii = row - kr * sr;
        if (kr >= ngr) continue;
        const int nr = sel4(kr & 3, nr0, nr1, nr2, nr3);
        const int t = g.unit_out[u * 16 + kr * 4 + kc];
        if (t >= 0 && ii < nr) {
            const int64_t e = g.tile_off[t] + (int64_t)jj * nr + ii;
            const float hi = (float)acc[r];
            C[e] = hi;
            C[ns + e] = (float)(acc[r] - (double)hi);
        }
    }
}

// Y = A X for an S-matrix A (tile layout) and a dense block X of r columns (column-major,
// leading dimension n, basis order), the product behind the paper's error estimator
// e_F (Section 5.1).  The tiles of block row nu are stored one after the other, so the
// row is a dense column-major panel of n_nu <= 32 rows; runs of tiles whose column
// clusters follow on in the basis cover contiguous basis columns, and the host cuts
// them into pieces of whole 16-column chunks.  One workgroup of kSpmmWaves waves per
// block row, the waves taking the pieces in turn; their partial sums are added in LDS
// in a fixed order.  Each piece is a small dense product (n_nu x w)(w x r):
//  - n_nu > 8: v_mfma_f64_16x16x4f64.  Per 16 columns, lane l loads A at row
//    16 rb + l%16 and X at column cc0 + 16 cb + l%16, both at piece columns
//    l/16 + 4s (s = 0..3), so every value of A and X is loaded once.
//  - n_nu <= 8 (where a 16-row MFMA would be mostly padding): plain FMAs.  Lane l takes
//    piece column l%16 of each chunk and X columns l/16 + 4m, and keeps n_nu x 4 CB sums,
//    folded over the 16 column lanes at the end; with at most four columns of X, lane l
//    takes piece column l of each 64-column step and all columns of X, so each entry of
//    A is loaded once.
// Four waves per workgroup, so that three workgroups fit on a CU.
constexpr int kSpmmWaves = 4;

// load at a uniform base plus a 32-bit byte offset (one VGPR per address)
__device__ __forceinline__ double ld_off(const double *base, uint32_t byte_off)
{
    return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(base) + byte_off);
}

template <int NRB, int CB>
__device__ __forceinline__ void spmm_mfma(int64_t q, int64_t p1, int nr, int64_t n, int r, int cc0,
                                          const int64_t *__restrict__ pc_off, const int64_t *__restrict__ pc_g,
                                          const int32_t *__restrict__ pc_w, const double *__restrict__ A,
                                          const double *__restrict__ X, double (*red)[16 * CB + 1])
{
    const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    dbl4 d[NRB][CB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) d[rb][cb] = dbl4{0.0, 0.0, 0.0, 0.0};
    for (; q < p1; q += kSpmmWaves) {
        const int w = pc_w[q];
        const double *aq = A + pc_off[q];
        const int64_t g = pc_g[q];
        const double *xr[CB];   // uniform: column cc0 + 16 cb of X at the piece's first basis column
        bool xon[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            xon[cb] = cc0 + 16 * cb + lr < r;
            xr[cb] = X + (int64_t)(cc0 + 16 * cb) * n + g;
        }
        const uint32_t xl = 8u * (uint32_t)(lr * n);
        // U chunks of 16 columns per step, all of their loads in flight together
        constexpr int U = NRB == 1 ? 4 : 2;
        for (int j0 = 0; j0 < w; j0 += 16 * U) {
            double av[U][NRB][4], xv[U][CB][4];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int sl = 0; sl < 4; ++sl) {
                    const int jc = j0 + 16 * u + lk + 4 * sl;
                    const bool jon = jc < w;
#pragma unroll
                    for (int rb = 0; rb < NRB; ++rb) {
                        const int row = 16 * rb + lr;
                        av[u][rb][sl] = (jon && row < nr) ? ld_off(aq, 8u * (uint32_t)(jc * nr + row)) : 0.0;
                    }
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        xv[u][cb][sl] = (jon && xon[cb]) ? ld_off(xr[cb], xl + 8u * (uint32_t)jc) : 0.0;
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int sl = 0; sl < 4; ++sl)
#pragma unroll
                    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb)
                            d[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][rb][sl], xv[u][cb][sl], d[rb][cb],
                                                                             0, 0, 0);
        }
    }
    // accumulator register k of lane l: row 16 rb + 4 k + l/16, column 16 cb + l%16
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int k = 0; k < 4; ++k) red[16 * rb + 4 * k + lk][16 * cb + lr] = d[rb][cb][k];
}

// CL groups of 64 / CL column lanes: with CL = 4 each group takes 4 CB columns of X (16 CB
// per pass, the four groups reading the same entries of A); with CL = 1 (at most four
// columns of X) every lane reads its own column of A, so each entry is loaded once.
template <int MAXR, int CB, int CL = 4>
__device__ __forceinline__ void spmm_thin(int64_t q, int64_t p1, int nr, int64_t n, int r, int cc0,
                                          const int64_t *__restrict__ pc_off, const int64_t *__restrict__ pc_g,
                                          const int32_t *__restrict__ pc_w, const double *__restrict__ A,
                                          const double *__restrict__ X, double (*red)[16 * CB + 1])
{
    constexpr int M = 4 * CB, JL = 64 / CL;
    const int lane = threadIdx.x & 63, jl = lane % JL, cl = lane / JL;
    double acc[MAXR][M];
#pragma unroll
    for (int i = 0; i < MAXR; ++i)
#pragma unroll
        for (int m = 0; m < M; ++m) acc[i][m] = 0.0;
    for (; q < p1; q += kSpmmWaves) {
        const int w = pc_w[q];
        const double *aq = A + pc_off[q];
        const int64_t g = pc_g[q];
        const double *xr[M];    // uniform: column cc0 + 4 m of X at the piece's first basis column
        bool xon[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            xon[m] = cc0 + cl + CL * m < r;
            xr[m] = X + (int64_t)(cc0 + CL * m) * n + g;
        }
        const uint32_t xl = 8u * (uint32_t)(cl * n);
        constexpr int U = MAXR <= 4 ? 4 : 2;
        for (int j0 = 0; j0 < w; j0 += JL * U) {
            double a[U][MAXR], x[U][M];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int jc = j0 + JL * u + jl;
                const bool jon = jc < w;
#pragma unroll
                for (int i = 0; i < MAXR; ++i)
                    a[u][i] = (jon && i < nr) ? ld_off(aq, 8u * (uint32_t)(jc * nr + i)) : 0.0;
#pragma unroll
                for (int m = 0; m < M; ++m) x[u][m] = (jon && xon[m]) ? ld_off(xr[m], xl + 8u * (uint32_t)jc) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int i = 0; i < MAXR; ++i)
#pragma unroll
                    for (int m = 0; m < M; ++m) acc[i][m] = fma(a[u][i], x[u][m], acc[i][m]);
        }
    }
    // fold the column lanes of each X-column group (a fixed butterfly)
#pragma unroll
    for (int i = 0; i < MAXR; ++i)
#pragma unroll
        for (int m = 0; m < M; ++m) {
            double v = acc[i][m];
#pragma unroll
            for (int o = 1; o < JL; o <<= 1) v += __shfl_xor(v, o, 64);
            if (jl == 0 && i < nr) red[i][cl + CL * m] = v;
        }
}

template <int CB>
__global__ __launch_bounds__(64 * kSpmmWaves, 3) void k_spmm(int32_t nc, int64_t n, int32_t r,
                                                          const int64_t *__restrict__ pc_rp,
                                                          const int64_t *__restrict__ pc_off,
                                                          const int64_t *__restrict__ pc_g,
                                                          const int32_t *__restrict__ pc_w,
                                                          const int32_t *__restrict__ nfun,
                                                          const int64_t *__restrict__ cstart,
                                                          const double *__restrict__ A, const double *__restrict__ X,
                                                          double *__restrict__ Y)
{
    __shared__ double red[kSpmmWaves][32][16 * CB + 1];
    const int c = blockIdx.x;
    if (c >= nc) return;
    const int nr = nfun[c];
    if (nr == 0) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t q0 = pc_rp[c] + wave, p1 = pc_rp[c + 1];
    for (int cc0 = 0; cc0 < r; cc0 += 16 * CB) {
        if (nr <= 4 && r <= 4) spmm_thin<4, 1, 1>(q0, p1, nr, n, r, cc0, pc_off, pc_g, pc_w, A, X, red[wave]);
        else if (nr <= 8 && r <= 4) spmm_thin<8, 1, 1>(q0, p1, nr, n, r, cc0, pc_off, pc_g, pc_w, A, X, red[wave]);
        else if (nr <= 4) spmm_thin<4, CB>(q0, p1, nr, n, r, cc0, pc_off, pc_g, pc_w, A, X, red[wave]);
        else if (nr <= 8) spmm_thin<8, CB>(q0, p1, nr, n, r, cc0, pc_off, pc_g, pc_w, A, X, red[wave]);
        else if (nr <= 16) spmm_mfma<1, CB>(q0, p1, nr, n, r, cc0, pc_off, pc_g, pc_w, A, X, red[wave]);
        else spmm_mfma<2, CB>(q0, p1, nr, n, r, cc0, pc_off, pc_g, pc_w, A, X, red[wave]);
        __syncthreads();
        const int rc = min(16 * CB, r - cc0);
        for (int o = threadIdx.x; o < nr * rc; o += blockDim.x) {
            const int ii = o % nr, cc = o / nr;
            double v = red[0][ii][cc];
#pragma unroll
            for (int w = 1; w < kSpmmWaves; ++w) v += red[w][ii][cc];
            Y[(int64_t)(cc0 + cc) * n + cstart[c] + ii] = v;
        }
        __syncthreads();
    }
}

// Raw buffer access (gfx9 resource word 3; byte offsets at or beyond the extent read 0 and
// are not written).
constexpr int kBufWord3 = 0x00020000;
constexpr int kBufOutside = 0x7fffffff;
template <typename T> struct BufWord;
template <> struct BufWord<double> { using type = unsigned long long; };
template <> struct BufWord<float> { using type = unsigned; };
template <typename T>
__device__ inline typename BufWord<T>::type buf_load(__amdgpu_buffer_rsrc_t r, int off)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(unsigned long long, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else
        return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}
template <typename T>
__device__ inline void buf_store(__amdgpu_buffer_rsrc_t r, int off, typename BufWord<T>::type v)
{
    using u32x2 = __attribute__((ext_vector_type(2))) unsigned;
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, 0);
}

// out = the tiles of in, each transposed into the place of its mirror tile.  One
// wavefront per run of kTrRun consecutive tiles: lane k loads the descriptors of tile
// t0 + k (one coalesced load per table) into LDS.  The run's input is contiguous in
// storage; it is staged through LDS kTrStage entries (whole tiles) at a time, read in
// order (coalesced, through a buffer resource of the run's extent, so lanes past its end
// read 0 without a branch), and every mirror tile is then written in order (coalesced),
// tile by tile, each lane gathering its entry from LDS.  Staged entry q sits at q + q / 32, so the gathers (stride n_rows)
// spread over the banks.
constexpr int kTrRun = 64;
constexpr int kTrStage = 1024;
constexpr int kTrUnroll = 16;
static_assert(kTrStage >= kMax * kMax, "a staged group holds at least one whole tile");
// Four independent wavefronts per workgroup (a 64-thread workgroup would be held to four
// per SIMD by the workgroup slots); each has its own LDS and orders its LDS accesses by
// wavefront-scope fences only.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(int64_t n_tiles, const int64_t *__restrict__ tile_off,
                                                  const int32_t *__restrict__ tile_row,
                                                  const int32_t *__restrict__ tile_col,
                                                  const int32_t *__restrict__ trans, const int32_t *__restrict__ nfun,
                                                  const T *__restrict__ in, T *__restrict__ out)
{
    using Word = typename BufWord<T>::type;
    __shared__ int32_t sh_off[4][kTrRun + 1]; // tile starts relative to the run's first entry
    __shared__ int64_t sh_dst[4][kTrRun];     // output offset of the mirror tile
    __shared__ int32_t sh_nr[4][kTrRun], sh_nc[4][kTrRun];
    __shared__ float sh_rnc[4][kTrRun];
    __shared__ Word sh_stage[4][kTrStage + kTrStage / 32];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int32_t *s_off = sh_off[w], *s_nr = sh_nr[w], *s_nc = sh_nc[w];
    int64_t *s_dst = sh_dst[w];
    float *s_rnc = sh_rnc[w];
    Word *stage = sh_stage[w];
    for (int64_t t0 = ((int64_t)blockIdx.x * 4 + w) * kTrRun; t0 < n_tiles; t0 += (int64_t)gridDim.x * 4 * kTrRun) {
        const int m = (int)min((int64_t)kTrRun, n_tiles - t0);
        const int64_t base = tile_off[t0];
        if (lane < m) {
            const int64_t t = t0 + lane;
            const int nc = nfun[tile_col[t]];
            s_off[lane] = (int32_t)(tile_off[t] - base);
            s_nr[lane] = nfun[tile_row[t]];
            s_nc[lane] = nc;
            s_rnc[lane] = 1.0f / (float)max(nc, 1);
            s_dst[lane] = tile_off[trans[t]];
        }
        if (lane == 0) s_off[m] = (int32_t)(tile_off[t0 + m] - base);
        wave_sync();
        const int E = s_off[m];                  // entries of the run (at most kTrRun * 1024)
        const __amdgpu_buffer_rsrc_t rin =
            __builtin_amdgcn_make_buffer_rsrc((void *)(in + base), 0, E * (int)sizeof(T), kBufWord3);
        // groups of whole tiles [ka, kb) with at most kTrStage entries (a tile has at most
        // kMax * kMax); the next group's loads are in flight while a group is written out
        auto group_end = [&](int ka) {
            int lo = ka + 1, hi = m;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] - s_off[ka] <= kTrStage) lo = mid;
                else hi = mid - 1;
            }
            return lo;
        };
        Word v[kTrUnroll];
        auto load_group = [&](int ka, int kb) {
            const int g0 = s_off[ka], G = s_off[kb] - g0;
#pragma unroll
            for (int u = 0; u < kTrUnroll; ++u) {
                const int q = 64 * u + lane;
                v[u] = buf_load<T>(rin, q < G ? (g0 + q) * (int)sizeof(T) : kBufOutside);
            }
        };
        int ka = 0, kb = group_end(0);
        load_group(ka, kb);
        while (ka < m) {
            const int g0 = s_off[ka], G = s_off[kb] - g0;
#pragma unroll
            for (int u = 0; u < kTrUnroll; ++u) {
                const int q = 64 * u + lane;
                if (q < G) stage[q + (q >> 5)] = v[u];
            }
            wave_sync();
            const int ka2 = kb, kb2 = kb < m ? group_end(kb) : kb;
            if (ka2 < m) load_group(ka2, kb2);
            for (int k = ka; k < kb; ++k) {
                const int nr = s_nr[k], nc = s_nc[k], off = s_off[k] - g0;
                const float rnc = s_rnc[k];
                T *dst = out + s_dst[k];
                for (int l = lane; l < nr * nc; l += 64) {
                    // output entry (i, j) of the mirror tile at l = i * nc + j; row i from l / nc:
                    // (l + 1/2) / nc is at least 1/(2 nc) away from an integer, far more than the
                    // float error for l < 1024
                    const int i = (int)(((float)l + 0.5f) * rnc), j = l - i * nc;
                    const int p = off + j * nr + i;             // staged input entry (i, j)
                    dst[l] = __builtin_bit_cast(T, stage[p + (p >> 5)]);
                }
            }
            wave_sync();
            ka = ka2;
            kb = kb2;
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

// The split-precision product runs on the matrix cores when the pattern was planned with
// cluster levels, every cluster size is even (k pairs never straddle two clusters) and
// every unit class has at most 7 blocks of 16 rows on a side; otherwise on the per-tile
// compensated kernel.
bool oz_ok(spm_pattern p)
{
    if (p->clevel.empty() || !p->all_even || p->nlev > 64) return false;
    for (const auto &L : p->launches)
        if (L.rb > 7 || L.cb > 7) return false;
    return true;
}

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

int ilog2_ceil(int x)
{
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

// Launches one grouped-product kernel with `lds` bytes of dynamic LDS (the attribute
// that allows more than 64 KiB is set on first use of each instantiation).
int launch_grp(const void *k, dim3 grid, int threads, size_t lds, hipStream_t s, GroupArgs &g, const double *A,
               const double *B, double *C)
{
    static std::mutex mu;
    static std::set<std::pair<int, const void *>> ready;   // (device, kernel)
    int dev = 0;
    SPM_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lock(mu);
        if (!ready.count({dev, k})) {
            SPM_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
            ready.insert({dev, k});
        }
    }
    void *args[] = {&g, &A, &B, &C};
    SPM_HIP(hipLaunchKernel(k, grid, dim3(threads), args, lds, s));
    return SPM_OK;
}

// C = P_S(A B^T) with the grouped kernel.
int launch_gemm_abt(spm_pattern p, const double *A, const double *B, double *C, hipStream_t s)
{
    GroupArgs g;
    g.grp_mem = p->d_grp_mem.ptr; g.grp_s = p->d_grp_s.ptr; g.grp_g = p->d_grp_g.ptr;
    g.unit_gr = p->d_unit_gr.ptr; g.unit_gc = p->d_unit_gc.ptr; g.unit_out = p->d_unit_out.ptr;
    g.unit_order = p->d_unit_order.ptr; g.pair_off = p->d_pair_off.ptr; g.pair_a = p->d_pair_a.ptr;
    g.pair_b = p->d_pair_b.ptr; g.gl_nm = p->d_gl_nm.ptr; g.gl_offd = p->d_gl_offd.ptr;
    g.stage_off = p->d_stage_off.ptr; g.stage_first = p->d_stage_first.ptr; g.tile_off = p->d_tile_off.ptr;
    g.nfun = p->d_nfun.ptr;
    const bool wide = p->all_even;   // two doubles per lane never straddle a cluster's functions
    for (const auto &L : p->launches) {
        g.first = L.first;
        g.count = L.count;
        g.RB = L.rb;
        g.CB = L.cb;
        g.lxa = std::max(4, ilog2_ceil(16 * L.rb));
        g.lxb = std::max(4, ilog2_ceil(16 * L.cb));
        const size_t pd = (size_t)kKS * ((1 << g.lxa) + (1 << g.lxb));
        const size_t lds = 2 * pd * sizeof(double) + 2 * sizeof(KTab);
        if (lds > 160 * 1024) return fail(SPM_EUNSUPPORTED, "grouped product: LDS budget exceeded");
        const dim3 grid((unsigned)L.count);
        if ((L.rb == 1 || L.cb == 1) && L.rb * L.cb <= 7) {
            // one side a single block: register-direct kernel, one wave per block plus the
            // record wave
            g.WR = g.WC = g.nsplit = 1;
            // record ring and staging, then with the shared-side copies (8 waves, even
            // sizes) their ring of six 4 KB slots
            const bool share = wide && L.rb * L.cb > 1;
            const size_t ring = share ? ring_bytes<5>() + 6 * 4096 : ring_bytes<3>();
            int st;
            const void *k;
            if (L.rb * L.cb == 1) k = wide ? (const void *)k_mgemm_thin<2, true> : (const void *)k_mgemm_thin<2, false>;
            else k = wide ? (const void *)k_mgemm_thin<8, true> : (const void *)k_mgemm_thin<8, false>;
            st = launch_grp(k, grid, L.rb * L.cb == 1 ? 128 : 512, ring, s, g, A, B, C);
            if (st) return st;
            continue;
        }
        if (L.rb * L.cb == 1) {
            // one 16 x 16 block: one MFMA wave plus a wave that keeps the stage records
            g.WR = g.WC = g.nsplit = 1;
            const void *k = wide ? (const void *)k_mgemm_grp<2, 16, 1, 1> : (const void *)k_mgemm_grp<2, 4, 1, 1>;
            int st = launch_grp(k, grid, 128, lds, s, g, A, B, C);
            if (st) return st;
            continue;
        }
        // wave patch MR x MC: fewest MFMAs per SIMD and k step (8 waves on 4 SIMDs), then
        // fewest fragment reads
        static const int shapes[10][2] = {{1, 1}, {1, 2}, {2, 1}, {2, 2}, {1, 4}, {4, 1}, {2, 4}, {4, 2}, {1, 7}, {7, 1}};
        int best = -1;
        auto simd_cost = [&](int q) {
            const int mr = shapes[q][0], mc = shapes[q][1];
            const int wr = (L.rb + mr - 1) / mr, wc = (L.cb + mc - 1) / mc;
            return ((wr * wc + 3) / 4) * mr * mc;
        };
        for (int q = 0; q < 10; ++q) {
            const int mr = shapes[q][0], mc = shapes[q][1];
            const int wr = (L.rb + mr - 1) / mr, wc = (L.cb + mc - 1) / mc;
            if (wr * wc > 8) continue;
            if (best < 0) { best = q; continue; }
            const int bm = simd_cost(best), qm = simd_cost(q);
            const int bs = shapes[best][0] + shapes[best][1], qs = mr + mc;
            if (qm < bm || (qm == bm && qs < bs)) best = q;
        }
        if (best < 0) return fail(SPM_EUNSUPPORTED, "grouped product: unit too large");
        const int mr = shapes[best][0], mc = shapes[best][1];
        g.WR = (L.rb + mr - 1) / mr;
        g.WC = (L.cb + mc - 1) / mc;
        g.nsplit = 8 / (g.WR * g.WC);
        if ((size_t)(g.nsplit - 1) * g.WR * g.WC * mr * mc * 256 > 2 * pd)
            return fail(SPM_EUNSUPPORTED, "grouped product: k-slice reduction exceeds LDS");
        const void *k = nullptr;
#define SPM_GRP_PICK(MR_, MC_)                                                                            \
        if (mr == MR_ && mc == MC_)                                                                       \
            k = wide ? (const void *)k_mgemm_grp<8, 16, MR_, MC_> : (const void *)k_mgemm_grp<8, 4, MR_, MC_>;
        SPM_GRP_PICK(1, 1) SPM_GRP_PICK(1, 2) SPM_GRP_PICK(2, 1) SPM_GRP_PICK(2, 2)
        SPM_GRP_PICK(1, 4) SPM_GRP_PICK(4, 1) SPM_GRP_PICK(2, 4) SPM_GRP_PICK(4, 2)
        SPM_GRP_PICK(1, 7) SPM_GRP_PICK(7, 1)
#undef SPM_GRP_PICK
        int st = launch_grp(k, grid, 512, lds, s, g, A, B, C);
        if (st) return st;
    }
    SPM_HIP(hipGetLastError());
    return SPM_OK;
}

template <typename T>
int launch_transpose(spm_pattern p, const T *in, T *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_transpose<T>, dim3(grid1d(p->n_tiles, 4 * kTrRun, 16384)), dim3(256), 0, s, p->n_tiles,
                       p->d_tile_off.ptr, p->d_tile_row.ptr, p->d_tile_col.ptr, p->d_trans.ptr, p->d_nfun.ptr, in, out);
    SPM_HIP(hipGetLastError());
    return SPM_OK;
}

size_t ws_align(size_t x) { return (x + 255) & ~(size_t)255; }

// F32ACC runs on the register-direct FP32 kernel when every unit class has at most 7 x 7
// blocks, else on the per-tile kernel.
bool f32acc_grouped(spm_pattern p)
{
    for (const auto &L : p->launches)
        if (L.rb > 7 || L.cb > 7) return false;
    return true;
}

// Workspace of one product C = P_S(op(A) op(B)): the grouped kernels compute
// P_S(A' B'^T) with A' = op(A) and B'^T = op(B), so A is transposed into the
// workspace when op(A) = A^T and B when op(B) = B.
size_t oz_ws_bytes(spm_pattern p)
{
    return 2 * ws_align((size_t)p->n_stored * 8) + 2 * ws_align((size_t)p->n * p->nlev * sizeof(int32_t));
}

size_t gemm_ws_bytes(spm_pattern p, int prec, int ta, int tb)
{
    if (p->n_tiles == 0) return 0;
    if (prec == SPM_F32SPLIT && oz_ok(p)) return oz_ws_bytes(p);
    size_t el;
    if (prec == SPM_F64) el = sizeof(double);
    else if (prec == SPM_F32ACC && f32acc_grouped(p)) el = sizeof(float);
    else return 0;                                   // per-tile kernel: reads both operands in place
    const size_t vb = ws_align((size_t)p->n_stored * el);
    return (ta ? vb : 0) + (tb ? 0 : vb);
}

// C = P_S(op(A) op(B)) with the grouped FP64 kernels; the transposed copies go to ws.
int gemm_grouped_ws(spm_pattern p, const double *A, int ta, const double *B, int tb, double *C, char *ws,
                    hipStream_t s)
{
    const size_t vb = ws_align((size_t)p->n_stored * sizeof(double));
    double *ta_buf = ta ? reinterpret_cast<double *>(ws) : nullptr;
    double *tb_buf = tb ? nullptr : reinterpret_cast<double *>(ws + (ta ? vb : 0));
    int st = SPM_OK;
    if (ta) st = launch_transpose(p, A, ta_buf, s);
    if (!st && !tb) st = launch_transpose(p, B, tb_buf, s);
    if (!st) st = launch_gemm_abt(p, ta ? ta_buf : A, tb ? B : tb_buf, C, s);
    return st;
}

// F32ACC: C = P_S(op(A) op(B)) with the register-direct FP32 kernel (unit classes of at
// most 7 x 7 blocks).
int gemm_f32acc_ws(spm_pattern p, const float *A, int ta, const float *B, int tb, float *C, char *ws, hipStream_t s)
{
    const size_t vb = ws_align((size_t)p->n_stored * sizeof(float));
    float *ta_buf = ta ? reinterpret_cast<float *>(ws) : nullptr;
    float *tb_buf = tb ? nullptr : reinterpret_cast<float *>(ws + (ta ? vb : 0));
    int st = SPM_OK;
    if (ta) st = launch_transpose(p, A, ta_buf, s);
    if (!st && !tb) st = launch_transpose(p, B, tb_buf, s);
    const float *Ap = ta ? ta_buf : A, *Bp = tb ? B : tb_buf;
    GroupArgs g;
    g.grp_mem = p->d_grp_mem.ptr; g.grp_s = p->d_grp_s.ptr; g.grp_g = p->d_grp_g.ptr;
    g.unit_gr = p->d_unit_gr.ptr; g.unit_gc = p->d_unit_gc.ptr; g.unit_out = p->d_unit_out.ptr;
    g.unit_order = p->d_unit_order.ptr; g.pair_off = p->d_pair_off.ptr; g.pair_a = p->d_pair_a.ptr;
    g.pair_b = p->d_pair_b.ptr; g.gl_nm = p->d_gl_nm.ptr; g.gl_offd = p->d_gl_offd.ptr;
    g.stage_off = p->d_stage_off.ptr; g.stage_first = p->d_stage_first.ptr; g.tile_off = p->d_tile_off.ptr;
    g.nfun = p->d_nfun.ptr;
    g.lxa = g.lxb = 4;
    g.WR = g.WC = g.nsplit = 1;
    const int lw = p->all_mult4 ? 4 : p->all_even ? 2 : 1;   // bytes per lane load / 4
    const size_t ring = ring_bytes<2>();
    for (const auto &L : p->launches) {
        if (st) break;
        g.first = L.first;
        g.count = L.count;
        g.RB = L.rb;
        g.CB = L.cb;
        const dim3 grid((unsigned)L.count);
        const void *k;
        int threads = 512;
        if (L.rb * L.cb == 1) {
            k = lw == 4 ? (const void *)k_mgemm_f32acc<2, 1, 4> : lw == 2 ? (const void *)k_mgemm_f32acc<2, 1, 2> : (const void *)k_mgemm_f32acc<2, 1, 1>;
            threads = 128;
        } else if (L.rb == 1 || L.cb == 1) {
            // one block per consumer wave (block rows or block columns)
            k = lw == 4 ? (const void *)k_mgemm_f32acc<8, 1, 4> : lw == 2 ? (const void *)k_mgemm_f32acc<8, 1, 2> : (const void *)k_mgemm_f32acc<8, 1, 1>;
        } else if (L.cb <= 2) {
            k = lw == 4 ? (const void *)k_mgemm_f32acc<8, 2, 4> : lw == 2 ? (const void *)k_mgemm_f32acc<8, 2, 2> : (const void *)k_mgemm_f32acc<8, 2, 1>;
        } else if (L.cb <= 4) {
            k = lw == 4 ? (const void *)k_mgemm_f32acc<8, 4, 4> : lw == 2 ? (const void *)k_mgemm_f32acc<8, 4, 2> : (const void *)k_mgemm_f32acc<8, 4, 1>;
        } else {
            k = lw == 4 ? (const void *)k_mgemm_f32acc<8, 7, 4> : lw == 2 ? (const void *)k_mgemm_f32acc<8, 7, 2> : (const void *)k_mgemm_f32acc<8, 7, 1>;
        }
        // a unit of one block row (RB == 1) with several column blocks gives each wave one
        // block; with several block rows each wave takes a row of blocks
        if (L.rb == 1 && L.cb > 1) g.RB = 1;
        st = launch_grp(k, grid, threads, ring, s, g, reinterpret_cast<const double *>(Ap),
                        reinterpret_cast<const double *>(Bp), reinterpret_cast<double *>(C));
    }
    return st;
}

// F32SPLIT on the matrix cores: slices of op(A) (rows) and of op(B)^T (columns of op(B))
// with their per-row-and-level exponents in ws, then one launch per unit class.
int gemm_oz_ws(spm_pattern p, const float *A, int ta, const float *B, int tb, float *C, char *ws, hipStream_t s)
{
    const size_t sb = ws_align((size_t)p->n_stored * 8), eb = ws_align((size_t)p->n * p->nlev * sizeof(int32_t));
    uint4 *SA = reinterpret_cast<uint4 *>(ws), *SB = reinterpret_cast<uint4 *>(ws + sb);
    int32_t *EA = reinterpret_cast<int32_t *>(ws + 2 * sb), *EB = reinterpret_cast<int32_t *>(ws + 2 * sb + eb);
    const size_t slds = (size_t)kMax * p->nlev * sizeof(int);
    // view of op(A): rows of A (ta = 0, strided in the tiles) or columns of A (ta = 1);
    // view of op(B)^T: columns of B (tb = 0, contiguous) or rows of B (tb = 1)
    hipLaunchKernelGGL(k_oz_slice, dim3((unsigned)p->nc), dim3(64 * kSliceWaves), slds, s, p->nc, p->nlev, ta ? 1 : 0,
                       p->n_stored, p->d_blk_rp.ptr, p->d_tile_col.ptr, p->d_tile_off.ptr, p->d_trans.ptr,
                       p->d_nfun.ptr, p->d_cstart.ptr, p->d_clevel.ptr, A, SA, EA);
    hipLaunchKernelGGL(k_oz_slice, dim3((unsigned)p->nc), dim3(64 * kSliceWaves), slds, s, p->nc, p->nlev, tb ? 0 : 1,
                       p->n_stored, p->d_blk_rp.ptr, p->d_tile_col.ptr, p->d_tile_off.ptr, p->d_trans.ptr,
                       p->d_nfun.ptr, p->d_cstart.ptr, p->d_clevel.ptr, B, SB, EB);
    SPM_HIP(hipGetLastError());
    GroupArgs g;
    g.grp_mem = p->d_grp_mem.ptr; g.grp_s = p->d_grp_s.ptr; g.grp_g = p->d_grp_g.ptr;
    g.unit_gr = p->d_unit_gr.ptr; g.unit_gc = p->d_unit_gc.ptr; g.unit_out = p->d_unit_out.ptr;
    g.unit_order = p->d_unit_order.ptr; g.pair_off = p->d_pair_off.ptr; g.pair_a = p->d_pair_a_lv.ptr;
    g.pair_b = p->d_pair_b_lv.ptr; g.gl_nm = p->d_gl_nml.ptr; g.gl_offd = p->d_gl_offT.ptr;
    g.stage_off = p->d_stage_off_lv.ptr; g.stage_first = p->d_stage_first_lv.ptr; g.tile_off = p->d_tile_off.ptr;
    g.nfun = p->d_nfun.ptr;
    g.lxa = g.lxb = 4;
    g.WR = g.WC = g.nsplit = 1;
    OzArgs z{EA, EB, p->d_cstart.ptr, p->nlev};
    static std::mutex mu;
    static std::set<std::pair<int, const void *>> ready;   // (device, kernel)
    int dev = 0;
    SPM_HIP(hipGetDevice(&dev));
    for (const auto &L : p->launches) {
        g.first = L.first;
        g.count = L.count;
        g.RB = L.rb;
        g.CB = L.cb;
        const int rows_split = L.rb > 1 && L.cb == 1 ? 1 : 0;
        const int sub_rows = L.rb > 1 && L.cb > 1 ? L.rb : 1;
        const int nconsumer = rows_split ? L.rb : L.cb;
        const int erows = rows_split ? 16 * L.rb : 16, ecols = rows_split ? 16 : 16 * L.cb;
        const bool share = nconsumer > 1;
        const size_t lds = (share ? ring_bytes<5, OzTab>() + 6 * 4096 : ring_bytes<3, OzTab>()) +
                           (size_t)(erows + ecols) * p->nlev * sizeof(int);
        const void *k = share ? (const void *)k_mgemm_oz<8, true> : (const void *)k_mgemm_oz<2, false>;
        const int threads = share ? 512 : 128;
        {
            std::lock_guard<std::mutex> lock(mu);
            if (!ready.count({dev, k})) {
                SPM_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
                ready.insert({dev, k});
            }
        }
        const int64_t nwg = sub_rows > 1 ? (L.count + 7) / 8 * 8 * sub_rows : L.count;
        const int64_t ns = p->n_stored;
        void *args[] = {&g, &z, (void *)&rows_split, (void *)&sub_rows, &SA, &SB, &C, (void *)&ns};
        SPM_HIP(hipLaunchKernel(k, dim3((unsigned)nwg), dim3(threads), args, lds, s));
    }
    return SPM_OK;
}

// C = P_S(op(A) op(B)) in precision prec with a workspace of at least
// gemm_ws_bytes(p, prec, ta, tb) bytes (256-byte aligned).
int gemm_ws(spm_pattern p, int prec, const void *A, int ta, const void *B, int tb, void *C, void *ws,
            hipStream_t s)
{
    if (p->n_tiles == 0) return SPM_OK;
    char *w = static_cast<char *>(ws);
    int st;
    if (prec == SPM_F64) {
        st = gemm_grouped_ws(p, static_cast<const double *>(A), ta, static_cast<const double *>(B), tb,
                             static_cast<double *>(C), w, s);
    } else if (prec == SPM_F32ACC && f32acc_grouped(p)) {
        st = gemm_f32acc_ws(p, static_cast<const float *>(A), ta, static_cast<const float *>(B), tb,
                            static_cast<float *>(C), w, s);
    } else if (prec == SPM_F32SPLIT && oz_ok(p)) {
        st = gemm_oz_ws(p, static_cast<const float *>(A), ta, static_cast<const float *>(B), tb,
                        static_cast<float *>(C), w, s);
    } else {
        GemmArgs g = gemm_args(p);
        dim3 grid((unsigned)p->n_tiles), block(64);
        const int sel = (ta ? 2 : 0) + (tb ? 1 : 0);
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
        st = SPM_OK;
    }
    if (st) return st;
    if (p->d_keep.ptr)
        hipLaunchKernelGGL(k_apply_keep, dim3(grid1d(p->n_stored, 256)), dim3(256), 0, s, p->n_stored, prec,
                           p->d_keep.ptr, C);
    SPM_HIP(hipGetLastError());
    return SPM_OK;
}

// The same with a stream-ordered temporary workspace.
int launch_gemm(spm_pattern p, int prec, const void *A, int ta, const void *B, int tb, void *C, hipStream_t s)
{
    const size_t need = gemm_ws_bytes(p, prec, ta, tb);
    void *ws = nullptr;
    if (need && hipMallocAsync(&ws, need, s) != hipSuccess)
        return fail(SPM_ENOMEM, "masked product: temporary workspace");
    const int st = gemm_ws(p, prec, A, ta, B, tb, C, ws, s);
    if (ws) (void)hipFreeAsync(ws, s);
    return st;
}

int launch_reduce(spm_pattern p, int op, int prec, const void *x, const void *y, const double *vec, double alpha,
                  int post, double scale, double *out, hipStream_t s)
{
    int64_t nb;
    if (op == RED_QUAD) {
        nb = std::max<int64_t>(1, (p->n_tiles + kRedTiles - 1) / kRedTiles);
        hipLaunchKernelGGL(k_reduce_tiles, dim3((unsigned)nb), dim3(kRedThreads), 0, s, op, p->n_tiles,
                           p->d_tile_off.ptr, p->d_tile_row.ptr, p->d_tile_col.ptr, p->d_nfun.ptr, p->d_cstart.ptr,
                           prec, p->n_stored, x, y, vec, alpha, p->d_partial.ptr);
    } else {
        const int64_t ns = p->n_stored, nseg = (ns + kFlatSeg - 1) / kFlatSeg;
        nb = std::max<int64_t>(1, std::min<int64_t>(kFlatBlocks, nseg));
        const int64_t *dg = p->d_diag_pos.ptr;
        const int64_t nd = (int64_t)p->d_diag_pos.n;
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(256), 0, s, ns, x, y, dg, nd, alpha, p->d_partial.ptr);
        };
        auto by_op = [&](auto pc) {
            constexpr int PC = decltype(pc)::value;
            if (op == RED_SQDIST) go(k_reduce_flat<PC, RED_SQDIST>);
            else if (op == RED_SQDIST_EYE) go(k_reduce_flat<PC, RED_SQDIST_EYE>);
            else go(k_reduce_flat<PC, RED_DOT>);
        };
        if (prec == SPM_F64) by_op(std::integral_constant<int, SPM_F64>());
        else if (prec == SPM_F32SPLIT) by_op(std::integral_constant<int, SPM_F32SPLIT>());
        else by_op(std::integral_constant<int, SPM_F32ACC>());
    }
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
    SPM_NEED_DEVICE(p, "spm_values_from_csr");
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
    SPM_NEED_DEVICE(p, "spm_values_to_csr");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_from_csr, dim3(grid1d(p->n_tiles, 1, 1 << 20)), dim3(64), 0, s, p->n_tiles,
                       p->d_tile_off.ptr, p->d_tile_row.ptr, p->d_tile_col.ptr, p->d_nfun.ptr, p->d_rowbase.ptr,
                       p->d_rowlen.ptr, p->d_colprefix.ptr, p->d_csr_pos.ptr, vals, csr, 1);
    SPM_HIP(hipGetLastError());
    return SPM_OK;
}

static int check_gemm_args(spm_pattern p, int prec, const void *A, int ta, const void *B, int tb, const void *C,
                           const char *name)
{
    if (!p || !A || !B || !C) return fail(SPM_EINVAL, std::string(name) + ": null pointer");
    SPM_NEED_DEVICE(p, name);
    if (!valid_prec(prec)) return fail(SPM_EINVAL, std::string(name) + ": bad precision");
    if ((ta != 0 && ta != 1) || (tb != 0 && tb != 1)) return fail(SPM_EINVAL, std::string(name) + ": bad transpose flag");
    const size_t vb = value_bytes(p, prec);
    if (overlap(A, C, vb) || overlap(B, C, vb)) return fail(SPM_EINVAL, std::string(name) + ": C aliases an operand");
    return SPM_OK;
}

extern "C" int spm_masked_gemm(spm_pattern p, int prec, const void *A, int ta, const void *B, int tb, void *C,
                               void *stream)
{
    int st = check_gemm_args(p, prec, A, ta, B, tb, C, "spm_masked_gemm");
    if (st) return st;
    return spm::launch_gemm(p, prec, A, ta, B, tb, C, (hipStream_t)stream);
}

extern "C" int spm_masked_gemm_workspace(spm_pattern p, int prec, int ta, int tb, size_t *bytes)
{
    if (!p || !bytes) return fail(SPM_EINVAL, "spm_masked_gemm_workspace: null pointer");
    if (!valid_prec(prec)) return fail(SPM_EINVAL, "spm_masked_gemm_workspace: bad precision");
    *bytes = spm::gemm_ws_bytes(p, prec, ta != 0, tb != 0);
    return SPM_OK;
}

// ws must not overlap A, B or C (the transposed operands are written there).
static int check_ws(spm_pattern p, int prec, const void *const *bufs, int nbufs, const void *ws, size_t bytes,
                    size_t need, const char *name)
{
    if (need == 0) return SPM_OK;
    if (!ws || bytes < need) return fail(SPM_EINVAL, std::string(name) + ": workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(SPM_EINVAL, std::string(name) + ": workspace not 256-byte aligned");
    const size_t vb = value_bytes(p, prec);
    for (int i = 0; i < nbufs; ++i)
        if (overlap2(bufs[i], vb, ws, need)) return fail(SPM_EINVAL, std::string(name) + ": workspace overlaps an operand");
    return SPM_OK;
}

extern "C" int spm_masked_gemm_ws(spm_pattern p, int prec, const void *A, int ta, const void *B, int tb, void *C,
                                  void *ws, size_t bytes, void *stream)
{
    int st = check_gemm_args(p, prec, A, ta, B, tb, C, "spm_masked_gemm_ws");
    if (st) return st;
    const void *bufs[3] = {A, B, C};
    if ((st = check_ws(p, prec, bufs, 3, ws, bytes, spm::gemm_ws_bytes(p, prec, ta, tb), "spm_masked_gemm_ws")))
        return st;
    return spm::gemm_ws(p, prec, A, ta, B, tb, C, ws, (hipStream_t)stream);
}

// ---------------------------------------------------------------- product without allocation
// A fixed device array serves as the product's workspace for callers that cannot
// allocate.  Host code never uses the array's name as an address: its device address
// is taken once per device with hipGetSymbolAddress and kept in `g_noalloc_ptr`.
static constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call there).
int noalloc_scratch(void **out)
{
    int dev = 0;
    SPM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SPM_EUNSUPPORTED, "spm_masked_gemm_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SPM_EHIP, std::string("spm_masked_gemm_noalloc: hipGetSymbolAddress failed: ") +
                                      hipGetErrorString(e));
        g_noalloc_ptr[dev] = ptr;
    }
    *out = g_noalloc_ptr[dev];
    return SPM_OK;
}
}  // namespace

extern "C" int spm_masked_gemm_noalloc_max_bytes(size_t *bytes)
{
    if (!bytes) return fail(SPM_EINVAL, "spm_masked_gemm_noalloc_max_bytes: null pointer");
    *bytes = kNoAllocScratchBytes;
    return SPM_OK;
}

extern "C" int spm_masked_gemm_noalloc(spm_pattern p, int prec, const void *A, int ta, const void *B, int tb, void *C,
                                       void *stream)
{
    int st = check_gemm_args(p, prec, A, ta, B, tb, C, "spm_masked_gemm_noalloc");
    if (st) return st;
    const size_t need = spm::gemm_ws_bytes(p, prec, ta, tb);
    if (need > kNoAllocScratchBytes)
        return fail(SPM_EINVAL, "spm_masked_gemm_noalloc: the product needs " + std::to_string(need) +
                                    " bytes of workspace, above the fixed " + std::to_string(kNoAllocScratchBytes) +
                                    " (use spm_masked_gemm_ws with a caller workspace)");
    void *ws = nullptr;
    if (need && (st = noalloc_scratch(&ws))) return st;
    return spm::gemm_ws(p, prec, A, ta, B, tb, C, ws, (hipStream_t)stream);
}

static size_t backward_ws_bytes(spm_pattern p, int prec)
{
    return std::max(spm::gemm_ws_bytes(p, prec, 0, 1), spm::gemm_ws_bytes(p, prec, 1, 0));
}

static int check_backward(spm_pattern p, int prec, const void *dC, const void *A, const void *B, void *dA, void *dB,
                          const char *name)
{
    if (!p || !dC || !A || !B) return fail(SPM_EINVAL, std::string(name) + ": null pointer");
    SPM_NEED_DEVICE(p, name);
    if (!valid_prec(prec)) return fail(SPM_EINVAL, std::string(name) + ": bad precision");
    const size_t vb = value_bytes(p, prec);
    for (void *o : {dA, dB})
        if (o && (overlap(o, dC, vb) || overlap(o, A, vb) || overlap(o, B, vb)))
            return fail(SPM_EINVAL, std::string(name) + ": output aliases an input");
    if (dA && dB && overlap(dA, dB, vb)) return fail(SPM_EINVAL, std::string(name) + ": dA aliases dB");
    return SPM_OK;
}

extern "C" int spm_masked_gemm_backward(spm_pattern p, int prec, const void *dC, const void *A, const void *B,
                                        void *dA, void *dB, void *stream)
{
    int st = check_backward(p, prec, dC, A, B, dA, dB, "spm_masked_gemm_backward");
    if (st) return st;
    if (dA && (st = spm::launch_gemm(p, prec, dC, 0, B, 1, dA, (hipStream_t)stream))) return st;   // P_S(dC B^T)
    if (dB && (st = spm::launch_gemm(p, prec, A, 1, dC, 0, dB, (hipStream_t)stream))) return st;   // P_S(A^T dC)
    return SPM_OK;
}

extern "C" int spm_masked_gemm_backward_workspace(spm_pattern p, int prec, size_t *bytes)
{
    if (!p || !bytes) return fail(SPM_EINVAL, "spm_masked_gemm_backward_workspace: null pointer");
    if (!valid_prec(prec)) return fail(SPM_EINVAL, "spm_masked_gemm_backward_workspace: bad precision");
    *bytes = backward_ws_bytes(p, prec);
    return SPM_OK;
}

extern "C" int spm_masked_gemm_backward_ws(spm_pattern p, int prec, const void *dC, const void *A, const void *B,
                                           void *dA, void *dB, void *ws, size_t bytes, void *stream)
{
    int st = check_backward(p, prec, dC, A, B, dA, dB, "spm_masked_gemm_backward_ws");
    if (st) return st;
    const void *bufs[5] = {dC, A, B, dA, dB};
    if ((st = check_ws(p, prec, bufs, 5, ws, bytes, backward_ws_bytes(p, prec), "spm_masked_gemm_backward_ws")))
        return st;
    hipStream_t s = (hipStream_t)stream;
    if (dA && (st = spm::gemm_ws(p, prec, dC, 0, B, 1, dA, ws, s))) return st;   // P_S(dC B^T)
    if (dB && (st = spm::gemm_ws(p, prec, A, 1, dC, 0, dB, ws, s))) return st;   // P_S(A^T dC)
    return SPM_OK;
}

extern "C" int spm_axpy(spm_pattern p, int prec, double alpha, const void *X, double beta, void *Y, void *stream)
{
    if (!p || !Y) return fail(SPM_EINVAL, "spm_axpy: null pointer");
    SPM_NEED_DEVICE(p, "spm_axpy");
    if (!valid_prec(prec)) return fail(SPM_EINVAL, "spm_axpy: bad precision");
    return spm::launch_axpy(p, prec, alpha, X, beta, Y, (hipStream_t)stream);
}

extern "C" int spm_convert(spm_pattern p, int pf, const void *X, int pt, void *Y, void *stream)
{
    if (!p || !X || !Y) return fail(SPM_EINVAL, "spm_convert: null pointer");
    SPM_NEED_DEVICE(p, "spm_convert");
    if (!valid_prec(pf) || !valid_prec(pt)) return fail(SPM_EINVAL, "spm_convert: bad precision");
    if (overlap2(X, value_bytes(p, pf), Y, value_bytes(p, pt)))
        return fail(SPM_EINVAL, "spm_convert: X and Y overlap");
    return spm::launch_convert(p, pf, X, pt, Y, (hipStream_t)stream);
}

extern "C" int spm_sqdist(spm_pattern p, int prec, const void *X, const void *Y, double *out, void *stream)
{
    if (!p || !X || !out) return fail(SPM_EINVAL, "spm_sqdist: null pointer");
    SPM_NEED_DEVICE(p, "spm_sqdist");
    if (!valid_prec(prec)) return fail(SPM_EINVAL, "spm_sqdist: bad precision");
    return spm::launch_reduce(p, RED_SQDIST, prec, X, Y, nullptr, 0.0, 0, 1.0, out, (hipStream_t)stream);
}

extern "C" int spm_sqdist_eye(spm_pattern p, int prec, double alpha, const void *X, double *out, void *stream)
{
    if (!p || !X || !out) return fail(SPM_EINVAL, "spm_sqdist_eye: null pointer");
    SPM_NEED_DEVICE(p, "spm_sqdist_eye");
    if (!valid_prec(prec)) return fail(SPM_EINVAL, "spm_sqdist_eye: bad precision");
    return spm::launch_reduce(p, RED_SQDIST_EYE, prec, X, nullptr, nullptr, alpha, 0, 1.0, out, (hipStream_t)stream);
}

extern "C" int spm_dot(spm_pattern p, const double *X, const double *Y, double *out, void *stream)
{
    if (!p || !X || !Y || !out) return fail(SPM_EINVAL, "spm_dot: null pointer");
    SPM_NEED_DEVICE(p, "spm_dot");
    return spm::launch_reduce(p, RED_DOT, SPM_F64, X, Y, nullptr, 0.0, 0, 1.0, out, (hipStream_t)stream);
}

extern "C" int spm_quadform(spm_pattern p, const double *X, const double *y, double *out, void *stream)
{
    if (!p || !X || !y || !out) return fail(SPM_EINVAL, "spm_quadform: null pointer");
    SPM_NEED_DEVICE(p, "spm_quadform");
    return spm::launch_reduce(p, RED_QUAD, SPM_F64, X, nullptr, y, 0.0, 0, 1.0, out, (hipStream_t)stream);
}

extern "C" int spm_fill_outer(spm_pattern p, double alpha, const double *y, double *X, void *stream)
{
    if (!p || !y || !X) return fail(SPM_EINVAL, "spm_fill_outer: null pointer");
    SPM_NEED_DEVICE(p, "spm_fill_outer");
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

// Newton-Schulz scratch: Y and T (FP64), the bulk-precision copies of A, X, Y, T, and
// the workspace of one product, each 256-byte aligned.
// Newton-Schulz scratch: Y and T (FP64), then a region used by the bulk iterations for
// the bulk-precision copies of A, X, Y, T and their product workspace, and afterwards
// by the FP64 iterations for theirs.  Every part is 256-byte aligned.
size_t ns_scratch(spm_pattern p, int bulk, int32_t nbulk)
{
    const size_t vb8 = spm::ws_align((size_t)p->n_stored * sizeof(double));
    size_t region = spm::gemm_ws_bytes(p, SPM_F64, 0, 0);
    if (bulk != SPM_F64 && nbulk > 0)
        region = std::max(region, 4 * spm::ws_align(value_bytes(p, bulk)) + spm::gemm_ws_bytes(p, bulk, 0, 0));
    return 2 * vb8 + region;
}

}  // namespace

extern "C" int spm_expm_taylor_scratch(spm_pattern p, size_t *bytes)
{
    if (!p || !bytes) return fail(SPM_EINVAL, "spm_expm_taylor_scratch: null pointer");
    *bytes = spm::ws_align((size_t)p->n_stored * sizeof(double)) + spm::gemm_ws_bytes(p, SPM_F64, 0, 0);
    return SPM_OK;
}

// Power series of exp(A) (end of Section 4.4) cut after `terms` terms, Horner's rule with
// formatted products: E = I; E <- I + P_S(A E) / k for k = terms .. 1.  The two value
// arrays E and scratch alternate; each step is one masked product and one pass that
// scales by 1/k and adds the identity.
extern "C" int spm_expm_taylor(spm_pattern p, const double *A, double *E, int32_t terms, void *scratch,
                               size_t scratch_bytes, void *stream)
{
    if (!p || !A || !E) return fail(SPM_EINVAL, "spm_expm_taylor: null pointer");
    SPM_NEED_DEVICE(p, "spm_expm_taylor");
    if (terms < 0) return fail(SPM_EINVAL, "spm_expm_taylor: negative number of terms");
    const size_t vb8 = (size_t)p->n_stored * sizeof(double), vba = spm::ws_align(vb8);
    const size_t need = vba + spm::gemm_ws_bytes(p, SPM_F64, 0, 0);
    if (terms > 0 && (!scratch || scratch_bytes < need)) return fail(SPM_EINVAL, "spm_expm_taylor: scratch too small");
    if (terms > 0 && reinterpret_cast<uintptr_t>(scratch) % 256)
        return fail(SPM_EINVAL, "spm_expm_taylor: scratch not 256-byte aligned");
    if (overlap(A, E, vb8) || (terms > 0 && (overlap2(A, vb8, scratch, need) || overlap2(E, vb8, scratch, need))))
        return fail(SPM_EINVAL, "spm_expm_taylor: buffers overlap");
    hipStream_t s = (hipStream_t)stream;
    const int64_t ns = p->n_stored;
    double *cur = E, *oth = static_cast<double *>(scratch);
    void *gw = static_cast<char *>(scratch) + vba;
    int st;
    hipLaunchKernelGGL(k_fill, dim3(grid1d(ns, 256)), dim3(256), 0, s, ns, (int)SPM_F64, 0.0, (void *)cur);
    if ((st = spm::launch_axpy(p, SPM_F64, 1.0, nullptr, 1.0, cur, s))) return st;
    for (int32_t k = terms; k >= 1; --k) {
        if ((st = spm::gemm_ws(p, SPM_F64, A, 0, cur, 0, oth, gw, s))) return st;
        if ((st = spm::launch_axpy(p, SPM_F64, 1.0, nullptr, 1.0 / k, oth, s))) return st;   // oth/k + I
        std::swap(cur, oth);
    }
    if (cur != E) SPM_HIP(hipMemcpyAsync(E, cur, vb8, hipMemcpyDeviceToDevice, s));
    return SPM_OK;
}

extern "C" int spm_spmm(spm_pattern p, const double *A, const double *X, int32_t r, double *Y, void *stream)
{
    if (!p) return fail(SPM_EINVAL, "spm_spmm: null pattern");
    SPM_NEED_DEVICE(p, "spm_spmm");
    if (r < 0) return fail(SPM_EINVAL, "spm_spmm: negative column count");
    if (r == 0 || p->nc == 0) return SPM_OK;                 // X and Y may then be null
    if (!A || !X || !Y) return fail(SPM_EINVAL, "spm_spmm: null pointer");
    if (p->n >= (int64_t(1) << 25)) return fail(SPM_EINVAL, "spm_spmm: n must be below 2^25");
    const size_t vb8 = (size_t)p->n_stored * sizeof(double), pb = (size_t)p->n * r * sizeof(double);
    if (overlap2(X, pb, Y, pb) || overlap2(A, vb8, Y, pb)) return fail(SPM_EINVAL, "spm_spmm: buffers overlap");
    hipStream_t s = (hipStream_t)stream;
    const dim3 g((unsigned)p->nc), b(64 * kSpmmWaves);
// passes of 16 columns of X
    hipLaunchKernelGGL(k_spmm<1>, g, b, 0, s, p->nc, (int64_t)p->n, r, p->d_pc_rp.ptr, p->d_pc_off.ptr,
                       p->d_pc_g.ptr, p->d_pc_w.ptr, p->d_nfun.ptr, p->d_cstart.ptr, A, X, Y);
    SPM_HIP(hipGetLastError());
    return SPM_OK;
}

extern "C" int spm_ns_sqrt_scratch(spm_pattern p, size_t *bytes)
{
    if (!p || !bytes) return fail(SPM_EINVAL, "spm_ns_sqrt_scratch: null pointer");
    *bytes = 3 * spm::ws_align((size_t)p->n_stored * sizeof(double)) + spm::gemm_ws_bytes(p, SPM_F64, 0, 0);
    return SPM_OK;
}

// Coupled Newton-Schulz iteration for A^{1/2} and A^{-1/2} with formatted products (the
// square root of Section 4.4, measured in Section 5.3): Y_0 = A, Z_0 = I,
// T_k = (3I - P_S(Z_k Y_k)) / 2, Y_{k+1} = P_S(Y_k T_k), Z_{k+1} = P_S(T_k Z_k).  Three
// masked products per iteration; the iterates alternate between the caller's arrays
// and the scratch.
extern "C" int spm_ns_sqrt(spm_pattern p, const double *A, double *Y, double *Z, int32_t iters,
                           double *residuals, void *scratch, size_t scratch_bytes, void *stream)
{
    if (!p || !A || !Y || !Z) return fail(SPM_EINVAL, "spm_ns_sqrt: null pointer");
    SPM_NEED_DEVICE(p, "spm_ns_sqrt");
    if (iters < 0) return fail(SPM_EINVAL, "spm_ns_sqrt: negative iteration count");
    const size_t vb8 = (size_t)p->n_stored * sizeof(double), vba = spm::ws_align(vb8);
    const size_t need = 3 * vba + spm::gemm_ws_bytes(p, SPM_F64, 0, 0);
    if (!scratch || scratch_bytes < need) return fail(SPM_EINVAL, "spm_ns_sqrt: scratch too small");
    if (reinterpret_cast<uintptr_t>(scratch) % 256) return fail(SPM_EINVAL, "spm_ns_sqrt: scratch not 256-byte aligned");
    if (overlap(A, Y, vb8) || overlap(A, Z, vb8) || overlap(Y, Z, vb8) || overlap2(A, vb8, scratch, need) ||
        overlap2(Y, vb8, scratch, need) || overlap2(Z, vb8, scratch, need))
        return fail(SPM_EINVAL, "spm_ns_sqrt: buffers overlap");
    hipStream_t s = (hipStream_t)stream;
    const int64_t ns = p->n_stored;
    const double rs = 1.0 / std::sqrt((double)p->n);
    char *sc = static_cast<char *>(scratch);
    double *W = reinterpret_cast<double *>(sc);
    double *y = Y, *z = Z, *yn = reinterpret_cast<double *>(sc + vba), *zn = reinterpret_cast<double *>(sc + 2 * vba);
    void *gw = sc + 3 * vba;
    int st;
    SPM_HIP(hipMemcpyAsync(y, A, vb8, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_fill, dim3(grid1d(ns, 256)), dim3(256), 0, s, ns, (int)SPM_F64, 0.0, (void *)z);
    if ((st = spm::launch_axpy(p, SPM_F64, 1.0, nullptr, 1.0, z, s))) return st;
    for (int32_t k = 0; k < iters; ++k) {
        if ((st = spm::gemm_ws(p, SPM_F64, z, 0, y, 0, W, gw, s))) return st;          // P_S(Z Y)
        if (residuals &&
            (st = spm::launch_reduce(p, 1, SPM_F64, W, nullptr, nullptr, 1.0, 1, rs, residuals + k, s)))
            return st;
        if ((st = spm::launch_axpy(p, SPM_F64, 1.5, nullptr, -0.5, W, s))) return st;  // T = (3I - W) / 2
        if ((st = spm::gemm_ws(p, SPM_F64, y, 0, W, 0, yn, gw, s))) return st;
        if ((st = spm::gemm_ws(p, SPM_F64, W, 0, z, 0, zn, gw, s))) return st;
        std::swap(y, yn);
        std::swap(z, zn);
    }
    if (y != Y) SPM_HIP(hipMemcpyAsync(Y, y, vb8, hipMemcpyDeviceToDevice, s));
    if (z != Z) SPM_HIP(hipMemcpyAsync(Z, z, vb8, hipMemcpyDeviceToDevice, s));
    return SPM_OK;
}

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
    SPM_NEED_DEVICE(p, "spm_newton_schulz");
    if (iters < 0 || nfin < 0) return fail(SPM_EINVAL, "spm_newton_schulz: negative iteration count");
    if (!valid_prec(bulk)) return fail(SPM_EINVAL, "spm_newton_schulz: bad precision");
    const int32_t nbulk = bulk == SPM_F64 ? 0 : std::max(0, iters - nfin);
    const size_t need = ns_scratch(p, bulk, nbulk);
    if (!scratch || scratch_bytes < need) return fail(SPM_EINVAL, "spm_newton_schulz: scratch too small");
    if (reinterpret_cast<uintptr_t>(scratch) % 256) return fail(SPM_EINVAL, "spm_newton_schulz: scratch not 256-byte aligned");
    const size_t vb8 = (size_t)p->n_stored * sizeof(double), vba = spm::ws_align(vb8);
    if (overlap(A, X, vb8) || overlap2(X, vb8, scratch, need) || overlap2(A, vb8, scratch, need))
        return fail(SPM_EINVAL, "spm_newton_schulz: buffers overlap");
    hipStream_t s = (hipStream_t)stream;
    const int64_t ns = p->n_stored;
    const double rs = 1.0 / std::sqrt((double)p->n);
    char *sc = static_cast<char *>(scratch);
    double *Y = reinterpret_cast<double *>(sc);
    double *T = reinterpret_cast<double *>(sc + vba);
    char *sp = sc + 2 * vba;
    const size_t vb = spm::ws_align(value_bytes(p, bulk));
    const bool lowp = bulk != SPM_F64 && nbulk > 0;
    void *As = sp, *Xs = sp + vb, *Ys = sp + 2 * vb, *Ts = sp + 3 * vb;
    void *gwb = sp + 4 * vb;                   // product workspace of the bulk iterations
    void *gw = sp;                             // of the FP64 ones (the bulk copies are dead by then)
    (void)lowp;
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
            if ((st = spm::gemm_ws(p, bulk, As, 0, Xs, 0, Ys, gwb, s))) return st;
            if ((st = spm::launch_reduce(p, 1, bulk, Ys, nullptr, nullptr, 1.0, 1, rs, res + k, s))) return st;
            if ((st = spm::launch_axpy(p, bulk, 2.0, nullptr, -1.0, Ys, s))) return st;
            if ((st = spm::gemm_ws(p, bulk, Xs, 0, Ys, 0, Ts, gwb, s))) return st;
            std::swap(Xs, Ts);
            if (k == nbulk - 1 && (st = spm::launch_convert(p, bulk, Xs, SPM_F64, cur, s))) return st;
        } else {
            if ((st = spm::gemm_ws(p, SPM_F64, A, 0, cur, 0, Y, gw, s))) return st;
            if ((st = spm::launch_reduce(p, 1, SPM_F64, Y, nullptr, nullptr, 1.0, 1, rs, res + k, s))) return st;
            if ((st = spm::launch_axpy(p, SPM_F64, 2.0, nullptr, -1.0, Y, s))) return st;
            if ((st = spm::gemm_ws(p, SPM_F64, cur, 0, Y, 0, oth, gw, s))) return st;
            std::swap(cur, oth);
        }
    }
    if (ckpt && ckpt[iters]) SPM_HIP(hipMemcpyAsync(ckpt[iters], cur, vb8, hipMemcpyDeviceToDevice, s));
    if ((st = spm::gemm_ws(p, SPM_F64, A, 0, cur, 0, Y, gw, s))) return st;
    if ((st = spm::launch_reduce(p, 1, SPM_F64, Y, nullptr, nullptr, 1.0, 1, rs, res + iters, s))) return st;
    if (cur != X) SPM_HIP(hipMemcpyAsync(X, cur, vb8, hipMemcpyDeviceToDevice, s));
    double first = 0.0, last = 0.0;
    SPM_HIP(hipMemcpyAsync(&first, res, sizeof(double), hipMemcpyDeviceToHost, s));
    SPM_HIP(hipMemcpyAsync(&last, res + iters, sizeof(double), hipMemcpyDeviceToHost, s));
    SPM_HIP(hipStreamSynchronize(s));
    if (!std::isfinite(last)) return fail(SPM_ENOTCONV, "spm_newton_schulz: residual is not finite");
    if (last > first)
        return fail(SPM_ENOTCONV, "spm_newton_schulz: final residual " + std::to_string(last) +
                                      " exceeds the initial residual " + std::to_string(first));
    return SPM_OK;
}


extern "C" int spm_contour_invsqrt_scratch(spm_pattern p, int32_t ns_iters, size_t *bytes)
{
    if (!p || !bytes) return fail(SPM_EINVAL, "spm_contour_invsqrt_scratch: null pointer");
    if (ns_iters < 0) return fail(SPM_EINVAL, "spm_contour_invsqrt_scratch: negative iteration count");
    *bytes = 2 * spm::ws_align((size_t)p->n_stored * sizeof(double)) + ns_scratch(p, SPM_F64, 0) +
             (size_t)(ns_iters + 1) * sizeof(double);
    return SPM_OK;
}

// A^{-1/2} by the contour quadrature of Section 4.4 (eq. ContInt): sum_k c_k X_k, X_k the
// masked Newton-Schulz inverse of A + w_k^2 I started from 2 / (lam_min + lam_max + 2 w_k^2) I.
extern "C" int spm_contour_invsqrt(spm_pattern p, const double *A, double lam_min, double lam_max, int32_t nodes,
                                   int32_t ns_iters, double *out, double *residuals, void *scratch,
                                   size_t scratch_bytes, void *stream)
{
    if (!p || !A || !out) return fail(SPM_EINVAL, "spm_contour_invsqrt: null pointer");
    SPM_NEED_DEVICE(p, "spm_contour_invsqrt");
    if (ns_iters < 0) return fail(SPM_EINVAL, "spm_contour_invsqrt: negative iteration count");
    std::vector<double> w2(std::max(nodes, 1)), cw(std::max(nodes, 1));
    int st;
    if ((st = spm_contour_rule(lam_min, lam_max, nodes, w2.data(), cw.data()))) return st;
    const size_t vb8 = (size_t)p->n_stored * sizeof(double), vba = spm::ws_align(vb8), nsb = ns_scratch(p, SPM_F64, 0);
    const size_t need = 2 * vba + nsb + (size_t)(ns_iters + 1) * sizeof(double);
    if (!scratch || scratch_bytes < need) return fail(SPM_EINVAL, "spm_contour_invsqrt: scratch too small");
    if (reinterpret_cast<uintptr_t>(scratch) % 256) return fail(SPM_EINVAL, "spm_contour_invsqrt: scratch not 256-byte aligned");
    if (overlap(A, out, vb8) || overlap2(A, vb8, scratch, need) || overlap2(out, vb8, scratch, need))
        return fail(SPM_EINVAL, "spm_contour_invsqrt: buffers overlap");
    hipStream_t s = (hipStream_t)stream;
    const int64_t ns = p->n_stored;
    double *As = static_cast<double *>(scratch);
    double *X = reinterpret_cast<double *>(static_cast<char *>(scratch) + vba);
    char *nsw = static_cast<char *>(scratch) + 2 * vba;
    double *res = reinterpret_cast<double *>(nsw + nsb);
    const bool progress = std::getenv("SPM_PROGRESS") != nullptr;   // one line per node on stderr
    hipLaunchKernelGGL(k_fill, dim3(grid1d(ns, 256)), dim3(256), 0, s, ns, (int)SPM_F64, 0.0, (void *)out);
    for (int32_t k = 0; k < nodes; ++k) {
        SPM_HIP(hipMemcpyAsync(As, A, vb8, hipMemcpyDeviceToDevice, s));
        if ((st = spm::launch_axpy(p, SPM_F64, w2[k], nullptr, 1.0, As, s))) return st;          // A + w_k^2 I
        const double alpha0 = 2.0 / (lam_min + lam_max + 2.0 * w2[k]);
        if ((st = spm_newton_schulz(p, As, X, ns_iters, ns_iters, SPM_F64, alpha0, res, nullptr, nsw, nsb, s)))
            return st;
        if (residuals) SPM_HIP(hipMemcpyAsync(residuals + k, res + ns_iters, sizeof(double), hipMemcpyDeviceToDevice, s));
        if ((st = spm::launch_axpy(p, SPM_F64, cw[k], X, 1.0, out, s))) return st;
        if (progress) std::fprintf(stderr, "[spm] contour_invsqrt: node %d of %d done\n", k + 1, nodes);
    }
    return SPM_OK;
}
