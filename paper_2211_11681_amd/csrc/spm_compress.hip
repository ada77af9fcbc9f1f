// Samplet compression of a Matern kernel matrix on the device (Section 3.3):
// vals = P_S(T K T^T), evaluated exactly with O(N^2) kernel evaluations.
//
// T is never formed.  Its action is the two-scale transform of Section 3.2 applied
// in place: every cluster maps the values at its input slots (its points for a
// leaf, the scaling slots of its two sons otherwise) by Q^T, writing output k to
// input slot k; the first outputs are the scaling coefficients handed up, the rest
// are samplet coefficients.
//
// K is processed in panels of rows: the rows of one subtree (points p0 .. p0+rows).
//   1. W = K(panel points, all points)                       rows x N
//   2. column transform: every row of W, all clusters, leaves first
//   3. row transform:   the subtree's clusters combine rows of W, leaves first
//   4. extract:         samplet rows of the subtree's clusters -> tiles on S
//   5. the subtree root's scaling rows move to a buffer U
// After all panels the clusters above the panel level combine rows of U the same
// way (step 3 and 4 on U).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <type_traits>
#include <vector>

#include "spm_internal.h"

using spm::fail;

namespace {

constexpr int kMaxIn = 64;   // largest number of inputs of one cluster transform

struct KParams {
    double c[4];     // polynomial P(s) coefficients, degree p
    int p;
    double sfac;     // s = sfac * r, sfac = sqrt(2p+1) / ell
    double ell, scale;
    int deriv;
};

__device__ inline double kernel_value(double r, const KParams &kp)
{
    const double s = kp.sfac * r;
    double poly = 0.0, dpoly = 0.0;
    for (int k = kp.p; k >= 0; --k) poly = fma(poly, s, kp.c[k]);
    for (int k = kp.p; k >= 1; --k) dpoly = fma(dpoly, s, k * kp.c[k]);
    const double ex = exp(-s);
    if (!kp.deriv) return kp.scale * ex * poly;
    return kp.scale * (-s / kp.ell) * (dpoly - poly) * ex;
}

__global__ void k_eval(double *__restrict__ W, const double *__restrict__ pts, int d, int64_t p0, int64_t rows,
                       int64_t n, KParams kp)
{
    const int64_t total = rows * n;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = idx / n, q = idx - r * n;
        const double *x = pts + (p0 + r) * d, *y = pts + q * d;
        double acc = 0.0;
        for (int a = 0; a < d; ++a) {
            const double df = x[a] - y[a];
            acc = fma(df, df, acc);
        }
        W[idx] = kernel_value(sqrt(acc), kp);
    }
}

// The transforms below keep Q (m x m; the row transform also the inputs of its 64
// lanes, m x 64) in dynamic LDS sized by the largest cluster of the launch, mmax, so
// that several workgroups share a CU (a fixed size for the limit of 64 inputs allowed
// two).
__host__ __device__ constexpr size_t tr_lds_bytes(int mmax) { return (size_t)(mmax * mmax + 64 * mmax) * sizeof(double); }

// Column transform of one tree level: block (cluster list entry, 64 rows), four waves
// taking the rows in turn.  Lane k of a wave owns slot k of the cluster: one coalesced
// load reads the row's inputs, lane k forms output k from all inputs (read out of the
// lanes that hold them) and Q^T kept in LDS, and stores it back to slot k.
__device__ __forceinline__ double lane_value(double v, int i)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), i);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), i);
    return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(256) void k_coltr(double *__restrict__ W, int64_t rows, int64_t n,
                                               const int32_t *__restrict__ clist, const int32_t *__restrict__ nin,
                                               const int64_t *__restrict__ qoff, const double *__restrict__ qmat,
                                               const int64_t *__restrict__ slotoff, const int64_t *__restrict__ slots,
                                               int mmax)
{
    extern __shared__ double tr_smem[];
    double *sQt = tr_smem;                           // sQt[i * m + k] = Q[k * m + i]
    const int c = clist[blockIdx.x];
    const int m = nin[c];
    const double *Q = qmat + qoff[c];
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) sQt[(e % m) * m + e / m] = Q[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t slot = lane < m ? slots[slotoff[c] + lane] : 0;
    for (int rr = wave; rr < 64; rr += 4) {
        const int64_t r = (int64_t)blockIdx.y * 64 + rr;
        if (r >= rows) break;
        double *row = W + r * n;
        const double v = lane < m ? row[slot] : 0.0;
        double acc = 0.0;
        for (int i = 0; i < m; ++i) acc = fma(sQt[i * m + min(lane, m - 1)], lane_value(v, i), acc);
        if (lane < m) row[slot] = acc;
    }
    (void)mmax;
}

// Row transform: block (cluster list entry, 64 columns); the cluster's input rows
// are R[(rowlist[i] - base) * n + q].
__global__ __launch_bounds__(64) void k_rowtr(double *__restrict__ R, int64_t n, int64_t base,
                                              const int32_t *__restrict__ clist, const int32_t *__restrict__ nin,
                                              const int64_t *__restrict__ qoff, const double *__restrict__ qmat,
                                              const int64_t *__restrict__ rloff, const int64_t *__restrict__ rlist,
                                              int mmax)
{
    extern __shared__ double tr_smem[];
    double *sQ = tr_smem, *sIn = tr_smem + mmax * mmax;
    const int c = clist[blockIdx.x];
    const int m = nin[c];
    const double *Q = qmat + qoff[c];
    for (int e = threadIdx.x; e < m * m; e += 64) sQ[e] = Q[e];
    const int64_t *rl = rlist + rloff[c];
    const int64_t q = (int64_t)blockIdx.y * 64 + threadIdx.x;
    __syncthreads();
    if (q >= n) return;
    for (int i = 0; i < m; ++i) sIn[i * 64 + threadIdx.x] = R[(rl[i] - base) * n + q];
    for (int k = 0; k < m; ++k) {
        double acc = 0.0;
        for (int i = 0; i < m; ++i) acc = fma(sQ[k * m + i], sIn[i * 64 + threadIdx.x], acc);
        R[(rl[k] - base) * n + q] = acc;
    }
}

// Inverse of the column transform for one tree level (levels run root first): the
// cluster's outputs, read at its slots, are mapped back by Q (Q is orthogonal and the
// forward step applies Q^T), writing input i to slot i.  Same layout as k_coltr: lane i
// forms input i from all outputs and Q kept in LDS.
__global__ __launch_bounds__(256) void k_coltr_t(double *__restrict__ W, int64_t rows, int64_t n,
                                                 const int32_t *__restrict__ clist, const int32_t *__restrict__ nin,
                                                 const int64_t *__restrict__ qoff, const double *__restrict__ qmat,
                                                 const int64_t *__restrict__ slotoff, const int64_t *__restrict__ slots,
                                                 int mmax)
{
    extern __shared__ double tr_smem[];
    double *sQ = tr_smem;                            // sQ[k * m + i] = Q[k * m + i]
    const int c = clist[blockIdx.x];
    const int m = nin[c];
    const double *Q = qmat + qoff[c];
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) sQ[e] = Q[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t slot = lane < m ? slots[slotoff[c] + lane] : 0;
    for (int rr = wave; rr < 64; rr += 4) {
        const int64_t r = (int64_t)blockIdx.y * 64 + rr;
        if (r >= rows) break;
        double *row = W + r * n;
        const double v = lane < m ? row[slot] : 0.0;
        double acc = 0.0;
        for (int k = 0; k < m; ++k) acc = fma(sQ[k * m + min(lane, m - 1)], lane_value(v, k), acc);
        if (lane < m) row[slot] = acc;
    }
    (void)mmax;
}

// Row-wise permutations of an r x n block: gather out[j][k] = in[j][idx[k]], scatter
// out[j][idx[k]] = in[j][k] (idx a permutation of 0 .. n-1).
__global__ void k_gather_rows(int64_t n, int64_t total, const int64_t *__restrict__ idx, const double *__restrict__ in,
                              double *__restrict__ out)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / n, k = e - j * n;
        out[e] = in[j * n + idx[k]];
    }
}

__global__ void k_scatter_rows(int64_t n, int64_t total, const int64_t *__restrict__ idx, const double *__restrict__ in,
                               double *__restrict__ out)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / n, k = e - j * n;
        out[j * n + idx[k]] = in[e];
    }
}

// Samplet rows of block rows -> tiles.  Element (i, j) of tile (r, c) is the value of
// basis row cstart[r] + i (output kb[r] + i of cluster r) at basis column cstart[c] + j.
__global__ void k_extract(double *__restrict__ vals, const double *__restrict__ R, int64_t n, int64_t base,
                          const int32_t *__restrict__ tlist, int64_t ntl, const int32_t *__restrict__ tile_row,
                          const int32_t *__restrict__ tile_col, const int64_t *__restrict__ tile_off,
                          const int32_t *__restrict__ nfun, const int64_t *__restrict__ cstart,
                          const int32_t *__restrict__ kb, const int64_t *__restrict__ rloff,
                          const int64_t *__restrict__ rlist, const int64_t *__restrict__ slot_of_basis,
                          const uint8_t *__restrict__ keep)
{
    for (int64_t w = blockIdx.x; w < ntl; w += gridDim.x) {
        const int t = tlist[w];
        const int r = tile_row[t], c = tile_col[t];
        const int nr = nfun[r], ncl = nfun[c];
        const int64_t off = tile_off[t];
        for (int e = threadIdx.x; e < nr * ncl; e += blockDim.x) {
            const int i = e % nr, j = e / nr;
            const int64_t row = rlist[rloff[r] + kb[r] + i] - base;
            const double v = R[row * n + slot_of_basis[cstart[c] + j]];
            vals[off + e] = (keep && !keep[off + e]) ? 0.0 : v;
        }
    }
}

template <typename T>
struct Dev {
    T *p = nullptr;
    ~Dev() { if (p) (void)hipFree(p); }
};

template <typename T>
int up(Dev<T> &d, const std::vector<T> &v, hipStream_t s)
{
    if (v.empty()) return SPM_OK;
    if (hipMalloc(&d.p, v.size() * sizeof(T)) != hipSuccess) { d.p = nullptr; return fail(SPM_ENOMEM, "spm_kernel_compress: device allocation"); }
    (void)s;
    SPM_HIP(hipMemcpy(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return SPM_OK;
}

double fact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

}  // namespace

extern "C" int spm_kernel_compress(spm_pattern p, spm_tree t, int32_t mp, double ell, double scale, int32_t deriv,
                                   double *vals, void *stream)
{
    if (!p || !t || !vals) return fail(SPM_EINVAL, "spm_kernel_compress: null pointer");
    SPM_NEED_DEVICE(p, "spm_kernel_compress");
    if (mp < 0 || mp > 3 || !(ell > 0.0)) return fail(SPM_EINVAL, "spm_kernel_compress: bad kernel parameters");
    if (p->n != t->n || p->nc != t->nc || p->cstart != t->cstart)
        return fail(SPM_EINVAL, "spm_kernel_compress: pattern was not built on this tree's clusters");
    const int nc = t->nc, d = t->d;
    const int64_t n = t->n;
    for (int c = 0; c < nc; ++c)
        if (t->nin[c] > kMaxIn) return fail(SPM_EUNSUPPORTED, "spm_kernel_compress: more than 64 inputs in one cluster");
    hipStream_t s = (hipStream_t)stream;

    KParams kp;
    kp.p = mp;
    for (int k = 0; k < 4; ++k) kp.c[k] = 0.0;
    for (int q = 0; q <= mp; ++q) {
        const int k = mp - q;
        kp.c[k] += fact(mp) / fact(2 * mp) * fact(mp + q) / (fact(q) * fact(mp - q)) * std::ldexp(1.0, k);
    }
    kp.sfac = std::sqrt(2.0 * mp + 1.0) / ell;
    kp.ell = ell;
    kp.scale = scale;
    kp.deriv = deriv ? 1 : 0;

    // ---- host plan
    std::vector<int32_t> kb(nc);
    for (int c = 0; c < nc; ++c) kb[c] = c == 0 ? 0 : t->nscal[c];
    std::vector<int64_t> sob(n);
    for (int c = 0; c < nc; ++c)
        for (int k = kb[c]; k < t->nin[c]; ++k) sob[t->cstart[c] + (k - kb[c])] = t->slots[t->slotoff[c] + k];
    const int depth = t->depth;
    std::vector<std::vector<int32_t>> bylevel(depth + 1);
    for (int c = 0; c < nc; ++c) bylevel[t->level[c]].push_back(c);

    // Panel level lp: the panel buffer holds the rows of the largest panel root, the
    // upper buffer the scaling rows of all panel roots, both n doubles wide.  Take the
    // level that needs the fewest rows in the two together, among the levels whose
    // panel fits the budget (the deepest level always qualifies as a fallback).
    const double budget = 16.0 * 1024 * 1024 * 1024;  // bytes of one panel
    int lp = depth;
    int64_t best = -1;
    for (int l = 0; l <= depth; ++l) {
        int64_t mx = 0, nup = 0;
        for (int c : bylevel[l]) { mx = std::max(mx, t->psize[c]); if (c != 0) nup += t->nscal[c]; }
        for (int k = 0; k < l; ++k)
            for (int c : bylevel[k])
                if (t->son0[c] < 0) { mx = std::max(mx, t->psize[c]); if (c != 0) nup += t->nscal[c]; }
        if ((double)mx * n * 8.0 > budget) continue;
        if (best < 0 || mx + nup < best) { best = mx + nup; lp = l; }
    }
    std::vector<int32_t> roots;                         // panel roots, in cluster order
    for (int c = 0; c < nc; ++c)
        if (t->level[c] == lp || (t->level[c] < lp && t->son0[c] < 0)) roots.push_back(c);
    int64_t maxrows = 0;
    for (int c : roots) maxrows = std::max(maxrows, t->psize[c]);

    // rows of U: panel roots get their scaling rows, upper clusters reuse their sons' rows in place
    std::vector<int64_t> urloff(nc + 1, 0), urows;
    std::vector<std::vector<int64_t>> ul(nc);
    int64_t nu = 0;
    for (int c : roots)
        if (c != 0) for (int k = 0; k < t->nscal[c]; ++k) ul[c].push_back(nu++);
    for (int l = lp - 1; l >= 0; --l)
        for (int c : bylevel[l]) {
            if (t->son0[c] < 0) continue;
            int a = t->son0[c], b = t->son1[c];
            ul[c].insert(ul[c].end(), ul[a].begin(), ul[a].begin() + t->nscal[a]);
            ul[c].insert(ul[c].end(), ul[b].begin(), ul[b].begin() + t->nscal[b]);
        }
    for (int c = 0; c < nc; ++c) { urloff[c + 1] = urloff[c] + (int64_t)ul[c].size(); urows.insert(urows.end(), ul[c].begin(), ul[c].end()); }
    // urloff indexes urows per cluster; make every cluster's list addressable (empty lists allowed)
    std::vector<int64_t> urloff_c(urloff.begin(), urloff.end() - 1);

    // ---- device copies
    Dev<double> dpts, dq, dW, dU;
    Dev<int32_t> dnin, dkb, dcl, dtl;
    Dev<int64_t> dqoff, dsloff, dslots, dsob, durloff, durows;
    int st;
    if ((st = up(dpts, t->pts, s)) || (st = up(dq, t->qmat, s)) || (st = up(dnin, t->nin, s)) ||
        (st = up(dkb, kb, s)) || (st = up(dqoff, t->qoff, s)) || (st = up(dsloff, t->slotoff, s)) ||
        (st = up(dslots, t->slots, s)) || (st = up(dsob, sob, s)) || (st = up(durloff, urloff_c, s)) ||
        (st = up(durows, urows, s)))
        return st;
    // cluster lists: all levels (column transform) + per panel subtree levels + upper levels, one flat array
    std::vector<int32_t> clist;
    std::vector<std::pair<int64_t, int64_t>> lvl_all(depth + 1);
    for (int l = depth; l >= 0; --l) {
        lvl_all[l] = {(int64_t)clist.size(), (int64_t)bylevel[l].size()};
        clist.insert(clist.end(), bylevel[l].begin(), bylevel[l].end());
    }
    struct Panel {
        int32_t root;
        std::vector<std::pair<int64_t, int64_t>> lv;   // per level, deepest first
        int64_t t0, nt;
    };
    std::vector<Panel> panels;
    std::vector<int32_t> tlist;
    for (int pr : roots) {
        Panel P;
        P.root = pr;
        std::vector<std::vector<int32_t>> sub(depth + 1);
        std::vector<int32_t> st2(1, pr);
        std::vector<int32_t> members;
        while (!st2.empty()) {
            int c = st2.back();
            st2.pop_back();
            sub[t->level[c]].push_back(c);
            members.push_back(c);
            if (t->son0[c] >= 0) { st2.push_back(t->son0[c]); st2.push_back(t->son1[c]); }
        }
        for (int l = depth; l >= 0; --l) {
            if (sub[l].empty()) continue;
            std::sort(sub[l].begin(), sub[l].end());
            P.lv.push_back({(int64_t)clist.size(), (int64_t)sub[l].size()});
            clist.insert(clist.end(), sub[l].begin(), sub[l].end());
        }
        std::sort(members.begin(), members.end());
        P.t0 = (int64_t)tlist.size();
        for (int c : members)
            for (int64_t tt = p->blk_rp[c]; tt < p->blk_rp[c + 1]; ++tt) tlist.push_back((int32_t)tt);
        P.nt = (int64_t)tlist.size() - P.t0;
        panels.push_back(std::move(P));
    }
    std::vector<std::pair<int64_t, int64_t>> lvl_up;
    std::vector<std::pair<int64_t, int64_t>> tl_up;
    for (int l = lp - 1; l >= 0; --l) {
        std::vector<int32_t> cs;
        for (int c : bylevel[l]) if (t->son0[c] >= 0) cs.push_back(c);
        if (cs.empty()) continue;
        lvl_up.push_back({(int64_t)clist.size(), (int64_t)cs.size()});
        clist.insert(clist.end(), cs.begin(), cs.end());
        int64_t t0 = (int64_t)tlist.size();
        for (int c : cs)
            for (int64_t tt = p->blk_rp[c]; tt < p->blk_rp[c + 1]; ++tt) tlist.push_back((int32_t)tt);
        tl_up.push_back({t0, (int64_t)tlist.size() - t0});
    }
    if ((st = up(dcl, clist, s)) || (st = up(dtl, tlist, s))) return st;
    if (hipMalloc(&dW.p, (size_t)maxrows * n * sizeof(double)) != hipSuccess) { dW.p = nullptr; return fail(SPM_ENOMEM, "spm_kernel_compress: panel buffer"); }
    if (nu > 0 && hipMalloc(&dU.p, (size_t)nu * n * sizeof(double)) != hipSuccess) { dU.p = nullptr; return fail(SPM_ENOMEM, "spm_kernel_compress: upper buffer"); }

    // largest number of inputs in a range of the cluster list (sizes the transforms' LDS)
    auto mmax_of = [&](int64_t o, int64_t cnt) {
        int mx = 1;
        for (int64_t i = o; i < o + cnt; ++i) mx = std::max(mx, t->nin[clist[i]]);
        return mx;
    };
    auto coltr = [&](int64_t rows) -> int {
        for (int l = depth; l >= 0; --l) {
            auto [o, cnt] = lvl_all[l];
            if (cnt == 0) continue;
            dim3 g((unsigned)cnt, (unsigned)((rows + 63) / 64));
            const int mx = mmax_of(o, cnt);
            hipLaunchKernelGGL(k_coltr, g, dim3(256), (size_t)mx * mx * sizeof(double), s, dW.p, rows, n, dcl.p + o,
                               dnin.p, dqoff.p, dq.p, dsloff.p, dslots.p, mx);
        }
        SPM_HIP(hipGetLastError());
        return SPM_OK;
    };
    auto extract = [&](double *R, int64_t base, int64_t t0, int64_t nt, const int64_t *rloff, const int64_t *rl) -> int {
        if (nt == 0) return SPM_OK;
        unsigned g = (unsigned)std::min<int64_t>(nt, 1 << 20);
        hipLaunchKernelGGL(k_extract, dim3(g), dim3(64), 0, s, vals, R, n, base, dtl.p + t0, nt, p->d_tile_row.ptr,
                           p->d_tile_col.ptr, p->d_tile_off.ptr, p->d_nfun.ptr, p->d_cstart.ptr, dkb.p, rloff, rl,
                           dsob.p, p->d_keep.ptr);
        SPM_HIP(hipGetLastError());
        return SPM_OK;
    };

    // progress on stderr (SPM_PROGRESS set): the construction is O(n^2) and runs for
    // minutes at a million points
    const bool progress = std::getenv("SPM_PROGRESS") != nullptr;
    const size_t tick = std::max<size_t>(1, panels.size() / 10);
    size_t done = 0;
    for (const Panel &P : panels) {
        if (progress && done > 0 && done % tick == 0) {
            SPM_HIP(hipStreamSynchronize(s));
            std::fprintf(stderr, "[spm] kernel_compress: %zu of %zu panels\n", done, panels.size());
        }
        ++done;
        const int64_t p0 = t->pstart[P.root], rows = t->psize[P.root];
        const int64_t total = rows * n;
        hipLaunchKernelGGL(k_eval, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20)), dim3(256), 0, s,
                           dW.p, dpts.p, d, p0, rows, n, kp);
        SPM_HIP(hipGetLastError());
        if ((st = coltr(rows))) return st;
        for (auto [o, cnt] : P.lv) {
            dim3 g((unsigned)cnt, (unsigned)((n + 63) / 64));
            const int mx = mmax_of(o, cnt);
            hipLaunchKernelGGL(k_rowtr, g, dim3(64), tr_lds_bytes(mx), s, dW.p, n, p0, dcl.p + o, dnin.p, dqoff.p, dq.p,
                               dsloff.p, dslots.p, mx);
        }
        SPM_HIP(hipGetLastError());
        if ((st = extract(dW.p, p0, P.t0, P.nt, dsloff.p, dslots.p))) return st;
        if (P.root != 0) {
            const int64_t *sl = t->slots.data() + t->slotoff[P.root];
            for (int k = 0; k < t->nscal[P.root]; ++k)
                SPM_HIP(hipMemcpyAsync(dU.p + ul[P.root][k] * n, dW.p + (sl[k] - p0) * n, n * sizeof(double),
                                       hipMemcpyDeviceToDevice, s));
        }
    }
    for (size_t i = 0; i < lvl_up.size(); ++i) {
        auto [o, cnt] = lvl_up[i];
        dim3 g((unsigned)cnt, (unsigned)((n + 63) / 64));
        const int mx = mmax_of(o, cnt);
        hipLaunchKernelGGL(k_rowtr, g, dim3(64), tr_lds_bytes(mx), s, dU.p, n, (int64_t)0, dcl.p + o, dnin.p, dqoff.p,
                           dq.p, durloff.p, durows.p, mx);
        SPM_HIP(hipGetLastError());
        if ((st = extract(dU.p, 0, tl_up[i].first, tl_up[i].second, durloff.p, durows.p))) return st;
    }
    SPM_HIP(hipStreamSynchronize(s));
    return SPM_OK;
}

// The tree's transform tables on the device, uploaded once (synchronous copies).
static int tree_tables(spm_tree t, spm::TreeDevice **out)
{
    spm::TreeDevice &D = *t->dev;
    std::lock_guard<std::mutex> lock(D.mu);
    if (!D.ready) {
        D.release();
        const int nc = t->nc, depth = t->depth;
        const int64_t n = t->n;
        std::vector<int32_t> kb(nc);
        for (int c = 0; c < nc; ++c) kb[c] = c == 0 ? 0 : t->nscal[c];
        std::vector<int64_t> sob(n);                   // basis index -> slot of its coefficient
        for (int c = 0; c < nc; ++c)
            for (int k = kb[c]; k < t->nin[c]; ++k) sob[t->cstart[c] + (k - kb[c])] = t->slots[t->slotoff[c] + k];
        std::vector<std::vector<int32_t>> bylevel(depth + 1);
        for (int c = 0; c < nc; ++c) bylevel[t->level[c]].push_back(c);
        std::vector<int32_t> clist;
        D.lvl.assign(depth + 1, {0, 0});
        D.lvl_mmax.assign(depth + 1, 1);
        for (int l = 0; l <= depth; ++l) {
            D.lvl[l] = {(int64_t)clist.size(), (int64_t)bylevel[l].size()};
            clist.insert(clist.end(), bylevel[l].begin(), bylevel[l].end());
            for (int c : bylevel[l]) D.lvl_mmax[l] = std::max(D.lvl_mmax[l], t->nin[c]);
        }
        auto put = [](auto *&dst, const auto &v) -> int {
            using T = typename std::decay_t<decltype(v)>::value_type;
            if (v.empty()) return SPM_OK;
            if (hipMalloc((void **)&dst, v.size() * sizeof(T)) != hipSuccess) {
                dst = nullptr;
                return fail(SPM_ENOMEM, "spm_fst: device tables");
            }
            SPM_HIP(hipMemcpy(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
            return SPM_OK;
        };
        int st;
        if ((st = put(D.q, t->qmat)) || (st = put(D.nin, t->nin)) || (st = put(D.qoff, t->qoff)) ||
            (st = put(D.sloff, t->slotoff)) || (st = put(D.slots, t->slots)) || (st = put(D.sob, sob)) ||
            (st = put(D.perm, t->perm)) || (st = put(D.clist, clist))) {
            D.release();
            return st;
        }
        D.ready = true;
    }
    *out = &D;
    return SPM_OK;
}

// Fast samplet transform of r vectors (Section 3.2): Y = T X with X in the points'
// original order and Y in basis order, or the inverse X = T^T Y.  The two-scale
// transform is applied level by level in place on a tree-ordered copy, as in the
// column transform of the compression above.
extern "C" int spm_fst(spm_tree t, const double *X, int32_t r, double *Y, int32_t inverse, void *stream)
{
    if (!t) return fail(SPM_EINVAL, "spm_fst: null tree");
    if (r < 0) return fail(SPM_EINVAL, "spm_fst: negative vector count");
    const int64_t n = t->n, total = (int64_t)r * n;
    if (r == 0 || n == 0) return SPM_OK;                     // X and Y may then be null
    if (!X || !Y) return fail(SPM_EINVAL, "spm_fst: null pointer");
    {
        const char *x0 = reinterpret_cast<const char *>(X), *y0 = reinterpret_cast<const char *>(Y);
        const size_t b = (size_t)total * sizeof(double);
        if (x0 < y0 + b && y0 < x0 + b) return fail(SPM_EINVAL, "spm_fst: X and Y overlap");
    }
    const int nc = t->nc, depth = t->depth;
    for (int c = 0; c < nc; ++c)
        if (t->nin[c] > kMaxIn) return fail(SPM_EUNSUPPORTED, "spm_fst: more than 64 inputs in one cluster");
    hipStream_t s = (hipStream_t)stream;
    spm::TreeDevice *D;
    int st;
    if ((st = tree_tables(t, &D))) return st;
    double *W = nullptr;                               // tree-ordered work copy, stream-ordered
    if (hipMallocAsync((void **)&W, (size_t)total * sizeof(double), s) != hipSuccess)
        return fail(SPM_ENOMEM, "spm_fst: work buffer");
    const unsigned g1 = (unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20);
    auto level = [&](int l, bool tr) {
        auto [o, cnt] = D->lvl[l];
        if (cnt == 0) return;
        dim3 g((unsigned)cnt, (unsigned)((r + 63) / 64));
        const int mx = D->lvl_mmax[l];
        if (tr)
            hipLaunchKernelGGL(k_coltr_t, g, dim3(256), (size_t)mx * mx * sizeof(double), s, W, (int64_t)r, n,
                               D->clist + o, D->nin, D->qoff, D->q, D->sloff, D->slots, mx);
        else
            hipLaunchKernelGGL(k_coltr, g, dim3(256), (size_t)mx * mx * sizeof(double), s, W, (int64_t)r, n,
                               D->clist + o, D->nin, D->qoff, D->q, D->sloff, D->slots, mx);
    };
    if (!inverse) {
        hipLaunchKernelGGL(k_gather_rows, dim3(g1), dim3(256), 0, s, n, total, D->perm, X, W);   // tree order
        for (int l = depth; l >= 0; --l) level(l, false);
        hipLaunchKernelGGL(k_gather_rows, dim3(g1), dim3(256), 0, s, n, total, D->sob, W, Y);    // basis order
    } else {
        hipLaunchKernelGGL(k_scatter_rows, dim3(g1), dim3(256), 0, s, n, total, D->sob, X, W);
        for (int l = 0; l <= depth; ++l) level(l, true);
        hipLaunchKernelGGL(k_scatter_rows, dim3(g1), dim3(256), 0, s, n, total, D->perm, W, Y);   // original order
    }
    const hipError_t e = hipGetLastError();
    (void)hipFreeAsync(W, s);
    if (e != hipSuccess) return fail(SPM_EHIP, std::string("spm_fst: launch failed: ") + hipGetErrorString(e));
    return SPM_OK;
}
