// Host side of libspm: cluster tree, samplet two-scale transforms, eta-admissibility
// block pattern, pattern validation and the tiled layout.
//
// Built with -ffp-contract=off: the admissibility test and the tree split compare
// floating-point values, and every operation there rounds on its own.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>

#include "spm_internal.h"

namespace spm {

static thread_local std::string g_last_error;

int fail(int status, const std::string &msg)
{
    g_last_error = msg;
    return status;
}

}  // namespace spm

using spm::fail;

extern "C" const char *spm_status_string(int s)
{
    switch (s) {
    case SPM_OK: return "ok";
    case SPM_EINVAL: return "invalid argument";
    case SPM_EPATTERN: return "invalid pattern";
    case SPM_ENOMEM: return "out of memory";
    case SPM_EHIP: return "HIP error";
    case SPM_ENOTCONV: return "not converged";
    case SPM_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

extern "C" const char *spm_last_error(void) { return spm::g_last_error.c_str(); }

// ----------------------------------------------------------------------------------
// Cluster tree and samplets (Section 3.2)
// ----------------------------------------------------------------------------------
namespace {

// Exponents of all monomials of total degree <= q in d variables: degree by degree,
// inside a degree in descending lexicographic order of the exponent tuple.
std::vector<std::vector<int>> monomials(int d, int q)
{
    std::vector<std::vector<int>> out;
    for (int deg = 0; deg <= q; ++deg) {
        std::vector<std::vector<int>> same;
        std::vector<int> e(d, 0);
        // enumerate all tuples with entries 0..deg, keep those summing to deg
        int total = 1;
        for (int a = 0; a < d; ++a) total *= (deg + 1);
        for (int code = 0; code < total; ++code) {
            int c = code, s = 0;
            for (int a = d - 1; a >= 0; --a) { e[a] = c % (deg + 1); c /= (deg + 1); s += e[a]; }
            if (s == deg) same.push_back(e);
        }
        std::sort(same.begin(), same.end(), std::greater<std::vector<int>>());
        out.insert(out.end(), same.begin(), same.end());
    }
    return out;
}

// In-place Householder QR of the column-major (n x m) matrix r, n > m; q (n x n,
// column-major) receives H_1 ... H_m.  Reflector of column k maps x = r[k:, k] to
// alpha e_1 with alpha = -sign(x_0) ||x|| (sign(0) = +1); zero columns are skipped.
void householder(int n, int m, double *r, double *q)
{
    std::fill(q, q + (size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) q[(size_t)i * n + i] = 1.0;
    std::vector<double> v(n);
    for (int k = 0; k < m; ++k) {
        double *x = r + (size_t)k * n;
        double ss = 0.0;
        for (int i = k; i < n; ++i) ss += x[i] * x[i];
        double nrm = std::sqrt(ss);
        if (nrm == 0.0) continue;
        double alpha = x[k] >= 0.0 ? -nrm : nrm;
        for (int i = k; i < n; ++i) v[i] = x[i];
        v[k] -= alpha;
        double vv = 0.0;
        for (int i = k; i < n; ++i) vv += v[i] * v[i];
        double beta = 2.0 / vv;
        for (int j = k; j < m; ++j) {             // R <- H R
            double *col = r + (size_t)j * n;
            double t = 0.0;
            for (int i = k; i < n; ++i) t += v[i] * col[i];
            t *= beta;
            for (int i = k; i < n; ++i) col[i] -= t * v[i];
        }
        for (int row = 0; row < n; ++row) {       // Q <- Q H
            double t = 0.0;
            for (int i = k; i < n; ++i) t += q[(size_t)i * n + row] * v[i];
            t *= beta;
            for (int i = k; i < n; ++i) q[(size_t)i * n + row] -= t * v[i];
        }
    }
}

}  // namespace

extern "C" int spm_tree_build(const double *points, int64_t n, int32_t d, int32_t leaf, int32_t q,
                              spm_tree *out)
{
    if (!points || !out) return fail(SPM_EINVAL, "spm_tree_build: null pointer");
    if (n < 1 || d < 1 || d > 3 || leaf < 1 || q < 0 || q > 8 || n > INT32_MAX)
        return fail(SPM_EINVAL, "spm_tree_build: bad size argument");
    *out = nullptr;
    spm_tree_s *t = new (std::nothrow) spm_tree_s;
    if (!t) return fail(SPM_ENOMEM, "spm_tree_build: host allocation");
    try {
        t->n = n; t->d = d; t->leaf = leaf; t->q = q;
        auto mons = monomials(d, q);
        const int m = (int)mons.size();
        t->m = m;
        std::vector<int64_t> perm(n);
        for (int64_t i = 0; i < n; ++i) perm[i] = i;
        auto X = [&](int64_t i, int a) { return points[i * d + a]; };

        // breadth-first splitting; clusters are appended level by level
        auto add = [&](int64_t s, int64_t sz, int lev, int par) {
            t->pstart.push_back(s); t->psize.push_back(sz); t->level.push_back(lev);
            t->parent.push_back(par); t->son0.push_back(-1); t->son1.push_back(-1);
            for (int a = 0; a < d; ++a) {
                double lo = X(perm[s], a), hi = lo;
                for (int64_t k = s + 1; k < s + sz; ++k) { lo = std::min(lo, X(perm[k], a)); hi = std::max(hi, X(perm[k], a)); }
                t->lo.push_back(lo); t->hi.push_back(hi);
            }
            return (int)t->pstart.size() - 1;
        };
        add(0, n, 0, -1);
        for (size_t c = 0; c < t->pstart.size(); ++c) {
            int64_t s = t->pstart[c], sz = t->psize[c];
            if (sz <= leaf) continue;
            int axis = 0;
            double best = t->hi[c * d] - t->lo[c * d];
            for (int a = 1; a < d; ++a) {
                double e = t->hi[c * d + a] - t->lo[c * d + a];
                if (e > best) { best = e; axis = a; }
            }
            std::sort(perm.begin() + s, perm.begin() + s + sz, [&](int64_t a, int64_t b) {
                double xa = X(a, axis), xb = X(b, axis);
                return xa < xb || (xa == xb && a < b);
            });
            int64_t h = sz / 2;
            int lev = t->level[c] + 1;
            int a0 = add(s, h, lev, (int)c);
            int a1 = add(s + h, sz - h, lev, (int)c);
            t->son0[c] = a0; t->son1[c] = a1;
        }
        const int nc = (int)t->pstart.size();
        t->nc = nc;
        t->depth = *std::max_element(t->level.begin(), t->level.end());
        t->perm = perm;
        t->pts.resize((size_t)n * d);
        for (int64_t k = 0; k < n; ++k)
            for (int a = 0; a < d; ++a) t->pts[k * d + a] = X(perm[k], a);

        // two-scale transforms, leaves first (sons are numbered after their father)
        t->nin.assign(nc, 0); t->nscal.assign(nc, 0);
        t->qoff.assign(nc + 1, 0); t->slotoff.assign(nc + 1, 0);
        std::vector<std::vector<double>> scal(nc);        // (size x nscal) column-major coefficients
        std::vector<std::vector<int64_t>> slots(nc);
        std::vector<std::vector<double>> qs(nc);
        for (int c = nc - 1; c >= 0; --c) {
            const int64_t s = t->pstart[c], sz = t->psize[c];
            std::vector<double> phi;      // (sz x nin) column-major
            std::vector<int64_t> sl;
            int nin;
            if (t->son0[c] < 0) {
                nin = (int)sz;
                phi.assign((size_t)sz * nin, 0.0);
                for (int k = 0; k < nin; ++k) { phi[(size_t)k * sz + k] = 1.0; sl.push_back(s + k); }
            } else {
                int a = t->son0[c], b = t->son1[c];
                int na = t->nscal[a], nb = t->nscal[b];
                int64_t sa = t->psize[a], sb = t->psize[b];
                nin = na + nb;
                phi.assign((size_t)sz * nin, 0.0);
                for (int k = 0; k < na; ++k)
                    std::memcpy(&phi[(size_t)k * sz], &scal[a][(size_t)k * sa], sa * sizeof(double));
                for (int k = 0; k < nb; ++k)
                    std::memcpy(&phi[(size_t)(na + k) * sz + sa], &scal[b][(size_t)k * sb], sb * sizeof(double));
                sl.insert(sl.end(), slots[a].begin(), slots[a].begin() + na);
                sl.insert(sl.end(), slots[b].begin(), slots[b].begin() + nb);
                std::vector<double>().swap(scal[a]);
                std::vector<double>().swap(scal[b]);
            }
            t->nin[c] = nin;
            std::vector<double> qm((size_t)nin * nin, 0.0);
            if (nin <= m) {
                for (int k = 0; k < nin; ++k) qm[(size_t)k * nin + k] = 1.0;
                t->nscal[c] = nin;
                scal[c] = phi;
            } else {
                // moment matrix transposed: mt[k][alpha] = sum_p phi_k(p) mono_alpha(p), (nin x m) column-major
                double ctr[3], half = 0.0;
                for (int a = 0; a < d; ++a) {
                    ctr[a] = 0.5 * (t->lo[c * d + a] + t->hi[c * d + a]);
                    half = std::max(half, 0.5 * (t->hi[c * d + a] - t->lo[c * d + a]));
                }
                if (half == 0.0) half = 1.0;
                std::vector<double> vmono((size_t)sz * m);
                for (int64_t p = 0; p < sz; ++p) {
                    double y[3];
                    for (int a = 0; a < d; ++a) y[a] = (t->pts[(s + p) * d + a] - ctr[a]) / half;
                    for (int al = 0; al < m; ++al) {
                        double v = 1.0;
                        for (int a = 0; a < d; ++a)
                            for (int e = 0; e < mons[al][a]; ++e) v *= y[a];
                        vmono[(size_t)al * sz + p] = v;
                    }
                }
                std::vector<double> mt((size_t)nin * m, 0.0);
                for (int al = 0; al < m; ++al)
                    for (int k = 0; k < nin; ++k) {
                        double acc = 0.0;
                        const double *f = &phi[(size_t)k * sz];
                        const double *v = &vmono[(size_t)al * sz];
                        for (int64_t p = 0; p < sz; ++p) acc += f[p] * v[p];
                        mt[(size_t)al * nin + k] = acc;
                    }
                householder(nin, m, mt.data(), qm.data());
                t->nscal[c] = m;
                scal[c].assign((size_t)sz * m, 0.0);           // phi Q[:, :m]
                for (int j = 0; j < m; ++j)
                    for (int k = 0; k < nin; ++k) {
                        double w = qm[(size_t)j * nin + k];
                        if (w == 0.0) continue;
                        const double *f = &phi[(size_t)k * sz];
                        double *o = &scal[c][(size_t)j * sz];
                        for (int64_t p = 0; p < sz; ++p) o[p] += w * f[p];
                    }
            }
            qs[c] = std::move(qm);
            slots[c] = std::move(sl);
        }
        // flatten transforms; basis ranges
        t->cstart.assign(nc + 1, 0);
        for (int c = 0; c < nc; ++c) {
            t->qoff[c + 1] = t->qoff[c] + (int64_t)t->nin[c] * t->nin[c];
            t->slotoff[c + 1] = t->slotoff[c] + t->nin[c];
            int64_t cnt = (c == 0) ? t->nin[0] : (t->nin[c] - t->nscal[c]);
            t->cstart[c + 1] = t->cstart[c] + cnt;
        }
        if (t->cstart[nc] != n) { delete t; return fail(SPM_EINVAL, "spm_tree_build: basis size mismatch"); }
        t->qmat.resize(t->qoff[nc]);
        t->slots.resize(t->slotoff[nc]);
        for (int c = 0; c < nc; ++c) {
            std::copy(qs[c].begin(), qs[c].end(), t->qmat.begin() + t->qoff[c]);
            std::copy(slots[c].begin(), slots[c].end(), t->slots.begin() + t->slotoff[c]);
            if (t->cstart[c + 1] - t->cstart[c] > spm::kMaxFun) {
                delete t;
                return fail(SPM_EUNSUPPORTED, "spm_tree_build: a cluster owns more than 32 basis functions");
            }
        }
    } catch (const std::bad_alloc &) {
        delete t;
        return fail(SPM_ENOMEM, "spm_tree_build: host allocation");
    }
    *out = t;
    return SPM_OK;
}

extern "C" int spm_tree_destroy(spm_tree t)
{
    delete t;
    return SPM_OK;
}

extern "C" int spm_tree_info(spm_tree t, int32_t *nc, int32_t *depth, int32_t *m)
{
    if (!t) return fail(SPM_EINVAL, "spm_tree_info: null tree");
    if (nc) *nc = t->nc;
    if (depth) *depth = t->depth;
    if (m) *m = t->m;
    return SPM_OK;
}

extern "C" int spm_tree_arrays(spm_tree t, int64_t *perm, int64_t *cstart, int32_t *level,
                               int64_t *pstart, int64_t *psize)
{
    if (!t) return fail(SPM_EINVAL, "spm_tree_arrays: null tree");
    if (perm) std::copy(t->perm.begin(), t->perm.end(), perm);
    if (cstart) std::copy(t->cstart.begin(), t->cstart.end(), cstart);
    if (level) std::copy(t->level.begin(), t->level.end(), level);
    if (pstart) std::copy(t->pstart.begin(), t->pstart.end(), pstart);
    if (psize) std::copy(t->psize.begin(), t->psize.end(), psize);
    return SPM_OK;
}

// ----------------------------------------------------------------------------------
// eta-admissibility (Section 3.3, eq. (cutoff)) by pruned descent of the tree:
// admissibility of (c, c') is inherited by the sons of c' (their boxes lie inside
// B_c', so the gap can only grow and the diameter only shrink).
// ----------------------------------------------------------------------------------
extern "C" int spm_tree_block_pattern(spm_tree t, double eta, int64_t *rp, int32_t *col, int64_t *nblocks)
{
    if (!t || !rp || !nblocks) return fail(SPM_EINVAL, "spm_tree_block_pattern: null pointer");
    if (!(eta > 0.0)) return fail(SPM_EINVAL, "spm_tree_block_pattern: eta must be positive");
    const int nc = t->nc, d = t->d;
    std::vector<double> diam(nc);
    for (int c = 0; c < nc; ++c) {
        double acc = 0.0;
        for (int a = 0; a < d; ++a) {
            double e = t->hi[c * d + a] - t->lo[c * d + a];
            acc = acc + e * e;
        }
        diam[c] = std::sqrt(acc);
    }
    auto keep = [&](int c, int c2) {
        double acc = 0.0;
        for (int a = 0; a < d; ++a) {
            double g = std::max(0.0, std::max(t->lo[c2 * d + a] - t->hi[c * d + a], t->lo[c * d + a] - t->hi[c2 * d + a]));
            acc = acc + g * g;
        }
        double dist = std::sqrt(acc);
        double bound = eta * std::max(diam[c], diam[c2]);
        return dist < bound;
    };
    std::vector<std::vector<int32_t>> rows(nc);
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nth; ++w)
        th.emplace_back([&, w]() {
            std::vector<int32_t> stack;
            for (int c = (int)w; c < nc; c += (int)nth) {
                auto &r = rows[c];
                stack.assign(1, 0);
                while (!stack.empty()) {
                    int c2 = stack.back();
                    stack.pop_back();
                    if (!keep(c, c2)) continue;
                    r.push_back(c2);
                    if (t->son0[c2] >= 0) { stack.push_back(t->son1[c2]); stack.push_back(t->son0[c2]); }
                }
                std::sort(r.begin(), r.end());
            }
        });
    for (auto &x : th) x.join();
    rp[0] = 0;
    for (int c = 0; c < nc; ++c) rp[c + 1] = rp[c] + (int64_t)rows[c].size();
    *nblocks = rp[nc];
    if (col)
        for (int c = 0; c < nc; ++c) std::copy(rows[c].begin(), rows[c].end(), col + rp[c]);
    return SPM_OK;
}

// ----------------------------------------------------------------------------------
// Pattern validation and tiled layout
// ----------------------------------------------------------------------------------
namespace {

int check_clusters(int64_t n, int32_t nc, const int64_t *cs)
{
    if (nc < 1) return fail(SPM_EPATTERN, "cluster count must be positive");
    if (cs[0] != 0 || cs[nc] != n) return fail(SPM_EPATTERN, "cluster ranges do not tile [0, n)");
    for (int32_t c = 0; c < nc; ++c) {
        if (cs[c + 1] < cs[c]) return fail(SPM_EPATTERN, "cluster ranges decrease");
        if (cs[c + 1] - cs[c] > spm::kMaxFun)
            return fail(SPM_EUNSUPPORTED, "a cluster owns more than 32 basis functions");
    }
    return SPM_OK;
}

// Sorted unique columns per row, all in [0, ncols).
int check_csr(int64_t nrows, int64_t ncols, const int64_t *rp, const int32_t *col, const char *what)
{
    if (rp[0] != 0) return fail(SPM_EPATTERN, std::string(what) + ": row_ptr[0] != 0");
    for (int64_t i = 0; i < nrows; ++i) {
        if (rp[i + 1] < rp[i]) return fail(SPM_EPATTERN, std::string(what) + ": row_ptr decreases");
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (col[e] < 0 || col[e] >= ncols) return fail(SPM_EPATTERN, std::string(what) + ": column out of range");
            if (e > rp[i] && col[e] <= col[e - 1])
                return fail(SPM_EPATTERN, std::string(what) + ": columns not sorted and unique");
        }
    }
    return SPM_OK;
}

bool has(const int64_t *rp, const int32_t *col, int64_t i, int32_t j)
{
    return std::binary_search(col + rp[i], col + rp[i + 1], j);
}

int check_symmetric_diag(int64_t nrows, const int64_t *rp, const int32_t *col, const std::vector<int32_t> *need_diag,
                         const char *what)
{
    for (int64_t i = 0; i < nrows; ++i) {
        bool want = need_diag ? (*need_diag)[i] > 0 : true;
        if (want && !has(rp, col, i, (int32_t)i)) return fail(SPM_EPATTERN, std::string(what) + ": diagonal entry missing");
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (!has(rp, col, col[e], (int32_t)i)) return fail(SPM_EPATTERN, std::string(what) + ": pattern not symmetric");
    }
    return SPM_OK;
}

inline int ceil4(int x) { return (x + 3) & ~3; }

// Grouped schedule of the FP64 product.  Consecutive clusters of equal size form
// groups of up to 4 (at most 128 rows); with clusters numbered level by level these
// are neighbours in the tree.  A unit is a pair of groups (G_r, G_c) holding at
// least one output tile; it sums over the clusters mu in U(G_r) cap U(G_c), where
// U(G) is the union of the members' block rows.
void build_groups(spm_pattern_s *p)
{
    const int nc = p->nc;
    std::vector<int32_t> gid(nc, -1);
    p->grp_mem.clear(); p->grp_s.clear(); p->grp_g.clear(); p->grp_R.clear();
    p->kmax = 4;
    for (int c = 0; c < nc; ++c) p->kmax = std::max(p->kmax, ceil4(p->nfun[c]));
    int c = 0;
    while (c < nc) {
        if (p->nfun[c] == 0) { ++c; continue; }
        const int s = ceil4(p->nfun[c]);
        // slots of up to 16 functions fill one 16-row block (four of 4, two of 8, one
        // of 12 or 16), so their units have a single 16-row side and run on the
        // register-direct kernel
        const int gmax = s <= 16 ? 16 / s : std::max(1, std::min(4, 128 / s));
        int k = 0;
        const int g = (int)p->grp_s.size();
        while (c < nc && k < gmax && ceil4(p->nfun[c]) == s && p->nfun[c] > 0) {
            p->grp_mem.push_back(c);
            gid[c] = g;
            ++k; ++c;
        }
        for (int r = k; r < 4; ++r) p->grp_mem.push_back(-1);
        p->grp_s.push_back(s);
        p->grp_g.push_back(k);
        p->grp_R.push_back(((k * s) + 15) / 16 * 16);
    }
    const int ng = (int)p->grp_s.size();
    p->ng = ng;
    p->all_even = true;
    p->all_mult4 = true;
    for (int q = 0; q < nc; ++q) {
        p->all_even = p->all_even && (p->nfun[q] % 2 == 0);
        p->all_mult4 = p->all_mult4 && (p->nfun[q] % 4 == 0);
    }
    // union lists
    p->gl_rp.assign(ng + 1, 0);
    p->gl_mu.clear(); p->gl_tile.clear();
    for (int g = 0; g < ng; ++g) {
        std::vector<std::pair<int32_t, int32_t>> ent;    // (mu, k * 2^28 + position) sorted by mu
        std::vector<int32_t> mus;
        for (int k = 0; k < p->grp_g[g]; ++k) {
            int r = p->grp_mem[g * 4 + k];
            for (int64_t t = p->blk_rp[r]; t < p->blk_rp[r + 1]; ++t) mus.push_back(p->tile_col[t]);
        }
        std::sort(mus.begin(), mus.end());
        mus.erase(std::unique(mus.begin(), mus.end()), mus.end());
        const size_t base = p->gl_mu.size();
        p->gl_mu.insert(p->gl_mu.end(), mus.begin(), mus.end());
        p->gl_tile.resize((base + mus.size()) * 4, -1);
        for (int k = 0; k < p->grp_g[g]; ++k) {
            int r = p->grp_mem[g * 4 + k];
            size_t e = 0;
            for (int64_t t = p->blk_rp[r]; t < p->blk_rp[r + 1]; ++t) {
                while (mus[e] != p->tile_col[t]) ++e;
                p->gl_tile[(base + e) * 4 + k] = (int32_t)t;
            }
        }
        p->gl_rp[g + 1] = (int64_t)p->gl_mu.size();
    }
    // units
    p->unit_gr.clear(); p->unit_gc.clear(); p->unit_out.clear();
    for (int g = 0; g < ng; ++g) {
        std::vector<int32_t> cg;
        for (int64_t e = p->gl_rp[g]; e < p->gl_rp[g + 1]; ++e) cg.push_back(gid[p->gl_mu[e]]);
        cg.erase(std::unique(cg.begin(), cg.end()), cg.end());   // entries sorted by cluster -> groups ascending
        for (int h : cg) {
            p->unit_gr.push_back(g);
            p->unit_gc.push_back(h);
            int32_t out[16];
            for (int q = 0; q < 16; ++q) out[q] = -1;
            const int32_t *b = p->gl_mu.data() + p->gl_rp[g], *e = p->gl_mu.data() + p->gl_rp[g + 1];
            for (int kc = 0; kc < p->grp_g[h]; ++kc) {
                int32_t cc = p->grp_mem[h * 4 + kc];
                const int32_t *f = std::lower_bound(b, e, cc);
                if (f == e || *f != cc) continue;
                int64_t ent = f - p->gl_mu.data();
                for (int kr = 0; kr < p->grp_g[g]; ++kr) out[kr * 4 + kc] = p->gl_tile[ent * 4 + kr];
            }
            p->unit_out.insert(p->unit_out.end(), out, out + 16);
        }
    }
    const int64_t nu = (int64_t)p->unit_gr.size();
    // middle clusters of each unit (merge of the two union lists) and its cost:
    // rows x cols x padded k
    std::vector<double> cost(nu, 0.0);
    std::vector<int64_t> cnt(nu, 0);
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto merge = [&](int64_t u, int32_t *pa, int32_t *pb) {
        int g = p->unit_gr[u], h = p->unit_gc[u];
        const int64_t a0 = p->gl_rp[g], a1 = p->gl_rp[g + 1], b0 = p->gl_rp[h], b1 = p->gl_rp[h + 1];
        int64_t a = a0, b = b0, k = 0, np = 0;
        while (a < a1 && b < b1) {
            const int32_t x = p->gl_mu[a], y = p->gl_mu[b];
            if (x < y) ++a;
            else if (y < x) ++b;
            else {
                if (pa) { pa[np] = (int32_t)a; pb[np] = (int32_t)b; }
                ++np;
                k += p->nfun[x];
                ++a; ++b;
            }
        }
        cnt[u] = np;
        cost[u] = (double)p->grp_R[g] * p->grp_R[h] * (double)k;
    };
    {
        std::vector<std::thread> th;
        for (unsigned w = 0; w < nth; ++w)
            th.emplace_back([&, w]() { for (int64_t u = w; u < nu; u += nth) merge(u, nullptr, nullptr); });
        for (auto &x : th) x.join();
    }
    p->pair_off.assign(nu + 1, 0);
    for (int64_t u = 0; u < nu; ++u) p->pair_off[u + 1] = p->pair_off[u] + cnt[u];
    p->pair_a.resize(p->pair_off[nu]);
    p->pair_b.resize(p->pair_off[nu]);
    p->pair_a_lv.assign(!p->clevel.empty() ? p->pair_off[nu] : 0, 0);
    p->pair_b_lv.assign(!p->clevel.empty() ? p->pair_off[nu] : 0, 0);
    // Order of a unit's middle clusters (the sum over mu may run in any order).  Both
    // kernels skip work per stage: the register-direct one a 16-column (or 16-row) block
    // of the wide side none of whose members has a tile in the stage, the staged one a
    // 16 x 16 block whose row or column members have none.  So the clusters are first
    // grouped by the sets of wide-side members with a tile (fewer stages in which a
    // block has work).  Inside a group they go largest first, each stage topped up from
    // the small end while its 32 k rows and 8 clusters allow (a 28-function leaf shares
    // its stage with a 4-function cluster instead of leaving 4 rows empty).
    struct Item { int32_t key, size, level; int64_t q; };
    const bool lev = !p->clevel.empty();
    // by_level: inside a key group, level by level (finest first), topped up within a level
    auto reorder = [&](int64_t u, int32_t *pa, int32_t *pb, int64_t np, std::vector<Item> &it,
                       std::vector<int32_t> &tmp, bool by_level) {
        if (np < 2) return;
        const bool wide_c = p->grp_R[p->unit_gc[u]] > 16, wide_r = p->grp_R[p->unit_gr[u]] > 16;
        it.resize(np);
        for (int64_t q = 0; q < np; ++q) {
            int32_t key = 0;   // row members with a tile in bits 4..7, column members in bits 0..3
            for (int k = 0; k < 4; ++k) {
                if (wide_r) key |= (p->gl_tile[(int64_t)pa[q] * 4 + k] >= 0 ? 1 : 0) << (4 + k);
                if (wide_c) key |= (p->gl_tile[(int64_t)pb[q] * 4 + k] >= 0 ? 1 : 0) << k;
            }
            const int32_t mu = p->gl_mu[pa[q]];
            it[q] = {key, p->nfun[mu], by_level ? p->clevel[mu] : 0, q};
        }
        std::stable_sort(it.begin(), it.end(), [](const Item &x, const Item &y) {
            if (x.key != y.key) return x.key < y.key;
            if (x.level != y.level) return x.level > y.level;
            return x.size > y.size;
        });
        tmp.clear();
        for (int64_t g0 = 0; g0 < np;) {
            int64_t g1 = g0;
            while (g1 < np && it[g1].key == it[g0].key && it[g1].level == it[g0].level) ++g1;
            int64_t i = g0, j = g1 - 1;
            while (i <= j) {
                int kacc = it[i].size, n = 1;
                tmp.push_back((int32_t)it[i++].q);
                while (i <= j && n < 8 && kacc + it[j].size <= 32) {
                    kacc += it[j].size;
                    ++n;
                    tmp.push_back((int32_t)it[j--].q);
                }
            }
            g0 = g1;
        }
        std::vector<int32_t> na(np), nb(np);
        for (int64_t q = 0; q < np; ++q) { na[q] = pa[tmp[q]]; nb[q] = pb[tmp[q]]; }
        std::copy(na.begin(), na.end(), pa);
        std::copy(nb.begin(), nb.end(), pb);
    };
    {
        std::vector<std::thread> th;
        for (unsigned w = 0; w < nth; ++w)
            th.emplace_back([&, w]() {
                std::vector<Item> it;
                std::vector<int32_t> tmp;
                for (int64_t u = w; u < nu; u += nth) {
                    int32_t *pa = p->pair_a.data() + p->pair_off[u], *pb = p->pair_b.data() + p->pair_off[u];
                    merge(u, pa, pb);
                    if (lev) {
                        int32_t *qa = p->pair_a_lv.data() + p->pair_off[u], *qb = p->pair_b_lv.data() + p->pair_off[u];
                        std::copy(pa, pa + cnt[u], qa);
                        std::copy(pb, pb + cnt[u], qb);
                        reorder(u, qa, qb, cnt[u], it, tmp, true);
                    }
                    reorder(u, pa, pb, cnt[u], it, tmp, false);
                }
            });
        for (auto &x : th) x.join();
    }
    p->padded_macs = 0.0;
    for (double x : cost) p->padded_macs += x;
    // per union entry: cluster size and the element offsets of the member tiles
    const int64_t ne = (int64_t)p->gl_mu.size();
    p->gl_nm.resize(ne);
    p->gl_offd.assign(ne * 4 + 4, -1);   // padded: 16-byte reads of the last entry stay in bounds
    if (lev) {
        p->gl_nml.resize(ne);
        p->gl_offT.assign(ne * 4 + 4, -1);
    }
    for (int64_t e = 0; e < ne; ++e) {
        p->gl_nm[e] = p->nfun[p->gl_mu[e]];
        if (lev) p->gl_nml[e] = p->gl_nm[e] | p->clevel[p->gl_mu[e]] << 8;
        for (int k = 0; k < 4; ++k) {
            const int32_t t = p->gl_tile[e * 4 + k];
            if (t >= 0) p->gl_offd[e * 4 + k] = p->tile_off[t];
            if (t >= 0 && lev) p->gl_offT[e * 4 + k] = p->tile_off[p->trans[t]];
        }
    }
    // stages: consecutive middle clusters of a unit packed while their sizes sum to at most
    // 32 k rows (a cluster may start at any row; only the stage's last k step is padded).
    // With levels a second list of stages (by_level) holds clusters of one level each, for
    // the split-precision product; the FP64 and FP32 stages may span two levels.
    std::vector<int64_t> nst(nu, 0);
    auto pack_list = [&](int64_t u, int32_t *out, bool by_level) {
        int64_t ns = 0;
        int kacc = 0, np = 0;
        const int64_t f0 = p->pair_off[u], f1 = p->pair_off[u + 1];
        int lv = -1;
        const int32_t *pa = by_level ? p->pair_a_lv.data() : p->pair_a.data();
        for (int64_t f = f0; f < f1; ++f) {
            const int km = p->gl_nm[pa[f]];
            const int lf = by_level ? p->clevel[p->gl_mu[pa[f]]] : 0;
            if (np == 0 || kacc + km > 32 || np == 8 || lf != lv) {
                lv = lf;
                if (out) out[ns] = (int32_t)(f - f0);
                ++ns;
                kacc = 0;
                np = 0;
            }
            kacc += km;
            ++np;
        }
        // a stage count that is a multiple of the kernels' loop trip (two stages for the
        // FP64 and FP32 kernels, two or three for the split-precision ones), so that the
        // loops have a single exit; the extra stages are empty (they start at the end of the
        // list)
        const int mult = by_level ? 6 : 2;
        while (ns % mult) {
            if (out) out[ns] = (int32_t)(f1 - f0);
            ++ns;
        }
        nst[u] = ns;
    };
    auto pack_all = [&](bool by_level, std::vector<int64_t> &off, std::vector<int32_t> &first) {
        {
            std::vector<std::thread> th;
            for (unsigned w = 0; w < nth; ++w)
                th.emplace_back([&, w]() { for (int64_t u = w; u < nu; u += nth) pack_list(u, nullptr, by_level); });
            for (auto &x : th) x.join();
        }
        off.assign(nu + 1, 0);
        for (int64_t u = 0; u < nu; ++u) off[u + 1] = off[u] + nst[u];
        first.resize(off[nu]);
        std::vector<std::thread> th;
        for (unsigned w = 0; w < nth; ++w)
            th.emplace_back([&, w]() {
                for (int64_t u = w; u < nu; u += nth) pack_list(u, first.data() + off[u], by_level);
            });
        for (auto &x : th) x.join();
    };
    pack_all(false, p->stage_off, p->stage_first);
    if (lev) pack_all(true, p->stage_off_lv, p->stage_first_lv);
    else {
        p->stage_off_lv.clear();
        p->stage_first_lv.clear();
    }
    // Launch classes by (row blocks, column blocks).  Inside a class the units are cut
    // into strips that share one operand group: the column group when the columns are
    // the wider side, else the row group.  A strip's units run back to back on one XCD,
    // so the shared panel is re-read from that XCD's L2 instead of HBM.  Strips go to
    // the XCD with the least work so far, heaviest first, and inside a strip the
    // heaviest units start first.  Workgroups are dispatched to the 8 XCDs round robin,
    // so the launch order interleaves the eight per-XCD lists.
    auto key = [&](int64_t u) { return p->grp_R[p->unit_gr[u]] / 16 * 16 + p->grp_R[p->unit_gc[u]] / 16; };
    std::vector<int64_t> idx(nu);
    for (int64_t u = 0; u < nu; ++u) idx[u] = u;
    std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
        const int kx = key(x), ky = key(y);
        return kx != ky ? kx < ky : x < y;
    });
    {
        std::vector<int64_t> out;
        out.reserve(nu);
        int64_t c0 = 0;
        while (c0 < nu) {
            int64_t c1 = c0;
            while (c1 < nu && key(idx[c1]) == key(idx[c0])) ++c1;
            const int k = key(idx[c0]);
            const int rb = k / 16, cb = k % 16;
            // strips of the class
            std::vector<std::pair<int64_t, int64_t>> bu;   // (strip key, unit)
            bu.reserve(c1 - c0);
            for (int64_t i = c0; i < c1; ++i) {
                const int64_t u = idx[i];
                bu.push_back({cb > rb ? p->unit_gc[u] : p->unit_gr[u], u});
            }
            std::sort(bu.begin(), bu.end(), [&](const std::pair<int64_t, int64_t> &x, const std::pair<int64_t, int64_t> &y) {
                if (x.first != y.first) return x.first < y.first;
                if (cost[x.second] != cost[y.second]) return cost[x.second] > cost[y.second];
                return x.second < y.second;
            });
            struct Blk { int64_t b0, b1; double w; };
            std::vector<Blk> blks;
            for (int64_t i = 0; i < (int64_t)bu.size();) {
                int64_t j = i;
                double w = 0.0;
                while (j < (int64_t)bu.size() && bu[j].first == bu[i].first) w += cost[bu[j++].second];
                blks.push_back({i, j, w});
                i = j;
            }
            std::stable_sort(blks.begin(), blks.end(), [](const Blk &x, const Blk &y) { return x.w > y.w; });
            std::vector<std::vector<int64_t>> lists(8);
            double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (const auto &B : blks) {
                int x = 0;
                for (int y = 1; y < 8; ++y)
                    if (load[y] < load[x]) x = y;
                load[x] += B.w;
                for (int64_t i = B.b0; i < B.b1; ++i) lists[x].push_back(bu[i].second);
            }
            std::vector<size_t> pos(8, 0);
            for (int64_t n = c0; n < c1; ++n) {
                int x = (int)((n - c0) % 8);
                if (pos[x] >= lists[x].size()) {       // list exhausted: take from the longest remaining one
                    int best = 0;
                    for (int y = 1; y < 8; ++y)
                        if (lists[y].size() - pos[y] > lists[best].size() - pos[best]) best = y;
                    x = best;
                }
                out.push_back(lists[x][pos[x]++]);
            }
            c0 = c1;
        }
        idx.swap(out);
    }
    p->unit_order.resize(nu);
    p->launches.clear();
    for (int64_t i = 0; i < nu; ++i) {
        p->unit_order[i] = (int32_t)idx[i];
        int k = key(idx[i]);
        if (p->launches.empty() || key(p->unit_order[p->launches.back().first]) != k) {
            spm_pattern_s::Launch L;
            L.rb = k / 16;
            L.cb = k % 16;
            L.waves = L.rb * L.cb == 1 ? 1 : 4;
            L.first = i;
            L.count = 0;
            L.smax_r = 0;
            L.smax_c = 0;
            L.out_tiles = 0;
            L.exact_macs = 0.0;
            L.padded_macs = 0.0;
            p->launches.push_back(L);
        }
        auto &B = p->launches.back();
        const int64_t u = idx[i];
        B.count++;
        B.smax_r = std::max(B.smax_r, p->grp_s[p->unit_gr[u]]);
        B.smax_c = std::max(B.smax_c, p->grp_s[p->unit_gc[u]]);
        B.padded_macs += cost[u];
        for (int q = 0; q < 16; ++q) {
            const int32_t t = p->unit_out[u * 16 + q];
            if (t < 0) continue;
            B.out_tiles++;
            B.exact_macs += p->tile_macs[t];
        }
    }
}

// Fill the layout of p from its block CSR (p->blk_rp, p->tile_col, p->nfun set).
void build_layout(spm_pattern_s *p)
{
    const int nc = p->nc;
    const int64_t nt = p->blk_rp[nc];
    p->n_tiles = nt;
    p->tile_row.resize(nt);
    p->tile_off.resize(nt + 1);
    p->trans.resize(nt);
    p->colprefix.resize(nt);
    p->rowbase.resize(nc);
    p->rowlen.resize(nc);
    p->diag_tile.assign(nc, -1);
    p->tile_off[0] = 0;
    int64_t base = 0;
    p->max_rowlen = 0;
    for (int r = 0; r < nc; ++r) {
        int64_t len = 0;
        p->max_rowlen = std::max<int32_t>(p->max_rowlen, (int32_t)(p->blk_rp[r + 1] - p->blk_rp[r]));
        for (int64_t t = p->blk_rp[r]; t < p->blk_rp[r + 1]; ++t) {
            int c = p->tile_col[t];
            p->tile_row[t] = r;
            p->colprefix[t] = len;
            len += p->nfun[c];
            p->tile_off[t + 1] = p->tile_off[t] + (int64_t)p->nfun[r] * p->nfun[c];
            if (c == r) p->diag_tile[r] = (int32_t)t;
            const int32_t *b = p->tile_col.data() + p->blk_rp[c];
            const int32_t *e = p->tile_col.data() + p->blk_rp[c + 1];
            p->trans[t] = (int32_t)(p->blk_rp[c] + (std::lower_bound(b, e, r) - b));
        }
        p->rowlen[r] = len;
        p->rowbase[r] = base;
        base += len * p->nfun[r];
    }
    p->n_stored = p->tile_off[nt];
    p->diag_pos.clear();
    for (int r = 0; r < nc; ++r) {
        const int64_t t = p->diag_tile[r];
        if (t < 0) continue;
        for (int i = 0; i < p->nfun[r]; ++i) p->diag_pos.push_back(p->tile_off[t] + (int64_t)i * (p->nfun[r] + 1));
    }
    // pieces for the S x dense product
    p->pc_rp.assign(nc + 1, 0);
    p->pc_off.clear();
    p->pc_g.clear();
    p->pc_w.clear();
    for (int r = 0; r < nc; ++r) {
        const int nr = p->nfun[r];
        // whole 16-column chunks of at most kPieceEntries entries (at least one chunk)
        const int32_t wmax = nr > 0 ? std::max(16, spm::kPieceEntries / nr / 16 * 16) : 16;
        for (int64_t t = p->blk_rp[r]; t < p->blk_rp[r + 1];) {
            // extend the run while the next tile's columns follow on in the basis
            int64_t e = t + 1;
            while (e < p->blk_rp[r + 1] &&
                   p->cstart[p->tile_col[e]] == p->cstart[p->tile_col[e - 1]] + p->nfun[p->tile_col[e - 1]])
                ++e;
            const int64_t g0 = p->cstart[p->tile_col[t]];
            const int64_t w = p->cstart[p->tile_col[e - 1]] + p->nfun[p->tile_col[e - 1]] - g0;
            if (nr > 0)
                for (int64_t j = 0; j < w; j += wmax) {
                    p->pc_off.push_back(p->tile_off[t] + j * nr);
                    p->pc_g.push_back(g0 + j);
                    p->pc_w.push_back((int32_t)std::min<int64_t>(wmax, w - j));
                }
            t = e;
        }
        p->pc_rp[r + 1] = (int64_t)p->pc_w.size();
    }
    // exact multiply-adds of one product: merge of the two sorted block rows per tile
    std::vector<double> part(16, 0.0);
    p->tile_macs.assign(nt, 0.0);
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nth; ++w)
        th.emplace_back([&, w]() {
            double acc = 0.0;
            for (int64_t t = w; t < nt; t += nth) {
                int r = p->tile_row[t], c = p->tile_col[t];
                const int32_t *a = p->tile_col.data() + p->blk_rp[r], *ae = p->tile_col.data() + p->blk_rp[r + 1];
                const int32_t *b = p->tile_col.data() + p->blk_rp[c], *be = p->tile_col.data() + p->blk_rp[c + 1];
                int64_t k = 0;
                while (a < ae && b < be) {
                    if (*a < *b) ++a;
                    else if (*b < *a) ++b;
                    else { k += p->nfun[*a]; ++a; ++b; }
                }
                p->tile_macs[t] = (double)p->nfun[r] * p->nfun[c] * (double)k;
                acc += p->tile_macs[t];
            }
            part[w] = acc;
        });
    for (auto &x : th) x.join();
    p->macs = 0.0;
    for (unsigned w = 0; w < nth; ++w) p->macs += part[w];
    // schedule: tiles in storage order (one workgroup per output tile)
    p->order.resize(nt);
    for (int64_t t = 0; t < nt; ++t) p->order[t] = (int32_t)t;
    build_groups(p);
    std::vector<double>().swap(p->tile_macs);   // only the per-class sums are kept
}

}  // namespace

// Levels of the clusters (optional): every value in [0, 64).
static int check_levels(int32_t nc, const int32_t *lev)
{
    if (!lev) return SPM_OK;
    for (int32_t c = 0; c < nc; ++c)
        if (lev[c] < 0 || lev[c] >= 64) return fail(SPM_EINVAL, "cluster level out of [0, 64)");
    return SPM_OK;
}

static void set_levels(spm_pattern_s *p, const int32_t *lev)
{
    p->clevel.clear();
    p->nlev = 0;
    if (!lev) return;
    p->clevel.assign(lev, lev + p->nc);
    for (int32_t c = 0; c < p->nc; ++c) p->nlev = std::max(p->nlev, lev[c] + 1);
}

extern "C" int spm_block_pattern_plan(int64_t n, int32_t nc, const int64_t *cs, const int64_t *brp,
                                      const int32_t *bcol, const int32_t *lev, spm_pattern *out)
{
    if (!cs || !brp || !bcol || !out) return fail(SPM_EINVAL, "spm_block_pattern_plan: null pointer");
    if (n < 1 || n > INT32_MAX) return fail(SPM_EINVAL, "spm_block_pattern_plan: bad n");
    *out = nullptr;
    int st = check_clusters(n, nc, cs);
    if (st) return st;
    if ((st = check_csr(nc, nc, brp, bcol, "block pattern"))) return st;
    if ((st = check_levels(nc, lev))) return st;
    std::vector<int32_t> nf(nc);
    for (int c = 0; c < nc; ++c) nf[c] = (int32_t)(cs[c + 1] - cs[c]);
    if ((st = check_symmetric_diag(nc, brp, bcol, &nf, "block pattern"))) return st;
    if (brp[nc] > INT32_MAX) return fail(SPM_EUNSUPPORTED, "more than 2^31-1 tiles");
    spm_pattern_s *p = new (std::nothrow) spm_pattern_s;
    if (!p) return fail(SPM_ENOMEM, "host allocation");
    try {
        p->n = n; p->nc = nc;
        p->cstart.assign(cs, cs + nc + 1);
        p->nfun = nf;
        // drop tiles of clusters without basis functions
        p->blk_rp.assign(nc + 1, 0);
        for (int r = 0; r < nc; ++r) {
            if (nf[r] > 0)
                for (int64_t e = brp[r]; e < brp[r + 1]; ++e)
                    if (nf[bcol[e]] > 0) p->tile_col.push_back(bcol[e]);
            p->blk_rp[r + 1] = (int64_t)p->tile_col.size();
        }
        set_levels(p, lev);
        build_layout(p);
        p->nnz = p->n_stored;
        p->masked = false;
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(SPM_ENOMEM, "host allocation");
    }
    *out = p;
    return SPM_OK;
}

extern "C" int spm_compress_pattern_plan(int64_t n, const int64_t *rp, const int32_t *col, int32_t nc,
                                         const int64_t *cs, const int32_t *lev, spm_pattern *out)
{
    if (!rp || !col || !cs || !out) return fail(SPM_EINVAL, "spm_compress_pattern_plan: null pointer");
    if (n < 1 || n > INT32_MAX) return fail(SPM_EINVAL, "spm_compress_pattern_plan: bad n");
    *out = nullptr;
    int st = check_clusters(n, nc, cs);
    if (st) return st;
    if ((st = check_csr(n, n, rp, col, "pattern"))) return st;
    if ((st = check_symmetric_diag(n, rp, col, nullptr, "pattern"))) return st;
    if ((st = check_levels(nc, lev))) return st;
    spm_pattern_s *p = new (std::nothrow) spm_pattern_s;
    if (!p) return fail(SPM_ENOMEM, "host allocation");
    try {
        p->n = n; p->nc = nc;
        p->cstart.assign(cs, cs + nc + 1);
        p->nfun.resize(nc);
        for (int c = 0; c < nc; ++c) p->nfun[c] = (int32_t)(cs[c + 1] - cs[c]);
        std::vector<int32_t> clus(n);
        for (int c = 0; c < nc; ++c)
            for (int64_t i = cs[c]; i < cs[c + 1]; ++i) clus[i] = c;
        // tiles: cluster pairs holding at least one entry
        p->blk_rp.assign(nc + 1, 0);
        std::vector<int32_t> mark(nc, -1);
        for (int r = 0; r < nc; ++r) {
            std::vector<int32_t> cols;
            for (int64_t i = cs[r]; i < cs[r + 1]; ++i)
                for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                    int c = clus[col[e]];
                    if (mark[c] != r) { mark[c] = r; cols.push_back(c); }
                }
            std::sort(cols.begin(), cols.end());
            p->tile_col.insert(p->tile_col.end(), cols.begin(), cols.end());
            p->blk_rp[r + 1] = (int64_t)p->tile_col.size();
        }
        if (p->blk_rp[nc] > INT32_MAX) { delete p; return fail(SPM_EUNSUPPORTED, "more than 2^31-1 tiles"); }
        set_levels(p, lev);
        build_layout(p);
        p->nnz = rp[n];
        p->csr_rp.assign(rp, rp + n + 1);
        p->csr_col.assign(col, col + rp[n]);
        p->csr_pos.assign(p->n_stored, -1);
        for (int64_t t = 0; t < p->n_tiles; ++t) {
            int r = p->tile_row[t], c = p->tile_col[t];
            int nr = p->nfun[r], ncl = p->nfun[c];
            for (int i = 0; i < nr; ++i) {
                int64_t row = cs[r] + i;
                const int32_t *b = col + rp[row], *e = col + rp[row + 1];
                for (int j = 0; j < ncl; ++j) {
                    int32_t cc = (int32_t)(cs[c] + j);
                    const int32_t *f = std::lower_bound(b, e, cc);
                    if (f < e && *f == cc) p->csr_pos[p->tile_off[t] + (int64_t)j * nr + i] = rp[row] + (f - col - rp[row]);
                }
            }
        }
        p->masked = p->nnz != p->n_stored;
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(SPM_ENOMEM, "host allocation");
    }
    *out = p;
    return SPM_OK;
}

// Planned pattern + device tables in a block the library allocates.
static int upload_owned(spm_pattern p, void *stream, spm_pattern *out)
{
    int st;
    if ((st = spm::upload_pattern_device(p, nullptr, 0, (hipStream_t)stream))) {
        spm::free_pattern_device(p);
        delete p;
        *out = nullptr;
        return st;
    }
    return SPM_OK;
}

extern "C" int spm_block_pattern_upload(int64_t n, int32_t nc, const int64_t *cs, const int64_t *brp,
                                        const int32_t *bcol, void *stream, spm_pattern *out)
{
    if (!out) return fail(SPM_EINVAL, "spm_block_pattern_upload: null pointer");
    const int st = spm_block_pattern_plan(n, nc, cs, brp, bcol, nullptr, out);
    return st ? st : upload_owned(*out, stream, out);
}

extern "C" int spm_compress_pattern_upload(int64_t n, const int64_t *rp, const int32_t *col, int32_t nc,
                                           const int64_t *cs, void *stream, spm_pattern *out)
{
    if (!out) return fail(SPM_EINVAL, "spm_compress_pattern_upload: null pointer");
    const int st = spm_compress_pattern_plan(n, rp, col, nc, cs, nullptr, out);
    return st ? st : upload_owned(*out, stream, out);
}

extern "C" int spm_pattern_upload(spm_pattern p, void *stream)
{
    if (!p) return fail(SPM_EINVAL, "spm_pattern_upload: null pattern");
    if (p->uploaded) return fail(SPM_EINVAL, "spm_pattern_upload: pattern already uploaded");
    int st = spm::upload_pattern_device(p, nullptr, 0, (hipStream_t)stream);
    if (st) spm::free_pattern_device(p);
    return st;
}

extern "C" int spm_pattern_workspace_bytes(spm_pattern p, size_t *bytes)
{
    if (!p || !bytes) return fail(SPM_EINVAL, "spm_pattern_workspace_bytes: null pointer");
    *bytes = spm::pattern_device_bytes(p);
    return SPM_OK;
}

extern "C" int spm_pattern_upload_workspace(spm_pattern p, void *ws, size_t bytes, void *stream)
{
    if (!p || !ws) return fail(SPM_EINVAL, "spm_pattern_upload_workspace: null pointer");
    if (p->uploaded) return fail(SPM_EINVAL, "spm_pattern_upload_workspace: pattern already uploaded");
    int st = spm::upload_pattern_device(p, ws, bytes, (hipStream_t)stream);
    if (st) spm::free_pattern_device(p);
    return st;
}

extern "C" int spm_pattern_classes(spm_pattern p, int32_t *n_classes, int32_t *row_blocks, int32_t *col_blocks,
                                   int64_t *units, int64_t *out_tiles, double *exact_macs, double *padded_macs)
{
    if (!p || !n_classes) return fail(SPM_EINVAL, "spm_pattern_classes: null pointer");
    const int32_t nl = (int32_t)p->launches.size();
    if (row_blocks || col_blocks || units || out_tiles || exact_macs || padded_macs) {
        if (*n_classes < nl) return fail(SPM_EINVAL, "spm_pattern_classes: arrays too short");
        for (int32_t i = 0; i < nl; ++i) {
            const auto &L = p->launches[i];
            if (row_blocks) row_blocks[i] = L.rb;
            if (col_blocks) col_blocks[i] = L.cb;
            if (units) units[i] = L.count;
            if (out_tiles) out_tiles[i] = L.out_tiles;
            if (exact_macs) exact_macs[i] = L.exact_macs;
            if (padded_macs) padded_macs[i] = L.padded_macs;
        }
    }
    *n_classes = nl;
    return SPM_OK;
}

extern "C" int spm_pattern_destroy(spm_pattern p)
{
    if (!p) return SPM_OK;
    spm::free_pattern_device(p);
    delete p;
    return SPM_OK;
}

extern "C" int spm_pattern_info(spm_pattern p, int64_t *nnz, int64_t *n_stored, int64_t *n_tiles, double *macs)
{
    if (!p) return fail(SPM_EINVAL, "spm_pattern_info: null pattern");
    if (nnz) *nnz = p->nnz;
    if (n_stored) *n_stored = p->n_stored;
    if (n_tiles) *n_tiles = p->n_tiles;
    if (macs) *macs = p->macs;
    return SPM_OK;
}

extern "C" int spm_pattern_tiles(spm_pattern p, int32_t *tr, int32_t *tc, int64_t *to)
{
    if (!p) return fail(SPM_EINVAL, "spm_pattern_tiles: null pattern");
    if (tr) std::copy(p->tile_row.begin(), p->tile_row.end(), tr);
    if (tc) std::copy(p->tile_col.begin(), p->tile_col.end(), tc);
    if (to) std::copy(p->tile_off.begin(), p->tile_off.end() - 1, to);
    return SPM_OK;
}

extern "C" int spm_pattern_download_csr(spm_pattern p, int64_t *rp, int32_t *col)
{
    if (!p || !rp || !col) return fail(SPM_EINVAL, "spm_pattern_download_csr: null pointer");
    if (!p->csr_rp.empty()) {
        std::copy(p->csr_rp.begin(), p->csr_rp.end(), rp);
        std::copy(p->csr_col.begin(), p->csr_col.end(), col);
        return SPM_OK;
    }
    rp[0] = 0;
    int64_t e = 0;
    for (int r = 0; r < p->nc; ++r)
        for (int i = 0; i < p->nfun[r]; ++i) {
            for (int64_t t = p->blk_rp[r]; t < p->blk_rp[r + 1]; ++t) {
                int c = p->tile_col[t];
                for (int j = 0; j < p->nfun[c]; ++j) col[e++] = (int32_t)(p->cstart[c] + j);
            }
            rp[p->cstart[r] + i + 1] = e;
        }
    return SPM_OK;
}

// ---------------------------------------------------------------- contour quadrature rule
namespace {

// Jacobi elliptic functions sn, cn, dn of u for the parameter m (0 <= m < 1) by the
// arithmetic-geometric mean (descending Landen transformation): with a_0 = 1,
// b_0 = sqrt(1 - m), c_0 = sqrt(m) and a_{j+1} = (a_j + b_j)/2, b_{j+1} = sqrt(a_j b_j),
// c_{j+1} = (a_j - b_j)/2 until c_N vanishes, phi_N = 2^N a_N u and
// phi_{j-1} = (phi_j + asin(c_j sin(phi_j) / a_j)) / 2; then sn = sin phi_0,
// cn = cos phi_0, dn = cos phi_0 / cos(phi_1 - phi_0).  The quarter period is
// K(m) = pi / (2 a_N).
struct Agm {
    double a[40], c[40];
    int n = 0;
    explicit Agm(double m)
    {
        a[0] = 1.0;
        c[0] = std::sqrt(m);
        double b = std::sqrt(1.0 - m);
        while (n < 38 && c[n] > 1e-17 * a[n]) {
            a[n + 1] = 0.5 * (a[n] + b);
            c[n + 1] = 0.5 * (a[n] - b);
            b = std::sqrt(a[n] * b);
            ++n;
        }
    }
    double quarter_period() const { return 3.14159265358979323846 / (2.0 * a[n]); }
    void sncndn(double u, double &sn, double &cn, double &dn) const
    {
        double phi = std::ldexp(a[n] * u, n), phi1 = phi;
        for (int j = n; j >= 1; --j) {
            phi1 = phi;
            phi = 0.5 * (phi + std::asin(c[j] / a[j] * std::sin(phi)));
        }
        sn = std::sin(phi);
        cn = std::cos(phi);
        dn = n >= 1 ? cn / std::cos(phi1 - phi) : 1.0;
    }
};

}  // namespace

// Nodes and weights of A^{-1/2} ~ sum_k c_k (A + w_k^2 I)^{-1} for a spectrum in
// [lam_min, lam_max] (Section 4.4, eq. ContInt): the midpoint rule in t for
// A^{-1/2} = (2/pi) int_0^inf (A + w^2 I)^{-1} dw after w = sqrt(lam_min) sn(t)/cn(t),
// parameter 1 - lam_min/lam_max, t over one quarter period.
extern "C" int spm_contour_rule(double lam_min, double lam_max, int32_t nodes, double *w2, double *c)
{
    if (!w2 || !c) return fail(SPM_EINVAL, "spm_contour_rule: null pointer");
    if (!(lam_min > 0.0) || !(lam_max >= lam_min) || !std::isfinite(lam_max) || nodes < 1)
        return fail(SPM_EINVAL, "spm_contour_rule: need 0 < lam_min <= lam_max and nodes >= 1");
    const Agm g(1.0 - lam_min / lam_max);
    const double kq = g.quarter_period(), sm = std::sqrt(lam_min);
    for (int k = 0; k < nodes; ++k) {
        const double t = kq * (k + 0.5) / nodes;
        double sn, cn, dn;
        g.sncndn(t, sn, cn, dn);
        w2[k] = lam_min * (sn / cn) * (sn / cn);
        c[k] = 2.0 * kq * sm / (3.14159265358979323846 * nodes) * dn / (cn * cn);
    }
    return SPM_OK;
}
