/*
 * Plain C helpers of the FP64 oracle.  TEST INFRASTRUCTURE ONLY: nothing in the
 * GPU library links or includes this file.
 *
 * - the formatted product exactly on the pattern (Section 4.1, Theorem
 *   (product), eq. (product)): c_ij = sum over k in S_i and S_j of a_ik b_kj,
 *   evaluated entry by entry as a sorted merge of row i of A with column j of B,
 *   summing in ascending k;
 *   (also on a list of single entries, counting the multiply-adds);
 * - kernel sums sum_p w_p k(|x_q - x_p|) used to form single rows of
 *   K^Sigma = T K T^T (Section 3.3) without the full matrix.
 *
 * Built with -ffp-contract=off so that every multiply and add rounds on its own.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

/* Position of (j, i) for every stored (i, j) of a structurally symmetric CSR
 * pattern (binary search in row j).  Returns the number of entries whose
 * mirror is missing (0 for a symmetric pattern). */
int64_t oracle_transpose_positions(int64_t n, const int64_t *rp, const int32_t *col, int64_t *tpos)
{
    int64_t missing = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : missing)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            int64_t j = col[e];
            int64_t lo = rp[j], hi = rp[j + 1];
            while (lo < hi) {
                int64_t mid = lo + (hi - lo) / 2;
                if (col[mid] < i) lo = mid + 1; else hi = mid;
            }
            if (lo < rp[j + 1] && col[lo] == i) tpos[e] = lo;
            else { tpos[e] = -1; ++missing; }
        }
    }
    return missing;
}

/* One entry c_ij = sum_{k in S_i cap S_j} a_ik b_kj.  bt holds B^T on the same
 * pattern: bt[pos(j,k)] = b_kj. */
static double entry(const int64_t *rp, const int32_t *col, const double *a, const double *bt,
                    int64_t i, int64_t j)
{
    int64_t p = rp[i], pe = rp[i + 1], r = rp[j], re = rp[j + 1];
    double s = 0.0;
    while (p < pe && r < re) {
        int32_t ki = col[p], kj = col[r];
        if (ki < kj) ++p;
        else if (kj < ki) ++r;
        else { s += a[p] * bt[r]; ++p; ++r; }
    }
    return s;
}

/* C = P_S(A B) on every stored entry. */
void oracle_masked_product(int64_t n, const int64_t *rp, const int32_t *col,
                           const double *a, const double *bt, double *c)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            c[e] = entry(rp, col, a, bt, i, col[e]);
}

/* Same product on the rows listed in ``rows`` only; results are written to
 * c at the stored positions of those rows.  Returns the number of entries. */
int64_t oracle_masked_product_rows(int64_t nrows, const int64_t *rows, const int64_t *rp,
                                   const int32_t *col, const double *a, const double *bt, double *c)
{
    int64_t cnt = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : cnt)
    for (int64_t t = 0; t < nrows; ++t) {
        int64_t i = rows[t];
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            c[e] = entry(rp, col, a, bt, i, col[e]);
            ++cnt;
        }
    }
    return cnt;
}

/* Entries c_ij for a list of positions (i, j) of S (pos[t] = stored position of
 * (ii[t], jj[t]), where c is written); *macs receives the number of multiply-adds,
 * i.e. the sum of |S_i cap S_j| over the list. */
void oracle_masked_product_entries(int64_t np, const int64_t *ii, const int64_t *jj, const int64_t *pos,
                                   const int64_t *rp, const int32_t *col, const double *a, const double *bt,
                                   double *c, int64_t *macs)
{
    int64_t m = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : m)
    for (int64_t t = 0; t < np; ++t) {
        int64_t i = ii[t], j = jj[t];
        int64_t p = rp[i], pe = rp[i + 1], r = rp[j], re = rp[j + 1];
        double s = 0.0;
        int64_t k = 0;
        while (p < pe && r < re) {
            int32_t ki = col[p], kj = col[r];
            if (ki < kj) ++p;
            else if (kj < ki) ++r;
            else { s += a[p] * bt[r]; ++p; ++r; ++k; }
        }
        c[pos[t]] = s;
        m += k;
    }
    *macs = m;
}

static double fact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

/* Matern kernel nu = p + 1/2, paper's half-integer sum, or its lengthscale
 * derivative (term-by-term differentiation of the same sum). */
static double matern(double r, int p, double ell, int deriv)
{
    double nu = p + 0.5;
    double s = sqrt(2.0 * nu) * r / ell;
    double poly = 0.0, dpoly = 0.0;
    double pref = fact(p) / fact(2 * p);
    for (int q = 0; q <= p; ++q) {
        int k = p - q;
        double ck = pref * fact(p + q) / (fact(q) * fact(p - q)) * pow(2.0, k);
        poly += ck * pow(s, k);
        if (k > 0) dpoly += ck * k * pow(s, k - 1);
    }
    if (!deriv) return exp(-s) * poly;
    return (-s / ell) * (dpoly - poly) * exp(-s);
}

/* acc[q] = scale * sum_{t < m} w[t] k(|x_q - y_t|) for all n points x (row-major
 * n x d) and the m points y. */
void oracle_kernel_apply(int64_t n, int d, const double *x, int64_t m, const double *y,
                         const double *w, int p, double ell, double scale, int deriv, double *acc)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        double s = 0.0;
        for (int64_t t = 0; t < m; ++t) {
            double r2 = 0.0;
            for (int a = 0; a < d; ++a) {
                double df = x[q * d + a] - y[t * d + a];
                r2 += df * df;
            }
            s += w[t] * matern(sqrt(r2), p, ell, deriv);
        }
        acc[q] = scale * s;
    }
}

/* The same sums for k weight vectors at once (w row-major m x k): acc[q*k + c] =
 * scale * sum_{t < m} w[t*k + c] k(|x_q - y_t|), each sum in the order of the
 * single-vector call, so every column equals that call bit for bit. */
void oracle_kernel_apply_multi(int64_t n, int d, const double *x, int64_t m, const double *y,
                               const double *w, int k, int p, double ell, double scale, int deriv, double *acc)
{
#pragma omp parallel
    {
        double *s = (double *)malloc((size_t)k * sizeof(double));
#pragma omp for schedule(static)
        for (int64_t q = 0; q < n; ++q) {
            for (int c = 0; c < k; ++c) s[c] = 0.0;
            for (int64_t t = 0; t < m; ++t) {
                double r2 = 0.0;
                for (int a = 0; a < d; ++a) {
                    double df = x[q * d + a] - y[t * d + a];
                    r2 += df * df;
                }
                const double kv = matern(sqrt(r2), p, ell, deriv);
                for (int c = 0; c < k; ++c) s[c] += w[t * k + c] * kv;
            }
            for (int c = 0; c < k; ++c) acc[q * k + c] = scale * s[c];
        }
        free(s);
    }
}

/* OpenMP thread count for the calls above; returns the number of threads a
 * parallel region then actually runs with. */
int oracle_set_threads(int nthreads)
{
    int used = 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
    }
    return used;
}
