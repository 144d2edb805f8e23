/* Multi-core CPU comparison point for the resample + redistribute path.
 *
 * Measurement code for the benchmark only: neither the GPU library nor the
 * parity tests depend on it.  It computes the same exact-integer systematic
 * resampling as the GPU path:
 *   m = max l_i;  K = min(52, 61 - ceil(log2 N));
 *   q_i = min(2^K, floor(2^K det_exp(l_i - m)))      (64-bit fixed point)
 *   S_j = q_0 + ... + q_j;  U = floor(r S / 2^64);
 *   A_j = floor((N S_j + U) / S);  ncopies_j = A_j - A_{j-1}   (eq. ncopies)
 * and writes row j to outputs A_{j-1} .. A_j - 1 (the sequential order of
 * Alg 5).  Z = sum e_i and Z2 = sum e_i^2 (e_i = det_exp(l_i - m)) are formed
 * on the way, as the FP64 normalisation and ESS need them (eq. normalise,
 * eq. neff).
 *
 * Parallel form (OpenMP over chunks of the particle range): a parallel max;
 * pass 1 quantises each chunk and forms its totals; a serial prefix over the
 * chunk totals gives every chunk its S offset; pass 2 walks each chunk in
 * order, carrying A_j as quotient and remainder so that each step needs one
 * 64-bit division; pass 3 splits the outputs into equal blocks and copies
 * rows, finding each block's first source by binary search over A.
 *
 * det_exp is the deterministic exponential: Cody-Waite reduction by ln 2
 * split as in fdlibm (hi/lo), the Taylor polynomial of e^r to degree 13 with
 * coefficients 1/n! rounded once, evaluated by Horner's rule with fused
 * multiply-adds, then scaled by 2^k. */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

static const double LN2_HI = 6.93147180369123816490e-01;
static const double LN2_LO = 1.90821492927058770002e-10;
static const double LOG2E = 1.4426950408889634;

static double inv_fact[14];

static void init_inv_fact(void)
{
    double f = 1.0;
    inv_fact[0] = 1.0;
    for (int i = 1; i < 14; ++i) {
        f *= (double)i;
        inv_fact[i] = 1.0 / f;
    }
}

static inline double det_exp(double x)
{
    if (x != x) return x;
    if (x < -746.0) return 0.0;
    if (x > 709.0) return INFINITY;
    const double kd = rint(x * LOG2E);
    double r = fma(-kd, LN2_HI, x);
    r = fma(-kd, LN2_LO, r);
    double p = inv_fact[13];
    for (int n = 12; n >= 0; --n) p = fma(p, r, inv_fact[n]);
    return ldexp(p, (int)kd);
}

typedef struct {
    uint64_t S;
    u128 Q2;
    double Z, Z2;
} chunk_tot;

/* Pass 1 over [lo, hi): q_i into q, and the chunk's totals. */
__attribute__((target_clones("fma", "default")))
static void quantise_chunk(const double *lw, int64_t lo, int64_t hi, double m, int K,
                           uint64_t *q, chunk_tot *t)
{
    const uint64_t top = (uint64_t)1 << K;
    uint64_t S = 0;
    u128 Q2 = 0;
    double Z = 0.0, Z2 = 0.0;
    for (int64_t i = lo; i < hi; ++i) {
        const double e = det_exp(lw[i] - m);
        const uint64_t v = (uint64_t)floor(ldexp(e, K));
        const uint64_t qi = v > top ? top : v;
        q[i] = qi;
        S += qi;
        Q2 += (u128)qi * qi;
        Z += e;
        Z2 += e * e;
    }
    t->S = S;
    t->Q2 = Q2;
    t->Z = Z;
    t->Z2 = Z2;
}

int omp_threads(void) { return omp_get_max_threads(); }

/* Returns 0, or 1 for an argument error, 2 for a non-finite log-weight, 3 when
 * every weight is zero.  x and x_out hold n rows of row_bytes bytes; q is n
 * words of scratch; res (nullable) receives S, U, Q2 hi/lo and K; zres
 * (nullable) receives Z, Z2 and m. */
int omp_resample_redistribute(const double *lw, int64_t n, uint64_t r, const void *x,
                              int64_t row_bytes, void *x_out, int64_t *ncopies, uint64_t *q,
                              uint64_t *res, double *zres)
{
    if (n < 1 || row_bytes < 1 || !lw || !x || !x_out || !ncopies || !q) return 1;
    if (inv_fact[0] == 0.0) init_inv_fact();
    double m = -INFINITY;
    int bad = 0;
#pragma omp parallel for reduction(max : m) reduction(| : bad) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double v = lw[i];
        if (v != v || v == INFINITY) bad |= 1;
        m = v > m ? v : m;
    }
    if (bad) return 2;
    if (m == -INFINITY) return 3;
    int c = 0;
    while (((int64_t)1 << c) < n) ++c;
    const int K = 61 - c < 52 ? 61 - c : 52;

    const int nth = omp_get_max_threads();
    int64_t nch = (int64_t)nth * 8;
    if (nch > n) nch = n;
    chunk_tot *tot = (chunk_tot *)calloc((size_t)nch, sizeof(chunk_tot));
    uint64_t *soff = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nch);
    if (!tot || !soff) {
        free(tot);
        free(soff);
        return 1;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nch; ++k)
        quantise_chunk(lw, n * k / nch, n * (k + 1) / nch, m, K, q, &tot[k]);
    uint64_t S = 0;
    u128 Q2 = 0;
    double Z = 0.0, Z2 = 0.0;
    for (int64_t k = 0; k < nch; ++k) {
        soff[k] = S;
        S += tot[k].S;
        Q2 += tot[k].Q2;
        Z += tot[k].Z;
        Z2 += tot[k].Z2;
    }
    const uint64_t U = (uint64_t)(((u128)r * S) >> 64);
    /* Pass 2: ncopies, and A_j (the end of row j's outputs) in place of q_j. */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nch; ++k) {
        const int64_t lo = n * k / nch, hi = n * (k + 1) / nch;
        const u128 num = (u128)n * soff[k] + U;
        uint64_t A = (uint64_t)(num / S);
        uint64_t R = (uint64_t)(num - (u128)A * S);  /* R < S <= 2^61 */
        for (int64_t j = lo; j < hi; ++j) {
            R += (uint64_t)n * q[j];                  /* n q_j <= 2^61: no overflow */
            const uint64_t dA = R / S;
            R -= dA * S;
            ncopies[j] = (int64_t)dA;
            A += dA;
            q[j] = A;
        }
    }
    /* Pass 3: equal blocks of outputs; the first source of a block by binary
     * search over A, so a row with millions of copies is spread over threads. */
    const unsigned char *src = (const unsigned char *)x;
    unsigned char *dst = (unsigned char *)x_out;
    const int64_t nblk = nch, per = (n + nblk - 1) / nblk;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nblk; ++b) {
        const uint64_t p0 = (uint64_t)(b * per), p1e = (uint64_t)((b + 1) * per);
        const uint64_t p1 = p1e < (uint64_t)n ? p1e : (uint64_t)n;
        if (p0 >= p1) continue;
        int64_t lo = 0, hi = n - 1;                   /* first j with A_j > p0 */
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (q[mid] > p0) hi = mid;
            else lo = mid + 1;
        }
        uint64_t p = p0;
        for (int64_t j = lo; p < p1; ++j) {
            const uint64_t end = q[j] < p1 ? q[j] : p1;
            const unsigned char *row = src + j * row_bytes;
            for (; p < end; ++p) memcpy(dst + p * row_bytes, row, (size_t)row_bytes);
        }
    }
    if (res) {
        res[0] = S;
        res[1] = U;
        res[2] = (uint64_t)(Q2 >> 64);
        res[3] = (uint64_t)Q2;
        res[4] = (uint64_t)K;
    }
    if (zres) {
        zres[0] = Z;
        zres[1] = Z2;
        zres[2] = m;
    }
    free(tot);
    free(soff);
    return 0;
}

/* Logistic-regression log-likelihood on every host core: for each of the n
 * particles theta_i (rows of d values), the sum over the m rows of X of
 * y_r z - softplus(z), z = X_r . theta_i, softplus in the overflow-safe form
 * max(z, 0) + log1p(exp(-|z|)).  The particles are split over the threads;
 * X is transposed once so that z for 64 rows at a time is a vector loop. */
enum { LR_ROWS = 64 };

__attribute__((target_clones("avx2", "default")))
static void logreg_one(const double *th, int d, const double *Xt, const double *y, int64_t m,
                       double *out)
{
    double acc = 0.0;
    double z[LR_ROWS];
    for (int64_t r0 = 0; r0 < m; r0 += LR_ROWS) {
        const int nr = m - r0 < LR_ROWS ? (int)(m - r0) : LR_ROWS;
        for (int j = 0; j < LR_ROWS; ++j) z[j] = 0.0;
        for (int k = 0; k < d; ++k) {
            const double *xk = Xt + (int64_t)k * m + r0;
            const double t = th[k];
            for (int j = 0; j < nr; ++j) z[j] += xk[j] * t;
        }
        for (int j = 0; j < nr; ++j) {
            const double sp = (z[j] > 0.0 ? z[j] : 0.0) + log1p(exp(-fabs(z[j])));
            acc += y[r0 + j] * z[j] - sp;
        }
    }
    *out = acc;
}

int omp_logreg_loglik(const double *theta, int64_t n, int d, const double *X, const double *y,
                      int64_t m, double *out)
{
    double *Xt = (double *)malloc(sizeof(double) * (size_t)m * (size_t)d);
    if (!Xt) return 1;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < m; ++r)
        for (int k = 0; k < d; ++k) Xt[(int64_t)k * m + r] = X[r * d + k];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) logreg_one(theta + i * d, d, Xt, y, m, out + i);
    free(Xt);
    return 0;
}
