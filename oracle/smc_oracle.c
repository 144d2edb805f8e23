/*
 * smc_oracle.c -- plain, slow, single-threaded FP64 CPU oracle for one
 * SMC-sampler iteration and its resampling step.
 *
 * TEST INFRASTRUCTURE ONLY.  The product path (the HIP library and its Python
 * binding) never links, loads or calls this file.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark use it.  It shares no
 * code, header, table or constant generator with the HIP library.
 *
 * Method: Varsi, Kekempanos, Thiyagalingam, Maskell, "A Single SMC Sampler on
 * MPI that Outperforms a Single MCMC Sampler" (arXiv:1905.10252).
 *   - Alg 2 (SMC sampler with recycling), eq. smcs_drawing_weights with the
 *     backward kernel equal to the forward random-walk kernel (Sec. 5.2.3),
 *     eq. normalise, eq. neff, eq. estimation_at_t, eq. normconst,
 *     eq. recycling.
 *   - Alg 4 (minimum variance / systematic resampling) and eq. ncopies.
 *   - Alg 5 (sequential redistribute, S-R), with the copied row taken from the
 *     source index j (the printed listing indexes the source by the output
 *     counter, which cannot be meant).
 *
 * The paper never prints the MVR formula.  This oracle takes the standard
 * systematic scheme written in exact integers:
 *   K   = min(52, 61 - ceil(log2 N))
 *   q_i = min(2^K, floor(2^K * det_exp(l_i - max l)))     (uint64)
 *   S_j = q_0 + ... + q_j,  S = S_{N-1}  (exact, <= 2^61)
 *   U   = floor(r * S / 2^64) for a 64-bit draw r        (0 <= U < S)
 *   A_j = floor((N * S_j + U) / S),  ncopies_j = A_j - A_{j-1},  A_{-1} = 0
 * which is systematic resampling with offset u = 1 - U/S in (0, 1] applied to
 * the CDF S_j / S.  Resampling is triggered when the effective sample size is
 * below ess_num/ess_den * N, decided exactly in integers:
 *   ess_den * S^2 < ess_num * N * sum(q_i^2).
 * The FP64 path (max, log-sum-exp, normalised weights, FP64 ESS, estimates)
 * uses libm exp and Neumaier-compensated sums; it is a tolerance output.
 *
 * Determinism spec implemented here independently of the GPU library:
 *   - Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
 *   - det_exp: Cody-Waite reduction with the fdlibm split of ln 2, Taylor
 *     polynomial of degree 13 by Horner with fused multiply-add, ldexp.
 *   - det_log: reduction to m in [sqrt(1/2), sqrt(2)), log m = 2 atanh(f),
 *     f = (m-1)/(m+1), odd series to f^23 by Horner in f^2 with FMA.
 *   - det_atan: atan(1/a) = pi/2 - atan(a) folds |z| to [0, 1]; two argument
 *     halvings a <- a / (1 + sqrt(1 + a^2)) bring it below tan(pi/16); odd
 *     Taylor series to a^25; times 4.
 *   - normals: Marsaglia-Bray polar method on Philox uniforms.
 *
 * SIR particle filter (Alg 1) on the bearing-only tracking model of Sec. 5.2.2:
 * constant-velocity state [x, vx, y, vy], process noise with the paper's block
 * covariance, bearing measurement arctan(y / x) plus Gaussian noise; the
 * proposal is the transition, so the weight update is the likelihood.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

enum { ORC_OK = 0, ORC_E_ARG = 1, ORC_E_NONFINITE = 2, ORC_E_DEGENERATE = 3 };
enum { ORC_MODE_AUTO = 0, ORC_MODE_FORCE = 1, ORC_MODE_NEVER = 2 };
enum { ORC_TAG_INIT = 1, ORC_TAG_PROPOSE = 2, ORC_TAG_RESAMPLE = 3 };
enum { ORC_T_GAUSS = 1, ORC_T_STUDENT = 2, ORC_T_LOGREG = 3, ORC_T_GAUSS_CHOL = 5 };

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: 10 rounds of the Philox S-box on a 4x32-bit counter with a  */
/* 2x32-bit key; multipliers 0xD2511F53, 0xCD9E8D57 and Weyl key increments */
/* 0x9E3779B9, 0xBB67AE85 as published by Salmon et al.                     */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter layout used by every random draw of the sampler. */
static void orc_draw(uint64_t seed, uint32_t tag, uint32_t sampler_id, uint32_t t,
                     uint32_t idx, uint32_t sub, uint32_t out[4])
{
    uint32_t ctr[4] = { idx, sub, t, (tag << 24) | (sampler_id & 0xFFFFFFu) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    orc_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Deterministic exp / log (same spec on both sides, written separately).    */
/* ------------------------------------------------------------------------ */
static const double ORC_LN2_HI = 6.93147180369123816490e-01; /* fdlibm ln2_hi */
static const double ORC_LN2_LO = 1.90821492927058770002e-10; /* fdlibm ln2_lo */
static const double ORC_LOG2E = 1.4426950408889634;          /* 1/ln 2 rounded */
static const double ORC_SQRT1_2 = 0.70710678118654752440;    /* sqrt(1/2) rounded */

static double orc_factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i; /* exact for n <= 18 */
    return f;
}

double orc_det_exp(double x)
{
    if (x != x) return x;
    if (x < -746.0) return 0.0;
    if (x > 709.0) return INFINITY;
    double kd = rint(x * ORC_LOG2E);
    double r = fma(-kd, ORC_LN2_HI, x);
    r = fma(-kd, ORC_LN2_LO, r);
    /* Taylor series of e^r to degree 13, coefficients 1/n! rounded once. */
    double p = 1.0 / orc_factorial(13);
    for (int n = 12; n >= 0; --n) p = fma(p, r, 1.0 / orc_factorial(n));
    return ldexp(p, (int)kd);
}

double orc_det_log(double x)
{
    if (!(x > 0.0)) return x == 0.0 ? -INFINITY : NAN;
    if (isinf(x)) return x;
    int e;
    double m = frexp(x, &e); /* x = m * 2^e, m in [0.5, 1) */
    if (m < ORC_SQRT1_2) { m = m * 2.0; e = e - 1; }
    double f = (m - 1.0) / (m + 1.0);
    double s = f * f;
    /* log m = 2 atanh f = sum_k 2 f^(2k+1) / (2k+1), k = 0..11 */
    double p = 2.0 / 23.0;
    for (int k = 10; k >= 0; --k) p = fma(p, s, 2.0 / (double)(2 * k + 1));
    double lm = f * p;
    double E = (double)e;
    return fma(E, ORC_LN2_HI, fma(E, ORC_LN2_LO, lm));
}

static const double ORC_PI_2_HI = 1.57079632679489655800e+00; /* pi/2 rounded */
static const double ORC_PI_2_LO = 6.12323399573676603587e-17; /* pi/2 - PI_2_HI */

double orc_det_atan(double z)
{
    if (z != z) return z;
    int neg = z < 0.0;
    double a = neg ? -z : z;
    int inv = a > 1.0;
    if (inv) a = 1.0 / a;
    a = a / (1.0 + sqrt(fma(a, a, 1.0)));
    a = a / (1.0 + sqrt(fma(a, a, 1.0)));
    double s = a * a;
    /* atan(a) / a = sum_k (-1)^k s^k / (2k + 1), k = 0..12 */
    double p = 1.0 / 25.0;
    for (int k = 11; k >= 0; --k) {
        double c = 1.0 / (double)(2 * k + 1);
        p = fma(p, -s, c);
    }
    double r = 4.0 * (a * p);
    if (inv) r = (ORC_PI_2_HI - r) + ORC_PI_2_LO;
    return neg ? -r : r;
}

/* ------------------------------------------------------------------------ */
/* Standard normals by the Marsaglia-Bray polar method.  Pair k of particle  */
/* idx uses counter sub-word (k << 16) | attempt; after 32 rejected attempts */
/* (probability ~1e-21) the pair is (0, 0).  With one coordinate a particle, */
/* particles 2p and 2p + 1 share pair 0 of index p.                          */
/* ------------------------------------------------------------------------ */
static void orc_normal_pair(uint64_t seed, uint32_t tag, uint32_t sampler_id, uint32_t t,
                            uint32_t idx, uint32_t pair, double *z1, double *z2)
{
    for (uint32_t a = 0; a < 32; ++a) {
        uint32_t w[4];
        orc_draw(seed, tag, sampler_id, t, idx, (pair << 16) | a, w);
        uint64_t b1 = ((uint64_t)w[1] << 32) | w[0];
        uint64_t b2 = ((uint64_t)w[3] << 32) | w[2];
        double v1 = (double)(b1 >> 11) * 0x1p-52 - 1.0; /* uniform on [-1, 1) */
        double v2 = (double)(b2 >> 11) * 0x1p-52 - 1.0;
        double s = v1 * v1 + v2 * v2;
        if (s > 0.0 && s < 1.0) {
            double lg = orc_det_log(s);
            double c = (-2.0 * lg) / s;
            double f = sqrt(c);
            *z1 = v1 * f;
            *z2 = v2 * f;
            return;
        }
    }
    *z1 = 0.0;
    *z2 = 0.0;
}

void orc_normals(uint64_t seed, uint32_t tag, uint32_t sampler_id, uint32_t t, uint32_t idx,
                 int32_t d, double *z)
{
    if (d == 1) {
        /* one coordinate a particle: particles 2p and 2p + 1 take the two
           values of pair 0 drawn for index p, so no draw is discarded */
        double a, b;
        orc_normal_pair(seed, tag, sampler_id, t, idx >> 1, 0u, &a, &b);
        z[0] = (idx & 1u) ? b : a;
        return;
    }
    for (int32_t k = 0; 2 * k < d; ++k) {
        double a, b;
        orc_normal_pair(seed, tag, sampler_id, t, idx, (uint32_t)k, &a, &b);
        z[2 * k] = a;
        if (2 * k + 1 < d) z[2 * k + 1] = b;
    }
}

/* 64-bit draw used as the systematic offset source r. */
uint64_t orc_resample_draw(uint64_t seed, uint32_t sampler_id, uint32_t t)
{
    uint32_t w[4];
    orc_draw(seed, ORC_TAG_RESAMPLE, sampler_id, t, 0u, 0u, w);
    return ((uint64_t)w[1] << 32) | w[0];
}

/* ------------------------------------------------------------------------ */
/* Resampling (Alg 4: MVR -> redistribute -> reset).                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    double m, logZ, ess, Z, Z2;
    uint64_t S, U, Q2_hi, Q2_lo;
    int32_t K, resampled, err, pad;
    int64_t unique; /* number of sources that receive at least one copy */
} orc_resample_info;

static void neu_add(double *sum, double *comp, double v)
{
    double s = *sum, t = s + v;
    if (fabs(s) >= fabs(v)) *comp += (s - t) + v;
    else *comp += (v - t) + s;
    *sum = t;
}

int32_t orc_quant_bits(int64_t n)
{
    int c = 0;
    while (((int64_t)1 << c) < n) ++c; /* ceil(log2 n) */
    int K = 61 - c;
    return K < 52 ? K : 52;
}

/* q_i = min(2^K, floor(2^K * det_exp(l_i - m))). */
void orc_quantise(const double *logw, int64_t n, int32_t K, double m, uint64_t *q)
{
    uint64_t top = (uint64_t)1 << K;
    for (int64_t i = 0; i < n; ++i) {
        double e = orc_det_exp(logw[i] - m);
        double v = floor(ldexp(e, K));
        uint64_t qi = (uint64_t)v;
        q[i] = qi > top ? top : qi;
    }
}

/* Systematic ncopies from quantised weights and offset U (0 <= U < S). */
int orc_systematic_ncopies(const uint64_t *q, int64_t n, uint64_t U, int64_t *ncopies)
{
    u128 S = 0;
    for (int64_t i = 0; i < n; ++i) S += q[i];
    if (S == 0 || (u128)U >= S) return ORC_E_ARG;
    u128 Sj = 0, Aprev = 0;
    for (int64_t j = 0; j < n; ++j) {
        Sj += q[j];
        u128 A = ((u128)n * Sj + U) / S;
        ncopies[j] = (int64_t)(A - Aprev);
        Aprev = A;
    }
    return ORC_OK;
}

int orc_resample(const double *logw, int64_t n, uint64_t r, int32_t mode, int32_t ess_num,
                 int32_t ess_den, int64_t *ncopies, orc_resample_info *info)
{
    memset(info, 0, sizeof(*info));
    if (n < 1 || ess_num < 0 || ess_den < 1 || ess_num > 16 || ess_den > 16) {
        info->err = ORC_E_ARG;
        return ORC_E_ARG;
    }
    /* validation: NaN and +inf are errors; -inf is a zero weight */
    double m = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double v = logw[i];
        if (v != v || v == INFINITY) { info->err = ORC_E_NONFINITE; return ORC_E_NONFINITE; }
        if (v > m) m = v;
    }
    if (m == -INFINITY) { info->err = ORC_E_DEGENERATE; return ORC_E_DEGENERATE; }
    info->m = m;

    /* FP64 path: eq. normalise and eq. neff through log-sum-exp. */
    double Z = 0.0, cz = 0.0, Z2 = 0.0, cz2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double e = exp(logw[i] - m);
        neu_add(&Z, &cz, e);
        neu_add(&Z2, &cz2, e * e);
    }
    Z += cz;
    Z2 += cz2;
    info->Z = Z;
    info->Z2 = Z2;
    info->logZ = m + log(Z);
    info->ess = (Z * Z) / Z2;

    /* Fixed-point weights and exact integer sums. */
    int32_t K = orc_quant_bits(n);
    info->K = K;
    uint64_t *q = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    if (!q) { info->err = ORC_E_ARG; return ORC_E_ARG; }
    orc_quantise(logw, n, K, m, q);
    u128 S = 0, Q2 = 0;
    for (int64_t i = 0; i < n; ++i) {
        S += q[i];
        Q2 += (u128)q[i] * q[i];
    }
    info->S = (uint64_t)S;
    info->Q2_hi = (uint64_t)(Q2 >> 64);
    info->Q2_lo = (uint64_t)Q2;

    int resample;
    if (mode == ORC_MODE_FORCE) resample = 1;
    else if (mode == ORC_MODE_NEVER) resample = 0;
    else resample = ((u128)ess_den * S * S) < ((u128)ess_num * (u128)n * Q2);
    info->resampled = resample;
    info->U = (uint64_t)(((u128)r * S) >> 64);

    int64_t unique = 0;
    if (resample) {
        orc_systematic_ncopies(q, n, info->U, ncopies);
        for (int64_t j = 0; j < n; ++j) unique += ncopies[j] > 0;
    } else {
        for (int64_t j = 0; j < n; ++j) ncopies[j] = 1;
        unique = n;
    }
    info->unique = unique;
    free(q);
    return ORC_OK;
}

/* eq. normalise: w~_i = w_i / sum_j w_j with w_i = exp(l_i), taken as
 * exp(l_i - m) / Z, m = max l, Z = sum exp(l_j - m) (libm exp, Neumaier sum).
 * Errors as orc_resample: NaN or +inf, or every weight zero. */
int orc_normalised_weights(const double *logw, int64_t n, double *w)
{
    if (n < 1) return ORC_E_ARG;
    double m = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double v = logw[i];
        if (v != v || v == INFINITY) return ORC_E_NONFINITE;
        if (v > m) m = v;
    }
    if (m == -INFINITY) return ORC_E_DEGENERATE;
    double Z = 0.0, cz = 0.0;
    for (int64_t i = 0; i < n; ++i) neu_add(&Z, &cz, exp(logw[i] - m));
    Z += cz;
    for (int64_t i = 0; i < n; ++i) w[i] = exp(logw[i] - m) / Z;
    return ORC_OK;
}

/* Alg 5, sequential redistribute: copy row j ncopies_j times, in source
 * order.  anc (nullable) receives the source index of every output row. */
int orc_redistribute(int64_t n, const int64_t *ncopies, const void *x, int64_t row_bytes,
                     void *x_out, int64_t *anc)
{
    int64_t total = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (ncopies[j] < 0) return ORC_E_ARG;
        total += ncopies[j];
    }
    if (total != n) return ORC_E_ARG;
    const unsigned char *src = (const unsigned char *)x;
    unsigned char *dst = (unsigned char *)x_out;
    int64_t i = 0;
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t k = 0; k < ncopies[j]; ++k) {
            memcpy(dst + i * row_bytes, src + j * row_bytes, (size_t)row_bytes);
            if (anc) anc[i] = j;
            ++i;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* SMC sampler (Alg 2) with a Gaussian random-walk proposal and L = q.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    int32_t d, target, mode, ess_num, ess_den;
    uint32_t sampler_id;
    uint64_t seed;
    double rw_sd;
    double init_mean, init_sd, init_log_norm; /* q0 = N(init_mean, init_sd^2 I) */
    double log_norm;                          /* additive constant of log pi */
    const double *mean, *prec;                /* Gaussian target, [d] each */
    double nu, mu;                            /* Student-t target (d = 1) */
    int64_t m_rows;                           /* logistic regression: X [M][d], y [M] */
    const double *X, *y;
    double prior_prec;
    const double *chol;                       /* Gaussian with full precision P = U^T U: */
                                              /* U upper triangular [d][d], row-major    */
} orc_smc_cfg;

#define ORC_DMAX 64

typedef struct {
    double logZ_prev;         /* log sum_i w_{t-1}^i */
    double lc_max;            /* running max of log c_t (scaling for the sums) */
    double den;               /* sum_t c_t * exp(-lc_max) */
    double num[2 * ORC_DMAX]; /* sum_t c_t f_t * exp(-lc_max) (mean, then 2nd moment) */
    int32_t steps;
    int32_t pad;
} orc_recycle;

typedef struct {
    orc_resample_info info;
    double log_c;              /* log c_t, eq. normconst */
    double est[2 * ORC_DMAX];  /* f_t = sum w~ x, then sum w~ x^2 */
    double rec[2 * ORC_DMAX];  /* recycled estimate, eq. recycling */
} orc_step_out;

static double orc_softplus(double z)
{
    return z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z));
}

/* log pi(x) for one particle. */
double orc_log_target(const orc_smc_cfg *c, const double *x)
{
    if (c->target == ORC_T_GAUSS) {
        double acc = 0.0;
        for (int32_t k = 0; k < c->d; ++k) {
            double t = x[k] - c->mean[k];
            acc = acc + (t * t) * c->prec[k];
        }
        return c->log_norm - 0.5 * acc;
    }
    if (c->target == ORC_T_GAUSS_CHOL) {
        /* (x - mean)^T P (x - mean) = |U (x - mean)|^2: row i of U from its
         * diagonal on, each term a fused multiply-add, rows summed in order */
        double acc = 0.0;
        for (int32_t i = 0; i < c->d; ++i) {
            double r = 0.0;
            for (int32_t k = i; k < c->d; ++k)
                r = fma(c->chol[(int64_t)i * c->d + k], x[k] - c->mean[k], r);
            acc = fma(r, r, acc);
        }
        return c->log_norm - 0.5 * acc;
    }
    if (c->target == ORC_T_STUDENT) {
        double inv_nu = 1.0 / c->nu;
        double hnu1 = 0.5 * (c->nu + 1.0);
        double t = x[0] - c->mu;
        double w = 1.0 + (t * t) * inv_nu;
        return c->log_norm - hnu1 * orc_det_log(w);
    }
    if (c->target == ORC_T_LOGREG) {
        double pr = 0.0;
        for (int32_t k = 0; k < c->d; ++k) pr += x[k] * x[k];
        double ll = 0.0, comp = 0.0;
        for (int64_t r = 0; r < c->m_rows; ++r) {
            double z = 0.0;
            for (int32_t k = 0; k < c->d; ++k) z += c->X[r * c->d + k] * x[k];
            neu_add(&ll, &comp, c->y[r] * z - orc_softplus(z));
        }
        return c->log_norm - 0.5 * c->prior_prec * pr + (ll + comp);
    }
    return NAN;
}

/* Batch of log-target values (used for per-step parity of costly targets). */
void orc_log_target_batch(const orc_smc_cfg *c, const double *x, int64_t n, double *lp)
{
    for (int64_t i = 0; i < n; ++i) lp[i] = orc_log_target(c, x + i * c->d);
}

static double orc_log_q0(const orc_smc_cfg *c, const double *x)
{
    double prec0 = 1.0 / (c->init_sd * c->init_sd);
    double acc = 0.0;
    for (int32_t k = 0; k < c->d; ++k) {
        double t = x[k] - c->init_mean;
        acc = acc + (t * t) * prec0;
    }
    return c->init_log_norm - 0.5 * acc;
}

/* Alg 2 initialisation: x0 ~ q0, w0 = pi(x0) / q0(x0), in logs. */
int orc_smc_init(const orc_smc_cfg *c, double *x, double *logw, double *lp, orc_recycle *rec)
{
    if (c->n < 1 || c->d < 1 || c->d > ORC_DMAX) return ORC_E_ARG;
    double z[ORC_DMAX];
    for (int64_t i = 0; i < c->n; ++i) {
        double *xi = x + i * c->d;
        orc_normals(c->seed, ORC_TAG_INIT, c->sampler_id, 0u, (uint32_t)i, c->d, z);
        for (int32_t k = 0; k < c->d; ++k) xi[k] = c->init_mean + c->init_sd * z[k];
        lp[i] = orc_log_target(c, xi);
        logw[i] = lp[i] - orc_log_q0(c, xi);
    }
    /* log sum w0 (log-sum-exp, FP64 with compensated sum) */
    double m = -INFINITY;
    for (int64_t i = 0; i < c->n; ++i) if (logw[i] > m) m = logw[i];
    double Z = 0.0, cz = 0.0;
    for (int64_t i = 0; i < c->n; ++i) neu_add(&Z, &cz, exp(logw[i] - m));
    memset(rec, 0, sizeof(*rec));
    rec->logZ_prev = m + log(Z + cz);
    rec->lc_max = -INFINITY;
    return ORC_OK;
}

/* One iteration t >= 1 of Alg 2: importance sampling, normalise, estimate,
 * ESS, resample if needed; plus the recycling sums (eq. normconst, eq.
 * recycling).  The normalising constant c_t is taken after importance
 * sampling at iteration t (the listing computes it before, where w_t does not
 * yet exist). */
int orc_smc_step(const orc_smc_cfg *c, uint32_t t, double *x, double *logw, double *lp,
                 orc_recycle *rec, orc_step_out *out)
{
    int64_t n = c->n;
    int32_t d = c->d;
    double z[ORC_DMAX];
    memset(out, 0, sizeof(*out));
    /* importance sampling: x' = x + rw_sd * z, l += log pi(x') - log pi(x) */
    for (int64_t i = 0; i < n; ++i) {
        double *xi = x + i * d;
        orc_normals(c->seed, ORC_TAG_PROPOSE, c->sampler_id, t, (uint32_t)i, d, z);
        for (int32_t k = 0; k < d; ++k) xi[k] = xi[k] + c->rw_sd * z[k];
        double lpn = orc_log_target(c, xi);
        logw[i] = logw[i] + (lpn - lp[i]);
        lp[i] = lpn;
    }
    /* resampling decision and ncopies (also normalise / ESS in FP64) */
    int64_t *nc = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!nc) return ORC_E_ARG;
    uint64_t r = orc_resample_draw(c->seed, c->sampler_id, t);
    int rc = orc_resample(logw, n, r, c->mode, c->ess_num, c->ess_den, nc, &out->info);
    if (rc != ORC_OK) { free(nc); return rc; }
    /* estimate f_t = sum w~ x (and sum w~ x^2), eq. estimation_at_t */
    double m = out->info.m, Z = out->info.Z;
    for (int32_t k = 0; k < d; ++k) {
        double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double e = exp(logw[i] - m);
            double xv = x[i * d + k];
            neu_add(&s1, &c1, e * xv);
            neu_add(&s2, &c2, e * xv * xv);
        }
        out->est[k] = (s1 + c1) / Z;
        out->est[d + k] = (s2 + c2) / Z;
    }
    /* normalising constant and recycling */
    double logc = out->info.logZ - rec->logZ_prev;
    out->log_c = logc;
    if (logc > rec->lc_max) {
        double sc = rec->steps ? exp(rec->lc_max - logc) : 0.0;
        rec->den *= sc;
        for (int32_t k = 0; k < 2 * d; ++k) rec->num[k] *= sc;
        rec->lc_max = logc;
    }
    double wgt = exp(logc - rec->lc_max);
    rec->den += wgt;
    for (int32_t k = 0; k < 2 * d; ++k) rec->num[k] += wgt * out->est[k];
    rec->steps += 1;
    for (int32_t k = 0; k < 2 * d; ++k) out->rec[k] = rec->num[k] / rec->den;
    /* resampling: redistribute x and the cached log-target, reset weights */
    if (out->info.resampled) {
        double *xn = (double *)malloc(sizeof(double) * (size_t)(n * d));
        double *lpn = (double *)malloc(sizeof(double) * (size_t)n);
        if (!xn || !lpn) { free(nc); free(xn); free(lpn); return ORC_E_ARG; }
        orc_redistribute(n, nc, x, (int64_t)d * 8, xn, NULL);
        orc_redistribute(n, nc, lp, 8, lpn, NULL);
        memcpy(x, xn, sizeof(double) * (size_t)(n * d));
        memcpy(lp, lpn, sizeof(double) * (size_t)n);
        double reset = -log((double)n);
        for (int64_t i = 0; i < n; ++i) logw[i] = reset;
        rec->logZ_prev = 0.0; /* sum of reset weights is 1 */
        free(xn);
        free(lpn);
    } else {
        rec->logZ_prev = out->info.logZ;
    }
    free(nc);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* SIR particle filter (Alg 1), bearing-only tracking (Sec. 5.2.2).          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    int32_t mode, ess_num, ess_den;
    uint32_t sampler_id;
    uint64_t seed;
    double delta;         /* sampling period */
    double obs_var;       /* variance of the bearing noise */
    double obs_log_norm;  /* -0.5 log(2 pi obs_var) */
    double init_mean[4];  /* X0 ~ N(init_mean, init_sd^2 I) */
    double init_sd;
    const double *y;      /* measurements y[t-1] for t = 1..T */
    int32_t T;
    int32_t pad;
} orc_pf_cfg;

typedef struct {
    orc_resample_info info;
    double log_c;       /* log of sum w_t / sum w_{t-1}: evidence increment */
    double mean[4];     /* weighted mean after resampling (Alg 1 order) */
    double m2[4];
} orc_pf_out;

/* Cholesky factor of the 2x2 process-noise block [[5 D^3/3, 5 D^2/2], [5 D^2/2, 5 D]]. */
static void orc_pf_chol(double D, double *l11, double *l21, double *l22)
{
    double s11 = 5.0 * D * D * D / 3.0, s21 = 5.0 * D * D / 2.0, s22 = 5.0 * D;
    *l11 = sqrt(s11);
    *l21 = s21 / *l11;
    *l22 = sqrt(s22 - *l21 * *l21);
}

int orc_pf_init(const orc_pf_cfg *c, double *x, double *logw, double *logZ_prev)
{
    if (c->n < 1) return ORC_E_ARG;
    double z[4];
    double reset = -log((double)c->n);
    for (int64_t i = 0; i < c->n; ++i) {
        orc_normals(c->seed, ORC_TAG_INIT, c->sampler_id, 0u, (uint32_t)i, 4, z);
        for (int k = 0; k < 4; ++k) x[i * 4 + k] = c->init_mean[k] + c->init_sd * z[k];
        logw[i] = reset;
    }
    *logZ_prev = 0.0;
    return ORC_OK;
}

/* Bearing log-likelihood of one particle: log N(y; atan(x2 / x0), obs_var). */
double orc_pf_loglik(const orc_pf_cfg *c, const double *xi, double y)
{
    double h = orc_det_atan(xi[2] / xi[0]);
    double e = y - h;
    double prec = 1.0 / c->obs_var;
    return c->obs_log_norm - 0.5 * ((e * e) * prec);
}

int orc_pf_step(const orc_pf_cfg *c, uint32_t t, double *x, double *logw, double *logZ_prev,
                orc_pf_out *out)
{
    if (t < 1 || (int32_t)t > c->T) return ORC_E_ARG;
    int64_t n = c->n;
    double l11, l21, l22, z[4];
    orc_pf_chol(c->delta, &l11, &l21, &l22);
    double y = c->y[t - 1];
    memset(out, 0, sizeof(*out));
    /* importance sampling with the transition as proposal */
    for (int64_t i = 0; i < n; ++i) {
        double *xi = x + i * 4;
        orc_normals(c->seed, ORC_TAG_PROPOSE, c->sampler_id, t, (uint32_t)i, 4, z);
        double v0 = l11 * z[0];
        double v1 = l21 * z[0] + l22 * z[1];
        double v2 = l11 * z[2];
        double v3 = l21 * z[2] + l22 * z[3];
        double n0 = (xi[0] + c->delta * xi[1]) + v0;
        double n1 = xi[1] + v1;
        double n2 = (xi[2] + c->delta * xi[3]) + v2;
        double n3 = xi[3] + v3;
        xi[0] = n0; xi[1] = n1; xi[2] = n2; xi[3] = n3;
        logw[i] = logw[i] + orc_pf_loglik(c, xi, y);
    }
    int64_t *nc = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!nc) return ORC_E_ARG;
    uint64_t r = orc_resample_draw(c->seed, c->sampler_id, t);
    int rc = orc_resample(logw, n, r, c->mode, c->ess_num, c->ess_den, nc, &out->info);
    if (rc != ORC_OK) { free(nc); return rc; }
    out->log_c = out->info.logZ - *logZ_prev;
    if (out->info.resampled) {
        double *xn = (double *)malloc(sizeof(double) * (size_t)(n * 4));
        if (!xn) { free(nc); return ORC_E_ARG; }
        orc_redistribute(n, nc, x, 32, xn, NULL);
        memcpy(x, xn, sizeof(double) * (size_t)(n * 4));
        free(xn);
        double reset = -log((double)n);
        for (int64_t i = 0; i < n; ++i) logw[i] = reset;
        *logZ_prev = 0.0;
    } else {
        *logZ_prev = out->info.logZ;
    }
    free(nc);
    /* weighted mean of the particles after resampling */
    double m = -INFINITY;
    for (int64_t i = 0; i < n; ++i) if (logw[i] > m) m = logw[i];
    double Z = 0.0, cz = 0.0;
    for (int64_t i = 0; i < n; ++i) neu_add(&Z, &cz, exp(logw[i] - m));
    Z += cz;
    for (int k = 0; k < 4; ++k) {
        double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double e = exp(logw[i] - m), xv = x[i * 4 + k];
            neu_add(&s1, &c1, e * xv);
            neu_add(&s2, &c2, e * xv * xv);
        }
        out->mean[k] = (s1 + c1) / Z;
        out->m2[k] = (s2 + c2) / Z;
    }
    return ORC_OK;
}
