/*
 * smc.h -- C ABI of libsmc, an MI355X (gfx950) implementation of one
 * SMC-sampler iteration and its resampling hot path.
 *
 * Method: Varsi, Kekempanos, Thiyagalingam, Maskell, "A Single SMC Sampler on
 * MPI that Outperforms a Single MCMC Sampler" (arXiv:1905.10252):
 *   Alg 2 (SMC sampler with recycling), Alg 4 (minimum variance resampling:
 *   ncopies, redistribute, reset), Alg 5 (sequential redistribute, whose
 *   output order this library reproduces), eq. neff, eq. normalise,
 *   eq. ncopies, eq. smcs_drawing_weights, eq. estimation_at_t,
 *   eq. normconst, eq. recycling.
 *
 * Conventions shared by every entry point:
 *   - Every pointer argument is a DEVICE pointer unless its name starts with
 *     h_.  The caller owns every buffer, including the workspace; the library
 *     never allocates device memory.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Every call only
 *     enqueues work on that stream and returns; nothing synchronises.
 *   - Argument errors are returned at once as the smc_status value and
 *     nothing is enqueued.  Errors found on the device (a NaN or +inf
 *     log-weight, all weights zero, bad foreign ncopies) are written to the
 *     `err` field of the device-side info block when one is given, and latch
 *     in the context until smc_sync_error() reads and clears them.
 *   - A context is not thread-safe and its calls must be issued on one stream
 *     (or on streams ordered by the caller): they share its workspace.
 *   - Row-major particle arrays: x is [n][d] elements of the configured type,
 *     i.e. n rows of row_bytes bytes.
 */
#ifndef SMC_H
#define SMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum smc_status {
    SMC_OK = 0,
    SMC_E_ARG = 1,          /* invalid argument or foreign ncopies not summing to N   */
    SMC_E_NONFINITE = 2,    /* a log-weight is NaN or +inf                              */
    SMC_E_DEGENERATE = 3,   /* every log-weight is -inf (all weights zero)              */
    SMC_E_NOMEM = 4,        /* workspace smaller than smc_workspace_bytes()             */
    SMC_E_DEVICE = 5,       /* a HIP runtime call failed                                */
    SMC_E_UNSUPPORTED = 6   /* a configuration this build does not implement            */
} smc_status;

enum { SMC_DTYPE_F32 = 0, SMC_DTYPE_F64 = 1 };
/* Targets of smc_step: the SMC sampler of Alg 2 on a Gaussian, Student-t or
 * logistic-regression posterior (random-walk proposal, L = q), or the SIR
 * particle filter of Alg 1 on the bearing-only tracking model (Sec. 5.2.2). */
enum { SMC_TARGET_NONE = 0, SMC_TARGET_GAUSS = 1, SMC_TARGET_STUDENT = 2, SMC_TARGET_LOGREG = 3,
       SMC_TARGET_BEARING = 4 };
/* Resampling trigger: the ESS rule of Alg 2 (resample when ESS < N*), always,
 * or never. */
enum { SMC_MODE_AUTO = 0, SMC_MODE_FORCE = 1, SMC_MODE_NEVER = 2 };
enum { SMC_PREC_F64 = 0, SMC_PREC_BF16 = 1 };

typedef struct smc_ctx smc_ctx; /* opaque, host-side */

/* Sampler configuration, copied at smc_init.  For resample/redistribute-only
 * use set target = SMC_TARGET_NONE; then only n, d, x_dtype, ess_num and
 * ess_den matter. */
typedef struct smc_config {
    int64_t n;               /* particles N, 1 <= N <= 2^31 - 1                       */
    int32_t d;               /* state dimension, 1 <= d <= 64 for samplers            */
    int32_t x_dtype;         /* SMC_DTYPE_*; samplers require SMC_DTYPE_F64            */
    int32_t target;          /* SMC_TARGET_*                                           */
    int32_t mode;            /* trigger used by smc_step, SMC_MODE_*                   */
    int32_t ess_num;         /* N* = ess_num / ess_den * N (Alg 2 default 1/2);        */
    int32_t ess_den;         /*   0 <= ess_num <= 16, 1 <= ess_den <= 16               */
    uint32_t sampler_id;     /* low 24 bits enter the random-number counter            */
    int32_t loglik_precision;/* SMC_PREC_* for SMC_TARGET_LOGREG                       */
    uint64_t seed;           /* Philox4x32-10 key                                      */
    double rw_sd;            /* random-walk proposal standard deviation                */
    double init_mean;        /* q0 = N(init_mean, init_sd^2 I)                         */
    double init_sd;
    double init_log_norm;    /* additive constant of log q0                            */
    double log_norm;         /* additive constant of log pi                            */
    const double *mean;      /* GAUSS: [d] target mean; BEARING: [4] mean of X0        */
    const double *prec;      /* GAUSS: [d] target precision (1 / variance)             */
    double nu, mu;           /* STUDENT (d = 1): degrees of freedom, location          */
    int64_t m_rows;          /* LOGREG: data rows M                                    */
    const void *X;           /* LOGREG: [M][d] row-major, FP64 or BF16 (precision)     */
    const double *y;         /* LOGREG: [M] labels in {0, 1}                           */
    double prior_prec;       /* LOGREG: prior N(0, I / prior_prec)                     */
    const double *obs;       /* BEARING: [n_obs] bearings, y_t used at iteration t     */
    int32_t n_obs;           /* BEARING: number of measurements (iterations allowed)   */
    int32_t lazy_reset;      /* 1: a resampling smc_step leaves logw unwritten (below)  */
    double delta;            /* BEARING: sampling period                               */
    double obs_var;          /* BEARING: bearing noise variance                        */
    double obs_log_norm;     /* BEARING: -0.5 log(2 pi obs_var)                        */
} smc_config;

/* Per-call summary written on the device (nullable everywhere). */
typedef struct smc_resample_info {
    double m;          /* max_i l_i (exact)                                         */
    double logZ;       /* log sum_i exp(l_i) (FP64, eq. normalise denominator)      */
    double ess;        /* FP64 effective sample size, eq. neff                      */
    double Z, Z2;      /* sum exp(l_i - m), sum exp(2 (l_i - m)) (FP64)             */
    uint64_t S;        /* sum of the 64-bit fixed-point weights q_i (exact)        */
    uint64_t U;        /* systematic offset, floor(r S / 2^64)                      */
    uint64_t Q2_hi, Q2_lo; /* sum q_i^2 as a 128-bit integer (exact)               */
    int32_t K;         /* fixed-point fraction bits                                 */
    int32_t resampled; /* 1 when the ESS rule (or force) chose to resample         */
    int32_t err;       /* smc_status found on the device, 0 if none                */
    int32_t pad;
    double log_c;      /* smc_step: log c_t, eq. normconst                          */
} smc_resample_info;

/* Bytes of device workspace smc_init needs for this configuration (256-byte
 * aligned base).  Returns 0 for an invalid configuration. */
size_t smc_workspace_bytes(const smc_config *h_cfg);

/* Creates a context bound to the caller's workspace.  For a sampler target
 * it also draws x0 ~ q0 and sets logw0 = log pi(x0) - log q0(x0) (Alg 2
 * initialisation); x and logw may be NULL for SMC_TARGET_NONE.  The config's
 * device arrays (mean, prec, X, y) must stay valid for the context's life. */
smc_status smc_init(smc_ctx **h_out, const smc_config *h_cfg, void *workspace,
                    size_t workspace_bytes, void *x, double *logw, void *stream);

/* One iteration t = 1, 2, ... of Alg 2 in place on (x, logw): random-walk
 * proposal and L = q reweighting (eq. smcs_drawing_weights), normalise,
 * estimate, ESS, and resampling when the configured trigger fires (then x
 * holds the redistributed particles and logw = -ln N).  est (nullable, [4d])
 * receives f_t (eq. estimation_at_t), sum w~ x^2, and the recycled estimates
 * of both (eq. recycling).  For SMC_TARGET_BEARING it is one iteration of
 * Alg 1 instead: transition proposal, likelihood weight, normalise, ESS,
 * resampling, then the weighted mean (est[0..d)) and second moment
 * (est[d..2d)) of the resampled population; info->log_c is then the log
 * evidence increment.  Returns SMC_E_ARG past the last measurement. */
smc_status smc_step(smc_ctx *ctx, void *x, double *logw, smc_resample_info *info, double *est,
                    void *stream);

/* With lazy_reset = 1 a resampling iteration does not write logw = -ln N
 * (Alg 4 reset, 8 bytes a particle); it marks the weights uniform in the
 * workspace, and the next iteration reads -ln N in place of logw.  Everything
 * else is unchanged.  smc_sync_weights writes the pending -ln N into logw (a
 * no-op otherwise); call it before reading logw between iterations.
 * Populations of at most 2048 particles always write logw. */
smc_status smc_sync_weights(smc_ctx *ctx, double *logw, void *stream);

/* nsteps >= 1 consecutive iterations of Alg 2 (Alg 1 for SMC_TARGET_BEARING),
 * enqueued one after another: results identical bit for bit to nsteps calls
 * of smc_step.  info (nullable) receives nsteps records and est (nullable)
 * nsteps blocks of 4d doubles, in iteration order.  SMC_E_ARG for nsteps < 1,
 * a misaligned pointer, or (filter) fewer measurements left than nsteps. */
smc_status smc_steps(smc_ctx *ctx, void *x, double *logw, int32_t nsteps,
                     smc_resample_info *info, double *est, void *stream);

/* Alg 4 up to ncopies on log-weights logw[n] (n = the configured N): exact
 * max, FP64 log-sum-exp and ESS, 64-bit fixed-point weights and their
 * exact integer prefix sum (tile-local prefixes plus tile offsets), the
 * integer ESS decision (mode), and
 * systematic ncopies with offset floor(r S / 2^64).  The prefix is kept in the
 * workspace for the next smc_redistribute; ncopies (nullable, int64[n]) is
 * also written when given.  When the decision is not to resample, ncopies is
 * all ones. */
smc_status smc_resample(smc_ctx *ctx, const double *logw, int64_t n, uint64_t r, int32_t mode,
                        int64_t *ncopies, smc_resample_info *info, void *stream);

/* For callers that cannot allocate device memory or create a context
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation): smc_resample on n <= SMC_NOALLOC_MAX_N log-weights with the
 * same results, bit for bit, as smc_resample with ncopies on a context of
 * that N (ess_num / ess_den as in smc_config).  Its workspace is a fixed
 * array in device memory, one per GPU (about 8.6 MB, held until the process
 * ends); calls allocate nothing.  ncopies (int64[n]) is required; info is
 * nullable and receives device-found errors (no context latches them).
 * Every call on a GPU uses that GPU's one array: calls that overlap on one
 * GPU (different streams or host threads without ordering) race and give
 * wrong results.  The device is the current one; the stream must belong to
 * it.  n > SMC_NOALLOC_MAX_N returns SMC_E_NOMEM; other argument errors
 * SMC_E_ARG. */
#define SMC_NOALLOC_MAX_N (1 << 20)
smc_status smc_resample_noalloc(const double *logw, int64_t n, uint64_t r, int32_t mode,
                                int32_t ess_num, int32_t ess_den, int64_t *ncopies,
                                smc_resample_info *info, void *stream);

/* eq. normalise: w[i] = exp(logw[i] - m) / Z, with m and the FP64 sum Z of
 * the last smc_resample on this context (call it with the same logw[n]);
 * exp is the deterministic one of the fixed-point weights.  Nothing is
 * written when that call found an error (info->err).  w must not overlap
 * logw. */
smc_status smc_normalised_weights(smc_ctx *ctx, const double *logw, int64_t n, double *w,
                                  void *stream);

/* Alg 5 semantics, load-balanced: x_out row p = x row anc(p) where the
 * ancestors are non-decreasing and source j appears ncopies_j times.
 * ncopies == NULL uses the pending result of the last smc_resample on this
 * context; otherwise the given int64[n] counts are scanned first (each >= 0,
 * summing to n, else err = SMC_E_ARG on the device and nothing is written).
 * row_bytes is a positive multiple of 4 of at most 2^20 (1 MiB), and
 * n * row_bytes at most 2^46; x_out must not overlap x.
 * ncopies_out and anc (int64[n], nullable) receive the counts and the source
 * index of every output row. */
smc_status smc_redistribute(smc_ctx *ctx, const int64_t *ncopies, const void *x, void *x_out,
                            int64_t n, int32_t row_bytes, int64_t *ncopies_out, int64_t *anc,
                            void *stream);

/* Evaluates log pi at n particles x[n][d] (FP64) into lp[n] with the
 * context's target and precision; used to check likelihood kernels. */
smc_status smc_log_target(smc_ctx *ctx, const double *x, int64_t n, double *lp, void *stream);

/* Waits for the stream, then returns and clears the context's latched device
 * error (SMC_OK if none). */
smc_status smc_sync_error(smc_ctx *ctx, void *stream);

/* Releases the host-side context (the workspace stays the caller's). */
smc_status smc_destroy(smc_ctx *ctx);

const char *smc_status_string(smc_status s);

#ifdef __cplusplus
}
#endif
#endif /* SMC_H */
