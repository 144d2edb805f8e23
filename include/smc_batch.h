/*
 * smc_batch.h -- C ABI of libsmc's batched SMC sampler: many independent
 * samplers of uneven size and dimension advanced by one shared sequence of
 * launches (segmented scans over per-sampler tiles), for throughput when each
 * sampler alone is too small to fill the GPU.
 *
 * Each sampler runs Alg 2 of Varsi et al., arXiv:1905.10252 (SMC sampler with
 * recycling: random-walk proposal, L = q so the incremental weight is
 * pi(x_t)/pi(x_{t-1}) by eq. smcs_drawing_weights, normalise and ESS by
 * eq. normalise and eq. neff, estimates by eq. estimation_at_t before
 * resampling, c_t by eq. normconst, recycling by eq. recycling) with the
 * resampling of Alg 4 (systematic ncopies in exact 64-bit fixed point, S-R
 * output order of Alg 5, reset to 1/N).  The target is a Gaussian with a full
 * precision matrix P = U^T U (U upper triangular):
 *   log pi(x) = log_norm - |U (x - mean)|^2 / 2,
 * with |U t|^2 = sum_i (sum_{k >= i} U_ik t_k)^2 summed in index order, each
 * term a fused multiply-add.
 *
 * A sampler's results depend only on its own description (seed, sampler id,
 * sizes, target), never on which other samplers share the batch: a sampler
 * run alone and in a mix gives the same bits.
 *
 * Conventions (as in smc.h): pointers are device pointers unless prefixed
 * h_; the caller owns every buffer (the batch workspace, each sampler's state
 * and workspace); calls enqueue on `stream` (a hipStream_t, NULL = null
 * stream) and return; argument errors return at once; errors found on the
 * device go to the sampler's info record.  A batch is not thread-safe.
 */
#ifndef SMC_BATCH_H
#define SMC_BATCH_H

#include <stddef.h>
#include <stdint.h>

#include "smc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smc_batch smc_batch; /* opaque, host-side */

enum { SMC_BATCH_DMAX = 64, SMC_BATCH_EST_STRIDE = 256 };

/* One sampler of a batch, copied at smc_batch_attach. */
typedef struct smc_batch_sampler {
    int64_t n;               /* particles N_s, 1 <= N_s <= 2^28                       */
    int32_t d;               /* dimension, 1 <= d <= 64                                */
    int32_t mode;            /* SMC_MODE_* resampling trigger                          */
    int32_t ess_num;         /* N* = ess_num / ess_den * N_s (Alg 2 default 1/2)       */
    int32_t ess_den;
    uint32_t sampler_id;     /* low 24 bits enter the random-number counter            */
    int32_t pad0;
    uint64_t seed;           /* Philox4x32-10 key                                      */
    double rw_sd;            /* random-walk proposal standard deviation                */
    double init_mean;        /* q0 = N(init_mean, init_sd^2 I)                         */
    double init_sd;
    double init_log_norm;    /* additive constant of log q0                            */
    double log_norm;         /* additive constant of log pi: -d/2 log 2pi + log det U  */
    const double *mean;      /* [d] target mean                                        */
    const double *chol;      /* [d][d] row-major upper-triangular U, P = U^T U          */
    double *x;               /* [N_s][d] initial particle array (FP64); see            */
                             /*   smc_batch_particles for where they are after a step   */
    double *logw;            /* [N_s] log-weights                                      */
    void *ws;                /* sampler workspace, 256-byte aligned                    */
    size_t ws_bytes;         /* >= smc_batch_sampler_bytes(this)                       */
} smc_batch_sampler;

/* Bytes of per-sampler workspace; 0 for an invalid description. */
size_t smc_batch_sampler_bytes(const smc_batch_sampler *h_s);

/* Bytes of batch workspace for `capacity` slots (1 <= capacity <= 4096). */
size_t smc_batch_workspace_bytes(int32_t capacity);

/* Creates an empty batch with `capacity` slots over the caller's workspace. */
smc_status smc_batch_create(smc_batch **h_out, int32_t capacity, void *ws, size_t ws_bytes,
                            void *stream);

/* Puts a sampler into free slot `slot` and runs its Alg 2 initialisation
 * (x0 ~ q0, logw0 = log pi(x0) - log q0(x0)).  The description's device arrays
 * must stay valid until the slot is detached.  SMC_E_ARG if the slot is taken
 * or the description is invalid. */
smc_status smc_batch_attach(smc_batch *b, int32_t slot, const smc_batch_sampler *h_s,
                            void *stream);

/* Frees a slot; the sampler's buffers are the caller's again once the work
 * already enqueued on the stream has finished. */
smc_status smc_batch_detach(smc_batch *b, int32_t slot, void *stream);

/* One iteration t = 1, 2, ... (counted per sampler from its attach) for every
 * attached sampler.  info (nullable) is indexed by slot [capacity]; est
 * (nullable) holds SMC_BATCH_EST_STRIDE doubles per slot: f_t [0, d),
 * sum w~ x^2 [d, 2d), and their recycled estimates [2d, 3d), [3d, 4d).
 * info->log_c is log c_t.  With graphs enabled (the default) the launches of
 * a step are captured once per set of attached samplers (and info/est
 * pointers) and replayed as one HIP graph. */
smc_status smc_batch_step(smc_batch *b, smc_resample_info *info, double *est, void *stream);

/* Where slot `slot`'s particles are now (waits for the stream).  Resampling
 * writes the redistributed particles into the sampler's workspace copy and
 * the two copies then alternate (no copy back), so the current particles
 * [N_s][d] and cached log-targets [N_s] are either the description's x and
 * the workspace's log-target array, or the two workspace copies.  The
 * log-weights always stay in the description's logw. */
smc_status smc_batch_particles(smc_batch *b, int32_t slot, double **h_x, double **h_lp,
                               void *stream);

/* Coordinate pairs per proposal work unit (a unit is 256 particles times
 * `pairs` pairs of coordinates; 1 <= pairs <= 8, default 8).  A tuning knob:
 * results do not depend on it. */
smc_status smc_batch_set_group(smc_batch *b, int32_t pairs, void *stream);

/* Occupancy the target kernel of smc_batch_step (the log-density and
 * weight update of eq. smcs_drawing_weights for samplers whose dimension
 * falls in bucket `bucket`, i.e. d in (8 bucket, 8 bucket + 8]) is compiled to
 * aim at: `waves` wavefronts per SIMD, 1 <= waves <= 4, bucket 0..7, clamped
 * to what the bucket's kernel can reach (4 for d <= 40, 3 above), which is
 * also the default.  Fewer waves leave more registers per
 * thread for the longer rows.  A tuning knob: results do not depend on it. */
smc_status smc_batch_set_bucket_waves(smc_batch *b, int32_t bucket, int32_t waves);

/* Enables (1) or disables (0) graph capture of the step. */
smc_status smc_batch_set_graph(smc_batch *b, int32_t enable);

/* Number of attached samplers, and the total particle tiles (4096 particles
 * each) a step covers. */
smc_status smc_batch_counts(const smc_batch *b, int32_t *h_samplers, int64_t *h_tiles);

/* Waits for the stream, then returns and clears the latched device error of
 * slot `slot` (SMC_OK if none). */
smc_status smc_batch_sync_error(smc_batch *b, int32_t slot, void *stream);

/* Releases the host-side batch (every workspace stays the caller's). */
smc_status smc_batch_destroy(smc_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* SMC_BATCH_H */
