// Sampler (Alg 2) launch sequences: initialisation, one iteration, and the
// batch log-target evaluation.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/smc.h"
#include "kernels.hpp"

namespace smc {

constexpr int kMaxDim = 64;

// Grid of the sampler kernels: one full residency of the update kernel on
// this device, at most kIsBlocks and at most one block per 256 particles;
// 0 if the device cannot be queried.
int sampler_grid(const smc_config &cfg);
// par: parity of the max slots this call uses (alternates between calls).
smc_status step_init(const smc_config &cfg, const Work &w, int par, double *x, double *logw,
                     hipStream_t s);
smc_status step_run(const smc_config &cfg, const Work &w, int K, int par, uint32_t t, double *x,
                    double *logw, smc_resample_info *info, double *est, hipStream_t s);
// nsteps iterations t0, t0 + 1, ... with parities par0, par0 ^ 1, ... (one
// step_run each); info and est (nullable) receive one record per iteration.
smc_status step_run_n(const smc_config &cfg, const Work &w, int K, int par0, uint32_t t0,
                      int nsteps, double *x, double *logw, smc_resample_info *info, double *est,
                      hipStream_t s);
// Lazy reset: writes -ln N into logw when the last iteration left the weights
// marked uniform.
smc_status step_sync_weights(const smc_config &cfg, const Work &w, double *logw, hipStream_t s);
smc_status step_log_target(const smc_config &cfg, const Work &w, const double *x, int64_t n,
                           double *lp, hipStream_t s);

}  // namespace smc
