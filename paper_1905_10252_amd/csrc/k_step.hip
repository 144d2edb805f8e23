#include "step.hpp"

namespace smc {

smc_status step_init(const smc_config &, const Work &, double *, double *, hipStream_t)
{
    return SMC_E_UNSUPPORTED;
}
smc_status step_run(const smc_config &, const Work &, int, uint32_t, double *, double *,
                    smc_resample_info *, double *, hipStream_t)
{
    return SMC_E_UNSUPPORTED;
}
smc_status step_log_target(const smc_config &, const Work &, const double *, int64_t, double *,
                           hipStream_t)
{
    return SMC_E_UNSUPPORTED;
}

}  // namespace smc
