// The sampler's per-iteration statistics as a block-level routine, shared by
// the statistics kernel and the fused decision kernel.
#pragma once

#include "../../include/smc.h"
#include "common.hpp"
#include "det.hpp"
#include "kernels.hpp"

namespace smc {

constexpr int kStatsMaxDim = 64;

// Estimates of eq. estimation_at_t, c_t (eq. normconst) and the recycling
// sums (eq. recycling) from the per-block partials of the update, by one
// workgroup of NT threads (sums in a fixed order for a given NT).
template <int NT>
__device__ inline void step_stats_block(Ctrl *ctrl, const double *is_part, int nblk, int d,
                                        double *rec_num, double *est, smc_resample_info *info,
                                        int init)
{
    constexpr int NW = NT / 64;
    __shared__ double s_col[2 + 2 * kStatsMaxDim];
    __shared__ double s_red[NW][2 + 2 * kStatsMaxDim];
    __shared__ double s_sc, s_wgt, s_den;
    __shared__ u64 s_mk[NW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int ncol = 2 + 2 * d;
    // reference: the largest block reference (blocks with no weight carry -inf)
    u64 mk = 0;
    for (int b = tid; b < nblk; b += NT) {
        const u64 k = okey(is_part[(i64)b * ncol]);
        mk = k > mk ? k : mk;
    }
    mk = wave_max_u64(mk);
    if ((tid & 63) == 0) s_mk[tid >> 6] = mk;
    __syncthreads();
    for (int i = 1; i < NW; ++i) mk = s_mk[i] > mk ? s_mk[i] : mk;
    mk = s_mk[0] > mk ? s_mk[0] : mk;
    const double m = okey_inv(mk);
    // thread tid folds blocks tid, tid + NT, ... (nblk <= kIsBlocks), then a
    // fixed-order wave and block sum per column
    constexpr int kPer = (kIsBlocks + NT - 1) / NT;
    double sc[kPer];
    for (int j = 0; j < kPer; ++j) {
        const int b = tid + NT * j;
        const double mb = b < nblk ? is_part[(i64)b * ncol] : -__builtin_huge_val();
        sc[j] = mb > -__builtin_huge_val() ? det_exp(mb - m) : 0.0;
    }
    // four columns at a time: their loads are all issued before the first
    // sum waits on them (the per-column sums and their order are unchanged)
    constexpr int CU = 4;
    for (int c0 = 1; c0 < ncol; c0 += CU) {
        double v[CU][kPer];
#pragma unroll
        for (int q = 0; q < CU; ++q)
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                const int b = tid + NT * j;
                v[q][j] = (c0 + q < ncol && b < nblk && sc[j] != 0.0)
                              ? is_part[(i64)b * ncol + c0 + q]
                              : 0.0;
            }
#pragma unroll
        for (int q = 0; q < CU; ++q) {
            if (c0 + q >= ncol) break;
            double acc = 0.0;
            for (int j = 0; j < kPer; ++j) {
                const int b = tid + NT * j;
                if (b < nblk && sc[j] != 0.0) acc += sc[j] * v[q][j];
            }
            acc = wave_sum_f64(acc);
            if (lane == 0) s_red[wid][c0 + q] = acc;
        }
    }
    __syncthreads();
    for (int c = 1 + tid; c < ncol; c += NT) {
        double v = s_red[0][c];
        for (int w = 1; w < NW; ++w) v += s_red[w][c];
        s_col[c] = v;
    }
    __syncthreads();
    const double E0 = s_col[1];
    if (init) {
        if (tid == 0) {
            ctrl->logZ_prev = m + log(E0);
            ctrl->lc_max = -__builtin_huge_val();
            ctrl->rec_den = 0.0;
            ctrl->rec_steps = 0;
        }
        for (int c = tid; c < 2 * d; c += NT) rec_num[c] = 0.0;
        return;
    }
    // an iteration whose decision found an error (NaN / +inf weight, all
    // weights zero) leaves c_t, the recycling sums and the estimates as they
    // were, as the iteration stops at the resampling step
    __shared__ unsigned s_err;
    if (tid == 0) s_err = ctrl->err_call;
    __syncthreads();
    if (s_err) return;
    if (tid == 0) {
        const double logc = ctrl->logZ - ctrl->logZ_prev;
        double sc = 1.0;
        double den = ctrl->rec_den;
        if (logc > ctrl->lc_max) {
            sc = ctrl->rec_steps ? exp(ctrl->lc_max - logc) : 0.0;
            den *= sc;
            ctrl->lc_max = logc;
        }
        const double wgt = exp(logc - ctrl->lc_max);
        den += wgt;
        ctrl->rec_den = den;
        ctrl->rec_steps += 1;
        ctrl->log_c = logc;
        ctrl->logZ_prev = ctrl->resample ? 0.0 : ctrl->logZ;
        s_sc = sc;
        s_wgt = wgt;
        s_den = den;
        if (info) info->log_c = logc;
    }
    __syncthreads();
    for (int k = tid; k < 2 * d; k += NT) {
        const double f = s_col[2 + k] / E0;
        const double num = rec_num[k] * s_sc + s_wgt * f;
        rec_num[k] = num;
        if (est) {
            est[k] = f;
            est[2 * d + k] = num / s_den;
        }
    }
}


}  // namespace smc
