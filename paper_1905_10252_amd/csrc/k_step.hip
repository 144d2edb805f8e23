// Sampler kernels of Alg 2 (SMC sampler with recycling), random-walk proposal
// and backward kernel L = q (so the incremental weight is pi(x_t)/pi(x_{t-1}),
// eq. smcs_drawing_weights):
//   k_is<target, init>  draws x0 ~ q0 or x_t = x_{t-1} + rw_sd z, evaluates the
//                       cheap targets, updates the log-weights, and leaves per
//                       block estimate sums (block-local max) and the grid max.
//   k_reweight<init>    the weight update for targets whose log-density comes
//                       from a separate likelihood kernel.
//   k_step_stats        estimates f_t (eq. estimation_at_t), c_t
//                       (eq. normconst) and the recycled estimate
//                       (eq. recycling).
//   k_copyback          after an in-place update and redistribute: particles
//                       and cached log-target back in place, weights reset to
//                       1/N (Alg 4 Reset).
//   k_reset_est         after a redistribution straight into x: the reset,
//                       and for the filter the post-resampling sums.
//   k_is<BEARING>       one SIR particle-filter update (Alg 1, Sec. 5.2.2):
//                       constant-velocity transition as proposal, bearing
//                       likelihood as weight; the expand then adds up the rows
//                       it writes for the mean of the resampled population.
//   k_logreg_f64 / k_logreg_bf16 + k_logreg_sum
//                       Bayesian logistic regression log-likelihood
//                       sum_m [y_m z_m - softplus(z_m)], z = X theta, in FP64 or
//                       as a BF16 MFMA contraction with FP32 accumulation.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/smc.h"
#include "common.hpp"
#include "det.hpp"
#include "kernels.hpp"
#include "reduce.hpp"
#include "rng_wave.hpp"
#include "stats.hpp"
#include "step.hpp"

static_assert(smc::kStatsMaxDim == smc::kMaxDim, "statistics width");

namespace smc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

struct TArgs {
    int kind, d, dp;
    const double *mean, *prec;
    double log_norm, mu, inv_nu, hnu1;
    double init_mean, init_sd, init_prec, init_log_norm, rw_sd;
    uint64_t seed;
    uint32_t sampler;
    unsigned short *thb;  // bf16 copy of the particles times log2 e [npad][dp] (nullable)
    // bearing-only particle filter
    const unsigned *uniform;  // lazy reset flag (NULL: weights always in logw)
    const double *obs;    // measurements, y_t = obs[t - 1]
    double delta, l11, l21, l22, obs_prec, obs_log_norm, reset;
};

__device__ inline unsigned short to_bf16(double v)
{
    const float f = (float)v;
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ inline double from_bf16(unsigned short h) { return (double)__uint_as_float((unsigned)h << 16); }

// The BF16 likelihood works in base 2: the bf16 particles hold theta log2 e, so
// that the MFMA yields t log2 e and the epilogue's exponentials need no scaling.
constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;

// ------------------------------------------------------------------ partials
// Per-block sums for the estimates with the block's own max (rescaled later):
// part = [m_b, sum e, sum e x_k (k < d), sum e x_k^2 (k < d)], e = exp(l - m_b).
__device__ inline void is_block_finish(i64 n, int d, const double *x, const double *logw, u64 key,
                                       unsigned bad, u64 *slots_p, double *is_part)
{
    __shared__ double s_acc[4][2 + 2 * kMaxDim];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const i64 gtid = (i64)blockIdx.x * 256 + tid, gsz = (i64)gridDim.x * 256;
    const u64 bk = block_max_key(key, bad);
    const double mb = okey_inv(bk);
    const bool live = mb > -__builtin_huge_val() && mb == mb;
    double e0 = 0.0;
    for (i64 i = gtid; i < n; i += gsz) e0 += live ? det_exp(logw[i] - mb) : 0.0;
    e0 = wave_sum_f64(e0);
    if (lane == 0) s_acc[wid][1] = e0;
    for (int k = 0; k < d; ++k) {
        double s1 = 0.0, s2 = 0.0;
        for (i64 i = gtid; i < n; i += gsz) {
            const double e = live ? det_exp(logw[i] - mb) : 0.0;
            const double ex = e * x[i * d + k];
            s1 += ex;
            s2 += ex * x[i * d + k];
        }
        s1 = wave_sum_f64(s1);
        s2 = wave_sum_f64(s2);
        if (lane == 0) {
            s_acc[wid][2 + k] = s1;
            s_acc[wid][2 + d + k] = s2;
        }
    }
    __syncthreads();
    const int ncol = 2 + 2 * d;
    double *part = is_part + (i64)blockIdx.x * ncol;
    for (int c = tid; c < ncol; c += 256)
        part[c] = c == 0 ? mb : ((s_acc[0][c] + s_acc[1][c]) + s_acc[2][c]) + s_acc[3][c];
    slot_publish(slots_p, bk, bad);
}

// One-pass variant for small d (the row stays in registers): each thread keeps
// a reference and sums e = exp(l - ref), so the rows are read once; blocks
// combine the thread references by det_exp rescaling.  The reference is the
// first finite weight and moves (rescaling the sums) only when a weight exceeds
// it by more than kOnlineSlack nats: terms stay below e^64, far from FP64
// overflow, and a lane no longer pays a second exponential at every new
// maximum, which in a wave of 64 lanes happened on most iterations.
constexpr double kOnlineSlack = 64.0;

template <int DT>
struct Online {
    double m, e0, e1[DT], e2[DT];
    __device__ void init()
    {
        m = -__builtin_huge_val();
        e0 = 0.0;
        for (int k = 0; k < DT; ++k) e1[k] = e2[k] = 0.0;
    }
    __device__ void add(double lw, const double *xv)
    {
        if (!(lw > -__builtin_huge_val())) return;  // zero weight, or NaN (flagged elsewhere)
        if (lw > m + kOnlineSlack) {
            if (m > -__builtin_huge_val()) {
                const double sc = det_exp(m - lw);
                e0 *= sc;
                for (int k = 0; k < DT; ++k) {
                    e1[k] *= sc;
                    e2[k] *= sc;
                }
            }
            m = lw;
        }
        const double e = det_exp(lw - m);
        e0 += e;
        for (int k = 0; k < DT; ++k) {
            const double ex = e * xv[k];
            e1[k] += ex;
            e2[k] += ex * xv[k];
        }
    }
    // Block combine into part = [m_b, sum e, sum e x_k, sum e x_k^2].
    __device__ void finish(double *part)
    {
        __shared__ double s_m[4], s_acc[4][1 + 2 * DT];
        const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
        const double mw = wave_max_f64(m);
        const double sc = m > -__builtin_huge_val() ? det_exp(m - mw) : 0.0;
        const double a0 = wave_sum_f64(e0 * sc);
        double a1[DT], a2[DT];
        for (int k = 0; k < DT; ++k) {
            a1[k] = wave_sum_f64(e1[k] * sc);
            a2[k] = wave_sum_f64(e2[k] * sc);
        }
        if (lane == 0) {
            s_m[wid] = mw;
            s_acc[wid][0] = a0;
            for (int k = 0; k < DT; ++k) {
                s_acc[wid][1 + k] = a1[k];
                s_acc[wid][1 + DT + k] = a2[k];
            }
        }
        __syncthreads();
        if (tid == 0) {
            double mb = s_m[0];
            for (int w = 1; w < 4; ++w) mb = fmax(mb, s_m[w]);
            double scw[4];
            for (int w = 0; w < 4; ++w)
                scw[w] = s_m[w] > -__builtin_huge_val() ? det_exp(s_m[w] - mb) : 0.0;
            part[0] = mb;
            for (int c = 0; c < 1 + 2 * DT; ++c) {
                double v = 0.0;
                for (int w = 0; w < 4; ++w) v += scw[w] * s_acc[w][c];
                part[1 + c] = v;
            }
        }
    }
};

// ------------------------------------------------------- proposal + weights
typedef double f64x2s __attribute__((ext_vector_type(2)));
// DT > 0: d == DT and the estimate sums are accumulated in one pass; DT == 0:
// any d, sums in a second pass over the block's particles.  The particle filter
// takes its estimate after resampling, so its update kernel skips them.
// kOut: the proposal and its log-target go to xo / lpo (the redistribution
// then maps them back into x); otherwise they overwrite x / lp in place.
// At least four waves per SIMD (up to 128 VGPRs): the 1-D Gaussian and
// Student-t updates need 102-110 VGPRs and the 4-D Gaussian ones 116-119;
// held to 96 for five waves they spilled 20-92 bytes a lane, and the Student-t
// iteration at N = 2^24 ran 6 % slower.  The other instances need fewer
// registers and keep six or seven waves.
template <int kKind, bool kInit, int DT, bool kOut>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_is(
    TArgs a, i64 n, uint32_t t, double *__restrict__ x, double *__restrict__ logw,
    double *__restrict__ lp, u64 *slots_p, double *is_part, double *__restrict__ xo,
    double *__restrict__ lpo)
{
    constexpr bool kEst = kKind != SMC_TARGET_BEARING;
    constexpr int DA = DT > 0 ? DT : 1;
    __shared__ uint4 s_xch[4][64];  // normal generator exchange, one row per wave
    const int tid = threadIdx.x;
    const i64 gtid = (i64)blockIdx.x * 256 + tid, gsz = (i64)gridDim.x * 256;
    const int d = DT == 1 ? 1 : a.d;  // DT > 0 is launched only for d == DT
    const bool uni = !kInit && a.uniform && *a.uniform;  // lazy reset: weights are -ln N
    const uint32_t tag = kInit ? (uint32_t)kTagInit : (uint32_t)kTagPropose;
    const uint32_t tt_ = kInit ? 0u : t;
    u64 key = 0;
    unsigned bad = 0;
    Online<DA> on;
    on.init();
    double xv[DA];
    // The weight and what follows it, for particle i whose new row is xw
    // (and, with DT > 0, also in xv); acc and acc0 are the quadratic forms of
    // the Gaussian target and of q0.
    auto tail = [&](i64 i, const double *xw, double acc, double acc0) {
        const double lq0 = kInit ? a.init_log_norm - 0.5 * acc0 : 0.0;
        if (kKind == SMC_TARGET_LOGREG) {
            if (kInit) logw[i] = lq0;  // combined with log pi by k_reweight
            return;
        }
        double lpn;
        if (kKind == SMC_TARGET_GAUSS) {
            lpn = a.log_norm - 0.5 * acc;
        } else {
            const double tt = xw[0] - a.mu;
            const double w = 1.0 + (tt * tt) * a.inv_nu;
            lpn = a.log_norm - a.hnu1 * det_log(w);
        }
        const double lw = kInit ? lpn - lq0 : (uni ? a.reset : logw[i]) + (lpn - lp[i]);
        (kOut ? lpo : lp)[i] = lpn;
        logw[i] = lw;
        bad |= (lw != lw) | (lw == __builtin_huge_val());
        const u64 kk = okey(lw);
        key = kk > key ? kk : key;
        if (DT > 0) on.add(lw, xv);
    };
    // Log-target of a 1-D particle of the Gaussian or Student-t target: the
    // same operations as tail's, so a value recomputed from a particle equals
    // the one computed when the particle was proposed, bit for bit.
    auto lpt1 = [&](double v) {
        if (kKind == SMC_TARGET_GAUSS) {
            const double tt = v - a.mean[0];
            return a.log_norm - 0.5 * ((tt * tt) * a.prec[0]);
        }
        const double tt = v - a.mu;
        const double w = 1.0 + (tt * tt) * a.inv_nu;
        return a.log_norm - a.hnu1 * det_log(w);
    };
    // tail's weight for such a particle with new value xk, previous weight
    // lw_old and previous log-target lp_old; returns the weight, lpn the new
    // log-target.
    auto weigh1 = [&](double xk, double lw_old, double lp_old, double &lpn) {
        double lq0 = 0.0;
        if (kInit) {
            const double t0 = xk - a.init_mean;
            lq0 = a.init_log_norm - 0.5 * ((t0 * t0) * a.init_prec);
        }
        lpn = lpt1(xk);
        const double lw = kInit ? lpn - lq0 : lw_old + (lpn - lp_old);
        bad |= (lw != lw) | (lw == __builtin_huge_val());
        const u64 kk = okey(lw);
        key = kk > key ? kk : key;
        if (DT > 0) {
            xv[0] = xk;
            on.add(lw, xv);
        }
        return lw;
    };
    constexpr bool kMay1 = kKind != SMC_TARGET_BEARING && DT <= 1;  // d == 1 possible
    if (kMay1 && d == 1) {
        // One coordinate a particle: particles 2p and 2p + 1 take the two
        // values of the pair drawn for index p, so each lane draws one pair
        // for two particles (a wave-uniform trip count over the pairs).  The
        // Gaussian and Student-t targets keep no cached log-target here: the
        // previous one is recomputed from the particle (for the Student-t one
        // more logarithm, against 16 bytes less read and written per particle
        // here and in the redistribution, which then moves 8-byte rows only).
        // The initial pass still writes it, for the one-workgroup iteration
        // that small populations step with.
        const i64 np = (n + 1) >> 1;
        // v2 (n even, 16-byte aligned arrays, Gaussian or Student-t target): a
        // lane moves its two particles' values as one 16-byte access per
        // array, so every wave instruction uses whole cache lines (about 2 %
        // faster per iteration at N = 2^24); otherwise 8-byte accesses
        const uintptr_t al = (uintptr_t)x | (uintptr_t)logw | (uintptr_t)lp | (uintptr_t)xo |
                             (uintptr_t)lpo;
        const bool v2 = kKind != SMC_TARGET_LOGREG && (n & 1) == 0 && (al & 15) == 0 &&
                        a.thb == nullptr;
        for (i64 base = gtid - (tid & 63); base < np; base += gsz) {
            const i64 p = base + (tid & 63);
            const bool pact = p < np;
            // the pair's rows are requested before the normals are drawn, so the
            // loads overlap the generator (the empty asm keeps the compiler from
            // sinking them into their use): about 1 % faster
            double xa0 = 0.0, xa1 = 0.0;
            if (v2) {
                const i64 pc = pact ? p : np - 1;
                if (!kInit) {
                    const f64x2s v = *reinterpret_cast<const f64x2s *>(x + 2 * pc);
                    xa0 = v[0];
                    xa1 = v[1];
                }
            } else if (!kInit) {
                const i64 ic0 = 2 * p < n ? 2 * p : n - 1, ic1 = 2 * p + 1 < n ? 2 * p + 1 : n - 1;
                xa0 = x[ic0];
                xa1 = x[ic1];
            }
            asm volatile("" ::: "memory");
            double z[2];
            normal_pair_wave(a.seed, tag, a.sampler, tt_, (uint32_t)p, 0u, pact, z[0], z[1],
                             s_xch[tid >> 6]);
            if (!pact) continue;
            if (v2) {
                double lwa = a.reset, lwb = a.reset;
                if (!kInit && !uni) {
                    const f64x2s w = *reinterpret_cast<const f64x2s *>(logw + 2 * p);
                    lwa = w[0];
                    lwb = w[1];
                }
                double xn0 = 0.0, xn1 = 0.0, lw0 = 0.0, lw1 = 0.0;
#pragma unroll 1
                for (int h = 0; h < 2; ++h) {
                    const double zh = h == 0 ? z[0] : z[1];
                    const double xh = h == 0 ? xa0 : xa1;
                    const double xk = kInit ? a.init_mean + a.init_sd * zh : xh + a.rw_sd * zh;
                    double lpn;
                    const double lw = weigh1(xk, h == 0 ? lwa : lwb, kInit ? 0.0 : lpt1(xh), lpn);
                    // the one-workgroup iteration (N <= 2048) reads the cache
                    if (kInit) lp[2 * p + h] = lpn;
                    if (h == 0) {
                        xn0 = xk;
                        lw0 = lw;
                    } else {
                        xn1 = xk;
                        lw1 = lw;
                    }
                }
                *reinterpret_cast<f64x2s *>((kOut ? xo : x) + 2 * p) = f64x2s{xn0, xn1};
                *reinterpret_cast<f64x2s *>(logw + 2 * p) = f64x2s{lw0, lw1};
                continue;
            }
            if constexpr (kKind != SMC_TARGET_LOGREG) {
#pragma unroll 1
                for (int h = 0; h < 2; ++h) {
                    const i64 i = 2 * p + h;
                    if (i >= n) break;
                    const double zh = h == 0 ? z[0] : z[1];
                    const double xh = h == 0 ? xa0 : xa1;
                    const double xk = kInit ? a.init_mean + a.init_sd * zh : xh + a.rw_sd * zh;
                    (kOut ? xo : x)[i] = xk;
                    const double lw_old = (kInit || uni) ? a.reset : logw[i];
                    double lpn;
                    logw[i] = weigh1(xk, lw_old, kInit ? 0.0 : lpt1(xh), lpn);
                    if (kInit) lp[i] = lpn;
                }
                continue;
            }
            // logistic regression: the likelihood kernels take its weight
#pragma unroll 1
            for (int h = 0; h < 2; ++h) {
                const i64 i = 2 * p + h;
                if (i >= n) break;
                double *xw = (kOut ? xo : x) + i;
                const double zh = h == 0 ? z[0] : z[1];
                const double xh = h == 0 ? xa0 : xa1;
                const double xk = kInit ? a.init_mean + a.init_sd * zh : xh + a.rw_sd * zh;
                xw[0] = xk;
                if (DT > 0) xv[0] = xk;
                if (a.thb) a.thb[i * a.dp] = to_bf16(xk * kLog2e);
                double acc = 0.0, acc0 = 0.0;
                if (kKind == SMC_TARGET_GAUSS) {
                    const double tt = xk - a.mean[0];
                    acc = acc + (tt * tt) * a.prec[0];
                }
                if (kInit) {
                    const double t0 = xk - a.init_mean;
                    acc0 = acc0 + (t0 * t0) * a.init_prec;
                }
                tail(i, xw, acc, acc0);
            }
        }
    }
    // wave-uniform trip count: the normal generator is wave-cooperative
    for (i64 base = gtid - (tid & 63); base < (kMay1 && d == 1 ? 0 : n); base += gsz) {
        const i64 i = base + (tid & 63);
        const bool act = i < n;
        double *xi = x + i * d;
        double *xw = (kOut ? xo : x) + i * d;
        if (kKind == SMC_TARGET_BEARING) {
            double z[4];
            // the particle's state and weight are requested before the
            // normals are drawn, so the loads overlap the generator
            const i64 ic = act ? i : 0;
            const double s0 = kInit ? 0.0 : x[ic * 4], s1 = kInit ? 0.0 : x[ic * 4 + 1];
            const double s2 = kInit ? 0.0 : x[ic * 4 + 2], s3 = kInit ? 0.0 : x[ic * 4 + 3];
            const double lw0 = (kInit || uni) ? 0.0 : logw[ic];
            asm volatile("" ::: "memory");
            // coefficients as scalar operands (coef()): 1.5 % faster here;
            // no gain for the other targets, whose uniform values already
            // fill the scalar registers
            normal_pair_wave<true>(a.seed, tag, a.sampler, tt_, (uint32_t)i, 0u, act, z[0], z[1],
                                   s_xch[tid >> 6]);
            normal_pair_wave<true>(a.seed, tag, a.sampler, tt_, (uint32_t)i, 1u, act, z[2], z[3],
                                   s_xch[tid >> 6]);
            if (!act) continue;
            double lw;
            if (kInit) {
                for (int k = 0; k < 4; ++k) xi[k] = a.mean[k] + a.init_sd * z[k];
                lw = a.reset;
                lp[i] = 0.0;
            } else {
                const double v0 = a.l11 * z[0];
                const double v1 = a.l21 * z[0] + a.l22 * z[1];
                const double v2 = a.l11 * z[2];
                const double v3 = a.l21 * z[2] + a.l22 * z[3];
                const double n0 = (s0 + a.delta * s1) + v0;
                const double n1 = s1 + v1;
                const double n2 = (s2 + a.delta * s3) + v2;
                const double n3 = s3 + v3;
                xw[0] = n0;
                xw[1] = n1;
                xw[2] = n2;
                xw[3] = n3;
                const double e = a.obs[t - 1] - det_atan<true>(n2 / n0);
                lw = (uni ? a.reset : lw0) + (a.obs_log_norm - 0.5 * ((e * e) * a.obs_prec));
            }
            logw[i] = lw;
            bad |= (lw != lw) | (lw == __builtin_huge_val());
            const u64 kk = okey(lw);
            key = kk > key ? kk : key;
            continue;
        }
        double acc = 0.0, acc0 = 0.0;
        for (int k = 0; 2 * k < d; ++k) {
            double z[2];
            normal_pair_wave(a.seed, tag, a.sampler, tt_, (uint32_t)i, (uint32_t)k, act, z[0],
                             z[1], s_xch[tid >> 6]);
            if (!act) continue;
            for (int h = 0; h < 2; ++h) {
                const int kk = 2 * k + h;
                if (kk >= d) break;
                const double xk = kInit ? a.init_mean + a.init_sd * z[h] : xi[kk] + a.rw_sd * z[h];
                xw[kk] = xk;
                if (DT > 0 && kk < DT) xv[kk] = xk;
                if (a.thb) a.thb[i * a.dp + kk] = to_bf16(xk * kLog2e);
                if (kKind == SMC_TARGET_GAUSS) {
                    const double tt = xk - a.mean[kk];
                    acc = acc + (tt * tt) * a.prec[kk];
                }
                if (kInit) {
                    const double t0 = xk - a.init_mean;
                    acc0 = acc0 + (t0 * t0) * a.init_prec;
                }
            }
        }
        if (!act) continue;
        tail(i, xw, acc, acc0);
    }
    if (kKind == SMC_TARGET_LOGREG) return;
    if (!kEst || DT > 0) {
        const u64 bk = block_max_key(key, bad);
        if (kEst) on.finish(is_part + (i64)blockIdx.x * (2 + 2 * DA));
        slot_publish(slots_p, bk, bad);
        return;
    }
    is_block_finish(n, d, kOut ? xo : x, logw, key, bad, slots_p, is_part);
}

template <bool kInit>
__global__ __launch_bounds__(256) void k_reweight(i64 n, int d, const double *__restrict__ x,
                                                  const double *__restrict__ lp_new,
                                                  double *__restrict__ logw,
                                                  double *__restrict__ lp, u64 *slots_p,
                                                  double *is_part, const unsigned *uniform,
                                                  double reset)
{
    const int tid = threadIdx.x;
    const i64 gtid = (i64)blockIdx.x * 256 + tid, gsz = (i64)gridDim.x * 256;
    const bool uni = !kInit && uniform && *uniform;
    u64 key = 0;
    unsigned bad = 0;
    for (i64 i = gtid; i < n; i += gsz) {
        const double lpn = lp_new[i];
        const double lw = kInit ? lpn - logw[i] : (uni ? reset : logw[i]) + (lpn - lp[i]);
        lp[i] = lpn;
        logw[i] = lw;
        bad |= (lw != lw) | (lw == __builtin_huge_val());
        const u64 kk = okey(lw);
        key = kk > key ? kk : key;
    }
    is_block_finish(n, d, x, logw, key, bad, slots_p, is_part);
}

// -------------------------------------------- estimates, c_t and recycling
template <int NT>
__global__ __launch_bounds__(NT) void k_step_stats(Ctrl *ctrl, const double *is_part, int nblk,
                                                   int d, double *rec_num, double *est,
                                                   smc_resample_info *info, int init)
{
    step_stats_block<NT>(ctrl, is_part, nblk, d, rec_num, est, info, init);
}

// uniform (lazy reset): instead of writing logw, mark the weights uniform.
__global__ __launch_bounds__(256) void k_copyback(Ctrl *ctrl, i64 n, int d, double *x,
                                                  const double *x_scr, double *lp,
                                                  const double *lp_scr, double *logw,
                                                  double reset, unsigned *uniform)
{
    if (!ctrl->resample || ctrl->err_call) return;
    const i64 gtid = (i64)blockIdx.x * 256 + threadIdx.x, gsz = (i64)gridDim.x * 256;
    for (i64 i = gtid; i < n * d; i += gsz) x[i] = x_scr[i];
    for (i64 i = gtid; i < n; i += gsz) {
        if (lp_scr) lp[i] = lp_scr[i];
        if (!uniform) logw[i] = reset;
    }
    if (uniform && gtid == 0) *uniform = 1u;
}

// After a redistribution straight into x: weights reset to 1/N when it
// resampled; with DT > 0 (the particle filter) also the post-resampling sums
// of Alg 1: when resampled, the equal-weight sums the expand formed from the
// rows it wrote (epart, one row per expand workgroup; NULL when x was not
// 16-byte aligned for it), gathered into block b's row from workgroups
// b, b + grid, ... in that order; else read from x, with equal weights when
// resampled and the current ones against the exact max otherwise.  A step that found an error
// redistributes nothing: the proposal (and its log-target) is copied into
// place instead, as the in-place update would have left it.
template <int DT>
__global__ __launch_bounds__(256) void k_reset_est(const Ctrl *ctrl, i64 n, int d,
                                                   double *__restrict__ x,
                                                   const double *__restrict__ x_scr,
                                                   double *__restrict__ lp,
                                                   const double *__restrict__ lp_scr,
                                                   double *__restrict__ logw, double reset,
                                                   double *is_part, const double *epart,
                                                   i64 nseg, unsigned *uniform)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const i64 gtid = (i64)blockIdx.x * 256 + tid, gsz = (i64)gridDim.x * 256;
    if (ctrl->err_call) {
        for (i64 e = gtid; e < n * d; e += gsz) x[e] = x_scr[e];
        if (lp_scr)
            for (i64 i = gtid; i < n; i += gsz) lp[i] = lp_scr[i];
        if (DT > 0 && tid == 0) {  // no estimate for a failed step
            double *part = is_part + (i64)blockIdx.x * (2 + 2 * DT);
            part[0] = -__builtin_huge_val();
            for (int c = 1; c < 2 + 2 * DT; ++c) part[c] = 0.0;
        }
        return;
    }
    const bool rs = ctrl->resample;
    // lazy reset: the weights are marked uniform instead of written
    const bool wr = rs && !uniform;
    if (rs && uniform && gtid == 0) *uniform = 1u;
    if (DT == 0) {
        if (wr)
            for (i64 i = gtid; i < n; i += gsz) logw[i] = reset;
        return;
    }
    constexpr int DA = DT > 0 ? DT : 1;
    if (rs && epart) {
        static_assert(DT == 0 || 2 + 2 * DA == kEstCols, "filter row layout");
        if (wr)
            for (i64 i = gtid; i < n; i += gsz) logw[i] = reset;
        if (tid < kEstCols) {
            double v = 0.0;
            for (i64 g = blockIdx.x; g < nseg; g += gridDim.x) v += epart[g * kEstCols + tid];
            is_part[(i64)blockIdx.x * kEstCols + tid] = tid == 0 ? reset : v;
        }
        return;
    }
    __shared__ double s_acc[4][1 + 2 * DA];
    const double m = rs ? reset : ctrl->m;
    double e0 = 0.0, e1[DA], e2[DA];
    for (int k = 0; k < DA; ++k) e1[k] = e2[k] = 0.0;
    for (i64 i = gtid; i < n; i += gsz) {
        double e = 1.0;
        if (rs) {
            if (wr) logw[i] = reset;
        } else {
            e = det_exp(logw[i] - m);
        }
        e0 += e;
        for (int k = 0; k < DA; ++k) {
            const double xk = x[i * DA + k];
            const double ex = e * xk;
            e1[k] += ex;
            e2[k] += ex * xk;
        }
    }
    e0 = wave_sum_f64(e0);
    for (int k = 0; k < DA; ++k) {
        e1[k] = wave_sum_f64(e1[k]);
        e2[k] = wave_sum_f64(e2[k]);
    }
    if (lane == 0) {
        s_acc[wid][0] = e0;
        for (int k = 0; k < DA; ++k) {
            s_acc[wid][1 + k] = e1[k];
            s_acc[wid][1 + DA + k] = e2[k];
        }
    }
    __syncthreads();
    double *part = is_part + (i64)blockIdx.x * (2 + 2 * DA);
    for (int c = tid; c < 2 + 2 * DA; c += 256)
        part[c] = c == 0 ? m : ((s_acc[0][c - 1] + s_acc[1][c - 1]) + s_acc[2][c - 1]) +
                                   s_acc[3][c - 1];
}

// Weighted sums of the population after resampling (Alg 1 takes its mean
// after the resampling step), in the block-partial layout of is_block_finish
// with one common reference weight.
template <int DT>
__global__ __launch_bounds__(256) void k_post_est(const Ctrl *ctrl, i64 n, int d,
                                                  const double *__restrict__ x,
                                                  const double *__restrict__ logw, double reset,
                                                  double *is_part)
{
    __shared__ double s_acc[4][1 + 2 * DT];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const i64 gtid = (i64)blockIdx.x * 256 + tid, gsz = (i64)gridDim.x * 256;
    const double m = (ctrl->resample && !ctrl->err_call) ? reset : ctrl->m;
    double e0 = 0.0, e1[DT], e2[DT];
    for (int k = 0; k < DT; ++k) e1[k] = e2[k] = 0.0;
    for (i64 i = gtid; i < n; i += gsz) {
        const double e = det_exp(logw[i] - m);
        e0 += e;
        for (int k = 0; k < DT; ++k) {
            const double xk = x[i * DT + k];
            const double ex = e * xk;
            e1[k] += ex;
            e2[k] += ex * xk;
        }
    }
    e0 = wave_sum_f64(e0);
    for (int k = 0; k < DT; ++k) {
        e1[k] = wave_sum_f64(e1[k]);
        e2[k] = wave_sum_f64(e2[k]);
    }
    if (lane == 0) {
        s_acc[wid][0] = e0;
        for (int k = 0; k < DT; ++k) {
            s_acc[wid][1 + k] = e1[k];
            s_acc[wid][1 + DT + k] = e2[k];
        }
    }
    __syncthreads();
    double *part = is_part + (i64)blockIdx.x * (2 + 2 * DT);
    for (int c = tid; c < 2 + 2 * DT; c += 256)
        part[c] = c == 0 ? m : ((s_acc[0][c - 1] + s_acc[1][c - 1]) + s_acc[2][c - 1]) +
                                   s_acc[3][c - 1];
}


// ------------------------------------------------- small-N fused iteration
// One workgroup of 1024 threads runs a whole iteration of Alg 2 for N <= 2048
// particles of a cheap target (Gaussian d <= 16, Student-t): proposal and
// weights, exact max, fixed-point weights and their inclusive prefix in LDS,
// FP64 sums, estimates, the integer decision, c_t and recycling, then the
// redistribution (ancestor by binary search on the LDS prefix) and reset.
// Same arithmetic per particle and same integers as the multi-kernel path;
// only the order of the FP64 sums differs.  It keeps the control block as
// the multi-kernel path does and clears the other parity's max slots.
constexpr int kSmallN = 2048, kSmallD = 16, kSmallT = 1024, kSmallI = kSmallN / kSmallT;

template <int CTRL>
__device__ inline double sdpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// sum of each 16-lane row, in the row's last lane (DPP only, no LDS trips)
__device__ inline double srow16(double v)
{
    v += sdpp_f64<0x111>(v);
    v += sdpp_f64<0x112>(v);
    v += sdpp_f64<0x114>(v);
    v += sdpp_f64<0x118>(v);
    return v;
}

// One whole iteration t of a population of at most kSmallN particles by one
// workgroup of kSmallT threads.  kD1 (d = 1): each thread keeps its items'
// new coordinate and log-target in registers, and the redistribution gathers
// them from LDS (no scratch rows in global memory).
template <int kKind, bool kD1>
__device__ __forceinline__ void small_iteration(const TArgs &a, i64 n, uint32_t t, int K,
                                                int mode, int ess_num, int ess_den,
                                                double *__restrict__ x,
                                                double *__restrict__ logw,
                                                double *__restrict__ lp,
                                                double *__restrict__ x_scr,
                                                double *__restrict__ lp_scr, Ctrl *ctrl,
                                                double *rec_num, smc_resample_info *info,
                                                double *est, double reset)
{
    constexpr int NW = kSmallT / 64;  // waves of the block
    __shared__ double s_e[kSmallN];
    __shared__ u64 s_S[kSmallN];
    __shared__ double s_col[NW][2 * kSmallD];
    __shared__ uint4 s_xch[NW][64];
    __shared__ double s_tot[2 * kSmallD];
    __shared__ double s_z[16], s_z2[16];
    __shared__ u64 s_key[16], s_wsum[16], s_lo[16], s_hi[16];
    __shared__ unsigned s_bad[16];
    __shared__ double s_bc[4];
    __shared__ u64 s_bu[4];
    __shared__ double s_lpv[kD1 ? kSmallN : 1];
    constexpr int DM = kD1 ? 1 : kSmallD;  // coordinates a thread handles
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int d = kD1 ? 1 : a.d;
    const u64 r = resample_word(a.seed, a.sampler, t);
    double xr[kSmallI], lpr[kSmallI];  // kD1: the items' new x and log-target

    // proposal and weights (items tid + 1024 j; with d = 1 items 2 tid + j,
    // the two particles that share the pair drawn for index tid)
    static_assert(kSmallI == 2, "one pair per thread covers its two 1-D items");
    u64 key = 0;
    unsigned bad = 0;
    double zp[2] = {0.0, 0.0};
    if (kD1)
        normal_pair_wave(a.seed, kTagPropose, a.sampler, t, (uint32_t)tid, 0u, 2 * (i64)tid < n,
                         zp[0], zp[1], s_xch[wid]);
    for (int j = 0; j < kSmallI; ++j) {
        const i64 i = kD1 ? 2 * (i64)tid + j : tid + (i64)kSmallT * j;
        const bool act = i < n;
        double *xi = x + i * d;
        double acc = 0.0;
        for (int k = 0; 2 * k < d; ++k) {
            double z[2] = {zp[j == 0 ? 0 : 1], 0.0};
            if (!kD1)
                normal_pair_wave(a.seed, kTagPropose, a.sampler, t, (uint32_t)i, (uint32_t)k, act,
                                 z[0], z[1], s_xch[wid]);
            if (!act) continue;
            for (int h = 0; h < 2; ++h) {
                const int kk = 2 * k + h;
                if (kk >= d) break;
                const double xk = xi[kk] + a.rw_sd * z[h];
                xi[kk] = xk;
                if (kD1) xr[j] = xk;
                if (kKind == SMC_TARGET_GAUSS) {
                    const double tt = xk - a.mean[kk];
                    acc = acc + (tt * tt) * a.prec[kk];
                }
            }
        }
        if (!act) continue;
        double lpn;
        if (kKind == SMC_TARGET_GAUSS) {
            lpn = a.log_norm - 0.5 * acc;
        } else {
            const double tt = xi[0] - a.mu;
            lpn = a.log_norm - a.hnu1 * det_log(1.0 + (tt * tt) * a.inv_nu);
        }
        const double lw = logw[i] + (lpn - lp[i]);
        lp[i] = lpn;
        if (kD1) lpr[j] = lpn;
        logw[i] = lw;
        s_e[i] = lw;
        bad |= (lw != lw) | (lw == __builtin_huge_val());
        const u64 kk = okey(lw);
        key = kk > key ? kk : key;
    }
    key = wave_max_u64(key);
    bad = wave_or(bad);
    if (lane == 0) {
        s_key[wid] = key;
        s_bad[wid] = bad;
    }
    __syncthreads();
    key = s_key[0];
    bad = s_bad[0];
    for (int w = 1; w < 16; ++w) {
        key = s_key[w] > key ? s_key[w] : key;
        bad |= s_bad[w];
    }
    const double m = okey_inv(key);

    // fixed-point weights of consecutive items per thread, FP64 sums, prefix
    const u64 top = 1ull << K;
    double z = 0.0, z2 = 0.0;
    U128 q2{0, 0};
    u64 loc[kSmallI];
    u64 run = 0;
    for (int j = 0; j < kSmallI; ++j) {
        const i64 i = (i64)tid * kSmallI + j;
        u64 q = 0;
        double e = 0.0;
        if (i < n) {
            e = det_exp(s_e[i] - m);  // s_e holds l_i here, e_i after this loop
            if (e >= 0.0) {
                z += e;
                z2 += e * e;
                q = (u64)floor(ldexp(e, K));
                q = q > top ? top : q;
                q2 = add128(q2, mul64(q, q));
            } else {
                e = 0.0;
            }
        }
        run += q;
        loc[j] = run;
        if (i < n) s_e[i] = e;  // the thread's own items: no hazard
    }
    const u64 incl = wave_incl_scan_u64(run);
    if (lane == 63) s_wsum[wid] = incl;
    z = wave_sum_f64(z);
    z2 = wave_sum_f64(z2);
    q2 = wave_sum_u128(q2);
    __syncthreads();
    u64 wpre = 0;
    for (int w = 0; w < wid; ++w) wpre += s_wsum[w];
    const u64 pre = wpre + incl - run;
    for (int j = 0; j < kSmallI; ++j) {
        const i64 i = (i64)tid * kSmallI + j;
        if (i < n) s_S[i] = pre + loc[j];
    }
    if (lane == 0) {
        s_z[wid] = z;
        s_z2[wid] = z2;
        s_lo[wid] = q2.lo;
        s_hi[wid] = q2.hi;
    }
    __syncthreads();

    // estimate sums: a DPP sum per 16-lane row, rows in order
    {
        double s1[DM], s2[DM];
        for (int k = 0; k < DM; ++k) s1[k] = s2[k] = 0.0;
        for (int j = 0; j < kSmallI; ++j) {
            const i64 i = kD1 ? 2 * (i64)tid + j : tid + (i64)kSmallT * j;
            if (i >= n) continue;
            const double e = s_e[i];
#pragma unroll
            for (int k = 0; k < DM; ++k) {
                if (k < d) {
                    const double xv = kD1 ? xr[j] : x[i * d + k];
                    const double ex = e * xv;
                    s1[k] += ex;
                    s2[k] += ex * xv;
                }
            }
        }
        // a DPP sum per 16-lane row, then the wave's four rows in order
#pragma unroll
        for (int k = 0; k < DM; ++k) {
            if (k < d) {
                const double a1 = srow16(s1[k]), a2 = srow16(s2[k]);
                const double w1 = ((lane_f64(a1, 15) + lane_f64(a1, 31)) + lane_f64(a1, 47)) +
                                  lane_f64(a1, 63);
                const double w2 = ((lane_f64(a2, 15) + lane_f64(a2, 31)) + lane_f64(a2, 47)) +
                                  lane_f64(a2, 63);
                if (lane == 0) {
                    s_col[wid][k] = w1;
                    s_col[wid][kSmallD + k] = w2;
                }
            }
        }
    }
    __syncthreads();
    if (kD1) {
        // s_e is free now (the decision below does not read it)
        for (int j = 0; j < kSmallI; ++j) {
            const i64 i = 2 * (i64)tid + j;
            if (i < n) {
                s_e[i] = xr[j];
                s_lpv[i] = lpr[j];
            }
        }
    }
    if (tid < 2 * d) {
        const int c = tid < d ? tid : kSmallD + (tid - d);
        double acc = 0.0;
        for (int w = 0; w < NW; ++w) acc += s_col[w][c];
        s_tot[tid] = acc;
    }
    __syncthreads();

    // decision, offset, log Z, ESS, c_t and recycling (one thread)
    if (tid == 0) {
        double Z = s_z[0], Z2 = s_z2[0];
        U128 Q2{s_lo[0], s_hi[0]};
        for (int w = 1; w < 16; ++w) {
            Z += s_z[w];
            Z2 += s_z2[w];
            Q2 = add128(Q2, U128{s_lo[w], s_hi[w]});
        }
        const u64 S = s_S[n - 1];
        unsigned err = 0;
        if (bad) err = kErrNonfinite;
        else if (key <= okey(-__builtin_huge_val())) err = kErrDegenerate;
        int resample;
        if (mode == SMC_MODE_FORCE) {
            resample = 1;
        } else if (mode == SMC_MODE_NEVER) {
            resample = 0;
        } else {
            const U128 lhs = mul128_small(mul64(S, S), (u64)ess_den);
            const U128 rhs = mul128_small(mul128_small(Q2, (u64)n), (u64)ess_num);
            resample = lt128(lhs, rhs) ? 1 : 0;
        }
        if (err) resample = 0;
        const u64 U = mul64(r, S).hi;
        const double logZ = m + log(Z);
        const double ess = (Z * Z) / Z2;
        ctrl->mkey = key;
        ctrl->m = m;
        ctrl->err_call = err;
        if (err && !ctrl->err_latch) ctrl->err_latch = err;
        ctrl->S = S;
        ctrl->U = U;
        ctrl->Q2lo = Q2.lo;
        ctrl->Q2hi = Q2.hi;
        ctrl->Z = Z;
        ctrl->Z2 = Z2;
        ctrl->logZ = logZ;
        ctrl->ess = ess;
        ctrl->K = K;
        ctrl->resample = (unsigned)resample;
        ctrl->pending = 0;
        // c_t and the recycling sums; an iteration that found an error leaves
        // them (and the estimates) unchanged
        double logc = 0.0, sc = 1.0, wgt = 0.0, den = ctrl->rec_den;
        if (!err) {
            logc = logZ - ctrl->logZ_prev;
            if (logc > ctrl->lc_max) {
                sc = ctrl->rec_steps ? exp(ctrl->lc_max - logc) : 0.0;
                den *= sc;
                ctrl->lc_max = logc;
            }
            wgt = exp(logc - ctrl->lc_max);
            den += wgt;
            ctrl->rec_den = den;
            ctrl->rec_steps += 1;
            ctrl->log_c = logc;
            ctrl->logZ_prev = resample ? 0.0 : logZ;
        }
        if (info) {
            info->m = m;
            info->logZ = logZ;
            info->ess = ess;
            info->Z = Z;
            info->Z2 = Z2;
            info->S = S;
            info->U = U;
            info->Q2_hi = Q2.hi;
            info->Q2_lo = Q2.lo;
            info->K = K;
            info->resampled = resample;
            info->err = (int)err;
            info->pad = 0;
            info->log_c = logc;
        }
        s_bc[0] = sc;
        s_bc[1] = wgt;
        s_bc[2] = den;
        s_bc[3] = Z;
        s_bu[0] = S;
        s_bu[1] = U;
        s_bu[2] = (u64)resample;
        s_bu[3] = (u64)err;
    }
    __syncthreads();
    if (tid < 2 * d && !s_bu[3]) {
        const double f = s_tot[tid] / s_bc[3];
        const double num = rec_num[tid] * s_bc[0] + s_bc[1] * f;
        rec_num[tid] = num;
        if (est) {
            est[tid] = f;
            est[2 * d + tid] = num / s_bc[2];
        }
    }
    if (!s_bu[2]) return;

    // redistribution: output p takes row anc(p), the first j with
    // N S_j + U >= (p + 1) S; staged in the scratch rows, then back in place
    // (kD1: gathered from LDS straight into place)
    const u64 S = s_bu[0], U = s_bu[1];
    for (int j = 0; j < kSmallI; ++j) {
        const i64 p = tid + (i64)kSmallT * j;
        if (p >= n) continue;
        const U128 rhs = mul64((u64)(p + 1), S);
        i64 lo = 0, hi = n - 1;
        while (lo < hi) {
            const i64 mid = (lo + hi) >> 1;
            if (lt128(add128(mul64((u64)n, s_S[mid]), U), rhs)) lo = mid + 1;
            else hi = mid;
        }
        if (kD1) {
            x[p] = s_e[lo];
            lp[p] = s_lpv[lo];
            logw[p] = reset;
        } else {
            for (int k = 0; k < d; ++k) x_scr[p * d + k] = x[lo * d + k];
            lp_scr[p] = lp[lo];
        }
    }
    if (kD1) return;
    __syncthreads();
    for (int j = 0; j < kSmallI; ++j) {
        const i64 p = tid + (i64)kSmallT * j;
        if (p >= n) continue;
        for (int k = 0; k < d; ++k) x[p * d + k] = x_scr[p * d + k];
        lp[p] = lp_scr[p];
        logw[p] = reset;
    }
}

// One iteration in one launch.  slots: the other parity's max slots are
// cleared for the call that follows.
template <int kKind, bool kD1>
__global__ __launch_bounds__(1024) void k_small_step(TArgs a, i64 n, uint32_t t, int K, int mode,
                                                     int ess_num, int ess_den,
                                                     double *__restrict__ x,
                                                     double *__restrict__ logw,
                                                     double *__restrict__ lp,
                                                     double *__restrict__ x_scr,
                                                     double *__restrict__ lp_scr, Ctrl *ctrl,
                                                     u64 *slots_other, double *rec_num,
                                                     smc_resample_info *info, double *est,
                                                     double reset)
{
    for (int k = threadIdx.x; k < kSlots * kSlotStride; k += kSmallT) slots_other[k] = 0;
    small_iteration<kKind, kD1>(a, n, t, K, mode, ess_num, ess_den, x, logw, lp, x_scr, lp_scr,
                                ctrl, rec_num, info, est, reset);
}

// ------------------------------------------------------ cheap log-targets
__global__ __launch_bounds__(256) void k_lp_cheap(TArgs a, i64 n, const double *x, double *lp)
{
    const i64 gtid = (i64)blockIdx.x * 256 + threadIdx.x, gsz = (i64)gridDim.x * 256;
    for (i64 i = gtid; i < n; i += gsz) {
        const double *xi = x + i * a.d;
        if (a.kind == SMC_TARGET_GAUSS) {
            double acc = 0.0;
            for (int k = 0; k < a.d; ++k) {
                const double tt = xi[k] - a.mean[k];
                acc = acc + (tt * tt) * a.prec[k];
            }
            lp[i] = a.log_norm - 0.5 * acc;
        } else {
            const double tt = xi[0] - a.mu;
            lp[i] = a.log_norm - a.hnu1 * det_log(1.0 + (tt * tt) * a.inv_nu);
        }
    }
}

// --------------------------------------------- logistic regression, FP64
// With s_m = 1 - 2 y_m and u = s_m z_m, y_m z_m - softplus(z_m) = -softplus(u),
// and softplus(u) = (u + |u|) / 2 + log1p(e^(-|u|)).  The kernel sums |u| and
// the logs of products of 64 factors 1 + e^(-|u|) in (1, 2] (at most 2^64);
// the sum of u over all rows, theta . (sum_m s_m x_m), is added once per
// particle by k_logreg_sum.
//
// u = (X s) theta runs on v_mfma_f64_16x16x4_f64, so the matrix unit takes the
// contraction while the vector ALU runs the exponentials.  One wavefront owns
// 16 particles (MFMA columns) and streams 16-row tiles of X s (MFMA rows) from
// xf, where each tile is stored in the order the MFMA A operand is read:
// xf[tile][lane][s] = s_m x_{m,k}, m = 16 tile + lane % 16, k = 4 s + lane / 16
// (zero beyond M and d), so a lane's KS values are contiguous and a tile is
// one contiguous 512 KS-byte read per wavefront.  The epilogue relies only on
// each lane's accumulators belonging to column lane % 16: it sums a column's
// rows whatever their order across lanes.
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2v __attribute__((ext_vector_type(2)));

__device__ inline void softplus_acc64(double u, double &sa, double &prod)
{
    const double au = fabs(u);
    prod = fma(prod, exp(-au), prod);
    sa += au;
}

template <int KS>
__global__ __launch_bounds__(256) void k_logreg_f64(const double *__restrict__ theta, i64 n, int d,
                                                    const double *__restrict__ xf, i64 m_rows,
                                                    i64 mpad, double *__restrict__ lpart)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const i64 p0 = ((i64)blockIdx.x * 4 + wid) * 16;
    if (p0 >= n) return;
    const int col = lane & 15, kq = lane >> 4;
    const i64 p = p0 + col;
    double b[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int k = 4 * s + kq;
        b[s] = (p < n && k < d) ? theta[p * d + k] : 0.0;
    }
    const i64 tiles = mpad / 16;
    const i64 per = (tiles + gridDim.y - 1) / gridDim.y;
    const i64 t0 = (i64)blockIdx.y * per;
    const i64 t1 = t0 + per < tiles ? t0 + per : tiles;
    double sa = 0.0, lg = 0.0, prod = 1.0;
    int cnt = 0;
    for (i64 tt = t0; tt < t1; ++tt) {
        const double *ap = xf + (tt * 64 + lane) * KS;
        double a[KS];
        if constexpr (KS == 1) {
            a[0] = ap[0];
        } else {
#pragma unroll
            for (int s = 0; s < KS; s += 2) {
                const f64x2v v = *reinterpret_cast<const f64x2v *>(ap + s);
                a[s] = v[0];
                a[s + 1] = v[1];
            }
        }
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KS; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) softplus_acc64(acc[v], sa, prod);
        if (++cnt == 16) {
            lg += log(prod);
            prod = 1.0;
            cnt = 0;
        }
    }
    double sp = 0.5 * sa + (lg + log(prod));
    sp += __shfl_xor(sp, 16, kWave);
    sp += __shfl_xor(sp, 32, kWave);
    // Rows of the last tile beyond M are zero: u = 0 there, and each added a
    // factor of exactly 2 (and nothing to |u|), whichever lane held it.
    const i64 lo = t0 * 16 > m_rows ? t0 * 16 : m_rows, hi = t1 * 16;
    if (hi > lo) sp -= (double)(hi - lo) * kLn2;
    if (lane < 16 && p < n) lpart[(i64)blockIdx.y * n + p] = -sp;
}

// xf (above) from the caller's X and y.
__global__ __launch_bounds__(256) void k_prep_xf(const double *X, const double *y, i64 m_rows,
                                                 int d, i64 mpad, int ks, double *xf)
{
    const i64 gtid = (i64)blockIdx.x * 256 + threadIdx.x, gsz = (i64)gridDim.x * 256;
    const i64 per_tile = 64 * (i64)ks;
    for (i64 e = gtid; e < mpad * 4 * ks; e += gsz) {
        const i64 t = e / per_tile;
        const int rem = (int)(e - t * per_tile);
        const int lane = rem / ks, sidx = rem - lane * ks;
        const i64 m = 16 * t + (lane & 15);
        const int k = 4 * sidx + (lane >> 4);
        double v = 0.0;
        if (m < m_rows && k < d) {
            v = X[m * d + k];
            if (y[m] != 0.0) v = -v;
        }
        xf[e] = v;
    }
}

// Column sums of X s (rows below m_rows), one workgroup per column, FP64 in
// a fixed order.
__global__ __launch_bounds__(256) void k_x_colsum(const double *X, const double *y, i64 m_rows,
                                                  int d, double *csum)
{
    __shared__ double red[4];
    const int k = blockIdx.x, tid = threadIdx.x;
    double v = 0.0;
    for (i64 m = tid; m < m_rows; m += 256) {
        const double xv = X[m * d + k];
        v += y[m] != 0.0 ? -xv : xv;
    }
    v = wave_sum_f64(v);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) csum[k] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ------------------------------------ logistic regression, BF16 MFMA (gfx950)
// X is stored pre-multiplied by s_m = 1 - 2 y_m (exact in bf16), so that
// y_m z_m - softplus(z_m) = -softplus(s_m z_m) and the epilogue needs no labels.
// One wavefront owns 32 particles (MFMA columns) and streams 32-row tiles of X
// (MFMA rows) through v_mfma_f32_32x32x16_bf16; the softplus epilogue runs on
// the FP32 accumulators, which hold u = t log2 e for t = s_m z_m.
// softplus(t) = ln 2 [(u + |u|) / 2 + log2(1 + 2^(-|u|))].  A lane's 16
// accumulator values of one tile each give a factor 1 + 2^(-|u|) in (1, 2];
// their product (at most 2^16) takes one log2 per tile.  The kernel sums |u|
// and the log2 terms; the sum of u over all rows is theta . (sum_m x_m s_m)
// log2 e, added once per particle by k_logreg_sum from the column sums of X.
__device__ inline void softplus_acc(float u, float &sa, float &prod)
{
    const float e = __builtin_amdgcn_exp2f(-fabsf(u));
    prod = fmaf(prod, e, prod);
    sa += fabsf(u);
}

template <int KS>
__global__ __launch_bounds__(256) void k_logreg_bf16(const unsigned short *__restrict__ thb, i64 n,
                                                     const unsigned short *__restrict__ xs,
                                                     i64 m_rows, i64 mpad, int dp,
                                                     double *__restrict__ lpart)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const i64 p0 = ((i64)blockIdx.x * 4 + wid) * 32;
    if (p0 >= n) return;
    const int col = lane & 31, kh = lane >> 5;
    bf16x8 bfr[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s)
        bfr[s] = *reinterpret_cast<const bf16x8 *>(thb + (p0 + col) * dp + 16 * s + 8 * kh);
    const i64 tiles = mpad / 32;
    const i64 per = (tiles + gridDim.y - 1) / gridDim.y;
    const i64 t0 = (i64)blockIdx.y * per;
    const i64 t1 = t0 + per < tiles ? t0 + per : tiles;
    float sa = 0.0f, lg = 0.0f;
    for (i64 tt = t0; tt < t1; ++tt) {
        const i64 m0 = tt * 32;
        f32x16 acc = {};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const bf16x8 afr =
                *reinterpret_cast<const bf16x8 *>(xs + (m0 + col) * dp + 16 * s + 8 * kh);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr, bfr[s], acc, 0, 0, 0);
        }
        float prod = 1.0f;
        if (m0 + 32 <= m_rows) {
#pragma unroll
            for (int r = 0; r < 16; ++r) softplus_acc(acc[r], sa, prod);
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const i64 row = m0 + 8 * (r >> 2) + 4 * kh + (r & 3);
                if (row < m_rows) softplus_acc(acc[r], sa, prod);
            }
        }
        lg += __builtin_amdgcn_logf(prod);
    }
    float sp = 0.5f * sa + lg;
    sp += __shfl_xor(sp, 32, kWave);
    if (lane < 32 && p0 + lane < n) lpart[(i64)blockIdx.y * n + p0 + lane] = -kLn2 * (double)sp;
}

// Column sums of the stored bf16 X s (rows below m_rows; padding is zero), one
// workgroup per column, FP64 in a fixed order.
__global__ __launch_bounds__(256) void k_xs_colsum(const unsigned short *xs, i64 m_rows, int dp,
                                                   double *csum)
{
    __shared__ double red[4];
    const int k = blockIdx.x, tid = threadIdx.x;
    double v = 0.0;
    for (i64 m = tid; m < m_rows; m += 256) v += from_bf16(xs[m * dp + k]);
    v = wave_sum_f64(v);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) csum[k] = (red[0] + red[1]) + (red[2] + red[3]);
}

// log pi = log_norm - prior_prec |theta|^2 / 2 + the partial likelihoods
// - usc (theta' . csum), where theta' is the bf16 copy thb when given (it holds
// theta log2 e) and theta otherwise.
__global__ __launch_bounds__(256) void k_logreg_sum(const double *theta, i64 n, int d,
                                                    const double *lpart, int msplit,
                                                    double log_norm, double prior_prec,
                                                    const unsigned short *thb, int dp,
                                                    const double *csum, double usc, double *lp)
{
    const i64 gtid = (i64)blockIdx.x * 256 + threadIdx.x, gsz = (i64)gridDim.x * 256;
    for (i64 i = gtid; i < n; i += gsz) {
        double pr = 0.0;
        for (int k = 0; k < d; ++k) pr += theta[i * d + k] * theta[i * d + k];
        double s = 0.0;
        for (int j = 0; j < msplit; ++j) s += lpart[(i64)j * n + i];
        double su = 0.0;
        for (int k = 0; k < d; ++k)
            su += (thb ? from_bf16(thb[i * dp + k]) : theta[i * d + k]) * csum[k];
        lp[i] = log_norm - 0.5 * prior_prec * pr + (s - usc * su);
    }
}

__global__ __launch_bounds__(256) void k_prep_x(const double *X, const double *y, i64 m_rows,
                                                int d, i64 mpad, int dp, unsigned short *xs,
                                                unsigned short *thb, i64 thb_elems)
{
    const i64 gtid = (i64)blockIdx.x * 256 + threadIdx.x, gsz = (i64)gridDim.x * 256;
    for (i64 e = gtid; e < mpad * dp; e += gsz) {
        const i64 m = e / dp;
        const int k = (int)(e - m * dp);
        double v = 0.0;
        if (m < m_rows && k < d) v = (y[m] != 0.0 ? -1.0 : 1.0) * X[m * d + k];
        xs[e] = to_bf16(v);
    }
    for (i64 e = gtid; e < thb_elems; e += gsz) thb[e] = 0;
}

__global__ __launch_bounds__(256) void k_theta_bf16(const double *x, i64 n, int d, int dp,
                                                    unsigned short *thb)
{
    const i64 gtid = (i64)blockIdx.x * 256 + threadIdx.x, gsz = (i64)gridDim.x * 256;
    for (i64 e = gtid; e < n * d; e += gsz) {
        const i64 i = e / d;
        const int k = (int)(e - i * d);
        thb[i * dp + k] = to_bf16(x[e] * kLog2e);
    }
}

// ================================================================= host side
namespace {

TArgs targs(const smc_config &c, const Work &w, bool with_bf16)
{
    TArgs a;
    a.kind = c.target;
    a.d = c.d;
    a.dp = w.dp;
    a.mean = c.mean;
    a.prec = c.prec;
    a.log_norm = c.log_norm;
    a.mu = c.mu;
    a.inv_nu = c.target == SMC_TARGET_STUDENT ? 1.0 / c.nu : 0.0;
    a.hnu1 = 0.5 * (c.nu + 1.0);
    a.init_mean = c.init_mean;
    a.init_sd = c.init_sd;
    a.init_prec = 1.0 / (c.init_sd * c.init_sd);
    a.init_log_norm = c.init_log_norm;
    a.rw_sd = c.rw_sd;
    a.seed = c.seed;
    a.sampler = c.sampler_id;
    a.thb = with_bf16 ? w.thb : nullptr;
    a.obs = c.obs;
    a.delta = c.delta;
    const double s11 = 5.0 * c.delta * c.delta * c.delta / 3.0;
    const double s21 = 5.0 * c.delta * c.delta / 2.0;
    const double s22 = 5.0 * c.delta;
    a.l11 = std::sqrt(s11);
    a.l21 = s21 / a.l11;
    a.l22 = std::sqrt(s22 - a.l21 * a.l21);
    a.obs_prec = c.target == SMC_TARGET_BEARING ? 1.0 / c.obs_var : 0.0;
    a.obs_log_norm = c.obs_log_norm;
    a.reset = -std::log((double)c.n);
    a.uniform = c.lazy_reset ? &w.ctrl->uniform : nullptr;
    return a;
}

int grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > kMaxBlocks ? kMaxBlocks : b));
}

bool is_bf16(const smc_config &c)
{
    return c.target == SMC_TARGET_LOGREG && c.loglik_precision == SMC_PREC_BF16;
}

// log pi at x[n][d] into lp (the likelihood kernels of the costly target).
hipError_t logreg_lp(const smc_config &c, const Work &w, const double *x, int64_t n, double *lp,
                     bool theta_ready, hipStream_t s)
{
    if (c.target != SMC_TARGET_LOGREG || !w.lpart || !w.csum || (is_bf16(c) && (!w.xs || !w.thb)) ||
        (!is_bf16(c) && !w.xf))
        return hipErrorInvalidValue;
    const int msplit = kLogregSplit;
    if (is_bf16(c)) {
        if (!theta_ready) {
            hipLaunchKernelGGL(k_theta_bf16, dim3(grid_for(n * c.d)), dim3(256), 0, s, x, (i64)n,
                               c.d, w.dp, w.thb);
        }
        const dim3 grid((unsigned)((n + 127) / 128), msplit);
        const unsigned short *xs = w.xs;
        switch (w.dp / 16) {
        case 1: hipLaunchKernelGGL(k_logreg_bf16<1>, grid, dim3(256), 0, s, w.thb, (i64)n, xs, c.m_rows, w.mpad, w.dp, w.lpart); break;
        case 2: hipLaunchKernelGGL(k_logreg_bf16<2>, grid, dim3(256), 0, s, w.thb, (i64)n, xs, c.m_rows, w.mpad, w.dp, w.lpart); break;
        case 3: hipLaunchKernelGGL(k_logreg_bf16<3>, grid, dim3(256), 0, s, w.thb, (i64)n, xs, c.m_rows, w.mpad, w.dp, w.lpart); break;
        default: hipLaunchKernelGGL(k_logreg_bf16<4>, grid, dim3(256), 0, s, w.thb, (i64)n, xs, c.m_rows, w.mpad, w.dp, w.lpart); break;
        }
    } else {
        const dim3 grid((unsigned)((n + 63) / 64), msplit);
        const double *xf = w.xf;
        switch (lr_ks(c.d)) {
        case 1: hipLaunchKernelGGL(k_logreg_f64<1>, grid, dim3(256), 0, s, x, (i64)n, c.d, xf, c.m_rows, w.mpad, w.lpart); break;
        case 2: hipLaunchKernelGGL(k_logreg_f64<2>, grid, dim3(256), 0, s, x, (i64)n, c.d, xf, c.m_rows, w.mpad, w.lpart); break;
        case 4: hipLaunchKernelGGL(k_logreg_f64<4>, grid, dim3(256), 0, s, x, (i64)n, c.d, xf, c.m_rows, w.mpad, w.lpart); break;
        case 8: hipLaunchKernelGGL(k_logreg_f64<8>, grid, dim3(256), 0, s, x, (i64)n, c.d, xf, c.m_rows, w.mpad, w.lpart); break;
        default: hipLaunchKernelGGL(k_logreg_f64<16>, grid, dim3(256), 0, s, x, (i64)n, c.d, xf, c.m_rows, w.mpad, w.lpart); break;
        }
    }
    const bool bf = is_bf16(c);
    hipLaunchKernelGGL(k_logreg_sum, dim3(grid_for(n)), dim3(256), 0, s, x, (i64)n, c.d, w.lpart,
                       msplit, c.log_norm, c.prior_prec, bf ? w.thb : nullptr, w.dp, w.csum,
                       bf ? 0.5 * kLn2 : 0.5, lp);
    return hipGetLastError();
}

template <int kKind, bool kInit, int DT>
void launch_is_k(dim3 g, hipStream_t s, const TArgs &a, i64 n, uint32_t t, double *x, double *logw,
                 const Work &w, u64 *sp, bool out)
{
    if (!kInit && out)
        hipLaunchKernelGGL((k_is<kKind, false, DT, true>), g, dim3(256), 0, s, a, n, t, x, logw,
                           w.lp, sp, w.is_part, w.x_scr, w.lp_scr);
    else
        hipLaunchKernelGGL((k_is<kKind, kInit, DT, false>), g, dim3(256), 0, s, a, n, t, x, logw,
                           w.lp, sp, w.is_part, (double *)nullptr,
                           (double *)nullptr);
}

// out: the proposal goes to the workspace copies (x_scr, lp_scr).
template <bool kInit>
hipError_t launch_is(const smc_config &c, const Work &w, int par, uint32_t t, double *x,
                     double *logw, hipStream_t s, bool out = false)
{
    const TArgs a = targs(c, w, is_bf16(c));
    const dim3 g(w.is_grid);
    const i64 n = c.n;
    u64 *sp = w.slots + (par & 1) * kSlots * kSlotStride;
    switch (c.target) {
    case SMC_TARGET_GAUSS:
        if (c.d == 1) launch_is_k<SMC_TARGET_GAUSS, kInit, 1>(g, s, a, n, t, x, logw, w, sp, out);
        else if (c.d == 4)
            launch_is_k<SMC_TARGET_GAUSS, kInit, 4>(g, s, a, n, t, x, logw, w, sp, out);
        else launch_is_k<SMC_TARGET_GAUSS, kInit, 0>(g, s, a, n, t, x, logw, w, sp, out);
        break;
    case SMC_TARGET_STUDENT:
        launch_is_k<SMC_TARGET_STUDENT, kInit, 1>(g, s, a, n, t, x, logw, w, sp, out);
        break;
    case SMC_TARGET_BEARING:
        launch_is_k<SMC_TARGET_BEARING, kInit, 4>(g, s, a, n, t, x, logw, w, sp, out);
        break;
    case SMC_TARGET_LOGREG:
        launch_is_k<SMC_TARGET_LOGREG, kInit, 0>(g, s, a, n, t, x, logw, w, sp, false);
        if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
        if (logreg_lp(c, w, x, n, w.lp_new, true, s) != hipSuccess) return hipErrorLaunchFailure;
        hipLaunchKernelGGL(k_reweight<kInit>, g, dim3(256), 0, s, n, c.d, x, w.lp_new, logw,
                           w.lp, sp, w.is_part, a.uniform, a.reset);
        break;
    default:
        return hipErrorInvalidValue;
    }
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    // initialisation has no scan; its max is folded on its own
    return kInit ? launch_fold(w, par, s) : hipSuccess;
}

template <int kKind, int DT>
int resident_blocks()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_is<kKind, false, DT, false>, 256, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

}  // namespace

int sampler_grid(const smc_config &c)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    int per_cu = 0;
    switch (c.target) {
    case SMC_TARGET_GAUSS:
        per_cu = c.d == 1 ? resident_blocks<SMC_TARGET_GAUSS, 1>()
                 : c.d == 4 ? resident_blocks<SMC_TARGET_GAUSS, 4>()
                            : resident_blocks<SMC_TARGET_GAUSS, 0>();
        break;
    case SMC_TARGET_STUDENT: per_cu = resident_blocks<SMC_TARGET_STUDENT, 1>(); break;
    case SMC_TARGET_BEARING: per_cu = resident_blocks<SMC_TARGET_BEARING, 4>(); break;
    case SMC_TARGET_LOGREG: per_cu = resident_blocks<SMC_TARGET_LOGREG, 0>(); break;
    default: return 0;
    }
    if (per_cu < 1) return 0;
    int64_t g = (int64_t)per_cu * cus;
    const int64_t need = (c.n + 255) / 256;
    g = g < need ? g : need;
    g = g < kIsBlocks ? g : kIsBlocks;
    return (int)(g < 1 ? 1 : g);
}

smc_status step_init(const smc_config &c, const Work &w, int par, double *x, double *logw,
                     hipStream_t s)
{
    if (c.target == SMC_TARGET_LOGREG && is_bf16(c)) {
        const int64_t thb_elems = w.npad * w.dp;
        hipLaunchKernelGGL(k_prep_x, dim3(grid_for(w.mpad * w.dp)), dim3(256), 0, s,
                           reinterpret_cast<const double *>(c.X), c.y, (i64)c.m_rows, c.d,
                           (i64)w.mpad, w.dp, w.xs, w.thb, (i64)thb_elems);
        hipLaunchKernelGGL(k_xs_colsum, dim3(c.d), dim3(256), 0, s, w.xs, (i64)c.m_rows, w.dp,
                           w.csum);
        if (hipGetLastError() != hipSuccess) return SMC_E_DEVICE;
    } else if (c.target == SMC_TARGET_LOGREG) {
        const int ks = lr_ks(c.d);
        hipLaunchKernelGGL(k_prep_xf, dim3(grid_for(w.mpad * 4 * ks)), dim3(256), 0, s,
                           reinterpret_cast<const double *>(c.X), c.y, (i64)c.m_rows, c.d,
                           (i64)w.mpad, ks, w.xf);
        hipLaunchKernelGGL(k_x_colsum, dim3(c.d), dim3(256), 0, s,
                           reinterpret_cast<const double *>(c.X), c.y, (i64)c.m_rows, c.d, w.csum);
        if (hipGetLastError() != hipSuccess) return SMC_E_DEVICE;
    }
    if (launch_is<true>(c, w, par, 0u, x, logw, s) != hipSuccess) return SMC_E_DEVICE;
    if (c.target == SMC_TARGET_BEARING)  // equal initial weights: sums from the common reference
        hipLaunchKernelGGL(k_post_est<4>, dim3(w.is_grid), dim3(256), 0, s, w.ctrl, (i64)c.n,
                           c.d, x, logw, -std::log((double)c.n), w.is_part);
    hipLaunchKernelGGL(k_step_stats<1024>, dim3(1), dim3(1024), 0, s, w.ctrl, w.is_part, w.is_grid,
                       c.d, w.rec_num, (double *)nullptr, (smc_resample_info *)nullptr, 1);
    return hipGetLastError() == hipSuccess ? SMC_OK : SMC_E_DEVICE;
}

bool small_path(const smc_config &c)
{
    return c.n <= kSmallN && c.d <= kSmallD &&
           (c.target == SMC_TARGET_GAUSS || c.target == SMC_TARGET_STUDENT);
}

// Small population: the whole iteration in one workgroup and one launch.
smc_status small_step(const smc_config &c, const Work &w, int K, int par, uint32_t t, double *x,
                      double *logw, smc_resample_info *info, double *est, hipStream_t s)
{
    const int64_t n = c.n;
    const TArgs a = targs(c, w, false);
    const double reset = -std::log((double)n);
    u64 *other = w.slots + ((par & 1) ^ 1) * kSlots * kSlotStride;
    auto kern = c.target == SMC_TARGET_GAUSS
                    ? (c.d == 1 ? k_small_step<SMC_TARGET_GAUSS, true>
                                : k_small_step<SMC_TARGET_GAUSS, false>)
                    : (c.d == 1 ? k_small_step<SMC_TARGET_STUDENT, true>
                                : k_small_step<SMC_TARGET_STUDENT, false>);
    hipLaunchKernelGGL(kern, dim3(1), dim3(kSmallT), 0, s, a, (i64)n, t, K, c.mode, c.ess_num,
                       c.ess_den, x, logw, w.lp, w.x_scr, w.lp_scr, w.ctrl, other, w.rec_num, info,
                       est, reset);
    return hipGetLastError() == hipSuccess ? SMC_OK : SMC_E_DEVICE;
}

smc_status step_run_n(const smc_config &c, const Work &w, int K, int par0, uint32_t t0,
                      int nsteps, double *x, double *logw, smc_resample_info *info, double *est,
                      hipStream_t s)
{
    for (int i = 0; i < nsteps; ++i) {
        const smc_status st = step_run(c, w, K, par0 ^ (i & 1), t0 + (uint32_t)i, x, logw,
                                       info ? info + i : nullptr,
                                       est ? est + (int64_t)i * 4 * c.d : nullptr, s);
        if (st != SMC_OK) return st;
    }
    return SMC_OK;
}

smc_status step_run(const smc_config &c, const Work &w, int K, int par, uint32_t t, double *x,
                    double *logw, smc_resample_info *info, double *est, hipStream_t s)
{
    if (small_path(c)) return small_step(c, w, K, par, t, x, logw, info, est, s);
    const int64_t n = c.n;
    const bool pf = c.target == SMC_TARGET_BEARING;
    // With resampling forced every iteration the proposal goes to the
    // workspace copy and the redistribution writes straight into x (an
    // identity copy if the step found an error or kept the weights): no copy
    // back.  The particle filter always takes this path (its weights collapse
    // almost every update, and the expand forms its post-resampling sums from
    // the rows it writes).  With the ESS rule a sampler is updated in place,
    // and only resampling steps move rows.
    const bool fwd = (c.mode == SMC_MODE_FORCE && c.target != SMC_TARGET_LOGREG) || pf;
    if (launch_is<false>(c, w, par, t, x, logw, s, fwd) != hipSuccess) return SMC_E_DEVICE;
    if (launch_quant_scan(w, logw, n, K, par, s, c.lazy_reset != 0) != hipSuccess)
        return SMC_E_DEVICE;
    const uint64_t r = resample_word(c.seed, c.sampler_id, t);
    // Alg 2 estimates come before resampling: the decision's workgroup forms
    // them (the filter takes its mean after resampling, below)
    StatsArgs st;
    if (!pf) {
        st.is_part = w.is_part;
        st.nblk = w.is_grid;
        st.d = c.d;
        st.rec_num = w.rec_num;
        st.est = est;
    }
    if (launch_decide(w, par, n, K, r, c.mode, c.ess_num, c.ess_den, info, s, st) != hipSuccess)
        return SMC_E_DEVICE;
    const double reset = -std::log((double)n);
    unsigned *uni = c.lazy_reset ? &w.ctrl->uniform : nullptr;
    // the particle filter and the 1-D Gaussian and Student-t samplers carry no
    // cached log-target
    const bool lpc = !pf && !(c.d == 1 && (c.target == SMC_TARGET_GAUSS ||
                                           c.target == SMC_TARGET_STUDENT));
    double *lp = lpc ? w.lp : nullptr, *lp_scr = lpc ? w.lp_scr : nullptr;
    if (fwd) {
        // the filter's row sums ride on 16-byte chunks of its 32-byte rows
        double *ep = (pf && ((uintptr_t)x & 15) == 0) ? w.epart : nullptr;
        if (launch_expand(w, n, 0, w.x_scr, x, c.d * 8, lp_scr, lp, 8, nullptr, nullptr, s,
                          false, ep) != hipSuccess)
            return SMC_E_DEVICE;
        if (pf) {  // Alg 1 takes the mean after resampling
            hipLaunchKernelGGL(k_reset_est<4>, dim3(w.is_grid), dim3(256), 0, s, w.ctrl, (i64)n,
                               c.d, x, w.x_scr, (double *)nullptr, (const double *)nullptr,
                               logw, reset, w.is_part, (const double *)ep,
                               (i64)expand_segments(n), uni);
            hipLaunchKernelGGL(k_step_stats<1024>, dim3(1), dim3(1024), 0, s, w.ctrl, w.is_part,
                               w.is_grid, c.d, w.rec_num, est, info, 0);
        } else {
            hipLaunchKernelGGL(k_reset_est<0>, dim3(w.is_grid), dim3(256), 0, s, w.ctrl, (i64)n,
                               c.d, x, w.x_scr, lp, lp_scr, logw, reset, w.is_part,
                               (const double *)nullptr, (i64)0, uni);
        }
        return hipGetLastError() == hipSuccess ? SMC_OK : SMC_E_DEVICE;
    }
    if (launch_expand(w, n, 0, x, w.x_scr, c.d * 8, lp, lp_scr, 8, nullptr, nullptr, s, true) !=
        hipSuccess)
        return SMC_E_DEVICE;
    hipLaunchKernelGGL(k_copyback, dim3(grid_for(n * c.d)), dim3(256), 0, s, w.ctrl, (i64)n, c.d,
                       x, w.x_scr, lp, lp_scr, logw, reset, uni);
    return hipGetLastError() == hipSuccess ? SMC_OK : SMC_E_DEVICE;
}

__global__ __launch_bounds__(256) void k_sync_weights(const Ctrl *ctrl, i64 n, double *logw,
                                                      double reset)
{
    if (!ctrl->uniform) return;
    const i64 gtid = (i64)blockIdx.x * 256 + threadIdx.x, gsz = (i64)gridDim.x * 256;
    for (i64 i = gtid; i < n; i += gsz) logw[i] = reset;
}

smc_status step_sync_weights(const smc_config &c, const Work &w, double *logw, hipStream_t s)
{
    if (!c.lazy_reset) return SMC_OK;
    hipLaunchKernelGGL(k_sync_weights, dim3(grid_for(c.n)), dim3(256), 0, s, w.ctrl, (i64)c.n,
                       logw, -std::log((double)c.n));
    return hipGetLastError() == hipSuccess ? SMC_OK : SMC_E_DEVICE;
}

smc_status step_log_target(const smc_config &c, const Work &w, const double *x, int64_t n,
                           double *lp, hipStream_t s)
{
    if (n > c.n) return SMC_E_ARG;
    if (c.target == SMC_TARGET_LOGREG) {
        return logreg_lp(c, w, x, n, lp, false, s) == hipSuccess ? SMC_OK : SMC_E_DEVICE;
    }
    const TArgs a = targs(c, w, false);
    hipLaunchKernelGGL(k_lp_cheap, dim3(grid_for(n)), dim3(256), 0, s, a, (i64)n, x, lp);
    return hipGetLastError() == hipSuccess ? SMC_OK : SMC_E_DEVICE;
}

}  // namespace smc
