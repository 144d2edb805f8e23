// Resampling kernels of Alg 4 (minimum variance resampling):
//   k_max            exact FP64 max of the log-weights (stability shift of
//                    eq. normalise) + non-finite detection; clears the scan
//                    state for the next pass.
//   k_scan<Quant>    one pass over the log-weights: 64-bit fixed-point weights
//                    q_i = min(2^K, floor(2^K det_exp(l_i - m))), FP64 sums for
//                    log-sum-exp and ESS (eq. normalise, eq. neff), exact
//                    sum q_i^2, and the inclusive prefix S_j by a single-pass
//                    decoupled-lookback scan (the Cumulative Sum of MVR).
//   k_scan<Counts>   the same scan over caller-supplied int64 ncopies.
//   k_finalize       exact integer ESS decision, systematic offset
//                    U = floor(r S / 2^64), log Z, FP64 ESS.
//   k_ncopies        ncopies_j = A_j - A_{j-1}, A_j = floor((N S_j + U) / S)
//                    (eq. ncopies holds by telescoping).
#include <hip/hip_runtime.h>

#include "../../include/smc.h"
#include "common.hpp"
#include "det.hpp"
#include "kernels.hpp"

namespace smc {

// ------------------------------------------------------------- control init
__global__ void k_init_ctrl(Ctrl *ctrl)
{
    u64 *p = reinterpret_cast<u64 *>(ctrl);
    for (int i = threadIdx.x; i < (int)(sizeof(Ctrl) / 8); i += blockDim.x) p[i] = 0;
}

hipError_t launch_init_ctrl(const Work &w, hipStream_t s)
{
    static_assert(sizeof(Ctrl) % 8 == 0, "ctrl size");
    hipLaunchKernelGGL(k_init_ctrl, dim3(1), dim3(64), 0, s, w.ctrl);
    return hipGetLastError();
}

// ------------------------------------------------------------- exact max
// Every block reduces a grid-stride share to one order key; the last block to
// finish combines the per-block keys (max is order-free, so the result is
// exact and independent of scheduling) and resets the counters of the scan.
__global__ __launch_bounds__(256) void k_max(const double *__restrict__ lw, i64 n, int vec2,
                                             Ctrl *ctrl, u64 *blk_key, unsigned *blk_bad,
                                             u64 *status, int n_status)
{
    __shared__ u64 s_key[4];
    __shared__ unsigned s_bad[4];
    __shared__ int s_last;
    const int tid = threadIdx.x;
    const i64 gtid = (i64)blockIdx.x * 256 + tid, gsz = (i64)gridDim.x * 256;
    for (i64 i = gtid; i < n_status; i += gsz) status[i] = 0;

    u64 key = 0;
    unsigned bad = 0;
    if (vec2) {
        const i64 npair = n >> 1;
        const double2 *lw2 = reinterpret_cast<const double2 *>(lw);
        for (i64 i = gtid; i < npair; i += gsz) {
            const double2 v = lw2[i];
            bad |= (v.x != v.x) | (v.x == __builtin_huge_val()) | (v.y != v.y) |
                   (v.y == __builtin_huge_val());
            const u64 ka = okey(v.x), kb = okey(v.y);
            key = ka > key ? ka : key;
            key = kb > key ? kb : key;
        }
        if ((n & 1) && gtid == 0) {
            const double v = lw[n - 1];
            bad |= (v != v) | (v == __builtin_huge_val());
            const u64 k = okey(v);
            key = k > key ? k : key;
        }
    } else {
        for (i64 i = gtid; i < n; i += gsz) {
            const double v = lw[i];
            bad |= (v != v) | (v == __builtin_huge_val());
            const u64 k = okey(v);
            key = k > key ? k : key;
        }
    }
    key = wave_max_u64(key);
    bad = wave_or(bad);
    if ((tid & 63) == 0) {
        s_key[tid >> 6] = key;
        s_bad[tid >> 6] = bad;
    }
    __syncthreads();
    if (tid == 0) {
        u64 k = s_key[0];
        unsigned b = s_bad[0];
        for (int i = 1; i < 4; ++i) {
            k = s_key[i] > k ? s_key[i] : k;
            b |= s_bad[i];
        }
        blk_key[blockIdx.x] = k;
        blk_bad[blockIdx.x] = b;
        __threadfence();
        s_last = atomicAdd(&ctrl->blk_done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    key = 0;
    bad = 0;
    for (int i = tid; i < (int)gridDim.x; i += 256) {
        const u64 k = __hip_atomic_load(&blk_key[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        key = k > key ? k : key;
        bad |= __hip_atomic_load(&blk_bad[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    key = wave_max_u64(key);
    bad = wave_or(bad);
    __syncthreads();
    if ((tid & 63) == 0) {
        s_key[tid >> 6] = key;
        s_bad[tid >> 6] = bad;
    }
    __syncthreads();
    if (tid == 0) {
        u64 k = s_key[0];
        unsigned b = s_bad[0];
        for (int i = 1; i < 4; ++i) {
            k = s_key[i] > k ? s_key[i] : k;
            b |= s_bad[i];
        }
        unsigned err = 0;
        if (b) err = kErrNonfinite;
        else if (k <= okey(-__builtin_huge_val())) err = kErrDegenerate;
        ctrl->mkey = k;
        ctrl->m = okey_inv(k);
        ctrl->err_call = err;
        if (err && !ctrl->err_latch) ctrl->err_latch = err;
        ctrl->blk_done = 0;
        ctrl->tile_next = 0;
        ctrl->pending = 0;
    }
}

hipError_t launch_max(const Work &w, const double *lw, int64_t n, hipStream_t s)
{
    const int vec2 = ((uintptr_t)lw & 15) == 0;
    hipLaunchKernelGGL(k_max, dim3(max_blocks_of(n)), dim3(256), 0, s, lw, (i64)n, vec2, w.ctrl,
                       w.blk_key, w.blk_bad, w.status, w.n_tiles);
    return hipGetLastError();
}

// -------------------------------------------------- decoupled-lookback scan
// Tile = 256 threads x 16 items.  Loads and stores are coalesced 16-byte row
// accesses (rows of 512 elements); an LDS transpose (one pad word per 16
// entries against bank conflicts) gives each thread 16 consecutive items for
// the sequential part of the scan.
constexpr int kPad(int i) { return i + (i >> 4); }

struct QuantIn {
    const double *lw;
    int K;
    int vec2;
};

struct CountIn {
    const i64 *nc;
    i64 n;
};

// Fixed-point weight of one log-weight; accumulates the FP64 and exact sums.
__device__ inline u64 quant_one(double v, double m, int K, u64 top, double &z, double &z2, U128 &q2)
{
    const double e = det_exp(v - m);
    if (!(e >= 0.0)) return 0;  // NaN input: the max pass has flagged it
    z += e;
    z2 += e * e;
    const double f = floor(ldexp(e, K));
    u64 q = (u64)f;
    q = q > top ? top : q;
    q2 = add128(q2, mul64(q, q));
    return q;
}

template <bool kQuant>
__global__ __launch_bounds__(256) void k_scan(QuantIn qin, CountIn cin, i64 n, Ctrl *ctrl,
                                              u64 *status, TilePart *tpart, u64 *__restrict__ out)
{
    __shared__ u64 sq[kTile + kTile / 16];
    __shared__ u64 s_wsum[4];
    __shared__ double s_z[4], s_z2[4];
    __shared__ u64 s_q2lo[4], s_q2hi[4];
    __shared__ unsigned s_tile, s_bad[4];
    __shared__ u64 s_prefix;

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) s_tile = atomicAdd(&ctrl->tile_next, 1u);
    __syncthreads();
    const unsigned tile = s_tile;
    const i64 base = (i64)tile * kTile;

    double z = 0.0, z2 = 0.0;
    U128 q2{0, 0};
    unsigned bad = 0;
    const u64 top = kQuant ? (1ull << qin.K) : 0;
    const double m = kQuant ? ctrl->m : 0.0;  // written by the max pass
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int s0 = r * 512 + 2 * tid;
        const i64 i0 = base + s0;
        u64 qa = 0, qb = 0;
        if (kQuant) {
            double a = -__builtin_huge_val(), b = -__builtin_huge_val();
            if (i0 + 1 < n) {
                if (qin.vec2) {
                    const double2 v = *reinterpret_cast<const double2 *>(qin.lw + i0);
                    a = v.x;
                    b = v.y;
                } else {
                    a = qin.lw[i0];
                    b = qin.lw[i0 + 1];
                }
            } else if (i0 < n) {
                a = qin.lw[i0];
            }
            if (i0 < n) qa = quant_one(a, m, qin.K, top, z, z2, q2);
            if (i0 + 1 < n) qb = quant_one(b, m, qin.K, top, z, z2, q2);
        } else {
            i64 a = 0, b = 0;
            if (i0 < n) a = cin.nc[i0];
            if (i0 + 1 < n) b = cin.nc[i0 + 1];
            bad |= (a < 0) | (a > cin.n) | (b < 0) | (b > cin.n);
            qa = (a < 0 || a > cin.n) ? 0 : (u64)a;
            qb = (b < 0 || b > cin.n) ? 0 : (u64)b;
        }
        sq[kPad(s0)] = qa;
        sq[kPad(s0 + 1)] = qb;
    }
    __syncthreads();

    // sequential inclusive scan of this thread's 16 consecutive items
    u64 loc[kScanItems];
    u64 run = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        run += sq[kPad(tid * kScanItems + j)];
        loc[j] = run;
    }
    // block scan of the per-thread totals
    const u64 incl = wave_incl_scan_u64(run);
    if (lane == 63) s_wsum[wid] = incl;
    __syncthreads();
    u64 wpre = 0, agg = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        wpre += (i < wid) ? s_wsum[i] : 0;
        agg += s_wsum[i];
    }
    const u64 texcl = wpre + incl - run;

    // decoupled lookback (wave 0)
    if (wid == 0) {
        u64 excl = 0;
        if (tile == 0) {
            if (lane == 0) st_relaxed(&status[0], kFlagInc | agg);
        } else {
            if (lane == 0) st_relaxed(&status[tile], kFlagAgg | agg);
            i64 top_idx = (i64)tile - 1;
            while (true) {
                const i64 idx = top_idx - lane;
                const u64 sv = idx >= 0 ? ld_relaxed(&status[idx]) : kFlagInc;
                const u64 flag = sv >> 62;
                const u64 inc_mask = __ballot(flag == 2);
                const u64 zero_mask = __ballot(flag == 0);
                const int first_inc = inc_mask ? __ffsll((long long)inc_mask) - 1 : 64;
                const u64 need = first_inc >= 64 ? ~0ull : ((1ull << first_inc) - 1);
                if (zero_mask & need) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                u64 v = lane <= first_inc ? (sv & kValMask) : 0;
                for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
                excl += v;
                if (first_inc < 64) break;
                top_idx -= 64;
            }
            if (lane == 0) st_relaxed(&status[tile], kFlagInc | (excl + agg));
        }
        if (lane == 0) s_prefix = excl;
    }

    // tile partial sums (fixed reduction order: deterministic)
    if (kQuant) {
        z = wave_sum_f64(z);
        z2 = wave_sum_f64(z2);
        q2 = wave_sum_u128(q2);
        if (lane == 0) {
            s_z[wid] = z;
            s_z2[wid] = z2;
            s_q2lo[wid] = q2.lo;
            s_q2hi[wid] = q2.hi;
        }
    } else {
        bad = wave_or(bad);
        if (lane == 0) s_bad[wid] = bad;
    }
    __syncthreads();
    if (tid == 0) {
        if (kQuant) {
            TilePart p;
            p.Z = ((s_z[0] + s_z[1]) + s_z[2]) + s_z[3];
            p.Z2 = ((s_z2[0] + s_z2[1]) + s_z2[2]) + s_z2[3];
            U128 t{s_q2lo[0], s_q2hi[0]};
            for (int i = 1; i < 4; ++i) t = add128(t, U128{s_q2lo[i], s_q2hi[i]});
            p.q2lo = t.lo;
            p.q2hi = t.hi;
            tpart[tile] = p;
        } else if (s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3]) {
            atomicOr(&ctrl->ncopy_bad, 1u);
        }
    }
    const u64 pre = s_prefix + texcl;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) sq[kPad(tid * kScanItems + j)] = pre + loc[j];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int s0 = r * 512 + 2 * tid;
        const i64 i0 = base + s0;
        if (i0 + 1 < n) {
            ulonglong2 v;
            v.x = sq[kPad(s0)];
            v.y = sq[kPad(s0 + 1)];
            *reinterpret_cast<ulonglong2 *>(out + i0) = v;
        } else if (i0 < n) {
            out[i0] = sq[kPad(s0)];
        }
    }
}


hipError_t launch_quant_scan(const Work &w, const double *lw, int64_t n, int K, hipStream_t s)
{
    QuantIn q{lw, K, ((uintptr_t)lw & 15) == 0};
    CountIn c{nullptr, 0};
    hipLaunchKernelGGL(k_scan<true>, dim3(w.n_tiles), dim3(256), 0, s, q, c, (i64)n, w.ctrl,
                       w.status, w.tpart, w.pref);
    return hipGetLastError();
}

// Resets the scan state before a scan that no max pass precedes.
__global__ __launch_bounds__(256) void k_clear_scan(Ctrl *ctrl, u64 *status, int n_status)
{
    const i64 gtid = (i64)blockIdx.x * 256 + threadIdx.x, gsz = (i64)gridDim.x * 256;
    for (i64 i = gtid; i < n_status; i += gsz) status[i] = 0;
    if (gtid == 0) {
        ctrl->tile_next = 0;
        ctrl->ncopy_bad = 0;
        ctrl->err_call = 0;
        ctrl->pending = 0;
    }
}

hipError_t launch_clear_scan(const Work &w, hipStream_t s)
{
    int blocks = (w.n_tiles + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > kMaxBlocks ? kMaxBlocks : blocks);
    hipLaunchKernelGGL(k_clear_scan, dim3(blocks), dim3(256), 0, s, w.ctrl, w.status, w.n_tiles);
    return hipGetLastError();
}

hipError_t launch_count_scan(const Work &w, const int64_t *ncopies, int64_t n, hipStream_t s)
{
    QuantIn q{nullptr, 0, 0};
    CountIn c{reinterpret_cast<const i64 *>(ncopies), (i64)n};
    hipLaunchKernelGGL(k_scan<false>, dim3(w.n_tiles), dim3(256), 0, s, q, c, (i64)n, w.ctrl,
                       w.status, w.tpart, w.pref);
    return hipGetLastError();
}

// ------------------------------------------------------------- finalize
// One workgroup.  Tile partials are summed in a fixed order, so the FP64
// outputs are reproducible run to run; the integer outputs are exact.
__global__ __launch_bounds__(256) void k_finalize_resample(Ctrl *ctrl, const TilePart *tpart,
                                                           const u64 *status, int n_tiles, i64 n,
                                                           u64 r, int mode, int ess_num,
                                                           int ess_den, int K,
                                                           smc_resample_info *info)
{
    __shared__ double s_z[4], s_z2[4];
    __shared__ u64 s_lo[4], s_hi[4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double z = 0.0, z2 = 0.0;
    U128 q2{0, 0};
    for (int t = tid; t < n_tiles; t += 256) {
        const TilePart p = tpart[t];
        z += p.Z;
        z2 += p.Z2;
        q2 = add128(q2, U128{p.q2lo, p.q2hi});
    }
    z = wave_sum_f64(z);
    z2 = wave_sum_f64(z2);
    q2 = wave_sum_u128(q2);
    if (lane == 0) {
        s_z[wid] = z;
        s_z2[wid] = z2;
        s_lo[wid] = q2.lo;
        s_hi[wid] = q2.hi;
    }
    __syncthreads();
    if (tid != 0) return;
    const double Z = ((s_z[0] + s_z[1]) + s_z[2]) + s_z[3];
    const double Z2 = ((s_z2[0] + s_z2[1]) + s_z2[2]) + s_z2[3];
    U128 Q2{s_lo[0], s_hi[0]};
    for (int i = 1; i < 4; ++i) Q2 = add128(Q2, U128{s_lo[i], s_hi[i]});
    const u64 S = status[n_tiles - 1] & kValMask;
    const unsigned err = ctrl->err_call;
    const double m = ctrl->m;

    int resample;
    if (mode == SMC_MODE_FORCE) {
        resample = 1;
    } else if (mode == SMC_MODE_NEVER) {
        resample = 0;
    } else {
        // ess_den * S^2 < ess_num * N * Q2, both sides < 2^127
        const U128 lhs = mul128_small(mul64(S, S), (u64)ess_den);
        const U128 rhs = mul128_small(mul128_small(Q2, (u64)n), (u64)ess_num);
        resample = lt128(lhs, rhs) ? 1 : 0;
    }
    if (err) resample = 0;
    const u64 U = mul64(r, S).hi;
    const double logZ = m + log(Z);
    const double ess = (Z * Z) / Z2;

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
    ctrl->pending = err ? 0 : 1;
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
        info->log_c = 0.0;
    }
}

hipError_t launch_finalize_resample(const Work &w, int64_t n, uint64_t r, int mode, int ess_num,
                                    int ess_den, int K, void *info, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_resample, dim3(1), dim3(256), 0, s, w.ctrl, w.tpart, w.status,
                       w.n_tiles, (i64)n, (u64)r, mode, ess_num, ess_den, K,
                       reinterpret_cast<smc_resample_info *>(info));
    return hipGetLastError();
}

}  // namespace smc
