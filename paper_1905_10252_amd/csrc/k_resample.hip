// Resampling kernels of Alg 4 (minimum variance resampling):
//   k_max          exact FP64 max of the log-weights (the stability shift of
//                  eq. normalise) and non-finite detection.
//   k_fold         combines the max slots, records the error of the call
//                  (used where no scan follows the max pass).
//   k_scan<true>   one pass over the log-weights: 64-bit fixed-point weights
//                  q_i = min(2^K, floor(2^K det_exp(l_i - m))), FP64 sums for
//                  log-sum-exp and ESS (eq. normalise, eq. neff), the exact
//                  sum of q_i^2, and the prefix sums of q within each tile of
//                  4096 weights, plus the tile's total.
//   k_scan<false>  the same tile scan over caller-supplied int64 ncopies.
//   k_decide       the exclusive prefix of the tile totals (so that the
//                  inclusive prefix S_j of the Cumulative Sum of MVR is the
//                  tile-local value plus its tile's offset), the error of the
//                  call, the exact integer ESS decision (resample when
//                  ESS < N*, Alg 2), the systematic offset U = floor(r S / 2^64),
//                  log Z and the FP64 ESS from the tile partials; clears the
//                  other parity's max slots.
//   k_tile_prefix  the tile offsets alone, for caller-supplied counts.
// No tile waits on another: the scan is split into tile-local prefixes and
// one small scan over the tile totals, so no kernel here spins, and none uses
// a device-wide fence or a contended atomic.
// Every 64th tile-local prefix value is also written to a sample array, a
// coarse index for the merge-path searches of the expand kernel.
#include <hip/hip_runtime.h>

#include "../../include/smc.h"
#include "common.hpp"
#include "det.hpp"
#include "kernels.hpp"
#include "stats.hpp"
#include "reduce.hpp"

namespace smc {

// ------------------------------------------------------------- control init
__global__ void k_init_ctrl(Ctrl *ctrl, u64 *slots)
{
    u64 *p = reinterpret_cast<u64 *>(ctrl);
    for (int i = threadIdx.x; i < (int)(sizeof(Ctrl) / 8); i += blockDim.x) p[i] = 0;
    for (int i = threadIdx.x; i < kSlotWords; i += blockDim.x) slots[i] = 0;
}

hipError_t launch_init_ctrl(const Work &w, hipStream_t s)
{
    static_assert(sizeof(Ctrl) % 8 == 0, "ctrl size");
    hipLaunchKernelGGL(k_init_ctrl, dim3(1), dim3(256), 0, s, w.ctrl, w.slots);
    return hipGetLastError();
}

// ------------------------------------------------------------- exact max
// Grid-stride share per block, four 16-byte loads in flight per thread; each
// block publishes its max order key into the slots of this call's parity.
// The loads are non-temporal, here and in the scan: the weights are read once
// by each pass, and streaming them past the caches measured faster on MI355X
// than keeping them (N = 2^24: about 10 us less for the resample call).
typedef double f64x2_t __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_max(const double *__restrict__ lw, i64 n, int vec2,
                                             u64 *slots_p)
{
    // two 16-byte loads in flight per thread: 1-2 us faster per call at
    // N = 2^24 than four or eight (and than one)
    constexpr int U = 2;
    const int tid = threadIdx.x;
    const i64 gtid = (i64)blockIdx.x * 256 + tid, gsz = (i64)gridDim.x * 256;

    u64 key = 0;
    unsigned bad = 0;
    const double ninf = -__builtin_huge_val();
    auto take = [&](double v) {
        bad |= (v != v) | (v == __builtin_huge_val());
        const u64 k = okey(v);
        key = k > key ? k : key;
    };
    if (vec2) {
        const i64 npair = n >> 1;
        const f64x2_t *lw2 = reinterpret_cast<const f64x2_t *>(lw);
        for (i64 i = gtid; i < npair; i += U * gsz) {
            f64x2_t v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const i64 j = i + u * gsz;
                v[u] = j < npair ? __builtin_nontemporal_load(lw2 + j) : f64x2_t{ninf, ninf};
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                take(v[u].x);
                take(v[u].y);
            }
        }
        if ((n & 1) && gtid == 0) take(lw[n - 1]);
    } else {
        for (i64 i = gtid; i < n; i += gsz) take(lw[i]);
    }
    const u64 bk = block_max_key(key, bad);
    slot_publish(slots_p, bk, bad);
}

hipError_t launch_max(const Work &w, const double *lw, int64_t n, int par, hipStream_t s)
{
    const int vec2 = ((uintptr_t)lw & 15) == 0;
    hipLaunchKernelGGL(k_max, dim3(max_blocks_of(n)), dim3(256), 0, s, lw, (i64)n, vec2,
                       w.slots + (par & 1) * kSlots * kSlotStride);
    return hipGetLastError();
}

// One wavefront: max over the 64 slots of parity par, the call's error
// (NaN or +inf seen: non-finite; max = -inf: every weight zero), and a clear
// of the other parity's slots for the next call.
__global__ __launch_bounds__(64) void k_fold(u64 *slots, int par, Ctrl *ctrl)
{
    const int lane = threadIdx.x;
    u64 *cur = slots + (par & 1) * kSlots * kSlotStride;
    u64 *nxt = slots + ((par & 1) ^ 1) * kSlots * kSlotStride;
    const u64 key = wave_max_u64(cur[lane * kSlotStride]);
    const unsigned bad = wave_or((unsigned)cur[lane * kSlotStride + 1]);
    nxt[lane * kSlotStride] = 0;
    nxt[lane * kSlotStride + 1] = 0;
    if (lane == 0) {
        unsigned err = 0;
        if (bad) err = kErrNonfinite;
        else if (key <= okey(-__builtin_huge_val())) err = kErrDegenerate;
        ctrl->mkey = key;
        ctrl->m = okey_inv(key);
        ctrl->err_call = err;
        if (err && !ctrl->err_latch) ctrl->err_latch = err;
        ctrl->pending = 0;
    }
}

hipError_t launch_fold(const Work &w, int par, hipStream_t s)
{
    hipLaunchKernelGGL(k_fold, dim3(1), dim3(64), 0, s, w.slots, par, w.ctrl);
    return hipGetLastError();
}

// ------------------------------------------------------------ tile scan
// Tile = kScanThreads threads x kScanItems items; tile t is workgroup t.
// Global loads and stores are coalesced 16-byte accesses over rows of
// 2 kScanThreads elements; an LDS transpose gives each thread kScanItems
// consecutive items for the sequential part of the scan.  Entry i of the
// transpose sits at slot (i ^ (i >> 5)) & 15 of its 16-entry block (a
// bijection): in both the striped and the per-thread accesses at most two
// lanes of a wave meet on a bank pair, the minimum for 8-byte accesses, with
// no pad words.
// The prefix written is local to the tile; the tile's total goes to tsum[t],
// which the following single-workgroup pass turns into tile offsets.  A
// chained scan (each tile waiting for its predecessors' totals) costs a
// round trip through the memory system per tile in flight; this split costs
// one small pass over 8 bytes per 4096 weights instead.
__host__ __device__ constexpr int kPad(int i) { return (i & ~15) | ((i ^ (i >> 5)) & 15); }
constexpr int kScanWaves = kScanThreads / 64;
constexpr int kScanRow = 2 * kScanThreads;  // elements per striped row
static_assert(kScanItems % 2 == 0 && 64 % kScanItems == 0, "scan tile shape");

struct ScanArgs {
    const double *lw;   // quantise mode input
    const i64 *nc;      // count mode input
    i64 n;
    int K, vec2;
    Ctrl *ctrl;
    u64 *tsum;          // [n_tiles] tile totals
    TilePart *tpart;
    u64 *out;           // [n] tile-local inclusive prefix
    u64 *out64;         // [n / 64] every 64th tile-local prefix value
    const u64 *slots_p; // max slots of this call's parity (quantise mode)
    unsigned *uniform;  // lazy-reset flag to clear (nullable)
    int n_tiles;
};

// Fixed-point weight of one log-weight; accumulates the FP64 and exact sums.
// The exponential takes its coefficients as scalar operands (coef()): with
// sixteen of them per thread the vector moves would otherwise be a sixth of
// the scan's vector instructions (measured: 2 to 3 us less per call at
// N = 2^24).
__device__ inline u64 quant_one(double v, double m, int K, u64 top, double &z, double &z2, U128 &q2)
{
    const double e = det_exp<true>(v - m);
    if (!(e >= 0.0)) return 0;  // NaN input: the max pass has flagged it
    z += e;
    z2 += e * e;
    const double f = floor(ldexp(e, K));
    u64 q = (u64)f;
    q = q > top ? top : q;
    // q < 2^53: q = h 2^32 + l, q^2 = l^2 + 2 h l 2^32 + h^2 2^64
    const unsigned l = (unsigned)q, h = (unsigned)(q >> 32);
    const u64 ll = (u64)l * l, hl = (u64)h * l, hh = (u64)h * h;
    const u64 lo1 = q2.lo + ll;
    const u64 c1 = lo1 < ll ? 1ull : 0ull;
    const u64 s = hl << 33;
    const u64 lo2 = lo1 + s;
    const u64 c2 = lo2 < s ? 1ull : 0ull;
    q2.lo = lo2;
    q2.hi += hh + (hl >> 31) + c1 + c2;
    return q;
}

template <bool kQuant>
__global__ __launch_bounds__(kScanThreads) void k_scan(ScanArgs a)
{
    __shared__ u64 sq[kTile];
    __shared__ u64 s_wsum[kScanWaves];
    __shared__ double s_z[kScanWaves], s_z2[kScanWaves];
    __shared__ u64 s_q2lo[kScanWaves], s_q2hi[kScanWaves];
    __shared__ unsigned s_bad[kScanWaves];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const i64 n = a.n;
    const unsigned tile = blockIdx.x;
    const i64 base = (i64)tile * kTile;
    const bool full = base + kTile <= n;

    double z = 0.0, z2 = 0.0;
    U128 q2{0, 0};
    unsigned bad = 0;
    u64 q[kScanItems];  // striped: q[2r + h] is element base + kScanRow r + 2 tid + h
    if (kQuant) {
        // every wave folds the 64 max slots itself (cached lines; no barrier)
        const double m = okey_inv(wave_max_u64(a.slots_p[lane * kSlotStride]));
        const int K = a.K;
        const u64 top = 1ull << K;
        double v[kScanItems];
        if (full && a.vec2) {
#pragma unroll
            for (int r = 0; r < kScanItems / 2; ++r) {
                const f64x2_t t = __builtin_nontemporal_load(
                    reinterpret_cast<const f64x2_t *>(a.lw + base + r * kScanRow + 2 * tid));
                v[2 * r] = t.x;
                v[2 * r + 1] = t.y;
            }
        } else {
#pragma unroll
            for (int e = 0; e < kScanItems; ++e) {
                const i64 i = base + (e >> 1) * kScanRow + 2 * tid + (e & 1);
                v[e] = i < n ? a.lw[i] : -__builtin_huge_val();
            }
        }
#pragma unroll
        for (int e = 0; e < kScanItems; ++e) q[e] = quant_one(v[e], m, K, top, z, z2, q2);
    } else {
        i64 c[kScanItems];
#pragma unroll
        for (int e = 0; e < kScanItems; ++e) {
            const i64 i = base + (e >> 1) * kScanRow + 2 * tid + (e & 1);
            c[e] = i < n ? a.nc[i] : 0;
        }
#pragma unroll
        for (int e = 0; e < kScanItems; ++e) {
            const bool ok = c[e] >= 0 && c[e] <= n;
            bad |= ok ? 0u : 1u;
            q[e] = ok ? (u64)c[e] : 0ull;
        }
    }
#pragma unroll
    for (int e = 0; e < kScanItems; ++e) sq[kPad((e >> 1) * kScanRow + 2 * tid + (e & 1))] = q[e];
    __syncthreads();

    // sequential inclusive scan of this thread's 16 consecutive items
    u64 loc[kScanItems];
    u64 run = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        run += sq[kPad(tid * kScanItems + j)];
        loc[j] = run;
    }
    const u64 incl = wave_incl_scan_u64(run);
    if (lane == 63) s_wsum[wid] = incl;
    // tile partial sums (fixed reduction order: reproducible)
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
    u64 wpre = 0, agg = 0;
#pragma unroll
    for (int i = 0; i < kScanWaves; ++i) {
        wpre += (i < wid) ? s_wsum[i] : 0;
        agg += s_wsum[i];
    }
    // each thread rewrites only the 16 entries it read above
    const u64 pre = wpre + incl - run;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) sq[kPad(tid * kScanItems + j)] = pre + loc[j];
    // every 64th prefix value (item 64g + 63 is the last item of its thread)
    if (((tid + 1) * kScanItems) % 64 == 0) {
        const i64 gi = base + tid * kScanItems + (kScanItems - 1);
        if (gi < n) a.out64[gi >> 6] = pre + loc[kScanItems - 1];
    }
    if (tid == 0) {
        if (a.uniform && tile == 0) *a.uniform = 0u;
        a.tsum[tile] = agg;
        if (kQuant) {
            TilePart p;
            double Z = s_z[0], Z2 = s_z2[0];
            U128 t{s_q2lo[0], s_q2hi[0]};
            for (int i = 1; i < kScanWaves; ++i) {
                Z += s_z[i];
                Z2 += s_z2[i];
                t = add128(t, U128{s_q2lo[i], s_q2hi[i]});
            }
            p.Z = Z;
            p.Z2 = Z2;
            p.q2lo = t.lo;
            p.q2hi = t.hi;
            a.tpart[tile] = p;
        } else {
            unsigned b = 0;
            for (int i = 0; i < kScanWaves; ++i) b |= s_bad[i];
            if (b) atomicOr(&a.ctrl->ncopy_bad, 1u);
        }
    }
    __syncthreads();
    if (full) {
#pragma unroll
        for (int r = 0; r < kScanItems / 2; ++r) {
            const int s0 = r * kScanRow + 2 * tid;
            ulonglong2 v;
            v.x = sq[kPad(s0)];
            v.y = sq[kPad(s0 + 1)];
            *reinterpret_cast<ulonglong2 *>(a.out + base + s0) = v;
        }
    } else {
#pragma unroll
        for (int e = 0; e < kScanItems; ++e) {
            const int s0 = (e >> 1) * kScanRow + 2 * tid + (e & 1);
            if (base + s0 < n) a.out[base + s0] = sq[kPad(s0)];
        }
    }
}

// Exclusive prefix of the tile totals, in place, by one workgroup of 1024
// threads (each a contiguous run of tiles); returns the grand total to every
// thread.
__device__ inline u64 tile_offsets(u64 *tsum, int n_tiles, u64 *s_w)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int per = (n_tiles + 1023) / 1024;
    const int t0 = tid * per;
    u64 run = 0;
    for (int i = 0; i < per; ++i)
        if (t0 + i < n_tiles) run += tsum[t0 + i];
    const u64 incl = wave_incl_scan_u64(run);
    if (lane == 63) s_w[wid] = incl;
    __syncthreads();
    u64 pre = 0, total = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        pre += (i < wid) ? s_w[i] : 0;
        total += s_w[i];
    }
    pre += incl - run;
    for (int i = 0; i < per; ++i)
        if (t0 + i < n_tiles) {
            const u64 v = tsum[t0 + i];
            tsum[t0 + i] = pre;
            pre += v;
        }
    return total;
}

// Caller-supplied counts: tile offsets and their total (checked against N by
// the expand).
__global__ __launch_bounds__(1024) void k_tile_prefix(Ctrl *ctrl, u64 *tsum, int n_tiles)
{
    __shared__ u64 s_w[16];
    const u64 total = tile_offsets(tsum, n_tiles, s_w);
    if (threadIdx.x == 0) ctrl->ctotal = total;
}

// ---------------------------------------------------------------- decision
// One workgroup: tile offsets; tile partials summed in a fixed order
// (reproducible FP64); exact integer decision and offset.
__global__ __launch_bounds__(1024) void k_decide(Ctrl *ctrl, u64 *slots, int par,
                                                 const TilePart *tpart, u64 *tsum,
                                                 int n_tiles, i64 n, int K, u64 r, int mode,
                                                 int ess_num, int ess_den,
                                                 smc_resample_info *info, StatsArgs st)
{
    __shared__ double s_z[16], s_z2[16];
    __shared__ u64 s_lo[16], s_hi[16];
    __shared__ u64 s_key, s_w[16];
    __shared__ unsigned s_badf;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const u64 S = tile_offsets(tsum, n_tiles, s_w);
    if (wid == 0) {
        u64 *cur = slots + (par & 1) * kSlots * kSlotStride;
        u64 *nxt = slots + ((par & 1) ^ 1) * kSlots * kSlotStride;
        const u64 key = wave_max_u64(cur[lane * kSlotStride]);
        const unsigned bad = wave_or((unsigned)cur[lane * kSlotStride + 1]);
        nxt[lane * kSlotStride] = 0;
        nxt[lane * kSlotStride + 1] = 0;
        if (lane == 0) {
            s_key = key;
            s_badf = bad;
        }
    }
    double z = 0.0, z2 = 0.0;
    U128 q2{0, 0};
    constexpr int FU = 4;  // partials in flight per thread; summed in tile order
    for (int t0 = tid; t0 < n_tiles; t0 += 1024 * FU) {
        TilePart p[FU];
#pragma unroll
        for (int u = 0; u < FU; ++u) {
            const int t = t0 + 1024 * u;
            p[u] = t < n_tiles ? tpart[t] : TilePart{0.0, 0.0, 0ull, 0ull};
        }
#pragma unroll
        for (int u = 0; u < FU; ++u) {
            z += p[u].Z;
            z2 += p[u].Z2;
            q2 = add128(q2, U128{p[u].q2lo, p[u].q2hi});
        }
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
    if (tid == 0) {
        double Z = s_z[0], Z2 = s_z2[0];
        U128 Q2{s_lo[0], s_hi[0]};
        for (int i = 1; i < 16; ++i) {
            Z += s_z[i];
            Z2 += s_z2[i];
            Q2 = add128(Q2, U128{s_lo[i], s_hi[i]});
        }
        const u64 key = s_key;
        const double m = okey_inv(key);
        unsigned err = 0;
        if (s_badf) err = kErrNonfinite;
        else if (key <= okey(-__builtin_huge_val())) err = kErrDegenerate;
        ctrl->mkey = key;
        ctrl->m = m;
        ctrl->err_call = err;
        if (err && !ctrl->err_latch) ctrl->err_latch = err;
        int resample;
        if (mode == SMC_MODE_FORCE) {
            resample = 1;
        } else if (mode == SMC_MODE_NEVER) {
            resample = 0;
        } else {
            // ess_den * S^2 < ess_num * N * Q2; both sides stay below 2^127
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
    // a sampler iteration's statistics follow the decision in the same
    // workgroup (they read the log Z and the decision written above)
    if (st.is_part) {
        __syncthreads();
        step_stats_block<1024>(ctrl, st.is_part, st.nblk, st.d, st.rec_num, st.est, info, 0);
    }
}

hipError_t launch_decide(const Work &w, int par, int64_t n, int K, uint64_t r, int mode,
                         int ess_num, int ess_den, void *info, hipStream_t s,
                         const StatsArgs &st)
{
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(1024), 0, s, w.ctrl, w.slots, par, w.tpart,
                       w.tsum, w.n_tiles, (i64)n, K, (u64)r, mode, ess_num, ess_den,
                       reinterpret_cast<smc_resample_info *>(info), st);
    return hipGetLastError();
}

hipError_t launch_quant_scan(const Work &w, const double *lw, int64_t n, int K, int par,
                             hipStream_t s, bool clear_uniform)
{
    ScanArgs a;
    a.uniform = clear_uniform ? &w.ctrl->uniform : nullptr;
    a.lw = lw;
    a.nc = nullptr;
    a.n = n;
    a.K = K;
    a.vec2 = ((uintptr_t)lw & 15) == 0;
    a.ctrl = w.ctrl;
    a.tsum = w.tsum;
    a.tpart = w.tpart;
    a.out = w.pref;
    a.out64 = w.pref64;
    a.slots_p = w.slots + (par & 1) * kSlots * kSlotStride;
    a.n_tiles = w.n_tiles;
    hipLaunchKernelGGL(k_scan<true>, dim3(w.n_tiles), dim3(kScanThreads), 0, s, a);
    return hipGetLastError();
}

// eq. normalise: w_i = exp(l_i - m) / Z with the max and the FP64 sum of
// the last decision (nothing is written when that call found an error).
__global__ __launch_bounds__(256) void k_weights(const Ctrl *ctrl, const double *lw, i64 n,
                                                 double *w)
{
    if (ctrl->err_call) return;
    const double m = ctrl->m, Z = ctrl->Z;
    const i64 gtid = (i64)blockIdx.x * 256 + threadIdx.x, gsz = (i64)gridDim.x * 256;
    for (i64 i = gtid; i < n; i += gsz) w[i] = det_exp(lw[i] - m) / Z;
}

hipError_t launch_weights(const Work &w, const double *lw, int64_t n, double *out, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    blocks = blocks > 8192 ? 8192 : blocks;
    hipLaunchKernelGGL(k_weights, dim3((unsigned)blocks), dim3(256), 0, s, w.ctrl, lw, (i64)n, out);
    return hipGetLastError();
}

// Resets the per-call flags before a scan of caller-supplied counts.
__global__ void k_clear_scan(Ctrl *ctrl)
{
    ctrl->ncopy_bad = 0;
    ctrl->err_call = 0;
    ctrl->pending = 0;
}

hipError_t launch_clear_scan(const Work &w, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_scan, dim3(1), dim3(1), 0, s, w.ctrl);
    return hipGetLastError();
}

hipError_t launch_count_scan(const Work &w, const int64_t *ncopies, int64_t n, hipStream_t s)
{
    ScanArgs a;
    a.uniform = nullptr;
    a.lw = nullptr;
    a.nc = reinterpret_cast<const i64 *>(ncopies);
    a.n = n;
    a.K = 0;
    a.vec2 = 0;
    a.ctrl = w.ctrl;
    a.tsum = w.tsum;
    a.tpart = w.tpart;
    a.out = w.pref;
    a.out64 = w.pref64;
    a.slots_p = nullptr;
    a.n_tiles = w.n_tiles;
    hipLaunchKernelGGL(k_scan<false>, dim3(w.n_tiles), dim3(kScanThreads), 0, s, a);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    hipLaunchKernelGGL(k_tile_prefix, dim3(1), dim3(1024), 0, s, w.ctrl, w.tsum, w.n_tiles);
    return hipGetLastError();
}

}  // namespace smc
