// Device-side building blocks shared by the libsmc kernels: the workspace
// control block, 128-bit integer helpers, wave-level reductions and scans for
// 64-wide CDNA wavefronts, and the ordered-integer image of FP64 values.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

typedef unsigned long long u64;
typedef long long i64;

constexpr int kWave = 64;

// Decoupled-lookback status word: 2 flag bits above a 62-bit prefix value.
constexpr u64 kFlagAgg = 1ull << 62;   // tile aggregate published
constexpr u64 kFlagInc = 2ull << 62;   // inclusive prefix published
constexpr u64 kValMask = (1ull << 62) - 1;

// Error bits found on the device (same numbering as smc_status).
constexpr unsigned kErrArg = 1, kErrNonfinite = 2, kErrDegenerate = 3;

// Control block at the start of the workspace.  Every kernel of one call
// sequence communicates through it; no host round trip is needed.
struct Ctrl {
    u64 mkey;            // order key of the max log-weight (written by the fold)
    u64 ctotal;          // total of caller-supplied counts (count scan)
    unsigned err_call;   // device error of the current call (0 = none)
    unsigned err_latch;  // sticky error, cleared by smc_sync_error
    unsigned resample;   // decision of the last resample (1 = resample)
    unsigned ncopy_bad;  // foreign ncopies: a negative count was seen
    u64 S, U, Q2hi, Q2lo;
    double m, logZ, ess, Z, Z2;
    int K;
    int pending;         // 1: S prefix in the workspace belongs to the last resample
    // sampler state
    double logZ_prev;    // log sum w_{t-1} (0 after a reset)
    double lc_max;       // running max of log c_t
    double rec_den;      // sum_t c_t exp(-lc_max)
    double log_c;
    int rec_steps;
    unsigned uniform;    // lazy reset: the weights are -ln N, logw in memory is stale
    double pad1[4];
};

// ------------------------------------------------------------ 128-bit ints
struct U128 {
    u64 lo, hi;
};

__host__ __device__ inline U128 mul64(u64 a, u64 b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return U128{a * b, __umul64hi(a, b)};
#else
    unsigned __int128 p = (unsigned __int128)a * b;
    return U128{(u64)p, (u64)(p >> 64)};
#endif
}

// a * b for a below 2^32: two 32 x 32 -> 64 products instead of a full
// 64 x 64 -> 128 one
__host__ __device__ inline U128 mul32x64(unsigned a, u64 b)
{
    const u64 lo = (u64)a * (unsigned)b;
    const u64 hi = (u64)a * (unsigned)(b >> 32);
    const u64 rlo = lo + (hi << 32);
    return U128{rlo, (hi >> 32) + (rlo < lo ? 1ull : 0ull)};
}

__host__ __device__ inline U128 add128(U128 a, U128 b)
{
    U128 r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (r.lo < a.lo ? 1ull : 0ull);
    return r;
}

__host__ __device__ inline U128 add128(U128 a, u64 b)
{
    U128 r;
    r.lo = a.lo + b;
    r.hi = a.hi + (r.lo < a.lo ? 1ull : 0ull);
    return r;
}

__host__ __device__ inline bool lt128(U128 a, U128 b)
{
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

// (a * b) mod 2^128 for a 128-bit a and a small b (b < 2^32).
__host__ __device__ inline U128 mul128_small(U128 a, u64 b)
{
    U128 lo = mul64(a.lo, b);
    lo.hi += a.hi * b;
    return lo;
}

// ------------------------------------------------------- FP64 order keys
__host__ __device__ inline u64 okey(double v)
{
    u64 b = (u64)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__host__ __device__ inline double okey_inv(u64 k)
{
    u64 b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// -------------------------------------------------- wave-level primitives
// Built on DPP lane moves (a VALU operand modifier, no LDS round trip).  GFX9
// controls: row_shr:n = 0x110 + n moves lane l - n of the same 16-lane row to
// lane l; row_bcast:15 = 0x142 moves lane 15 of each row to the next row (row
// mask 0xA: rows 1 and 3); row_bcast:31 = 0x143 moves lane 31 to rows 2 and 3
// (row mask 0xC).  A lane with no source (or outside the row mask) receives
// `fill`, the identity of the operation.  A scan is Hillis-Steele within each
// row (shifts 1, 2, 4, 8), then the row totals carried forward by the two
// broadcasts; lane 63 then holds the total, which a reduction broadcasts to
// every lane.  All 64 lanes must take part.
template <int CTRL, int ROW_MASK>
__device__ inline u64 dpp_u64(u64 v, u64 fill)
{
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)fill, (int)(unsigned)v, CTRL,
                                               ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(fill >> 32),
                                               (int)(unsigned)(v >> 32), CTRL, ROW_MASK, 0xF,
                                               false);
    return ((u64)(unsigned)hi << 32) | (u64)(unsigned)lo;
}

__device__ inline u64 lane63_u64(u64 v)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
    return ((u64)hi << 32) | lo;
}

// Inclusive scan over the wave of v under op (associative, identity `fill`).
template <class Op>
__device__ inline u64 wave_scan_u64(u64 v, u64 fill, Op op)
{
    v = op(v, dpp_u64<0x111, 0xF>(v, fill));
    v = op(v, dpp_u64<0x112, 0xF>(v, fill));
    v = op(v, dpp_u64<0x114, 0xF>(v, fill));
    v = op(v, dpp_u64<0x118, 0xF>(v, fill));
    v = op(v, dpp_u64<0x142, 0xA>(v, fill));
    v = op(v, dpp_u64<0x143, 0xC>(v, fill));
    return v;
}

__device__ inline u64 wave_max_u64(u64 v)
{
    return lane63_u64(wave_scan_u64(v, 0ull, [](u64 a, u64 b) { return b > a ? b : a; }));
}

// FP64 sum in a fixed order (the scan's): reproducible run to run.
__device__ inline double wave_sum_f64(double v)
{
    const u64 r = wave_scan_u64((u64)__double_as_longlong(v), 0ull, [](u64 a, u64 b) {
        return (u64)__double_as_longlong(__longlong_as_double((long long)a) +
                                         __longlong_as_double((long long)b));
    });
    return __longlong_as_double((long long)lane63_u64(r));
}

__device__ inline double wave_max_f64(double v)
{
    const u64 ninf = (u64)__double_as_longlong(-__builtin_huge_val());
    const u64 r = wave_scan_u64((u64)__double_as_longlong(v), ninf, [](u64 a, u64 b) {
        return (u64)__double_as_longlong(fmax(__longlong_as_double((long long)a),
                                              __longlong_as_double((long long)b)));
    });
    return __longlong_as_double((long long)lane63_u64(r));
}

__device__ inline double lane_f64(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((u64)hi << 32) | lo));
}

template <int CTRL, int ROW_MASK>
__device__ inline U128 dpp_u128(U128 v)
{
    return U128{dpp_u64<CTRL, ROW_MASK>(v.lo, 0ull), dpp_u64<CTRL, ROW_MASK>(v.hi, 0ull)};
}

__device__ inline U128 wave_sum_u128(U128 v)
{
    v = add128(v, dpp_u128<0x111, 0xF>(v));
    v = add128(v, dpp_u128<0x112, 0xF>(v));
    v = add128(v, dpp_u128<0x114, 0xF>(v));
    v = add128(v, dpp_u128<0x118, 0xF>(v));
    v = add128(v, dpp_u128<0x142, 0xA>(v));
    v = add128(v, dpp_u128<0x143, 0xC>(v));
    return U128{lane63_u64(v.lo), lane63_u64(v.hi)};
}

__device__ inline unsigned wave_or(unsigned v)
{
    return (unsigned)lane63_u64(wave_scan_u64(v, 0ull, [](u64 a, u64 b) { return a | b; }));
}

// Inclusive scan of u64 across the 64 lanes of a wavefront.
__device__ inline u64 wave_incl_scan_u64(u64 v)
{
    return wave_scan_u64(v, 0ull, [](u64 a, u64 b) { return a + b; });
}

// Device-scope relaxed atomics on 64-bit words (coherent across XCDs).
__device__ inline u64 ld_relaxed(const u64 *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void st_relaxed(u64 *p, u64 v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace smc
