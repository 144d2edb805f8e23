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
    unsigned unused1;
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
__device__ inline u64 wave_max_u64(u64 v)
{
    for (int o = 32; o > 0; o >>= 1) {
        u64 w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

__device__ inline double wave_sum_f64(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ inline double wave_max_f64(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ inline U128 wave_sum_u128(U128 v)
{
    for (int o = 32; o > 0; o >>= 1) {
        U128 w;
        w.lo = __shfl_xor(v.lo, o, kWave);
        w.hi = __shfl_xor(v.hi, o, kWave);
        v = add128(v, w);
    }
    return v;
}

__device__ inline unsigned wave_or(unsigned v)
{
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, kWave);
    return v;
}

// Inclusive scan of u64 across the 64 lanes of a wavefront.
__device__ inline u64 wave_incl_scan_u64(u64 v)
{
    const int lane = threadIdx.x & (kWave - 1);
    for (int o = 1; o < kWave; o <<= 1) {
        u64 w = __shfl_up(v, o, kWave);
        if (lane >= o) v += w;
    }
    return v;
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
