// Grid-wide exact max of the log-weights without fences or contended
// atomics: every block publishes its max order key (and a non-finite flag)
// with one device-scope atomic into one of 64 slots, each on its own cache
// line, so the atomics do not serialise.  The slots are double-buffered by the
// parity of the call: a small fold kernel combines the current parity (max is
// order-free, so the result is exact) and clears the other parity for the
// next call.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace smc {

constexpr int kSlots = 64;
constexpr int kSlotStride = 16;  // u64 words: one 128-byte line per slot
constexpr int kSlotWords = 2 * kSlots * kSlotStride;

// Call with every thread of a 256-thread block; key/bad are per-thread values.
// Returns the block's max key (and OR of flags in bad) to every thread.
__device__ inline u64 block_max_key(u64 key, unsigned &bad)
{
    __shared__ u64 s_k[4];
    __shared__ unsigned s_b[4];
    const int tid = threadIdx.x;
    key = wave_max_u64(key);
    bad = wave_or(bad);
    if ((tid & 63) == 0) {
        s_k[tid >> 6] = key;
        s_b[tid >> 6] = bad;
    }
    __syncthreads();
    u64 k = s_k[0];
    unsigned b = s_b[0];
    for (int i = 1; i < 4; ++i) {
        k = s_k[i] > k ? s_k[i] : k;
        b |= s_b[i];
    }
    __syncthreads();
    bad = b;
    return k;
}

// slots_p: the kSlots slots of this call's parity.
__device__ inline void slot_publish(u64 *slots_p, u64 key, unsigned bad)
{
    if (threadIdx.x == 0) {
        u64 *s = slots_p + (blockIdx.x & (kSlots - 1)) * kSlotStride;
        atomicMax(s, key);
        if (bad) atomicOr(s + 1, 1ull);
    }
}

}  // namespace smc
