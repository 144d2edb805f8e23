// Grid-wide exact max of the log-weights with the last-block-done pattern:
// each block publishes its max order key and non-finite flag; the block that
// finishes last combines them (max is order-free, so the result is exact and
// does not depend on scheduling), records the error of the call and resets
// the counters the following scan pass relies on.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace smc {

// Call with every thread of a 256-thread block; key/bad are per-thread values.
// Returns the block's max key to every thread.
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

__device__ inline void grid_max_combine(u64 blk_k, unsigned blk_b, Ctrl *ctrl, u64 *blk_key,
                                        unsigned *blk_bad)
{
    __shared__ int s_last;
    const int tid = threadIdx.x;
    if (tid == 0) {
        blk_key[blockIdx.x] = blk_k;
        blk_bad[blockIdx.x] = blk_b;
        __threadfence();
        s_last = atomicAdd(&ctrl->blk_done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    u64 key = 0;
    unsigned bad = 0;
    for (int i = tid; i < (int)gridDim.x; i += blockDim.x) {
        const u64 k = __hip_atomic_load(&blk_key[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        key = k > key ? k : key;
        bad |= __hip_atomic_load(&blk_bad[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    key = block_max_key(key, bad);
    if (tid == 0) {
        unsigned err = 0;
        if (bad) err = kErrNonfinite;
        else if (key <= okey(-__builtin_huge_val())) err = kErrDegenerate;
        ctrl->mkey = key;
        ctrl->m = okey_inv(key);
        ctrl->err_call = err;
        if (err && !ctrl->err_latch) ctrl->err_latch = err;
        ctrl->blk_done = 0;
        ctrl->tile_next = 0;
        ctrl->pending = 0;
    }
}

}  // namespace smc
