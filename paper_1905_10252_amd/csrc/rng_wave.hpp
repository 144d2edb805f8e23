// Wave-cooperative standard normals, bit-identical to normal_pair().
//
// The polar method accepts a Philox draw with probability pi/4, so a wave of
// 64 lanes that retries in lockstep runs about 3.5 attempts (the maximum of 64
// geometric counts) although each lane needs 1.27 on average, and repeats the
// logarithm for every attempt in which some lane accepts.  Here every lane
// first tries attempt 0 of its own pair; the pairs still pending are then
// spread over the whole wave, L = floor(64 / pending) lanes per pair, each
// lane trying one later attempt of its pair.  A pair takes the lowest attempt
// that accepted, which is the draw the sequential definition takes, and the
// logarithm runs once per lane at the end.  All 64 lanes must call it in
// convergent control flow; lanes without a pair pass active = false.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "det.hpp"

namespace smc {

// Position of the n-th (0-based) set bit of m; requires n < popcount(m).
__device__ inline int nth_set_bit(uint64_t m, int n)
{
    int pos = 0;
#pragma unroll
    for (int sh = 32; sh; sh >>= 1) {
        const int c = __popcll((m >> pos) & ((1ull << sh) - 1ull));
        if (n >= c) {
            n -= c;
            pos += sh;
        }
    }
    return pos;
}

__device__ inline bool polar_uniforms(uint64_t seed, uint32_t tag, uint32_t sampler, uint32_t t,
                                      uint32_t idx, uint32_t sub, double &v1, double &v2)
{
    const Philox4 w = draw(seed, tag, sampler, t, idx, sub);
    const uint64_t b1 = ((uint64_t)w.v[1] << 32) | w.v[0];
    const uint64_t b2 = ((uint64_t)w.v[3] << 32) | w.v[2];
    v1 = (double)(b1 >> 11) * 0x1p-52 - 1.0;
    v2 = (double)(b2 >> 11) * 0x1p-52 - 1.0;
    const double s = v1 * v1 + v2 * v2;
    return s > 0.0 && s < 1.0;
}

__device__ inline void normal_pair_wave(uint64_t seed, uint32_t tag, uint32_t sampler, uint32_t t,
                                        uint32_t idx, uint32_t pair, bool active, double &z1,
                                        double &z2)
{
    constexpr uint32_t kAttempts = 32;
    const int lane = (int)__lane_id();
    double v1 = 0.0, v2 = 0.0;
    bool ok = active && polar_uniforms(seed, tag, sampler, t, idx, pair << 16, v1, v2);
    bool dead = false;         // all attempts rejected: the pair is (0, 0)
    uint32_t next = 1;         // next attempt of this lane's pair
    uint64_t pend = __ballot(active && !ok);
    while (pend) {
        const int r = __popcll(pend);
        const int L = 64 / r;
        const int j = lane / L, k = lane - j * L;
        const bool helper = j < r;
        const int owner = helper ? nth_set_bit(pend, j) : lane;
        const uint32_t o_idx = (uint32_t)__shfl((int)idx, owner);
        const uint32_t o_pair = (uint32_t)__shfl((int)pair, owner);
        const uint32_t a = (uint32_t)__shfl((int)next, owner) + (uint32_t)k;
        double h1 = 0.0, h2 = 0.0;
        const bool hok = helper && a < kAttempts &&
                         polar_uniforms(seed, tag, sampler, t, o_idx, (o_pair << 16) | a, h1, h2);
        const uint64_t acc = __ballot(hok);
        const bool own = (pend >> lane) & 1ull;
        const int rank = __popcll(pend & ((1ull << lane) - 1ull));
        const uint64_t seg = own ? (acc >> (rank * L)) & (L == 64 ? ~0ull : ((1ull << L) - 1ull))
                                 : 0ull;
        const int src = seg ? rank * L + __ffsll((long long)seg) - 1 : lane;
        const double f1 = __shfl(h1, src), f2 = __shfl(h2, src);
        if (seg) {
            v1 = f1;
            v2 = f2;
            ok = true;
        } else if (own) {
            next += (uint32_t)L;
            dead = next >= kAttempts;
        }
        pend = __ballot(own && !ok && !dead);
    }
    if (ok) {
        const double s = v1 * v1 + v2 * v2;
        const double c = (-2.0 * det_log(s)) / s;
        const double f = det_sqrt(c);
        z1 = v1 * f;
        z2 = v2 * f;
    } else {
        z1 = 0.0;
        z2 = 0.0;
    }
}

}  // namespace smc
