// Wave-cooperative standard normals, bit-identical to normal_pair().
//
// The polar method accepts a Philox draw with probability pi/4, so a wave of
// 64 lanes that retries in lockstep runs about 3.5 attempts (the maximum of 64
// geometric counts) although each lane needs 1.27 on average, and repeats the
// logarithm for every attempt in which some lane accepts.  Here every lane
// first tries attempt 0 of its own pair; the pairs still pending are then
// spread over the whole wave, L = floor(64 / pending) lanes per pair, each
// lane trying one later attempt of its pair (jobs and results pass through a
// per-wave LDS buffer).  A pair takes the lowest attempt
// that accepted, which is the draw the sequential definition takes, and the
// logarithm runs once per lane at the end.  All 64 lanes must call it in
// convergent control flow; lanes without a pair pass active = false.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "det.hpp"

namespace smc {

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

// xch: this wave's 64-entry exchange buffer in LDS (16 bytes a lane).  Lanes
// of one wave read and write it in program order, so no barrier is needed.
// kSc: the logarithm's coefficients as scalar operands (see coef()).
template <bool kSc = false>
__device__ inline void normal_pair_wave(uint64_t seed, uint32_t tag, uint32_t sampler, uint32_t t,
                                        uint32_t idx, uint32_t pair, bool active, double &z1,
                                        double &z2, uint4 *xch)
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
        const bool own = (pend >> lane) & 1ull;
        const int rank = (int)__builtin_amdgcn_mbcnt_hi(
            (unsigned)(pend >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)pend, 0u));
        // pending pair number `rank` is posted at entry `rank`; helpers of
        // pair j (L lanes each) read entry j and try the next L attempts
        if (own) xch[rank] = make_uint4(idx, pair, next, 0u);
        __builtin_amdgcn_wave_barrier();
        const int j = lane / L, k = lane - j * L;
        const bool helper = j < r;
        const uint4 job = helper ? xch[j] : make_uint4(0u, 0u, 0u, 0u);
        const uint32_t a = job.z + (uint32_t)k;
        double h1 = 0.0, h2 = 0.0;
        const bool hok = helper && a < kAttempts &&
                         polar_uniforms(seed, tag, sampler, t, job.x, (job.y << 16) | a, h1, h2);
        const uint64_t acc = __ballot(hok);
        __builtin_amdgcn_wave_barrier();
        xch[lane] = make_uint4((uint32_t)__double2loint(h1), (uint32_t)__double2hiint(h1),
                               (uint32_t)__double2loint(h2), (uint32_t)__double2hiint(h2));
        __builtin_amdgcn_wave_barrier();
        const uint64_t seg = own ? (acc >> (rank * L)) & (L == 64 ? ~0ull : ((1ull << L) - 1ull))
                                 : 0ull;
        if (seg) {
            const uint4 h = xch[rank * L + __ffsll((long long)seg) - 1];
            v1 = __hiloint2double((int)h.y, (int)h.x);
            v2 = __hiloint2double((int)h.w, (int)h.z);
            ok = true;
        } else if (own) {
            next += (uint32_t)L;
            dead = next >= kAttempts;
        }
        __builtin_amdgcn_wave_barrier();
        pend = __ballot(own && !ok && !dead);
    }
    if (ok) {
        const double s = v1 * v1 + v2 * v2;
        const double c = (-2.0 * det_log<kSc>(s)) / s;
        const double f = det_sqrt(c);
        z1 = v1 * f;
        z2 = v2 * f;
    } else {
        z1 = 0.0;
        z2 = 0.0;
    }
}

}  // namespace smc
