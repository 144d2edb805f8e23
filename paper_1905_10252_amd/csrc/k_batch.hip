// Batched SMC samplers: every attached sampler runs Alg 2 (random-walk
// proposal, L = q weights by eq. smcs_drawing_weights, estimates before
// resampling by eq. estimation_at_t, the exact-integer ESS decision and
// systematic resampling of Alg 4 in S-R order, reset to 1/N, c_t and
// recycling by eq. normconst and eq. recycling) on a Gaussian target with
// precision U^T U.  One step is one sequence of launches for all samplers:
//
//   k_bprop     per chunk of 256 particles of every sampler: the random-walk
//               proposal in place (normals generated wave-cooperatively).
//   k_bquad<DB> per chunk of samplers whose dimension falls in the bucket
//               (DB - 8, DB]: |U (x - mean)|^2 with U staged in LDS and the row
//               in registers, weight update, chunk max key and estimate sums
//               against the chunk's max.  One launch per bucket.  From
//               DB = 24 up, k_bquad_mx: the same results with the product
//               U (x - mean) on the FP64 matrix cores.
//   k_bscan     per tile of 4096 particles of every sampler: the sampler's max
//               from its chunk keys, 64-bit fixed-point weights, FP64 sums,
//               the exact sum of squares, and the inclusive prefix by a
//               decoupled lookback that stays inside the sampler's own tiles
//               (segmented scan); the tile's chunk estimate sums rescaled to
//               the sampler's max.
//   k_bdecide   one workgroup per sampler: tile partials in a fixed order,
//               integer decision, offset, log Z, ESS, estimates, c_t,
//               recycling, the sampler's info record.
//   k_bexpand   per 256 outputs of resampling samplers: ancestor by binary
//               search on the prefix, rows copied by whole wavefronts.
//   k_bflip     per sampler that resampled: the redistributed copy becomes
//               the current one (particles alternate between the caller's
//               array and the workspace copy; no copy back).
//
// Tiles never straddle samplers, a tile waits only on earlier tiles of its own
// sampler, and every reduction runs in a fixed order over that sampler's
// tiles, so a sampler's results do not depend on the rest of the batch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "../../include/smc.h"
#include "../../include/smc_batch.h"
#include "common.hpp"
#include "det.hpp"
#include "kernels.hpp"
#include "rng_wave.hpp"

namespace smc {
namespace {

constexpr int kBT = 256;               // threads per workgroup
constexpr int kBItems = 16;            // particles per thread and tile
constexpr int kBTile = kBT * kBItems;  // particles per tile
// LDS position of tile entry i: entries stay in their run of 16, rotated by
// bits 5..8 of i, so that both the striped and the per-thread accesses of a
// wave spread over the banks
__host__ __device__ constexpr int kBPad(int i) { return (i & ~15) | ((i ^ (i >> 5)) & 15); }
typedef double f64x2b_t __attribute__((ext_vector_type(2)));
constexpr int kBChunk = 256;           // particles of an update / expand / copy workgroup
constexpr int kChunksPerTile = kBTile / kBChunk;
constexpr int kMaxGroup = 8;           // coordinate pairs of a proposal unit (16 columns of LDS)
constexpr int kBSpin = 1 << 22;        // lookback poll bound
constexpr int kBuckets = 8;            // dimension buckets (8b, 8b + 8]
constexpr int kBMaxCap = 4096;
constexpr int kBStage = 2048;          // prefix values of one expand chunk staged in LDS
constexpr int64_t kBMaxN = 1ll << 28;

// The per-sampler arrays are reached through pointers read from the slot
// table, which the compiler would address as generic (flat) memory; flat
// accesses also count against the LDS wait counter, so every wave shuffle
// would drain them.  These casts keep them on the global path.
#define GLB(T) __attribute__((address_space(1))) T
template <class T>
__device__ inline GLB(T) *glb(T *p)
{
    return (GLB(T) *)p;
}
// Read-only data that is the same for the whole wave (the target's U and
// mean) is read through the constant address space: scalar loads into SGPRs,
// no LDS or vector-memory traffic per lane.
#define CST(T) __attribute__((address_space(4))) T

// Per-sampler control block (in the sampler's workspace).
struct BCtrl {
    u64 S, U, Q2lo, Q2hi, mkey;
    double m, logZ, ess, Z, Z2, log_c;
    double logZ_prev, lc_max, rec_den;
    unsigned t;          // iteration of the next step (1, 2, ...)
    unsigned resample;   // decision of the last step
    unsigned err_call, err_latch, spin_fail, bad, rec_steps;
    unsigned cur;        // 0: particles and log-targets in (x, lp); 1: in (x_scr, lp_scr)
};

// Per-chunk max key and non-finite flag of the update kernel.
struct BTileIS {
    u64 key;
    unsigned bad, pad;
};

// Device descriptor of one slot (n == 0: free).
struct BSlot {
    i64 n;
    int d, mode, ess_num, ess_den, K, ntile, nchunk, bucket;
    uint32_t sampler, pad;
    u64 seed;
    double rw_sd, init_mean, init_sd, init_prec, init_log_norm, log_norm, reset;
    const double *mean, *chol;
    double *x, *logw;
    BCtrl *ctrl;
    double *lp, *x_scr, *lp_scr, *epart, *cpart, *rec_num;
    double *upad;  // [DB][DB] U zero-padded to the bucket width, then [DB] mean
    u64 *pref, *status;
    TilePart *tpart;
    BTileIS *tis;
};

struct BTabs {
    int *n_act;       // [1 + kBuckets]: attached samplers, then per bucket
    int *act;         // [cap] attached slots, ascending
    int *tile_pref;   // [cap + 1] tile prefix over act
    int *chunk_pref;  // [cap + 1] expand-chunk prefix over act
    int *unit_pref;   // [cap + 1] proposal-unit prefix over act (chunk x pair group)
    int *bact;        // [kBuckets][cap]
    int *btile_pref;  // [kBuckets][cap + 1] chunk prefix over bact
};

// Sum of each 16-lane row of the wave, left in the row's last lane (lanes
// 15, 31, 47, 63), by DPP row shifts: VALU only, no LDS round trips.  Lanes
// whose shifted source lies outside the row add 0.
template <int CTRL>
__device__ inline double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Offset of row r in a packed upper triangle of a DB x DB matrix.
template <int DB>
__device__ constexpr int tri_off(int r) { return r * DB - r * (r - 1) / 2; }

__device__ inline double row16_sum(double v)
{
    v += dpp_f64<0x111>(v);  // row_shr:1
    v += dpp_f64<0x112>(v);  // row_shr:2
    v += dpp_f64<0x114>(v);  // row_shr:4
    v += dpp_f64<0x118>(v);  // row_shr:8
    return v;
}

// Position of block b in a prefix table: slot and index within the slot.
// Rows [0, cnt) x columns [0, w) of a row-major block (row stride d, w <= 16)
// into LDS as whole lines: 16 lanes a row, 16 rows per pass.  Every load of a
// thread is issued before the first wait (its address is clamped into the
// block, so the loads need no branch); a loop that waits for each load in
// turn spends most of a wave's life on memory latency.
template <int CW>
__device__ inline void stage_rows(double (*sx)[CW], const GLB(double) *xb, int d, int cnt, int w)
{
    const int tid = threadIdx.x, lc = tid & 15, lr = tid >> 4;
    const int cc = lc < w ? lc : w - 1;
    double v[kBChunk / 16];
#pragma unroll
    for (int j = 0; j < kBChunk / 16; ++j) {
        const int r = lr + 16 * j;
        v[j] = xb[(i64)(r < cnt ? r : cnt - 1) * d + cc];
    }
#pragma unroll
    for (int j = 0; j < kBChunk / 16; ++j) {
        const int r = lr + 16 * j;
        if (r < cnt && lc < w) sx[r][lc] = v[j];
    }
}

__device__ inline bool locate(const int *pref, const int *act, int nact, int b, int &slot,
                              int &local)
{
    if (nact <= 0 || b >= pref[nact]) return false;
    int lo = 0, hi = nact;  // pref[lo] <= b < pref[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pref[mid] <= b) lo = mid;
        else hi = mid;
    }
    slot = act[lo];
    local = b - pref[lo];
    return true;
}

// ------------------------------------------------------------------ tables
__global__ void k_bslot_set(BSlot v, BSlot *dst) { *dst = v; }

// U zero-padded to DB x DB (lower triangle and beyond d are zero) and the
// mean zero-padded to DB, so the quadratic form needs no per-element guard:
// the extra terms are fma(0, 0, s) = s.
__global__ __launch_bounds__(256) void k_bpad(const BSlot *slots, int slot)
{
    const BSlot S = slots[slot];
    const int d = S.d, DB = 8 * (S.bucket + 1);
    for (int e = blockIdx.x * 256 + threadIdx.x; e < DB * DB + DB; e += gridDim.x * 256) {
        double v = 0.0;
        if (e < DB * DB) {
            const int r = e / DB, k = e - r * DB;
            if (r < d && k < d && k >= r) v = S.chol[r * d + k];
        } else if (e - DB * DB < d) {
            v = S.mean[e - DB * DB];
        }
        S.upad[e] = v;
    }
}

__global__ void k_bslots_clear(BSlot *slots, int cap)
{
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < cap; s += gridDim.x * blockDim.x)
        slots[s].n = 0;
}

// Tables of the attached slots in slot order; thread t owns a contiguous
// range of slots, counts are combined by a block scan.
__device__ __host__ inline int units_of(int nchunk, int d, int G)
{
    return nchunk * (((d + 1) / 2 + G - 1) / G);
}

__global__ __launch_bounds__(256) void k_btables(const BSlot *slots, int cap, int G, BTabs tb)
{
    constexpr int NV = 4 + 2 * kBuckets;  // act, tiles, chunks, bucket counts, bucket chunks, units
    __shared__ int s_v[NV][256];
    const int tid = threadIdx.x;
    const int per = (cap + 255) / 256;
    const int s0 = tid * per, s1 = (s0 + per < cap) ? s0 + per : cap;
    int v[NV];
    for (int q = 0; q < NV; ++q) v[q] = 0;
    for (int s = s0; s < s1; ++s) {
        if (slots[s].n <= 0) continue;
        const int b = slots[s].bucket;
        v[0] += 1;
        v[1] += slots[s].ntile;
        v[2] += slots[s].nchunk;
        v[3 + b] += 1;
        v[3 + kBuckets + b] += slots[s].nchunk;
        v[3 + 2 * kBuckets] += units_of(slots[s].nchunk, slots[s].d, G);
    }
    for (int q = 0; q < NV; ++q) s_v[q][tid] = v[q];
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {  // inclusive Hillis-Steele scan
        int add[NV];
        for (int q = 0; q < NV; ++q) add[q] = tid >= o ? s_v[q][tid - o] : 0;
        __syncthreads();
        for (int q = 0; q < NV; ++q) s_v[q][tid] += add[q];
        __syncthreads();
    }
    int off[NV];
    for (int q = 0; q < NV; ++q) off[q] = s_v[q][tid] - v[q];
    for (int s = s0; s < s1; ++s) {
        if (slots[s].n <= 0) continue;
        const int b = slots[s].bucket;
        tb.act[off[0]] = s;
        tb.tile_pref[off[0]] = off[1];
        tb.chunk_pref[off[0]] = off[2];
        tb.unit_pref[off[0]] = off[3 + 2 * kBuckets];
        tb.bact[b * cap + off[3 + b]] = s;
        tb.btile_pref[b * (cap + 1) + off[3 + b]] = off[3 + kBuckets + b];
        off[0] += 1;
        off[1] += slots[s].ntile;
        off[2] += slots[s].nchunk;
        off[3 + b] += 1;
        off[3 + kBuckets + b] += slots[s].nchunk;
        off[3 + 2 * kBuckets] += units_of(slots[s].nchunk, slots[s].d, G);
    }
    if (tid == 255) {
        const int na = s_v[0][255];
        tb.n_act[0] = na;
        tb.tile_pref[na] = s_v[1][255];
        tb.chunk_pref[na] = s_v[2][255];
        tb.unit_pref[na] = s_v[3 + 2 * kBuckets][255];
        for (int b = 0; b < kBuckets; ++b) {
            const int nb = s_v[3 + b][255];
            tb.n_act[1 + b] = nb;
            tb.btile_pref[b * (cap + 1) + nb] = s_v[3 + kBuckets + b][255];
        }
    }
}

// ---------------------------------------------------------------- proposal
// One workgroup per chunk of 256 particles (one per thread), every sampler in
// one launch (single >= 0: the chunks of that slot only).  Draws the proposal
// (or x0 ~ q0) in place; at initialisation also leaves the quadratic term of
// log q0 in lp_scr.  Kept apart from the target so that its register use, and
// with it the occupancy of the normal generation, does not depend on d.
// CW: row stride of the step's LDS staging block, at least 2 G + 1 doubles.
template <bool kInit, int CW = 17>
__global__ __launch_bounds__(256) void k_bprop(const BSlot *slots, const int *n_act,
                                               const int *act_list, const int *unit_pref, int G,
                                               int single)
{
    const int tid = threadIdx.x;
    int slot, unit;
    if (single >= 0) {
        slot = single;
        unit = blockIdx.x;
    } else if (!locate(unit_pref, act_list, n_act[0], blockIdx.x, slot, unit)) {
        return;
    }
    // a local copy: stores through the sampler's arrays cannot alias it
    const BSlot S = slots[__builtin_amdgcn_readfirstlane(slot)];
    const i64 n = S.n;
    const int d = S.d;
    // a unit is one chunk of 256 particles and a group of G coordinate pairs
    // (all pairs at initialisation, where log q0 sums over the whole row)
    __shared__ uint4 s_xch[4][64];  // normal generator exchange, one row per wave
    const int npair = (d + 1) / 2;
    const int ng = kInit ? 1 : (npair + G - 1) / G;
    const int chunk = unit / ng, grp = unit - chunk * ng;
    const int kp0 = kInit ? 0 : grp * G;
    const int kp1 = kInit ? npair : (kp0 + G < npair ? kp0 + G : npair);
    if (tid == 0 && grp == 0 && (chunk % kChunksPerTile) == 0) S.status[chunk / kChunksPerTile] = 0;
    const uint32_t t = kInit ? 0u : S.ctrl->t;
    const uint32_t tag = kInit ? (uint32_t)kTagInit : (uint32_t)kTagPropose;
    if (d == 1) {
        // One coordinate a particle: particles 2p and 2p + 1 take the two
        // values of the pair drawn for index p; the chunk's (at most 128)
        // pairs go to its first two wavefronts, one pair a lane.
        if (tid >= kBChunk / 2) return;  // whole wavefronts
        const i64 p = (i64)chunk * (kBChunk / 2) + tid;
        const i64 i0 = 2 * p;
        const bool pact = i0 < n;
        double z[2];
        normal_pair_wave(S.seed, tag, S.sampler, t, (uint32_t)p, 0u, pact, z[0], z[1],
                         s_xch[tid >> 6]);
        if (!pact) return;
        GLB(double) *xr = glb(kInit ? S.x : (S.ctrl->cur ? S.x_scr : S.x));
        for (int h = 0; h < 2; ++h) {
            const i64 i = i0 + h;
            if (i >= n) break;
            const double zh = h == 0 ? z[0] : z[1];
            if (kInit) {
                const double xk = S.init_mean + S.init_sd * zh;
                xr[i] = xk;
                const double t0 = xk - S.init_mean;
                glb(S.lp_scr)[i] = 0.0 + (t0 * t0) * S.init_prec;
            } else {
                xr[i] = xr[i] + S.rw_sd * zh;
            }
        }
        return;
    }
    const i64 i = (i64)chunk * kBChunk + tid;
    const bool act = i < n;
    GLB(double) *xi = glb(S.x) + i * d;
    double acc0 = 0.0;
    if (!kInit) {
        // Step: the unit's block of rows [base, base + cnt) x columns
        // [k0, k0 + w), w <= 16, moves between HBM and LDS as whole 128-byte
        // lines (16 lanes per row); each thread then updates its own row in
        // LDS.  Strided per-thread row accesses would touch 64 lines per
        // wave instruction.
        __shared__ double sx[kBChunk][CW];
        const int k0 = 2 * kp0, w = (2 * kp1 < d ? 2 * kp1 : d) - k0;
        const i64 base = (i64)chunk * kBChunk;
        const int cnt = (int)((n - base) < kBChunk ? (n - base) : kBChunk);
        const int lc = tid & 15, lr = tid >> 4;
        GLB(double) *xb = glb(S.ctrl->cur ? S.x_scr : S.x) + base * d + k0;
        stage_rows(sx, xb, d, cnt, w);
        __syncthreads();
        for (int k2 = kp0; k2 < kp1; ++k2) {
            double z[2];
            normal_pair_wave(S.seed, tag, S.sampler, t, (uint32_t)i, (uint32_t)k2, act, z[0],
                             z[1], s_xch[tid >> 6]);
            const int c = 2 * k2 - k0;
            if (act) {
                sx[tid][c] = sx[tid][c] + S.rw_sd * z[0];
                if (c + 1 < w) sx[tid][c + 1] = sx[tid][c + 1] + S.rw_sd * z[1];
            }
        }
        __syncthreads();
        for (int r = lr; r < cnt; r += 16)
            if (lc < w) xb[(i64)r * d + lc] = sx[r][lc];
        return;
    }
    // Initialisation (whole rows, all pairs; log q0 sums over the row)
    for (int k2 = kp0; k2 < kp1; ++k2) {
        const int k0 = 2 * k2;
        double z[2];
        normal_pair_wave(S.seed, tag, S.sampler, t, (uint32_t)i, (uint32_t)k2, act, z[0], z[1],
                         s_xch[tid >> 6]);
        if (act) {
            for (int h = 0; h < 2; ++h) {
                const int kk = k0 + h;
                if (kk >= d) break;
                const double xk = S.init_mean + S.init_sd * z[h];
                xi[kk] = xk;
                const double t0 = xk - S.init_mean;
                acc0 = acc0 + (t0 * t0) * S.init_prec;
            }
        }
    }
    if (kInit && act) glb(S.lp_scr)[i] = acc0;
}

// ------------------------------------------------------ target + weights
// One workgroup per chunk of samplers whose dimension falls in the bucket
// (DB - 8, DB] (single >= 0: the chunks of that slot): |U (x - mean)|^2 with U
// staged in LDS and the row in registers, the weight update, the chunk's max
// key, non-finite flag and estimate sums against the chunk's own max m_b:
// [m_b, sum e, sum e x_k, sum e x_k^2], e = exp(l - m_b).
// W: the occupancy the register allocation aims at (waves per SIMD), a
// per-bucket speed knob (smc_batch_set_bucket_waves); results do not depend
// on it.
template <int DB, bool kInit, int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) void k_bquad(
    const BSlot *slots, const int *n_act, const int *bact, const int *bchunk_pref, int bucket,
    int cap, int single)
{
    __shared__ u64 s_key[4];
    __shared__ unsigned s_bad[4];
    __shared__ double s_col[16][1 + 2 * DB];  // one partial per 16-lane row
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int slot, chunk;
    if (single >= 0) {
        slot = single;
        chunk = blockIdx.x;
    } else if (!locate(bchunk_pref + bucket * (cap + 1), bact + bucket * cap, n_act[1 + bucket],
                       blockIdx.x, slot, chunk)) {
        return;
    }
    // a local copy: stores through the sampler's arrays cannot alias it
    const BSlot S = slots[__builtin_amdgcn_readfirstlane(slot)];
    const i64 n = S.n;
    const int d = S.d;
    const CST(double) *sM = (const CST(double) *)S.upad + DB * DB;
    const i64 i = (i64)chunk * kBChunk + tid;
    const bool act = i < n;
    const bool alt = !kInit && S.ctrl->cur;
    GLB(double) *lpg = glb(alt ? S.lp_scr : S.lp);
    GLB(double) *lwg = glb(S.logw);
    double lw = -__builtin_huge_val();
    // The chunk's rows come in through LDS in slices of 16 columns, each
    // moved as whole 128-byte lines (16 lanes per row).
    __shared__ double sx[kBChunk][17];
    constexpr int PW = DB < 16 ? DB : 16;
    const i64 base = (i64)chunk * kBChunk;
    const int cnt = (int)((n - base) < kBChunk ? (n - base) : kBChunk);
    const GLB(double) *xb = glb(alt ? S.x_scr : S.x) + base * d;
    constexpr int NQ = (DB + PW - 1) / PW;
    double tv[DB];
    // U's upper triangle, packed by rows (row r holds k = r .. DB - 1 from
    // offset tri_off(r)), in LDS: every lane reads the same element, so the
    // reads are broadcasts, and many can be in flight (unlike scalar loads).
    __shared__ double sT[DB * (DB + 1) / 2];
    {
        constexpr int kPer = (DB * DB + 255) / 256;
        const GLB(double) *ug = glb(S.upad);
        double uv[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int e = tid + 256 * j;
            uv[j] = e < DB * DB ? ug[e] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int e = tid + 256 * j;
            const int r = e / DB, k = e - r * DB;
            if (e < DB * DB && k >= r) sT[tri_off<DB>(r) + k - r] = uv[j];
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (q * PW < d) {
            stage_rows(sx, xb + q * PW, d, cnt, d - q * PW < PW ? d - q * PW : PW);
            __syncthreads();
#pragma unroll
            for (int c = 0; c < PW; ++c) {
                const int k = q * PW + c;
                if (k < DB) tv[k] = (act && k < d) ? sx[tid][c] - sM[k] : 0.0;
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int c = 0; c < PW; ++c)
                if (q * PW + c < DB) tv[q * PW + c] = 0.0;
        }
    }
    if (act) {
        // rows r and r + 1 advance together (two independent FMA chains);
        // each row still sums k = r, r + 1, ... in order
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < DB; r += 2) {
            const double *u0 = sT + tri_off<DB>(r) - r, *u1 = sT + tri_off<DB>(r + 1) - (r + 1);
            double s0 = fma(u0[r], tv[r], 0.0), s1 = 0.0;
#pragma unroll
            for (int k = r + 1; k < DB; ++k) {
                s0 = fma(u0[k], tv[k], s0);
                s1 = fma(u1[k], tv[k], s1);
            }
            acc = fma(s0, s0, acc);
            acc = fma(s1, s1, acc);
        }
        const double lpn = S.log_norm - 0.5 * acc;
        lw = kInit ? lpn - (S.init_log_norm - 0.5 * glb(S.lp_scr)[i]) : lwg[i] + (lpn - lpg[i]);
        lpg[i] = lpn;
        lwg[i] = lw;
    }
    const unsigned bad = wave_or((lw != lw) | (lw == __builtin_huge_val()));
    const u64 key = wave_max_u64(act ? okey(lw) : 0ull);
    if (lane == 0) {
        s_key[wid] = key;
        s_bad[wid] = bad;
    }
    __syncthreads();
    u64 bk = s_key[0];
    unsigned bb = s_bad[0];
    for (int w = 1; w < 4; ++w) {
        bk = s_key[w] > bk ? s_key[w] : bk;
        bb |= s_bad[w];
    }
    const double mb = okey_inv(bk);
    const bool live = act && mb > -__builtin_huge_val();
    const double e = live ? det_exp(lw - mb) : 0.0;
    // column sums over the chunk: a DPP sum per 16-lane row, then the 16 row
    // partials in order.  The row is taken from the registers as
    // (x - mean) + mean, within an ulp of x: these sums feed FP64 estimates,
    // not the particle trajectories.
    const int prow = tid >> 4;
    const bool last = (lane & 15) == 15;
    {
        const double se = row16_sum(e);
        if (last) s_col[prow][0] = se;
    }
#pragma unroll
    for (int k = 0; k < DB; ++k) {
        if (k < d) {
            const double xk = act ? tv[k] + sM[k] : 0.0;
            const double ex = e * xk;
            const double s1 = row16_sum(ex), s2 = row16_sum(ex * xk);
            if (last) {
                s_col[prow][1 + k] = s1;
                s_col[prow][1 + d + k] = s2;
            }
        }
    }
    __syncthreads();
    double *cp = S.cpart + (i64)chunk * (2 + 2 * d);
    for (int c = tid; c < 1 + 2 * d; c += 256) {
        double a = s_col[0][c];
        for (int r = 1; r < 16; ++r) a += s_col[r][c];
        cp[1 + c] = a;
    }
    if (tid == 0) {
        cp[0] = mb;
        BTileIS o;
        o.key = bk;
        o.bad = bb;
        o.pad = 0;
        S.tis[chunk] = o;
    }
}

// The same update with the quadratic form on the FP64 matrix cores.  Every
// wavefront takes its 64 particles in tiles of 16: Y^T = U T^T (T: the tile's
// x - mean, 16 x DB) by v_mfma_f64_16x16x4f64 over k in steps of four, one
// accumulator per block of 16 rows of U (blocks of U wholly below the
// diagonal are skipped).  The instruction adds its four products to the
// accumulator one fused multiply-add at a time, in k order (checked bit for
// bit against a sequential fma chain on MI355X, subnormal products and zero
// operands included), so row r of Y is the chain fma(U_rk, t_k, .) from +0
// over k: the terms k < r leave it +0, and it equals the row-by-row form above
// bit for bit.  The accumulators then hold Y in exactly the operand layout of
// the same instruction (lane (g, p16), element v of block R: Y of particle
// p16, row 16 R + 4 v + g), so Y Y^T over the row blocks and elements in
// order is, on its diagonal, the chain fma(y_r, y_r, .) from +0 over r in row
// order: the sum of squares of the row-by-row form, bit for bit (rows past d
// are +0 and add nothing).  No LDS holds Y, which leaves the LDS footprint
// small enough that registers alone set the occupancy.  A particle with a
// non-finite difference (possible only with non-finite parameters, where a
// zero of U times inf gives NaN instead of the row-by-row result) takes the
// row-by-row loop instead.
// U's operands and the mean wait in LDS.  The estimate sums re-read the
// chunk's rows (from cache) once the chunk's max is known, per lane over its
// four particles, then across the 16 lanes of each row, then over the
// wavefronts in order: the same sums as above within rounding.
template <int DB>
__host__ __device__ constexpr int mx_pair(int R, int c)
{
    int p = 0;
    for (int q = 0; q < R; ++q) p += DB / 4 - 4 * q;
    return p + c - 4 * R;
}

typedef double f64x4_t __attribute__((ext_vector_type(4)));

template <int DB, bool kInit, int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) void k_bquad_mx(
    const BSlot *slots, const int *n_act, const int *bact, const int *bchunk_pref, int bucket,
    int cap, int single)
{
    constexpr int NC = DB / 4;           // k steps of four coordinates
    constexpr int NRB = (DB + 15) / 16;  // blocks of 16 rows of U
    constexpr int NP = mx_pair<DB>(NRB, 4 * NRB);
    static_assert(DB % 8 == 0 && NP > 0, "bucket width");
    __shared__ double sU[NP][64];         // B operands, one per lane and step
    __shared__ double sMean[DB];
    __shared__ double s_q[kBChunk];
    __shared__ double s_e[kBChunk];
    __shared__ double s_col[4][1 + 2 * DB];  // one partial per wavefront
    __shared__ u64 s_key[4];
    __shared__ unsigned s_bad[4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int slot, chunk;
    if (single >= 0) {
        slot = single;
        chunk = blockIdx.x;
    } else if (!locate(bchunk_pref + bucket * (cap + 1), bact + bucket * cap, n_act[1 + bucket],
                       blockIdx.x, slot, chunk)) {
        return;
    }
    // a local copy: stores through the sampler's arrays cannot alias it
    const BSlot S = slots[__builtin_amdgcn_readfirstlane(slot)];
    const i64 n = S.n;
    const int d = S.d;
    const CST(double) *sM = (const CST(double) *)S.upad + DB * DB;
    const GLB(double) *ug = glb(S.upad);
    const i64 base = (i64)chunk * kBChunk;
    const int cnt = (int)((n - base) < kBChunk ? (n - base) : kBChunk);
    const bool alt = !kInit && S.ctrl->cur;
    const GLB(double) *xb = glb(alt ? S.x_scr : S.x) + base * d;
    const int p16 = lane & 15, g = lane >> 4;

    // lane (g, p16) of step (R, c) multiplies U[16 R + p16][4 c + g]
#pragma unroll
    for (int R = 0; R < NRB; ++R)
#pragma unroll
        for (int c = 4 * R; c < NC; ++c)
            if (mx_pair<DB>(R, c) % 4 == wid) {
                const int r = 16 * R + p16;
                sU[mx_pair<DB>(R, c)][lane] = r < DB ? ug[r * DB + 4 * c + g] : 0.0;
            }
    for (int k = tid; k < DB; k += 256) sMean[k] = k < d ? sM[k] : 0.0;
    __syncthreads();

#pragma unroll 1
    for (int tile = 0; tile < 4; ++tile) {
        if (wid * 64 + tile * 16 >= cnt) break;  // past the chunk's last particle
        const int pl = wid * 64 + tile * 16 + p16;
        const bool pact = pl < cnt;
        const int plc = pact ? pl : 0;
        // every load of the tile is issued before the first is used (the
        // empty asm keeps the compiler from sinking each load into its use)
        double xv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) xv[c] = xb[(i64)plc * d + (4 * c + g < d ? 4 * c + g : d - 1)];
        asm volatile("" ::: "memory");
        f64x4_t acc[NRB];
#pragma unroll
        for (int R = 0; R < NRB; ++R) acc[R] = f64x4_t{0.0, 0.0, 0.0, 0.0};
        bool nf = false;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int k = 4 * c + g;
            const double t = (pact && k < d) ? xv[c] - sMean[k] : 0.0;
            nf |= !__builtin_isfinite(t);
#pragma unroll
            for (int R = 0; R < NRB; ++R)
                if (4 * R <= c)
                    acc[R] = __builtin_amdgcn_mfma_f64_16x16x4f64(sU[mx_pair<DB>(R, c)][lane], t,
                                                                  acc[R], 0, 0, 0);
        }
        const u64 nfm = __ballot(nf);
        // element v of lane (g, p16) in block R is Y[p16][16 R + 4 v + g]
        f64x4_t q2 = f64x4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int R = 0; R < NRB; ++R)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                q2 = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[R][v], acc[R][v], q2, 0, 0, 0);
        if ((p16 & 3) == g) {
            const int pt = wid * 64 + tile * 16 + p16;
            const int vq = p16 >> 2;
            double q = vq == 0 ? q2[0] : (vq == 1 ? q2[1] : (vq == 2 ? q2[2] : q2[3]));
            if (((nfm >> p16) & 0x0001000100010001ull) && pt < cnt) {
                q = 0.0;
                const GLB(double) *xr = xb + (i64)pt * d;
                for (int r = 0; r < d; ++r) {
                    double sr = 0.0;
                    for (int k = r; k < d; ++k) sr = fma(ug[r * DB + k], xr[k] - sMean[k], sr);
                    q = fma(sr, sr, q);
                }
            }
            if (pt < cnt) s_q[pt] = q;
        }
    }
    __syncthreads();

    const i64 i = base + tid;
    const bool act = tid < cnt;
    GLB(double) *lpg = glb(alt ? S.lp_scr : S.lp);
    GLB(double) *lwg = glb(S.logw);
    double lw = -__builtin_huge_val();
    if (act) {
        const double lpn = S.log_norm - 0.5 * s_q[tid];
        lw = kInit ? lpn - (S.init_log_norm - 0.5 * glb(S.lp_scr)[i]) : lwg[i] + (lpn - lpg[i]);
        lpg[i] = lpn;
        lwg[i] = lw;
    }
    const unsigned bad = wave_or((lw != lw) | (lw == __builtin_huge_val()));
    const u64 key = wave_max_u64(act ? okey(lw) : 0ull);
    if (lane == 0) {
        s_key[wid] = key;
        s_bad[wid] = bad;
    }
    __syncthreads();
    u64 bk = s_key[0];
    unsigned bb = s_bad[0];
    for (int w = 1; w < 4; ++w) {
        bk = s_key[w] > bk ? s_key[w] : bk;
        bb |= s_bad[w];
    }
    const double mb = okey_inv(bk);
    const bool live = act && mb > -__builtin_huge_val();
    s_e[tid] = live ? det_exp(lw - mb) : 0.0;
    __syncthreads();

    // estimate sums: lane (g, p16) takes coordinates 4 c + g of particles
    // wid * 64 + 16 tile + p16, then the 16 lanes of each row are added up
    double s1[NC], s2[NC], s0 = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) s1[c] = s2[c] = 0.0;
#pragma unroll 1
    for (int tile = 0; tile < 4; ++tile) {
        if (wid * 64 + tile * 16 >= cnt) break;
        const int pl = wid * 64 + tile * 16 + p16;
        const bool pact = pl < cnt;
        const int plc = pact ? pl : 0;
        const double e = s_e[pl];
        s0 += e;
        double xv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) xv[c] = xb[(i64)plc * d + (4 * c + g < d ? 4 * c + g : d - 1)];
        asm volatile("" ::: "memory");
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int k = 4 * c + g;
            const double xk = (pact && k < d) ? xv[c] : 0.0;
            const double ex = e * xk;
            s1[c] += ex;
            s2[c] += ex * xk;
        }
    }
    s0 = row16_sum(s0);
    if (lane == 15) s_col[wid][0] = s0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double v1 = row16_sum(s1[c]), v2 = row16_sum(s2[c]);
        const int k = 4 * c + g;
        if (p16 == 15 && k < d) {
            s_col[wid][1 + k] = v1;
            s_col[wid][1 + d + k] = v2;
        }
    }
    __syncthreads();
    double *cp = S.cpart + (i64)chunk * (2 + 2 * d);
    for (int c = tid; c < 1 + 2 * d; c += 256) {
        double a = s_col[0][c];
        for (int w = 1; w < 4; ++w) a += s_col[w][c];
        cp[1 + c] = a;
    }
    if (tid == 0) {
        cp[0] = mb;
        BTileIS o;
        o.key = bk;
        o.bad = bb;
        o.pad = 0;
        S.tis[chunk] = o;
    }
}

// Initialisation statistics: log sum w_0 from the chunk partials (fixed
// order), error of the initial weights, cleared recycling sums.
__global__ __launch_bounds__(64) void k_binit(const BSlot *slots, int slot)
{
    // a local copy: stores through the sampler's arrays cannot alias it
    const BSlot S = slots[__builtin_amdgcn_readfirstlane(slot)];
    BCtrl *c = S.ctrl;
    const int lane = threadIdx.x;
    const int cw = 2 + 2 * S.d;
    for (int k = lane; k < 2 * S.d; k += 64) S.rec_num[k] = 0.0;
    if (lane != 0) return;
    u64 key = 0;
    unsigned bad = 0;
    double m = -__builtin_huge_val();
    for (int k = 0; k < S.nchunk; ++k) {
        key = S.tis[k].key > key ? S.tis[k].key : key;
        bad |= S.tis[k].bad;
        m = fmax(m, S.cpart[(i64)k * cw]);
    }
    double E = 0.0;
    for (int k = 0; k < S.nchunk; ++k) {
        const double mk = S.cpart[(i64)k * cw];
        if (mk > -__builtin_huge_val()) E += S.cpart[(i64)k * cw + 1] * det_exp(mk - m);
    }
    unsigned err = 0;
    if (bad) err = kErrNonfinite;
    else if (key <= okey(-__builtin_huge_val())) err = kErrDegenerate;
    c->logZ_prev = m + log(E);
    c->lc_max = -__builtin_huge_val();
    c->rec_den = 0.0;
    c->rec_steps = 0;
    c->t = 1;
    c->cur = 0;
    c->resample = 0;
    c->err_call = err;
    c->err_latch = err;
    c->spin_fail = 0;
    c->bad = 0;
}

// --------------------------------------------------------- segmented scan
// One workgroup per tile of 4096 particles (16 consecutive per thread).
__global__ __launch_bounds__(256) void k_bscan(const BSlot *slots, const int *n_act,
                                               const int *act, const int *tile_pref)
{
    __shared__ u64 s_k[4], s_wsum[4], s_lo[4], s_hi[4];
    __shared__ unsigned s_b[4];
    __shared__ double s_z[4], s_z2[4];
    __shared__ u64 s_prefix;
    __shared__ u64 s_t[kBTile];  // the tile's log-weights in, its prefix out
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int slot, tile;
    if (!locate(tile_pref, act, n_act[0], blockIdx.x, slot, tile)) return;
    // a local copy: stores through the sampler's arrays cannot alias it
    const BSlot S = slots[__builtin_amdgcn_readfirstlane(slot)];
    const i64 n = S.n;
    const int d = S.d, K = S.K, ntile = S.ntile, nchunk = S.nchunk;

    // the sampler's max and non-finite flag from its chunk keys
    u64 key = 0;
    unsigned bad = 0;
    for (int k = tid; k < nchunk; k += 256) {
        const u64 kk = S.tis[k].key;
        key = kk > key ? kk : key;
        bad |= S.tis[k].bad;
    }
    key = wave_max_u64(key);
    bad = wave_or(bad);
    if (lane == 0) {
        s_k[wid] = key;
        s_b[wid] = bad;
    }
    __syncthreads();
    key = s_k[0];
    bad = s_b[0];
    for (int w = 1; w < 4; ++w) {
        key = s_k[w] > key ? s_k[w] : key;
        bad |= s_b[w];
    }
    const double m = okey_inv(key);
    if (tile == 0 && tid == 0) {
        S.ctrl->mkey = key;
        S.ctrl->bad = bad;
    }

    // estimate sums of the tile's chunks, rescaled to the sampler's max
    const int cw = 2 + 2 * d;
    const int c0 = tile * kChunksPerTile;
    const int c1 = (c0 + kChunksPerTile < nchunk) ? c0 + kChunksPerTile : nchunk;
    if (tid < 2 * d) {
        double a = 0.0;
        for (int c = c0; c < c1; ++c) {
            const double mc = S.cpart[(i64)c * cw];
            if (mc > -__builtin_huge_val()) a += det_exp(mc - m) * S.cpart[(i64)c * cw + 2 + tid];
        }
        S.epart[(i64)tile * 2 * d + tid] = a;
    }

    // fixed-point weights of 16 consecutive particles, FP64 and exact sums
    const i64 base = (i64)tile * kBTile;
    const u64 top = 1ull << K;
    double z = 0.0, z2 = 0.0;
    U128 q2{0, 0};
    u64 loc[kBItems];
    u64 run = 0;
    // the tile's log-weights arrive by striped, coalesced loads and pass
    // through LDS, so that every thread still takes 16 consecutive particles
    // in order (the same sums as a direct per-thread read, which touched 64
    // cache lines per wave instruction)
    {
        const GLB(double) *lwt = glb(S.logw) + base;
        if (base + kBTile <= n && ((uintptr_t)lwt & 15) == 0) {
#pragma unroll
            for (int r = 0; r < kBItems / 2; ++r) {
                const int s0 = r * 2 * kBT + 2 * tid;
                const GLB(f64x2b_t) *p2 = reinterpret_cast<const GLB(f64x2b_t) *>(lwt + s0);
                const f64x2b_t t2 = *p2;
                s_t[kBPad(s0)] = (u64)__double_as_longlong(t2.x);
                s_t[kBPad(s0 + 1)] = (u64)__double_as_longlong(t2.y);
            }
        } else {
#pragma unroll
            for (int e = 0; e < kBItems; ++e) {
                const int s0 = (e >> 1) * 2 * kBT + 2 * tid + (e & 1);
                const double v = base + s0 < n ? lwt[s0] : -__builtin_huge_val();
                s_t[kBPad(s0)] = (u64)__double_as_longlong(v);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBItems; ++j) {
        const double v = __longlong_as_double((long long)s_t[kBPad(tid * kBItems + j)]);
        const double e = det_exp(v - m);
        u64 q = 0;
        if (e >= 0.0) {
            z += e;
            z2 += e * e;
            q = (u64)floor(ldexp(e, K));
            q = q > top ? top : q;
            q2 = add128(q2, mul64(q, q));
        }
        run += q;
        loc[j] = run;
    }
    const u64 incl = wave_incl_scan_u64(run);
    if (lane == 63) s_wsum[wid] = incl;
    __syncthreads();
    u64 wpre = 0, agg = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        wpre += (w < wid) ? s_wsum[w] : 0;
        agg += s_wsum[w];
    }
    const u64 texcl = wpre + incl - run;

    // decoupled lookback over this sampler's earlier tiles
    if (wid == 0) {
        u64 excl = 0;
        if (tile == 0) {
            if (lane == 0) st_relaxed(&S.status[0], kFlagInc | agg);
        } else {
            if (lane == 0) st_relaxed(&S.status[tile], kFlagAgg | agg);
            i64 top_idx = (i64)tile - 1;
            int spins = 0;
            while (true) {
                const i64 idx = top_idx - lane;
                const u64 sv = idx >= 0 ? ld_relaxed(&S.status[idx]) : kFlagInc;
                const u64 flag = sv >> 62;
                const u64 inc_mask = __ballot(flag == 2);
                const u64 zero_mask = __ballot(flag == 0);
                const int first_inc = inc_mask ? __ffsll((long long)inc_mask) - 1 : 64;
                const u64 need = first_inc >= 64 ? ~0ull : ((1ull << first_inc) - 1);
                if (zero_mask & need) {
                    if (++spins > kBSpin) {
                        if (lane == 0) S.ctrl->spin_fail = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                u64 acc = lane <= first_inc ? (sv & kValMask) : 0;
                for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
                excl += acc;
                if (first_inc < 64) break;
                top_idx -= 64;
            }
            if (lane == 0) st_relaxed(&S.status[tile], kFlagInc | (excl + agg));
        }
        if (lane == 0) s_prefix = excl;
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
    const u64 pre = s_prefix + texcl;
    // each thread rewrites the 16 entries it read; the prefix then leaves by
    // striped, coalesced stores
#pragma unroll
    for (int j = 0; j < kBItems; ++j) s_t[kBPad(tid * kBItems + j)] = pre + loc[j];
    __syncthreads();
    {
        GLB(u64) *pt = glb(S.pref) + base;
#pragma unroll
        for (int e = 0; e < kBItems; ++e) {
            const int s0 = (e >> 1) * 2 * kBT + 2 * tid + (e & 1);
            if (base + s0 < n) pt[s0] = s_t[kBPad(s0)];
        }
    }
    if (tid == 0) {
        TilePart p;
        p.Z = ((s_z[0] + s_z[1]) + s_z[2]) + s_z[3];
        p.Z2 = ((s_z2[0] + s_z2[1]) + s_z2[2]) + s_z2[3];
        U128 t{s_lo[0], s_hi[0]};
        for (int w = 1; w < 4; ++w) t = add128(t, U128{s_lo[w], s_hi[w]});
        p.q2lo = t.lo;
        p.q2hi = t.hi;
        S.tpart[tile] = p;
    }
    (void)ntile;
}

// ------------------------------------------------------- per-sampler decide
__global__ __launch_bounds__(256) void k_bdecide(const BSlot *slots, const int *n_act,
                                                 const int *act, smc_resample_info *info,
                                                 double *est)
{
    __shared__ double s_z[4], s_z2[4];
    __shared__ u64 s_lo[4], s_hi[4];
    __shared__ double s_col[2 * SMC_BATCH_DMAX];
    __shared__ double s_sc, s_wgt, s_den, s_Z;
    __shared__ unsigned s_err;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if ((int)blockIdx.x >= n_act[0]) return;
    const int slot = act[blockIdx.x];
    // a local copy: stores through the sampler's arrays cannot alias it
    const BSlot S = slots[__builtin_amdgcn_readfirstlane(slot)];
    BCtrl *c = S.ctrl;
    const int d = S.d, ntile = S.ntile;
    const i64 n = S.n;
    double z = 0.0, z2 = 0.0;
    U128 q2{0, 0};
    for (int k = tid; k < ntile; k += 256) {
        const TilePart p = S.tpart[k];
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
    if (tid < 2 * d) {  // estimate columns, tiles in order
        double a = 0.0;
        for (int k = 0; k < ntile; ++k) a += S.epart[(i64)k * 2 * d + tid];
        s_col[tid] = a;
    }
    __syncthreads();
    if (tid == 0) {
        const double Z = ((s_z[0] + s_z[1]) + s_z[2]) + s_z[3];
        const double Z2 = ((s_z2[0] + s_z2[1]) + s_z2[2]) + s_z2[3];
        U128 Q2{s_lo[0], s_hi[0]};
        for (int w = 1; w < 4; ++w) Q2 = add128(Q2, U128{s_lo[w], s_hi[w]});
        const u64 Ssum = S.status[ntile - 1] & kValMask;
        const u64 key = c->mkey;
        const double m = okey_inv(key);
        unsigned err = 0;
        if (c->bad) err = kErrNonfinite;
        else if (key <= okey(-__builtin_huge_val())) err = kErrDegenerate;
        else if (c->spin_fail) err = SMC_E_DEVICE;
        c->spin_fail = 0;
        int resample;
        if (S.mode == SMC_MODE_FORCE) {
            resample = 1;
        } else if (S.mode == SMC_MODE_NEVER) {
            resample = 0;
        } else {
            const U128 lhs = mul128_small(mul64(Ssum, Ssum), (u64)S.ess_den);
            const U128 rhs = mul128_small(mul128_small(Q2, (u64)n), (u64)S.ess_num);
            resample = lt128(lhs, rhs) ? 1 : 0;
        }
        if (err) resample = 0;
        const unsigned t = c->t;
        const u64 r = resample_word(S.seed, S.sampler, t);
        const u64 U = mul64(r, Ssum).hi;
        const double logZ = m + log(Z);
        const double ess = (Z * Z) / Z2;
        // normalising constant (eq. normconst) and recycling (eq. recycling);
        // an iteration that found an error leaves them and the estimates
        double logc = 0.0, sc = 1.0, wgt = 0.0, den = c->rec_den;
        if (!err) {
            logc = logZ - c->logZ_prev;
            if (logc > c->lc_max) {
                sc = c->rec_steps ? exp(c->lc_max - logc) : 0.0;
                den *= sc;
                c->lc_max = logc;
            }
            wgt = exp(logc - c->lc_max);
            den += wgt;
            c->rec_den = den;
            c->rec_steps += 1;
            c->log_c = logc;
            c->logZ_prev = resample ? 0.0 : logZ;
        }
        c->S = Ssum;
        c->U = U;
        c->Q2lo = Q2.lo;
        c->Q2hi = Q2.hi;
        c->m = m;
        c->Z = Z;
        c->Z2 = Z2;
        c->logZ = logZ;
        c->ess = ess;
        c->resample = (unsigned)resample;
        c->err_call = err;
        if (err && !c->err_latch) c->err_latch = err;
        c->t = t + 1;
        s_sc = sc;
        s_wgt = wgt;
        s_den = den;
        s_Z = Z;
        s_err = err;
        if (info) {
            smc_resample_info *o = info + slot;
            o->m = m;
            o->logZ = logZ;
            o->ess = ess;
            o->Z = Z;
            o->Z2 = Z2;
            o->S = Ssum;
            o->U = U;
            o->Q2_hi = Q2.hi;
            o->Q2_lo = Q2.lo;
            o->K = S.K;
            o->resampled = resample;
            o->err = (int)err;
            o->pad = 0;
            o->log_c = logc;
        }
    }
    __syncthreads();
    if (tid < 2 * d && !s_err) {
        const double f = s_col[tid] / s_Z;
        const double num = S.rec_num[tid] * s_sc + s_wgt * f;
        S.rec_num[tid] = num;
        if (est) {
            est[(i64)slot * SMC_BATCH_EST_STRIDE + tid] = f;
            est[(i64)slot * SMC_BATCH_EST_STRIDE + 2 * d + tid] = num / s_den;
        }
    }
}

// ------------------------------------------------------------ redistribute
__global__ __launch_bounds__(256) void k_bexpand(const BSlot *slots, const int *n_act,
                                                 const int *act, const int *chunk_pref)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int slot, ch;
    if (!locate(chunk_pref, act, n_act[0], blockIdx.x, slot, ch)) return;
    // a local copy: stores through the sampler's arrays cannot alias it
    const BSlot S = slots[__builtin_amdgcn_readfirstlane(slot)];
    const BCtrl *c = S.ctrl;
    if (!c->resample || c->err_call) return;
    const i64 n = S.n;
    const int d = S.d;
    const u64 Ssum = c->S, U = c->U;
    // from the current copy into the other one
    const bool alt = c->cur;
    const double *xs = alt ? S.x_scr : S.x, *lps = alt ? S.lp_scr : S.lp;
    double *xd = alt ? S.x : S.x_scr, *lpd = alt ? S.lp : S.lp_scr;
    const i64 p = (i64)ch * kBChunk + tid;
    // anc(p) = first j with N S_j + U >= (p + 1) S (it exists: j = n - 1).
    // The chunk's outputs have non-decreasing ancestors in [a0, a1]: two
    // wavefronts find those ends by rounds of 64 probes, the prefix values in
    // between are staged into LDS when they fit, and every output searches
    // its ancestor there (in global memory, within [a0, a1], when they do not)
    __shared__ u64 s_pref[kBStage];
    __shared__ i64 s_a[2];
    const GLB(u64) *pg = glb(S.pref);
    if (wid < 2) {
        const i64 pe = wid == 0 ? (i64)ch * kBChunk
                                : ((i64)ch * kBChunk + kBChunk < n ? (i64)ch * kBChunk + kBChunk : n) - 1;
        const U128 rhs = mul64((u64)(pe + 1), Ssum);
        i64 lo = 0, hi = n;  // first index in [lo, hi) where the test fails
        while (hi > lo) {
            const i64 len = hi - lo;
            const i64 stride = (len + 63) / 64;
            const i64 pos = lo + (i64)lane * stride;
            const bool t = pos < hi ? lt128(add128(mul64((u64)n, pg[pos]), U), rhs) : false;
            const int cnt = __popcll(__ballot(t));
            if (cnt == 0) {
                hi = lo;
                break;
            }
            const i64 nlo = lo + (i64)(cnt - 1) * stride + 1;
            i64 nhi = lo + (i64)cnt * stride;
            if (nhi > hi) nhi = hi;
            lo = nlo;
            hi = nhi;
        }
        if (lane == 0) s_a[wid] = lo < n ? lo : n - 1;
    }
    __syncthreads();
    const i64 a0 = s_a[0], a1 = s_a[1];
    const bool staged = a1 - a0 + 1 <= kBStage;
    if (staged)
        for (i64 k = tid; k <= a1 - a0; k += 256) s_pref[k] = pg[a0 + k];
    __syncthreads();
    i64 lo = a0, hi = a1;
    if (p < n) {
        const U128 rhs = mul64((u64)(p + 1), Ssum);
        while (lo < hi) {
            const i64 mid = (lo + hi) >> 1;
            const u64 pm = staged ? s_pref[mid - a0] : pg[mid];
            if (lt128(add128(mul64((u64)n, pm), U), rhs)) lo = mid + 1;
            else hi = mid;
        }
        glb(lpd)[p] = glb(lps)[lo];
        glb(S.logw)[p] = S.reset;
    }
    // the chunk's new rows are contiguous: they are copied as one flat array
    // of cnt * d values, 256 consecutive values per step of the workgroup,
    // value e being column e mod d of output row e / d (quotient from an
    // FP32 reciprocal, corrected by one: e < 2^14); UB steps' loads are
    // issued before the first wait (indices clamped, so no branch)
    __shared__ i64 s_anc[kBChunk];
    s_anc[tid] = lo;
    __syncthreads();
    const int cnt = (int)(n - (i64)ch * kBChunk < kBChunk ? n - (i64)ch * kBChunk : kBChunk);
    const int nel = cnt * d;
    const i64 dst0 = (i64)ch * kBChunk * d;
    const float inv_d = 1.0f / (float)d;
    constexpr int UB = 8;
    for (int e0 = 0; e0 < nel; e0 += 256 * UB) {
        double v[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int e = e0 + u * 256 + tid;
            const int ec = e < nel ? e : nel - 1;
            int o = (int)((float)ec * inv_d);
            int col = ec - o * d;
            if (col < 0) {
                --o;
                col += d;
            } else if (col >= d) {
                ++o;
                col -= d;
            }
            v[u] = glb(xs)[s_anc[o] * d + col];
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int e = e0 + u * 256 + tid;
            if (e < nel) glb(xd)[dst0 + e] = v[u];
        }
    }
}

// After redistribution the new copy becomes the current one.
__global__ __launch_bounds__(64) void k_bflip(const BSlot *slots, const int *n_act,
                                              const int *act)
{
    const int k = blockIdx.x * 64 + threadIdx.x;
    if (k >= n_act[0]) return;
    BCtrl *c = slots[act[k]].ctrl;
    if (c->resample && !c->err_call) c->cur ^= 1u;
}

// ------------------------------------------------------------------- host
struct SamplerLayout {
    size_t ctrl, lp, x_scr, lp_scr, pref, status, tpart, tis, epart, cpart, rec_num, upad, total;
};

inline int64_t ntile_of(int64_t n) { return (n + kBTile - 1) / kBTile; }
inline int64_t nchunk_of(int64_t n) { return (n + kBChunk - 1) / kBChunk; }

SamplerLayout sampler_layout(int64_t n, int d)
{
    SamplerLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t nt = (size_t)ntile_of(n);
    L.ctrl = take(sizeof(BCtrl));
    L.lp = take(8 * (size_t)n);
    L.x_scr = take(8 * (size_t)n * d);
    L.lp_scr = take(8 * (size_t)n);
    L.pref = take(8 * (size_t)n);
    L.status = take(8 * nt);
    L.tpart = take(sizeof(TilePart) * nt);
    L.tis = take(sizeof(BTileIS) * (size_t)nchunk_of(n));
    L.epart = take(8 * 2 * (size_t)d * nt);
    L.cpart = take(8 * (2 + 2 * (size_t)d) * (size_t)nchunk_of(n));
    L.rec_num = take(8 * 2 * (size_t)d);
    const size_t DB = (size_t)(d + 7) / 8 * 8;
    L.upad = take(8 * (DB * DB + DB));
    L.total = off;
    return L;
}

struct BatchLayout {
    size_t slots, n_act, act, tile_pref, chunk_pref, unit_pref, bact, btile_pref, total;
};

BatchLayout batch_layout(int cap)
{
    BatchLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    L.slots = take(sizeof(BSlot) * (size_t)cap);
    L.n_act = take(4 * (1 + kBuckets));
    L.act = take(4 * (size_t)cap);
    L.tile_pref = take(4 * (size_t)(cap + 1));
    L.chunk_pref = take(4 * (size_t)(cap + 1));
    L.unit_pref = take(4 * (size_t)(cap + 1));
    L.bact = take(4 * (size_t)kBuckets * cap);
    L.btile_pref = take(4 * (size_t)kBuckets * (cap + 1));
    L.total = off;
    return L;
}

bool finite(double v) { return v == v && v != HUGE_VAL && v != -HUGE_VAL; }

bool desc_ok(const smc_batch_sampler *s)
{
    if (!s || s->n < 1 || s->n > kBMaxN || s->d < 1 || s->d > SMC_BATCH_DMAX) return false;
    if (s->mode < SMC_MODE_AUTO || s->mode > SMC_MODE_NEVER) return false;
    if (s->ess_num < 0 || s->ess_num > 16 || s->ess_den < 1 || s->ess_den > 16) return false;
    if (!finite(s->rw_sd) || !(s->rw_sd > 0.0) || !finite(s->init_sd) || !(s->init_sd > 0.0))
        return false;
    if (!finite(s->init_mean) || !finite(s->init_log_norm) || !finite(s->log_norm)) return false;
    if (!s->mean || !s->chol || !s->x || !s->logw) return false;
    return true;
}

}  // namespace
}  // namespace smc

using namespace smc;

struct smc_batch {
    int cap;
    unsigned char *ws;
    BSlot *d_slots;
    BTabs tabs;
    std::vector<BSlot> h_slots;
    // host mirror of the tables (grid sizes)
    int n_act, total_tiles, total_chunks;
    int64_t total_units;
    int G;  // coordinate pairs per proposal unit
    int quad_waves[kBuckets];  // occupancy aim of k_bquad per dimension bucket
    int btiles[kBuckets];
    // graph of one step for the current membership and output pointers
    bool graph_on;
    hipStream_t cap_stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
    unsigned version, g_version, e_version;
    int eager_same;  // eager steps since the last membership change
    smc_resample_info *g_info;
    double *g_est;
};

namespace {

inline hipStream_t HS(void *s) { return reinterpret_cast<hipStream_t>(s); }

void mirror_update(smc_batch *b)
{
    b->n_act = b->total_tiles = b->total_chunks = 0;
    b->total_units = 0;
    for (int q = 0; q < kBuckets; ++q) b->btiles[q] = 0;
    for (int s = 0; s < b->cap; ++s) {
        const BSlot &v = b->h_slots[s];
        if (v.n <= 0) continue;
        b->n_act += 1;
        b->total_tiles += v.ntile;
        b->total_chunks += v.nchunk;
        b->total_units += units_of(v.nchunk, v.d, b->G);
        b->btiles[v.bucket] += v.nchunk;
    }
    b->version += 1;
    b->eager_same = 0;
}

hipError_t launch_tables(smc_batch *b, hipStream_t s)
{
    hipLaunchKernelGGL(k_btables, dim3(1), dim3(256), 0, s, (const BSlot *)b->d_slots, b->cap,
                       b->G, b->tabs);
    return hipGetLastError();
}

// Buckets from this width up take the matrix-core form of the update (below
// it the vector form measured as fast: a 16-row block is mostly padding).
constexpr int kQuadMxMin = 24;

// Highest occupancy aim the kernel of bucket width DB can meet (LDS and
// registers of the wider rows; the matrix-core kernel needs 166 VGPRs at
// width 64, 150 at 56, 122 at 48); larger requests are clamped to it.
constexpr int max_quad_waves(int DB)
{
    return DB >= kQuadMxMin ? (DB <= 40 ? 4 : 3) : (DB <= 16 ? 4 : (DB <= 40 ? 3 : 2));
}

template <int DB, bool kInit>
void launch_quad_waves(int w, dim3 g, hipStream_t s, const smc_batch *b, int q, int single)
{
    const BSlot *sl = b->d_slots;
    const BTabs &t = b->tabs;
    w = w < max_quad_waves(DB) ? w : max_quad_waves(DB);
    switch (w) {
#define SMC_BQW_CASE(W)                                                                        \
    case W:                                                                                    \
        if constexpr (W <= max_quad_waves(DB)) {                                               \
            if constexpr (DB >= kQuadMxMin)                                                    \
                hipLaunchKernelGGL((k_bquad_mx<DB, kInit, W>), g, dim3(256), 0, s, sl,         \
                                   t.n_act, t.bact, t.btile_pref, q, b->cap, single);          \
            else                                                                               \
                hipLaunchKernelGGL((k_bquad<DB, kInit, W>), g, dim3(256), 0, s, sl, t.n_act,   \
                                   t.bact, t.btile_pref, q, b->cap, single);                   \
        }                                                                                      \
        break;
        SMC_BQW_CASE(1) SMC_BQW_CASE(2) SMC_BQW_CASE(3) SMC_BQW_CASE(4)
#undef SMC_BQW_CASE
    default: break;
    }
}

template <bool kInit>
void launch_quad_bucket(int q, dim3 g, hipStream_t s, const smc_batch *b, int single)
{
    const int w = b->quad_waves[q];
    switch (q) {
    case 0: launch_quad_waves<8, kInit>(w, g, s, b, q, single); break;
    case 1: launch_quad_waves<16, kInit>(w, g, s, b, q, single); break;
    case 2: launch_quad_waves<24, kInit>(w, g, s, b, q, single); break;
    case 3: launch_quad_waves<32, kInit>(w, g, s, b, q, single); break;
    case 4: launch_quad_waves<40, kInit>(w, g, s, b, q, single); break;
    case 5: launch_quad_waves<48, kInit>(w, g, s, b, q, single); break;
    case 6: launch_quad_waves<56, kInit>(w, g, s, b, q, single); break;
    case 7: launch_quad_waves<64, kInit>(w, g, s, b, q, single); break;
    default: break;
    }
}

// Default occupancy aim of the quadratic-form kernel per bucket: the highest
// it reaches (the widest rows need the registers of two waves per SIMD).
inline int default_quad_waves(int q) { return max_quad_waves(8 * (q + 1)); }

hipError_t enqueue_step(smc_batch *b, smc_resample_info *info, double *est, hipStream_t s)
{
    const BSlot *sl = b->d_slots;
    const BTabs &t = b->tabs;
    // the staging block is sized for the unit (2 G columns, one of padding):
    // at 5 or 6 pairs its LDS lets 6 or 5 workgroups share a CU instead of 4
    // (and the kernel needs 73 or 81 VGPRs instead of 97)
    if (b->G <= 5)
        hipLaunchKernelGGL((k_bprop<false, 11>), dim3((unsigned)b->total_units), dim3(256), 0, s, sl,
                           t.n_act, t.act, t.unit_pref, b->G, -1);
    else if (b->G == 6)
        hipLaunchKernelGGL((k_bprop<false, 13>), dim3((unsigned)b->total_units), dim3(256), 0, s, sl,
                           t.n_act, t.act, t.unit_pref, b->G, -1);
    else
        hipLaunchKernelGGL((k_bprop<false, 17>), dim3((unsigned)b->total_units), dim3(256), 0, s, sl,
                           t.n_act, t.act, t.unit_pref, b->G, -1);
    for (int q = 0; q < kBuckets; ++q)
        if (b->btiles[q] > 0) launch_quad_bucket<false>(q, dim3(b->btiles[q]), s, b, -1);
    hipLaunchKernelGGL(k_bscan, dim3(b->total_tiles), dim3(256), 0, s, sl, t.n_act, t.act,
                       t.tile_pref);
    hipLaunchKernelGGL(k_bdecide, dim3(b->n_act), dim3(256), 0, s, sl, t.n_act, t.act, info, est);
    hipLaunchKernelGGL(k_bexpand, dim3(b->total_chunks), dim3(256), 0, s, sl, t.n_act, t.act,
                       t.chunk_pref);
    hipLaunchKernelGGL(k_bflip, dim3((b->n_act + 63) / 64), dim3(64), 0, s, sl, t.n_act, t.act);
    return hipGetLastError();
}

void drop_graph(smc_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

}  // namespace

extern "C" {

size_t smc_batch_sampler_bytes(const smc_batch_sampler *h_s)
{
    if (!desc_ok(h_s)) return 0;
    return sampler_layout(h_s->n, h_s->d).total;
}

size_t smc_batch_workspace_bytes(int32_t capacity)
{
    if (capacity < 1 || capacity > kBMaxCap) return 0;
    return batch_layout(capacity).total;
}

smc_status smc_batch_create(smc_batch **h_out, int32_t capacity, void *ws, size_t ws_bytes,
                            void *stream)
{
    if (!h_out || capacity < 1 || capacity > kBMaxCap || !ws) return SMC_E_ARG;
    if (((uintptr_t)ws & 255) != 0) return SMC_E_ARG;
    const BatchLayout L = batch_layout(capacity);
    if (ws_bytes < L.total) return SMC_E_NOMEM;
    smc_batch *b = new (std::nothrow) smc_batch;
    if (!b) return SMC_E_NOMEM;
    b->cap = capacity;
    b->ws = reinterpret_cast<unsigned char *>(ws);
    b->d_slots = reinterpret_cast<BSlot *>(b->ws + L.slots);
    b->tabs.n_act = reinterpret_cast<int *>(b->ws + L.n_act);
    b->tabs.act = reinterpret_cast<int *>(b->ws + L.act);
    b->tabs.tile_pref = reinterpret_cast<int *>(b->ws + L.tile_pref);
    b->tabs.chunk_pref = reinterpret_cast<int *>(b->ws + L.chunk_pref);
    b->tabs.unit_pref = reinterpret_cast<int *>(b->ws + L.unit_pref);
    b->tabs.bact = reinterpret_cast<int *>(b->ws + L.bact);
    b->tabs.btile_pref = reinterpret_cast<int *>(b->ws + L.btile_pref);
    b->h_slots.assign((size_t)capacity, BSlot());
    for (auto &v : b->h_slots) v.n = 0;
    b->graph_on = true;
    b->G = 8;
    for (int q = 0; q < kBuckets; ++q) b->quad_waves[q] = default_quad_waves(q);
    b->graph = nullptr;
    b->exec = nullptr;
    b->version = 0;
    b->g_version = ~0u;
    b->e_version = ~0u;
    b->eager_same = 0;
    b->g_info = nullptr;
    b->g_est = nullptr;
    if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return SMC_E_DEVICE;
    }
    mirror_update(b);
    hipLaunchKernelGGL(k_bslots_clear, dim3((capacity + 255) / 256), dim3(256), 0, HS(stream),
                       b->d_slots, capacity);
    if (hipGetLastError() != hipSuccess || launch_tables(b, HS(stream)) != hipSuccess) {
        (void)hipStreamDestroy(b->cap_stream);
        delete b;
        return SMC_E_DEVICE;
    }
    *h_out = b;
    return SMC_OK;
}

smc_status smc_batch_attach(smc_batch *b, int32_t slot, const smc_batch_sampler *h_s,
                            void *stream)
{
    if (!b || slot < 0 || slot >= b->cap || !desc_ok(h_s)) return SMC_E_ARG;
    if (b->h_slots[slot].n > 0) return SMC_E_ARG;
    if (!h_s->ws || ((uintptr_t)h_s->ws & 255) != 0) return SMC_E_ARG;
    const SamplerLayout L = sampler_layout(h_s->n, h_s->d);
    if (h_s->ws_bytes < L.total) return SMC_E_NOMEM;
    const int64_t nt = ntile_of(h_s->n), nc = nchunk_of(h_s->n);
    if ((int64_t)b->total_tiles + nt > 0x7fffffff || (int64_t)b->total_chunks + nc > 0x7fffffff ||
        b->total_units + units_of((int)nc, h_s->d, 1) > 0x7fffffff)
        return SMC_E_UNSUPPORTED;
    unsigned char *w = reinterpret_cast<unsigned char *>(h_s->ws);
    BSlot v;
    v.n = h_s->n;
    v.d = h_s->d;
    v.mode = h_s->mode;
    v.ess_num = h_s->ess_num;
    v.ess_den = h_s->ess_den;
    {
        int c = 0;
        while ((1LL << c) < h_s->n) ++c;
        v.K = 61 - c < 52 ? 61 - c : 52;
    }
    v.ntile = (int)nt;
    v.nchunk = (int)nc;
    v.bucket = (h_s->d - 1) / 8;
    v.sampler = h_s->sampler_id;
    v.pad = 0;
    v.seed = h_s->seed;
    v.rw_sd = h_s->rw_sd;
    v.init_mean = h_s->init_mean;
    v.init_sd = h_s->init_sd;
    v.init_prec = 1.0 / (h_s->init_sd * h_s->init_sd);
    v.init_log_norm = h_s->init_log_norm;
    v.log_norm = h_s->log_norm;
    v.reset = -std::log((double)h_s->n);
    v.mean = h_s->mean;
    v.chol = h_s->chol;
    v.x = h_s->x;
    v.logw = h_s->logw;
    v.ctrl = reinterpret_cast<BCtrl *>(w + L.ctrl);
    v.lp = reinterpret_cast<double *>(w + L.lp);
    v.x_scr = reinterpret_cast<double *>(w + L.x_scr);
    v.lp_scr = reinterpret_cast<double *>(w + L.lp_scr);
    v.epart = reinterpret_cast<double *>(w + L.epart);
    v.cpart = reinterpret_cast<double *>(w + L.cpart);
    v.upad = reinterpret_cast<double *>(w + L.upad);
    v.rec_num = reinterpret_cast<double *>(w + L.rec_num);
    v.pref = reinterpret_cast<u64 *>(w + L.pref);
    v.status = reinterpret_cast<u64 *>(w + L.status);
    v.tpart = reinterpret_cast<TilePart *>(w + L.tpart);
    v.tis = reinterpret_cast<BTileIS *>(w + L.tis);
    const hipStream_t s = HS(stream);
    hipLaunchKernelGGL(k_bslot_set, dim3(1), dim3(1), 0, s, v, b->d_slots + slot);
    hipLaunchKernelGGL(k_bpad, dim3(4), dim3(256), 0, s, (const BSlot *)b->d_slots, slot);
    hipLaunchKernelGGL(k_bprop<true>, dim3(v.nchunk), dim3(256), 0, s, (const BSlot *)b->d_slots,
                       b->tabs.n_act, b->tabs.act, b->tabs.unit_pref, b->G, slot);
    launch_quad_bucket<true>(v.bucket, dim3(v.nchunk), s, b, slot);
    hipLaunchKernelGGL(k_binit, dim3(1), dim3(64), 0, s, (const BSlot *)b->d_slots, slot);
    if (hipGetLastError() != hipSuccess) return SMC_E_DEVICE;
    b->h_slots[slot] = v;
    mirror_update(b);
    return launch_tables(b, s) == hipSuccess ? SMC_OK : SMC_E_DEVICE;
}

smc_status smc_batch_detach(smc_batch *b, int32_t slot, void *stream)
{
    if (!b || slot < 0 || slot >= b->cap || b->h_slots[slot].n <= 0) return SMC_E_ARG;
    BSlot v = BSlot();
    v.n = 0;
    const hipStream_t s = HS(stream);
    hipLaunchKernelGGL(k_bslot_set, dim3(1), dim3(1), 0, s, v, b->d_slots + slot);
    if (hipGetLastError() != hipSuccess) return SMC_E_DEVICE;
    b->h_slots[slot].n = 0;
    mirror_update(b);
    return launch_tables(b, s) == hipSuccess ? SMC_OK : SMC_E_DEVICE;
}

smc_status smc_batch_step(smc_batch *b, smc_resample_info *info, double *est, void *stream)
{
    if (!b) return SMC_E_ARG;
    if (b->n_act == 0) return SMC_OK;
    const hipStream_t s = HS(stream);
    if (b->graph_on) {
        const bool same = b->g_version == b->version && b->g_info == info && b->g_est == est;
        if (same && b->exec)
            return hipGraphLaunch(b->exec, s) == hipSuccess ? SMC_OK : SMC_E_DEVICE;
        // capture once the membership has held for two eager steps
        if (b->e_version == b->version && b->eager_same >= 2) {
            drop_graph(b);
            hipGraph_t g = nullptr;
            if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) !=
                hipSuccess)
                return SMC_E_DEVICE;
            const hipError_t le = enqueue_step(b, info, est, b->cap_stream);
            const hipError_t ce = hipStreamEndCapture(b->cap_stream, &g);
            if (le != hipSuccess || ce != hipSuccess || !g) {
                if (g) (void)hipGraphDestroy(g);
                return SMC_E_DEVICE;
            }
            b->graph = g;
            if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
                drop_graph(b);
                return SMC_E_DEVICE;
            }
            b->g_version = b->version;
            b->g_info = info;
            b->g_est = est;
            return hipGraphLaunch(b->exec, s) == hipSuccess ? SMC_OK : SMC_E_DEVICE;
        }
    }
    if (b->e_version != b->version) {
        b->e_version = b->version;
        b->eager_same = 0;
    }
    b->eager_same += 1;
    return enqueue_step(b, info, est, s) == hipSuccess ? SMC_OK : SMC_E_DEVICE;
}

smc_status smc_batch_particles(smc_batch *b, int32_t slot, double **h_x, double **h_lp,
                               void *stream)
{
    if (!b || slot < 0 || slot >= b->cap || b->h_slots[slot].n <= 0) return SMC_E_ARG;
    if (hipStreamSynchronize(HS(stream)) != hipSuccess) return SMC_E_DEVICE;
    const BSlot &v = b->h_slots[slot];
    unsigned cur = 0;
    if (hipMemcpy(&cur, &v.ctrl->cur, sizeof(cur), hipMemcpyDeviceToHost) != hipSuccess)
        return SMC_E_DEVICE;
    if (h_x) *h_x = cur ? v.x_scr : v.x;
    if (h_lp) *h_lp = cur ? v.lp_scr : v.lp;
    return SMC_OK;
}

smc_status smc_batch_set_group(smc_batch *b, int32_t pairs, void *stream)
{
    if (!b || pairs < 1 || pairs > kMaxGroup) return SMC_E_ARG;
    if (pairs == b->G) return SMC_OK;
    b->G = pairs;
    mirror_update(b);
    return launch_tables(b, HS(stream)) == hipSuccess ? SMC_OK : SMC_E_DEVICE;
}

smc_status smc_batch_set_bucket_waves(smc_batch *b, int32_t bucket, int32_t waves)
{
    if (!b || bucket < 0 || bucket >= kBuckets || waves < 1 || waves > 4) return SMC_E_ARG;
    if (b->quad_waves[bucket] == waves) return SMC_OK;
    b->quad_waves[bucket] = waves;
    b->version += 1;  // a captured step holds the old kernel: capture again
    b->eager_same = 0;
    return SMC_OK;
}

smc_status smc_batch_set_graph(smc_batch *b, int32_t enable)
{
    if (!b) return SMC_E_ARG;
    b->graph_on = enable != 0;
    if (!b->graph_on) {
        drop_graph(b);
        b->g_version = ~0u;
    }
    return SMC_OK;
}

smc_status smc_batch_counts(const smc_batch *b, int32_t *h_samplers, int64_t *h_tiles)
{
    if (!b) return SMC_E_ARG;
    if (h_samplers) *h_samplers = b->n_act;
    if (h_tiles) *h_tiles = b->total_tiles;
    return SMC_OK;
}

smc_status smc_batch_sync_error(smc_batch *b, int32_t slot, void *stream)
{
    if (!b || slot < 0 || slot >= b->cap || b->h_slots[slot].n <= 0) return SMC_E_ARG;
    if (hipStreamSynchronize(HS(stream)) != hipSuccess) return SMC_E_DEVICE;
    BCtrl *c = b->h_slots[slot].ctrl;
    unsigned e = 0;
    if (hipMemcpy(&e, &c->err_latch, sizeof(e), hipMemcpyDeviceToHost) != hipSuccess)
        return SMC_E_DEVICE;
    const unsigned zero = 0;
    if (e && hipMemcpy(&c->err_latch, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
        return SMC_E_DEVICE;
    return (smc_status)e;
}

smc_status smc_batch_destroy(smc_batch *b)
{
    if (!b) return SMC_E_ARG;
    drop_graph(b);
    (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return SMC_OK;
}

}  // extern "C"
