// Redistribute (Alg 5 semantics) as a load-balanced expand.
//
// With A_j = (number of output rows taken from sources 0..j), output row p
// comes from anc(p) = #{j : A_j <= p}, so the ancestors are non-decreasing and
// the output order is exactly that of the sequential redistribute.  Copies per
// source range from 0 to N, so a source-parallel copy is unbalanced; instead
// the merge of the two sorted sequences (A_j + j over sources, p over outputs)
// is cut into equal segments of kSegLen merge steps (merge path).  Every
// workgroup owns one segment: a few sources and a few outputs, never more than
// kSegLen in total, whatever the weights.
//
// A_j is computed from the fixed-point prefix as floor((N S_j + U) / S), or is
// the prefix of caller-supplied counts, or j + 1 when the ESS rule decided not
// to resample.  A prefix value is the scan's tile-local value plus the offset
// of its tile of 4096.  The segment boundaries are found by a 64-ary search
// run by one wavefront; the test A_j + j < k is evaluated as
// N S_j + U < (k - j) S in 128-bit integers (no division).  Inside a segment
// the outputs find their sources without a search: each source with copies
// marks its first output, and a max-scan over the outputs carries the marks.
#include <hip/hip_runtime.h>

#include "../../include/smc.h"
#include "common.hpp"
#include "kernels.hpp"

namespace smc {

// n is below 2^31 (the library's limit), so n, A_j <= n and k - j <= 2n all
// fit 32 bits and every product below is a 32 x 64-bit one.
struct AFun {
    i64 n;
    const u64 *pref;  // tile-local inclusive prefix
    const u64 *tpre;  // exclusive prefix of the tile totals
    int mode;  // 0: identity, 1: systematic from S_j, 2: caller counts (A_j = prefix)
    u64 S, U;
    double invS;

    __device__ inline u64 at(i64 j) const { return pref[j] + tpre[j >> kTileShift]; }

    // A_j + j < k, given the prefix value pj of source j
    __device__ inline bool pred_at(i64 j, u64 pj, i64 k) const
    {
        if (mode == 0) return 2 * j + 1 < k;
        if (mode == 2) return (i64)pj + j < k;
        const i64 c = k - j;
        if (c <= 0) return false;
        const U128 lhs = add128(mul32x64((unsigned)n, pj), U);
        const U128 rhs = mul32x64((unsigned)c, S);
        return lt128(lhs, rhs);
    }

    __device__ inline bool pred(i64 j, i64 k) const
    {
        return pred_at(j, mode == 0 ? 0ull : at(j), k);
    }

    __device__ inline u64 A(i64 j) const { return A_of(j, mode == 0 ? 0ull : at(j)); }

    // A_j given the prefix value sj of source j
    __device__ inline u64 A_of(i64 j, u64 sj) const
    {
        if (mode == 0) return (u64)(j + 1);
        if (mode == 2) return sj;
        const U128 num = add128(mul32x64((unsigned)n, sj), U);
        const double est = ((double)n * (double)sj + (double)U) * invS;
        u64 a = est > 0.0 ? (u64)est : 0ull;
        a = a <= (u64)n ? a : (u64)n;  // A_j <= n: keeps a within 32 bits
        // exact correction to a S <= num < (a + 1) S
        U128 aS = mul32x64((unsigned)a, S);
        while (lt128(num, aS)) {
            --a;
            aS = mul32x64((unsigned)a, S);
        }
        U128 a1S = add128(aS, S);
        while (!lt128(num, a1S)) {
            ++a;
            a1S = add128(a1S, S);
        }
        return a;
    }
};

// First index in [lo, hi) where a predicate that is true on a prefix turns
// false (hi if none), by rounds of 64 probes, one per lane.
template <class P>
__device__ inline i64 wave_first_false(const P &pred, i64 lo, i64 hi)
{
    const int lane = threadIdx.x & 63;
    while (hi > lo) {
        const i64 len = hi - lo;
        const i64 stride = (len + 63) / 64;
        const i64 pos = lo + (i64)lane * stride;
        const bool t = pos < hi ? pred(pos) : false;
        const int c = __popcll(__ballot(t));
        if (c == 0) {
            hi = lo;
            break;
        }
        const i64 nlo = lo + (i64)(c - 1) * stride + 1;
        i64 nhi = lo + (i64)c * stride;
        if (nhi > hi) nhi = hi;
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// j(k) = #{j : A_j + j < k}, the number of sources consumed after k merge
// steps, known to lie in [lo, hi].  The test is monotone in j, so it is first
// searched on the sampled prefix values S_{64g+63} (a small array that stays
// in cache), then among the 64 consecutive sources of one group.
__device__ inline i64 wave_search(const AFun &f, const u64 *pref64, i64 k, i64 lo, i64 hi)
{
    if (f.mode == 0) {
        auto p = [&](i64 j) { return f.pred(j, k); };
        return wave_first_false(p, lo, hi);
    }
    const i64 G = f.n >> 6;  // full groups, each with a sample
    const i64 glo = lo >> 6;
    i64 ghi = (hi >> 6) + 1;
    ghi = ghi < G ? ghi : G;
    i64 g = glo;
    if (ghi > glo) {
        auto ps = [&](i64 gg) {
            return f.pred_at(gg * 64 + 63, pref64[gg] + f.tpre[gg >> (kTileShift - 6)], k);
        };
        g = wave_first_false(ps, glo, ghi);
    }
    i64 lo2 = g * 64 > lo ? g * 64 : lo;
    lo2 = lo2 < hi ? lo2 : hi;
    i64 hi2 = g * 64 + 64 < hi ? g * 64 + 64 : hi;
    hi2 = hi2 > lo2 ? hi2 : lo2;
    auto p = [&](i64 j) { return f.pred(j, k); };
    return wave_first_false(p, lo2, hi2);
}

// Chooses the A function of this call; false if nothing may be written.
__device__ inline bool make_afun(const Ctrl *ctrl, const u64 *pref, const u64 *tpre, i64 n,
                                 int count_mode, AFun &f, bool report)
{
    f.n = n;
    f.pref = pref;
    f.tpre = tpre;
    f.S = 1;
    f.U = 0;
    f.invS = 1.0;
    if (count_mode) {
        if (ctrl->ncopy_bad || ctrl->ctotal != (u64)n) {
            if (report) {
                const unsigned err = kErrArg;
                Ctrl *c = const_cast<Ctrl *>(ctrl);
                c->err_call = err;
                if (!c->err_latch) c->err_latch = err;
            }
            return false;
        }
        f.mode = 2;
        return true;
    }
    if (!ctrl->pending || ctrl->err_call) return false;
    f.mode = ctrl->resample ? 1 : 0;
    f.S = ctrl->S;
    f.U = ctrl->U;
    f.invS = 1.0 / (double)ctrl->S;
    return true;
}

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

template <int VEC>
struct VecT;
template <>
struct VecT<16> {
    typedef u32x4 T;
};
template <>
struct VecT<8> {
    typedef u32x2 T;
};
template <>
struct VecT<4> {
    typedef unsigned T;
};

// Copies np rows [p0, p0 + np) of dst from rows sAnc[] of src, VEC bytes per
// lane access; consecutive lanes write consecutive addresses.  The bulk of the
// stores is non-temporal: the new population is not read again by this call,
// and keeping it out of the caches spares the next resample the write-back
// of a cache full of dirty rows (about 5 us per call at N = 2^24 on MI355X).
// kNtLoad: the source rows are read non-temporally too.  A segment whose
// outputs are mostly distinct sources reads each line about once; streaming
// those lines past the caches measured 48 us faster per call at N = 2^24,
// s = 0.5 (HBM read requests are whole 128-byte lines either way).  Where a
// few sources fill many outputs (heavy degeneracy) the cached reads are
// faster, the same lines serving the whole segment.
// kSum (VEC = 16, rows of four FP64 values): the thread also adds up the two
// values of every chunk it copies, and their squares, into acc; its chunks all
// sit in the same half of a row (the lane stride is a multiple of two chunks).
__device__ inline void add_chunk(const u32x4 &v, double *acc)
{
    const double lo = __hiloint2double((int)v.y, (int)v.x);
    const double hi = __hiloint2double((int)v.w, (int)v.z);
    acc[0] += lo;
    acc[1] += hi;
    acc[2] += lo * lo;
    acc[3] += hi * hi;
}

template <int VEC, bool kSum = false, bool kNtLoad = false>
__device__ inline void copy_rows(const unsigned char *__restrict__ src,
                                 unsigned char *__restrict__ dst, int row_bytes, int cpr_shift,
                                 const unsigned *sAnc, i64 p0, int np, double *acc = nullptr)
{
    static_assert(!kSum || VEC == 16, "row sums take 16-byte chunks");
    typedef typename VecT<VEC>::T V;
    const int cpr = row_bytes / VEC;
    const int total = np * cpr;
    const int tid = threadIdx.x;
    constexpr int U = 4;
    int c = tid;
    for (; c + (U - 1) * kExpandThreads < total; c += U * kExpandThreads) {
        V v[U];
        i64 doff[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int cc = c + u * kExpandThreads;
            int r, col;
            if (cpr_shift >= 0) {
                r = cc >> cpr_shift;
                col = cc & (cpr - 1);
            } else {
                r = cc / cpr;
                col = cc - r * cpr;
            }
            const V *sp = reinterpret_cast<const V *>(src + (i64)sAnc[r] * row_bytes + col * VEC);
            v[u] = kNtLoad ? __builtin_nontemporal_load(sp) : *sp;
            doff[u] = (p0 + r) * (i64)row_bytes + col * VEC;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], reinterpret_cast<V *>(dst + doff[u]));
        if constexpr (kSum) {
#pragma unroll
            for (int u = 0; u < U; ++u) add_chunk(v[u], acc);
        }
    }
    for (; c < total; c += kExpandThreads) {
        int r, col;
        if (cpr_shift >= 0) {
            r = c >> cpr_shift;
            col = c & (cpr - 1);
        } else {
            r = c / cpr;
            col = c - r * cpr;
        }
        const V v = *reinterpret_cast<const V *>(src + (i64)sAnc[r] * row_bytes + col * VEC);
        *reinterpret_cast<V *>(dst + (p0 + r) * (i64)row_bytes + col * VEC) = v;
        if constexpr (kSum) add_chunk(v, acc);
    }
}

// Rows of 8 bytes with an 8-byte side row each (a 1-D sampler's particle and
// its cached log-target): both copies in one loop, twice the loads in flight;
// kNtLoad as in copy_rows.
template <bool kNtLoad>
__device__ inline void copy_rows_8x2(const unsigned char *__restrict__ src,
                                     unsigned char *__restrict__ dst,
                                     const unsigned char *__restrict__ src2,
                                     unsigned char *__restrict__ dst2, const unsigned *sAnc,
                                     i64 p0, int np)
{
    typedef unsigned long long V;
    const V *s1 = reinterpret_cast<const V *>(src), *s2 = reinterpret_cast<const V *>(src2);
    V *d1 = reinterpret_cast<V *>(dst) + p0, *d2 = reinterpret_cast<V *>(dst2) + p0;
    constexpr int U = 4;
    int r = threadIdx.x;
    for (; r + (U - 1) * kExpandThreads < np; r += U * kExpandThreads) {
        V v[U], w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned j = sAnc[r + u * kExpandThreads];
            v[u] = kNtLoad ? __builtin_nontemporal_load(s1 + j) : s1[j];
            w[u] = kNtLoad ? __builtin_nontemporal_load(s2 + j) : s2[j];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            __builtin_nontemporal_store(v[u], d1 + r + u * kExpandThreads);
            __builtin_nontemporal_store(w[u], d2 + r + u * kExpandThreads);
        }
    }
    for (; r < np; r += kExpandThreads) {
        const unsigned j = sAnc[r];
        d1[r] = s1[j];
        d2[r] = s2[j];
    }
}

// Sums of the rows one workgroup wrote (rows of four FP64 values, two 16-byte
// chunks each): lanes of equal parity hold the same half of a row; their sums
// are combined in a fixed order and written in the filter's estimate layout
// (column 0 unused here, 1 the row count, 2 + k the sum of value k, 6 + k the
// sum of its square).
__device__ inline void store_row_sums(double *acc, int np, double *out)
{
    __shared__ double s_acc[kExpandThreads / 64][2][4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        for (int o = 2; o < 64; o <<= 1) acc[k] += __shfl_xor(acc[k], o, 64);
    if (lane < 2)
        for (int k = 0; k < 4; ++k) s_acc[wid][lane][k] = acc[k];
    __syncthreads();
    if (tid < kEstCols) {
        double v = tid == 1 ? (double)np : 0.0;
        if (tid >= 2) {
            const int k = (tid - 2) & 3;                  // value k = 2 h + half
            const int j = (tid >= 6 ? 2 : 0) + (k & 1);   // its sum, or its square's
            v = s_acc[0][k >> 1][j];
            for (int w = 1; w < kExpandThreads / 64; ++w) v += s_acc[w][k >> 1][j];
        }
        out[tid] = v;
    }
}

struct ExpandArgs {
    i64 n;
    const u64 *pref;
    const u64 *pref64;
    const u64 *tpre;
    const Ctrl *ctrl;
    int count_mode;
    const unsigned char *x;
    unsigned char *xo;
    int row_bytes, cpr_shift;
    const unsigned char *aux;
    unsigned char *auxo;
    int aux_bytes, aux_shift;
    i64 *nc_out;
    i64 *anc_out;
    int skip_identity;  // when the decision is "no resample", write nothing
    double *est_part;   // kSum: [segments][kEstCols] sums of the rows written
};

template <int VEC, bool kSum = false>
__global__ __launch_bounds__(kExpandThreads) void k_expand(ExpandArgs a)
{
    __shared__ unsigned sA[kSegLen + 1];
    __shared__ __attribute__((aligned(16))) unsigned sAnc[kSegLen];
    __shared__ i64 s_j[2];
    __shared__ u64 s_wmax[kExpandThreads / 64];
    const int tid = threadIdx.x, wid = tid >> 6;
    AFun f;
    if (!make_afun(a.ctrl, a.pref, a.tpre, a.n, a.count_mode, f, blockIdx.x == 0 && tid == 0))
        return;
    if (a.skip_identity && f.mode == 0) return;

    const i64 n = a.n;
    const i64 k0 = (i64)blockIdx.x * kSegLen;
    const i64 k1 = (k0 + kSegLen < 2 * n) ? k0 + kSegLen : 2 * n;
    if (wid < 2) {
        const i64 k = wid == 0 ? k0 : k1;
        const i64 lo = k - n > 0 ? k - n : 0;
        const i64 hi = k < n ? k : n;
        const i64 j = wave_search(f, a.pref64, k, lo, hi);
        if ((tid & 63) == 0) s_j[wid] = j;
    }
    __syncthreads();
    const i64 j0 = s_j[0], j1 = s_j[1];
    const i64 p0 = k0 - j0;
    const int ns = (int)(j1 - j0), np = (int)((k1 - j1) - p0);

    // sources j0 - 1 .. j1 - 1 (at most kSegLen + 1 < 4096) lie in at most two
    // tiles: their offsets are read once
    const i64 ta = (j0 > 0 ? j0 - 1 : 0) >> kTileShift;
    const i64 ntl = (n + kTile - 1) >> kTileShift;
    const u64 off_a = f.mode ? f.tpre[ta] : 0ull;
    const u64 off_b = (f.mode && ta + 1 < ntl) ? f.tpre[ta + 1] : 0ull;
    for (int i = tid; i <= ns; i += kExpandThreads) {
        const i64 j = j0 - 1 + i;
        if (j < 0) {
            sA[i] = 0u;
            continue;
        }
        const u64 sj = f.mode ? a.pref[j] + ((j >> kTileShift) == ta ? off_a : off_b) : 0ull;
        sA[i] = (unsigned)f.A_of(j, sj);
    }
    __syncthreads();
    if (a.nc_out)
        for (int i = tid; i < ns; i += kExpandThreads)
            a.nc_out[j0 + i] = (i64)sA[i + 1] - (i64)sA[i];
    // Output p comes from local source t, the first with sA[1 + t] > p, so
    // sA[t] <= p < sA[1 + t] (sA[0] <= p0 by the merge-path cut).  Each source
    // with copies marks the first of its outputs inside the segment with
    // t + 1; an inclusive max-scan over the outputs carries every mark over
    // the rest of its source's outputs.  Local source ns (source j1) owns
    // whatever follows sA[ns].  Marks land on distinct outputs (sources with
    // copies start at distinct outputs) and output p0 always holds one.
    for (int r = tid; r < np; r += kExpandThreads) sAnc[r] = 0u;
    __syncthreads();
    for (int t = tid; t <= ns; t += kExpandThreads) {
        const i64 lo = sA[t];
        const i64 hi = t < ns ? (i64)sA[t + 1] : INT64_MAX;
        if (hi > lo && hi > p0) {
            const i64 st = (lo > p0 ? lo : p0) - p0;
            if (st < np) sAnc[st] = (unsigned)(t + 1);
        }
    }
    __syncthreads();
    {
        constexpr int E = kSegLen / kExpandThreads;  // outputs per thread, contiguous
        static_assert(E == 8, "two 16-byte LDS reads per thread");
        const int lane = tid & 63;
        // entries past np are stale; they reach only positions past np
        const uint4 q0 = reinterpret_cast<const uint4 *>(sAnc)[2 * tid];
        const uint4 q1 = reinterpret_cast<const uint4 *>(sAnc)[2 * tid + 1];
        unsigned v[E] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
        unsigned run = 0u;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            run = v[e] > run ? v[e] : run;
            v[e] = run;
        }
        const u64 incl = wave_scan_u64((u64)run, 0ull, [](u64 x, u64 y) { return y > x ? y : x; });
        if (lane == 63) s_wmax[wid] = incl;
        u64 carry = (u64)__shfl_up((long long)incl, 1, 64);
        carry = lane ? carry : 0ull;
        __syncthreads();
        for (int w = 0; w < wid; ++w) carry = s_wmax[w] > carry ? s_wmax[w] : carry;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int r = tid * E + e;
            if (r < np) {
                const unsigned m = v[e] > (unsigned)carry ? v[e] : (unsigned)carry;
                i64 anc = j0 + (i64)m - 1;
                anc = anc < n ? anc : n - 1;
                sAnc[r] = (unsigned)anc;
                if (a.anc_out) a.anc_out[p0 + r] = anc;
            }
        }
    }
    __syncthreads();
    if constexpr (kSum) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (np < 2 * ns)
            copy_rows<VEC, true, true>(a.x, a.xo, a.row_bytes, a.cpr_shift, sAnc, p0, np, acc);
        else
            copy_rows<VEC, true>(a.x, a.xo, a.row_bytes, a.cpr_shift, sAnc, p0, np, acc);
        store_row_sums(acc, np, a.est_part + (i64)blockIdx.x * kEstCols);
    } else if (VEC == 8 && a.row_bytes == 8 && a.aux && a.aux_bytes == 8) {
        if (np < 2 * ns) copy_rows_8x2<true>(a.x, a.xo, a.aux, a.auxo, sAnc, p0, np);
        else copy_rows_8x2<false>(a.x, a.xo, a.aux, a.auxo, sAnc, p0, np);
        return;
    } else if (np < 2 * ns) {
        // fewer than two outputs per source in this segment
        copy_rows<VEC, false, true>(a.x, a.xo, a.row_bytes, a.cpr_shift, sAnc, p0, np);
    } else {
        copy_rows<VEC>(a.x, a.xo, a.row_bytes, a.cpr_shift, sAnc, p0, np);
    }
    if (a.aux) {
        if (np < 2 * ns)
            copy_rows<8, false, true>(a.aux, a.auxo, a.aux_bytes, a.aux_shift, sAnc, p0, np);
        else
            copy_rows<8>(a.aux, a.auxo, a.aux_bytes, a.aux_shift, sAnc, p0, np);
    }
}

static int shift_of(int v)
{
    if (v <= 0 || (v & (v - 1))) return -1;
    int s = 0;
    while ((1 << s) < v) ++s;
    return s;
}

hipError_t launch_expand(const Work &w, int64_t n, int count_mode, const void *x, void *x_out,
                         int row_bytes, const void *aux, void *aux_out, int aux_bytes,
                         int64_t *ncopies_out, int64_t *anc_out, hipStream_t s,
                         bool skip_identity, double *est_part)
{
    ExpandArgs a;
    a.skip_identity = skip_identity ? 1 : 0;
    a.n = n;
    a.pref = w.pref;
    a.pref64 = w.pref64;
    a.tpre = w.tsum;
    a.ctrl = w.ctrl;
    a.count_mode = count_mode;
    a.x = reinterpret_cast<const unsigned char *>(x);
    a.xo = reinterpret_cast<unsigned char *>(x_out);
    a.row_bytes = row_bytes;
    a.aux = reinterpret_cast<const unsigned char *>(aux);
    a.auxo = reinterpret_cast<unsigned char *>(aux_out);
    a.aux_bytes = aux_bytes;
    a.aux_shift = shift_of(aux_bytes / 8);
    a.nc_out = reinterpret_cast<i64 *>(ncopies_out);
    a.anc_out = reinterpret_cast<i64 *>(anc_out);
    a.est_part = est_part;
    const uintptr_t al = (uintptr_t)x | (uintptr_t)x_out | (uintptr_t)row_bytes;
    const int64_t segs = expand_segments(n);
    if (est_part) {
        if ((al & 15) != 0 || row_bytes != 32) return hipErrorInvalidValue;
        a.cpr_shift = 1;
        hipLaunchKernelGGL((k_expand<16, true>), dim3((unsigned)segs), dim3(kExpandThreads), 0, s,
                           a);
    } else if ((al & 15) == 0) {
        a.cpr_shift = shift_of(row_bytes / 16);
        hipLaunchKernelGGL(k_expand<16>, dim3((unsigned)segs), dim3(kExpandThreads), 0, s, a);
    } else if ((al & 7) == 0) {
        a.cpr_shift = shift_of(row_bytes / 8);
        hipLaunchKernelGGL(k_expand<8>, dim3((unsigned)segs), dim3(kExpandThreads), 0, s, a);
    } else {
        a.cpr_shift = shift_of(row_bytes / 4);
        hipLaunchKernelGGL(k_expand<4>, dim3((unsigned)segs), dim3(kExpandThreads), 0, s, a);
    }
    return hipGetLastError();
}

// ncopies_j = A_j - A_{j-1} for every source (elementwise).
__global__ __launch_bounds__(256) void k_ncopies(const Ctrl *ctrl, const u64 *pref,
                                                 const u64 *tpre, i64 n, int count_mode, i64 *nc)
{
    AFun f;
    if (!make_afun(ctrl, pref, tpre, n, count_mode, f, false)) return;
    const i64 gtid = (i64)blockIdx.x * 256 + threadIdx.x, gsz = (i64)gridDim.x * 256;
    for (i64 j = gtid; j < n; j += gsz) {
        const u64 a1 = f.A(j);
        const u64 a0 = j > 0 ? f.A(j - 1) : 0;
        nc[j] = (i64)(a1 - a0);
    }
}

hipError_t launch_ncopies(const Work &w, int64_t n, int count_mode, int64_t *ncopies,
                          hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    blocks = blocks > 4096 ? 4096 : blocks;
    hipLaunchKernelGGL(k_ncopies, dim3((unsigned)blocks), dim3(256), 0, s, w.ctrl, w.pref, w.tsum,
                       (i64)n, count_mode, reinterpret_cast<i64 *>(ncopies));
    return hipGetLastError();
}

}  // namespace smc
