// Host-side launchers of the libsmc kernels (one translation unit per kernel
// family).  Every launcher enqueues on `s` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace smc {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kTile = kScanThreads * kScanItems;  // 4096 elements per scan tile
constexpr int kTileShift = 12;
static_assert(kTile == 1 << kTileShift, "tile size");
constexpr int kMaxBlocks = 1024;                  // grid of the max / reweight passes
constexpr int kIsBlocks = 2048;                   // max grid of the sampler kernels
constexpr int kExpandThreads = 256;
constexpr int kSegLen = 2048;                     // merge-path steps per expand workgroup
// Largest row of smc_redistribute: a segment's 32-bit chunk count
// (kSegLen rows of row_bytes / 4 chunks) then stays below 2^31.
constexpr int kMaxRowBytes = 1 << 20;
static_assert((long long)kSegLen * (kMaxRowBytes / 4) < (1ll << 31), "expand chunk count");
constexpr int kEstCols = 10;                      // 2 + 2 d sums of a filter row (d = 4)
static_assert(kSegLen + 1 <= kTile, "an expand segment spans at most two scan tiles");
constexpr int kLogregSplit = 8;                   // row blocks of the likelihood contraction

struct TilePart {
    double Z, Z2;
    u64 q2lo, q2hi;
};

// Device pointers into the caller's workspace.
struct Work {
    Ctrl *ctrl;
    u64 *slots;         // [2][64][16] max / non-finite slots, double-buffered by parity
    u64 *tsum;          // [n_tiles] tile totals, then their exclusive prefix
    TilePart *tpart;    // [n_tiles]
    u64 *pref;          // [n] tile-local inclusive prefix (of q, or of foreign counts)
    u64 *pref64;        // [n / 64 + 1] every 64th tile-local prefix value
    // sampler state (NULL when no target)
    double *lp;         // [n] cached log-target of the current particles
    double *lp_new;     // [n] proposal log-target (costly targets)
    double *x_scr;      // [n * d] redistribute destination
    double *lp_scr;     // [n]
    double *is_part;    // [kIsBlocks * (2 + 2d)] per-block estimate sums
    double *rec_num;    // [2d] recycled estimate sums
    double *epart;      // particle filter: [expand segments][kEstCols] row sums of the
                        // redistributed rows (NULL otherwise)
    // logistic regression (NULL otherwise)
    unsigned short *xs;   // [mpad][dp] bf16 rows of X times (1 - 2 y)
    unsigned short *thb;  // [npad][dp] bf16 copy of the particles times log2 e
    double *csum;         // [dp] column sums of X (1 - 2 y) (of xs for BF16)
    double *xf;           // FP64: [mpad / 16][64][lr_ks(d)] X (1 - 2 y) in MFMA operand order
    double *lpart;        // [kLogregSplit][n] partial log-likelihoods
    int64_t mpad, npad;
    int dp;
    int n_tiles;
    int is_grid;        // blocks of the sampler kernels (rows of is_part)
};

// FP64 likelihood: MFMA k-steps of four columns, d padded to a power of two.
inline int lr_ks(int d) { return d <= 4 ? 1 : d <= 8 ? 2 : d <= 16 ? 4 : d <= 32 ? 8 : 16; }
inline int n_tiles_of(int64_t n) { return (int)((n + kTile - 1) / kTile); }
inline int max_blocks_of(int64_t n)
{
    int64_t b = (n + 2 * 256 * 8 - 1) / (2 * 256 * 8);
    return (int)(b < 1 ? 1 : (b > kMaxBlocks ? kMaxBlocks : b));
}


hipError_t launch_init_ctrl(const Work &w, hipStream_t s);
// Max pass into the slots of parity par, then the fold of those slots.
hipError_t launch_max(const Work &w, const double *lw, int64_t n, int par, hipStream_t s);
hipError_t launch_fold(const Work &w, int par, hipStream_t s);
// Quantise + scan; reads the max slots of parity par.
// clear_uniform: also clears the lazy-reset flag (an iteration's scan runs
// after the kernels that read it).
hipError_t launch_quant_scan(const Work &w, const double *lw, int64_t n, int K, int par,
                             hipStream_t s, bool clear_uniform = false);
// A sampler iteration's statistics, computed by the decision's workgroup
// right after the decision (is_part NULL: none).
struct StatsArgs {
    const double *is_part = nullptr;
    int nblk = 0, d = 0;
    double *rec_num = nullptr, *est = nullptr;
};

// Error and decision of the call from the max slots of parity par and the
// scan; info is a device smc_resample_info (nullable).
hipError_t launch_decide(const Work &w, int par, int64_t n, int K, uint64_t r, int mode,
                         int ess_num, int ess_den, void *info, hipStream_t s,
                         const StatsArgs &st = StatsArgs());
hipError_t launch_clear_scan(const Work &w, hipStream_t s);
// Normalised weights exp(l_i - m) / Z from the last decision.
hipError_t launch_weights(const Work &w, const double *lw, int64_t n, double *out, hipStream_t s);
hipError_t launch_count_scan(const Work &w, const int64_t *ncopies, int64_t n, hipStream_t s);
hipError_t launch_ncopies(const Work &w, int64_t n, int count_mode, int64_t *ncopies,
                          hipStream_t s);
// est_part (nullable; rows of four FP64 values only): per workgroup, the
// count, sums and sums of squares of the rows it wrote, kEstCols doubles.
hipError_t launch_expand(const Work &w, int64_t n, int count_mode, const void *x, void *x_out,
                         int row_bytes, const void *aux, void *aux_out, int aux_bytes,
                         int64_t *ncopies_out, int64_t *anc_out, hipStream_t s,
                         bool skip_identity, double *est_part = nullptr);
inline int64_t expand_segments(int64_t n) { return (2 * n + kSegLen - 1) / kSegLen; }

}  // namespace smc
