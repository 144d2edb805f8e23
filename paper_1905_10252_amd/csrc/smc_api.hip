// libsmc C ABI: argument checking, workspace layout and the launch sequence
// of each entry point.  No entry point allocates device memory or
// synchronises (except smc_sync_error); everything is enqueued on the
// caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/smc.h"
#include "common.hpp"
#include "kernels.hpp"
#include "reduce.hpp"
#include "step.hpp"

using namespace smc;

// Workspace of smc_resample_noalloc: a resample-only context's sections for
// up to SMC_NOALLOC_MAX_N weights (as layout_of() places them in a caller's
// workspace), in a fixed device array, one copy per GPU, held until the
// process ends (about 8.6 MB).
static constexpr size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
static constexpr size_t kNaTiles = ((size_t)SMC_NOALLOC_MAX_N + kTile - 1) / kTile;
static constexpr size_t kNaCtrl = 0;
static constexpr size_t kNaSlots = kNaCtrl + al256(sizeof(Ctrl));
static constexpr size_t kNaTsum = kNaSlots + al256(8 * (size_t)kSlotWords);
static constexpr size_t kNaTpart = kNaTsum + al256(8 * kNaTiles);
static constexpr size_t kNaPref = kNaTpart + al256(sizeof(TilePart) * kNaTiles);
static constexpr size_t kNaPref64 = kNaPref + al256(8 * (size_t)SMC_NOALLOC_MAX_N);
static constexpr size_t kNaBytes = kNaPref64 + al256(8 * ((size_t)SMC_NOALLOC_MAX_N / 64 + 1));
static __device__ __align__(256) unsigned char scratch[kNaBytes];

struct smc_ctx {
    smc_config cfg;
    Work w;
    void *ws;
    size_t ws_bytes;
    int K;
    bool pending;   // the workspace prefix belongs to the last smc_resample
    uint32_t t;     // sampler iteration counter (Alg 2 t)
    int par;        // parity of the max slots used by the next call
};

namespace {

struct Layout {
    size_t ctrl, slots, tsum, tpart, pref, pref64;
    size_t lp, lp_new, x_scr, lp_scr, is_part, rec_num, epart;
    size_t xs, thb, csum, xf, lpart;
    int64_t mpad, npad;
    int dp;
    size_t total;
};

bool config_ok(const smc_config *c)
{
    if (!c) return false;
    if (c->n < 1 || c->n > 0x7fffffffLL) return false;
    if (c->d < 1) return false;
    if (c->x_dtype != SMC_DTYPE_F32 && c->x_dtype != SMC_DTYPE_F64) return false;
    if (c->ess_num < 0 || c->ess_num > 16 || c->ess_den < 1 || c->ess_den > 16) return false;
    if (c->mode < SMC_MODE_AUTO || c->mode > SMC_MODE_NEVER) return false;
    if (c->target < SMC_TARGET_NONE || c->target > SMC_TARGET_BEARING) return false;
    if (c->lazy_reset != 0 && c->lazy_reset != 1) return false;
    if (c->target != SMC_TARGET_NONE) {
        if (c->d > kMaxDim || c->x_dtype != SMC_DTYPE_F64) return false;
        if (!(c->rw_sd >= 0.0) || !(c->init_sd > 0.0)) return false;
        if (c->target == SMC_TARGET_GAUSS && (!c->mean || !c->prec)) return false;
        if (c->target == SMC_TARGET_STUDENT && (c->d != 1 || !(c->nu > 0.0))) return false;
        if (c->target == SMC_TARGET_BEARING &&
            (c->d != 4 || !c->mean || !c->obs || c->n_obs < 1 || !(c->delta > 0.0) ||
             !(c->obs_var > 0.0)))
            return false;
        if (c->target == SMC_TARGET_LOGREG &&
            (!c->X || !c->y || c->m_rows < 1 || !(c->prior_prec > 0.0) ||
             (c->loglik_precision != SMC_PREC_F64 && c->loglik_precision != SMC_PREC_BF16)))
            return false;
    }
    return true;
}

Layout layout_of(const smc_config *c)
{
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t n = (size_t)c->n, d = (size_t)c->d;
    const size_t nt = (size_t)n_tiles_of(c->n);
    L.ctrl = take(sizeof(Ctrl));
    L.slots = take(8 * (size_t)kSlotWords);
    L.tsum = take(8 * nt);
    L.tpart = take(sizeof(TilePart) * nt);
    L.pref = take(8 * n);
    L.pref64 = take(8 * (n / 64 + 1));
    L.lp = L.lp_new = L.x_scr = L.lp_scr = L.is_part = L.rec_num = L.epart = 0;
    L.xs = L.thb = L.csum = L.xf = L.lpart = 0;
    L.dp = (int)((d + 15) / 16 * 16);
    L.mpad = (c->m_rows + 31) / 32 * 32;
    L.npad = (int64_t)((n + 31) / 32 * 32);
    if (c->target != SMC_TARGET_NONE) {
        L.lp = take(8 * n);
        L.lp_new = take(8 * n);
        L.x_scr = take(8 * n * d);
        L.lp_scr = take(8 * n);
        L.is_part = take(8 * (size_t)kIsBlocks * (2 + 2 * d));
        L.rec_num = take(8 * 2 * d);
        if (c->target == SMC_TARGET_BEARING)
            L.epart = take(8 * (size_t)kEstCols * (size_t)expand_segments(c->n));
        if (c->target == SMC_TARGET_LOGREG) {
            L.lpart = take(8 * (size_t)kLogregSplit * n);
            L.csum = take(8 * (size_t)L.dp);
            if (c->loglik_precision == SMC_PREC_BF16) {
                L.xs = take(2 * (size_t)L.mpad * L.dp);
                L.thb = take(2 * (size_t)L.npad * L.dp);
            } else {
                L.xf = take(8 * (size_t)L.mpad * 4 * lr_ks(c->d));
            }
        }
    }
    L.total = off;
    return L;
}

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------ smc_resample_noalloc
// Per-device address of `scratch`, looked up once per device (the array's
// name is not a device address in host code).
constexpr int kNaMaxDevices = 64;
std::mutex g_na_mutex;
unsigned char *g_na_ptr[kNaMaxDevices];

unsigned char *noalloc_scratch()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNaMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_na_mutex);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_na_ptr[dev] = reinterpret_cast<unsigned char *>(p);
    }
    return g_na_ptr[dev];
}

bool overlap(const void *a, const void *b, size_t bytes)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bytes && y < x + bytes;
}

}  // namespace

extern "C" {

const char *smc_status_string(smc_status s)
{
    switch (s) {
    case SMC_OK: return "ok";
    case SMC_E_ARG: return "invalid argument";
    case SMC_E_NONFINITE: return "non-finite log-weight (NaN or +inf)";
    case SMC_E_DEGENERATE: return "all weights are zero";
    case SMC_E_NOMEM: return "workspace too small";
    case SMC_E_DEVICE: return "HIP runtime error";
    case SMC_E_UNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

size_t smc_workspace_bytes(const smc_config *h_cfg)
{
    if (!config_ok(h_cfg)) return 0;
    return layout_of(h_cfg).total;
}

smc_status smc_init(smc_ctx **h_out, const smc_config *h_cfg, void *workspace,
                    size_t workspace_bytes, void *x, double *logw, void *stream)
{
    if (!h_out) return SMC_E_ARG;
    *h_out = nullptr;
    if (!config_ok(h_cfg) || !workspace || ((uintptr_t)workspace & 255)) return SMC_E_ARG;
    const Layout L = layout_of(h_cfg);
    if (workspace_bytes < L.total) return SMC_E_NOMEM;
    if (h_cfg->target != SMC_TARGET_NONE && (!x || !logw)) return SMC_E_ARG;
    smc_ctx *ctx = new (std::nothrow) smc_ctx;
    if (!ctx) return SMC_E_NOMEM;
    ctx->cfg = *h_cfg;
    ctx->ws = workspace;
    ctx->ws_bytes = workspace_bytes;
    ctx->pending = false;
    ctx->t = 0;
    ctx->par = 0;
    {
        int c = 0;
        while ((1LL << c) < h_cfg->n) ++c;
        ctx->K = 61 - c < 52 ? 61 - c : 52;
    }
    unsigned char *b = reinterpret_cast<unsigned char *>(workspace);
    Work &w = ctx->w;
    w.ctrl = reinterpret_cast<Ctrl *>(b + L.ctrl);
    w.slots = reinterpret_cast<u64 *>(b + L.slots);
    w.tsum = reinterpret_cast<u64 *>(b + L.tsum);
    w.tpart = reinterpret_cast<TilePart *>(b + L.tpart);
    w.pref = reinterpret_cast<u64 *>(b + L.pref);
    w.pref64 = reinterpret_cast<u64 *>(b + L.pref64);
    w.n_tiles = n_tiles_of(h_cfg->n);
    const bool samp = h_cfg->target != SMC_TARGET_NONE;
    w.lp = samp ? reinterpret_cast<double *>(b + L.lp) : nullptr;
    w.lp_new = samp ? reinterpret_cast<double *>(b + L.lp_new) : nullptr;
    w.x_scr = samp ? reinterpret_cast<double *>(b + L.x_scr) : nullptr;
    w.lp_scr = samp ? reinterpret_cast<double *>(b + L.lp_scr) : nullptr;
    w.is_part = samp ? reinterpret_cast<double *>(b + L.is_part) : nullptr;
    w.rec_num = samp ? reinterpret_cast<double *>(b + L.rec_num) : nullptr;
    w.epart = L.epart ? reinterpret_cast<double *>(b + L.epart) : nullptr;
    w.lpart = L.lpart ? reinterpret_cast<double *>(b + L.lpart) : nullptr;
    w.xs = L.xs ? reinterpret_cast<unsigned short *>(b + L.xs) : nullptr;
    w.thb = L.thb ? reinterpret_cast<unsigned short *>(b + L.thb) : nullptr;
    w.csum = L.csum ? reinterpret_cast<double *>(b + L.csum) : nullptr;
    w.xf = L.xf ? reinterpret_cast<double *>(b + L.xf) : nullptr;
    w.mpad = L.mpad;
    w.npad = L.npad;
    w.dp = L.dp;
    w.is_grid = samp ? sampler_grid(ctx->cfg) : 0;
    if ((samp && w.is_grid < 1) || launch_init_ctrl(w, S(stream)) != hipSuccess) {
        delete ctx;
        return SMC_E_DEVICE;
    }
    if (samp) {
        const smc_status st = step_init(ctx->cfg, w, ctx->par, reinterpret_cast<double *>(x),
                                        logw, S(stream));
        ctx->par ^= 1;
        if (st != SMC_OK) {
            delete ctx;
            return st;
        }
    }
    *h_out = ctx;
    return SMC_OK;
}

smc_status smc_resample(smc_ctx *ctx, const double *logw, int64_t n, uint64_t r, int32_t mode,
                        int64_t *ncopies, smc_resample_info *info, void *stream)
{
    if (!ctx || !logw || n != ctx->cfg.n) return SMC_E_ARG;
    if (mode < SMC_MODE_AUTO || mode > SMC_MODE_NEVER) return SMC_E_ARG;
    if (((uintptr_t)logw & 7) || ((uintptr_t)ncopies & 7) || ((uintptr_t)info & 7))
        return SMC_E_ARG;
    const Work &w = ctx->w;
    hipStream_t s = S(stream);
    const int par = ctx->par;
    ctx->par ^= 1;
    if (launch_max(w, logw, n, par, s) != hipSuccess) return SMC_E_DEVICE;
    if (launch_quant_scan(w, logw, n, ctx->K, par, s) != hipSuccess) return SMC_E_DEVICE;
    if (launch_decide(w, par, n, ctx->K, r, mode, ctx->cfg.ess_num, ctx->cfg.ess_den, info, s) !=
        hipSuccess)
        return SMC_E_DEVICE;
    ctx->pending = true;
    if (ncopies && launch_ncopies(w, n, 0, ncopies, s) != hipSuccess) return SMC_E_DEVICE;
    return SMC_OK;
}

smc_status smc_resample_noalloc(const double *logw, int64_t n, uint64_t r, int32_t mode,
                                int32_t ess_num, int32_t ess_den, int64_t *ncopies,
                                smc_resample_info *info, void *stream)
{
    if (!logw || !ncopies || n < 1) return SMC_E_ARG;
    if (n > SMC_NOALLOC_MAX_N) return SMC_E_NOMEM;
    if (mode < SMC_MODE_AUTO || mode > SMC_MODE_NEVER) return SMC_E_ARG;
    if (ess_num < 0 || ess_num > 16 || ess_den < 1 || ess_den > 16) return SMC_E_ARG;
    if (((uintptr_t)logw & 7) || ((uintptr_t)ncopies & 7) || ((uintptr_t)info & 7))
        return SMC_E_ARG;
    unsigned char *b = noalloc_scratch();
    if (!b) return SMC_E_DEVICE;
    Work w{};
    w.ctrl = reinterpret_cast<Ctrl *>(b + kNaCtrl);
    w.slots = reinterpret_cast<u64 *>(b + kNaSlots);
    w.tsum = reinterpret_cast<u64 *>(b + kNaTsum);
    w.tpart = reinterpret_cast<TilePart *>(b + kNaTpart);
    w.pref = reinterpret_cast<u64 *>(b + kNaPref);
    w.pref64 = reinterpret_cast<u64 *>(b + kNaPref64);
    w.n_tiles = n_tiles_of(n);
    int c = 0;
    while ((1LL << c) < n) ++c;
    const int K = 61 - c < 52 ? 61 - c : 52;
    hipStream_t s = S(stream);
    // the last call's control block and max slots are cleared by a kernel
    // (no memset node if the caller captures the stream); parity 0 always
    if (launch_init_ctrl(w, s) != hipSuccess) return SMC_E_DEVICE;
    if (launch_max(w, logw, n, 0, s) != hipSuccess) return SMC_E_DEVICE;
    if (launch_quant_scan(w, logw, n, K, 0, s) != hipSuccess) return SMC_E_DEVICE;
    if (launch_decide(w, 0, n, K, r, mode, ess_num, ess_den, info, s) != hipSuccess)
        return SMC_E_DEVICE;
    if (launch_ncopies(w, n, 0, ncopies, s) != hipSuccess) return SMC_E_DEVICE;
    return SMC_OK;
}

smc_status smc_normalised_weights(smc_ctx *ctx, const double *logw, int64_t n, double *w,
                                  void *stream)
{
    if (!ctx || !logw || !w || n != ctx->cfg.n) return SMC_E_ARG;
    if (((uintptr_t)logw & 7) || ((uintptr_t)w & 7)) return SMC_E_ARG;
    if (overlap(logw, w, (size_t)n * 8)) return SMC_E_ARG;
    return launch_weights(ctx->w, logw, n, w, S(stream)) == hipSuccess ? SMC_OK : SMC_E_DEVICE;
}

smc_status smc_redistribute(smc_ctx *ctx, const int64_t *ncopies, const void *x, void *x_out,
                            int64_t n, int32_t row_bytes, int64_t *ncopies_out, int64_t *anc,
                            void *stream)
{
    if (!ctx || !x || !x_out || n != ctx->cfg.n) return SMC_E_ARG;
    if (row_bytes <= 0 || (row_bytes & 3) || row_bytes > kMaxRowBytes) return SMC_E_ARG;
    if (((uintptr_t)x & 3) || ((uintptr_t)x_out & 3)) return SMC_E_ARG;
    if (((uintptr_t)ncopies & 7) || ((uintptr_t)ncopies_out & 7) || ((uintptr_t)anc & 7))
        return SMC_E_ARG;
    if ((uint64_t)n * (uint64_t)row_bytes > (1ull << 46)) return SMC_E_ARG;
    if (overlap(x, x_out, (size_t)n * (size_t)row_bytes)) return SMC_E_ARG;
    if (!ncopies && !ctx->pending) return SMC_E_ARG;
    const Work &w = ctx->w;
    hipStream_t s = S(stream);
    int count_mode = 0;
    if (ncopies) {
        if (launch_clear_scan(w, s) != hipSuccess) return SMC_E_DEVICE;
        if (launch_count_scan(w, ncopies, n, s) != hipSuccess) return SMC_E_DEVICE;
        ctx->pending = false;
        count_mode = 1;
    }
    if (launch_expand(w, n, count_mode, x, x_out, row_bytes, nullptr, nullptr, 0, ncopies_out, anc,
                      s, false) != hipSuccess)
        return SMC_E_DEVICE;
    return SMC_OK;
}

smc_status smc_step(smc_ctx *ctx, void *x, double *logw, smc_resample_info *info, double *est,
                    void *stream)
{
    if (!ctx || !x || !logw || ctx->cfg.target == SMC_TARGET_NONE) return SMC_E_ARG;
    if (((uintptr_t)x & 7) || ((uintptr_t)logw & 7) || ((uintptr_t)info & 7) ||
        ((uintptr_t)est & 7))
        return SMC_E_ARG;
    if (ctx->cfg.target == SMC_TARGET_BEARING && (int64_t)ctx->t >= (int64_t)ctx->cfg.n_obs)
        return SMC_E_ARG;  // no measurement left
    ctx->t += 1;
    const int par = ctx->par;
    ctx->par ^= 1;
    const smc_status st = step_run(ctx->cfg, ctx->w, ctx->K, par, ctx->t,
                                   reinterpret_cast<double *>(x), logw, info, est, S(stream));
    ctx->pending = false;  // the step reuses the prefix buffer
    return st;
}

smc_status smc_steps(smc_ctx *ctx, void *x, double *logw, int32_t nsteps,
                     smc_resample_info *info, double *est, void *stream)
{
    if (!ctx || !x || !logw || nsteps < 1 || ctx->cfg.target == SMC_TARGET_NONE) return SMC_E_ARG;
    if (((uintptr_t)x & 7) || ((uintptr_t)logw & 7) || ((uintptr_t)info & 7) ||
        ((uintptr_t)est & 7))
        return SMC_E_ARG;
    if ((uint64_t)ctx->t + (uint64_t)nsteps > 0xFFFFFFFFull) return SMC_E_ARG;
    if (ctx->cfg.target == SMC_TARGET_BEARING &&
        (int64_t)ctx->t + nsteps > (int64_t)ctx->cfg.n_obs)
        return SMC_E_ARG;  // not enough measurements left
    const uint32_t t0 = ctx->t + 1;
    const int par0 = ctx->par;
    ctx->t += (uint32_t)nsteps;
    ctx->par ^= nsteps & 1;
    const smc_status st = step_run_n(ctx->cfg, ctx->w, ctx->K, par0, t0, nsteps,
                                     reinterpret_cast<double *>(x), logw, info, est, S(stream));
    ctx->pending = false;
    return st;
}

smc_status smc_sync_weights(smc_ctx *ctx, double *logw, void *stream)
{
    if (!ctx || !logw || ctx->cfg.target == SMC_TARGET_NONE || ((uintptr_t)logw & 7))
        return SMC_E_ARG;
    return step_sync_weights(ctx->cfg, ctx->w, logw, S(stream));
}

smc_status smc_log_target(smc_ctx *ctx, const double *x, int64_t n, double *lp, void *stream)
{
    if (!ctx || !x || !lp || n < 1 || ctx->cfg.target == SMC_TARGET_NONE ||
        ctx->cfg.target == SMC_TARGET_BEARING)
        return SMC_E_ARG;
    return step_log_target(ctx->cfg, ctx->w, x, n, lp, S(stream));
}

smc_status smc_sync_error(smc_ctx *ctx, void *stream)
{
    if (!ctx) return SMC_E_ARG;
    if (hipStreamSynchronize(S(stream)) != hipSuccess) return SMC_E_DEVICE;
    unsigned err = 0;
    if (hipMemcpy(&err, &ctx->w.ctrl->err_latch, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess)
        return SMC_E_DEVICE;
    if (err) {
        const unsigned zero = 0;
        if (hipMemcpy(&ctx->w.ctrl->err_latch, &zero, sizeof(zero), hipMemcpyHostToDevice) !=
            hipSuccess)
            return SMC_E_DEVICE;
    }
    return (smc_status)err;
}

smc_status smc_destroy(smc_ctx *ctx)
{
    delete ctx;
    return SMC_OK;
}

}  // extern "C"
