"""Python face of libsmc: argument marshalling over the C ABI.

Every step of the computation runs in the HIP kernels of libsmc; this module
only checks tensors, hands device pointers and torch's current HIP stream to
the library, and decodes the small device-side info block.
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import _lib as L


# Normalising constants of the targets (log of the constant factor of each
# density), the defaults of Sampler and Batch.attach; a caller may pass its own.
def q0_log_norm(d: int, init_sd: float) -> float:
    """log of (2 pi init_sd^2)^(-d/2): x0 ~ N(init_mean, init_sd^2 I)."""
    return -0.5 * d * math.log(2.0 * math.pi * init_sd * init_sd)


def gauss_log_norm(var) -> float:
    """Diagonal Gaussian with variances `var`: -(d log 2 pi + sum log var) / 2."""
    v = [float(a) for a in torch.as_tensor(var, dtype=torch.float64).reshape(-1)]
    return -0.5 * (len(v) * math.log(2.0 * math.pi) + sum(math.log(a) for a in v))


def student_log_norm(nu: float) -> float:
    """Student-t with nu degrees of freedom, unit scale."""
    return math.lgamma(0.5 * (nu + 1.0)) - math.lgamma(0.5 * nu) - 0.5 * math.log(nu * math.pi)


def logreg_log_norm(d: int, prior_var: float) -> float:
    """The logistic regression's N(0, prior_var I) prior on the d weights."""
    return -0.5 * d * math.log(2.0 * math.pi * prior_var)


def bearing_obs_log_norm(obs_var: float) -> float:
    """The bearing-only model's N(0, obs_var) observation noise."""
    return -0.5 * math.log(2.0 * math.pi * obs_var)


def chol_log_norm(U) -> float:
    """Gaussian with precision U^T U (U upper triangular): -(d/2) log 2 pi + sum log U_ii."""
    Ut = torch.as_tensor(U, dtype=torch.float64)
    d = Ut.shape[0]
    return -0.5 * d * math.log(2.0 * math.pi) + float(torch.log(torch.diagonal(Ut)).sum())


def _stream():
    # torch's current HIP stream; the raw getter skips building a Stream
    # object (about 0.3 instead of 4 us a call)
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        return C.c_void_p(raw(torch.cuda.current_device()))
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, dtype, n=None, name="tensor"):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if n is not None and t.shape[0] != n:
        raise ValueError("%s must have %d rows, got %d" % (name, n, t.shape[0]))


def decode_info(buf: torch.Tensor) -> dict:
    """Copies a device info block back and decodes it (synchronises)."""
    raw = bytes(buf.cpu().numpy().tobytes())
    info = L.SmcInfo.from_buffer_copy(raw[:L.INFO_BYTES])
    return {f: getattr(info, f) for f, _ in L.SmcInfo._fields_ if f != "pad"}


class Resampler:
    """Resample + redistribute for N particles (Alg 4 with Alg 5 semantics).

    ``resample(logw, r)`` -> ncopies (optional); ``redistribute(x)`` -> x_new.
    The workspace (about 8 N bytes) is a torch allocation owned here.
    """

    def __init__(self, n: int, *, ess_num: int = 1, ess_den: int = 2, device=None):
        lib = L.load()
        self.n = int(n)
        self.device = torch.device(device or "cuda")
        cfg = L.SmcConfig()
        cfg.n, cfg.d, cfg.x_dtype, cfg.target = self.n, 1, L.DTYPE_F32, L.TARGET_NONE
        cfg.ess_num, cfg.ess_den, cfg.mode = ess_num, ess_den, L.MODE_AUTO
        self.ws_bytes = lib.smc_workspace_bytes(C.byref(cfg))
        if self.ws_bytes == 0:
            raise L.SmcError(L.SMC_E_ARG, "smc_workspace_bytes")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.info_buf = torch.zeros(L.INFO_BYTES, dtype=torch.uint8, device=self.device)
        self.ctx = C.c_void_p()
        L.check(lib.smc_init(C.byref(self.ctx), C.byref(cfg), _ptr(self.ws), self.ws_bytes,
                             None, None, _stream()), "smc_init")
        self._lib = lib

    def __del__(self):
        # the handle is dropped, not reset: module globals may already be gone
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self._lib.smc_destroy(ctx)
            self.ctx = None

    def resample(self, logw: torch.Tensor, r: int, mode: int = L.MODE_AUTO,
                 ncopies: torch.Tensor | None = None, info: bool = True):
        _need(logw, torch.float64, self.n, "logw")
        if ncopies is not None:
            _need(ncopies, torch.int64, self.n, "ncopies")
        L.check(self._lib.smc_resample(self.ctx, _ptr(logw), self.n, int(r) & (2**64 - 1), mode,
                                       _ptr(ncopies), _ptr(self.info_buf) if info else None,
                                       _stream()), "smc_resample")
        return ncopies

    def normalised_weights(self, logw: torch.Tensor,
                           out: torch.Tensor | None = None) -> torch.Tensor:
        """eq. normalise, exp(l_i - m) / Z with m and Z of the last resample()
        (call it with the same logw)."""
        _need(logw, torch.float64, self.n, "logw")
        if out is None:
            out = torch.empty_like(logw)
        _need(out, torch.float64, self.n, "out")
        L.check(self._lib.smc_normalised_weights(self.ctx, _ptr(logw), self.n, _ptr(out),
                                                 _stream()), "smc_normalised_weights")
        return out

    def redistribute(self, x: torch.Tensor, x_out: torch.Tensor | None = None,
                     ncopies: torch.Tensor | None = None,
                     ncopies_out: torch.Tensor | None = None,
                     anc: torch.Tensor | None = None) -> torch.Tensor:
        if not x.is_cuda or not x.is_contiguous() or x.shape[0] != self.n:
            raise ValueError("x must be a contiguous device tensor with N rows")
        if x_out is None:
            x_out = torch.empty_like(x)
        elif x_out.shape != x.shape or x_out.dtype != x.dtype or not x_out.is_contiguous():
            raise ValueError("x_out must match x")
        row_bytes = x.numel() * x.element_size() // self.n
        for t, nm in ((ncopies, "ncopies"), (ncopies_out, "ncopies_out"), (anc, "anc")):
            if t is not None:
                _need(t, torch.int64, self.n, nm)
        L.check(self._lib.smc_redistribute(self.ctx, _ptr(ncopies), _ptr(x), _ptr(x_out), self.n,
                                           row_bytes, _ptr(ncopies_out), _ptr(anc), _stream()),
                "smc_redistribute")
        return x_out

    def info(self) -> dict:
        return decode_info(self.info_buf)

    def sync_error(self) -> int:
        return self._lib.smc_sync_error(self.ctx, _stream())


_RESAMPLERS: dict = {}


def _resampler(n: int, device) -> Resampler:
    """The Resampler kept for (N, device); module-level calls share it, so a
    redistribute() without counts follows the last resample() of that N.  Its
    workspace is shared too: module-level calls of one N on one device must
    not overlap on different streams (use a Resampler each instead)."""
    dev = torch.device(device)
    key = (int(n), dev.type, dev.index if dev.index is not None else torch.cuda.current_device())
    rs = _RESAMPLERS.get(key)
    if rs is None:
        rs = _RESAMPLERS[key] = Resampler(n, device=dev)
    return rs


def release() -> None:
    """Drops the contexts (and workspaces) kept by the module-level calls."""
    _RESAMPLERS.clear()


def resample(logw: torch.Tensor, r: int, mode: int = L.MODE_AUTO,
             ncopies: torch.Tensor | None = None) -> torch.Tensor:
    """Alg 4 on the log-weights ``logw`` (float64 [N], device) with the
    systematic offset ``r`` (a 64-bit integer, U = floor(r S / 2^64)); returns
    the copy counts (int64 [N], allocated when not given).  When the ESS rule
    (``mode``) decides not to resample, every count is one."""
    rs = _resampler(logw.shape[0], logw.device)
    if ncopies is None:
        ncopies = torch.empty(rs.n, dtype=torch.int64, device=logw.device)
    return rs.resample(logw, r, mode, ncopies=ncopies, info=False)


def resample_noalloc(logw: torch.Tensor, r: int, ncopies: torch.Tensor,
                     mode: int = L.MODE_AUTO, info: torch.Tensor | None = None,
                     ess_num: int = 1, ess_den: int = 2) -> torch.Tensor:
    """``resample`` through smc_resample_noalloc: no context, no workspace and
    no allocation in the library (N <= 2^20; the caller passes ``ncopies``
    and, optionally, a uint8 device buffer ``info`` of INFO_BYTES)."""
    n = logw.shape[0]
    _need(logw, torch.float64, n, "logw")
    _need(ncopies, torch.int64, n, "ncopies")
    if info is not None:
        _need(info, torch.uint8, L.INFO_BYTES, "info")
    L.check(L.load().smc_resample_noalloc(_ptr(logw), n, int(r) & (2**64 - 1), mode, ess_num,
                                          ess_den, _ptr(ncopies), _ptr(info), _stream()),
            "smc_resample_noalloc")
    return ncopies


def redistribute(x: torch.Tensor, ncopies: torch.Tensor | None = None,
                 x_out: torch.Tensor | None = None) -> torch.Tensor:
    """Alg 5 semantics on the rows of ``x`` ([N][...], contiguous, device):
    returns the new population (row p is a copy of row anc(p), ancestors in
    non-decreasing order, source j copied ncopies_j times).  Without
    ``ncopies`` the counts of the last ``resample`` on N rows on this device
    are used."""
    return _resampler(x.shape[0], x.device).redistribute(x, x_out=x_out, ncopies=ncopies)


class Sampler:
    """One SMC sampler (Alg 2) driven through smc_init / smc_step.

    Particles x [N][d] and log-weights logw [N] are FP64 device tensors owned
    here; every step runs the library's kernels in place on them.
    Targets: "gauss" (mean, var), "student" (nu, mu; d = 1), "logreg"
    (X [M][d], y [M], prior_var; precision "f64" or "bf16"), and "bearing",
    the SIR particle filter of Alg 1 (mean = X0 mean, obs = bearings, delta,
    obs_var; d = 4).
    """

    def __init__(self, n: int, d: int, target: str, *, seed: int = 0, sampler_id: int = 0,
                 rw_sd: float = 0.5, init_mean: float = 0.0, init_sd: float = 3.0,
                 mode: int = L.MODE_AUTO, ess_num: int = 1, ess_den: int = 2, mean=None,
                 var=None, nu=None, mu=None, X=None, y=None, prior_var=None,
                 precision: str = "f64", log_norm=None, init_log_norm=None, obs=None,
                 delta: float = 1.0, obs_var: float = 1e-4, lazy_reset: bool = False,
                 device=None):
        lib = L.load()
        self._lib = lib
        self.n, self.d = int(n), int(d)
        self.device = torch.device(device or "cuda")
        dev = self.device
        cfg = L.SmcConfig()
        cfg.lazy_reset = 1 if lazy_reset else 0
        cfg.n, cfg.d, cfg.x_dtype = self.n, self.d, L.DTYPE_F64
        cfg.mode, cfg.ess_num, cfg.ess_den = mode, ess_num, ess_den
        cfg.sampler_id, cfg.seed = sampler_id, int(seed) & (2**64 - 1)
        cfg.rw_sd, cfg.init_mean, cfg.init_sd = rw_sd, init_mean, init_sd
        cfg.init_log_norm = (init_log_norm if init_log_norm is not None
                             else q0_log_norm(d, init_sd))
        self._keep = []
        if target == "gauss":
            cfg.target = L.TARGET_GAUSS
            m = torch.as_tensor(mean, dtype=torch.float64).reshape(-1).to(dev)
            v = torch.as_tensor(var, dtype=torch.float64).reshape(-1)
            pr = (1.0 / v).to(dev)
            self._keep += [m, pr]
            cfg.mean, cfg.prec = m.data_ptr(), pr.data_ptr()
            cfg.log_norm = log_norm if log_norm is not None else gauss_log_norm(v)
        elif target == "student":
            cfg.target = L.TARGET_STUDENT
            cfg.nu, cfg.mu = nu, mu
            cfg.log_norm = log_norm if log_norm is not None else student_log_norm(nu)
        elif target == "logreg":
            cfg.target = L.TARGET_LOGREG
            Xd = torch.as_tensor(X, dtype=torch.float64).contiguous().to(dev)
            yd = torch.as_tensor(y, dtype=torch.float64).contiguous().to(dev)
            self._keep += [Xd, yd]
            cfg.m_rows, cfg.X, cfg.y = Xd.shape[0], Xd.data_ptr(), yd.data_ptr()
            cfg.prior_prec = 1.0 / prior_var
            cfg.loglik_precision = L.PREC_BF16 if precision == "bf16" else L.PREC_F64
            cfg.log_norm = log_norm if log_norm is not None else logreg_log_norm(d, prior_var)
        elif target == "bearing":
            # SIR particle filter (Alg 1): mean = X0 mean [4], obs = bearings
            if d != 4:
                raise ValueError("the bearing-only model has d = 4")
            cfg.target = L.TARGET_BEARING
            m = torch.as_tensor(mean, dtype=torch.float64).reshape(-1).to(dev)
            ob = torch.as_tensor(obs, dtype=torch.float64).reshape(-1).to(dev)
            self._keep += [m, ob]
            cfg.mean, cfg.obs, cfg.n_obs = m.data_ptr(), ob.data_ptr(), ob.numel()
            cfg.delta, cfg.obs_var = delta, obs_var
            cfg.obs_log_norm = (log_norm if log_norm is not None
                                else bearing_obs_log_norm(obs_var))
        else:
            raise ValueError("unknown target %r" % target)
        self.cfg = cfg
        self.ws_bytes = lib.smc_workspace_bytes(C.byref(cfg))
        if self.ws_bytes == 0:
            raise L.SmcError(L.SMC_E_ARG, "smc_workspace_bytes")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.x = torch.empty((self.n, self.d), dtype=torch.float64, device=dev)
        self.logw = torch.empty(self.n, dtype=torch.float64, device=dev)
        self.info_buf = torch.zeros(L.INFO_BYTES, dtype=torch.uint8, device=dev)
        self.est = torch.zeros(4 * self.d, dtype=torch.float64, device=dev)
        self.ctx = C.c_void_p()
        L.check(lib.smc_init(C.byref(self.ctx), C.byref(cfg), _ptr(self.ws), self.ws_bytes,
                             _ptr(self.x), _ptr(self.logw), _stream()), "smc_init")
        self.t = 0

    def __del__(self):
        # the handle is dropped, not reset: module globals may already be gone
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self._lib.smc_destroy(ctx)
            self.ctx = None

    def step(self, info: bool = True, est: bool = True) -> None:
        L.check(self._lib.smc_step(self.ctx, _ptr(self.x), _ptr(self.logw),
                                   _ptr(self.info_buf) if info else None,
                                   _ptr(self.est) if est else None, _stream()), "smc_step")
        self.t += 1

    def steps(self, k: int, info: bool = False, est: bool = False) -> dict:
        """k iterations in one call (smc_steps).  With info / est, returns the
        per-iteration records (decoded info dicts; a [k, 4d] estimate tensor);
        the last also lands where info() and estimates() read."""
        k = int(k)
        dev = self.x.device
        ib = torch.zeros(k * L.INFO_BYTES, dtype=torch.uint8, device=dev) if info else None
        eb = torch.zeros(k * 4 * self.d, dtype=torch.float64, device=dev) if est else None
        L.check(self._lib.smc_steps(self.ctx, _ptr(self.x), _ptr(self.logw), k,
                                    _ptr(ib) if info else None, _ptr(eb) if est else None,
                                    _stream()), "smc_steps")
        self.t += k
        out = {}
        if info:
            self.info_buf.copy_(ib[(k - 1) * L.INFO_BYTES:])
            out["info"] = [decode_info(ib[i * L.INFO_BYTES:(i + 1) * L.INFO_BYTES])
                           for i in range(k)]
        if est:
            self.est.copy_(eb[(k - 1) * 4 * self.d:])
            out["est"] = eb.view(k, 4 * self.d)
        return out

    def sync_weights(self) -> None:
        """With lazy_reset: writes the pending -ln N of a resampling iteration
        into logw (smc_sync_weights; nothing to do otherwise)."""
        L.check(self._lib.smc_sync_weights(self.ctx, _ptr(self.logw), _stream()),
                "smc_sync_weights")

    def info(self) -> dict:
        return decode_info(self.info_buf)

    def estimates(self) -> dict:
        e = self.est.cpu().numpy()
        d = self.d
        return {"mean": e[:d], "m2": e[d:2 * d], "rec_mean": e[2 * d:3 * d],
                "rec_m2": e[3 * d:4 * d]}

    def log_target(self, x: torch.Tensor) -> torch.Tensor:
        _need(x, torch.float64, None, "x")
        lp = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
        L.check(self._lib.smc_log_target(self.ctx, _ptr(x), x.shape[0], _ptr(lp), _stream()),
                "smc_log_target")
        return lp

    def sync_error(self) -> int:
        return self._lib.smc_sync_error(self.ctx, _stream())


def _aligned(nbytes: int, device) -> tuple:
    """A uint8 device buffer and its first 256-byte aligned address."""
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    return buf, (buf.data_ptr() + 255) & ~255


class Batch:
    """Many independent samplers advanced by one sequence of launches
    (include/smc_batch.h): Gaussian targets with precision U^T U, each
    sampler of its own size N and dimension d <= 64.

    ``attach(slot, ...)`` allocates the sampler's particles and workspace as
    torch tensors and initialises it; ``step()`` advances every attached
    sampler one iteration; ``detach(slot)`` frees the slot.  A sampler's
    results depend only on its own arguments, not on the rest of the batch.
    """

    def __init__(self, capacity: int, *, graph: bool = True, device=None):
        lib = L.load()
        self._lib = lib
        self.capacity = int(capacity)
        self.device = torch.device(device or "cuda")
        nb = lib.smc_batch_workspace_bytes(self.capacity)
        if nb == 0:
            raise L.SmcError(L.SMC_E_ARG, "smc_batch_workspace_bytes")
        self._ws, ws = _aligned(nb, self.device)
        self.info_buf = torch.zeros(self.capacity * L.INFO_BYTES, dtype=torch.uint8,
                                    device=self.device)
        self.est = torch.zeros(self.capacity * L.BATCH_EST_STRIDE, dtype=torch.float64,
                               device=self.device)
        self.h = C.c_void_p()
        L.check(lib.smc_batch_create(C.byref(self.h), self.capacity, C.c_void_p(ws), nb,
                                     _stream()), "smc_batch_create")
        L.check(lib.smc_batch_set_graph(self.h, 1 if graph else 0), "smc_batch_set_graph")
        self.slots = {}

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self._lib.smc_batch_destroy(h)
            self.h = None

    def attach(self, slot: int, n: int, d: int, mean, chol, *, seed: int = 0,
               sampler_id: int = 0, rw_sd: float = 0.5, init_mean: float = 0.0,
               init_sd: float = 3.0, mode: int = L.MODE_AUTO, ess_num: int = 1,
               ess_den: int = 2, log_norm=None, init_log_norm=None, logw=None) -> None:
        """logw: optionally the caller's own float64 [n] device tensor for the
        log-weights (any 8-byte aligned view); allocated here otherwise."""
        dev = self.device
        n, d = int(n), int(d)
        m = torch.as_tensor(mean, dtype=torch.float64).reshape(-1).contiguous()
        U = torch.as_tensor(chol, dtype=torch.float64).reshape(d, d).contiguous()
        if m.numel() != d:
            raise ValueError("mean must have d entries")
        desc = L.SmcBatchSampler()
        desc.n, desc.d, desc.mode = n, d, mode
        desc.ess_num, desc.ess_den = ess_num, ess_den
        desc.sampler_id, desc.seed = sampler_id, int(seed) & (2**64 - 1)
        desc.rw_sd, desc.init_mean, desc.init_sd = rw_sd, init_mean, init_sd
        desc.init_log_norm = (init_log_norm if init_log_norm is not None
                              else q0_log_norm(d, init_sd))
        desc.log_norm = log_norm if log_norm is not None else chol_log_norm(U)
        md, Ud = m.to(dev), U.to(dev)
        x = torch.empty((n, d), dtype=torch.float64, device=dev)
        if logw is None:
            logw = torch.empty(n, dtype=torch.float64, device=dev)
        else:
            _need(logw, torch.float64, n, "logw")
        desc.mean, desc.chol = md.data_ptr(), Ud.data_ptr()
        desc.x, desc.logw = x.data_ptr(), logw.data_ptr()
        nb = self._lib.smc_batch_sampler_bytes(C.byref(desc))
        if nb == 0:
            raise L.SmcError(L.SMC_E_ARG, "smc_batch_sampler_bytes")
        wsb, ws = _aligned(nb, dev)
        desc.ws, desc.ws_bytes = ws, nb
        L.check(self._lib.smc_batch_attach(self.h, int(slot), C.byref(desc), _stream()),
                "smc_batch_attach")
        self.slots[int(slot)] = {"n": n, "d": d, "x": x, "logw": logw, "ws": wsb,
                                 "mean": md, "chol": Ud, "desc": desc}

    def detach(self, slot: int) -> None:
        L.check(self._lib.smc_batch_detach(self.h, int(slot), _stream()), "smc_batch_detach")
        self.slots.pop(int(slot))

    def step(self, info: bool = True, est: bool = True) -> None:
        L.check(self._lib.smc_batch_step(self.h, _ptr(self.info_buf) if info else None,
                                         _ptr(self.est) if est else None, _stream()),
                "smc_batch_step")

    def set_group(self, pairs: int) -> None:
        L.check(self._lib.smc_batch_set_group(self.h, int(pairs), _stream()),
                "smc_batch_set_group")

    def set_bucket_waves(self, bucket: int, waves: int) -> None:
        """Occupancy aim (1-4 waves per SIMD) of the target kernel for samplers
        with d in (8 bucket, 8 bucket + 8]; speed only."""
        L.check(self._lib.smc_batch_set_bucket_waves(self.h, int(bucket), int(waves)),
                "smc_batch_set_bucket_waves")

    def set_graph(self, enable: bool) -> None:
        L.check(self._lib.smc_batch_set_graph(self.h, 1 if enable else 0), "smc_batch_set_graph")

    def counts(self) -> tuple:
        ns, nt = C.c_int32(), C.c_int64()
        L.check(self._lib.smc_batch_counts(self.h, C.byref(ns), C.byref(nt)), "smc_batch_counts")
        return ns.value, nt.value

    def x(self, slot: int) -> torch.Tensor:
        """The slot's current particles [N][d] (waits for the stream): the
        attach-time array or the workspace copy, which alternate."""
        e = self.slots[int(slot)]
        px = C.c_void_p()
        L.check(self._lib.smc_batch_particles(self.h, int(slot), C.byref(px), None, _stream()),
                "smc_batch_particles")
        if px.value == e["x"].data_ptr():
            return e["x"]
        off = px.value - e["ws"].data_ptr()
        nb = 8 * e["n"] * e["d"]
        return e["ws"][off:off + nb].view(torch.float64).view(e["n"], e["d"])

    def logw(self, slot: int) -> torch.Tensor:
        return self.slots[int(slot)]["logw"]

    def info(self, slot: int) -> dict:
        o = int(slot) * L.INFO_BYTES
        return decode_info(self.info_buf[o:o + L.INFO_BYTES])

    def estimates(self, slot: int) -> dict:
        d = self.slots[int(slot)]["d"]
        o = int(slot) * L.BATCH_EST_STRIDE
        e = self.est[o:o + 4 * d].cpu().numpy()
        return {"mean": e[:d], "m2": e[d:2 * d], "rec_mean": e[2 * d:3 * d],
                "rec_m2": e[3 * d:4 * d]}

    def sync_error(self, slot: int) -> int:
        return self._lib.smc_batch_sync_error(self.h, int(slot), _stream())
