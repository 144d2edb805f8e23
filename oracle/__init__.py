"""ctypes shim over the plain FP64 CPU oracle (``smc_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product package never does.
It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODE_AUTO, MODE_FORCE, MODE_NEVER = 0, 1, 2
E_OK, E_ARG, E_NONFINITE, E_DEGENERATE = 0, 1, 2, 3
T_GAUSS, T_STUDENT, T_LOGREG, T_GAUSS_CHOL = 1, 2, 3, 5
TAG_INIT, TAG_PROPOSE, TAG_RESAMPLE = 1, 2, 3
DMAX = 64


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
            "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class ResampleInfo(C.Structure):
    _fields_ = [("m", C.c_double), ("logZ", C.c_double), ("ess", C.c_double),
                ("Z", C.c_double), ("Z2", C.c_double),
                ("S", C.c_uint64), ("U", C.c_uint64), ("Q2_hi", C.c_uint64), ("Q2_lo", C.c_uint64),
                ("K", C.c_int32), ("resampled", C.c_int32), ("err", C.c_int32), ("pad", C.c_int32),
                ("unique", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class SmcCfg(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("target", C.c_int32), ("mode", C.c_int32),
                ("ess_num", C.c_int32), ("ess_den", C.c_int32), ("sampler_id", C.c_uint32),
                ("seed", C.c_uint64), ("rw_sd", C.c_double),
                ("init_mean", C.c_double), ("init_sd", C.c_double), ("init_log_norm", C.c_double),
                ("log_norm", C.c_double),
                ("mean", C.POINTER(C.c_double)), ("prec", C.POINTER(C.c_double)),
                ("nu", C.c_double), ("mu", C.c_double),
                ("m_rows", C.c_int64), ("X", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
                ("prior_prec", C.c_double), ("chol", C.POINTER(C.c_double))]


class Recycle(C.Structure):
    _fields_ = [("logZ_prev", C.c_double), ("lc_max", C.c_double), ("den", C.c_double),
                ("num", C.c_double * (2 * DMAX)), ("steps", C.c_int32), ("pad", C.c_int32)]


class StepOut(C.Structure):
    _fields_ = [("info", ResampleInfo), ("log_c", C.c_double),
                ("est", C.c_double * (2 * DMAX)), ("rec", C.c_double * (2 * DMAX))]


class PfCfg(C.Structure):
    _fields_ = [("n", C.c_int64), ("mode", C.c_int32), ("ess_num", C.c_int32),
                ("ess_den", C.c_int32), ("sampler_id", C.c_uint32), ("seed", C.c_uint64),
                ("delta", C.c_double), ("obs_var", C.c_double), ("obs_log_norm", C.c_double),
                ("init_mean", C.c_double * 4), ("init_sd", C.c_double),
                ("y", C.POINTER(C.c_double)), ("T", C.c_int32), ("pad", C.c_int32)]


class PfOut(C.Structure):
    _fields_ = [("info", ResampleInfo), ("log_c", C.c_double), ("mean", C.c_double * 4),
                ("m2", C.c_double * 4)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P = C.POINTER
        L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.orc_det_exp.argtypes = [C.c_double]
        L.orc_det_exp.restype = C.c_double
        L.orc_det_log.argtypes = [C.c_double]
        L.orc_det_log.restype = C.c_double
        L.orc_det_atan.argtypes = [C.c_double]
        L.orc_det_atan.restype = C.c_double
        L.orc_pf_init.argtypes = [P(PfCfg), P(C.c_double), P(C.c_double), P(C.c_double)]
        L.orc_pf_init.restype = C.c_int
        L.orc_pf_step.argtypes = [P(PfCfg), C.c_uint32, P(C.c_double), P(C.c_double),
                                  P(C.c_double), P(PfOut)]
        L.orc_pf_step.restype = C.c_int
        L.orc_pf_loglik.argtypes = [P(PfCfg), P(C.c_double), C.c_double]
        L.orc_pf_loglik.restype = C.c_double
        L.orc_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                  C.c_int32, P(C.c_double)]
        L.orc_resample_draw.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32]
        L.orc_resample_draw.restype = C.c_uint64
        L.orc_quant_bits.argtypes = [C.c_int64]
        L.orc_quant_bits.restype = C.c_int32
        L.orc_quantise.argtypes = [P(C.c_double), C.c_int64, C.c_int32, C.c_double, P(C.c_uint64)]
        L.orc_systematic_ncopies.argtypes = [P(C.c_uint64), C.c_int64, C.c_uint64, P(C.c_int64)]
        L.orc_systematic_ncopies.restype = C.c_int
        L.orc_resample.argtypes = [P(C.c_double), C.c_int64, C.c_uint64, C.c_int32, C.c_int32,
                                   C.c_int32, P(C.c_int64), P(ResampleInfo)]
        L.orc_resample.restype = C.c_int
        L.orc_redistribute.argtypes = [C.c_int64, P(C.c_int64), C.c_void_p, C.c_int64, C.c_void_p,
                                       P(C.c_int64)]
        L.orc_normalised_weights.argtypes = [P(C.c_double), C.c_int64, P(C.c_double)]
        L.orc_normalised_weights.restype = C.c_int
        L.orc_redistribute.restype = C.c_int
        L.orc_log_target_batch.argtypes = [P(SmcCfg), P(C.c_double), C.c_int64, P(C.c_double)]
        L.orc_smc_init.argtypes = [P(SmcCfg), P(C.c_double), P(C.c_double), P(C.c_double),
                                   P(Recycle)]
        L.orc_smc_init.restype = C.c_int
        L.orc_smc_step.argtypes = [P(SmcCfg), C.c_uint32, P(C.c_double), P(C.c_double),
                                   P(C.c_double), P(Recycle), P(StepOut)]
        L.orc_smc_step.restype = C.c_int
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


# ---------------------------------------------------------------- primitives
def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def det_exp(x: float) -> float:
    return lib().orc_det_exp(float(x))


def det_log(x: float) -> float:
    return lib().orc_det_log(float(x))


def det_atan(x: float) -> float:
    return lib().orc_det_atan(float(x))


def normals(seed, tag, sampler_id, t, idx, d):
    z = np.zeros(max(d, 1), dtype=np.float64)
    lib().orc_normals(seed, tag, sampler_id, t, idx, d, _p(z, C.c_double))
    return z[:d]


def resample_draw(seed, sampler_id, t):
    return int(lib().orc_resample_draw(seed, sampler_id, t))


def quant_bits(n: int) -> int:
    return int(lib().orc_quant_bits(n))


def quantise(logw, K, m):
    lw = np.ascontiguousarray(logw, dtype=np.float64)
    q = np.zeros(lw.size, dtype=np.uint64)
    lib().orc_quantise(_p(lw, C.c_double), lw.size, K, float(m), _p(q, C.c_uint64))
    return q


def systematic_ncopies(q, U):
    qq = np.ascontiguousarray(q, dtype=np.uint64)
    nc = np.zeros(qq.size, dtype=np.int64)
    rc = lib().orc_systematic_ncopies(_p(qq, C.c_uint64), qq.size, int(U), _p(nc, C.c_int64))
    if rc != E_OK:
        raise ValueError("systematic_ncopies: bad arguments")
    return nc


def resample(logw, r, mode=MODE_AUTO, ess_num=1, ess_den=2):
    """Alg 4 up to ncopies.  Returns (ncopies, info dict)."""
    lw = np.ascontiguousarray(logw, dtype=np.float64)
    nc = np.zeros(max(lw.size, 1), dtype=np.int64)
    info = ResampleInfo()
    lib().orc_resample(_p(lw, C.c_double), lw.size, int(r) & (2**64 - 1), mode, ess_num,
                       ess_den, _p(nc, C.c_int64), C.byref(info))
    return nc[:lw.size], info.as_dict()


def normalised_weights(logw):
    """eq. normalise: exp(l_i - m) / sum_j exp(l_j - m); raises on the
    resample errors (status in the message)."""
    lw = np.ascontiguousarray(logw, dtype=np.float64)
    w = np.zeros(lw.shape[0], dtype=np.float64)
    rc = lib().orc_normalised_weights(_p(lw, C.c_double), lw.shape[0], _p(w, C.c_double))
    if rc != E_OK:
        raise ValueError("normalised_weights failed: status %d" % rc)
    return w


def redistribute(ncopies, x):
    """Alg 5 (S-R) over the rows of x.  Returns (x_new, anc)."""
    nc = np.ascontiguousarray(ncopies, dtype=np.int64)
    xa = np.ascontiguousarray(x)
    n = nc.size
    row_bytes = xa.nbytes // max(n, 1)
    out = np.empty_like(xa)
    anc = np.zeros(max(n, 1), dtype=np.int64)
    rc = lib().orc_redistribute(n, _p(nc, C.c_int64), xa.ctypes.data, row_bytes,
                                out.ctypes.data, _p(anc, C.c_int64))
    if rc != E_OK:
        raise ValueError("redistribute: ncopies must be >= 0 and sum to N")
    return out, anc[:n]


# ------------------------------------------------------------------ sampler
class Sampler:
    """Alg 2 driven step by step on host arrays (x [N][d], logw, lp)."""

    def __init__(self, n, d, target, *, seed=0, sampler_id=0, rw_sd=0.5, init_mean=0.0,
                 init_sd=3.0, mode=MODE_AUTO, ess_num=1, ess_den=2, mean=None, var=None,
                 nu=None, mu=None, X=None, y=None, prior_var=None, log_norm=None,
                 init_log_norm=None, chol=None):
        import math
        self.cfg = SmcCfg()
        c = self.cfg
        c.n, c.d, c.target, c.mode = n, d, target, mode
        c.ess_num, c.ess_den, c.sampler_id, c.seed = ess_num, ess_den, sampler_id, seed
        c.rw_sd, c.init_mean, c.init_sd = rw_sd, init_mean, init_sd
        c.init_log_norm = -0.5 * d * math.log(2.0 * math.pi * init_sd * init_sd)
        self._keep = []
        if target == T_GAUSS:
            mean = np.ascontiguousarray(mean, dtype=np.float64)
            var = np.ascontiguousarray(var, dtype=np.float64)
            prec = np.ascontiguousarray(1.0 / var)
            self._keep += [mean, prec]
            c.mean, c.prec = _p(mean, C.c_double), _p(prec, C.c_double)
            c.log_norm = gauss_log_norm(var)
        elif target == T_GAUSS_CHOL:
            mean = np.ascontiguousarray(mean, dtype=np.float64)
            U = np.ascontiguousarray(chol, dtype=np.float64)
            self._keep += [mean, U]
            c.mean, c.chol = _p(mean, C.c_double), _p(U, C.c_double)
            c.log_norm = gauss_chol_log_norm(U)
        elif target == T_STUDENT:
            c.nu, c.mu = nu, mu
            c.log_norm = student_log_norm(nu)
        elif target == T_LOGREG:
            Xa = np.ascontiguousarray(X, dtype=np.float64)
            ya = np.ascontiguousarray(y, dtype=np.float64)
            self._keep += [Xa, ya]
            c.m_rows, c.X, c.y = Xa.shape[0], _p(Xa, C.c_double), _p(ya, C.c_double)
            c.prior_prec = 1.0 / prior_var
            c.log_norm = -0.5 * d * math.log(2.0 * math.pi * prior_var)
        if log_norm is not None:
            c.log_norm = log_norm
        if init_log_norm is not None:
            c.init_log_norm = init_log_norm
        self.x = np.zeros((n, d), dtype=np.float64)
        self.logw = np.zeros(n, dtype=np.float64)
        self.lp = np.zeros(n, dtype=np.float64)
        self.rec = Recycle()
        self.t = 0

    def init(self):
        rc = lib().orc_smc_init(C.byref(self.cfg), _p(self.x, C.c_double),
                                _p(self.logw, C.c_double), _p(self.lp, C.c_double),
                                C.byref(self.rec))
        if rc != E_OK:
            raise ValueError("oracle init failed: %d" % rc)
        self.t = 0

    def step(self):
        self.t += 1
        out = StepOut()
        rc = lib().orc_smc_step(C.byref(self.cfg), self.t, _p(self.x, C.c_double),
                                _p(self.logw, C.c_double), _p(self.lp, C.c_double),
                                C.byref(self.rec), C.byref(out))
        if rc != E_OK:
            raise ValueError("oracle step failed: %d" % rc)
        d = self.cfg.d
        return {"info": out.info.as_dict(), "log_c": out.log_c,
                "mean": np.array(out.est[:d]), "m2": np.array(out.est[d:2 * d]),
                "rec_mean": np.array(out.rec[:d]), "rec_m2": np.array(out.rec[d:2 * d])}

    def log_target(self, x):
        xa = np.ascontiguousarray(x, dtype=np.float64)
        n = xa.shape[0]
        lp = np.zeros(n, dtype=np.float64)
        lib().orc_log_target_batch(C.byref(self.cfg), _p(xa, C.c_double), n, _p(lp, C.c_double))
        return lp


def gauss_chol_log_norm(U) -> float:
    """Additive constant of a Gaussian log-density with precision U^T U:
    -d/2 log(2 pi) + log det U (U triangular, so its diagonal)."""
    import math
    U = np.asarray(U, dtype=np.float64)
    d = U.shape[0]
    return -0.5 * d * math.log(2.0 * math.pi) + float(np.sum(np.log(np.diag(U))))


def gauss_log_norm(var) -> float:
    """Additive constant of a diagonal Gaussian log-density."""
    import math
    v = np.asarray(var, dtype=np.float64)
    return float(-0.5 * (v.size * math.log(2.0 * math.pi) + sum(math.log(float(a)) for a in v)))


def student_log_norm(nu: float) -> float:
    import math
    return math.lgamma(0.5 * (nu + 1.0)) - math.lgamma(0.5 * nu) - 0.5 * math.log(nu * math.pi)


class ParticleFilter:
    """Alg 1 (SIR) on the bearing-only tracking model, host arrays x [N][4]."""

    def __init__(self, n, y, *, seed=0, sampler_id=0, mode=MODE_AUTO, ess_num=1, ess_den=2,
                 delta=1.0, obs_var=1e-4, init_mean=(0.0, 0.0, 0.0, 0.0), init_sd=1.0,
                 obs_log_norm=None):
        import math
        self.y = np.ascontiguousarray(y, dtype=np.float64)
        c = self.cfg = PfCfg()
        c.n, c.mode, c.ess_num, c.ess_den = n, mode, ess_num, ess_den
        c.sampler_id, c.seed, c.delta, c.obs_var = sampler_id, seed, delta, obs_var
        c.obs_log_norm = (obs_log_norm if obs_log_norm is not None
                          else -0.5 * math.log(2.0 * math.pi * obs_var))
        for k in range(4):
            c.init_mean[k] = init_mean[k]
        c.init_sd, c.y, c.T = init_sd, _p(self.y, C.c_double), self.y.size
        self.x = np.zeros((n, 4), dtype=np.float64)
        self.logw = np.zeros(n, dtype=np.float64)
        self.logZ_prev = C.c_double(0.0)
        self.t = 0

    def init(self):
        if lib().orc_pf_init(C.byref(self.cfg), _p(self.x, C.c_double), _p(self.logw, C.c_double),
                             C.byref(self.logZ_prev)) != E_OK:
            raise ValueError("pf init failed")
        self.t = 0

    def step(self):
        self.t += 1
        out = PfOut()
        rc = lib().orc_pf_step(C.byref(self.cfg), self.t, _p(self.x, C.c_double),
                               _p(self.logw, C.c_double), C.byref(self.logZ_prev),
                               C.byref(out))
        if rc != E_OK:
            raise ValueError("pf step failed: %d" % rc)
        return {"info": out.info.as_dict(), "log_c": out.log_c, "mean": np.array(out.mean[:]),
                "m2": np.array(out.m2[:])}

    def loglik(self, x, y):
        xa = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc_pf_loglik(C.byref(self.cfg), _p(xa, C.c_double), float(y))
