"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only draws inputs (numpy PCG64 streams) and states workload
shapes; it holds none of the method's arithmetic.  The paper's own redistribute
and sorting experiments feed Gaussian random numbers through MVR (Sec. 5.1.1);
the workloads below follow that recipe at the sizes used here.
"""
from __future__ import annotations

import math

import numpy as np

# Resample + redistribute alone: N = 2^24 particles, d = 16 FP32 state,
# log-weights N(0, s^2) with s in {0.5, 2, 8}.
RESAMPLE_N = 1 << 24
RESAMPLE_D = 16
RESAMPLE_SCALES = (0.5, 2.0, 8.0)
LOGW_SEEDS = {0.5: 101, 2.0: 102, 8.0: 103}
X_SEED = 100
R_SEED = 7


def logw_normal(n: int, s: float, seed: int) -> np.ndarray:
    """Log-weights l_i = s * z_i, z_i iid N(0, 1), FP64."""
    rng = np.random.default_rng(seed)
    return s * rng.standard_normal(n)


def particles(n: int, d: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Particle rows [n][d], iid N(0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, d), dtype=np.float64 if dtype == np.float64 else np.float32
                               ).astype(dtype, copy=False)


# Largest N the library takes; its log-weights repeat a seeded pattern so the
# exact prefix of the fixed-point weights has a closed form at any index.
MAX_N = (1 << 31) - 1
MAX_PERIOD = 1000


def offset_word(seed: int) -> int:
    """One 64-bit word used as the systematic offset source."""
    rng = np.random.default_rng(seed)
    return int(rng.integers(0, 2**64, dtype=np.uint64))


# 1-D Gaussian target N(2, 1), q0 = N(0, 9), random walk sd 0.5, N = 1024,
# 20 iterations.
GAUSS1D = dict(n=1024, d=1, mean=[2.0], var=[1.0], init_mean=0.0, init_sd=3.0, rw_sd=0.5,
               iters=20)


def gauss_log_norm(var) -> float:
    """Additive constant -0.5 * sum log(2 pi var_k) of a diagonal Gaussian."""
    v = [float(a) for a in np.asarray(var, dtype=np.float64).ravel()]
    return float(-0.5 * (len(v) * math.log(2.0 * math.pi) + sum(math.log(a) for a in v)))


def iso_gauss_log_norm(d: int, sd: float) -> float:
    return float(-0.5 * d * math.log(2.0 * math.pi * sd * sd))


def student_log_norm(nu: float) -> float:
    return (math.lgamma(0.5 * (nu + 1.0)) - math.lgamma(0.5 * nu)
            - 0.5 * math.log(nu * math.pi))


# Bayesian logistic regression: M rows, D features iid N(0, 1) (rounded to
# bf16 at generation so both precisions read the same data), theta* ~ N(0, I),
# labels ~ Bernoulli(sigmoid(x . theta*)), prior N(0, 10 I).
LOGREG = dict(m_rows=65536, d=32, n=1 << 16, iters=50, prior_var=10.0, rw_sd=0.01)


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), as FP32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def logreg_data(m_rows: int, d: int, seed: int):
    rng = np.random.default_rng(seed)
    X = bf16_round(rng.standard_normal((m_rows, d), dtype=np.float32))
    theta = rng.standard_normal(d)
    z = X.astype(np.float64) @ theta
    p = 1.0 / (1.0 + np.exp(-z))
    y = (rng.random(m_rows) < p).astype(np.float64)
    return X, y, theta


# Bearing-only tracking (SIR particle filter): constant-velocity state
# [x, vx, y, vy], sampling period 1 s, process noise covariance per axis
# [[5/3, 5/2], [5/2, 5]], bearing noise variance 1e-4, X0 ~ N(true X0, I).
BEARING = dict(delta=1.0, obs_var=1e-4, x0=(10.0, -1.0, 10.0, 1.0), init_sd=1.0, T=100)


def bearing_track(T: int, seed: int, x0=BEARING["x0"], delta=BEARING["delta"],
                  obs_var=BEARING["obs_var"]):
    """Simulated true states [T+1][4] and bearings y[T] = arctan(x2/x0) + noise."""
    rng = np.random.default_rng(seed)
    A = np.array([[1, delta, 0, 0], [0, 1, 0, 0], [0, 0, 1, delta], [0, 0, 0, 1]], float)
    blk = np.array([[5 * delta**3 / 3, 5 * delta**2 / 2], [5 * delta**2 / 2, 5 * delta]])
    Q = np.zeros((4, 4))
    Q[:2, :2] = blk
    Q[2:, 2:] = blk
    L = np.linalg.cholesky(Q)
    xs = [np.asarray(x0, float)]
    ys = []
    for _ in range(T):
        xs.append(A @ xs[-1] + L @ rng.standard_normal(4))
        ys.append(np.arctan(xs[-1][2] / xs[-1][0]) + np.sqrt(obs_var) * rng.standard_normal())
    return np.array(xs), np.array(ys)


# Batched samplers: many independent Gaussian targets of uneven size and
# dimension.  N log-uniform in [2^8, 2^16], d uniform in 1..64, mean ~ N(0, I),
# covariance W / (d + 2) with W ~ Wishart(I, d + 2) (so its mean is I),
# q0 = N(0, 9 I), random-walk sd 0.5 / sqrt(d).
BATCH = dict(count=256, n_lo=1 << 8, n_hi=1 << 16, d_lo=1, d_hi=64, init_sd=3.0, seed=300,
             iters=20)


def wishart_target(d: int, rng: np.random.Generator):
    """Mean, upper-triangular U with precision U^T U, and the covariance."""
    g = rng.standard_normal((d + 2, d))
    cov = (g.T @ g) / (d + 2)
    prec = np.linalg.inv(cov)
    prec = 0.5 * (prec + prec.T)
    U = np.ascontiguousarray(np.linalg.cholesky(prec).T)
    mean = rng.standard_normal(d)
    return mean, U, cov


def batch_specs(count: int = BATCH["count"], seed: int = BATCH["seed"],
                n_lo: int = BATCH["n_lo"], n_hi: int = BATCH["n_hi"],
                d_lo: int = BATCH["d_lo"], d_hi: int = BATCH["d_hi"]) -> list:
    """Per-sampler sizes, targets, proposal scale and random-number keys."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        d = int(rng.integers(d_lo, d_hi + 1))
        mean, U, cov = wishart_target(d, rng)
        out.append(dict(n=n, d=d, mean=mean, chol=U, cov=cov, rw_sd=0.5 / math.sqrt(d),
                        seed=(seed << 32) + s, sampler_id=s, init_mean=0.0,
                        init_sd=BATCH["init_sd"]))
    return out



# Serving: a stream of sampler requests mixing the shapes above.  Gaussian
# requests (the 1-D workload's and the batched workload's kind) with N
# log-uniform in [2^10, 2^20] and d uniform in 1..64; logistic-regression
# requests with N log-uniform in [2^10, 2^16], D uniform in 8..64 and M rows
# log-uniform in [2^10, 2^16]; iterations uniform in 20..100; exponential
# inter-arrival gaps (a Poisson process) of mean 1 / rate.
SERVE = dict(requests=2000, seed=400, logreg_share=1.0 / 3.0, n_lo=1 << 10, n_hi=1 << 20,
             lr_n_hi=1 << 16, m_lo=1 << 10, m_hi=1 << 16, d_lr_lo=8, d_lr_hi=64, t_lo=20,
             t_hi=100)


def serve_requests(count: int, rate: float, seed: int = SERVE["seed"], scale: float = 1.0):
    """Request descriptions (dicts) in arrival order; ``scale`` shrinks every
    N and M (for quick runs)."""
    rng = np.random.default_rng(seed)
    c = SERVE
    out, t = [], 0.0
    for k in range(count):
        t += float(rng.exponential(1.0 / rate)) if rate > 0 else 0.0
        iters = int(rng.integers(c["t_lo"], c["t_hi"] + 1))
        if rng.uniform() < c["logreg_share"]:
            n = int(round(math.exp(rng.uniform(math.log(c["n_lo"]), math.log(c["lr_n_hi"])))))
            m = int(round(math.exp(rng.uniform(math.log(c["m_lo"]), math.log(c["m_hi"])))))
            d = int(rng.integers(c["d_lr_lo"], c["d_lr_hi"] + 1))
            n, m = max(64, int(n * scale)), max(64, int(m * scale))
            X, y, _ = logreg_data(m, d, int(rng.integers(0, 2**31)))
            out.append(dict(kind="logreg", n=n, d=d, iters=iters, arrival=t,
                            seed=(seed << 32) + k, sampler_id=k,
                            params=dict(X=X.astype(np.float64), y=y, prior_var=10.0,
                                        rw_sd=0.01)))
        else:
            n = int(round(math.exp(rng.uniform(math.log(c["n_lo"]), math.log(c["n_hi"])))))
            d = int(rng.integers(1, 65))
            n = max(1, int(n * scale))
            mean, U, _ = wishart_target(d, rng)
            out.append(dict(kind="gauss", n=n, d=d, iters=iters, arrival=t,
                            seed=(seed << 32) + k, sampler_id=k,
                            params=dict(mean=mean, chol=U, rw_sd=0.5 / math.sqrt(d),
                                        init_sd=3.0)))
    return out
