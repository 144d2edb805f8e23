"""GPU parity of smc_init / smc_step (Alg 2) against the CPU oracle.

For the cheap targets every operation on a particle is a fixed IEEE sequence
and resampling is integer-exact, so whole trajectories (particles and
log-weights) must match bit for bit; estimates, c_t and the recycled
estimate are FP64 sums in a different order (relative 1e-12).  For logistic
regression the likelihood is a long FP64 sum (GPU order differs: 1e-11
relative) or a BF16 MFMA contraction (1e-2 relative, per the stated
tolerance), so its parity is per step.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_1905_10252_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def smc(dev):
    from paper_1905_10252_amd import smc as S
    return S


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def assert_close(a, b, rtol, what):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    scale = np.maximum(np.abs(b), 1.0)
    err = np.max(np.abs(a - b) / scale) if a.size else 0.0
    assert err <= rtol, "%s: rel err %.3g > %.3g" % (what, err, rtol)


MODES = {"auto": O.MODE_AUTO, "force": O.MODE_FORCE, "never": O.MODE_NEVER}


def pair_gauss(smc, dev, n, mean, var, seed, mode, rw_sd=0.5, init_sd=3.0):
    d = len(mean)
    ln, iln = I.gauss_log_norm(var), I.iso_gauss_log_norm(d, init_sd)
    g = smc.Sampler(n, d, "gauss", seed=seed, rw_sd=rw_sd, init_mean=0.0, init_sd=init_sd,
                    mean=mean, var=var, mode=mode, log_norm=ln, init_log_norm=iln, device=dev)
    o = O.Sampler(n, d, O.T_GAUSS, seed=seed, rw_sd=rw_sd, init_mean=0.0, init_sd=init_sd,
                  mean=mean, var=var, mode=mode, log_norm=ln, init_log_norm=iln)
    o.init()
    return g, o


def run_and_compare(g, o, steps):
    assert np.array_equal(bits(g.x.cpu().numpy()), bits(o.x)), "x0"
    assert np.array_equal(bits(g.logw.cpu().numpy()), bits(o.logw)), "logw0"
    for t in range(1, steps + 1):
        g.step()
        out = o.step()
        info = g.info()
        oi = out["info"]
        for k in ("S", "U", "Q2_hi", "Q2_lo", "resampled", "K", "err"):
            assert info[k] == oi[k], (t, k, info[k], oi[k])
        assert info["m"] == oi["m"], t
        assert np.array_equal(bits(g.x.cpu().numpy()), bits(o.x)), "x at t=%d" % t
        assert np.array_equal(bits(g.logw.cpu().numpy()), bits(o.logw)), "logw at t=%d" % t
        assert_close(info["logZ"], oi["logZ"], 1e-12, "logZ t=%d" % t)
        assert_close(info["ess"], oi["ess"], 1e-12, "ess t=%d" % t)
        assert abs(info["log_c"] - out["log_c"]) <= 1e-11, ("log_c", t)
        e = g.estimates()
        for k in ("mean", "m2", "rec_mean", "rec_m2"):
            assert_close(e[k], out[k], 1e-11, "%s t=%d" % (k, t))
    assert g.sync_error() == 0


def test_gauss_1d_twenty_iterations_bit_exact(smc, dev):
    """N = 1024, target N(2, 1), q0 = N(0, 9), random walk sd 0.5."""
    g = I.GAUSS1D
    G, Or = pair_gauss(smc, dev, g["n"], g["mean"], g["var"], 0, O.MODE_AUTO)
    run_and_compare(G, Or, g["iters"])


@pytest.mark.parametrize("mode", ["auto", "force", "never"])
def test_gauss_3d_ragged(smc, dev, mode):
    _say("gauss 3d", mode)
    G, Or = pair_gauss(smc, dev, 3001, [1.0, -2.0, 0.5], [0.5, 2.0, 1.5], 17, MODES[mode],
                       rw_sd=0.3)
    run_and_compare(G, Or, 6)


@pytest.mark.parametrize("n", [1, 7, 1 << 10, 4096, 70001, 1 << 17])
def test_student_t(smc, dev, n):
    _say("student n=%d" % n)
    nu, mu = 5.0, 1.0
    ln, iln = I.student_log_norm(nu), I.iso_gauss_log_norm(1, 3.0)
    g = smc.Sampler(n, 1, "student", seed=5, rw_sd=0.5, nu=nu, mu=mu, mode=O.MODE_FORCE,
                    log_norm=ln, init_log_norm=iln, device=dev)
    o = O.Sampler(n, 1, O.T_STUDENT, seed=5, rw_sd=0.5, nu=nu, mu=mu, mode=O.MODE_FORCE,
                  log_norm=ln, init_log_norm=iln)
    o.init()
    run_and_compare(g, o, 5)


@pytest.mark.parametrize("n,mode", [(6000, "auto"), (6000, "force"), (6001, "never")])
def test_gauss_1d_multi_kernel(smc, dev, n, mode):
    """The 1-D Gaussian above one workgroup: even n moves each lane's two
    particles as 16-byte accesses, odd n takes 8-byte ones; both bit-exact."""
    _say("gauss 1d n=%d" % n, mode)
    G, Or = pair_gauss(smc, dev, n, [2.0], [1.0], 41, MODES[mode])
    run_and_compare(G, Or, 6)


@pytest.mark.parametrize("kind", ["student", "gauss"])
def test_one_dimensional_update_unaligned_arrays(smc, dev, kind):
    """x and logw handed to smc_step one element past a 16-byte boundary: the
    update takes its 8-byte accesses and the trajectory stays bit-exact."""
    import torch
    _say("unaligned", kind)
    n = 4096
    if kind == "student":
        ln, iln = I.student_log_norm(5.0), I.iso_gauss_log_norm(1, 3.0)
        g = smc.Sampler(n, 1, "student", seed=9, rw_sd=0.5, nu=5.0, mu=1.0,
                        mode=O.MODE_AUTO, log_norm=ln, init_log_norm=iln, device=dev)
        o = O.Sampler(n, 1, O.T_STUDENT, seed=9, rw_sd=0.5, nu=5.0, mu=1.0,
                      mode=O.MODE_AUTO, log_norm=ln, init_log_norm=iln)
        o.init()
    else:
        g, o = pair_gauss(smc, dev, n, [2.0], [1.0], 9, O.MODE_AUTO)
    bx = torch.empty((n + 1, 1), dtype=torch.float64, device=dev)
    bw = torch.empty(n + 1, dtype=torch.float64, device=dev)
    bx[1:] = g.x
    bw[1:] = g.logw
    g.x, g.logw = bx[1:], bw[1:]
    assert g.x.data_ptr() % 16 == 8 and g.logw.data_ptr() % 16 == 8
    run_and_compare(g, o, 6)


def test_many_samplers_independent_streams(smc, dev):
    """Different seeds / sampler ids give different draws; same ones repeat."""
    g = I.GAUSS1D
    outs = []
    for seed, sid in [(1, 0), (1, 0), (2, 0), (1, 3)]:
        s = smc.Sampler(256, 1, "gauss", seed=seed, sampler_id=sid, mean=g["mean"],
                        var=g["var"], device=dev)
        s.step()
        outs.append(s.x.cpu().numpy().copy())
    assert np.array_equal(outs[0], outs[1])
    assert not np.array_equal(outs[0], outs[2])
    assert not np.array_equal(outs[0], outs[3])


# ------------------------------------------------------ logistic regression
def logreg_pair(smc, dev, m_rows, d, n, precision, mode=O.MODE_NEVER, seed=3):
    X, y, _ = I.logreg_data(m_rows, d, 200 + m_rows)
    ln = I.iso_gauss_log_norm(d, math.sqrt(10.0))
    iln = I.iso_gauss_log_norm(d, math.sqrt(10.0))
    kw = dict(seed=seed, rw_sd=0.01, init_mean=0.0, init_sd=math.sqrt(10.0), mode=mode)
    g = smc.Sampler(n, d, "logreg", X=X.astype(np.float64), y=y, prior_var=10.0,
                    precision=precision, log_norm=ln, init_log_norm=iln, device=dev, **kw)
    o = O.Sampler(n, d, O.T_LOGREG, X=X.astype(np.float64), y=y, prior_var=10.0, log_norm=ln,
                  init_log_norm=iln, **kw)
    return g, o


# (M, d, scale of theta): every operand width of both kernels (FP64: 1, 2, 4, 8
# and 16 MFMA k-steps; BF16: 1 to 4), M below one tile, a single row, and
# |z| in the hundreds (e^-|z| underflows; the product of factors stays 1).
LR_CASES = [(1000, 8, 0.3), (333, 3, 0.3), (2048, 32, 0.3), (100, 64, 0.3), (500, 13, 0.3),
            (777, 40, 0.3), (17, 13, 0.3), (1, 4, 0.3), (1000, 8, 30.0)]


@pytest.mark.parametrize("m_rows,d,scale", LR_CASES)
def test_logreg_f64_log_target(smc, dev, m_rows, d, scale):
    import torch
    g, o = logreg_pair(smc, dev, m_rows, d, 600, "f64")
    th = np.random.default_rng(9).standard_normal((600, d)) * scale
    lp = g.log_target(torch.from_numpy(th).to(dev)).cpu().numpy()
    ref = o.log_target(th)
    assert_close(lp, ref, 1e-11, "logreg f64 lp")


@pytest.mark.parametrize("m_rows,d,scale", LR_CASES)
def test_logreg_bf16_log_target(smc, dev, m_rows, d, scale):
    import torch
    g, o = logreg_pair(smc, dev, m_rows, d, 600, "bf16")
    th = np.random.default_rng(9).standard_normal((600, d)) * scale
    lp = g.log_target(torch.from_numpy(th).to(dev)).cpu().numpy()
    ref = o.log_target(th)
    rel = np.abs(lp - ref) / np.abs(ref)
    _say("bf16 lp (M=%d, d=%d): max rel %.3g, max abs %.3g nats" % (m_rows, d, rel.max(),
                                                                     np.abs(lp - ref).max()))
    assert rel.max() < 1e-2


def test_logreg_full_size_likelihood(smc, dev):
    """M = 65536 rows, D = 32, N = 2^16 particles: both precisions on the GPU
    for every particle; the oracle on a 256-particle sample."""
    import torch
    cfg = I.LOGREG
    m_rows, d, n = cfg["m_rows"], cfg["d"], cfg["n"]
    X, y, theta_star = I.logreg_data(m_rows, d, 200)
    th = theta_star[None, :] + 0.05 * np.random.default_rng(4).standard_normal((n, d))
    tth = torch.from_numpy(th).to(dev)
    lps = {}
    for prec in ("f64", "bf16"):
        g = smc.Sampler(n, d, "logreg", X=X.astype(np.float64), y=y, prior_var=10.0,
                        precision=prec, init_sd=math.sqrt(10.0), rw_sd=0.01, device=dev)
        lps[prec] = g.log_target(tth).cpu().numpy()
    o = O.Sampler(n, d, O.T_LOGREG, X=X.astype(np.float64), y=y, prior_var=10.0,
                  init_sd=math.sqrt(10.0))
    o.cfg.log_norm = g.cfg.log_norm
    idx = np.linspace(0, n - 1, 256).astype(np.int64)
    ref = o.log_target(th[idx])
    assert_close(lps["f64"][idx], ref, 1e-11, "f64 full size")
    rel = np.abs(lps["bf16"][idx] - ref) / np.abs(ref)
    _say("full-size bf16: max rel %.3g, median abs %.3g nats, max abs %.3g nats"
         % (rel.max(), np.median(np.abs(lps["bf16"][idx] - ref)),
            np.abs(lps["bf16"][idx] - ref).max()))
    assert rel.max() < 1e-2
    relg = np.abs(lps["bf16"] - lps["f64"]) / np.abs(lps["f64"])
    assert relg.max() < 1e-2


@pytest.mark.parametrize("precision,tol", [("f64", 1e-11), ("bf16", 1e-2)])
def test_logreg_steps_per_step_parity(smc, dev, precision, tol):
    """Proposals are bit-exact; log-weights within the likelihood tolerance;
    the resampling decision on the GPU's own weights is bit-exact."""
    import torch
    n, d = 3000, 8
    g, o = logreg_pair(smc, dev, 1500, d, n, precision)
    o.init()
    assert np.array_equal(bits(g.x.cpu().numpy()), bits(o.x))
    assert_close(g.logw.cpu().numpy(), o.logw, tol, "logw0")
    R = smc.Resampler(n, device=dev)
    for t in range(1, 4):
        g.step()
        o.step()
        assert np.array_equal(bits(g.x.cpu().numpy()), bits(o.x)), t
        gl = g.logw.cpu().numpy()
        # the weights telescope to log pi(x_t) - log q0(x_0) up to FP64 rounding
        # of the running sum, so they carry the likelihood's own tolerance
        assert_close(gl, o.logw, tol, "logw t=%d" % t)
        nc = torch.zeros(n, dtype=torch.int64, device=dev)
        R.resample(g.logw, 77 + t, O.MODE_FORCE, ncopies=nc)
        onc, _ = O.resample(gl, 77 + t, O.MODE_FORCE)
        assert np.array_equal(nc.cpu().numpy(), onc)


def test_logreg_one_feature_proposals(smc, dev):
    """d = 1 on the general update path: particles 2p and 2p + 1 share the
    pair drawn for index p; initial particles and proposals bit for bit
    against the oracle over an odd population, weights within tolerance."""
    n = 3001
    g, o = logreg_pair(smc, dev, 400, 1, n, "f64")
    o.init()
    assert np.array_equal(bits(g.x.cpu().numpy()), bits(o.x))
    for t in range(1, 4):
        g.step()
        o.step()
        assert np.array_equal(bits(g.x.cpu().numpy()), bits(o.x)), t
        assert_close(g.logw.cpu().numpy(), o.logw, 1e-11, "logw t=%d" % t)


def test_logreg_force_step_structure(smc, dev):
    """A resampling step leaves copies of proposed particles, equal weights."""
    n, d = 2000, 8
    g, o = logreg_pair(smc, dev, 700, d, n, "f64", mode=O.MODE_FORCE)
    o.init()
    g.step()
    o.step()
    assert g.info()["resampled"] == 1
    assert np.all(g.logw.cpu().numpy() == -math.log(n))
    gx = g.x.cpu().numpy()
    assert np.array_equal(bits(gx), bits(o.x)) or set(map(tuple, gx)) <= set(map(tuple, o.x))


@pytest.mark.parametrize("n,d", [(2048, 16), (2049, 16), (1500, 5)])
def test_gauss_small_population_paths(smc, dev, n, d):
    """N <= 2048 and d <= 16 run as one fused workgroup; 2049 takes the
    multi-kernel path.  Both are bit-exact against the oracle."""
    _say("gauss small n=%d d=%d" % (n, d))
    rng = np.random.default_rng(n + d)
    mean, var = rng.standard_normal(d), rng.uniform(0.5, 2.0, d)
    G, Or = pair_gauss(smc, dev, n, mean, var, 23, O.MODE_AUTO, rw_sd=0.4)
    run_and_compare(G, Or, 5)


def test_resample_call_after_fused_steps(smc, dev):
    """smc_resample on a context whose steps ran fused: the max slots it uses
    were left clear, so its exact max and integers match the oracle."""
    import ctypes as C
    import torch
    g = I.GAUSS1D
    G, Or = pair_gauss(smc, dev, g["n"], g["mean"], g["var"], 3, O.MODE_AUTO)
    for _ in range(3):
        G.step()
        Or.step()
    lib = smc.L.load()
    for k in range(3):
        lw = torch.from_numpy(np.random.default_rng(k).standard_normal(g["n"]) * (k + 1)).to(dev)
        info = torch.zeros(smc.L.INFO_BYTES, dtype=torch.uint8, device=dev)
        r = 0x9E3779B97F4A7C15 * (k + 1) & (2**64 - 1)
        smc.L.check(lib.smc_resample(G.ctx, C.c_void_p(lw.data_ptr()), g["n"], r, O.MODE_FORCE,
                                     None, C.c_void_p(info.data_ptr()), smc._stream()),
                    "smc_resample")
        got = smc.decode_info(info)
        ref = O.resample(lw.cpu().numpy(), r, O.MODE_FORCE)[1]
        for key in ("m", "S", "U", "Q2_hi", "Q2_lo", "K", "err"):
            assert got[key] == ref[key], (k, key)


def test_forced_and_in_place_paths_agree_on_an_error_step(smc, dev):
    """A target with zero density everywhere (variance 1e-320, so the
    precision overflows) makes the step fail on the device: the forced path
    (proposal written to the workspace copy) and the in-place path report the
    same error, resample nothing and leave the same proposal in x."""
    _say("degenerate step, forced vs in place")
    n, d = 5000, 2
    res = []
    for mode in (O.MODE_FORCE, O.MODE_AUTO):
        g = smc.Sampler(n, d, "gauss", seed=4, rw_sd=0.5, mean=[0.0, 0.0], var=[1e-320, 1e-320],
                        mode=mode, device=dev)
        g.sync_error()
        g.step()
        res.append((g.sync_error(), g.x.cpu().numpy().copy(), g.info()["resampled"]))
    assert res[0][0] != 0 and res[0][0] == res[1][0]
    assert res[0][2] == 0 and res[1][2] == 0
    assert np.array_equal(bits(res[0][1]), bits(res[1][1]))


def test_student_t_full_size(smc, dev):
    """The Student-t workload as timed (N = 2^24, nu = 5, mu = 1, resampling
    every iteration): initial population and two iterations bit for bit."""
    _say("student n=2^24 (oracle about 15 s)")
    n = 1 << 24
    g = smc.Sampler(n, 1, "student", seed=1, rw_sd=0.5, nu=5.0, mu=1.0, mode=O.MODE_FORCE,
                    device=dev)
    o = O.Sampler(n, 1, O.T_STUDENT, seed=1, rw_sd=0.5, nu=5.0, mu=1.0, mode=O.MODE_FORCE,
                  log_norm=g.cfg.log_norm, init_log_norm=g.cfg.init_log_norm)
    o.init()
    run_and_compare(g, o, 2)


def test_runs_repeat_bit_for_bit(smc, dev):
    """The same sampler run twice gives the same bits (no dependence on
    scheduling, atomics order or leftover workspace contents); another seed
    gives other bits."""
    _say("repeat runs")

    def run(seed):
        g = smc.Sampler(70001, 1, "student", seed=seed, rw_sd=0.5, nu=5.0, mu=1.0,
                        mode=O.MODE_AUTO, device=dev)
        outs = []
        for _ in range(6):
            g.step()
            outs.append((g.info()["S"], g.estimates()["mean"].copy()))
        return bits(g.x.cpu().numpy()), bits(g.logw.cpu().numpy()), outs

    a, b, c = run(21), run(21), run(22)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for (sa, ea), (sb, eb) in zip(a[2], b[2]):
        assert sa == sb and np.array_equal(bits(ea), bits(eb))
    assert not np.array_equal(a[0], c[0])


def _steps_pair(smc, dev, kind, n, d, mode, seed):
    if kind == "student":
        nu, mu = 5.0, 1.0
        ln, iln = I.student_log_norm(nu), I.iso_gauss_log_norm(1, 3.0)
        mk = lambda: smc.Sampler(n, 1, "student", seed=seed, rw_sd=0.5, nu=nu, mu=mu, mode=mode,
                                 log_norm=ln, init_log_norm=iln, device=dev)
        o = O.Sampler(n, 1, O.T_STUDENT, seed=seed, rw_sd=0.5, nu=nu, mu=mu, mode=mode,
                      log_norm=ln, init_log_norm=iln)
    else:
        mean = np.linspace(-1.0, 1.5, d)
        var = np.linspace(0.5, 2.0, d)
        ln, iln = I.gauss_log_norm(var), I.iso_gauss_log_norm(d, 3.0)
        mk = lambda: smc.Sampler(n, d, "gauss", seed=seed, rw_sd=0.4, init_mean=0.0, init_sd=3.0,
                                 mean=mean, var=var, mode=mode, log_norm=ln, init_log_norm=iln,
                                 device=dev)
        o = O.Sampler(n, d, O.T_GAUSS, seed=seed, rw_sd=0.4, init_mean=0.0, init_sd=3.0,
                      mean=mean, var=var, mode=mode, log_norm=ln, init_log_norm=iln)
    o.init()
    return mk(), mk(), o


@pytest.mark.parametrize("kind,n,d,mode,k", [
    ("gauss", 1024, 1, O.MODE_AUTO, 20),     # the 1-D workload
    ("gauss", 2048, 16, O.MODE_FORCE, 7),    # the largest one-workgroup population
    ("student", 1500, 1, O.MODE_AUTO, 9),
    ("gauss", 1, 2, O.MODE_AUTO, 3),
    ("gauss", 2049, 3, O.MODE_AUTO, 4),      # the multi-kernel path
])
def test_steps_equal_single_steps_and_the_oracle(smc, dev, kind, n, d, mode, k):
    """smc_steps(k) leaves the bits k calls of smc_step leave, records every
    iteration's info and estimates, and matches the oracle."""
    _say("steps %s n=%d d=%d k=%d" % (kind, n, d, k))
    A, B, o = _steps_pair(smc, dev, kind, n, d, mode, 41)
    infos, ests = [], []
    for _ in range(k):
        A.step(info=True, est=True)
        infos.append(A.info())
        ests.append(A.est.cpu().numpy().copy())
    out = B.steps(k, info=True, est=True)
    assert np.array_equal(bits(A.x.cpu().numpy()), bits(B.x.cpu().numpy()))
    assert np.array_equal(bits(A.logw.cpu().numpy()), bits(B.logw.cpu().numpy()))
    be = out["est"].cpu().numpy()
    for t in range(k):
        assert out["info"][t] == infos[t], t
        assert np.array_equal(bits(be[t]), bits(ests[t])), t
    for _ in range(k):
        o.step()
    assert np.array_equal(bits(B.x.cpu().numpy()), bits(o.x))
    assert np.array_equal(bits(B.logw.cpu().numpy()), bits(o.logw))
    # the contexts continue alike: one more single step each
    A.step(info=True, est=False)
    B.step(info=True, est=False)
    assert A.info() == B.info()
    assert np.array_equal(bits(A.x.cpu().numpy()), bits(B.x.cpu().numpy()))
    assert B.sync_error() == 0


def test_steps_argument_errors(smc, dev):
    g = I.GAUSS1D
    S = smc.Sampler(64, 1, "gauss", seed=1, mean=g["mean"], var=g["var"], device=dev)
    lib = smc.L.load()
    import ctypes as C
    rc = lib.smc_steps(S.ctx, C.c_void_p(S.x.data_ptr()), C.c_void_p(S.logw.data_ptr()), 0,
                       None, None, smc._stream())
    assert rc == smc.L.SMC_E_ARG
    rc = lib.smc_steps(S.ctx, C.c_void_p(S.x.data_ptr() + 4), C.c_void_p(S.logw.data_ptr()), 2,
                       None, None, smc._stream())
    assert rc == smc.L.SMC_E_ARG


def _lazy_pair(smc, dev, kind, n, mode):
    def mk(lazy):
        if kind == "student":
            return smc.Sampler(n, 1, "student", seed=5, rw_sd=0.5, nu=5.0, mu=1.0, mode=mode,
                               lazy_reset=lazy, device=dev)
        if kind == "gauss":
            return smc.Sampler(n, 3, "gauss", seed=17, rw_sd=0.3, mean=[1.0, -2.0, 0.5],
                               var=[0.5, 2.0, 1.5], mode=mode, lazy_reset=lazy, device=dev)
        if kind == "bearing":
            B = I.BEARING
            _, ys = I.bearing_track(12, 7)
            return smc.Sampler(n, 4, "bearing", seed=3, mean=B["x0"], init_sd=B["init_sd"],
                               obs=ys, delta=B["delta"], obs_var=B["obs_var"], mode=mode,
                               lazy_reset=lazy, device=dev)
        X, y, _ = I.logreg_data(500, 8, 300)
        return smc.Sampler(n, 8, "logreg", seed=3, X=X.astype(np.float64), y=y, prior_var=10.0,
                           rw_sd=0.01, init_sd=math.sqrt(10.0), mode=mode, lazy_reset=lazy,
                           device=dev)
    return mk(False), mk(True)


@pytest.mark.parametrize("kind,n,mode", [("student", 1 << 24, O.MODE_FORCE),
                                         ("student", 70001, O.MODE_FORCE),
                                         ("gauss", 3001, O.MODE_AUTO),
                                         ("bearing", 20000, O.MODE_AUTO),
                                         ("logreg", 3000, O.MODE_FORCE),
                                         ("gauss", 1500, O.MODE_FORCE)])
def test_lazy_reset_matches_eager(smc, dev, kind, n, mode):
    """A lazy-reset sampler follows the eager one bit for bit; its logw catches
    up on smc_sync_weights (synced on every other iteration here, so that
    iterations also start from stale memory marked uniform)."""
    _say("lazy %s n=%d" % (kind, n))
    E, Lz = _lazy_pair(smc, dev, kind, n, mode)
    resampled = 0
    for t in range(1, 9):
        E.step(info=True, est=True)
        Lz.step(info=True, est=True)
        ie, il = E.info(), Lz.info()
        assert ie == il, t
        resampled += ie["resampled"]
        assert np.array_equal(bits(E.x.cpu().numpy()), bits(Lz.x.cpu().numpy())), t
        assert np.array_equal(bits(E.est.cpu().numpy()), bits(Lz.est.cpu().numpy())), t
        if t % 2 == 0:
            Lz.sync_weights()
            assert np.array_equal(bits(E.logw.cpu().numpy()), bits(Lz.logw.cpu().numpy())), t
    assert resampled > 0
    assert Lz.sync_error() == 0


def test_lazy_reset_with_steps(smc, dev):
    """smc_steps on a lazy-reset sampler: the same bits as eager single steps."""
    E, Lz = _lazy_pair(smc, dev, "student", 9000, O.MODE_FORCE)
    for _ in range(5):
        E.step(info=False, est=False)
    out = Lz.steps(5, info=True)
    assert out["info"][-1]["resampled"] == 1
    assert np.array_equal(bits(E.x.cpu().numpy()), bits(Lz.x.cpu().numpy()))
    Lz.sync_weights()
    assert np.array_equal(bits(E.logw.cpu().numpy()), bits(Lz.logw.cpu().numpy()))


@pytest.mark.parametrize("mode", ["auto", "force"])
def test_gauss_4d_multi_kernel_path(smc, dev, mode):
    """d = 4 above the one-workgroup size: the update kernel's four-coordinate
    one-pass estimate; bit-exact trajectories against the oracle."""
    _say("gauss 4d", mode)
    G, Or = pair_gauss(smc, dev, 5000, [0.5, -1.0, 2.0, 0.0], [1.0, 0.5, 2.0, 1.5], 29,
                       MODES[mode], rw_sd=0.4)
    run_and_compare(G, Or, 6)


@pytest.mark.parametrize("d,mode", [(1, "never"), (4, "never"), (1, "auto")])
def test_estimate_reference_over_wide_weight_spread(smc, dev, d, mode):
    """Log-weights spread over 400 nats at N = 2^20 + 3: the update kernel runs
    one full residency, so each thread folds several particles into its one-pass
    estimate sums and meets weights far above (the reference moves, the sums
    are rescaled) and far below its reference (terms underflow harmlessly).
    Trajectories bit for bit, estimates within the FP64-sum tolerance."""
    import torch
    _say("estimate reference d=%d %s" % (d, mode))
    n = (1 << 20) + 3
    rng = np.random.default_rng(5 + d)
    G, Or = pair_gauss(smc, dev, n, rng.standard_normal(d), rng.uniform(0.5, 2.0, d), 31,
                       MODES[mode], rw_sd=0.3)
    lw = rng.uniform(-400.0, 0.0, n)
    G.logw.copy_(torch.from_numpy(lw).to(dev))
    Or.logw[:] = lw
    run_and_compare(G, Or, 2)


@pytest.mark.parametrize("kind,n,d", [("gauss", 3001, 3), ("gauss", 1024, 1),
                                      ("student", 70001, 1)])
def test_failed_iteration_leaves_recycling(smc, dev, kind, n, d):
    """A NaN log-weight makes one iteration fail at the resampling step (the
    oracle returns there): c_t, the recycling sums and log Z_{t-1} stay as they
    were, so once the weight is repaired the run continues as the oracle's
    does, recycled estimates included."""
    import torch
    _say("failed iteration %s n=%d d=%d" % (kind, n, d))
    if kind == "student":
        _, G, Or = _steps_pair(smc, dev, "student", n, 1, O.MODE_AUTO, 13)
    else:
        rng = np.random.default_rng(d)
        G, Or = pair_gauss(smc, dev, n, rng.standard_normal(d), rng.uniform(0.5, 2.0, d), 13,
                           O.MODE_AUTO, rw_sd=0.4)
    for _ in range(3):
        G.step()
        Or.step()
    G.logw[5] = float("nan")
    Or.logw[5] = np.nan
    G.step()
    with pytest.raises(ValueError):
        Or.step()
    assert G.info()["err"] == O.E_NONFINITE
    assert G.sync_error() == O.E_NONFINITE
    assert np.array_equal(bits(G.x.cpu().numpy()), bits(Or.x))
    G.logw[5] = 0.25
    Or.logw[5] = 0.25
    for t in range(3):
        G.step()
        out = Or.step()
        assert np.array_equal(bits(G.x.cpu().numpy()), bits(Or.x)), t
        assert np.array_equal(bits(G.logw.cpu().numpy()), bits(Or.logw)), t
        assert abs(G.info()["log_c"] - out["log_c"]) <= 1e-11, t
        e = G.estimates()
        for k in ("mean", "m2", "rec_mean", "rec_m2"):
            assert_close(e[k], out[k], 1e-11, "%s after the failed iteration, t=%d" % (k, t))
    assert G.sync_error() == 0
    del torch


@pytest.mark.parametrize("precision,tol", [("f64", 1e-11), ("bf16", 1e-2)])
def test_logreg_full_size_resampling_step(smc, dev, precision, tol):
    """One resampling iteration of the timed logistic-regression workload
    (N = 2^16, M = 65536, D = 32) in each precision, against the oracle:
    initial particles and proposals bit for bit (the oracle's normals); log pi
    of 256 particles within the likelihood tolerance (the oracle's plain FP64
    sum); and with the oracle fed the GPU's own weights (Alg 2 reweighting of
    the GPU's log-targets), the resampling integers and the redistributed
    particles bit for bit."""
    import torch
    c = I.LOGREG
    m_rows, d, n = c["m_rows"], c["d"], c["n"]
    X, y, _ = I.logreg_data(m_rows, d, 200)
    seed, rw_sd, init_sd = 9, c["rw_sd"], math.sqrt(c["prior_var"])
    _say("logreg full size %s" % precision)
    kw = dict(X=X.astype(np.float64), y=y, prior_var=c["prior_var"], precision=precision,
              rw_sd=rw_sd, init_sd=init_sd, seed=seed, device=dev)
    G = smc.Sampler(n, d, "logreg", mode=O.MODE_FORCE, **kw)
    Gn = smc.Sampler(n, d, "logreg", mode=O.MODE_NEVER, **kw)
    x0 = G.x.cpu().numpy().copy()
    lw0 = G.logw.cpu().numpy().copy()
    # x0 ~ q0 and the proposal x' = x0 + rw_sd z from the oracle's normals
    z0 = np.stack([O.normals(seed, O.TAG_INIT, 0, 0, i, d) for i in range(n)])
    assert np.array_equal(bits(x0), bits(0.0 + init_sd * z0))
    z1 = np.stack([O.normals(seed, O.TAG_PROPOSE, 0, 1, i, d) for i in range(n)])
    xp = x0 + rw_sd * z1
    Gn.step()
    assert np.array_equal(bits(Gn.x.cpu().numpy()), bits(xp))
    # log pi at x0 and x' on the GPU; 256 of them against the oracle
    lp0 = G.log_target(torch.from_numpy(x0).to(dev)).cpu().numpy()
    lp1 = G.log_target(torch.from_numpy(xp).to(dev)).cpu().numpy()
    o = O.Sampler(n, d, O.T_LOGREG, X=X.astype(np.float64), y=y, prior_var=c["prior_var"],
                  init_sd=init_sd, log_norm=G.cfg.log_norm)
    idx = np.linspace(0, n - 1, 256).astype(np.int64)
    ref = o.log_target(xp[idx])
    err = np.abs(lp1[idx] - ref)
    _say("%s log pi at N=2^16, M=65536: max rel %.3g, max abs %.3g nats, median abs %.3g nats"
         % (precision, np.max(err / np.abs(ref)), err.max(), np.median(err)))
    assert_close(lp1[idx], ref, tol, "%s log pi" % precision)
    # the resampling iteration on the GPU, and the oracle's on the GPU's weights
    G.step()
    info = G.info()
    lw1 = lw0 + (lp1 - lp0)
    onc, oinfo = O.resample(lw1, O.resample_draw(seed, 0, 1), O.MODE_FORCE)
    for k in ("S", "U", "Q2_hi", "Q2_lo", "K", "resampled", "err"):
        assert info[k] == oinfo[k], (k, info[k], oinfo[k])
    assert info["m"] == oinfo["m"]
    ox, _ = O.redistribute(onc, xp)
    assert np.array_equal(bits(G.x.cpu().numpy()), bits(ox))
    assert np.all(G.logw.cpu().numpy() == -math.log(n))
    assert G.sync_error() == 0 and Gn.sync_error() == 0
