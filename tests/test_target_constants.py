"""Normalising constants the binding supplies by default, against scipy's
densities (CPU).  Both the oracle and the GPU path take these constants as
inputs, so parity between them cannot catch a wrong one; here each is checked
against an independent implementation of the same density."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_1905_10252_amd import smc
from paper_1905_10252_amd import inputs as I


def test_q0_constant():
    # x0 ~ N(init_mean, init_sd^2 I): log q0(x) = c - |x - m|^2 / (2 sd^2)
    rng = np.random.default_rng(1)
    for d, sd in ((1, 3.0), (4, 0.5), (16, 2.0)):
        x = rng.standard_normal(d)
        ref = stats.multivariate_normal(np.full(d, 0.25), sd * sd * np.eye(d)).logpdf(x)
        got = smc.q0_log_norm(d, sd) - 0.5 * np.sum((x - 0.25) ** 2) / (sd * sd)
        assert got == pytest.approx(ref, rel=1e-13, abs=1e-13)


def test_diagonal_gauss_constant():
    rng = np.random.default_rng(2)
    for d in (1, 3, 8):
        var = rng.uniform(0.2, 3.0, d)
        mean = rng.standard_normal(d)
        x = rng.standard_normal(d)
        ref = stats.multivariate_normal(mean, np.diag(var)).logpdf(x)
        got = smc.gauss_log_norm(var) - 0.5 * np.sum((x - mean) ** 2 / var)
        assert got == pytest.approx(ref, rel=1e-13, abs=1e-13)


def test_student_constant():
    for nu in (1.0, 2.5, 5.0, 30.0):
        for x in (-3.0, 0.1, 1.0, 7.5):
            ref = stats.t(df=nu, loc=1.0).logpdf(x)
            t = x - 1.0
            got = smc.student_log_norm(nu) - 0.5 * (nu + 1.0) * math.log1p(t * t / nu)
            assert got == pytest.approx(ref, rel=1e-13, abs=1e-13)


def test_logreg_prior_and_bearing_noise_constants():
    rng = np.random.default_rng(3)
    d, pv = I.LOGREG["d"], I.LOGREG["prior_var"]
    th = rng.standard_normal(d)
    ref = stats.multivariate_normal(np.zeros(d), pv * np.eye(d)).logpdf(th)
    assert smc.logreg_log_norm(d, pv) - 0.5 * th @ th / pv == pytest.approx(ref, rel=1e-13)
    for ov in (1e-4, 0.01):
        e = 0.003
        ref = stats.norm(0.0, math.sqrt(ov)).logpdf(e)
        assert smc.bearing_obs_log_norm(ov) - 0.5 * e * e / ov == pytest.approx(ref, rel=1e-13)


def test_precision_factor_constant():
    # Gaussian with precision U^T U, the batched samplers' target
    rng = np.random.default_rng(4)
    for d in (1, 5, 17, 64):
        mean, U, cov = I.wishart_target(d, rng)
        x = mean + rng.standard_normal(d)
        ref = stats.multivariate_normal(mean, cov).logpdf(x)
        r = U @ (x - mean)
        got = smc.chol_log_norm(U) - 0.5 * r @ r
        assert got == pytest.approx(ref, rel=1e-10, abs=1e-10)
