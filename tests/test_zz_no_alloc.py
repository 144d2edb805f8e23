"""smc_resample_noalloc (no context, no workspace, nothing allocated) against
smc_resample with ncopies on a context of the same N, through the C ABI: the
same bits in every output, on consecutive calls of decreasing size (the fixed
array keeps the last call's contents), and against the oracle."""
import ctypes as C
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


def run_pair(smc, dev, lw, r, mode):
    import torch
    n = lw.size
    L = smc.L
    lib = L.load()
    tlw = torch.from_numpy(lw).to(dev)
    # the existing entry point on a context of this N
    R = smc.Resampler(n, device=dev)
    nc_ref = torch.full((n,), -3, dtype=torch.int64, device=dev)
    R.resample(tlw, r, mode, ncopies=nc_ref)
    # the no-allocation one
    nc = torch.full((n,), -5, dtype=torch.int64, device=dev)
    info = torch.zeros(L.INFO_BYTES, dtype=torch.uint8, device=dev)
    L.check(lib.smc_resample_noalloc(C.c_void_p(tlw.data_ptr()), n, r, mode, 1, 2,
                                     C.c_void_p(nc.data_ptr()), C.c_void_p(info.data_ptr()),
                                     smc._stream()), "smc_resample_noalloc")
    torch.cuda.synchronize()
    return nc.cpu().numpy(), smc.decode_info(info), nc_ref.cpu().numpy(), R.info()


@pytest.mark.parametrize("mode", [O.MODE_FORCE, O.MODE_AUTO])
def test_noalloc_equals_resample_on_consecutive_calls(smc, dev, mode):
    cases = [(smc.L.NOALLOC_MAX_N, 2.0, 31), (70001, 0.5, 32), (4097, 8.0, 33), (1, 1.0, 34)]
    for n, s, seed in cases:
        _say("noalloc n=%d s=%g mode=%d" % (n, s, mode))
        lw = I.logw_normal(n, s, seed)
        r = I.offset_word(seed)
        nc, info, nc_ref, info_ref = run_pair(smc, dev, lw, r, mode)
        assert np.array_equal(nc, nc_ref), n
        assert info == info_ref, (n, info, info_ref)
        onc, oinfo = O.resample(lw, r, mode)
        assert np.array_equal(nc, onc), n
        for k in ("S", "U", "Q2_hi", "Q2_lo", "K", "resampled", "err"):
            assert info[k] == oinfo[k], (n, k)
        assert info["m"] == oinfo["m"]
        assert abs(info["logZ"] - oinfo["logZ"]) <= 1e-12 * max(1.0, abs(oinfo["logZ"]))


def test_noalloc_errors(smc, dev):
    import torch
    L = smc.L
    lib = L.load()
    n = L.NOALLOC_MAX_N + 1
    lw = torch.zeros(n, dtype=torch.float64, device=dev)
    nc = torch.zeros(n, dtype=torch.int64, device=dev)
    rc = lib.smc_resample_noalloc(C.c_void_p(lw.data_ptr()), n, 1, O.MODE_FORCE, 1, 2,
                                  C.c_void_p(nc.data_ptr()), None, smc._stream())
    assert rc == L.SMC_E_NOMEM
    rc = lib.smc_resample_noalloc(C.c_void_p(lw.data_ptr()), 10, 1, O.MODE_FORCE, 1, 2, None,
                                  None, smc._stream())
    assert rc == L.SMC_E_ARG
    # a NaN weight: reported in info, nothing latched, the next call is clean
    bad = I.logw_normal(5000, 1.0, 7)
    bad[17] = np.nan
    info = torch.zeros(L.INFO_BYTES, dtype=torch.uint8, device=dev)
    tb = torch.from_numpy(bad).to(dev)
    nc = torch.zeros(5000, dtype=torch.int64, device=dev)
    L.check(lib.smc_resample_noalloc(C.c_void_p(tb.data_ptr()), 5000, 1, O.MODE_FORCE, 1, 2,
                                     C.c_void_p(nc.data_ptr()), C.c_void_p(info.data_ptr()),
                                     smc._stream()), "smc_resample_noalloc")
    assert smc.decode_info(info)["err"] == L.SMC_E_NONFINITE
    good = I.logw_normal(5000, 1.0, 8)
    got, gi, ref, ri = run_pair(smc, dev, good, 99, O.MODE_FORCE)
    assert gi["err"] == 0 and np.array_equal(got, ref) and gi == ri
