"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and its host-only helpers behave.  No device work is launched."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    out = set()
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            text = open(os.path.join(inc, f)).read()
            out |= set(re.findall(r"^\s*(?:size_t|smc_status|const char \*)\s*(smc_\w+)\s*\(",
                                  text, re.M))
    return sorted(out)


@pytest.fixture(scope="module")
def lib():
    from paper_1905_10252_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1905_10252_amd import build
        build.build()
    return L.load()


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for s in ("smc_init", "smc_step", "smc_resample", "smc_redistribute", "smc_workspace_bytes",
              "smc_destroy", "smc_status_string", "smc_batch_create", "smc_batch_attach",
              "smc_batch_step", "smc_batch_detach"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_python_binding_covers_exports():
    from paper_1905_10252_amd import _lib as L
    assert sorted(L.EXPORTS) == declared_symbols()


def test_workspace_bytes(lib):
    from paper_1905_10252_amd import _lib as L
    cfg = L.SmcConfig()
    cfg.n, cfg.d, cfg.x_dtype, cfg.target, cfg.ess_num, cfg.ess_den = 1 << 24, 16, 0, 0, 1, 2
    b = lib.smc_workspace_bytes(C.byref(cfg))
    assert 8 * (1 << 24) < b < 8 * (1 << 24) + (1 << 24) // 8 + (1 << 21)  # prefix + 1/64 samples
    cfg.n = 0
    assert lib.smc_workspace_bytes(C.byref(cfg)) == 0
    cfg.n, cfg.ess_den = 10, 0
    assert lib.smc_workspace_bytes(C.byref(cfg)) == 0
    # sampler workspace grows with d
    cfg.ess_den, cfg.target, cfg.x_dtype, cfg.d, cfg.rw_sd, cfg.init_sd = 2, 2, 1, 1, 0.5, 3.0
    cfg.nu = 5.0
    assert lib.smc_workspace_bytes(C.byref(cfg)) > 0
    cfg.x_dtype = 0  # samplers need FP64 particles
    assert lib.smc_workspace_bytes(C.byref(cfg)) == 0
    cfg.x_dtype, cfg.lazy_reset = 1, 1
    assert lib.smc_workspace_bytes(C.byref(cfg)) > 0
    cfg.lazy_reset = 2  # a flag: 0 or 1
    assert lib.smc_workspace_bytes(C.byref(cfg)) == 0


def test_status_strings(lib):
    for code in range(7):
        assert lib.smc_status_string(code)
    assert b"unknown" in lib.smc_status_string(99)


def test_struct_sizes_match_header():
    from paper_1905_10252_amd import _lib as L
    assert C.sizeof(L.SmcInfo) == 96
    assert C.sizeof(L.SmcConfig) == 192  # sizeof(smc_config) on x86-64 (gcc)


def test_batch_workspace_bytes(lib):
    from paper_1905_10252_amd import _lib as L
    assert C.sizeof(L.SmcBatchSampler) == 128
    assert lib.smc_batch_workspace_bytes(0) == 0
    assert lib.smc_batch_workspace_bytes(4097) == 0
    assert lib.smc_batch_workspace_bytes(256) > 256 * 200
    d = L.SmcBatchSampler()
    d.n, d.d, d.mode, d.ess_num, d.ess_den = 10000, 33, 0, 1, 2
    d.rw_sd, d.init_sd = 0.1, 3.0
    d.mean = d.chol = d.x = d.logw = 256
    b = lib.smc_batch_sampler_bytes(C.byref(d))
    assert 8 * 10000 * (3 + 33) < b < 8 * 10000 * (3 + 33) + (1 << 16)  # lp, scratch, prefix
    d.d = 65
    assert lib.smc_batch_sampler_bytes(C.byref(d)) == 0
    d.d, d.n = 4, 0
    assert lib.smc_batch_sampler_bytes(C.byref(d)) == 0
    d.n, d.chol = 5, None
    assert lib.smc_batch_sampler_bytes(C.byref(d)) == 0
