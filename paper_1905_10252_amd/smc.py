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


def _stream():
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
        if getattr(self, "ctx", None) and self.ctx.value:
            self._lib.smc_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def resample(self, logw: torch.Tensor, r: int, mode: int = L.MODE_AUTO,
                 ncopies: torch.Tensor | None = None, info: bool = True):
        _need(logw, torch.float64, self.n, "logw")
        if ncopies is not None:
            _need(ncopies, torch.int64, self.n, "ncopies")
        L.check(self._lib.smc_resample(self.ctx, _ptr(logw), self.n, int(r) & (2**64 - 1), mode,
                                       _ptr(ncopies), _ptr(self.info_buf) if info else None,
                                       _stream()), "smc_resample")
        return ncopies

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


def reset_logw(logw: torch.Tensor) -> torch.Tensor:
    """Reset step of Alg 4: every weight 1/N (log-weight -ln N)."""
    return logw.fill_(-math.log(logw.shape[0]))
