"""Autotuner for the batched sampler's launch shape.

Times whole batched steps on the device for each candidate proposal-unit size
(coordinate pairs per 256-particle unit) on a scratch batch holding the
caller's workload shapes, and returns the fastest.  The choice changes only
speed: every candidate gives the same bits.
"""
from __future__ import annotations

import torch

from . import smc

GROUP_CANDIDATES = (2, 4, 8)


def tune_group(specs, *, device=None, steps: int = 3, candidates=GROUP_CANDIDATES) -> dict:
    """``specs``: sampler descriptions (dicts with n, d, mean, chol, seed,
    sampler_id, rw_sd, init_sd).  Returns {"best": pairs, "ms": {pairs: ms}}."""
    dev = torch.device(device or "cuda")
    b = smc.Batch(len(specs), graph=False, device=dev)
    for k, sp in enumerate(specs):
        b.attach(k, sp["n"], sp["d"], sp["mean"], sp["chol"], seed=sp["seed"],
                 sampler_id=sp["sampler_id"], rw_sd=sp["rw_sd"], init_sd=sp.get("init_sd", 3.0))
    times = {}
    for g in candidates:
        b.set_group(g)
        b.step(info=False, est=False)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            b.step(info=False, est=False)
        e1.record()
        torch.cuda.synchronize()
        times[g] = e0.elapsed_time(e1) / steps
    del b
    best = min(times, key=times.get)
    return {"best": best, "ms": times}
