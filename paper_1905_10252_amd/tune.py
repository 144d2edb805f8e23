"""Autotuner for the batched sampler's launch shape.

Times whole batched steps on the device on a scratch batch holding the
caller's workload shapes, for the knobs that change only speed (every
candidate gives the same bits):

  - ``k_bprop`` / unit_pairs: coordinate pairs per proposal work unit (2, 4, 8);
  - ``k_bquad`` / waves, per dimension bucket: the occupancy the target
    kernel of samplers with d in (8 q, 8 q + 8] aims at (1 up to what that
    bucket's kernel reaches), tuned one bucket at a time with the others at
    their current choice.

Results are kept in a JSON cache keyed by kernel, knob, bucket, device
architecture (gcnArchName, e.g. gfx950) and a digest of the workload's
(N, d) shapes, so a later run on the same device and workload reuses them
without timing.  The cache file is ``$SMC_TUNE_CACHE`` or
``~/.cache/paper_1905_10252_amd/tune.json``.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from . import smc

GROUP_CANDIDATES = (2, 4, 5, 6, 8)
BUCKETS = 8


def _max_waves(bucket: int) -> int:
    d = 8 * (bucket + 1)
    return 4 if d <= 40 else 3


def cache_path() -> str:
    return os.environ.get("SMC_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1905_10252_amd", "tune.json")


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: dict) -> None:
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # an unwritable cache only costs a retune next time


def arch(dev) -> str:
    return torch.cuda.get_device_properties(dev).gcnArchName.split(":")[0]


def workload_digest(specs) -> str:
    shapes = sorted((int(sp["n"]), int(sp["d"])) for sp in specs)
    return hashlib.sha1(repr(shapes).encode()).hexdigest()[:16]


def key(kernel: str, knob: str, bucket, arch_name: str, digest: str) -> str:
    return "%s|%s|%s|%s|%s" % (kernel, knob, "all" if bucket is None else bucket, arch_name,
                               digest)


def _scratch_batch(specs, dev):
    b = smc.Batch(len(specs), graph=False, device=dev)
    for k, sp in enumerate(specs):
        b.attach(k, sp["n"], sp["d"], sp["mean"], sp["chol"], seed=sp["seed"],
                 sampler_id=sp["sampler_id"], rw_sd=sp["rw_sd"], init_sd=sp.get("init_sd", 3.0))
    return b


def _time_steps(b, steps: int) -> float:
    b.step(info=False, est=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        b.step(info=False, est=False)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def tune_group(specs, *, device=None, steps: int = 3, candidates=GROUP_CANDIDATES,
               use_cache: bool = True) -> dict:
    """``specs``: sampler descriptions (dicts with n, d, mean, chol, seed,
    sampler_id, rw_sd, init_sd).  Returns {"best": pairs, "ms": {pairs: ms},
    "cached": bool}."""
    dev = torch.device(device or "cuda")
    path, k = cache_path(), key("k_bprop", "unit_pairs", None, arch(dev), workload_digest(specs))
    data = _load(path) if use_cache else {}
    if k in data:
        return {"best": data[k]["best"], "ms": data[k]["ms"], "cached": True}
    b = _scratch_batch(specs, dev)
    times = {}
    for g in candidates:
        b.set_group(g)
        times[g] = _time_steps(b, steps)
    del b
    best = min(times, key=times.get)
    if use_cache:
        data = _load(path)
        data[k] = {"best": best, "ms": {str(g): t for g, t in times.items()}}
        _store(path, data)
    return {"best": best, "ms": times, "cached": False}


def tune_buckets(specs, *, device=None, steps: int = 4, pairs: int | None = None,
                 use_cache: bool = True) -> dict:
    """Occupancy aim of the target kernel per dimension bucket present in the
    workload (one bucket at a time, whole-step timings).  Returns
    {"best": {bucket: waves}, "ms": {bucket: {waves: ms}}, "cached": [...]}."""
    dev = torch.device(device or "cuda")
    a, dg = arch(dev), workload_digest(specs)
    path = cache_path()
    data = _load(path) if use_cache else {}
    present = sorted({(int(sp["d"]) - 1) // 8 for sp in specs})
    best, ms, cached = {}, {}, []
    todo = []
    for q in present:
        k = key("k_bquad", "waves", q, a, dg)
        if k in data:
            best[q] = data[k]["best"]
            ms[q] = data[k]["ms"]
            cached.append(q)
        else:
            best[q] = _max_waves(q)
            todo.append(q)
    if todo:
        b = _scratch_batch(specs, dev)
        if pairs is not None:
            b.set_group(pairs)
        for q in present:
            b.set_bucket_waves(q, best[q])
        for q in todo:
            times = {}
            for w in range(1, _max_waves(q) + 1):
                b.set_bucket_waves(q, w)
                times[w] = _time_steps(b, steps)
            best[q] = min(times, key=times.get)
            b.set_bucket_waves(q, best[q])
            ms[q] = times
        del b
        if use_cache:
            data = _load(path)
            for q in todo:
                data[key("k_bquad", "waves", q, a, dg)] = {
                    "best": best[q], "ms": {str(w): t for w, t in ms[q].items()}}
            _store(path, data)
    return {"best": best, "ms": ms, "cached": cached}


def apply(batch, tuned_group: dict | None = None, tuned_buckets: dict | None = None) -> None:
    """Sets a batch's knobs to tuned choices."""
    if tuned_group is not None:
        batch.set_group(tuned_group["best"])
    if tuned_buckets is not None:
        for q, w in tuned_buckets["best"].items():
            batch.set_bucket_waves(int(q), int(w))
