"""Continuous-batching request loop over libsmc.

Requests are SMC-sampler runs (Alg 2) of their own size, dimension, target
and iteration count.  Each tick of the loop admits arrived requests while a
batch slot and the HBM budget allow (first come, first served), advances
every admitted request by one iteration, and retires the finished ones:

  - Gaussian requests (any N and d <= 64, full-precision target) share one
    batched step of ``smc.Batch``: all of them advance in the same launches;
  - logistic-regression requests each advance by one ``smc_step`` of their
    own context (BF16 MFMA likelihood), on further streams (contexts dealt
    round robin over them), so their kernels overlap the batched step and
    each other on the device.

Particle state stays on the device from admission to retirement.  A request's
result depends only on the request: the batch gives every sampler the same
bits alone and in a mix.  All device work is the library's (``DeviceBackend``);
the scheduler (``Server``) only decides what runs in which tick and keeps time,
and runs over any backend with the same methods.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import torch

from . import _lib as L
from . import smc


@dataclass
class Request:
    rid: int
    kind: str                 # "gauss" or "logreg"
    n: int
    d: int
    iters: int
    arrival: float            # seconds (or ticks) from the start of the run
    seed: int
    sampler_id: int
    params: dict = field(default_factory=dict)
    admitted: float | None = None
    finished: float | None = None
    result: dict | None = None

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


def request_bytes(r: Request) -> int:
    """Device bytes a request holds while admitted (state plus workspace)."""
    if r.kind == "gauss":
        # x, x scratch, lp, lp scratch, logw, prefix: (2d + 4) doubles a particle
        return 8 * r.n * (2 * r.d + 4) + 8 * r.d * (r.d + 1) + (1 << 16)
    m = r.params["X"].shape[0]
    dp = (r.d + 15) // 16 * 16
    # particles, scratch, weights, log-targets, prefix, 8 likelihood partials,
    # bf16 copies of the particles and of the data
    return 8 * r.n * (2 * r.d + 16) + 2 * r.n * dp + 2 * m * dp + 8 * m * (r.d + 1) + (1 << 16)


class DeviceBackend:
    """The device side of a server: one ``smc.Batch`` of ``capacity`` slots
    for the Gaussian requests, one ``smc.Sampler`` context per
    logistic-regression request on one of ``side_streams`` further streams
    (contexts dealt round robin, so that the small likelihood launches of
    different requests overlap), and retirement of results through pinned
    host memory behind events."""

    def __init__(self, capacity: int, *, graph: bool = True, keep_particles: bool = False,
                 device=None, side_streams: int = 3):
        self.device = torch.device(device or "cuda")
        self.batch = smc.Batch(capacity, graph=graph, device=self.device)
        self.keep = keep_particles
        self.main = torch.cuda.current_stream(self.device)
        # default priority; with the main stream, one per hardware queue
        self.sides = [torch.cuda.Stream(device=self.device) for _ in range(max(1, side_streams))]
        self.opened = 0
        self.t0 = None

    def attach(self, slot: int, r: Request) -> None:
        p = r.params
        self.batch.attach(slot, r.n, r.d, p["mean"], p["chol"], seed=r.seed,
                          sampler_id=r.sampler_id, rw_sd=p["rw_sd"],
                          init_mean=p.get("init_mean", 0.0), init_sd=p.get("init_sd", 3.0),
                          mode=p.get("mode", L.MODE_AUTO))

    def open(self, r: Request):
        p = r.params
        stream = self.sides[self.opened % len(self.sides)]
        self.opened += 1
        with torch.cuda.stream(stream):
            s = smc.Sampler(r.n, r.d, "logreg", seed=r.seed, sampler_id=r.sampler_id,
                            X=p["X"], y=p["y"], prior_var=p["prior_var"],
                            precision=p.get("precision", "bf16"), rw_sd=p["rw_sd"],
                            init_sd=math.sqrt(p["prior_var"]),
                            mode=p.get("mode", L.MODE_AUTO), device=self.device)
        s.serve_stream = stream
        return s

    def step(self, batch: bool, contexts) -> None:
        if batch:
            self.batch.step(info=False, est=True)
        for s in contexts:
            with torch.cuda.stream(s.serve_stream):
                s.step(info=False, est=True)

    def _token(self, est_dev, x_dev, stream):
        with torch.cuda.stream(stream):
            host = torch.empty(est_dev.numel(), dtype=torch.float64, pin_memory=True)
            host.copy_(est_dev, non_blocking=True)
            x = x_dev.cpu().numpy() if (self.keep and x_dev is not None) else None
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
        return (ev, host, x)

    def retire_slot(self, slot: int, r: Request):
        o = slot * L.BATCH_EST_STRIDE
        tok = self._token(self.batch.est[o:o + 4 * r.d],
                          self.batch.x(slot) if self.keep else None, self.main)
        self.batch.detach(slot)
        return tok

    def retire_context(self, s, r: Request):
        # the context's buffers were allocated on its stream: freeing them
        # with the sampler is ordered after its last use there
        return self._token(s.est[:4 * r.d], s.x if self.keep else None, s.serve_stream)

    def ready(self, tok) -> bool:
        return tok[0].query()

    def wait(self, tok) -> None:
        tok[0].synchronize()

    def fetch(self, tok):
        return tok[1].numpy(), tok[2]

    def start(self) -> None:
        torch.cuda.current_stream(self.device).synchronize()
        self.t0 = torch.cuda.Event(enable_timing=True)
        self.t0.record()

    def elapsed(self, tok) -> float:
        return self.t0.elapsed_time(tok[0]) / 1e3

    def finish(self) -> None:
        torch.cuda.synchronize(self.device)


class Server:
    """Admits requests into ``capacity`` batch slots under an HBM budget
    (bytes), first come first served, and advances all admitted requests one
    iteration per tick.

    A finished request's slot and bytes are free for the next tick at once;
    its results are retired through the backend (on the device: pinned host
    memory behind an event) and the request is finished once they have
    arrived, so ticks never wait for the device.  The default backend is the
    library's (``DeviceBackend``); any object with the same methods serves."""

    def __init__(self, capacity: int = 256, hbm_budget: int = 64 << 30, *, graph: bool = True,
                 keep_particles: bool = False, device=None, backend=None):
        self.be = backend if backend is not None else DeviceBackend(
            capacity, graph=graph, keep_particles=keep_particles, device=device)
        self.capacity = capacity
        self.budget = int(hbm_budget)
        self.used = 0
        self.free = list(range(capacity))[::-1]
        self.queue = collections.deque()
        self.gauss = {}    # slot -> [request, iterations left]
        self.logreg = {}   # rid -> [request, context, iterations left]
        self.retiring = [] # [request, backend token, d]
        self.iters_done = 0
        self.peak_used = 0
        self.peak_active = 0

    # --------------------------------------------------------------- admission
    def submit(self, r: Request) -> None:
        if request_bytes(r) > self.budget:
            raise ValueError("request %d needs more than the whole HBM budget" % r.rid)
        self.queue.append(r)

    def _fits(self, r: Request) -> bool:
        if self.used + request_bytes(r) > self.budget:
            return False
        return r.kind == "logreg" or bool(self.free)

    def _admit(self, now: float) -> None:
        while self.queue and self.queue[0].arrival <= now and self._fits(self.queue[0]):
            r = self.queue.popleft()
            if r.kind == "gauss":
                slot = self.free.pop()
                self.be.attach(slot, r)
                self.gauss[slot] = [r, r.iters]
            else:
                self.logreg[r.rid] = [r, self.be.open(r), r.iters]
            self.used += request_bytes(r)
            self.peak_used = max(self.peak_used, self.used)
            self.peak_active = max(self.peak_active, len(self.gauss) + len(self.logreg))
            r.admitted = now

    # -------------------------------------------------------------------- tick
    def busy(self) -> bool:
        return bool(self.gauss or self.logreg or self.retiring)

    def _collect(self, finish_time) -> list:
        out, keep = [], []
        for ent in self.retiring:
            r, tok, d = ent
            if not self.be.ready(tok):
                keep.append(ent)
                continue
            e, x = self.be.fetch(tok)
            r.result = {"mean": e[:d].copy(), "m2": e[d:2 * d].copy(),
                        "rec_mean": e[2 * d:3 * d].copy(), "rec_m2": e[3 * d:4 * d].copy()}
            if x is not None:
                r.result["x"] = x
            r.finished = finish_time(tok)
            out.append(r)
        self.retiring = keep
        return out

    def tick(self, now_fn, finish_time) -> list:
        """Admits, advances every admitted request by one iteration, starts
        retiring the finished ones; returns the requests whose results have
        arrived on the host."""
        self._admit(now_fn())
        if self.gauss or self.logreg:
            self.be.step(bool(self.gauss), [ent[1] for ent in self.logreg.values()])
            self.iters_done += len(self.gauss) + len(self.logreg)
        for slot, ent in list(self.gauss.items()):
            ent[1] -= 1
            if ent[1] == 0:
                r = ent[0]
                self.retiring.append([r, self.be.retire_slot(slot, r), r.d])
                self.free.append(slot)
                del self.gauss[slot]
                self.used -= request_bytes(r)
        for rid, ent in list(self.logreg.items()):
            ent[2] -= 1
            if ent[2] == 0:
                r = ent[0]
                self.retiring.append([r, self.be.retire_context(ent[1], r), r.d])
                del self.logreg[rid]
                self.used -= request_bytes(r)
        return self._collect(finish_time)

    # --------------------------------------------------------------------- run
    def run(self, requests: list, *, clock: str = "wall") -> dict:
        """Serves ``requests`` (arrival times in seconds, or in ticks with
        clock="tick") to completion; returns latency and throughput figures.
        With the wall clock a request finishes when its results reach the
        host (device event time); with the tick clock, at the tick whose
        collection found them there."""
        for r in sorted(requests, key=lambda q: (q.arrival, q.rid)):
            self.submit(r)
        ticks = [0]
        self.be.start()
        t0 = time.perf_counter()
        if clock == "tick":
            def now():
                return float(ticks[0])

            def finish_time(tok):
                return float(ticks[0])
        else:
            def now():
                return time.perf_counter() - t0

            finish_time = self.be.elapsed
        finished = []
        while len(finished) < len(requests):
            if not self.busy() and self.queue and self.queue[0].arrival > now():
                if clock == "tick":
                    ticks[0] = int(math.ceil(self.queue[0].arrival))
                else:
                    time.sleep(min(1e-3, max(0.0, self.queue[0].arrival - now())))
                continue
            if not (self.gauss or self.logreg) and self.retiring:
                self.be.wait(self.retiring[0][1])
            finished += self.tick(now, finish_time)
            ticks[0] += 1
        self.be.finish()
        wall = time.perf_counter() - t0
        lat = sorted(r.latency for r in finished)
        iters = sum(r.iters for r in finished)

        def pct(p):
            return lat[min(len(lat) - 1, int(round(p / 100.0 * (len(lat) - 1))))]

        return {"requests": len(finished), "wall_s": wall, "sampler_iters": iters,
                "sampler_iters_per_s": iters / wall, "p50_latency": pct(50),
                "p99_latency": pct(99), "ticks": ticks[0]}
