"""The serving scheduler without a GPU.

A backend that runs every request on the CPU oracle stands in for the device,
so the scheduler's own logic is checked on the host: first-come-first-served
admission under the slot count and the HBM budget (a request that does not fit
holds back the ones behind it; logistic-regression requests take no batch
slot), retirement that frees slot and bytes at the request's last tick, the
tick accounting of latencies, and that every request is advanced exactly its
own number of iterations (its result equals the same request run alone).
"""
import math
import time

import numpy as np
import pytest

import oracle as O
from paper_1905_10252_amd import inputs as I
from paper_1905_10252_amd import serve


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def oracle_sampler(r):
    p = r.params
    if r.kind == "gauss":
        s = O.Sampler(r.n, r.d, O.T_GAUSS_CHOL, seed=r.seed, sampler_id=r.sampler_id,
                      rw_sd=p["rw_sd"], init_mean=p.get("init_mean", 0.0),
                      init_sd=p.get("init_sd", 3.0), mean=p["mean"], chol=p["chol"],
                      mode=p.get("mode", O.MODE_AUTO))
    else:
        s = O.Sampler(r.n, r.d, O.T_LOGREG, seed=r.seed, sampler_id=r.sampler_id,
                      rw_sd=p["rw_sd"], init_sd=math.sqrt(p["prior_var"]), X=p["X"], y=p["y"],
                      prior_var=p["prior_var"], mode=p.get("mode", O.MODE_AUTO))
    s.init()
    return s


class OracleBackend:
    """The backend interface of serve.Server over oracle samplers.  Results
    reach the 'host' ``lag`` readiness polls after retirement (wait() makes
    them ready at the next poll)."""

    def __init__(self, capacity, lag=0):
        self.capacity = capacity
        self.lag = lag
        self.slots = {}
        self.open_contexts = 0
        self.steps = 0
        self.t0 = time.perf_counter()

    def attach(self, slot, r):
        assert 0 <= slot < self.capacity and slot not in self.slots, slot
        assert r.kind == "gauss"
        self.slots[slot] = [oracle_sampler(r), None]

    def open(self, r):
        assert r.kind == "logreg"
        self.open_contexts += 1
        return [oracle_sampler(r), None]

    def step(self, batch, contexts):
        assert batch == bool(self.slots)
        self.steps += 1
        for ent in list(self.slots.values()) + list(contexts):
            ent[1] = ent[0].step()

    def _token(self, ent):
        out = ent[1]
        est = np.concatenate([out["mean"], out["m2"], out["rec_mean"], out["rec_m2"]])
        return {"est": est, "x": ent[0].x.copy(), "polls": 0, "t": None}

    def retire_slot(self, slot, r):
        return self._token(self.slots.pop(slot))

    def retire_context(self, ent, r):
        self.open_contexts -= 1
        return self._token(ent)

    def ready(self, tok):
        tok["polls"] += 1
        if tok["polls"] > self.lag and tok["t"] is None:
            tok["t"] = time.perf_counter() - self.t0
        return tok["polls"] > self.lag

    def wait(self, tok):
        tok["polls"] = max(tok["polls"], self.lag)

    def fetch(self, tok):
        return tok["est"], tok["x"]

    def start(self):
        self.t0 = time.perf_counter()

    def elapsed(self, tok):
        return tok["t"]

    def finish(self):
        pass


def gauss(rid, n, d, iters, arrival, seed=0):
    mean, U, _ = I.wishart_target(d, np.random.default_rng(100 + rid + seed))
    return serve.Request(rid, "gauss", n, d, iters, float(arrival), seed=(seed << 32) + rid,
                         sampler_id=rid, params=dict(mean=mean, chol=U, rw_sd=0.5 / math.sqrt(d),
                                                     init_sd=3.0))


def logreg(rid, n, d, m, iters, arrival, seed=0):
    X, y, _ = I.logreg_data(m, d, 500 + rid + seed)
    return serve.Request(rid, "logreg", n, d, iters, float(arrival), seed=(seed << 32) + rid,
                         sampler_id=rid, params=dict(X=X.astype(np.float64), y=y,
                                                     prior_var=10.0, rw_sd=0.05))


def alone(r):
    s = oracle_sampler(r)
    for _ in range(r.iters):
        out = s.step()
    return s.x, out


def check_alone(r):
    x, out = alone(r)
    assert np.array_equal(bits(r.result["x"]), bits(x)), r.rid
    for k in ("mean", "m2", "rec_mean", "rec_m2"):
        assert np.array_equal(bits(r.result[k]), bits(out[k])), (r.rid, k)


def mixed_stream(count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(count):
        arrival = int(rng.integers(0, 12))
        iters = int(rng.integers(1, 6))
        if k % 4 == 3:
            reqs.append(logreg(k, int(rng.integers(16, 97)), int(rng.integers(2, 5)),
                               int(rng.integers(16, 49)), iters, arrival, seed))
        else:
            reqs.append(gauss(k, int(rng.integers(1, 400)), int(rng.integers(1, 7)), iters,
                              arrival, seed))
    return reqs


@pytest.mark.parametrize("lag", [0, 1, 3])
def test_scheduler_mixed_stream(lag):
    reqs = mixed_stream(20, seed=lag + 1)
    budget = int(2.5 * max(serve.request_bytes(r) for r in reqs))
    be = OracleBackend(3, lag=lag)
    srv = serve.Server(capacity=3, hbm_budget=budget, backend=be)
    stats = srv.run(reqs, clock="tick")
    assert stats["requests"] == len(reqs)
    assert stats["sampler_iters"] == sum(r.iters for r in reqs) == srv.iters_done
    assert srv.peak_used <= budget and srv.peak_active > 1
    assert srv.used == 0 and not srv.busy() and sorted(srv.free) == [0, 1, 2]
    assert not be.slots and be.open_contexts == 0
    order = sorted(reqs, key=lambda q: (q.arrival, q.rid))
    for a, b in zip(order, order[1:]):
        assert a.admitted <= b.admitted          # first come, first served
    for r in reqs:
        assert r.admitted >= r.arrival
        # steps at ticks admitted .. admitted + iters - 1; results polled from
        # the next tick on (or waited for when nothing else runs)
        if lag == 0:
            assert r.finished == r.admitted + r.iters - 1, r.rid
        else:
            assert r.admitted + r.iters <= r.finished <= r.admitted + r.iters - 1 + lag, r.rid
        check_alone(r)


def test_budget_holds_back_the_queue_in_order():
    big1, big2 = gauss(0, 2000, 2, 3, 0), gauss(1, 2000, 2, 2, 0)
    small = gauss(2, 10, 1, 1, 1)
    budget = serve.request_bytes(big1) + serve.request_bytes(small)
    assert budget < serve.request_bytes(big1) + serve.request_bytes(big2)
    srv = serve.Server(capacity=2, hbm_budget=budget, backend=OracleBackend(2))
    srv.run([small, big2, big1], clock="tick")
    # big2 waits for big1's bytes; small would fit beside big1 but queues behind big2
    assert (big1.admitted, big1.finished) == (0, 2)
    assert (big2.admitted, big2.finished) == (3, 4)
    assert (small.admitted, small.finished) == (3, 3)
    assert srv.peak_used == serve.request_bytes(big2) + serve.request_bytes(small)
    for r in (big1, big2, small):
        check_alone(r)


def test_logistic_requests_take_no_slot():
    g1, lr, g2 = gauss(0, 50, 3, 2, 0), logreg(1, 40, 3, 32, 4, 0), gauss(2, 60, 2, 2, 0)
    srv = serve.Server(capacity=1, hbm_budget=1 << 30, backend=OracleBackend(1))
    srv.run([g1, lr, g2], clock="tick")
    assert (g1.admitted, g1.finished) == (0, 1)
    assert (lr.admitted, lr.finished) == (0, 3)
    assert (g2.admitted, g2.finished) == (2, 3)
    assert srv.peak_active == 2
    for r in (g1, lr, g2):
        check_alone(r)


def test_idle_gaps_jump_to_the_next_arrival():
    a, b = gauss(0, 20, 1, 2, 0), gauss(1, 20, 1, 1, 40.5)
    srv = serve.Server(capacity=2, hbm_budget=1 << 30, backend=OracleBackend(2, lag=2))
    be = srv.be
    stats = srv.run([a, b], clock="tick")
    assert (a.admitted, b.admitted) == (0, 41)
    assert b.finished == 42                 # waited for: nothing else runs
    assert be.steps == 3 and stats["ticks"] == 43


def test_wall_clock_run_and_oversized_request():
    reqs = [gauss(k, 30 + k, 1 + k % 3, 2, 1e-3 * k) for k in range(5)]
    srv = serve.Server(capacity=2, hbm_budget=1 << 30, backend=OracleBackend(2, lag=1))
    stats = srv.run(reqs)
    assert stats["requests"] == 5 and stats["p99_latency"] >= stats["p50_latency"] >= 0.0
    for r in reqs:
        assert r.finished >= 0.0
        check_alone(r)
    big = gauss(9, 1 << 16, 4, 5, 0.0)
    with pytest.raises(ValueError):
        serve.Server(capacity=2, hbm_budget=1 << 20, backend=OracleBackend(2)).submit(big)
