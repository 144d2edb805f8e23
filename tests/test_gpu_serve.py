"""The serving loop (continuous batching over the batched sampler): requests
arriving while others run are admitted as slots and the HBM budget free up,
and every request's result equals the same request run alone, bit for bit
(particles and estimates)."""
import numpy as np
import pytest

from paper_1905_10252_amd import inputs as I

pytestmark = pytest.mark.gpu


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def small_requests(serve):
    rng = np.random.default_rng(9)
    reqs = []
    for k in range(12):
        arrival = float(rng.integers(0, 8))
        iters = int(rng.integers(3, 9))
        if k % 3 == 2:
            d, n, m = int(rng.integers(8, 17)), int(rng.integers(256, 2049)), int(rng.integers(512, 2049))
            X, y, _ = I.logreg_data(m, d, 1000 + k)
            reqs.append(serve.Request(k, "logreg", n, d, iters, arrival, seed=77 + k, sampler_id=k,
                                      params=dict(X=X.astype(np.float64), y=y, prior_var=10.0,
                                                  rw_sd=0.01)))
        else:
            d, n = int(rng.integers(1, 21)), int(rng.integers(100, 5001))
            mean, U, _ = I.wishart_target(d, rng)
            reqs.append(serve.Request(k, "gauss", n, d, iters, arrival, seed=77 + k, sampler_id=k,
                                      params=dict(mean=mean, chol=U, rw_sd=0.5 / np.sqrt(d),
                                                  init_sd=3.0)))
    return reqs


def alone(smc, r, dev):
    p = r.params
    if r.kind == "gauss":
        b = smc.Batch(1, device=dev)
        b.attach(0, r.n, r.d, p["mean"], p["chol"], seed=r.seed, sampler_id=r.sampler_id,
                 rw_sd=p["rw_sd"], init_sd=p["init_sd"])
        for _ in range(r.iters):
            b.step(info=False, est=True)
        return {"x": b.x(0).cpu().numpy(), **b.estimates(0)}
    s = smc.Sampler(r.n, r.d, "logreg", seed=r.seed, sampler_id=r.sampler_id, X=p["X"], y=p["y"],
                    prior_var=p["prior_var"], precision="bf16", rw_sd=p["rw_sd"],
                    init_sd=np.sqrt(p["prior_var"]), device=dev)
    for _ in range(r.iters):
        s.step(info=False, est=True)
    return {"x": s.x.cpu().numpy(), **s.estimates()}


def test_serving_admits_under_budget_and_matches_alone(dev):
    print("serving mix", flush=True)
    from paper_1905_10252_amd import serve, smc
    reqs = small_requests(serve)
    budget = max(serve.request_bytes(r) for r in reqs) * 3
    srv = serve.Server(capacity=4, hbm_budget=budget, keep_particles=True, device=dev)
    stats = srv.run(reqs, clock="tick")
    assert stats["requests"] == len(reqs)
    assert srv.peak_used <= budget
    assert 1 < srv.peak_active
    assert srv.used == 0 and not srv.busy() and len(srv.free) == 4
    for r in reqs:
        assert r.admitted >= r.arrival
        assert r.finished - r.admitted >= r.iters - 1
    # wall-clock serving of the same stream gives the same estimates
    again = small_requests(serve)
    for r in again:
        r.arrival *= 1e-3  # ticks read as milliseconds
    serve.Server(capacity=4, hbm_budget=budget, device=dev).run(again)
    for a, b in zip(reqs, again):
        for k in ("mean", "m2", "rec_mean", "rec_m2"):
            assert np.array_equal(bits(a.result[k]), bits(b.result[k])), (a.rid, k)
    for r in reqs:
        ref = alone(smc, r, dev)
        assert np.array_equal(bits(r.result["x"]), bits(ref["x"])), r.rid
        for k in ("mean", "m2", "rec_mean", "rec_m2"):
            assert np.array_equal(bits(r.result[k]), bits(ref[k])), (r.rid, k)


def test_serving_rejects_oversized_request(dev):
    from paper_1905_10252_amd import serve
    srv = serve.Server(capacity=2, hbm_budget=1 << 20, device=dev)
    mean, U, _ = I.wishart_target(4, np.random.default_rng(1))
    r = serve.Request(0, "gauss", 1 << 16, 4, 5, 0.0, seed=1, sampler_id=0,
                      params=dict(mean=mean, chol=U, rw_sd=0.25, init_sd=3.0))
    with pytest.raises(ValueError):
        srv.submit(r)
