"""Benchmark: resample + redistribute at N = 2^24 particles (d = 16 FP32).

One step = smc_resample (exact max, 64-bit fixed-point weights with a
tile-local prefix scan and one pass over the tile totals, integer ESS
decision) + smc_redistribute (merge-path expand writing the new particle array
and int64 ncopies) on one batch of synthetic log-weights.
Steps cycle through the log-weight scales s = 0.5, 2, 8 (mild to heavy
degeneracy), resampling forced.  Inputs are resident in HBM before timing.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
EXPAND_SRC = os.path.join(ROOT, "paper_1905_10252_amd", "csrc", "k_expand.hip")
COUNTERS = os.path.join(ROOT, "profiles", "k_expand_N2e24_hbm_counters.md")


def expand_traffic():
    """HBM bytes per expand launch from the committed rocprofv3 counter summary,
    or None when that summary was taken on another version of the kernel."""
    import hashlib
    if not os.path.exists(COUNTERS):
        return None
    digest = hashlib.sha256(open(EXPAND_SRC, "rb").read()).hexdigest()
    text = open(COUNTERS).read()
    src = [l.split("`")[1] for l in text.splitlines() if l.startswith("- source sha256:")]
    tot = [l.split("`")[1] for l in text.splitlines() if l.startswith("- traffic bytes per launch:")]
    if not src or not tot or src[0] != digest:
        return None
    return int(tot[0])


def progress(msg):
    """A progress line on stderr (the result goes to stdout as one JSON line)."""
    sys.stderr.write("bench: %s (%.1f s)\n" % (msg, time.perf_counter() - T_START))
    sys.stderr.flush()


T_START = time.perf_counter()


def pctl(v, q):
    v = sorted(v)
    if not v:
        return None
    i = min(len(v) - 1, max(0, int(round(q / 100.0 * (len(v) - 1)))))
    return v[i]


def cpu_baseline(budget_s: float = 10.0, max_calls: int = 12):
    """The plain single-threaded oracle on full-size inputs, cycling over the
    scales until the budget is spent (bounded sample)."""
    import oracle as O
    from paper_1905_10252_amd import inputs as I
    n, d = I.RESAMPLE_N, I.RESAMPLE_D
    x = I.particles(n, d, I.X_SEED)
    r = I.offset_word(I.R_SEED)
    lws = {s: I.logw_normal(n, s, I.LOGW_SEEDS[s]) for s in I.RESAMPLE_SCALES}
    done, spent, calls = 0, 0.0, 0
    while spent < budget_s and calls < max_calls:
        s = I.RESAMPLE_SCALES[calls % len(I.RESAMPLE_SCALES)]
        t0 = time.perf_counter()
        nc, _ = O.resample(lws[s], r, O.MODE_FORCE)
        O.redistribute(nc, x)
        spent += time.perf_counter() - t0
        done += n
        calls += 1
    return {"value": done / spent, "unit": "resampled particles/s", "cores": 1, "kind": "oracle",
            "sample": "%d full-size calls (N=2^24, d=16, s cycled over %s), %.1f s"
                      % (calls, "/".join("%g" % s for s in I.RESAMPLE_SCALES), spent)}


def cpu_openmp(budget_s: float = 4.0, max_calls: int = 30):
    """The same resample + redistribute on every host core (OpenMP build of the
    exact-integer systematic path, ``baseline/``), full-size inputs cycling
    over the scales; a comparison point beside the single-core oracle."""
    import baseline as B
    from paper_1905_10252_amd import inputs as I
    n, d = I.RESAMPLE_N, I.RESAMPLE_D
    x = I.particles(n, d, I.X_SEED)
    r = I.offset_word(I.R_SEED)
    lws = {s: I.logw_normal(n, s, I.LOGW_SEEDS[s]) for s in I.RESAMPLE_SCALES}
    ws = B.Workspace(n, x.shape[1:], x.dtype)
    B.resample_redistribute(lws[I.RESAMPLE_SCALES[0]], r, x, ws)  # first touch of the outputs
    done, spent, calls = 0, 0.0, 0
    while spent < budget_s and calls < max_calls:
        s = I.RESAMPLE_SCALES[calls % len(I.RESAMPLE_SCALES)]
        t0 = time.perf_counter()
        B.resample_redistribute(lws[s], r, x, ws)
        spent += time.perf_counter() - t0
        done += n
        calls += 1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    # the logistic-regression likelihood (the cost of one iteration of that
    # sampler) on a subset of the particles, extrapolated to N = 2^16
    import numpy as np
    c = I.LOGREG
    X, y, _ = I.logreg_data(c["m_rows"], c["d"], 200)
    sub = 1024
    th = np.random.default_rng(1).standard_normal((sub, c["d"])) * 0.3
    t0 = time.perf_counter()
    B.logreg_loglik(th, X, y)
    t_sub = time.perf_counter() - t0
    per_iter = t_sub * c["n"] / sub
    return {"value": done / spent, "unit": "resampled particles/s", "cores": B.threads(),
            "kind": "openmp", "cpu": model, "nproc": os.cpu_count(),
            "sample": "%d full-size calls (N=2^24, d=16, s cycled over %s), %.2f s"
                      % (calls, "/".join("%g" % s for s in I.RESAMPLE_SCALES), spent),
            "logreg_f64": {"s_per_iter_extrapolated": round(per_iter, 2),
                           "iters_per_s": round(1.0 / per_iter, 4),
                           "sample": "FP64 likelihood of %d of the N=2^16 particles (M=65536, "
                                     "D=32) in %.2f s, scaled by %d" % (sub, t_sub, c["n"] // sub)}}


def sampler_metrics(dev):
    """SMC iterations per second of whole smc_step iterations (Alg 2) on three
    workloads; each timed with events around whole runs after warm-up."""
    import math
    import numpy as np
    import torch
    from paper_1905_10252_amd import inputs as I
    from paper_1905_10252_amd import smc
    out = {}

    def timed_steps(S, k):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
        ev[0].record()
        for i in range(k):
            S.step(info=False, est=False)
            ev[i + 1].record()
        torch.cuda.synchronize()
        per = [ev[i].elapsed_time(ev[i + 1]) for i in range(k)]
        return ev[0].elapsed_time(ev[k]), per

    # 1-D Gaussian N(2,1), N = 1024, 20 iterations per run
    g = I.GAUSS1D
    runs, tot, lat = 10, 0.0, []
    for rep in range(runs + 2):
        S = smc.Sampler(g["n"], 1, "gauss", seed=rep, rw_sd=g["rw_sd"], init_sd=g["init_sd"],
                        mean=g["mean"], var=g["var"], device=dev)
        torch.cuda.synchronize()
        ms, per = timed_steps(S, g["iters"])
        if rep >= 2:
            tot += ms
            lat += per
    # the launch floor: one trivial kernel per step, timed the same way
    one = torch.zeros(1, device=dev)
    for _ in range(20):
        one.add_(1.0)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(201)]
    ev[0].record()
    for i in range(200):
        one.add_(1.0)
        ev[i + 1].record()
    torch.cuda.synchronize()
    floor = [ev[i].elapsed_time(ev[i + 1]) for i in range(200)]
    out["gauss1d_N1024"] = {"iters_per_s": round(runs * g["iters"] / (tot / 1e3), 1),
                            "us_per_iter": round(1e3 * tot / (runs * g["iters"]), 2),
                            "p50_us": round(1e3 * pctl(lat, 50), 2),
                            "p99_us": round(1e3 * pctl(lat, 99), 2),
                            "one_trivial_launch_p50_us": round(1e3 * pctl(floor, 50), 2)}
    # the paper's sampler workload: Student-t target (nu = 5, mu = 1), resampling
    # every iteration, T = 100 iterations, N = 2^10, 2^17 and 2^24
    for lg in (10, 17, 24):
        n = 1 << lg
        S = smc.Sampler(n, 1, "student", seed=1, rw_sd=0.5, nu=5.0, mu=1.0,
                        mode=smc.L.MODE_FORCE, device=dev)
        timed_steps(S, 3)
        ms, per = timed_steps(S, 100)
        out["student_t_N2e%d_force" % lg] = {"iters_per_s": round(100 / (ms / 1e3), 2),
                                             "ms_per_iter": round(ms / 100, 4),
                                             "particles_per_s": round(100 * n / (ms / 1e3), 1),
                                             "p50_ms": round(pctl(per, 50), 4),
                                             "p99_ms": round(pctl(per, 99), 4)}
        del S
    n = 1 << 24
    # the same with the lazy reset (weights marked uniform instead of written)
    S = smc.Sampler(n, 1, "student", seed=1, rw_sd=0.5, nu=5.0, mu=1.0, mode=smc.L.MODE_FORCE,
                    lazy_reset=True, device=dev)
    timed_steps(S, 3)
    ms, per = timed_steps(S, 100)
    out["student_t_N2e24_force"]["lazy_reset"] = {"ms_per_iter": round(ms / 100, 4),
                                                  "particles_per_s": round(100 * n / (ms / 1e3), 1)}
    del S
    # SIR particle filter (Alg 1), bearing-only tracking, N = 2^24, 50 updates
    B = I.BEARING
    _, ys = I.bearing_track(60, 7)
    S = smc.Sampler(n, 4, "bearing", seed=2, mean=B["x0"], init_sd=B["init_sd"], obs=ys,
                    delta=B["delta"], obs_var=B["obs_var"], device=dev)
    timed_steps(S, 3)
    ms, per = timed_steps(S, 50)
    out["bearing_pf_N2e24"] = {"iters_per_s": round(50 / (ms / 1e3), 2),
                               "ms_per_iter": round(ms / 50, 4),
                               "particles_per_s": round(50 * n / (ms / 1e3), 1),
                               "p50_ms": round(pctl(per, 50), 4),
                               "p99_ms": round(pctl(per, 99), 4)}
    del S
    S = smc.Sampler(n, 4, "bearing", seed=2, mean=B["x0"], init_sd=B["init_sd"], obs=ys,
                    delta=B["delta"], obs_var=B["obs_var"], lazy_reset=True, device=dev)
    timed_steps(S, 3)
    ms, per = timed_steps(S, 50)
    out["bearing_pf_N2e24"]["lazy_reset"] = {"ms_per_iter": round(ms / 50, 4),
                                             "particles_per_s": round(50 * n / (ms / 1e3), 1)}
    del S
    # Bayesian logistic regression: M = 65536, D = 32, N = 2^16
    c = I.LOGREG
    X, y, _ = I.logreg_data(c["m_rows"], c["d"], 200)
    for prec, k in (("bf16", 20), ("f64", 6)):
        S = smc.Sampler(c["n"], c["d"], "logreg", X=X.astype(np.float64), y=y,
                        prior_var=c["prior_var"], precision=prec, rw_sd=c["rw_sd"],
                        init_sd=math.sqrt(c["prior_var"]), device=dev)
        timed_steps(S, 1)
        ms, per = timed_steps(S, k)
        out["logreg_%s" % prec] = {"iters_per_s": round(k / (ms / 1e3), 2),
                                   "ms_per_iter": round(ms / k, 3),
                                   "p50_ms": round(pctl(per, 50), 4),
                                   "p99_ms": round(pctl(per, 99), 4)}
        del S
    progress("sampler workloads timed")
    out["logreg_bf16"]["vs_f64"] = logreg_precision_gap(dev)
    progress("logistic regression in both precisions")
    out["batch256"] = batch_metrics(dev, timed_steps)
    progress("batched samplers")
    out["serving"] = serve_metrics(dev)
    progress("serving")
    return out


def logreg_precision_gap(dev):
    """The configured logistic-regression run (N = 2^16, M = 65536, D = 32, 50
    iterations, ESS-triggered resampling) in both precisions from the same
    seed.  Reported: the BF16 likelihood's error against the FP64 one on the
    final BF16 population (every particle, the per-step comparison that
    matters: the two runs' trajectories part at the first resampling with
    different weights), how often each run resampled and its last ESS, and the
    posterior-mean estimates of both runs against each other and against the
    data's true coefficients, in units of the Laplace posterior standard
    deviation at those coefficients (host FP64: the inverse of
    X^T diag(p(1 - p)) X + I / prior_var)."""
    import math
    import numpy as np
    import torch
    from paper_1905_10252_amd import inputs as I
    from paper_1905_10252_amd import smc
    c = I.LOGREG
    X, y, theta_star = I.logreg_data(c["m_rows"], c["d"], 200)
    Xd = X.astype(np.float64)
    d = c["d"]
    z = Xd @ theta_star
    p = 1.0 / (1.0 + np.exp(-z))
    H = (Xd * (p * (1.0 - p))[:, None]).T @ Xd + np.eye(d) / c["prior_var"]
    lap_sd = np.sqrt(np.diag(np.linalg.inv(H)))
    runs = {}
    for prec in ("bf16", "f64"):
        S = smc.Sampler(c["n"], d, "logreg", X=Xd, y=y, seed=5, prior_var=c["prior_var"],
                        precision=prec, rw_sd=c["rw_sd"], init_sd=math.sqrt(c["prior_var"]),
                        device=dev)
        out = S.steps(c["iters"], info=True, est=True)
        e = out["est"][-1].cpu().numpy()
        runs[prec] = {"mean": e[:d], "resampled": sum(i["resampled"] for i in out["info"]),
                      "ess_last": out["info"][-1]["ess"], "S": S}
    b, f = runs["bf16"], runs["f64"]
    th = b["S"].x
    lb = b["S"].log_target(th).cpu().numpy()
    lf = f["S"].log_target(th).cpu().numpy()
    rel = np.abs(lb - lf) / np.abs(lf)
    res = {"iterations": c["iters"],
           "loglik_rel_err_max": float(rel.max()),
           "loglik_rel_err_median": float(np.median(rel)),
           "loglik_abs_err_nats_median": float(np.median(np.abs(lb - lf))),
           "loglik_abs_err_nats_max": float(np.abs(lb - lf).max()),
           "resampled": {"bf16": b["resampled"], "f64": f["resampled"]},
           "ess_last": {"bf16": round(b["ess_last"], 2), "f64": round(f["ess_last"], 2)},
           "laplace_sd_median": float(np.median(lap_sd)),
           "mean_gap_bf16_f64_laplace_sd": {
               "max": round(float(np.max(np.abs(b["mean"] - f["mean"]) / lap_sd)), 3),
               "median": round(float(np.median(np.abs(b["mean"] - f["mean"]) / lap_sd)), 3)},
           "mean_to_truth_laplace_sd_median": {
               "bf16": round(float(np.median(np.abs(b["mean"] - theta_star) / lap_sd)), 3),
               "f64": round(float(np.median(np.abs(f["mean"] - theta_star) / lap_sd)), 3)}}
    del runs, b, f
    torch.cuda.synchronize()
    return res


def serve_metrics(dev, count=None, sequential=60):
    """Continuous-batching server on the configured stream of mixed requests
    (2000 Gaussian and logistic-regression samplers, N up to 2^20, 20-100
    iterations): capacity from a closed loop (all requests queued at the
    start), then an open loop with Poisson arrivals at 0.7 x capacity (p50/p99
    latency, aggregate sampler-iterations/s); and on the first ``sequential``
    requests, the server against serving them one at a time with per-request
    launches.  The request descriptions are drawn once (unit-rate arrival
    gaps) and the gaps scaled to each rate."""
    import time
    import torch
    from paper_1905_10252_amd import inputs as I
    from paper_1905_10252_amd import serve, smc

    count = I.SERVE["requests"] if count is None else count
    base = I.serve_requests(count, 1.0)

    def reqs(rate, k=count):
        out = []
        for i, r in enumerate(base[:k]):
            r = dict(r)
            r["arrival"] = r["arrival"] / rate if rate > 0 else 0.0
            out.append(serve.Request(i, **r))
        return out

    def server():
        return serve.Server(capacity=256, hbm_budget=96 << 30, device=dev)

    res = {"requests": count}
    closed = server().run(reqs(0.0))
    cap = closed["requests"] / closed["wall_s"]
    res["closed_loop"] = {k: round(v, 4) if isinstance(v, float) else v for k, v in closed.items()}
    res["capacity_req_per_s"] = round(cap, 2)
    opened = server().run(reqs(0.7 * cap))
    res["open_loop_0.7"] = {k: round(v, 4) if isinstance(v, float) else v
                            for k, v in opened.items()}
    torch.cuda.synchronize()
    # one at a time, each request on its own launches, against the server
    sub = reqs(0.0, sequential)
    t0 = time.perf_counter()
    for r in sub:
        p = r.params
        if r.kind == "gauss":
            b = smc.Batch(1, graph=False, device=dev)
            b.attach(0, r.n, r.d, p["mean"], p["chol"], seed=r.seed, sampler_id=r.sampler_id,
                     rw_sd=p["rw_sd"], init_sd=p["init_sd"])
            for _ in range(r.iters):
                b.step(info=False, est=True)
        else:
            s_ = smc.Sampler(r.n, r.d, "logreg", seed=r.seed, sampler_id=r.sampler_id, X=p["X"],
                             y=p["y"], prior_var=p["prior_var"], precision="bf16",
                             rw_sd=p["rw_sd"], init_sd=p["prior_var"] ** 0.5, device=dev)
            for _ in range(r.iters):
                s_.step(info=False, est=True)
        torch.cuda.synchronize()
    seq_wall = time.perf_counter() - t0
    seq_iters = sum(r.iters for r in sub)
    batched = server().run(reqs(0.0, sequential))
    res["subset"] = {"requests": sequential,
                     "one_at_a_time_sampler_iters_per_s": round(seq_iters / seq_wall, 1),
                     "server_sampler_iters_per_s": round(batched["sampler_iters_per_s"], 1),
                     "speedup": round(batched["sampler_iters_per_s"] / (seq_iters / seq_wall), 2)}
    return res


def batch_metrics(dev, timed_steps):
    """256 Gaussian samplers (N log-uniform 2^8..2^16, d 1..64, Wishart
    covariances, ESS-triggered resampling): one batched step per iteration
    (graph replay) against per-sampler launch sequences, eager and graphed.
    Rates are sampler-iterations per second."""
    import torch
    from paper_1905_10252_amd import inputs as I
    from paper_1905_10252_amd import smc
    specs = I.batch_specs()
    ns = len(specs)

    def make(group, graph):
        b = smc.Batch(len(group), graph=graph, device=dev)
        for k, sp in enumerate(group):
            b.attach(k, sp["n"], sp["d"], sp["mean"], sp["chol"], seed=sp["seed"],
                     sampler_id=sp["sampler_id"], rw_sd=sp["rw_sd"], init_sd=sp["init_sd"])
        return b

    from paper_1905_10252_amd import tune
    res = {"samplers": ns, "particles": int(sum(sp["n"] for sp in specs)),
           "mean_d": round(sum(sp["d"] for sp in specs) / ns, 2)}
    tuned = tune.tune_group(specs, device=dev, use_cache=False)
    tb = tune.tune_buckets(specs, device=dev, pairs=tuned["best"], use_cache=False)
    res["unit_pairs"] = tuned["best"]
    res["tuning_ms_per_step"] = {str(g): round(v, 4) for g, v in tuned["ms"].items()}
    res["bucket_waves"] = {str(q): w for q, w in tb["best"].items()}
    res["bucket_tuning_ms_per_step"] = {str(q): {str(w): round(t, 4) for w, t in m.items()}
                                        for q, m in tb["ms"].items()}
    b = make(specs, True)
    tune.apply(b, tuned, tb)
    timed_steps(b, 4)  # the third eager step captures the graph
    k = 20
    ms, per = timed_steps(b, k)
    res.update({"sampler_iters_per_s": round(k * ns / (ms / 1e3), 1),
                "ms_per_step": round(ms / k, 4), "p50_ms": round(pctl(per, 50), 4),
                "p99_ms": round(pctl(per, 99), 4)})
    del b
    torch.cuda.synchronize()
    for name, graph in (("per_sampler_eager", False), ("per_sampler_graph", True)):
        bs = [make([sp], graph) for sp in specs]
        for _ in range(4):
            for one in bs:
                one.step(info=False, est=False)
        torch.cuda.synchronize()
        rounds = 5
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(rounds):
            for one in bs:
                one.step(info=False, est=False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        res[name] = {"sampler_iters_per_s": round(rounds * ns / (ms / 1e3), 1),
                     "ms_per_round": round(ms / rounds, 3)}
        del bs
        torch.cuda.synchronize()
    res["speedup_vs_eager"] = round(res["sampler_iters_per_s"]
                                    / res["per_sampler_eager"]["sampler_iters_per_s"], 2)
    return res


def only_workload(name, steps, warmup):
    """One sampler workload alone (a profiling target): the Student-t sampler
    or the bearing-only filter at N = 2^24 with resampling every iteration,
    the logistic-regression sampler (N = 2^16, M = 65536, D = 32) with a BF16 or
    FP64 likelihood, or one batched step of the 256-sampler workload; prints ms
    per iteration."""
    import math
    import numpy as np
    import torch
    from paper_1905_10252_amd import inputs as I
    from paper_1905_10252_amd import smc
    dev = torch.device("cuda:0")
    n = 1 << 24
    if name == "student":
        S = smc.Sampler(n, 1, "student", seed=1, rw_sd=0.5, nu=5.0, mu=1.0,
                        mode=smc.L.MODE_FORCE, device=dev)
    elif name.startswith("logreg"):
        c = I.LOGREG
        X, y, _ = I.logreg_data(c["m_rows"], c["d"], 200)
        S = smc.Sampler(c["n"], c["d"], "logreg", X=X.astype(np.float64), y=y,
                        prior_var=c["prior_var"], precision=name.split("_")[1], rw_sd=c["rw_sd"],
                        init_sd=math.sqrt(c["prior_var"]), device=dev)
    elif name == "bearing":
        B = I.BEARING
        _, ys = I.bearing_track(warmup + steps + 1, 7)
        S = smc.Sampler(n, 4, "bearing", seed=2, mean=B["x0"], init_sd=B["init_sd"], obs=ys,
                        delta=B["delta"], obs_var=B["obs_var"], mode=smc.L.MODE_FORCE, device=dev)
    else:
        specs = I.batch_specs()
        S = smc.Batch(len(specs), graph=False, device=dev)
        for k, sp in enumerate(specs):
            S.attach(k, sp["n"], sp["d"], sp["mean"], sp["chol"], seed=sp["seed"],
                     sampler_id=sp["sampler_id"], rw_sd=sp["rw_sd"], init_sd=sp["init_sd"])
    for _ in range(warmup):
        S.step(info=False, est=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        S.step(info=False, est=False)
    e1.record()
    torch.cuda.synchronize()
    print(json.dumps({"workload": name, "steps": steps,
                      "ms_per_iter": round(e0.elapsed_time(e1) / steps, 4)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baselines (oracle and OpenMP)")
    ap.add_argument("--no-samplers", action="store_true", help="skip the smc_step workloads")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after timing, run one plain device copy of the 1 GiB particle array "
                         "(reference for hardware byte counters)")
    ap.add_argument("--only", choices=("student", "bearing", "batch", "logreg_bf16", "logreg_f64"), default=None,
                    help="run only --steps iterations of one sampler workload (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one GPU only (the resample hot path on one "
              "MI355X); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.only:
        only_workload(args.only, args.steps, args.warmup)
        return

    import numpy as np
    import torch

    from paper_1905_10252_amd import inputs as I
    from paper_1905_10252_amd import smc

    dev = torch.device("cuda:0")
    n, d = I.RESAMPLE_N, I.RESAMPLE_D
    scales = I.RESAMPLE_SCALES
    lws = [torch.from_numpy(I.logw_normal(n, s, I.LOGW_SEEDS[s])).to(dev) for s in scales]
    x = torch.from_numpy(I.particles(n, d, I.X_SEED)).to(dev)
    x_out = torch.empty_like(x)
    ncopies = torch.empty(n, dtype=torch.int64, device=dev)
    r = I.offset_word(I.R_SEED)
    R = smc.Resampler(n, device=dev)
    FORCE = smc.L.MODE_FORCE

    def step(k, ev=None):
        lw = lws[k % len(scales)]
        if ev is not None:
            ev[0].record()
        R.resample(lw, r, FORCE, info=False)
        if ev is not None:
            ev[1].record()
        R.redistribute(x, x_out, ncopies_out=ncopies)
        if ev is not None:
            ev[2].record()

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    if R.sync_error() != 0:
        raise RuntimeError("device error during warmup")

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record()
    for k in range(args.steps):
        step(k, evs[k])
    stop.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(stop)
    step_ms = [e[0].elapsed_time(e[2]) for e in evs]
    res_ms = [e[0].elapsed_time(e[1]) for e in evs]
    exp_ms = [e[1].elapsed_time(e[2]) for e in evs]
    if R.sync_error() != 0:
        raise RuntimeError("device error during timing")
    if args.calib_copy:
        x_out.copy_(x)
        torch.cuda.synchronize()
    # measured stream-copy bandwidth of the 1 GiB particle array, outside the
    # timed region: the runtime's device copy, and torch's vectorised
    # elementwise kernel (x * 1); the faster is the reference
    def copy_rate(fn):
        ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        ce0.record()
        for _ in range(5):
            fn()
        ce1.record()
        torch.cuda.synchronize()
        return 2 * x.numel() * x.element_size() * 5 / (ce0.elapsed_time(ce1) / 1e3) / 1e9
    copy_rates = {"device_copy": copy_rate(lambda: x_out.copy_(x)),
                  "elementwise": copy_rate(lambda: torch.mul(x, 1.0, out=x_out))}
    copy_gbs = max(copy_rates.values())
    # sources that receive a copy, per scale (the strict read bound)
    uniq = []
    for i in range(len(scales)):
        step(i)
        uniq.append(int((ncopies > 0).sum().item()))

    per_s = {}
    for i, s in enumerate(scales):
        sel = [k for k in range(args.steps) if k % len(scales) == i]
        per_s["s=%g" % s] = {
            "ms_median": round(float(np.median([step_ms[k] for k in sel])), 4),
            "resample_ms": round(float(np.median([res_ms[k] for k in sel])), 4),
            "expand_ms": round(float(np.median([exp_ms[k] for k in sel])), 4),
        }
    ms_per_step = total_ms / args.steps
    value = n * args.steps / (total_ms / 1e3)

    # dominant kernel: the expand (smc_redistribute launches exactly one kernel).
    # Its algorithmic bytes are the strict ones: the ncopies write (8 B), the
    # new row (4d B) and the rows of the sources that receive a copy (4d B
    # each, u sources); reading every source row (dense, 8 + 8d B a particle)
    # is reported beside it as an upper bound only.
    exp_avg_s = float(np.mean(exp_ms)) / 1e3
    strict_b = {s: (8 + 4 * d) * n + 4 * d * u for s, u in zip(scales, uniq)}
    dense_b = (8 + 8 * d) * n
    sel = {s: [k for k in range(args.steps) if k % len(scales) == i] for i, s in enumerate(scales)}
    tot_strict = sum(strict_b[scales[k % len(scales)]] for k in range(args.steps))
    achieved = tot_strict / (float(np.sum(exp_ms)) / 1e3) / 1e9
    per_scale_roof = {}
    for i, s in enumerate(scales):
        t_s = float(np.mean([exp_ms[k] for k in sel[s]])) / 1e3
        a_s = strict_b[s] / t_s / 1e9
        per_scale_roof["s=%g" % s] = {
            "avg_launch_us": round(t_s * 1e6, 2), "unique_sources": uniq[i],
            "strict_bytes": int(strict_b[s]), "achieved": round(a_s, 1),
            "frac": round(a_s / HBM_PEAK_GBS, 4),
            "frac_of_copy": round(a_s / copy_gbs, 4)}
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": expand_traffic(),
                "kernel": "k_expand",
                "bytes": "strict: 8 + 4d + 4d*u/N per particle (ncopies write, new row, rows of "
                         "the u sources with ncopies > 0)",
                "avg_launch_us": round(exp_avg_s * 1e6, 2),
                "per_scale": per_scale_roof,
                "dense_upper_bound": {
                    "bytes_per_launch": dense_b,
                    "achieved": round(dense_b / exp_avg_s / 1e9, 1),
                    "frac": round(dense_b / exp_avg_s / 1e9 / HBM_PEAK_GBS, 4),
                    "note": "counts every source row as read; at s=8 most are not"}}
    # the whole call (resample + redistribute) per scale, on both byte counts:
    # strict 16 + 4d + 4d*u/N (log-weights read, ncopies write, new rows,
    # surviving rows), dense 16 + 8d (every row read)
    path = {}
    for i, s in enumerate(scales):
        t_s = float(np.median([step_ms[k] for k in sel[s]])) / 1e3
        ps = (16 + 4 * d) * n + 4 * d * uniq[i]
        pd = (16 + 8 * d) * n
        path["s=%g" % s] = {"ms_median": round(t_s * 1e3, 4),
                            "frac_strict": round(ps / t_s / 1e9 / HBM_PEAK_GBS, 4),
                            "frac_dense": round(pd / t_s / 1e9 / HBM_PEAK_GBS, 4),
                            "frac_strict_of_copy": round(ps / t_s / 1e9 / copy_gbs, 4)}
    path_bytes = (16 + 8 * d) * n  # logw read, ncopies write, row read + write
    out = {
        "metric": "resampled particles/s (resample+redistribute) @N=2^24",
        "value": round(value, 1), "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 weights, u64 fixed point, f32 rows",
        "data": "synthetic",
        "config": {"workload": "resample+redistribute N=2^24 d=16 fp32, logw~N(0,s^2), "
                               "s cycled over 0.5/2/8, systematic, forced",
                   "n": n, "d": d, "scales": list(scales)},
        "p50_ms": round(pctl(step_ms, 50), 4), "p99_ms": round(pctl(step_ms, 99), 4),
        "max_ms": round(max(step_ms), 4),
        "per_scale": per_s,
        "path_per_scale": path,
        "path_dense_frac": round(path_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "copy_GBs_measured": round(copy_gbs, 1),
        "copy_GBs_by_kernel": {k: round(v, 1) for k, v in copy_rates.items()},
        "wall_s": round(t_wall, 3),
        "roofline": roofline,
    }
    progress("resample + redistribute timed")
    if not args.no_samplers:
        out["smc_iters"] = sampler_metrics(dev)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
        progress("oracle on the host")
        out["cpu_openmp"] = cpu_openmp()
        progress("OpenMP baseline")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
