"""GPU parity of the batched sampler (include/smc_batch.h) against the CPU
oracle, sampler by sampler.

Particle rows and log-weights are fixed IEEE sequences (deterministic normals,
the quadratic form summed in index order) and resampling is integer-exact, so
they must match the oracle bit for bit; estimates, log Z and log c_t are FP64
sums in another order (1e-11 / 1e-10 relative).  A sampler's bits must not
depend on the other samplers of the batch, on graph replay, or on samplers
attached and detached around it.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1905_10252_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smc(dev):
    from paper_1905_10252_amd import smc as S
    return S


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def close(a, b, rtol):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1.0)) <= rtol


def spec(k, n, d, mode, seed=500):
    rng = np.random.default_rng(seed + k)
    mean, U, _ = I.wishart_target(d, rng)
    return dict(n=n, d=d, mean=mean, chol=U, rw_sd=0.5 / math.sqrt(d),
                seed=(seed << 32) + k, sampler_id=k, mode=mode)


def attach(B, slot, sp):
    B.attach(slot, sp["n"], sp["d"], sp["mean"], sp["chol"], seed=sp["seed"],
             sampler_id=sp["sampler_id"], rw_sd=sp["rw_sd"], init_mean=sp.get("init_mean", 0.0),
             init_sd=sp.get("init_sd", 3.0), mode=sp["mode"])


def oracle_of(B, slot, sp):
    desc = B.slots[slot]["desc"]
    o = O.Sampler(sp["n"], sp["d"], O.T_GAUSS_CHOL, seed=sp["seed"], sampler_id=sp["sampler_id"],
                  rw_sd=sp["rw_sd"], init_mean=sp.get("init_mean", 0.0),
                  init_sd=sp.get("init_sd", 3.0), mean=sp["mean"], chol=sp["chol"],
                  mode=sp["mode"], log_norm=desc.log_norm, init_log_norm=desc.init_log_norm)
    o.init()
    return o


def check_state(B, slot, o, where):
    assert np.array_equal(bits(B.x(slot).cpu().numpy()), bits(o.x)), where
    assert np.array_equal(bits(B.logw(slot).cpu().numpy()), bits(o.logw)), where


def check_step(B, slot, o, out, where):
    info = B.info(slot)
    for k in ("S", "U", "Q2_hi", "Q2_lo", "resampled", "err", "K"):
        assert info[k] == out["info"][k], (where, k, info[k], out["info"][k])
    check_state(B, slot, o, where)
    e = B.estimates(slot)
    assert close(e["mean"], out["mean"], 1e-11), where
    assert close(e["m2"], out["m2"], 1e-11), where
    assert close(e["rec_mean"], out["rec_mean"], 1e-10), where
    assert abs(info["log_c"] - out["log_c"]) <= 1e-10 * max(1.0, abs(out["log_c"])), where


# (n, d, mode): ragged tiles, every dimension bucket, all three triggers, and
# a 1-D sampler of odd N over several chunks (neighbours share a normal pair)
MIX = [(1, 1, O.MODE_AUTO), (255, 3, O.MODE_FORCE), (4096, 8, O.MODE_AUTO),
       (4097, 9, O.MODE_FORCE), (10000, 33, O.MODE_AUTO), (20000, 64, O.MODE_NEVER),
       (7000, 17, O.MODE_FORCE), (3000, 56, O.MODE_AUTO), (4099, 1, O.MODE_FORCE)]
SLOTS = [3, 0, 9, 1, 5, 2, 4, 7, 8]


def test_batch_mix_bit_exact_vs_oracle(smc, dev):
    print("batch mix", flush=True)
    B = smc.Batch(10, device=dev)
    specs = [spec(k, *m) for k, m in enumerate(MIX)]
    for slot, sp in zip(SLOTS, specs):
        attach(B, slot, sp)
    assert B.counts()[0] == len(MIX)
    orcs = {slot: oracle_of(B, slot, sp) for slot, sp in zip(SLOTS, specs)}
    for slot in SLOTS:
        check_state(B, slot, orcs[slot], ("init", slot))
    for t in range(1, 7):  # steps 3.. replay the captured graph
        B.step()
        for slot in SLOTS:
            check_step(B, slot, orcs[slot], orcs[slot].step(), (t, slot))
    for slot in SLOTS:
        assert B.sync_error(slot) == 0


def run_alone(smc, dev, sp, steps, graph=True):
    B = smc.Batch(1, graph=graph, device=dev)
    attach(B, 0, sp)
    for _ in range(steps):
        B.step()
    return B.x(0).cpu().numpy(), B.estimates(0)


def test_batch_results_independent_of_the_mix(smc, dev):
    print("batch alone vs mix", flush=True)
    specs = [spec(20 + k, *m) for k, m in enumerate(MIX)]
    B = smc.Batch(len(MIX), device=dev)
    for slot, sp in enumerate(specs):
        attach(B, slot, sp)
    for _ in range(5):
        B.step()
    for slot in (1, 4, 5):
        x, e = run_alone(smc, dev, specs[slot], 5, graph=(slot != 4))
        assert np.array_equal(bits(B.x(slot).cpu().numpy()), bits(x)), slot
        got = B.estimates(slot)
        for k in ("mean", "m2", "rec_mean", "rec_m2"):
            assert np.array_equal(bits(got[k]), bits(e[k])), (slot, k)


def test_batch_graph_replay_equals_eager(smc, dev):
    print("batch graph vs eager", flush=True)
    specs = [spec(40 + k, *m) for k, m in enumerate(MIX[:5])]
    outs = []
    for graph in (True, False):
        B = smc.Batch(5, graph=graph, device=dev)
        for slot, sp in enumerate(specs):
            attach(B, slot, sp)
        for _ in range(6):
            B.step()
        outs.append([B.x(s).cpu().numpy() for s in range(5)])
    for a, b in zip(*outs):
        assert np.array_equal(bits(a), bits(b))


def test_batch_attach_detach_midrun(smc, dev):
    print("batch attach/detach", flush=True)
    a, b, c = spec(60, 5000, 12, O.MODE_FORCE), spec(61, 9000, 40, O.MODE_AUTO), \
        spec(62, 300, 2, O.MODE_FORCE)
    B = smc.Batch(4, device=dev)
    attach(B, 0, a)
    attach(B, 1, b)
    oa, ob = oracle_of(B, 0, a), oracle_of(B, 1, b)
    for t in range(3):
        B.step()
        check_step(B, 0, oa, oa.step(), ("a", t))
        ob.step()
    B.detach(1)
    attach(B, 1, c)
    attach(B, 3, b | {"seed": b["seed"] + 1})
    oc = oracle_of(B, 1, c)
    for t in range(4):
        B.step()
        check_step(B, 0, oa, oa.step(), ("a2", t))
        check_step(B, 1, oc, oc.step(), ("c", t))
    assert B.counts()[0] == 3


def test_batch_large_sampler(smc, dev):
    print("batch n=2^20+5", flush=True)
    sp = spec(70, (1 << 20) + 5, 2, O.MODE_FORCE)
    B = smc.Batch(2, device=dev)
    attach(B, 1, sp)
    o = oracle_of(B, 1, sp)
    for t in range(2):
        B.step()
        check_step(B, 1, o, o.step(), t)


def test_batch_workload_sampled(smc, dev):
    """The 256-sampler workload (N log-uniform 2^8..2^16, d 1..64): sampled
    samplers bit-exact against the oracle over three steps."""
    print("batch workload 256 samplers", flush=True)
    specs = I.batch_specs()
    B = smc.Batch(len(specs), device=dev)
    for slot, sp in enumerate(specs):
        attach(B, slot, sp | {"mode": O.MODE_AUTO})
    ns = np.array([s["n"] for s in specs])
    ds = np.array([s["d"] for s in specs])
    pick = sorted({int(np.argmin(ns)), int(np.argmax(ns)), int(np.argmax(ds)), 17})
    orcs = {k: oracle_of(B, k, specs[k] | {"mode": O.MODE_AUTO}) for k in pick}
    for t in range(3):
        B.step()
        for k in pick:
            check_step(B, k, orcs[k], orcs[k].step(), (t, k))
    infos = [B.info(k) for k in range(len(specs))]
    assert all(i["err"] == 0 for i in infos)


def test_batch_rejects_bad_arguments(smc, dev):
    B = smc.Batch(2, device=dev)
    sp = spec(80, 100, 4, O.MODE_AUTO)
    attach(B, 0, sp)
    with pytest.raises(smc.L.SmcError):
        attach(B, 0, sp)          # slot taken
    with pytest.raises(smc.L.SmcError):
        attach(B, 2, sp)          # no such slot
    with pytest.raises(smc.L.SmcError):
        B.attach(1, 100, 65, np.zeros(65), np.eye(65))   # d > 64
    with pytest.raises(smc.L.SmcError):
        B.detach(1)               # free slot


def test_batch_unit_size_does_not_change_results(smc, dev):
    print("batch unit size", flush=True)
    specs = [spec(90 + k, *m) for k, m in enumerate(MIX)]
    outs = []
    for g in (1, 3, 6, 8):
        B = smc.Batch(len(MIX), device=dev)
        B.set_group(g)
        for slot, sp in enumerate(specs):
            attach(B, slot, sp)
        for _ in range(3):
            B.step()
        outs.append([(B.x(s).cpu().numpy(), B.estimates(s)["mean"]) for s in range(len(MIX))])
    for other in outs[1:]:
        for (xa, ea), (xb, eb) in zip(outs[0], other):
            assert np.array_equal(bits(xa), bits(xb))
            assert np.array_equal(bits(ea), bits(eb))
    with pytest.raises(smc.L.SmcError):
        B.set_group(9)


def test_batch_unaligned_log_weights(smc, dev):
    """A sampler whose log-weight array is 8-byte but not 16-byte aligned: the
    scan reads its full tiles element by element instead of in 16-byte
    pieces; the bits equal those of the same sampler on an aligned array."""
    import torch
    print("batch unaligned log-weights", flush=True)
    sp = spec(70, 3 * 4096 + 100, 5, O.MODE_FORCE)
    outs = []
    for off in (0, 1):
        B = smc.Batch(1, device=dev)
        buf = torch.empty(sp["n"] + 1, dtype=torch.float64, device=dev)
        lw = buf[off:off + sp["n"]]
        assert (lw.data_ptr() % 16 == 0) == (off == 0)
        B.attach(0, sp["n"], sp["d"], sp["mean"], sp["chol"], seed=sp["seed"],
                 sampler_id=sp["sampler_id"], rw_sd=sp["rw_sd"], mode=sp["mode"], logw=lw)
        for _ in range(3):
            B.step()
        outs.append((B.x(0).cpu().numpy(), lw.cpu().numpy(), B.estimates(0)["mean"]))
    for u, v in zip(*outs):
        assert np.array_equal(bits(u), bits(v))


def test_batch_bucket_waves_do_not_change_results(smc, dev):
    """The per-bucket occupancy aim of the target kernel is a speed knob:
    every setting gives the same bits (graph replay included)."""
    print("batch bucket waves", flush=True)
    specs = [spec(120 + k, *m) for k, m in enumerate(MIX)]
    outs = []
    for waves in (None, 1, 2, 3):
        B = smc.Batch(len(MIX), device=dev)
        if waves is not None:
            for q in range(8):
                B.set_bucket_waves(q, waves)
        for slot, sp in enumerate(specs):
            attach(B, slot, sp)
        for _ in range(4):
            B.step()
        outs.append([(B.x(s).cpu().numpy(), B.logw(s).cpu().numpy(), B.estimates(s)["mean"])
                     for s in range(len(MIX))])
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            for u, v in zip(a, b):
                assert np.array_equal(bits(u), bits(v))
    for bad in ((8, 2), (-1, 2), (3, 0), (3, 5)):
        with pytest.raises(smc.L.SmcError):
            B.set_bucket_waves(*bad)


def test_autotuner_picks_candidates_and_caches(dev, tmp_path, monkeypatch):
    from paper_1905_10252_amd import tune
    monkeypatch.setenv("SMC_TUNE_CACHE", str(tmp_path / "tune.json"))
    specs = I.batch_specs(count=12, seed=301)
    r = tune.tune_group(specs, device=dev, steps=1)
    assert not r["cached"]
    assert r["best"] in tune.GROUP_CANDIDATES and set(r["ms"]) == set(tune.GROUP_CANDIDATES)
    rb = tune.tune_buckets(specs, device=dev, steps=1, pairs=r["best"])
    present = sorted({(sp["d"] - 1) // 8 for sp in specs})
    assert sorted(rb["best"]) == present and not rb["cached"]
    for q, w in rb["best"].items():
        assert 1 <= w <= tune._max_waves(q)
    # the second call reads the cache (keyed by kernel, knob, bucket, device
    # architecture and workload shapes) instead of timing
    r2 = tune.tune_group(specs, device=dev, steps=1)
    rb2 = tune.tune_buckets(specs, device=dev, steps=1)
    assert r2["cached"] and r2["best"] == r["best"]
    assert sorted(rb2["cached"]) == present and rb2["best"] == rb["best"]
    import json
    keys = json.load(open(tmp_path / "tune.json"))
    arch = tune.arch(dev)
    assert any(k.startswith("k_bquad|waves|%d|%s|" % (present[0], arch)) for k in keys)


def test_batch_failed_iteration_leaves_recycling(smc, dev):
    """A NaN log-weight in one sampler fails that sampler's iteration at the
    resampling step: its c_t and recycling sums stay as they were (the oracle
    returns there), its neighbour is untouched, and after the repair both
    continue as the oracle's samplers do."""
    B = smc.Batch(2, graph=True, device=dev)
    sps = [spec(0, 3000, 5, O.MODE_AUTO, seed=610), spec(1, 5000, 12, O.MODE_AUTO, seed=610)]
    os_ = []
    for k, sp in enumerate(sps):
        attach(B, k, sp)
        os_.append(oracle_of(B, k, sp))
    for t in range(3):
        B.step()
        for k in range(2):
            check_step(B, k, os_[k], os_[k].step(), "before t=%d slot %d" % (t, k))
    B.logw(1)[7] = float("nan")
    os_[1].logw[7] = np.nan
    B.step()
    check_step(B, 0, os_[0], os_[0].step(), "failed step, slot 0")
    with pytest.raises(ValueError):
        os_[1].step()
    assert B.info(1)["err"] == O.E_NONFINITE
    assert B.sync_error(1) == O.E_NONFINITE
    check_state(B, 1, os_[1], "failed step, slot 1")
    B.logw(1)[7] = -0.5
    os_[1].logw[7] = -0.5
    for t in range(3):
        B.step()
        for k in range(2):
            check_step(B, k, os_[k], os_[k].step(), "after t=%d slot %d" % (t, k))
    assert B.sync_error(0) == 0 and B.sync_error(1) == 0


def test_batch_infinite_coordinate_matches_row_by_row(smc, dev):
    """A particle with one infinite coordinate: the oracle's row-by-row
    quadratic form makes every row through that coordinate infinite, so
    log pi = -inf and the particle's weight is zero.  The matrix-core form
    (d = 40 here) multiplies the zeros of U below the diagonal by that
    coordinate too, which would give NaN; such a particle must take the
    row-by-row path and match the oracle bit for bit (d = 12: the vector
    kernel).  Resampling is forced, so the particle is dropped after the
    step and the next step runs on finite rows again."""
    import torch
    print("batch infinite coordinate", flush=True)
    B = smc.Batch(2, graph=False, device=dev)
    specs = [spec(0, 3000, 40, O.MODE_FORCE), spec(1, 3000, 12, O.MODE_FORCE)]
    for slot, sp in enumerate(specs):
        attach(B, slot, sp)
    orcs = [oracle_of(B, slot, sp) for slot, sp in enumerate(specs)]
    rows = [5, 700, 1601, 2999]
    for slot, sp in enumerate(specs):
        xg = B.x(slot)
        for j, r in enumerate(rows):
            k = (7 * j + 3) % sp["d"]
            v = math.inf if j % 2 == 0 else -math.inf
            xg[r, k] = v
            orcs[slot].x[r, k] = v
    torch.cuda.synchronize()
    B.step()
    for slot in range(2):
        orcs[slot].step()
        x = B.x(slot).cpu().numpy()  # the rows with an infinite coordinate were dropped
        assert np.all(np.isfinite(x)), slot
        check_state(B, slot, orcs[slot], ("inf coordinate", slot))
        assert B.info(slot)["err"] == 0
    B.step()
    for slot in range(2):
        orcs[slot].step()
        check_state(B, slot, orcs[slot], ("after", slot))
