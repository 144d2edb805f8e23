"""GPU parity of smc_resample + smc_redistribute against the CPU oracle.

Integer outputs (ncopies, ancestors, redistributed rows, S, U, sum q^2,
decision) must be bit-exact; FP64 outputs (log Z, ESS) within 1e-12 relative.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_1905_10252_amd import inputs as I

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def smc(dev):
    from paper_1905_10252_amd import smc as S
    return S


def run_gpu(smc, dev, lw, x, r, mode, ncopies=True, anc=True):
    import torch
    n = lw.size
    R = smc.Resampler(n, device=dev)
    tlw = torch.from_numpy(lw).to(dev)
    tx = torch.from_numpy(x).to(dev)
    nc = torch.full((n,), -7, dtype=torch.int64, device=dev)
    an = torch.full((n,), -7, dtype=torch.int64, device=dev) if anc else None
    R.resample(tlw, r, mode)
    xo = R.redistribute(tx, ncopies_out=nc, anc=an)
    torch.cuda.synchronize()
    info = R.info()
    return (xo.cpu().numpy(), nc.cpu().numpy(), None if an is None else an.cpu().numpy(), info, R)


def compare(lw, x, r, mode, smc, dev):
    xo, nc, an, info, _ = run_gpu(smc, dev, lw, x, r, mode)
    onc, oinfo = O.resample(lw, r, mode)
    assert info["err"] == oinfo["err"] == 0
    for k in ("S", "U", "Q2_hi", "Q2_lo", "K", "resampled"):
        assert info[k] == oinfo[k], (k, info[k], oinfo[k])
    assert info["m"] == oinfo["m"]
    assert abs(info["logZ"] - oinfo["logZ"]) <= RTOL * max(1.0, abs(oinfo["logZ"]))
    assert abs(info["ess"] - oinfo["ess"]) <= RTOL * oinfo["ess"]
    assert np.array_equal(nc, onc)
    ox, oanc = O.redistribute(onc, x)
    assert np.array_equal(an, oanc)
    assert np.array_equal(xo.view(np.uint8), ox.view(np.uint8))
    return oinfo


SIZES = [1, 2, 3, 5, 64, 1023, 4096, 4097, 3 * 4096 + 17, 65537, (1 << 20) + 7]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("s", I.RESAMPLE_SCALES)
def test_resample_parity_forced(smc, dev, n, s):
    _say("case n=%d s=%g" % (n, s))
    lw = I.logw_normal(n, s, 1000 + n)
    x = I.particles(n, 3, 2000 + n)
    compare(lw, x, I.offset_word(3000 + n), O.MODE_FORCE, smc, dev)


@pytest.mark.parametrize("n", [7, 4097, 100000])
@pytest.mark.parametrize("s", [0.1, 0.5, 0.83, 2.0])
def test_resample_parity_auto(smc, dev, n, s):
    _say("case auto n=%d s=%g" % (n, s))
    lw = I.logw_normal(n, s, 11 + n)
    x = I.particles(n, 2, 12 + n, dtype=np.float64)
    compare(lw, x, I.offset_word(13), O.MODE_AUTO, smc, dev)


@pytest.mark.parametrize("row", [1, 2, 3, 5, 16, 64])
def test_row_widths(smc, dev, row):
    n = 9000
    lw = I.logw_normal(n, 2.0, 5)
    x = I.particles(n, row, 6)
    compare(lw, x, 99, O.MODE_FORCE, smc, dev)


def test_never_is_identity(smc, dev):
    n = 5000
    lw = I.logw_normal(n, 8.0, 5)
    x = I.particles(n, 4, 6)
    xo, nc, an, info, _ = run_gpu(smc, dev, lw, x, 1, O.MODE_NEVER)
    assert info["resampled"] == 0
    assert np.all(nc == 1) and np.array_equal(an, np.arange(n))
    assert np.array_equal(xo, x)


def test_equal_and_single_weights(smc, dev):
    n = 777
    x = I.particles(n, 2, 1)
    compare(np.full(n, 1.5), x, 5, O.MODE_FORCE, smc, dev)
    compare(np.full(n, 1.5), x, 5, O.MODE_AUTO, smc, dev)
    lw = np.full(n, -np.inf)
    lw[400] = -3.0
    info = compare(lw, x, 5, O.MODE_AUTO, smc, dev)
    assert info["resampled"] == 1


def test_heavy_tail_with_minus_inf(smc, dev):
    n = 70000
    lw = I.logw_normal(n, 8.0, 21)
    lw[::3] = -np.inf
    compare(lw, I.particles(n, 4, 22), 2**64 - 1, O.MODE_FORCE, smc, dev)
    compare(lw, I.particles(n, 4, 22), 0, O.MODE_FORCE, smc, dev)


@pytest.mark.parametrize("bad,code", [(np.nan, O.E_NONFINITE), (np.inf, O.E_NONFINITE)])
def test_nonfinite_reported(smc, dev, bad, code):
    import torch
    n = 5000
    lw = I.logw_normal(n, 1.0, 3)
    lw[1234] = bad
    x = I.particles(n, 2, 4)
    R = smc.Resampler(n, device=dev)
    tx = torch.from_numpy(x).to(dev)
    xo = torch.zeros_like(tx)
    R.resample(torch.from_numpy(lw).to(dev), 1, O.MODE_FORCE)
    R.redistribute(tx, xo)
    torch.cuda.synchronize()
    assert R.info()["err"] == code
    assert np.all(xo.cpu().numpy() == 0)  # nothing written
    assert R.sync_error() == code
    assert R.sync_error() == 0  # cleared


def test_all_zero_weights_reported(smc, dev):
    import torch
    n = 100
    R = smc.Resampler(n, device=dev)
    R.resample(torch.full((n,), -math.inf, dtype=torch.float64, device=dev), 1)
    torch.cuda.synchronize()
    assert R.info()["err"] == O.E_DEGENERATE
    assert R.sync_error() == O.E_DEGENERATE


def test_foreign_ncopies(smc, dev):
    import torch
    rng = np.random.default_rng(7)
    for n in [1, 10, 4097, 200003]:
        q = rng.integers(0, 3, n).astype(np.uint64)
        q[0] += 1
        onc = O.systematic_ncopies(q, int(rng.integers(0, int(q.sum()))))
        x = I.particles(n, 5, n)
        R = smc.Resampler(n, device=dev)
        an = torch.zeros(n, dtype=torch.int64, device=dev)
        xo = R.redistribute(torch.from_numpy(x).to(dev),
                            ncopies=torch.from_numpy(onc).to(dev), anc=an)
        ox, oanc = O.redistribute(onc, x)
        assert np.array_equal(xo.cpu().numpy(), ox)
        assert np.array_equal(an.cpu().numpy(), oanc)
        assert R.sync_error() == 0


def test_foreign_ncopies_rejected(smc, dev):
    import torch
    n = 1000
    x = torch.ones((n, 2), dtype=torch.float32, device=dev)
    R = smc.Resampler(n, device=dev)
    neg = np.ones(n, dtype=np.int64)
    neg[0], neg[1] = -1, 3  # sums to N but has a negative count
    for nc in (np.full(n, 2), neg):
        xo = torch.zeros_like(x)
        R.redistribute(x, xo, ncopies=torch.from_numpy(nc.astype(np.int64)).to(dev))
        torch.cuda.synchronize()
        assert np.all(xo.cpu().numpy() == 0)
        assert R.sync_error() == O.E_ARG


def test_repeat_calls_are_independent(smc, dev):
    import torch
    n = 30000
    R = smc.Resampler(n, device=dev)
    x = I.particles(n, 4, 1)
    tx = torch.from_numpy(x).to(dev)
    for it, s in enumerate([8.0, 0.5, 2.0, 8.0]):
        lw = I.logw_normal(n, s, 40 + it)
        nc = torch.zeros(n, dtype=torch.int64, device=dev)
        R.resample(torch.from_numpy(lw).to(dev), 1000 + it, O.MODE_FORCE, ncopies=nc)
        xo = R.redistribute(tx)
        onc, _ = O.resample(lw, 1000 + it, O.MODE_FORCE)
        assert np.array_equal(nc.cpu().numpy(), onc)
        assert np.array_equal(xo.cpu().numpy(), O.redistribute(onc, x)[0])


@pytest.mark.parametrize("s", I.RESAMPLE_SCALES)
def test_full_size_parity(smc, dev, s):
    """N = 2^24, d = 16 FP32: the configuration the benchmark times."""
    n, d = I.RESAMPLE_N, I.RESAMPLE_D
    _say("full-size case s=%g" % s)
    lw = I.logw_normal(n, s, I.LOGW_SEEDS[s])
    x = I.particles(n, d, I.X_SEED)
    oinfo = compare(lw, x, I.offset_word(I.R_SEED), O.MODE_FORCE, smc, dev)
    _say("  unique survivors %d of %d" % (oinfo["unique"], n))


def test_module_level_functions(smc, dev):
    """smc.resample / smc.redistribute keep one context per N: a
    redistribute without counts follows the last resample of the same N,
    whatever was resampled at other sizes in between."""
    import torch
    _say("module-level resample/redistribute")
    sizes = (3001, 70001)
    xs = {n: I.particles(n, 3, 7 + n) for n in sizes}
    lws = {n: I.logw_normal(n, 2.0, 11 + n) for n in sizes}
    nc = {n: smc.resample(torch.from_numpy(lws[n]).to(dev), 99 + n, O.MODE_FORCE) for n in sizes}
    for n in sizes[::-1]:
        onc, _ = O.resample(lws[n], 99 + n, O.MODE_FORCE)
        assert nc[n].dtype == torch.int64 and np.array_equal(nc[n].cpu().numpy(), onc)
        xo = smc.redistribute(torch.from_numpy(xs[n]).to(dev))
        assert np.array_equal(xo.cpu().numpy(), O.redistribute(onc, xs[n])[0])
    # explicit counts, and the ESS rule declining to resample (all ones)
    n = sizes[0]
    onc, _ = O.resample(lws[sizes[1]][:n], 5, O.MODE_FORCE)
    xo = smc.redistribute(torch.from_numpy(xs[n]).to(dev), torch.from_numpy(onc).to(dev))
    assert np.array_equal(xo.cpu().numpy(), O.redistribute(onc, xs[n])[0])
    flat = np.zeros(n)
    ones = smc.resample(torch.from_numpy(flat).to(dev), 1, O.MODE_AUTO)
    assert np.array_equal(ones.cpu().numpy(), np.ones(n, dtype=np.int64))
    assert np.array_equal(O.resample(flat, 1, O.MODE_AUTO)[0], np.ones(n, dtype=np.int64))
    smc.release()
    with pytest.raises(smc.L.SmcError):
        smc.redistribute(torch.from_numpy(xs[n]).to(dev))   # a new context has nothing pending


def test_maximum_size(smc, dev):
    """N = 2^31 - 1, the largest N the library takes (its last tile ragged),
    rows of one int32 holding their own source index.  The log-weights repeat
    a seeded pattern of P values, so the exact prefix has a closed form at any
    index: S_j = (j div P) Q + C[j mod P], with q of the pattern from the
    oracle's quantiser.  Exact checks: S, U, sum q^2 and K; sum ncopies = N;
    sampled counts (both outputs) and sampled output rows against the
    systematic definition evaluated on that prefix."""
    import torch
    n, P = I.MAX_N, I.MAX_PERIOD
    _say("maximum size N = 2^31 - 1 (about 80 GB of device memory)")
    base = I.logw_normal(P, 2.0, 404)
    K = O.quant_bits(n)
    q = [int(v) for v in O.quantise(base, K, float(base.max()))]
    C = np.cumsum(np.array(q, dtype=object))
    Q = int(C[-1])
    full, rem = divmod(n, P)

    def S_at(j):
        return (j // P) * Q + int(C[j % P])

    S = S_at(n - 1)
    q2 = full * sum(v * v for v in q) + sum(v * v for v in q[:rem])
    r = I.offset_word(I.R_SEED)
    U = (r * S) >> 64

    def A(j):
        return (n * S_at(j) + U) // S if j >= 0 else 0

    def anc(p):
        lo, hi = 0, n - 1          # first j with A_j > p
        while lo < hi:
            mid = (lo + hi) // 2
            if A(mid) > p:
                hi = mid
            else:
                lo = mid + 1
        return lo

    R = smc.Resampler(n, device=dev)
    lw = torch.from_numpy(base).to(dev).repeat(full + 1)[:n]
    x = torch.arange(n, dtype=torch.int32, device=dev)
    nc1 = torch.empty(n, dtype=torch.int64, device=dev)
    nc2 = torch.empty(n, dtype=torch.int64, device=dev)
    R.resample(lw, r, O.MODE_FORCE, ncopies=nc1)
    xo = R.redistribute(x, ncopies_out=nc2)
    info = R.info()
    assert info["err"] == 0 and info["resampled"] == 1 and info["K"] == K
    assert info["S"] == S and info["U"] == U
    assert (info["Q2_hi"] << 64) | info["Q2_lo"] == q2
    assert int(nc1.sum().item()) == n and int(nc2.sum().item()) == n
    rng = np.random.default_rng(5)
    js = sorted(set(rng.integers(0, n, 1500).tolist()) |
                {0, 1, 4095, 4096, P - 1, P, n // 2, n - 4096, n - 2, n - 1})
    idx = torch.tensor(js, dtype=torch.int64, device=dev)
    got1, got2 = nc1[idx].cpu().tolist(), nc2[idx].cpu().tolist()
    for j, a1, a2 in zip(js, got1, got2):
        want = A(j) - A(j - 1)
        assert a1 == want and a2 == want, (j, a1, a2, want)
    ps = sorted(set(rng.integers(0, n, 1500).tolist()) | {0, 1, n // 2, n - 2, n - 1})
    rows = xo[torch.tensor(ps, dtype=torch.int64, device=dev)].cpu().tolist()
    for p, row in zip(ps, rows):
        assert row == anc(p), (p, row)
    assert R.sync_error() == 0
    del R, lw, x, nc1, nc2, xo, idx
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,s", [(1, 1.0), (1000, 0.5), (70001, 8.0), (1 << 20, 2.0),
                                 (1 << 24, 8.0)])
def test_normalised_weights(smc, dev, n, s):
    """eq. normalise against the oracle: exp(l - m) / Z, zero weights zero,
    unit sum."""
    import torch
    lw = I.logw_normal(n, s, 31 + n)
    if n > 7:
        lw[::7] = -np.inf
    R = smc.Resampler(n, device=dev)
    t = torch.from_numpy(lw).to(dev)
    R.resample(t, 5, O.MODE_FORCE)
    w = R.normalised_weights(t).cpu().numpy()
    ref = O.normalised_weights(lw)
    pos = ref > 0
    assert np.array_equal(w[~pos], ref[~pos])
    assert np.max(np.abs(w[pos] / ref[pos] - 1.0)) < 1e-12
    assert abs(w.sum() - 1.0) < 1e-12


def test_redistribute_row_size_bound(smc, dev):
    """Rows up to 1 MiB are copied (the expand's 32-bit chunk count per
    segment stays in range); a larger row is an argument error, returned
    before anything is enqueued."""
    import ctypes as C
    import torch
    n = 5
    lw = np.array([0.0, -1.0, 2.0, -0.5, 1.0])
    R = smc.Resampler(n, device=dev)
    R.resample(torch.from_numpy(lw).to(dev), 12345, O.MODE_FORCE)
    row = 1 << 20
    x = torch.arange(n * row // 4, dtype=torch.int32, device=dev).view(n, row // 4)
    xo = R.redistribute(x)
    torch.cuda.synchronize()
    onc, _ = O.resample(lw, 12345, O.MODE_FORCE)
    ox, _ = O.redistribute(onc, x.cpu().numpy())
    assert np.array_equal(xo.cpu().numpy(), ox)
    big = torch.zeros(n * (row + 4), dtype=torch.uint8, device=dev)
    out = torch.zeros_like(big)
    lib = smc.L.load()
    rc = lib.smc_redistribute(R.ctx, None, C.c_void_p(big.data_ptr()), C.c_void_p(out.data_ptr()),
                              n, row + 4, None, None, smc._stream())
    assert rc == smc.L.SMC_E_ARG
    del x
