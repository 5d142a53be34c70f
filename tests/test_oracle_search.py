"""Pins of the oracle's search stages: brute-force dedispersion, moments, boxcar
search with threshold and best width, and the peak filter.

Each pin rests on something other than the oracle's own code: exhaustive brute
force on tiny inputs, invariants of the DM transform (DM-0 row = channel sum,
impulse response, linearity), numpy library routines (convolution, mean, std),
the Gaussian tail, and recovery of an injected pulse at its analytic S/N.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2606_27262_amd import synth
from paper_2606_27262_amd import workloads as W


# ---------------------------------------------------------------- dedispersion
def _brute(x, delays, n_dd):
    return np.array([[sum(int(x[c][t + delays[d][c]]) for c in range(x.shape[0]))
                      for t in range(n_dd)] for d in range(delays.shape[0])], dtype=np.int64)


def test_dedisperse_exhaustive_tiny():
    """All monotone delay tables with entries <= 2 for nch <= 3, values in {0, 1, 255}."""
    rng = np.random.default_rng(0)
    for nch in (1, 2, 3):
        rows = [r for r in itertools.product(range(3), repeat=nch) if list(r) == sorted(r)]
        for ndm in (1, 2):
            for table in itertools.product(rows, repeat=ndm):
                delays = np.array(table, dtype=np.int64)
                n_dd = 3
                n_in = n_dd + int(delays.max())
                x = rng.choice(np.array([0, 1, 255], np.uint8), size=(nch, n_in))
                assert np.array_equal(oracle.dedisperse(x, delays, n_dd), _brute(x, delays, n_dd))


def test_dm0_row_is_channel_sum_and_impulse_response():
    plan = W.plan_c1()
    dms = oracle.dm_trials(plan["dm_ranges"])
    D, _ = oracle.delay_table(plan["nchans"], plan["fch1"], plan["foff"], plan["tsamp"], dms)
    sz = oracle.sizes(D, plan["n_out"], plan["widths"])
    rng = np.random.default_rng(1)
    x = rng.integers(0, 256, size=(plan["nchans"], sz["n_in"]), dtype=np.uint8)
    X = oracle.dedisperse(x, D, sz["n_dd"])
    assert np.array_equal(X[0], x[:, :sz["n_dd"]].astype(np.int64).sum(0))
    # single 1 at (c, t0): appears at X[d, t0 - delay[d][c]] and nowhere else
    imp = np.zeros_like(x)
    c, t0 = 200, 12000
    imp[c, t0] = 1
    Xi = oracle.dedisperse(imp, D, sz["n_dd"])
    for d in range(D.shape[0]):
        nz = np.nonzero(Xi[d])[0]
        t = t0 - D[d, c]
        if 0 <= t < sz["n_dd"]:
            assert list(nz) == [t]
        else:
            assert nz.size == 0
    # linearity on values that cannot overflow a byte
    a = rng.integers(0, 128, size=x.shape, dtype=np.uint8)
    b = rng.integers(0, 128, size=x.shape, dtype=np.uint8)
    assert np.array_equal(oracle.dedisperse(a + b, D, sz["n_dd"]),
                          oracle.dedisperse(a, D, sz["n_dd"]) + oracle.dedisperse(b, D, sz["n_dd"]))


def test_dedisperse_single_channel_is_shift():
    x = np.arange(40, dtype=np.uint8).reshape(1, 40)
    D = np.array([[0], [3], [7]], np.int64)
    X = oracle.dedisperse(x, D, 20)
    for d in range(3):
        assert np.array_equal(X[d], x[0, D[d, 0]:D[d, 0] + 20])


# ---------------------------------------------------------------- moments
def test_moments_match_numpy_and_constant_rows():
    rng = np.random.default_rng(2)
    X = rng.integers(0, 1 << 20, size=(5, 300)).astype(np.int64)
    X[3] = 777
    n, s1, s2 = oracle.moments(X, 290, 100)
    assert n.tolist() == [[100, 100, 90]] * 5
    for d in range(5):
        for k in range(3):
            seg = X[d, 100 * k: min(100 * k + 100, 290)]
            assert s1[d, k] == int(seg.sum()) and s2[d, k] == int((seg * seg).sum())
            mu, sg = oracle.mu_sigma(n[d, k], s1[d, k], s2[d, k])
            assert math.isclose(mu, float(np.mean(seg)), rel_tol=1e-15)
            assert math.isclose(sg, float(np.std(seg)), rel_tol=1e-9, abs_tol=1e-12)
    assert oracle.mu_sigma(n[3, 0], s1[3, 0], s2[3, 0])[1] == 0.0
    # constant row: no hits at all
    h = oracle.search(np.full((1, 400), 5, np.int64), 300, 300, (1, 4), 1.0)
    assert h["d"].size == 0


def test_mu_sigma_128bit_exactness():
    # n*S2 and S1^2 both above 2^64; their difference is small and exact
    n = 32768
    v = 1_000_000
    s1 = n * v
    s2 = n * v * v + 12345 * n
    mu, sg = oracle.mu_sigma(n, s1, s2)
    assert mu == float(v)
    assert math.isclose(sg, math.sqrt(12345 * n * n) / n, rel_tol=1e-15)


# ---------------------------------------------------------------- boxcar search
def _numpy_snr_all(X, n_out, L, widths):
    """S/N of every (d, t, w) from numpy convolution, mean and std."""
    ndm, _ = X.shape
    out = np.full((ndm, n_out, len(widths)), -np.inf)
    for d in range(ndm):
        for k in range((n_out + L - 1) // L):
            lo, hi = k * L, min((k + 1) * L, n_out)
            seg = X[d, lo:hi].astype(np.float64)
            mu, sd = seg.mean(), seg.std()
            if sd == 0:
                continue
            for j, w in enumerate(widths):
                B = np.convolve(X[d].astype(np.float64), np.ones(w), "valid")[lo:hi]
                out[d, lo:hi, j] = (B - w * mu) / (sd * math.sqrt(w))
    return out


@pytest.mark.parametrize("L", [64, 250, 1000])
def test_search_against_numpy_definition(L):
    rng = np.random.default_rng(3)
    widths = (1, 2, 4, 8)
    n_out = 250
    X = rng.normal(1000, 30, size=(6, n_out + 7)).round().astype(np.int64)
    X[2, 100:104] += 150       # a pulse
    X[4] = 9                   # constant row
    theta = 2.5
    h = oracle.search(X, n_out, min(L, n_out), widths, theta)
    snr = _numpy_snr_all(X, n_out, min(L, n_out), widths)
    best = snr.max(axis=2)
    near = np.abs(best - theta) < 1e-9
    expect = (best >= theta) & ~near
    got = np.zeros_like(expect)
    got[h["d"], h["t"]] = True
    assert np.array_equal(got & ~near, expect)
    # (d, t) order, best width and exact boxcar sums
    key = h["d"].astype(np.int64) * 10 ** 6 + h["t"]
    assert np.all(np.diff(key) > 0)
    for d, t, w, B, s in zip(h["d"], h["t"], h["w"], h["B"], h["snr"]):
        assert B == int(X[d, t:t + w].sum())
        j = widths.index(int(w))
        assert math.isclose(s, snr[d, t, j], rel_tol=1e-9)
        assert s >= snr[d, t].max() - 1e-9


def test_best_width_tie_keeps_smaller_width():
    """A row with mean exactly 0 where B_4 = 2 B_1: both widths give the same S/N
    bit for bit (4/sigma), and the smaller width is reported."""
    X = np.zeros((1, 40), np.int64)
    X[0, 10] = 4
    X[0, 11] = 4
    X[0, 30] = -8
    h = oracle.search(X, 36, 36, (1, 4), 0.1)
    i = list(h["t"]).index(10)
    mu, sg = oracle.mu_sigma(36, 0, int((X[0, :36] ** 2).sum()))
    assert mu == 0.0
    assert oracle.snr(4, 1, mu, sg) == oracle.snr(8, 4, mu, sg)
    assert h["w"][i] == 1 and h["B"][i] == 4


def test_false_alarm_rate_single_width_matches_gaussian_tail():
    """Noise-only c1 block, width 1, threshold 3: fraction of (d, t) above threshold
    equals the Gaussian tail 1 - Phi(3) = 1.35e-3 (normaliser and sign pinned)."""
    plan = W.plan_c1()
    dms = oracle.dm_trials(plan["dm_ranges"])
    D, _ = oracle.delay_table(plan["nchans"], plan["fch1"], plan["foff"], plan["tsamp"], dms)
    sz = oracle.sizes(D, plan["n_out"], plan["widths"])
    _, x = W.c1_block(sz["n_in"], seed=11, with_pulse=False)
    X = oracle.dedisperse(x[:, :sz["n_in"]], D, sz["n_dd"])
    h = oracle.search(X, plan["n_out"], plan["n_out"], (1,), 3.0)
    frac = h["d"].size / (X.shape[0] * plan["n_out"])
    assert 0.8 * 1.35e-3 < frac < 1.2 * 1.35e-3
    # and at the real 6-sigma threshold with all widths, almost nothing
    h6 = oracle.search(X, plan["n_out"], plan["n_out"], plan["widths"], 6.0)
    assert h6["d"].size <= 3


def _expected_snr(spec, pulse, D, d, n_out, widths):
    """Analytic matched-boxcar S/N of the noise-free template dedispersed at trial d,
    normalised like the search (plain mean; sigma^2 = noise + template variance)."""
    amp = synth.pulse_amplitude(pulse, spec.nch, widths)
    starts, vals = synth.pulse_template(spec, pulse, amp)
    n_dd = n_out + max(widths) - 1
    T = np.zeros(n_dd)
    for c in range(spec.nch):
        a = int(starts[c]) - int(D[d, c])
        for k in range(vals.shape[1]):
            if 0 <= a + k < n_dd:
                T[a + k] += vals[c, k]
    sig_n2 = synth.QUANT_SIGMA ** 2 * spec.nch
    mean = T[:n_out].mean()
    sig = math.sqrt(sig_n2 + T[:n_out].var())
    best = 0.0
    for w in widths:
        B = np.convolve(T, np.ones(w), "valid")[:n_out]
        best = max(best, float(((B - w * mean) / (math.sqrt(w) * sig)).max()))
    return best


@pytest.mark.slow
def test_injected_pulse_recovered_at_analytic_snr():
    """c1: DM 250 (trial 64), FWHM 4, S/N 20.  Over 64 seeds the mean measured S/N is
    within 5% of the analytic matched-filter value; each seed within 4 units; the
    peak sits at trial 64, next to t0 = 4096."""
    plan = W.plan_c1()
    dms = oracle.dm_trials(plan["dm_ranges"])
    D, _ = oracle.delay_table(plan["nchans"], plan["fch1"], plan["foff"], plan["tsamp"], dms)
    sz = oracle.sizes(D, plan["n_out"], plan["widths"])
    measured = []
    spec = None
    for seed in range(100, 164):
        spec, x = W.c1_block(sz["n_in"], seed=seed)
        X = oracle.dedisperse(x[:, :sz["n_in"]], D, sz["n_dd"])
        h = oracle.search(X[60:69], plan["n_out"], plan["n_out"], plan["widths"], 6.0)
        sel = np.abs(h["t"] - 4096) <= 8
        assert sel.any()
        i = np.argmax(np.where(sel, h["snr"], -np.inf))
        assert h["d"][i] + 60 == 64
        measured.append(h["snr"][i])
    exp = _expected_snr(spec, spec.pulses[0], D, 64, plan["n_out"], plan["widths"])
    assert 18.0 < exp < 20.5
    m = np.array(measured)
    assert abs(m.mean() - exp) / exp < 0.05
    assert np.all(np.abs(m - exp) < 4.0)


# ---------------------------------------------------------------- peak filter
def _nms_brute(d, t, s, rd, rt, alive):
    keep = []
    for i in range(len(d)):
        if not alive[i]:
            keep.append(False)
            continue
        ok = True
        for j in range(len(d)):
            if j == i or not alive[j]:
                continue
            if abs(d[j] - d[i]) <= rd and abs(t[j] - t[i]) <= rt:
                if (s[j], -d[j], -t[j]) > (s[i], -d[i], -t[i]):
                    ok = False
                    break
        keep.append(ok)
    return np.array(keep)


def test_nms_matches_brute_force_with_ties():
    rng = np.random.default_rng(4)
    for trial in range(40):
        ndm, nt = 12, 30
        cells = rng.choice(ndm * nt, size=rng.integers(1, 120), replace=False)
        cells.sort()
        d = (cells // nt).astype(np.int32)
        t = (cells % nt).astype(np.int32)
        s = rng.integers(0, 4, size=cells.size).astype(np.float64)   # many ties
        hits = {"d": d, "t": t, "snr": s}
        a1 = _nms_brute(d, t, s, 1, 1, np.ones(d.size, bool))
        a2 = _nms_brute(d, t, s, 5, 5, a1)
        assert np.array_equal(oracle.nms(hits, ndm, nt, ((1, 1),)), a1)
        assert np.array_equal(oracle.nms(hits, ndm, nt), a2)
        # survivors are pairwise outside the last window
        sd, st = d[a2], t[a2]
        for i in range(sd.size):
            for j in range(i + 1, sd.size):
                assert abs(int(sd[i]) - int(sd[j])) > 5 or abs(int(st[i]) - int(st[j])) > 5


def test_corner_turn_small_worked_example():
    """Two spectra of three channels: the rows of the output are the channels."""
    x_tc = np.array([[1, 2, 3], [4, 5, 6]], np.uint8)
    assert oracle.corner_turn(x_tc).tolist() == [[1, 4], [2, 5], [3, 6]]


def test_corner_turn_feeds_the_dm0_sum():
    """The DM-0 row of the channel-major block equals the per-spectrum channel sum."""
    rng = np.random.default_rng(3)
    x_tc = rng.integers(0, 256, size=(50, 16), dtype=np.uint8)
    x = oracle.corner_turn(x_tc)
    X = oracle.dedisperse(x, np.zeros((1, 16), np.int64), 50)
    assert np.array_equal(X[0], x_tc.astype(np.int64).sum(axis=1))
