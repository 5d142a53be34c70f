"""Pins of the oracle's delay table (Eq. (1) of the dedispersion section).

Independent of the oracle's own code: physical scaling laws of the cold-plasma
delay, the printed dispersion constant, and an exact-rational evaluation of the
same real number that reproduces every rounding away from half-integer ties.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2606_27262_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "eq1_dispersion_constant.txt")


def _golden_constant():
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("dispersion_constant_MHz2_pc-1_cm3_s"):
                return line.split("=")[1].strip()
    raise AssertionError("constant missing from golden file")


def _plan_table(plan):
    dms = oracle.dm_trials(plan["dm_ranges"])
    D, ties = oracle.delay_table(plan["nchans"], plan["fch1"], plan["foff"], plan["tsamp"], dms)
    return dms, D, ties


def test_golden_constant_matches_oracle():
    assert Fraction(_golden_constant()) == Fraction("4148.8064239")
    assert oracle.DISPERSION_CONSTANT == float(_golden_constant())


def test_dm_zero_and_reference_channel_are_zero():
    for plan in (W.plan_c1(), W.plan_c2(), W.plan_band3_c4()):
        dms, D, _ = _plan_table(plan)
        assert dms[0] == 0.0
        assert np.all(D[0] == 0)
        assert np.all(D[:, 0] == 0)        # channel 0 is the highest frequency


def test_monotone_in_dm_and_frequency():
    for plan in (W.plan_c1(), W.plan_c2()):
        _, D, _ = _plan_table(plan)
        assert np.all(np.diff(D, axis=0) >= 0)   # more DM, more delay
        assert np.all(np.diff(D, axis=1) >= 0)   # lower frequency, more delay


def test_order_of_magnitude_4p149_ms_per_ghz2():
    # delay of 1 GHz relative to 2 GHz at DM 100: 4.1488 ms * 100 * (1 - 1/4)
    dms = np.array([100.0])
    D, _ = oracle.delay_table(2, 2000.0, -1000.0, 1e-6, dms)
    expect_s = 4.1488064239e-3 * 100 * (1.0 - 0.25)
    assert abs(D[0, 1] * 1e-6 - expect_s) <= 0.5e-6


def test_spot_value_band3_dm1000():
    # DM 1000 across 500 -> 300 MHz: 29.5026 s
    D, _ = oracle.delay_table(2, 500.0, -200.0, 1e-6, np.array([1000.0]))
    assert abs(D[0, 1] * 1e-6 - 29.5026) < 1e-4


def test_linear_in_dm_and_inverse_square_in_frequency():
    plan = W.plan_c2()
    dms = np.array([500.0, 1000.0, 2000.0])
    D, _ = oracle.delay_table(plan["nchans"], plan["fch1"], plan["foff"], 1e-7, dms)
    # rounding error at most 1/2 sample per entry
    assert np.all(np.abs(D[1] - 2 * D[0]) <= 1)
    assert np.all(np.abs(D[2] - 2 * D[1]) <= 1)
    f = plan["fch1"] + np.arange(plan["nchans"]) * plan["foff"]
    law = (f ** -2 - f[0] ** -2) / (f[-1] ** -2 - f[0] ** -2)
    assert np.allclose(D[2] / D[2, -1], law, atol=2.0 / D[2, -1])


def test_reversed_channel_order():
    # ascending frequency: the reference is the last channel
    nch = 64
    fch1, foff = W.synth.band_edges(nch, 300.0, 500.0)
    f_asc0 = fch1 + (nch - 1) * foff
    dms = np.array([0.0, 300.0])
    Dd, _ = oracle.delay_table(nch, fch1, foff, 1e-3, dms)
    Da, _ = oracle.delay_table(nch, f_asc0, -foff, 1e-3, dms)
    assert np.array_equal(Dd[:, ::-1], Da)
    assert np.all(Da[:, -1] == 0)


def _exact_round(dm, f, fref, tsamp, K):
    v = K * Fraction(dm) * (1 / (Fraction(f) ** 2) - 1 / (Fraction(fref) ** 2)) / Fraction(tsamp)
    return math.floor(v + Fraction(1, 2)), v


@pytest.mark.parametrize("mk", [W.plan_c1, W.plan_c2, W.plan_band3_c4])
def test_exact_rational_reevaluation(mk):
    """Every sampled entry equals round-half-up of the exact real value built from
    the FP64 inputs (no entry sits within 1e-9 of a tie)."""
    plan = mk()
    dms, D, ties = _plan_table(plan)
    assert ties == 0
    K = Fraction(_golden_constant())
    nch = plan["nchans"]
    f = [plan["fch1"] + c * plan["foff"] for c in range(nch)]   # channel centres, FP64
    fref = max(f)
    rng = np.random.default_rng(7)
    n = min(D.size, 3000)
    picks = rng.choice(D.size, size=n, replace=False)
    picks = np.concatenate([picks, [D.size - 1]])
    for k in picks:
        d, c = divmod(int(k), nch)
        r, v = _exact_round(dms[d], f[c], fref, plan["tsamp"], K)
        assert abs((v - math.floor(v)) - Fraction(1, 2)) > Fraction(1, 10 ** 9)
        assert D[d, c] == r, (d, c, float(v))


def test_plan_sizes_match_derived_table():
    # s_max and block length for the benchmark plans, from Eq. (1) by hand
    for mk, s_max, n_in in ((W.plan_c1, 11111, 19366), (W.plan_c2, 9666, 26305),
                            (W.plan_band3_c4, 44946, 77969), (W.plan_band4_c4, 14501, 31140)):
        plan = mk()
        _, D, _ = _plan_table(plan)
        sz = oracle.sizes(D, plan["n_out"], plan["widths"])
        assert sz["s_max"] == s_max and sz["n_in"] == n_in
        # largest delay from the continuous formula, lowest channel, last DM
        f = plan["fch1"] + (plan["nchans"] - 1) * plan["foff"]
        dm_last = oracle.dm_trials(plan["dm_ranges"])[-1]
        cont = 4148.8064239 * dm_last * (f ** -2 - plan["fch1"] ** -2) / plan["tsamp"]
        assert abs(cont - s_max) <= 0.5


def test_dm_250_is_trial_64_in_c1():
    dms = oracle.dm_trials(W.plan_c1()["dm_ranges"])
    assert dms.size == 128 and dms[64] == 250.0 and dms[1] == 3.90625


# ---------------------------------------------------------------- smearing-limited plans
def test_snr_kept_closed_forms():
    # no offset keeps everything
    assert oracle.snr_kept(0.0, 1.0, 200.0, 0.65) == 1.0
    # z = 1: (sqrt(pi)/2) erf(1) = integral of exp(-t^2) over [0, 1] = 0.746824132812427...
    ddm = 1.0 / (6.91e-3 * 200.0 / (1.0 * 0.65 ** 3))
    assert abs(oracle.snr_kept(ddm, 1.0, 200.0, 0.65) - 0.7468241328124271) < 1e-14
    # far off: the sqrt(pi) / (2 z) asymptote of the approximate form
    z = 6.0
    assert abs(oracle.snr_kept(z * ddm, 1.0, 200.0, 0.65) * 2 * z / math.sqrt(math.pi) - 1.0) < 1e-15


def _ranges_check(nch, fch1, foff, tsamp, lo, hi, loss, wmin=0.0):
    r = oracle.smearing_ranges(nch, fch1, foff, tsamp, lo, hi, loss, wmin)
    edge = [fch1, fch1 + (nch - 1) * foff]
    fl, fh = min(edge), max(edge)
    bw, nu_c, nu_lo = nch * abs(foff), (fl + fh) / 2e3, fl / 1e3

    def allowed(step, dm):
        tc = 8.3e-3 * dm * abs(foff) / nu_lo ** 3
        w = math.sqrt((wmin * 1e3) ** 2 + (tsamp * 1e3) ** 2 + tc ** 2)
        return oracle.snr_kept(step / 2, w, bw, nu_c) >= 1 - loss

    assert r[0][0] == lo
    for k, (start, step, n) in enumerate(r):
        assert n >= 1 and math.frexp(step)[0] == 0.5          # a power of two
        assert allowed(step, start)
        if k + 1 < len(r):
            nxt = r[k + 1]
            assert nxt[1] == 2 * step and nxt[0] == start + n * step   # contiguous, doubled
            assert allowed(2 * step, nxt[0])                            # switched when allowed ...
            assert n == 1 or not allowed(2 * step, start + (n - 1) * step)   # ... and not before
        else:
            assert start + (n - 1) * step >= hi and (n == 1 or start + (n - 2) * step < hi)
    assert not allowed(2 * r[0][1], lo)   # the first step is the largest allowed
    return r


@pytest.mark.parametrize("band", ["c1", "c2", "b3", "b5"])
def test_smearing_ranges_follow_their_definition(band):
    bands = {"c1": (256, 499.609375, -0.78125, 1.31072e-3), "c2": (4096, 749.9755859375, -0.048828125, 1.31072e-3),
             "b3": (2048, 499.951171875, -0.09765625, 0.65536e-3), "b5": (2048, 1459.90234375, -0.1953125, 0.65536e-3)}
    for loss in (0.05, 0.1, 0.2):
        r = _ranges_check(*bands[band], 0.0, 2000.0, loss)
        assert len(r) >= 1
    # a smaller tolerated loss needs more trials; a wider minimum pulse fewer
    n = lambda r: sum(x[2] for x in r)
    assert n(oracle.smearing_ranges(*bands[band], 0.0, 2000.0, 0.05)) > n(oracle.smearing_ranges(*bands[band], 0.0, 2000.0, 0.2))
    assert n(oracle.smearing_ranges(*bands[band], 0.0, 2000.0, 0.1, 2e-3)) < n(oracle.smearing_ranges(*bands[band], 0.0, 2000.0, 0.1))


def test_intra_channel_smearing_constant():
    """8.3 us per MHz of channel width and unit DM at 1 GHz (Cordes & McLaughlin): at
    1 GHz with 1 MHz channels a DM of 1000 smears 8.3 ms within a channel; the effective
    width the generator uses at that DM with 1 ms sampling is sqrt(1 + 8.3^2) ms."""
    tc = 8.3e-3 * 1000.0 * 1.0 / (1.0 ** 3)
    assert abs(tc - 8.3) < 1e-12
    # the generator's first step at DM 1000 equals the one for that width at DM 0
    r_hi = oracle.smearing_ranges(16, 1008.0, -1.0, 1e-3, 1000.0, 1001.0, 0.1)
    r_w = oracle.smearing_ranges(16, 1008.0, -1.0, 1e-3, 0.0, 1.0, 0.1, w_min_s=8.3e-3 * 1000 * 1.0 / (0.993 ** 3) * 1e-3)
    assert r_hi[0][1] == r_w[0][1]
