"""Pins of the quantised-domain injection oracle against what the appendix and the
mathematics fix: its printed 1-bit and 2-bit closed forms, the exact conditional
distribution it models (Monte Carlo of injection before quantisation), and the special
cases S = 0, S a whole number of states, and the top state."""
import math

import numpy as np
import pytest

from oracle import injection as inj


def _cdf(x, mu, sigma):
    # the appendix's noise CDF, from the standard library's erf (not the oracle's routine)
    return 0.5 * (1.0 + math.erf((x - mu) / (sigma * math.sqrt(2.0))))


MU, SIG, ELL = 0.3, 1.7, 0.8
SIGNALS = (0.05, 0.4, 1.0, 1.36, 1.9, 3.1, 6.0)


def _pos(v):
    # transitions whose intervals do not overlap have probability 0
    return max(0.0, v)


@pytest.mark.parametrize("S", SIGNALS)
def test_one_bit_closed_forms(S):
    """Eqs. P0to1 and P0to1_2: P(0->1) = 1 - phi(mu - S)/0.5, P(0->0) = phi(mu - S)/0.5,
    P(1->0) = 0, P(1->1) = 1."""
    P = inj.transition_matrix(S, inj.Quantiser(1, MU, SIG, ELL))
    phi = lambda x: _cdf(x, MU, SIG)
    assert P[0, 1] == pytest.approx(1 - phi(MU - S) / 0.5, abs=1e-14)
    assert P[0, 0] == pytest.approx(phi(MU - S) / 0.5, abs=1e-14)
    assert P[1, 0] == 0.0 and P[1, 1] == 1.0


@pytest.mark.parametrize("S", SIGNALS)
def test_two_bit_closed_forms(S):
    """The appendix's 2-bit equations P00, P01, P02, P03, P11, P12, P13, P22, P23, P33."""
    P = inj.transition_matrix(S, inj.Quantiser(2, MU, SIG, ELL))
    phi = lambda x: _cdf(x, MU, SIG)
    ls = ELL * SIG
    mu = MU
    want = {
        (0, 0): phi(mu - ls - S) / phi(mu - ls),
        (0, 1): _pos(phi(min(mu - S, mu - ls)) - phi(mu - ls - S)) / phi(mu - ls),
        (0, 2): _pos(phi(min(mu + ls - S, mu - ls)) - phi(mu - S)) / phi(mu - ls),
        (0, 3): _pos(phi(mu - ls) - phi(mu + ls - S)) / phi(mu - ls),
        (1, 1): _pos(phi(mu - S) - phi(mu - ls)) / (0.5 - phi(mu - ls)),
        (1, 2): _pos(phi(min(mu + ls - S, mu)) - phi(max(mu - S, mu - ls))) / (0.5 - phi(mu - ls)),
        (1, 3): _pos(0.5 - phi(max(mu + ls - S, mu - ls))) / (0.5 - phi(mu - ls)),
        (2, 2): _pos(phi(mu + ls - S) - 0.5) / (phi(mu + ls) - 0.5),
        (2, 3): _pos(phi(mu + ls) - phi(max(mu + ls - S, mu))) / (phi(mu + ls) - 0.5),
        (3, 3): 1.0,
    }
    for (a, b), v in want.items():
        assert P[a, b] == pytest.approx(v, abs=1e-13), (a, b)
    # below the diagonal: the signal only raises a sample
    assert np.all(np.tril(P, -1) == 0)


def _quantise_by_thresholds(x, q):
    # state = number of state edges at or below x (independent of the oracle's formula)
    half = q.levels // 2
    edges = q.mu + (np.arange(1 - half, half, dtype=np.float64) + q.offset) * q.level * q.sigma
    return np.searchsorted(edges, x, side="right")


QUANTISERS = [
    inj.Quantiser(1, 0.0, 1.0, 1.0),
    inj.Quantiser(2, 0.0, 1.0, 0.9),
    inj.Quantiser(3, 0.2, 1.3, 0.6, offset=0.25),
    inj.Quantiser(8, 0.0, 1.0, inj.paper_level_8bit()),
]


@pytest.mark.parametrize("qi", range(len(QUANTISERS)))
@pytest.mark.parametrize("S_states", (0.3, 1.7, 5.2))
def test_rows_match_injection_before_quantisation(qi, S_states):
    """The row P(n -> .) is the distribution of quantise(N + S) given quantise(N) = n for
    Gaussian N: compared with a Monte Carlo of that definition (binomial bound)."""
    q = QUANTISERS[qi]
    S = S_states * q.level * q.sigma
    rng = np.random.default_rng(1000 + 10 * qi + int(10 * S_states))
    N = rng.normal(q.mu, q.sigma, 3_000_000)
    a = _quantise_by_thresholds(N, q)
    b = _quantise_by_thresholds(N + S, q)
    P = inj.transition_matrix(S, q)
    checked = 0
    for n in np.unique(a):
        sel = b[a == n]
        if sel.size < 3000:
            continue
        emp = np.bincount(sel, minlength=q.levels) / sel.size
        tol = 6 * np.sqrt(P[n] * (1 - P[n]) / sel.size) + 3.0 / sel.size
        assert np.all(np.abs(emp - P[n]) <= tol), (n, emp[n:n + 4], P[n, n:n + 4])
        checked += 1
    assert checked >= min(q.levels, 2)


def test_synthetic_quantiser_matches_the_data_generator():
    """offset -1/2 with one level per unit is clip(round(128 + 16 n)), the synthetic blocks'
    quantiser: Monte Carlo of injection before that exact rounding."""
    q = inj.synthetic_quantiser()
    rng = np.random.default_rng(77)
    N = rng.normal(128.0, 16.0, 4_000_000)
    for S in (0.37, 2.5, 11.2):
        a = np.clip(np.rint(N), 0, 255).astype(np.int64)
        b = np.clip(np.rint(N + S), 0, 255).astype(np.int64)
        for n in (100, 128, 150):
            sel = b[a == n]
            P = inj.transition_rows([n], [S], q)[0]
            emp = np.bincount(sel, minlength=256) / sel.size
            tol = 6 * np.sqrt(P * (1 - P) / sel.size) + 3.0 / sel.size
            assert np.all(np.abs(emp - P) <= tol), (S, n)


@pytest.mark.parametrize("qi", range(len(QUANTISERS)))
def test_rows_are_distributions(qi):
    q = QUANTISERS[qi]
    for S in (0.0, 0.01, 0.77, 3.3, 40.0):
        P = inj.transition_matrix(S, q)
        assert np.all(P >= 0)
        assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
    assert np.array_equal(inj.transition_matrix(0.0, q), np.eye(q.levels))


def test_whole_state_shift_is_exact():
    """S an integer number k of state widths moves every interior state exactly k up
    (saturating at the top)."""
    q = inj.Quantiser(8, 0.0, 1.0, 0.125)
    for k in (1, 3, 7):
        P = inj.transition_matrix(k * 0.125, q)
        for n in range(1, 255):
            dest = min(255, n + k)
            assert P[n, dest] == pytest.approx(1.0, abs=1e-9), (k, n)


def test_strong_signal_saturates_and_state_zero_spreads():
    q = inj.Quantiser(8, 0.0, 1.0, inj.paper_level_8bit())
    P = inj.transition_matrix(100.0, q)
    assert np.allclose(P[:, 255], 1.0)
    P = inj.transition_matrix(0.5, q)
    # state 0 is unbounded below: a shift of ~16 states spreads it over many states
    assert np.count_nonzero(P[0] > 1e-6) > 5


def test_choose_sample_inverts_the_row_cdf():
    q = inj.Quantiser(3, 0.0, 1.0, 0.5)
    S = 0.9
    P = inj.transition_rows([2], [S], q)[0]
    u = (np.arange(100000) + 0.5) / 100000
    k = inj.choose(np.full(u.size, 2), np.full(u.size, S), u, q, inj.SAMPLE)
    freq = np.bincount(k, minlength=q.levels) / u.size
    assert np.allclose(freq, P, atol=2e-5)


def test_choose_argmax_and_ties():
    q = inj.synthetic_quantiser()
    # state 128 = [127.5, 128.5) is centred on the mean: a shift of half a state splits it
    # into two equal halves; the tie goes to the smaller state
    assert inj.choose([128], [0.5], None, q, inj.ARGMAX)[0] == 128
    assert inj.choose([128], [0.6], None, q, inj.ARGMAX)[0] == 129
    assert inj.choose([100], [2.2], None, q, inj.ARGMAX)[0] == 102
    assert inj.choose([100], [2.8], None, q, inj.ARGMAX)[0] == 103


def test_unchanged_samples():
    q = inj.Quantiser(2, 0.0, 1.0, 0.9)
    n = np.array([1, 1, 1, 5, 3])
    S = np.array([0.0, -1.0, np.nan, 2.0, 2.0])
    out = inj.choose(n, S, np.full(5, 0.99), q, inj.SAMPLE)
    assert out.tolist() == [1, 1, 1, 5, 3]


def test_inject_windows_and_block_edges():
    q = inj.synthetic_quantiser()
    rng = np.random.default_rng(5)
    block = np.clip(np.rint(rng.normal(128, 16, (3, 40))), 0, 255).astype(np.uint8)
    t_start = np.array([[-4, 10, 35]], np.int32)
    signal = np.full((1, 3, 8), 3.0, np.float32)
    words = rng.integers(0, 1 << 32, (1, 3, 8), dtype=np.uint32)
    out = inj.inject(block, 40, t_start, signal, words, q, inj.ARGMAX)
    d = out.astype(int) - block.astype(int)
    # an interior state shifted by exactly 3 states moves 3 up; outside the windows or
    # beyond [0, n_t) nothing changes
    assert np.all(d[0, :4] == 3) and np.all(d[0, 4:] == 0)
    assert np.all(d[1, 10:18] == 3) and np.all(d[1, :10] == 0) and np.all(d[1, 18:] == 0)
    assert np.all(d[2, 35:40] == 3) and np.all(d[2, :35] == 0)


def test_uniform_words_are_open_interval():
    u = inj.uniform_from_words(np.array([0, 0xFFFFFFFF], np.uint32))
    assert 0 < u[0] < 1e-9 and 1 - 1e-9 < u[1] < 1
