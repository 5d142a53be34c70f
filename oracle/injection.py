"""Oracle of the quantised-domain signal injector (the appendix on injecting a signal into
an M-bit quantised data stream, and the injection section it supports).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product path never imports it.

Model (the appendix).  Gaussian noise N ~ Normal(mu, sigma) is quantised into 2^M states.
With K = 2^M/2 - 1 and the state index n tied to i = n - K, state n covers
[mu + (i-1) l sigma, mu + i l sigma); state 0 reaches down to -inf and state 2^M - 1 up to
+inf.  A signal S >= 0 added to the noise moves a sample in state n to state n + m with
probability P(n -> n+m) = (Gaussian mass of the part of state n that lands in state n+m
after the shift) / (Gaussian mass of state n): Eq. Pn->n+m for the interior and
Eqs. P0->0, P0->m, Pn->max, P0->max, Pmax->max at the boundary states.

Readings (where the appendix is silent or inconsistent):
  * the state interval is the one the equations use, [mu + (i-1) l sigma, mu + i l sigma),
    not the one the preceding sentence names (shifted by one level); only the former
    agrees with the boundary-state intervals the appendix gives;
  * a transition whose two intervals do not overlap has probability 0 (the printed
    differences turn negative there);
  * ``offset`` shifts every state edge by offset*l*sigma: 0 is the appendix's quantiser,
    -1/2 the rounding quantiser clip(round(mu + x)) with l*sigma = 1 of the synthetic
    8-bit data;
  * the new state is drawn from the row P(n -> .) by inverse CDF with a uniform variate
    u in (0, 1) (mode "sample": the exact conditional distribution of the quantised sum
    given the quantised noise, as the injection method it follows intends), or is the
    most probable state of the row, the smaller one on ties (mode "argmax": the
    figure's description of a bit shift);
  * S <= 0 or NaN, a byte above 2^M - 1, or a state of zero Gaussian mass in binary64
    leaves the sample unchanged.
Each difference of two CDF values is evaluated as the Gaussian mass of the interval
between them, on the side of the mean where it does not cancel (scipy's ndtr), so rows
stay accurate in the far tails of a fine quantiser.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import ndtr

SAMPLE, ARGMAX = 0, 1


@dataclass(frozen=True)
class Quantiser:
    bits: int          # M
    mu: float          # noise mean
    sigma: float       # noise standard deviation
    level: float       # l: level spacing in units of sigma
    offset: float = 0.0

    @property
    def levels(self) -> int:
        return 1 << self.bits


def _mass(lo, hi, mu: float, sigma: float):
    """Gaussian probability of [lo, hi) (0 where hi <= lo); lo may be -inf, hi +inf."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    zl = (lo - mu) / sigma
    zh = (hi - mu) / sigma
    upper = (zl + zh) > 0          # interval centred above the mean: use upper tails
    with np.errstate(invalid="ignore"):
        below = ndtr(zh) - ndtr(zl)
        above = ndtr(-zl) - ndtr(-zh)
    return np.where(hi > lo, np.where(upper, above, below), 0.0)


def transition_rows(n, S, q: Quantiser) -> np.ndarray:
    """Rows P(n -> .) for arrays of source states n and signals S (float64 [E, 2^M])."""
    n = np.asarray(n, dtype=np.int64).reshape(-1, 1)
    S = np.asarray(S, dtype=np.float64).reshape(-1, 1)
    levels = q.levels
    top = levels - 1
    K = levels // 2 - 1
    L = q.level * q.sigma
    k = np.arange(levels, dtype=np.int64).reshape(1, -1)
    m = k - n
    i = n - K
    mu, sig = q.mu, q.sigma

    def a(j):
        return mu + (j + q.offset) * L

    def mass(lo, hi):
        return _mass(lo, hi, mu, sig)

    ninf, pinf = -np.inf, np.inf
    with np.errstate(invalid="ignore", divide="ignore"):
        # Eq. Pn->n+m: interior source, interior destination.
        p_int = mass(np.maximum(a(i + m - 1) - S, a(i - 1)), np.minimum(a(i + m) - S, a(i))) / mass(a(i - 1), a(i))
        # Eq. Pn->max: interior source, top destination.
        p_nmax = mass(np.maximum(a(K) - S, a(i - 1)), a(i)) / mass(a(i - 1), a(i))
        # Eq. P0->0 and Eq. P0->m: bottom source.
        p_00 = mass(ninf, a(-K) - S) / mass(ninf, a(-K))
        p_0m = mass(a(m - K - 1) - S, np.minimum(a(m - K) - S, a(-K))) / mass(ninf, a(-K))
        # Eq. P0->max: bottom source, top destination.
        p_0max = mass(a(K) - S, a(-K)) / mass(ninf, a(-K))
    kk = np.broadcast_to(k, (n.shape[0], levels))
    nn = np.broadcast_to(n, kk.shape)
    P = np.zeros(kk.shape, dtype=np.float64)
    src0, srctop = nn == 0, nn == top
    dsttop = kk == top
    inner = ~src0 & ~srctop
    P = np.where(inner & (kk >= nn) & ~dsttop, p_int, P)
    P = np.where(inner & dsttop, p_nmax, P)
    P = np.where(src0 & (kk == 0) & ~dsttop, p_00, P)
    P = np.where(src0 & (kk > 0) & ~dsttop, p_0m, P)
    P = np.where(src0 & dsttop, p_0max, P)
    # Eq. Pmax->max: the top state stays.
    P = np.where(srctop, (kk == top).astype(np.float64), P)
    return P


def transition_matrix(S: float, q: Quantiser) -> np.ndarray:
    """The appendix's (upper-triangular) matrix P_ij for one signal value S."""
    return transition_rows(np.arange(q.levels), np.full(q.levels, S), q)


def source_mass(n, q: Quantiser) -> np.ndarray:
    """Gaussian mass of each source state (0 means the sample is left unchanged)."""
    n = np.asarray(n, dtype=np.int64)
    K = q.levels // 2 - 1
    L = q.level * q.sigma
    i = n - K
    lo = np.where(n == 0, -np.inf, q.mu + (i - 1 + q.offset) * L)
    hi = np.where(n == q.levels - 1, np.inf, q.mu + (i + q.offset) * L)
    return _mass(lo, hi, q.mu, q.sigma)


def choose(n, S, u, q: Quantiser, mode: int) -> np.ndarray:
    """New state per sample: inverse CDF of the row at u (SAMPLE) or its argmax (ARGMAX)."""
    n = np.asarray(n, dtype=np.int64).reshape(-1)
    S = np.asarray(S, dtype=np.float64).reshape(-1)
    out = n.copy()
    live = (n <= q.levels - 1) & (S > 0) & (source_mass(np.minimum(n, q.levels - 1), q) > 0)
    idx = np.nonzero(live)[0]
    if idx.size == 0:
        return out
    P = transition_rows(n[idx], S[idx], q)
    if mode == ARGMAX:
        out[idx] = np.argmax(P, axis=1)          # first maximum: the smaller state on ties
    else:
        u = np.asarray(u, dtype=np.float64).reshape(-1)[idx]
        C = np.cumsum(P, axis=1)
        below = u[:, None] < C
        below[:, -1] = True                      # the top state closes the row
        out[idx] = np.argmax(below, axis=1)
    return out


def uniform_from_words(r) -> np.ndarray:
    """u = (r + 1/2) 2^-32 for 32-bit random words r: uniform on (0, 1), never 0 or 1."""
    return (np.asarray(r, dtype=np.uint32).astype(np.float64) + 0.5) * (1.0 / 4294967296.0)


def inject(block: np.ndarray, n_t: int, t_start: np.ndarray, signal: np.ndarray, words, q: Quantiser,
           mode: int) -> np.ndarray:
    """Inject windows of signal into a quantised block [nch][pitch] (returns a copy).

    Window w adds signal[w][c][j] to sample t_start[w][c] + j of channel c; samples outside
    [0, n_t) are skipped.  Windows are applied in order (they should not overlap).
    ``words`` holds one 32-bit random word per signal value (unused in ARGMAX mode)."""
    out = block.copy()
    signal = np.asarray(signal, dtype=np.float32)
    n_win, nch, n_sig = signal.shape
    for w in range(n_win):
        for c in range(nch):
            t = int(t_start[w][c]) + np.arange(n_sig, dtype=np.int64)
            ok = (t >= 0) & (t < n_t)
            if not ok.any():
                continue
            tt = t[ok]
            src = out[c, tt].astype(np.int64)
            u = uniform_from_words(words[w][c][ok]) if mode == SAMPLE else None
            out[c, tt] = choose(src, signal[w][c][ok].astype(np.float64), u, q, mode).astype(np.uint8)
    return out


def quantise(x, q: Quantiser) -> np.ndarray:
    """State of each value: n = floor((x - mu)/(l sigma) - offset) + 2^M/2, clipped to the
    states; the inverse of the state intervals above."""
    z = np.floor((np.asarray(x, dtype=np.float64) - q.mu) / (q.level * q.sigma) - q.offset)
    return np.clip(z + q.levels // 2, 0, q.levels - 1).astype(np.int64)


def paper_level_8bit() -> float:
    """The level spacing the appendix adopts for 8-bit data (in units of sigma)."""
    return 0.030765


def synthetic_quantiser() -> Quantiser:
    """The synthetic 8-bit blocks: clip(round(128 + 16 n)), one level per unit."""
    return Quantiser(bits=8, mu=128.0, sigma=16.0, level=1.0 / 16.0, offset=-0.5)

