"""Seeded synthetic filterbank blocks (stand-ins for uGMRT beam data).

This module only *makes inputs*: Gaussian receiver noise quantised to 8 bits,
dispersed Gaussian-profile pulses added before quantisation, and RFI.  It holds
none of the search's arithmetic (no delay table, no dedispersion, no boxcars);
the sky model below computes the continuous arrival time of each channel on its
own.  Both the HIP path and the CPU oracle consume its output.

Random numbers come from numpy's counter-based Philox generator keyed by
(seed, beam) with the channel chunk in the counter, so a block is independent of
thread count and of the order in which chunks are drawn.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
from scipy.special import ndtr

# Cold-plasma constant used by the sky model to place pulses (MHz^2 pc^-1 cm^3 s).
_KDM = 4148.8064239
NOISE_MEAN = 128.0
NOISE_SIGMA = 16.0
# Standard deviation of clip(round(128 + 16 n)) for n ~ N(0, 1): sqrt(256 + 1/12).
QUANT_SIGMA = math.sqrt(256.0 + 1.0 / 12.0)
_CHUNK = 64


@dataclass
class Pulse:
    t0: float        # arrival time (samples) at the highest channel centre
    dm: float        # pc cm^-3
    fwhm: float      # samples
    snr: float       # ideal matched-boxcar S/N (see pulse_amplitude)


@dataclass
class BlockSpec:
    nch: int
    fch1: float      # MHz, centre of channel 0 (highest frequency)
    foff: float      # MHz, negative: frequency falls with channel index
    tsamp: float     # s
    n_in: int        # samples per channel row
    pitch: int = 0   # row pitch in bytes (0: n_in rounded up to 256)
    pulses: list = field(default_factory=list)
    rfi_channels_persistent: tuple = ()
    rfi_channels_intermittent: tuple = ()
    zero_dm_bursts: list = field(default_factory=list)  # (t0, width, amp_sigma)

    def row_pitch(self) -> int:
        return self.pitch if self.pitch else (self.n_in + 255) // 256 * 256


def band_edges(nch: int, f_lo: float, f_hi: float):
    """Channel 0 is the highest frequency; channel centres sit half a channel
    inside the band edges."""
    df = (f_hi - f_lo) / nch
    return f_hi - df / 2.0, -df


def _rng(seed: int, beam: int, chunk: int, salt: int = 0) -> np.random.Generator:
    key = np.array([(seed & 0xFFFFFFFF) | ((salt & 0xFFFF) << 32), beam & 0xFFFFFFFFFFFFFFFF],
                   dtype=np.uint64)
    ctr = np.array([0, 0, 0, chunk], dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key, counter=ctr))


def _bin_profile(centre: float, fwhm: float, t_lo: int, n: int) -> np.ndarray:
    """Integral over each sample bin [t, t+1) of a unit-height Gaussian of the
    given FWHM centred at `centre` (samples)."""
    s = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    t = np.arange(t_lo, t_lo + n + 1, dtype=np.float64)
    cdf = ndtr((t - centre) / s)
    return s * math.sqrt(2.0 * math.pi) * np.diff(cdf)


def pulse_amplitude(p: Pulse, nch: int, widths) -> float:
    """Per-channel amplitude (quantisation units) giving the ideal S/N p.snr:
    perfectly dedispersed, noise-free, sigma_n = QUANT_SIGMA*sqrt(nch), best
    boxcar of the plan's widths at the best anchor."""
    s = p.fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    half = int(math.ceil(6 * s + max(widths) + 2))
    lo = int(math.floor(p.t0)) - half
    g = _bin_profile(p.t0, p.fwhm, lo, 2 * half + 1)
    best = 0.0
    c = np.concatenate([[0.0], np.cumsum(g)])
    for w in widths:
        if w > g.size:
            continue
        sums = c[w:] - c[:-w]
        best = max(best, float(sums.max()) / math.sqrt(w))
    return p.snr * QUANT_SIGMA / (math.sqrt(nch) * best)


def arrival_offsets(spec: BlockSpec, dm: float) -> np.ndarray:
    """Continuous arrival time of each channel relative to the highest channel
    centre, in samples (sky model)."""
    f = spec.fch1 + np.arange(spec.nch, dtype=np.float64) * spec.foff
    fref = f.max()
    return _KDM * dm * (1.0 / f ** 2 - 1.0 / fref ** 2) / spec.tsamp


def pulse_template(spec: BlockSpec, p: Pulse, amp: float):
    """Noise-free dispersed pulse as (row index, column start, values[nch, K])."""
    s = p.fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    K = int(math.ceil(12 * s)) + 4
    centres = p.t0 + arrival_offsets(spec, p.dm)
    starts = np.floor(centres - 6 * s).astype(np.int64) - 1
    t = starts[:, None] + np.arange(K + 1)[None, :]
    cdf = ndtr((t - centres[:, None]) / s)
    vals = amp * s * math.sqrt(2.0 * math.pi) * np.diff(cdf, axis=1)
    return starts, vals


def _chunk_rows(spec: BlockSpec, seed: int, beam: int, ci: int, widths, noise: bool = True) -> np.ndarray:
    c0 = ci * _CHUNK
    c1 = min(spec.nch, c0 + _CHUNK)
    if noise:
        rng = _rng(seed, beam, ci)
        v = rng.standard_normal((c1 - c0, spec.n_in), dtype=np.float32)
        v *= NOISE_SIGMA
        v += NOISE_MEAN
    else:
        v = np.full((c1 - c0, spec.n_in), NOISE_MEAN, np.float32)
    # persistent RFI: +3 sigma offset, twice the variance
    for c in spec.rfi_channels_persistent:
        if c0 <= c < c1:
            v[c - c0] = (v[c - c0] - NOISE_MEAN) * math.sqrt(2.0) + NOISE_MEAN + 3 * NOISE_SIGMA
    # intermittent RFI: on/off bursts of 10-500 samples, 20% duty, log-U(1, 8) sigma
    for c in spec.rfi_channels_intermittent:
        if c0 <= c < c1:
            r = _rng(seed, beam, c, salt=1)
            t = int(r.integers(0, 500))
            while t < spec.n_in:
                length = int(r.integers(10, 501))
                amp = math.exp(r.uniform(0.0, math.log(8.0))) * NOISE_SIGMA
                v[c - c0, t:t + length] += amp
                t += length + int(length * 4 * r.uniform(0.5, 1.5))
    for (t0, width, amp) in spec.zero_dm_bursts:
        lo, hi = max(0, int(t0)), min(spec.n_in, int(t0) + int(width))
        if hi > lo:
            v[:, lo:hi] += float(amp) * NOISE_SIGMA
    for p in spec.pulses:
        amp = pulse_amplitude(p, spec.nch, widths)
        starts, vals = pulse_template(spec, p, amp)
        for r in range(c0, c1):
            a = int(starts[r])
            b = a + vals.shape[1]
            lo, hi = max(a, 0), min(b, spec.n_in)
            if hi > lo:
                v[r - c0, lo:hi] += vals[r, lo - a:hi - a].astype(np.float32)
    np.rint(v, out=v)
    np.clip(v, 0, 255, out=v)
    return v.astype(np.uint8)


def make_block(spec: BlockSpec, seed: int, beam: int = 0, widths=(1, 2, 4, 8, 16, 32, 64),
               threads: int = 8, noise: bool = True) -> np.ndarray:
    """uint8 block [nch][pitch]; samples beyond n_in in each row are 0.  noise=False
    leaves the receiver noise out (every sample starts at the mean)."""
    pitch = spec.row_pitch()
    out = np.zeros((spec.nch, pitch), np.uint8)
    nchunks = (spec.nch + _CHUNK - 1) // _CHUNK

    def work(ci):
        rows = _chunk_rows(spec, seed, beam, ci, widths, noise)
        out[ci * _CHUNK: ci * _CHUNK + rows.shape[0], :spec.n_in] = rows

    if threads > 1 and nchunks > 1:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(work, range(nchunks)))
    else:
        for ci in range(nchunks):
            work(ci)
    return out


def make_block_torch(spec: BlockSpec, seed: int, beam: int = 0, widths=(1, 2, 4, 8, 16, 32, 64),
                     device="cuda", noise: bool = True):
    """The same recipe as make_block, evaluated with torch on `device` (for training sets
    of many blocks): Gaussian noise from torch's generator seeded by (seed, beam) (so the
    noise differs from make_block's Philox stream; everything else is the same sky
    model), RFI channels, zero-DM bursts and pulses added in float32 before rounding to
    the nearest integer (ties to even) and clipping to 0..255.  noise=False leaves the
    noise out (the deterministic part, for checking against make_block).  Returns a
    uint8 tensor [nch][pitch] on `device`; samples beyond n_in are 0."""
    import torch
    nch, n_in = spec.nch, spec.n_in
    if noise:
        g = torch.Generator(device=device)
        g.manual_seed((int(seed) * 1000003 + int(beam) * 7919 + 12345) & 0x7FFFFFFFFFFFFFFF)
        v = torch.randn((nch, n_in), generator=g, device=device, dtype=torch.float32)
        v.mul_(NOISE_SIGMA).add_(NOISE_MEAN)
    else:
        v = torch.full((nch, n_in), NOISE_MEAN, device=device, dtype=torch.float32)
    for c in spec.rfi_channels_persistent:
        v[c] = (v[c] - NOISE_MEAN) * math.sqrt(2.0) + NOISE_MEAN + 3 * NOISE_SIGMA
    if spec.rfi_channels_intermittent:
        add = np.zeros((len(spec.rfi_channels_intermittent), n_in), np.float32)
        for i, c in enumerate(spec.rfi_channels_intermittent):
            r = _rng(seed, beam, c, salt=1)
            t = int(r.integers(0, 500))
            while t < n_in:
                length = int(r.integers(10, 501))
                amp = math.exp(r.uniform(0.0, math.log(8.0))) * NOISE_SIGMA
                add[i, t:t + length] += amp
                t += length + int(length * 4 * r.uniform(0.5, 1.5))
        idx = torch.tensor(spec.rfi_channels_intermittent, device=device, dtype=torch.long)
        v.index_add_(0, idx, torch.from_numpy(add).to(device))
    for (t0, width, amp) in spec.zero_dm_bursts:
        lo, hi = max(0, int(t0)), min(n_in, int(t0) + int(width))
        if hi > lo:
            v[:, lo:hi] += float(amp) * NOISE_SIGMA
    flat = v.view(-1)
    rows = torch.arange(nch, device=device, dtype=torch.long)[:, None]
    for p in spec.pulses:
        amp = pulse_amplitude(p, nch, widths)
        s = p.fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
        K = int(math.ceil(12 * s)) + 4
        centres = torch.from_numpy(p.t0 + arrival_offsets(spec, p.dm)).to(device)
        starts = torch.floor(centres - 6 * s).to(torch.long) - 1
        t = starts[:, None] + torch.arange(K + 1, device=device, dtype=torch.long)[None, :]
        cdf = torch.special.ndtr((t.to(torch.float64) - centres[:, None]) / s)
        vals = (amp * s * math.sqrt(2.0 * math.pi) * torch.diff(cdf, dim=1)).to(torch.float32)
        cols = t[:, :K]
        ok = (cols >= 0) & (cols < n_in)
        flat.index_add_(0, (rows * n_in + cols)[ok], vals[ok])
    torch.round(v, out=v)
    v.clamp_(0.0, 255.0)
    out = torch.zeros((nch, spec.row_pitch()), dtype=torch.uint8, device=device)
    out[:, :n_in] = v.to(torch.uint8)
    return out


# --------------------------------------------------------------------------
# Workload recipes (the benchmark and test workloads: stand-ins for uGMRT data)
# --------------------------------------------------------------------------
def pulses_evenly(rng: np.random.Generator, n: int, n_out: int, dm_lo: float, dm_hi: float,
                  fwhm_lo: float, fwhm_hi: float, snr_lo: float, snr_hi: float):
    """n pulses in evenly spaced slots of the owned samples (small jitter),
    DM uniform, FWHM log-uniform, S/N uniform."""
    out = []
    slot = n_out / (n + 1)
    for i in range(n):
        t0 = slot * (i + 1) + rng.uniform(-0.1, 0.1) * slot
        dm = rng.uniform(dm_lo, dm_hi)
        fwhm = math.exp(rng.uniform(math.log(fwhm_lo), math.log(fwhm_hi)))
        snr = rng.uniform(snr_lo, snr_hi)
        out.append(Pulse(t0=t0, dm=dm, fwhm=fwhm, snr=snr))
    return out


def rfi_channels(rng: np.random.Generator, nch: int, frac: float = 0.02):
    k = int(round(frac * nch))
    ch = rng.choice(nch, size=k, replace=False)
    ch.sort()
    return tuple(int(c) for c in ch[: k // 2]), tuple(int(c) for c in ch[k // 2:])


def zero_dm_bursts(rng: np.random.Generator, n_in: int, tsamp: float, rate_hz: float = 0.2):
    k = rng.poisson(rate_hz * n_in * tsamp)
    return [(float(rng.integers(0, n_in)), int(rng.integers(1, 33)), float(rng.uniform(1.0, 4.0)))
            for _ in range(k)]


# --------------------------------------------------------------------------
# Inputs of the quantised-domain injector
# --------------------------------------------------------------------------
def burst_windows(spec: BlockSpec, pulses, widths=(1, 2, 4, 8, 16, 32, 64)):
    """Noise-free dispersed pulses as injector windows: (t_start int32 [n_win][nch],
    signal float32 [n_win][nch][n_sig]), one window per pulse, zero-padded to the widest
    window; the amplitudes are those make_block adds before quantisation."""
    temps = [pulse_template(spec, p, pulse_amplitude(p, spec.nch, widths)) for p in pulses]
    n_sig = max((v.shape[1] for _, v in temps), default=0)
    t_start = np.zeros((len(temps), spec.nch), np.int32)
    signal = np.zeros((len(temps), spec.nch, n_sig), np.float32)
    for w, (starts, vals) in enumerate(temps):
        t_start[w] = starts.astype(np.int32)
        signal[w, :, :vals.shape[1]] = vals
    return t_start, signal


def random_words(seed: int, shape, salt: int = 7) -> np.ndarray:
    """Uniform 32-bit words (the injector's random draws), seeded."""
    rng = _rng(seed, 0, 0, salt=salt)
    return rng.integers(0, 1 << 32, size=shape, dtype=np.uint32)
