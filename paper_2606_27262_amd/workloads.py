"""The benchmark and test workloads, as plan parameters plus a seeded input recipe.

Shapes follow the paper's setting (8-bit samples, uGMRT Band 3 300-500 MHz and
Band 4 550-750 MHz, 1.31072 ms sampling, DM up to 2000 and beyond, boxcar
widths in powers of two, a 6-sigma threshold).  The inputs are synthetic
stand-ins for the paper's beam data (see ``synth``).

A plan here is a plain dict:
  nchans, fch1, foff, tsamp, n_out, norm_window,
  dm_ranges [(start, step, n)], widths, threshold.
The block length n_in depends on the plan's delay table, so the recipes take it
as an argument: callers obtain it from the plan they built.
"""
from __future__ import annotations


import numpy as np

from . import synth

W64 = (1, 2, 4, 8, 16, 32, 64)
W256 = (1, 2, 4, 8, 16, 32, 64, 128, 256)


def make_plan(nchans, f_lo, f_hi, tsamp, n_out, dm_lo, dm_hi, n_trials, widths,
              threshold=6.0, norm_window=0):
    fch1, foff = synth.band_edges(nchans, f_lo, f_hi)
    # n trials uniformly spaced over [lo, hi): step (hi - lo)/n, end excluded
    return dict(nchans=nchans, fch1=fch1, foff=foff, tsamp=tsamp, n_out=n_out,
                norm_window=norm_window or n_out,
                dm_ranges=[(float(dm_lo), (dm_hi - dm_lo) / n_trials, int(n_trials))],
                widths=tuple(widths), threshold=float(threshold))


def plan_c1():
    """1 beam, 256 ch over 300-500 MHz, 8192 samples, 128 trials 0-500, widths 1..64."""
    return make_plan(256, 300.0, 500.0, 1.31072e-3, 8192, 0.0, 500.0, 128, W64)


def plan_c2():
    """1 beam, 4096 ch over 550-750 MHz, 16384 samples, 2048 trials 0-2000, widths 1..256."""
    return make_plan(4096, 550.0, 750.0, 1.31072e-3, 16384, 0.0, 2000.0, 2048, W256)


def plan_band3_c4():
    """2048 ch over 300-500 MHz at 0.65536 ms, 32768 samples, 1024 trials 0-1000."""
    return make_plan(2048, 300.0, 500.0, 0.65536e-3, 32768, 0.0, 1000.0, 1024, W256)


def plan_band4_c4():
    """4096 ch over 550-750 MHz at 1.31072 ms, 16384 samples, 3072 trials 0-3000."""
    return make_plan(4096, 550.0, 750.0, 1.31072e-3, 16384, 0.0, 3000.0, 3072, W256)


def block_spec(plan, n_in, pulses=(), rfi=None, zero_dm=()):
    pers, inter = rfi if rfi else ((), ())
    return synth.BlockSpec(nch=plan["nchans"], fch1=plan["fch1"], foff=plan["foff"],
                           tsamp=plan["tsamp"], n_in=n_in, pulses=list(pulses),
                           rfi_channels_persistent=pers, rfi_channels_intermittent=inter,
                           zero_dm_bursts=list(zero_dm))


def c1_block(n_in, seed=1, beam=0, with_pulse=True, snr=20.0):
    """One pulse at DM 250 (trial 64), FWHM 4 samples, S/N 20, t0 = 4096."""
    plan = plan_c1()
    pulses = [synth.Pulse(t0=4096.0, dm=250.0, fwhm=4.0, snr=snr)] if with_pulse else []
    spec = block_spec(plan, n_in, pulses)
    return spec, synth.make_block(spec, seed, beam, plan["widths"])


def c2_like_block(plan, n_in, seed, beam, n_pulses, dm_max_pulse=1800.0, rfi_frac=0.02,
                  zero_dm_rate=0.0, fwhm_hi=64.0):
    """Pulses with DM ~ U(50, dm_max_pulse), FWHM log-U(1, fwhm_hi), S/N ~ U(8, 50);
    2% RFI channels (half persistent, half intermittent); optional zero-DM bursts."""
    rng = np.random.default_rng([seed, beam, 12345])
    pulses = synth.pulses_evenly(rng, n_pulses, plan["n_out"], 50.0, dm_max_pulse,
                                 1.0, fwhm_hi, 8.0, 50.0)
    rfi = synth.rfi_channels(rng, plan["nchans"], rfi_frac) if rfi_frac > 0 else None
    zd = synth.zero_dm_bursts(rng, n_in, plan["tsamp"], zero_dm_rate) if zero_dm_rate > 0 else ()
    spec = block_spec(plan, n_in, pulses, rfi, zd)
    return spec, synth.make_block(spec, seed, beam, plan["widths"])


def c2_like_block_torch(plan, n_in, seed, beam, n_pulses, dm_max_pulse=1800.0, rfi_frac=0.02,
                        zero_dm_rate=0.0, fwhm_hi=64.0, device="cuda"):
    """c2_like_block's recipe (same pulses, RFI channels and zero-DM bursts for the same
    seed and beam) made with torch on `device` (synth.make_block_torch: torch's noise):
    a uint8 tensor [nch][pitch]."""
    rng = np.random.default_rng([seed, beam, 12345])
    pulses = synth.pulses_evenly(rng, n_pulses, plan["n_out"], 50.0, dm_max_pulse,
                                 1.0, fwhm_hi, 8.0, 50.0)
    rfi = synth.rfi_channels(rng, plan["nchans"], rfi_frac) if rfi_frac > 0 else None
    zd = synth.zero_dm_bursts(rng, n_in, plan["tsamp"], zero_dm_rate) if zero_dm_rate > 0 else ()
    spec = block_spec(plan, n_in, pulses, rfi, zd)
    return spec, synth.make_block_torch(spec, seed, beam, plan["widths"], device=device)


def stream_series(plan, n_blocks, n_in, seed, beam, n_pulses_per_block, dm_max_pulse=1800.0, rfi_frac=0.02,
                  zero_dm_rate=0.0, fwhm_hi=64.0, period=0, device=None):
    """A continuous stream of one beam, in blocks: block k owns stream samples
    [k n_out, (k+1) n_out) and reads [k n_out, k n_out + n_in) (the overlap tail of the
    plan).  Pulses with DM ~ U(50, dm_max_pulse), FWHM log-U(1, fwhm_hi), S/N ~ U(8, 50),
    n_pulses_per_block in evenly spaced slots of every block's owned samples, 2 % RFI
    channels, optional zero-DM bursts.

    period = 0: the series holds n_in + (n_blocks - 1) n_out samples.  period = m > 0:
    the series holds m n_out samples and the stream repeats it (block k reads it modulo
    its length, so blocks k and k + m are equal); a pulse's DM is capped so that its
    whole sweep ends before the period does (no pulse crosses the wrap).
    Returns the series uint8 [nch][length] (numpy; with a torch device, a tensor made
    there by synth.make_block_torch) and, per block of one period (or of the whole
    series), the pulses with t0 relative to that block's first sample."""
    n_out = plan["n_out"]
    length = period * n_out if period else n_in + (n_blocks - 1) * n_out
    n_own = period if period else n_blocks
    rng = np.random.default_rng([seed, beam, 54321])
    probe = block_spec(plan, length)
    k_bottom = float(synth.arrival_offsets(probe, 1.0).max())    # samples per unit DM, lowest channel
    pulses, per_block = [], []
    for k in range(n_own):
        ps = synth.pulses_evenly(rng, n_pulses_per_block, n_out, 50.0, dm_max_pulse, 1.0, fwhm_hi, 8.0, 50.0)
        mine = []
        for p in ps:
            t0 = p.t0 + k * n_out
            dm = p.dm
            if period:
                dm = min(dm, (length - t0 - 4.0 * p.fwhm - 8.0) / k_bottom)
            q = synth.Pulse(t0=t0, dm=max(dm, 0.0), fwhm=p.fwhm, snr=p.snr)
            pulses.append(q)
            mine.append(synth.Pulse(t0=p.t0, dm=q.dm, fwhm=p.fwhm, snr=p.snr))
        per_block.append(mine)
    rfi = synth.rfi_channels(rng, plan["nchans"], rfi_frac) if rfi_frac > 0 else None
    zd = synth.zero_dm_bursts(rng, length, plan["tsamp"], zero_dm_rate) if zero_dm_rate > 0 else ()
    spec = block_spec(plan, length, pulses, rfi, zd)
    if device is not None:
        return synth.make_block_torch(spec, seed, beam, plan["widths"], device=device)[:, :length], per_block
    x = synth.make_block(spec, seed, beam, plan["widths"])
    return x[:, :length], per_block


def stream_block(series, n_out, n_in, k):
    """Block k of a stream series (periodic when the series is shorter than the block's
    end): samples [k n_out, k n_out + n_in) modulo the series length."""
    L = series.shape[1]
    idx = (k * n_out + np.arange(n_in)) % L
    return series[:, idx]


def batch_c3_plans():
    """24 beams of the 4096-channel Band-4 plan (one GPU's share of 2000 beams on 90 GPUs)."""
    return [plan_c2() for _ in range(24)]


def batch_c4_plans():
    """32 beams alternating the Band-3 and Band-4 plans above."""
    return [plan_band3_c4() if b % 2 == 0 else plan_band4_c4() for b in range(32)]


def dm_max(plan):
    s, st, n = plan["dm_ranges"][-1]
    return s + st * n


def real_time_s(plan):
    """Duration of the samples one block owns."""
    return plan["n_out"] * plan["tsamp"]


def describe(plan):
    r = plan["dm_ranges"]
    if len(r) == 1:
        s, st, n = r[0]
        dm = f"dm={s}+{st}x{n}"
    else:
        dm = (f"dm={r[0][0]}-{r[-1][0] + (r[-1][2] - 1) * r[-1][1]} in {len(r)} ranges "
              f"(steps {'/'.join(str(x[1]) for x in r)}, {sum(x[2] for x in r)} trials)")
    return (f"{plan['nchans']}ch f1={plan['fch1']:.6f} df={plan['foff']:.6f} "
            f"ts={plan['tsamp'] * 1e3:.5f}ms n_out={plan['n_out']} {dm} "
            f"w<= {max(plan['widths'])}")


__all__ = ["make_plan", "plan_c1", "plan_c2", "plan_band3_c4", "plan_band4_c4", "block_spec",
           "c1_block", "c2_like_block", "c2_like_block_torch", "stream_series", "stream_block", "batch_c3_plans", "batch_c4_plans", "dm_max",
           "real_time_s", "describe"]
