"""The five workloads of the build, as plan parameters plus a seeded input recipe.

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
           "c1_block", "c2_like_block", "batch_c3_plans", "batch_c4_plans", "dm_max",
           "real_time_s", "describe"]
