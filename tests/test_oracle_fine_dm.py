"""Pins of the fine-DM DM-time plane of the oracle: its half-range against Eq. snrloss
and the corrected Eq. deltadm, its centre row against the (pinned) dedispersion of the
search, its other rows against a direct brute force, and the fall of a strong pulse's
peak across the plane against Eq. snrloss."""
import math

import numpy as np
import pytest

import oracle
from paper_2606_27262_amd import synth


def _band(nch, lo, hi):
    fch1, foff = synth.band_edges(nch, lo, hi)
    return fch1, foff


@pytest.mark.parametrize("nch,lo,hi,tsamp,width", [(4096, 550.0, 750.0, 1.31072e-3, 1),
                                                   (4096, 550.0, 750.0, 1.31072e-3, 64),
                                                   (2048, 300.0, 500.0, 0.65536e-3, 8)])
@pytest.mark.parametrize("keep", [0.1, 0.05])
def test_half_range_keeps_the_requested_snr(nch, lo, hi, tsamp, width, keep):
    """At dDM the full Eq. snrloss (with erf) gives `keep`: the large-zeta form is exact
    there since erf(zeta) = 1 for zeta = sqrt(pi)/(2 keep) >= 8.8."""
    fch1, foff = _band(nch, lo, hi)
    half = oracle.fine_dm_half_range(width, tsamp, fch1, foff, nch, keep)
    f = fch1 + np.arange(nch) * foff
    nu = (f.max() + f.min()) / 2 / 1000.0
    kept = oracle.snr_kept(half, width * tsamp * 1000.0, nch * abs(foff), nu)
    assert kept == pytest.approx(keep, rel=1e-12)


def test_half_range_is_corrected_eq_deltadm():
    """Eq. deltadm written with W in seconds and nu in MHz has the constant sqrt(pi)/13820;
    the printed sqrt(pi)/1382 is ten times larger (it drops a factor 10 when converting
    W_ms nu_GHz^3 to W_s nu_MHz^3)."""
    nch, tsamp, width, keep = 4096, 1.31072e-3, 4, 0.1
    fch1, foff = _band(nch, 550.0, 750.0)
    half = oracle.fine_dm_half_range(width, tsamp, fch1, foff, nch, keep)
    nu_mhz = 650.0
    w_s = width * tsamp
    corrected = math.sqrt(math.pi) / 13820 * w_s * (1 / keep) * nu_mhz ** 3 / (nch * abs(foff))
    assert half == pytest.approx(corrected, rel=1e-12)
    printed = math.sqrt(math.pi) / 1382 * w_s * (1 / keep) * nu_mhz ** 3 / (nch * abs(foff))
    assert printed == pytest.approx(10 * half, rel=1e-12)
    # the band-4 example: a 5 ms pulse, 90 % loss -> about 8.8 pc cm^-3
    h5 = oracle.fine_dm_half_range(1, 5e-3, fch1, foff, nch, 0.1)
    assert 8.7 < h5 < 8.9


def _block(nch, lo, hi, tsamp, n_in, pulses, seed=3):
    fch1, foff = _band(nch, lo, hi)
    spec = synth.BlockSpec(nch=nch, fch1=fch1, foff=foff, tsamp=tsamp, n_in=n_in, pulses=pulses)
    return spec, synth.make_block(spec, seed, 0)[:, :n_in]


def test_centre_row_is_the_search_dm_transform_row():
    """Row 32 sits exactly at the trial DM: it equals that trial's row of the search's DM
    transform (standardisation aside: compared before it, through the integer moments)."""
    nch, tsamp, n_in = 64, 1e-3, 3000
    spec, x = _block(nch, 400.0, 500.0, tsamp, n_in, [synth.Pulse(t0=900.0, dm=60.0, fwhm=3.0, snr=30.0)])
    dms = np.arange(0, 100, 1.0)
    D, _ = oracle.delay_table(nch, spec.fch1, spec.foff, tsamp, dms)
    n_dd = n_in - int(D.max())
    X = oracle.dedisperse(x, D, n_dd)
    d, t = 60, 900
    got = oracle.fine_dm_snippet(x, n_in, spec.fch1, spec.foff, tsamp, float(dms[d]), 2, t)
    # the plane rebuilt by brute force, standardised by its own exact moments
    ref = np.zeros((64, 256), np.int64)
    step = oracle.fine_dm_half_range(2, tsamp, spec.fch1, spec.foff, nch) / 32.0
    fd = np.array([dms[d] + (r - 32) * step for r in range(64)])
    FD, _ = oracle.delay_table(nch, spec.fch1, spec.foff, tsamp, fd)
    assert np.array_equal(FD[32], D[d])
    ts = np.arange(t - 128, t + 128)
    for r in range(64):
        for c in range(nch):
            ref[r] += x[c, ts + FD[r, c]]
    assert np.array_equal(ref[32], X[d, t - 128:t + 128])
    mu, sg = oracle._mu_sigma_exact(ref.reshape(-1))
    want = oracle.f32_to_bf16_bits(((ref - mu) / sg).astype(np.float32))
    assert np.array_equal(got, want)


def test_edges_invalid_and_zero():
    """Entries whose samples fall outside [0, n_in) for some channel are 0, and the
    moments cover only valid entries."""
    nch, tsamp, n_in = 32, 1e-3, 1200
    spec, x = _block(nch, 400.0, 500.0, tsamp, n_in, [])
    got = oracle.bf16_bits_to_f32(oracle.fine_dm_snippet(x, n_in, spec.fch1, spec.foff, tsamp, 40.0, 16, 60))
    step = oracle.fine_dm_half_range(16, tsamp, spec.fch1, spec.foff, nch) / 32.0
    fd = np.array([40.0 + (r - 32) * step for r in range(64)])
    FD, _ = oracle.delay_table(nch, spec.fch1, spec.foff, tsamp, fd)
    ts = np.arange(60 - 128, 60 + 128)
    for r in range(64):
        bad = (ts + FD[r].min() < 0) | (ts + FD[r].max() >= n_in)
        assert np.all(got[r, bad] == 0)
    assert np.all(got[:, :68] == 0)      # t < 0
    valid = got != 0
    assert valid.sum() > 100 and abs(float(got[valid].mean())) < 0.1


def test_strong_pulse_falls_to_keep_at_the_plane_edges():
    """A strong pulse (S/N 400, FWHM 6 samples) at its trial DM: row 32 holds the peak and
    the rows dDM away keep about 10 % of it (Eq. snrloss; loose: the boxcar width stands
    in for the FWHM and the sampling grid blurs the profile)."""
    nch, tsamp, n_in = 256, 1.31072e-3, 10000
    dm = 300.0                    # sweeps ~6750 samples across the band
    spec, x = _block(nch, 300.0, 500.0, tsamp, n_in, [synth.Pulse(t0=2000.0, dm=dm, fwhm=6.0, snr=400.0)])
    plane = oracle.bf16_bits_to_f32(oracle.fine_dm_snippet(x, n_in, spec.fch1, spec.foff, tsamp, dm, 6, 2000))
    peak = plane.max(axis=1)
    assert int(np.argmax(peak)) in range(30, 35)
    edge = 0.5 * (peak[0] + peak[63])
    assert 0.03 < edge / peak[32] < 0.3
    # symmetric fall-off either side of the centre
    assert abs(peak[16] - peak[48]) < 0.15 * peak[32]
