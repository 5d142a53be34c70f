"""The torch evaluation of the synthetic-block recipe (used for large training sets on
the GPU) against the numpy generator: identical blocks when the receiver noise is left
out (pulses, RFI channels, zero-DM bursts, rounding and clipping), and noise with the
quantised Gaussian's moments."""
import math

import numpy as np
import pytest

from paper_2606_27262_amd import synth
from paper_2606_27262_amd import workloads as W

torch = pytest.importorskip("torch")


def _spec(seed):
    pd = W.make_plan(256, 300.0, 500.0, 1.31072e-3, 4096, 0.0, 250.0, 64, W.W64)
    rng = np.random.default_rng(seed)
    pulses = synth.pulses_evenly(rng, 4, pd["n_out"], 20.0, 240.0, 1.0, 64.0, 6.0, 40.0)
    rfi = synth.rfi_channels(rng, pd["nchans"], 0.05)
    zd = synth.zero_dm_bursts(rng, 9000, pd["tsamp"], 2.0)
    assert zd and rfi[0] and rfi[1]
    return pd, W.block_spec(pd, 9000, pulses, rfi, zd)


def test_noise_free_blocks_are_identical():
    for seed in (1, 2):
        pd, spec = _spec(seed)
        a = synth.make_block_torch(spec, seed, 3, pd["widths"], device="cpu", noise=False).numpy()
        b = synth.make_block(spec, seed, 3, pd["widths"], noise=False)
        assert a.shape == b.shape and np.array_equal(a, b)


def test_noise_moments_and_seeding():
    spec = synth.BlockSpec(nch=64, fch1=500.0, foff=-1.0, tsamp=1e-3, n_in=40000)
    a = synth.make_block_torch(spec, 9, 0, device="cpu").numpy()[:, :spec.n_in].astype(np.float64)
    n = a.size
    # clip(round(128 + 16 n)): mean 128, variance 256 + 1/12 (clipping at 0 and 255 is 8 sigma away)
    assert abs(a.mean() - 128.0) < 5 * synth.QUANT_SIGMA / math.sqrt(n)
    assert abs(a.var() / synth.QUANT_SIGMA ** 2 - 1.0) < 5 * math.sqrt(2.0 / n)
    b = synth.make_block_torch(spec, 9, 0, device="cpu").numpy()
    c = synth.make_block_torch(spec, 9, 1, device="cpu").numpy()
    assert np.array_equal(a, b[:, :spec.n_in]) and not np.array_equal(b, c)
