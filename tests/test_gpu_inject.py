"""GPU parity of the quantised-domain injector (spl_inject_quantised) against the oracle.

The new state of a sample is an integer decided by binary64 probabilities: both sides
decide in binary64, and the whole block must match byte for byte (untouched bytes
included).  A decision could differ only where u falls within rounding (~1e-15) of a
cumulative row sum; the seeded cases below hold none."""
import sys

import numpy as np
import pytest

from oracle import injection as inj
from paper_2606_27262_amd import synth
from paper_2606_27262_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_27262_amd import spotlight
    return spotlight


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(a, dtype=None):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def _gpu_inject(spl, block, n_t, t_start, signal, words, q, mode):
    d = _dev(block)
    spl.inject_quantised(d, _dev(t_start.astype(np.int32)), _dev(signal.astype(np.float32)),
                         None if words is None else _dev(words), bits=q.bits, mu=q.mu, sigma=q.sigma,
                         level=q.level, offset=q.offset, mode=mode, n_t=n_t)
    torch.cuda.synchronize()
    return d.cpu().numpy()


QUANTISERS = {
    "1bit": inj.Quantiser(1, 0.0, 1.0, 1.0),
    "2bit": inj.Quantiser(2, 0.1, 1.2, 0.9),
    "3bit_offset": inj.Quantiser(3, 0.2, 1.3, 0.6, offset=0.25),
    "8bit_paper": inj.Quantiser(8, 0.0, 1.0, inj.paper_level_8bit()),
    "8bit_synthetic": inj.synthetic_quantiser(),
}


@pytest.mark.parametrize("mode", [inj.SAMPLE, inj.ARGMAX])
@pytest.mark.parametrize("name", list(QUANTISERS))
def test_random_windows_match_oracle(spl, name, mode):
    """Three windows of 150 samples (several 64-sample groups and a ragged tail) on 64
    channels: states uniform over all levels (bytes above the top state included for
    fewer than 8 bits), signals of zero, negative, NaN, small and large size, starts
    before the block and past n_t."""
    q = QUANTISERS[name]
    say(f"inject parity {name} mode={mode}")
    rng = np.random.default_rng(list(QUANTISERS).index(name) * 31 + 17 * mode)
    nch, n_sig, n_win, pitch, n_t = 64, 150, 3, 1024, 760
    hi = 256 if q.bits == 8 else min(256, q.levels + 3)
    block = rng.integers(0, hi, (nch, pitch)).astype(np.uint8)
    t_start = (np.arange(n_win)[:, None] * 330 + rng.integers(-20, 20, (n_win, nch))).astype(np.int32)
    width = q.level * q.sigma
    sig = rng.exponential(2.0 * width, (n_win, nch, n_sig))
    pick = rng.random(sig.shape)
    sig[pick < 0.05] = 0.0
    sig[(pick >= 0.05) & (pick < 0.08)] = -1.0
    sig[(pick >= 0.08) & (pick < 0.09)] = np.nan
    sig[(pick >= 0.09) & (pick < 0.12)] *= 40.0
    sig = sig.astype(np.float32)
    words = rng.integers(0, 1 << 32, sig.shape, dtype=np.uint32)
    got = _gpu_inject(spl, block, n_t, t_start, sig, words if mode == inj.SAMPLE else None, q, mode)
    want = inj.inject(block, n_t, t_start, sig, words, q, mode)
    bad = np.argwhere(got != want)
    assert bad.size == 0, (bad[:5], got[tuple(bad[0])], want[tuple(bad[0])])
    assert np.any(got != block)


FULL_GROUPS = 8


@pytest.fixture(scope="module")
def full_size(spl):
    """Ten bursts of the 4096-channel, 16384-sample workload (DM 50-1800, FWHM 1-64,
    S/N 8-50) injected into one quantised noise block of 26305 samples per channel in
    SAMPLE mode on the GPU, once for the tests below."""
    plan = W.plan_c2()
    n_in = 26305
    rng = np.random.default_rng(31)
    pulses = synth.pulses_evenly(rng, 10, plan["n_out"], 50.0, 1800.0, 1.0, 64.0, 8.0, 50.0)
    spec = W.block_spec(plan, n_in)
    block = synth.make_block(spec, seed=31, beam=0, widths=plan["widths"])
    t_start, sig = synth.burst_windows(W.block_spec(plan, n_in, pulses), pulses, plan["widths"])
    words = synth.random_words(31, sig.shape)
    q = inj.synthetic_quantiser()
    say(f"inject full size: {sig.shape} values")
    got = _gpu_inject(spl, block, n_in, t_start, sig, words, q, inj.SAMPLE)
    return {"plan": plan, "n_in": n_in, "block": block, "t_start": t_start, "sig": sig, "words": words, "q": q,
            "got": got}


@pytest.mark.parametrize("group", range(FULL_GROUPS))
def test_full_size_beam_every_channel(spl, full_size, group):
    """Channels 512 g .. 512 g + 511 of the full-size injection equal the oracle's, byte for
    byte (the eight groups together cover all 4096 channels)."""
    f = full_size
    nch = f["plan"]["nchans"]
    chans = np.arange(group * nch // FULL_GROUPS, (group + 1) * nch // FULL_GROUPS)
    want = inj.inject(f["block"][chans], f["n_in"], f["t_start"][:, chans], f["sig"][:, chans],
                      f["words"][:, chans], f["q"], inj.SAMPLE)
    bad = np.argwhere(f["got"][chans] != want)
    assert bad.size == 0, (group, bad[:5])


def test_full_size_beam_outside_windows(spl, full_size):
    """Every byte outside the windows is unchanged, and a positive signal only raises a
    sample."""
    f = full_size
    block, got, t_start, sig, n_in = f["block"], f["got"], f["t_start"], f["sig"], f["n_in"]
    covered = np.zeros(block.shape, bool)
    for w in range(sig.shape[0]):
        for c in range(block.shape[0]):
            a = max(0, int(t_start[w, c]))
            b = min(n_in, int(t_start[w, c]) + sig.shape[2])
            if b > a:
                covered[c, a:b] = True
    assert np.array_equal(got[~covered], block[~covered])
    assert np.all(got >= block) and np.count_nonzero(got != block) > 0


def test_degenerate_calls(spl):
    block = np.full((4, 256), 128, np.uint8)
    d = _dev(block)
    ts = _dev(np.zeros((1, 4), np.int32))
    sig = _dev(np.ones((1, 4, 0), np.float32))
    spl.inject_quantised(d, ts, sig, None, mode=spl.INJECT_ARGMAX)      # n_sig = 0: no-op
    sig = _dev(np.ones((1, 4, 8), np.float32))
    spl.inject_quantised(d, ts, sig, None, mode=spl.INJECT_ARGMAX, n_t=0)  # n_t = 0: no-op
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), block)
    with pytest.raises(spl.SplError):
        spl.inject_quantised(d, ts, sig, None, mode=spl.INJECT_SAMPLE)    # SAMPLE needs words
    with pytest.raises(spl.SplError):
        spl.inject_quantised(d, ts, sig, None, bits=9, mode=spl.INJECT_ARGMAX)
    with pytest.raises(spl.SplError):
        spl.inject_quantised(d, ts, sig, None, sigma=0.0, mode=spl.INJECT_ARGMAX)


def _best_snr(spl, plan_dict, block):
    p = spl.Plan.from_dict(plan_dict)
    b = spl.Batch([p])
    cands = spl.new_candidates(1 << 14)
    cands, stats = b.run([spl.upload_block(block)], cands)
    torch.cuda.synchronize()
    c = spl.candidates_to_numpy(cands, stats)
    near = c[(np.abs(c["t_sample"].astype(int) - 4096) <= 16) & (np.abs(c["dm_index"].astype(int) - 64) <= 2)]
    return float(near["snr"].max()) if near.size else 0.0


def test_injected_pulse_recovers_pre_quantisation_snr(spl):
    """The 256-channel case's pulse (DM 250, FWHM 4, S/N 20) added to quantised noise by
    the injector is found by the search at the S/N of the same pulse added before
    quantisation: the injector draws from the exact conditional distribution, so over
    16 noise seeds the two S/N agree to sampling scatter."""
    plan = W.plan_c1()
    n_in = 19366
    pulse = synth.Pulse(t0=4096.0, dm=250.0, fwhm=4.0, snr=20.0)
    q = inj.synthetic_quantiser()
    diffs, pre_all = [], []
    for seed in range(16):
        pre = synth.make_block(W.block_spec(plan, n_in, [pulse]), seed=100 + seed, beam=0, widths=plan["widths"])
        noise = synth.make_block(W.block_spec(plan, n_in), seed=100 + seed, beam=0, widths=plan["widths"])
        t_start, sig = synth.burst_windows(W.block_spec(plan, n_in, [pulse]), [pulse], plan["widths"])
        words = synth.random_words(100 + seed, sig.shape)
        post = _gpu_inject(spl, noise, n_in, t_start, sig, words, q, inj.SAMPLE)
        s_pre = _best_snr(spl, plan, pre[:, :n_in])
        s_post = _best_snr(spl, plan, post[:, :n_in])
        diffs.append(s_post - s_pre)
        pre_all.append(s_pre)
    say(f"pre-quantisation S/N mean {np.mean(pre_all):.2f}; injector minus pre: mean {np.mean(diffs):+.3f}, "
        f"max |d| {np.max(np.abs(diffs)):.3f}")
    assert abs(np.mean(pre_all) - 20.0) < 1.0
    assert abs(np.mean(diffs)) < 0.3 and np.max(np.abs(diffs)) < 1.0
