"""spl_batch_run_static (the search for callers that cannot allocate device memory)
against spl_batch_run on the same blocks: candidate lists and run statistics equal bit
for bit, on two calls in a row (the second with a smaller batch), and the ordinary
entry point still gives its results afterwards."""
import sys

import numpy as np
import pytest

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


def _blocks(spl, pd, plan, n_beams, seed):
    out = []
    for b in range(n_beams):
        spec = W.block_spec(pd, plan.info["n_in"], [synth.Pulse(t0=0.4 * pd["n_out"] + 37 * b, dm=250.0 - 40 * b,
                                                               fwhm=3.0 + b, snr=18.0)])
        out.append(spl.upload_block(synth.make_block(spec, seed, b, pd["widths"])[:, :plan.info["n_in"]]))
    return out


def _compare(spl, batch, blocks, cap, label):
    c_ref, s_ref = batch.run(blocks, spl.new_candidates(cap))
    c_st = torch.full((cap, 8), -7, dtype=torch.int32, device="cuda")
    s_st = torch.full((spl.STATS_WORDS,), -7, dtype=torch.int64, device="cuda")
    batch.run_static(blocks, c_st, s_st)
    torch.cuda.synchronize()
    a = spl.candidates_to_numpy(c_ref, s_ref)
    b = spl.candidates_to_numpy(c_st, s_st)
    say(f"{label}: {a.size} candidates, stats {spl.stats_dict(s_st)}")
    assert a.size > 0
    assert spl.stats_dict(s_ref) == spl.stats_dict(s_st)
    assert np.array_equal(a, b)
    return a


def test_static_entry_point_matches_batch_run(spl):
    # first call: three 256-channel beams of 8192 samples, 128 trials
    pd = W.plan_c1()
    plan = spl.Plan.from_dict(pd)
    big = spl.Batch([plan] * 3, hit_capacity=1 << 18)
    assert big.workspace_bytes() <= spl.STATIC_SCRATCH_BYTES
    xb = _blocks(spl, pd, plan, 3, seed=61)
    first = _compare(spl, big, xb, 1 << 14, "3 beams x 8192 samples")
    # second call: one beam of 2048 samples and fewer trials (a smaller input)
    ps = dict(pd, n_out=2048, norm_window=2048, dm_ranges=[(0.0, 3.90625, 100)])
    plan_s = spl.Plan.from_dict(ps)
    small = spl.Batch([plan_s], hit_capacity=1 << 16)
    xs = _blocks(spl, ps, plan_s, 1, seed=62)
    _compare(spl, small, xs, 1 << 12, "1 beam x 2048 samples")
    # the ordinary entry point of the first batch after the static calls
    c, s = big.run(xb, spl.new_candidates(1 << 14))
    torch.cuda.synchronize()
    assert np.array_equal(spl.candidates_to_numpy(c, s), first)


def test_static_entry_point_graph_batch(spl):
    """A batch created for the persistent graph mode runs eagerly through the static
    entry point, with the same results as its graph replay."""
    pd = W.plan_c1()
    plan = spl.Plan.from_dict(pd)
    batch = spl.Batch([plan] * 2, mode=spl.MODE_PERSISTENT_GRAPH, hit_capacity=1 << 18)
    xb = _blocks(spl, pd, plan, 2, seed=63)
    _compare(spl, batch, xb, 1 << 14, "graph batch, 2 beams")
