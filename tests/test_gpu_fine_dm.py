"""GPU parity of the fine-DM snippets (spl_ranker_snippets_fine) against the oracle:
plane 0 (the DM transform over DM* +- dDM at 64 fine DMs, standardised by exact
moments) and plane 1 (the frequency-time plane, the same in both snippet calls) bit
for bit against the oracle, BF16 included."""
import sys

import numpy as np
import pytest

import oracle
from paper_2606_27262_amd import synth
from paper_2606_27262_amd import workloads as W
from plan_tables import assert_library_tables, oracle_plan

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


def _run(spl, plan_d, x):
    plan = spl.Plan.from_dict(plan_d)
    assert_library_tables(plan)
    batch = spl.Batch([plan])
    xb = spl.upload_block(x)
    cands = spl.new_candidates(1 << 16)
    cands, stats = batch.run([xb], cands)
    torch.cuda.synchronize()
    return plan, batch, xb, spl.candidates_to_numpy(cands, stats)


def _check(spl, plan, plan_d, batch, x, recs, keep):
    info = plan.info
    dev = torch.from_numpy(np.ascontiguousarray(recs).view(np.int32).reshape(-1, 8).copy()).cuda()
    fine = spl.snippets(batch, dev, fine_keep=keep)
    coarse = spl.snippets(batch, dev)
    torch.cuda.synchronize()
    g = fine.cpu().numpy().view(np.uint16)
    gc = coarse.cpu().numpy().view(np.uint16)
    o = oracle_plan(plan)
    dms = o["dms"]
    pd = plan.info
    # plane 1 needs only the block and the delays: a zero-strided stand-in of the DM
    # transform gives the oracle's shapes without computing plane 0
    X0 = np.broadcast_to(np.int64(0), (o["D"].shape[0], o["n_dd"]))
    for i, r in enumerate(recs):
        ok = (r["beam"] == 0 and 0 <= r["dm_index"] < pd["ndm"] and 0 <= r["t_sample"] < pd["n_out"]
              and r["width"] >= 1)
        if not ok:
            assert not g[i].any(), (i, r)
            continue
        ref = oracle.fine_dm_snippet(x, o["n_in"], plan_d["fch1"], plan_d["foff"], plan_d["tsamp"],
                                     float(dms[int(r["dm_index"])]), int(r["width"]), int(r["t_sample"]), keep)
        bad = np.argwhere(g[i, 0] != ref)
        assert bad.size == 0, (i, r, bad[:4])
        ref1 = oracle.snippets(x, o["D"], X0, o["n_out"], o["L"], int(r["dm_index"]), int(r["t_sample"]))[1]
        assert np.array_equal(g[i, 1], ref1), (i, r)
        assert np.array_equal(gc[i, 1], ref1), (i, r)


def _small(seed=3):
    nch, n_out, L = 128, 700, 256
    plan_d = {"nchans": nch, "fch1": 499.609375, "foff": -1.5625, "tsamp": 1.31072e-3, "n_out": n_out,
              "dm_ranges": [(0.0, 2.0, 70)], "widths": (1, 2, 4, 8, 16, 32), "threshold": 4.5, "norm_window": L}
    pulses = [synth.Pulse(t0=300.0, dm=60.0, fwhm=3.0, snr=25.0), synth.Pulse(t0=20.0, dm=4.0, fwhm=12.0, snr=15.0)]
    return plan_d, pulses


@pytest.mark.parametrize("keep", [0.1, 0.3])
def test_fine_snippets_small_bit_exact(spl, keep):
    """Search candidates of a 128-channel block plus edge records (first and last owned
    samples, DM 0 whose fine rows go negative, the widest width) and records that name
    nothing (zero planes)."""
    plan_d, pulses = _small()
    spl_plan = spl.Plan.from_dict(plan_d)
    n_in = spl_plan.info["n_in"]
    x = synth.make_block(W.block_spec(plan_d, n_in, pulses), 3, 0, plan_d["widths"])[:, :n_in]
    plan, batch, xb, got = _run(spl, plan_d, x)
    say(f"fine snippets keep={keep}: {got.size} candidates")
    assert got.size >= 3
    extra = np.zeros(8, oracle.CAND_DTYPE)
    ndm, n_out = plan.info["ndm"], plan.info["n_out"]
    extra["dm_index"] = [0, ndm - 1, 5, 0, ndm - 1, 0, 0, 3]
    extra["t_sample"] = [0, n_out - 1, 3, 400, 0, n_out, 10, 50]
    extra["width"] = [1, 32, 4, 32, 1, 1, 1, 0]
    extra["beam"] = [0, 0, 0, 0, 0, 0, 1, 0]
    recs = np.concatenate([got[:200], extra])
    _check(spl, plan, plan_d, batch, x, recs, keep)
    del xb


def test_fine_snippets_full_size_sample(spl):
    """The 4096-channel, 16384-sample workload with ten pulses (64 channels per sub-band
    of plane 1): 24 of its candidates (the strongest and a spread of the rest) checked
    bit for bit."""
    pd = W.plan_c2()
    plan0 = spl.Plan.from_dict(pd)
    n_in = plan0.info["n_in"]
    spec, x = W.c2_like_block(pd, n_in, 2, 0, 10)
    x = x[:, :n_in]
    plan, batch, xb, got = _run(spl, pd, x)
    say(f"fine snippets full size: {got.size} candidates")
    order = np.argsort(-got["snr"])
    pick = np.unique(np.concatenate([order[:12], order[:: max(1, order.size // 12)][:12]]))
    _check(spl, plan, pd, batch, x, got[pick], 0.1)
    del xb
