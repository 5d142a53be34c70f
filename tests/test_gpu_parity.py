"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer results (DM transform, moments, candidate lists incl. widths and boxcar
sums) must match bit for bit; the float32 S/N of a candidate is the binary64 S/N
of the oracle rounded to float32, so it matches exactly too (tolerance 0).
"""
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


def gpu_run(spl, plans, blocks, mode=0, hit_capacity=0, cand_cap=1 << 16, batch=None):
    for p in {id(p): p for p in plans}.values():
        assert_library_tables(p)
    if batch is None:
        batch = spl.Batch(plans, mode=mode, hit_capacity=hit_capacity)
    tb = [spl.upload_block(x) for x in blocks]
    cands = spl.new_candidates(cand_cap)
    cands, stats = batch.run(tb, cands)
    torch.cuda.synchronize()
    out = {"cands": spl.candidates_to_numpy(cands, stats), "stats": spl.stats_dict(stats),
           "batch": batch, "X": [], "S1": [], "S2": []}
    for b, p in enumerate(plans):
        out["X"].append(batch.dm_transform(b)[:, :p.info["n_dd"]].cpu().numpy().astype(np.int64))
        s1, s2 = batch.moments(b)
        out["S1"].append(s1.cpu().numpy())
        out["S2"].append(s2.cpu().numpy())
    return out


def oracle_search(p, x, beam=0):
    """The oracle's whole search of one beam on its own view of the plan (delay table,
    DM values and sizes rebuilt from the plan's arguments), with its moments."""
    o = oracle_plan(p)
    r = oracle.search_beam(x[:, :o["n_in"]], o["D"], o["dms"], o["n_out"], o["L"], o["widths"], o["threshold"],
                           stencils=o["stencils"], beam=beam)
    n, s1, s2 = oracle.moments(r["X"], o["n_out"], o["L"])
    r["S1"], r["S2"] = s1, s2
    return r


def oracle_run(plans, blocks):
    res = [oracle_search(p, x, b) for b, (p, x) in enumerate(zip(plans, blocks))]
    cands = np.concatenate([r["cands"] for r in res]) if res else np.zeros(0, oracle.CAND_DTYPE)
    return res, cands


def make_plan(spl, nch, ndm, n_out, widths, theta, L=0, delays=None, dms=None, stencils=((1, 1), (5, 5)),
              plan_dict=None):
    if plan_dict is not None:
        return spl.Plan.from_dict(plan_dict, stencils=stencils)
    return spl.Plan(nch, 500.0, -0.5, 1e-3, n_out, widths=widths, threshold=theta, norm_window=L,
                    delays=delays, dms=dms, stencils=stencils)


def compare(g, ref_beams, ref_cands, check_X=True):
    for b, r in enumerate(ref_beams):
        if check_X:
            assert np.array_equal(g["X"][b], r["X"]), f"X differs (beam {b})"
            assert np.array_equal(g["S1"][b], r["S1"]) and np.array_equal(g["S2"][b], r["S2"]), f"moments (beam {b})"
    assert g["stats"]["hit_overflow"] == 0
    assert g["stats"]["n_hits"] == sum(r["hits"]["d"].size for r in ref_beams)
    assert g["cands"].size == ref_cands.size, (g["cands"].size, ref_cands.size)
    assert np.array_equal(g["cands"], ref_cands)


def test_normaliser_hook_matches_oracle(spl):
    rng = np.random.default_rng(0)
    n = rng.integers(1, 40000, 4000).astype(np.int64)
    v = rng.integers(0, 1_100_000, 4000).astype(np.int64)
    s1 = n * v + rng.integers(0, 1000, 4000)
    var = rng.integers(0, 1 << 40, 4000)
    s2 = np.minimum(n * v * v + var, (1 << 62))
    # consistent moments for the edge cases: constant rows (V = 0) and tiny V
    s1[:10] = n[:10] * v[:10]
    s2[:10] = n[:10] * v[:10] * v[:10]
    s2[10:20] = n[10:20] * v[10:20] * v[10:20] + 1
    s1[10:20] = n[10:20] * v[10:20]
    ok = (n.astype(object) * s2.astype(object) - s1.astype(object) ** 2) >= 0
    n, s1, s2 = n[ok], s1[ok], s2[ok]
    mu, sg = spl.debug_mu_sigma(torch.from_numpy(n).cuda(), torch.from_numpy(s1).cuda(), torch.from_numpy(s2).cuda())
    mu, sg = mu.cpu().numpy(), sg.cpu().numpy()
    for k in range(n.size):
        m, s = oracle.mu_sigma(n[k], s1[k], s2[k])
        assert mu[k] == m and sg[k] == s, (k, n[k], s1[k], s2[k], mu[k], m, sg[k], s)


def _random_monotone_delays(rng, ndm, nch, smax):
    steps = rng.integers(0, 3, size=(ndm, nch))
    D = np.cumsum(np.cumsum(steps, axis=1), axis=0)
    D = D - D[:, :1]
    if D.max() > smax:
        D = (D * smax) // max(1, D.max())
    return D.astype(np.int32)


@pytest.mark.parametrize("mode", [0, 1])
def test_small_random_batches(spl, mode):
    """Uneven small plans in one batch (ragged tiles, several segments, odd sizes)."""
    rng = np.random.default_rng(11 + mode)
    for trial in range(4):
        plans, blocks = [], []
        for b in range(int(rng.integers(1, 4))):
            nch = int(rng.integers(1, 80))
            ndm = int(rng.integers(1, 70))
            n_out = int(rng.integers(1, 3000))
            widths = tuple(sorted(set(int(w) for w in rng.choice([1, 2, 3, 4, 8, 16, 33], size=3))))
            widths = tuple(w for w in widths if w <= n_out) or (1,)
            L = int(rng.integers(1, n_out + 1)) if rng.random() < 0.5 else 0
            D = _random_monotone_delays(rng, ndm, nch, int(rng.integers(0, 400)))
            p = make_plan(spl, nch, ndm, n_out, widths, 2.0, L=L, delays=D)
            x = rng.integers(0, 256, size=(nch, p.info["n_in"]), dtype=np.uint8)
            if rng.random() < 0.3:
                x[:] = 7   # constant input: sigma = 0, no hits
            plans.append(p)
            blocks.append(x)
        say("trial", trial, [(p.info["nchans"], p.info["ndm"], p.info["n_out"]) for p in plans])
        g = gpu_run(spl, plans, blocks, mode=mode)
        ref, rc = oracle_run(plans, blocks)
        compare(g, ref, rc)


@pytest.mark.parametrize("mode", [0, 1])
def test_stencil_sets_of_every_length(spl, mode):
    """Plans with one to four peak filters of different sizes in one batch: the first
    filter runs over all hits, the later ones over its compacted survivors (a third and
    fourth filter read the flags of the compacted pass before), and beams whose plan has
    fewer filters pass the later ones unchanged.  Candidates bit for bit."""
    rng = np.random.default_rng(61 + mode)
    sets = [((1, 1),), ((1, 1), (3, 2), (5, 5)), ((2, 3), (4, 1), (1, 1), (6, 6)), ((1, 1), (5, 5)), ()]
    plans, blocks = [], []
    for b, st in enumerate(sets):
        nch, ndm, n_out = int(rng.integers(8, 48)), int(rng.integers(20, 60)), int(rng.integers(1500, 3000))
        D = _random_monotone_delays(rng, ndm, nch, int(rng.integers(20, 300)))
        p = make_plan(spl, nch, ndm, n_out, (1, 2, 4, 8), 2.0, delays=D, stencils=st)
        x = rng.integers(0, 256, size=(nch, p.info["n_in"]), dtype=np.uint8)
        plans.append(p)
        blocks.append(x)
    g = gpu_run(spl, plans, blocks, mode=mode)
    ref, rc = oracle_run(plans, blocks)
    say("stencil sets: hits", g["stats"]["n_hits"], "candidates", rc.size, "after each filter",
        g["stats"]["n_after_stencil"])
    compare(g, ref, rc)


def test_c1_full(spl):
    p = make_plan(spl, 0, 0, 0, None, 0, plan_dict=W.plan_c1())
    _, x = W.c1_block(p.info["n_in"], seed=1)
    blocks = [x[:, :p.info["n_in"]]]
    g = gpu_run(spl, [p], blocks)
    ref, rc = oracle_run([p], blocks)
    compare(g, ref, rc)
    best = g["cands"][np.argmax(g["cands"]["snr"])]
    assert best["dm_index"] == 64 and abs(int(best["t_sample"]) - 4096) <= 8


@pytest.mark.parametrize("mode", [0, 1])
def test_smearing_plan_batch(spl, mode):
    """A multi-range plan from the smearing-limited generator (seven sub-ranges, steps
    1/16 .. 4) on the 256-channel band, two beams with pulses at low and high DM:
    DM transform and candidates bit for bit."""
    pd = W.plan_c1()
    pd["n_out"] = pd["norm_window"] = 3000
    pd["dm_ranges"] = spl.smearing_ranges(pd["nchans"], pd["fch1"], pd["foff"], pd["tsamp"], 0.0, 500.0, 0.1)
    assert len(pd["dm_ranges"]) == 7
    p = make_plan(spl, 0, 0, 0, None, 0, plan_dict=pd)
    from paper_2606_27262_amd import synth
    blocks = []
    for b, dm in enumerate((30.0, 420.0)):
        spec = W.block_spec(pd, p.info["n_in"], [synth.Pulse(t0=1500.0, dm=dm, fwhm=3.0, snr=25.0)])
        blocks.append(synth.make_block(spec, 40 + b, b, pd["widths"])[:, :p.info["n_in"]])
    g = gpu_run(spl, [p, p], blocks, mode=mode)
    ref, rc = oracle_run([p, p], blocks)
    compare(g, ref, rc)
    for b, dm in enumerate((30.0, 420.0)):
        cb = g["cands"][g["cands"]["beam"] == b]
        best = cb[np.argmax(cb["snr"])]
        assert abs(float(best["dm"]) - dm) < 0.05 * dm and abs(int(best["t_sample"]) - 1500) <= 8


@pytest.mark.parametrize("mode", [0, 1])
def test_c2_full_size(spl, mode):
    """4096 channels, 2048 trials, 16384 samples, 20 pulses, 2% RFI, plain and graph
    modes: the whole DM transform, the moments and the candidate list equal the oracle's
    own search of the block, bit for bit."""
    pd = W.plan_c2()
    p = make_plan(spl, 0, 0, 0, None, 0, plan_dict=pd)
    i = p.info
    _, x = W.c2_like_block(pd, i["n_in"], seed=2, beam=0, n_pulses=20)
    x = x[:, :i["n_in"]]
    say("c2 block generated", x.shape)
    g = gpu_run(spl, [p], [x], mode=mode, cand_cap=1 << 18)
    ref, rc = oracle_run([p], [x])
    say("c2 hits", ref[0]["hits"]["d"].size, "candidates", rc.size)
    assert np.array_equal(g["X"][0][0], x[:, :i["n_dd"]].astype(np.int64).sum(0))
    compare(g, ref, rc)


@pytest.mark.parametrize("tiles", ["default", "one-buffer"])
def test_c4_mixed_beams_full_size(spl, tiles):
    """The 32-beam workload's two plans at full size in one persistent, graph-captured
    batch: a 2048-channel 300-500 MHz beam (0.65536 ms, 32768 samples, 1024 trials to
    DM 1000, delays up to 44,946 samples) and a 4096-channel beam with 3072 trials to DM
    3000, each with ten pulses, RFI channels and zero-DM bursts.  Per beam the whole DM
    transform, the moments and the candidate list equal the oracle's own search, bit for
    bit.  Default tiles, and 16-wavefront tiles with one LDS buffer (2 trials with
    16-channel chunks; 4 trials with 32-channel chunks); the 32-beam batch below runs the
    two-buffer tiles the autotuner picks."""
    pds = [W.plan_band3_c4(), W.plan_band4_c4()]
    plans = [make_plan(spl, 0, 0, 0, None, 0, plan_dict=pd) for pd in pds]
    batch = spl.Batch(plans, mode=1)
    if tiles == "one-buffer":
        batch.set_tiles(0, 2, 2, 16, waves=16, buffers=1)
        batch.set_tiles(1, 4, 2, 32, waves=16, buffers=1)
        say("tiles", batch.tiles(0), batch.tiles(1))
    blocks = []
    for b, (pd, p) in enumerate(zip(pds, plans)):
        _, x = W.c2_like_block(pd, p.info["n_in"], seed=4, beam=b, n_pulses=10,
                               dm_max_pulse=0.9 * W.dm_max(pd), zero_dm_rate=0.2)
        blocks.append(x[:, :p.info["n_in"]])
        say(f"c4 beam {b} block generated", blocks[-1].shape)
    g = gpu_run(spl, plans, blocks, cand_cap=1 << 20, batch=batch)
    ref, rc = oracle_run(plans, blocks)
    for b, r in enumerate(ref):
        say(f"c4 beam {b}: hits {r['hits']['d'].size}, candidates {r['cands'].size}")
    compare(g, ref, rc)


C3_BEAMS = 24
C3_GROUP = 4
C3_TILES = (4, 2, 16, 16, 2)    # trials per wavefront, time groups, channel chunk, wavefronts, LDS buffers


@pytest.fixture(scope="module")
def c3_batch(spl):
    """The 24-beam workload exactly as the benchmark searches it: 24 blocks of the
    4096-channel plan (seed 3, ten pulses and 2% RFI channels per beam), one persistent
    launch captured in a hipGraph, with the tiles the autotuner picks for this plan."""
    pd = W.plan_c2()
    p = make_plan(spl, 0, 0, 0, None, 0, plan_dict=pd)
    assert_library_tables(p)
    n_in = p.info["n_in"]
    blocks, dev = [], []
    for b in range(C3_BEAMS):
        _, x = W.c2_like_block(pd, n_in, 3, b, 10)
        blocks.append(np.ascontiguousarray(x[:, :n_in]))
        dev.append(spl.upload_block(blocks[-1]))
        if b % 8 == 7:
            say(f"c3 blocks generated: {b + 1}")
    batch = spl.Batch([p] * C3_BEAMS, mode=spl.MODE_PERSISTENT_GRAPH)
    dw, j, cc, nw, nbuf = C3_TILES
    for b in range(C3_BEAMS):
        batch.set_tiles(b, dw, j, cc, waves=nw, buffers=nbuf)
    cands = spl.new_candidates(1 << 20)
    cands, stats = batch.run(dev, cands)
    torch.cuda.synchronize()
    st = spl.stats_dict(stats)
    say("c3 batch searched:", st)
    assert st["hit_overflow"] == 0 and st["cand_overflow"] == 0
    return {"plan": p, "batch": batch, "blocks": blocks, "dev": dev, "cands_dev": cands,
            "cands": spl.candidates_to_numpy(cands, stats), "stats": st}


@pytest.mark.parametrize("group", range(C3_BEAMS // C3_GROUP))
def test_c3_batch_full_size(spl, c3_batch, group):
    """Beams 4g .. 4g+3 of the 24-beam persistent graph batch: the whole DM transform, the
    moments and the candidate list of every beam equal the oracle's own search of its
    block, bit for bit; then both snippet planes of a sample of each beam's candidates
    (the first, the last, the strongest and every 64th) equal the oracle's."""
    p, batch = c3_batch["plan"], c3_batch["batch"]
    i = p.info
    o = oracle_plan(p)
    for b in range(group * C3_GROUP, (group + 1) * C3_GROUP):
        x = c3_batch["blocks"][b]
        r = oracle_search(p, x, beam=b)
        X = batch.dm_transform(b)[:, :i["n_dd"]].cpu().numpy().astype(np.int64)
        assert np.array_equal(X, r["X"]), f"X differs (beam {b})"
        del X
        s1, s2 = batch.moments(b)
        assert np.array_equal(s1.cpu().numpy(), r["S1"]) and np.array_equal(s2.cpu().numpy(), r["S2"]), b
        got = c3_batch["cands"][c3_batch["cands"]["beam"] == b]
        say(f"c3 beam {b}: hits {r['hits']['d'].size}, candidates {got.size} / {r['cands'].size}")
        assert np.array_equal(got, r["cands"]), f"candidates differ (beam {b})"
        pick = sorted(set([0, got.size - 1, int(np.argmax(got["snr"]))] + list(range(0, got.size, 64))))
        recs = np.ascontiguousarray(got[pick])
        snip = spl.snippets(batch, torch.from_numpy(recs.view(np.int32).reshape(-1, 8).copy()).cuda())
        torch.cuda.synchronize()
        gs = snip.cpu().numpy().view(np.uint16)
        for k, c in enumerate(recs):
            want = oracle.snippets(x, o["D"], r["X"], o["n_out"], o["L"], int(c["dm_index"]), int(c["t_sample"]))
            assert np.array_equal(gs[k], want), (b, k, c)
        say(f"  snippets of {len(pick)} candidates bit-exact")


C4_BEAMS = 32
C4_GROUP = 4


@pytest.fixture(scope="module")
def c4_batch(spl):
    """The 32-beam uneven workload as the benchmark's uneven leg searches it: beams
    alternating the 2048-channel 300-500 MHz plan (even) and the 4096-channel 550-750 MHz
    plan with 3072 trials (odd), blocks made on the GPU with the workload's recipe (seed
    4, ten pulses, 2% RFI channels, zero-DM bursts), one persistent launch per band in one
    hipGraph with the tiles the autotuner picks for these plans."""
    pds = W.batch_c4_plans()
    uniq = {}
    plans = []
    for pd in pds:
        key = repr(sorted(pd.items()))
        if key not in uniq:
            uniq[key] = make_plan(spl, 0, 0, 0, None, 0, plan_dict=pd)
            assert_library_tables(uniq[key])
        plans.append(uniq[key])
    dev = []
    for b, (pd, p) in enumerate(zip(pds, plans)):
        _, x = W.c2_like_block_torch(pd, p.info["n_in"], 4, b, 10, dm_max_pulse=0.9 * W.dm_max(pd), zero_dm_rate=0.2)
        dev.append(x)
    batch = spl.Batch(plans, mode=spl.MODE_PERSISTENT_GRAPH, hit_capacity=1 << 28)
    batch.set_tiles(0, 2, 2, 8, waves=16, buffers=2)
    batch.set_tiles(1, 4, 2, 16, waves=16, buffers=2)
    cands = spl.new_candidates(1 << 22)
    cands, stats = batch.run(dev, cands)
    torch.cuda.synchronize()
    st = spl.stats_dict(stats)
    say("c4 batch searched:", st, batch.tiles(0), batch.tiles(1))
    assert st["hit_overflow"] == 0 and st["cand_overflow"] == 0
    return {"plans": plans, "batch": batch, "dev": dev, "cands": spl.candidates_to_numpy(cands, stats), "stats": st}


def _host_block(c4, b):
    p = c4["plans"][b]
    return c4["dev"][b][:, :p.info["n_in"]].cpu().numpy()


@pytest.mark.parametrize("group", range(C4_BEAMS // C4_GROUP))
def test_c4_batch_full_size(spl, c4_batch, group):
    """Beams 4g .. 4g+3 of the 32-beam uneven persistent graph batch (two of each band):
    the whole DM transform, the moments and the candidate list of every beam equal the
    oracle's own search of its block, bit for bit."""
    batch = c4_batch["batch"]
    assert len(c4_batch["plans"]) == C4_BEAMS
    for beam in range(group * C4_GROUP, (group + 1) * C4_GROUP):
        p = c4_batch["plans"][beam]
        x = _host_block(c4_batch, beam)
        r = oracle_search(p, x, beam=beam)
        X = batch.dm_transform(beam)[:, :p.info["n_dd"]].cpu().numpy().astype(np.int64)
        assert np.array_equal(X, r["X"]), f"X differs (beam {beam})"
        del X
        s1, s2 = batch.moments(beam)
        assert np.array_equal(s1.cpu().numpy(), r["S1"]) and np.array_equal(s2.cpu().numpy(), r["S2"]), beam
        got = c4_batch["cands"][c4_batch["cands"]["beam"] == beam]
        say(f"c4 beam {beam} ({p.info['nchans']} ch): hits {r['hits']['d'].size}, "
            f"candidates {got.size} / {r['cands'].size}")
        assert np.array_equal(got, r["cands"]), f"candidates differ (beam {beam})"


@pytest.mark.parametrize("band", ["300-500", "300-500-fine", "550-750"])
@pytest.mark.parametrize("nch", [512, 37])
def test_tile_shapes_give_identical_results(spl, nch, band):
    """Every compiled tile shape, staging depth and LDS buffer count the plan admits gives
    the oracle's results (37 channels: odd chunks, padded with the zero row; with two
    buffers and 4-channel chunks, ten chunks alternate between the buffers).  The 300-500 MHz plan
    (3 pc cm^-3 steps, ~67 samples of extra delay per trial at the lowest channel)
    admits only 16-trial tiles; with the 2048-channel band's sampling and trial step
    (~44 samples per trial) 32-trial tiles stage rows of 1-2 KB (two 16-byte vectors
    per lane); the 550-750 MHz plan with the 4096-channel band's trial step (~4.7
    samples per trial) admits every shape, up to the 64-trial tiles the autotuner picks
    for that band."""
    if band == "300-500":
        pd = W.make_plan(nch, 300.0, 500.0, 1.31072e-3, 3000, 0.0, 300.0, 100, W.W64)
    elif band == "300-500-fine":
        pd = W.make_plan(nch, 300.0, 500.0, 0.65536e-3, 3000, 0.0, 62.5, 64, W.W64)
    else:
        pd = W.make_plan(nch, 550.0, 750.0, 1.31072e-3, 3000, 0.0, 125.0, 128, W.W64)
    p = make_plan(spl, 0, 0, 0, None, 0, plan_dict=pd)
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, size=(nch, p.info["n_in"]), dtype=np.uint8)
    ref, rc = oracle_run([p], [x])
    batch = spl.Batch([p])
    shapes = ((2, 2, 8), (2, 4, 8), (4, 1, 4), (4, 2, 4), (4, 4, 4), (4, 1, 8), (4, 2, 8), (8, 1, 4),
              (8, 2, 4), (8, 1, 8), (16, 1, 4), (4, 1, 16), (4, 2, 16), (2, 2, 16))
    ran = set()
    for dw, j, nw in shapes:
        for nbuf in ((1, 2) if nw == 16 else (1,)):
            for cc in (0, 1, 4, 16, 32):
                try:
                    batch.set_tiles(0, dw, j, cc, waves=nw, buffers=nbuf)
                except spl.SplError:
                    continue
                say("tiles", dw, j, cc, nbuf, batch.tiles(0))
                g = gpu_run(spl, [p], [x], batch=batch)
                compare(g, ref, rc)
                ran.add((dw, j, nw, nbuf))
    say("shapes checked", sorted(ran))
    if band == "550-750":
        assert {(4, 2, 8, 1), (4, 2, 16, 1), (4, 1, 16, 1), (8, 1, 8, 1), (2, 2, 16, 1),
                (4, 2, 16, 2), (4, 1, 16, 2), (2, 2, 16, 2)} <= ran, ran
    elif band == "300-500-fine":
        assert {(4, 2, 8, 1), (2, 2, 16, 1), (2, 2, 16, 2)} <= ran, ran
    else:
        assert ran


def test_graph_replays_match_eager(spl):
    """Graph mode replayed on new block contents (same buffers) with eager runs in
    between; every replay equals the plain mode's result."""
    plans = [make_plan(spl, 0, 0, 0, None, 0, plan_dict=W.plan_c1()) for _ in range(3)]
    n_in = plans[0].info["n_in"]
    gb = spl.Batch(plans, mode=spl.MODE_PERSISTENT_GRAPH)
    eb = spl.Batch(plans, mode=spl.MODE_PLAIN_PER_BEAM)
    bufs = [torch.zeros((256, (n_in + 255) // 256 * 256), dtype=torch.uint8, device="cuda") for _ in range(3)]
    cg, ce = spl.new_candidates(1 << 14), spl.new_candidates(1 << 14)
    sg = torch.zeros(spl.STATS_WORDS, dtype=torch.int64, device="cuda")
    se = torch.zeros(spl.STATS_WORDS, dtype=torch.int64, device="cuda")
    for rep in range(4):
        for b in range(3):
            _, x = W.c1_block(n_in, seed=100 + 10 * rep + b, beam=b)
            bufs[b].copy_(torch.from_numpy(x[:, :bufs[b].shape[1]]).cuda())
        gb.run(bufs, cg, sg)
        eb.run(bufs, ce, se)
        torch.cuda.synchronize()
        a = spl.candidates_to_numpy(cg, sg)
        e = spl.candidates_to_numpy(ce, se)
        say("replay", rep, a.size)
        assert a.size > 0 and np.array_equal(a, e)
        assert spl.stats_dict(sg) == spl.stats_dict(se)


def test_capacity_flags(spl):
    p = make_plan(spl, 0, 0, 0, None, 0, plan_dict=W.plan_c1())
    _, x = W.c1_block(p.info["n_in"], seed=1)
    x = x[:, :p.info["n_in"]]
    ref, rc = oracle_run([p], [x])
    assert rc.size > 3
    g = gpu_run(spl, [p], [x], cand_cap=3)
    assert g["stats"]["cand_overflow"] == 1 and g["stats"]["n_candidates"] == rc.size
    assert np.array_equal(g["cands"], rc[:3])
    nh = ref[0]["hits"]["d"].size
    g2 = gpu_run(spl, [p], [x], hit_capacity=max(1, nh // 2))
    assert g2["stats"]["hit_overflow"] == 1 and g2["stats"]["n_hits"] == nh


def test_degenerate_shapes(spl):
    rng = np.random.default_rng(8)
    cases = [(1, 1, 1, (1,)), (1, 3, 5, (1, 2)), (3, 1, 7, (1, 7)), (64, 2, 1025, (1, 4)), (257, 5, 300, (1,))]
    for nch, ndm, n_out, widths in cases:
        D = _random_monotone_delays(rng, ndm, nch, 50)
        p = make_plan(spl, nch, ndm, n_out, widths, 1.0, delays=D, stencils=())
        x = rng.integers(0, 256, size=(nch, p.info["n_in"]), dtype=np.uint8)
        g = gpu_run(spl, [p], [x])
        ref, rc = oracle_run([p], [x])
        compare(g, ref, rc)


def test_autotune_keeps_results_and_caches(spl, tmp_path):
    """The autotuner times every compiled shape, verifies identical DM transforms,
    and caches its choice; the tuned batch still matches the oracle."""
    pd = W.make_plan(1024, 550.0, 750.0, 1.31072e-3, 4096, 0.0, 1000.0, 256, W.W256)
    p = make_plan(spl, 0, 0, 0, None, 0, plan_dict=pd)
    rng = np.random.default_rng(21)
    x = rng.integers(0, 256, size=(1024, p.info["n_in"]), dtype=np.uint8)
    ref, rc = oracle_run([p], [x])
    batch = spl.Batch([p, p], mode=spl.MODE_PERSISTENT_GRAPH)
    tb = [spl.upload_block(x), spl.upload_block(x)]
    cache = tmp_path / "tiles.txt"
    tiles = batch.autotune(tb, cache_path=str(cache))
    say("tuned", tiles)
    assert cache.exists() and len(cache.read_text().splitlines()) == 1
    g = gpu_run(spl, [p, p], [x, x], batch=batch)
    for b in range(2):
        assert np.array_equal(g["X"][b], ref[0]["X"])
    rc2 = np.concatenate([rc, rc.copy()])
    rc2["beam"][rc.size:] = 1
    assert np.array_equal(g["cands"], rc2)
    # a second batch reuses the cached choice
    b2 = spl.Batch([p])
    assert b2.autotune([tb[0]], cache_path=str(cache))[0] == tiles[0]
    # the cache line holds trials/wave, time groups, waves, LDS buffers, channel chunk, ms
    sig, *fields = cache.read_text().split()
    t = tiles[0]
    assert [int(v) for v in fields[:5]] == [t["dm_per_wave"], t["time_groups"], t["waves"], t["buffers"],
                                            t["chan_chunk"]]
    # a line of six fields (no buffer count) is dropped and the plan tuned again: the
    # batch's tiles then come from this tuning (timing decides between close shapes), and
    # the file holds one seven-field line that names them
    old = tmp_path / "old.txt"
    old.write_text(f"{sig} 8 1 8 16 1.0\n")
    b3 = spl.Batch([p])
    t3 = b3.autotune([tb[0]], cache_path=str(old))[0]
    lines = old.read_text().splitlines()
    assert len(lines) == 1, lines
    f3 = lines[0].split()
    assert len(f3) == 7 and f3[0] == sig, lines
    assert [int(v) for v in f3[1:6]] == [t3["dm_per_wave"], t3["time_groups"], t3["waves"], t3["buffers"],
                                         t3["chan_chunk"]]


def test_graph_batch_follows_new_block_pointers(spl):
    """A graph-mode batch given other block tensors on each run (new device pointers, as
    a caller that allocates blocks per run does): every run equals the plain mode's on
    the same blocks."""
    plans = [make_plan(spl, 0, 0, 0, None, 0, plan_dict=W.plan_c1()) for _ in range(2)]
    n_in = plans[0].info["n_in"]
    gb = spl.Batch(plans, mode=spl.MODE_PERSISTENT_GRAPH)
    eb = spl.Batch(plans, mode=spl.MODE_PLAIN_PER_BEAM)
    cg, ce = spl.new_candidates(1 << 14), spl.new_candidates(1 << 14)
    sg = torch.zeros(spl.STATS_WORDS, dtype=torch.int64, device="cuda")
    se = torch.zeros(spl.STATS_WORDS, dtype=torch.int64, device="cuda")
    keep = []
    for rep in range(4):
        bufs = []
        for b in range(2):
            _, x = W.c1_block(n_in, seed=300 + 10 * rep + b, beam=b)
            bufs.append(spl.upload_block(x[:, :n_in]))
        keep.append(bufs)   # earlier tensors stay allocated: every run sees new addresses
        gb.run(bufs, cg, sg)
        eb.run(bufs, ce, se)
        torch.cuda.synchronize()
        a = spl.candidates_to_numpy(cg, sg)
        e = spl.candidates_to_numpy(ce, se)
        say("new pointers", rep, a.size)
        assert a.size > 0 and np.array_equal(a, e)
