"""Benchmark of the single-pulse search hot path on one MI355X.

A step is one pass of the whole path (dedispersion, normaliser and thresholds,
boxcar search, peak filters, candidate compaction) over one block of every beam
of the workload, with the blocks already resident in HBM.  Prints one JSON line.

Workloads (synthetic stand-ins for uGMRT beam data, seeded):
  c3  24 beams of the c2 shape (one GPU's share of 2000 beams over 90 GPUs), persistent
      launch captured in a hipGraph, 10 injected pulses per beam       (default)
  c2  1 beam, 4096 ch 550-750 MHz, 16384 samples at 1.31072 ms, 2048 DM trials 0-2000,
      widths 1..256, 20 injected pulses, 2% RFI channels
  c4  32 beams alternating 2048 ch 300-500 MHz / 0.65536 ms / 32768 samples / 1024
      trials 0-1000 and 4096 ch 550-750 MHz / 1.31072 ms / 16384 samples / 3072 trials
      0-3000, zero-DM RFI bursts, persistent launch in a hipGraph
  c1  1 beam, 256 ch 300-500 MHz, 8192 samples, 128 trials 0-500, widths 1..64
  c2s, c3s  as c2 / c3 searched to DM 2000 with smearing-limited sub-ranges (5157 trials
      in steps 0.25, 0.5 and 1: spl_plan_smearing_ranges, 10% S/N loss half a step off)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_ADDS = 256 * 64 * 2.4e9      # int32 adds/s: 256 CUs x 64 lanes x 2.4 GHz, one add per lane per clock


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name, spl, W, keep_host=False):
    import numpy as np
    host = []
    if name == "c1":
        pds = [W.plan_c1()]
    elif name == "c2":
        pds = [W.plan_c2()]
    elif name == "c3":
        pds = W.batch_c3_plans()
    elif name == "c4":
        pds = W.batch_c4_plans()
    elif name in ("c2s", "c3s"):
        # the 4096-channel band searched to DM 2000 with smearing-limited sub-ranges
        pd = W.plan_c2()
        pd["dm_ranges"] = spl.smearing_ranges(pd["nchans"], pd["fch1"], pd["foff"], pd["tsamp"], 0.0, 2000.0, 0.1)
        pds = [pd] if name == "c2s" else [dict(pd) for _ in range(24)]
    else:
        raise SystemExit(f"unknown workload {name}")
    plans, cache = [], {}
    for pd in pds:
        key = json.dumps(pd, sort_keys=True, default=str)
        if key not in cache:
            cache[key] = spl.Plan.from_dict(pd)
        plans.append(cache[key])
    blocks, pulses = [], []
    seed = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c2s": 2, "c3s": 3}[name]
    for b, (pd, p) in enumerate(zip(pds, plans)):
        n_in = p.info["n_in"]
        if name == "c1":
            spec, x = W.c1_block(n_in, seed=seed)
        elif name in ("c2", "c2s"):
            spec, x = W.c2_like_block(pd, n_in, seed, b, 20)
        elif name in ("c3", "c3s"):
            spec, x = W.c2_like_block(pd, n_in, seed, b, 10)
        else:
            spec, x = W.c2_like_block(pd, n_in, seed, b, 10, dm_max_pulse=0.9 * W.dm_max(pd), zero_dm_rate=0.2)
        blocks.append(spl.upload_block(x[:, :n_in]))
        pulses.append(list(spec.pulses))
        if keep_host:
            import torch
            h = torch.empty(tuple(blocks[-1].shape), dtype=torch.uint8, pin_memory=True)
            h[:, :n_in] = torch.from_numpy(np.ascontiguousarray(x[:, :n_in]))
            host.append(h)
        del x
        if b % 8 == 7:
            log(f"generated {b + 1}/{len(pds)} blocks")
    return pds, plans, blocks, pulses, host


def end_to_end_leg(spl, W, pds, args, n_blocks=8, warmup=2, seed=33):
    """Sustained search of continuous beam streams (paper_2606_27262_amd.streaming): each
    beam's stream repeats a synthetic series of two blocks' owned samples (2 n_out, ten
    pulses per block, 2 % RFI channels; no pulse crosses the period end), so the stream
    alternates between two block contents.  The first block is uploaded whole; every
    later block receives the previous block's overlap tail on the device and only its
    n_out new samples from pinned host memory, overlapped with the search of the current
    block (one contiguous pinned copy per beam into a staging buffer; spl_stream_assemble
    then writes the block from the previous block's tail and the staged samples on the
    search stream), while the candidate stage of the previous block runs on the host.
    ms_per_block is the steady-state period on the search stream (first measured
    block's start to the last block's searched and copied records); the host wall time,
    which also holds the last block's unoverlapped candidate stage, is reported beside
    it.  Recall counts each block's own bursts; a candidate matching a burst of the
    neighbouring blocks is not a false alarm."""
    import tempfile

    import numpy as np
    import torch

    from paper_2606_27262_amd import ranking, streaming
    block_s = max(pd["n_out"] * pd["tsamp"] for pd in pds)
    ss = streaming.StreamingSearch(spl, pds,
                                   thresholds=ranking.beam_thresholds(pds, ranking.load_operating_point(
                                       args.operating_point)))
    ss.attach(tile_cache=None if args.no_autotune else
              (args.tile_cache or os.path.join(tempfile.gettempdir(), "spotlight_tiles.txt")))
    first, chunks, truth = [], [[], []], [[], []]
    for b, (pd, p) in enumerate(zip(pds, ss.plans)):
        n_in, n_out = p.info["n_in"], p.info["n_out"]
        series, per_block = W.stream_series(pd, 0, n_in, seed, b, 10, period=2, device="cuda")
        idx0 = torch.arange(n_in, device="cuda") % series.shape[1]
        h = torch.zeros(tuple(ss.dev[0][b].shape), dtype=torch.uint8, pin_memory=True)
        h[:, :n_in].copy_(series[:, idx0])
        first.append(h)
        for j, k in enumerate((1, 2)):
            idx = (k * n_out + (n_in - n_out) + torch.arange(n_out, device="cuda")) % series.shape[1]
            c = torch.empty((series.shape[0], n_out), dtype=torch.uint8, pin_memory=True)
            c.copy_(series[:, idx])
            chunks[j].append(c)
        truth[0].append(per_block[0])
        truth[1].append(per_block[1])
        del series
    torch.cuda.synchronize()

    def shifted(ps, dt):
        return [type(p)(t0=p.t0 + dt, dm=p.dm, fwhm=p.fwhm, snr=p.snr) for p in ps]

    n_outs = [p.info["n_out"] for p in ss.plans]
    context = [[shifted(truth[1 - q][b], -n_outs[b]) + shifted(truth[1 - q][b], n_outs[b]) for b in range(len(pds))]
               for q in (0, 1)]

    def on_block(k, final, ncand, recs):
        q = k % 2
        return ranking.recall_and_false_alarms(final, truth[q], pds, context_by_beam=context[q])

    out = {"blocks": n_blocks, "warmup": warmup, "stream": "period of two blocks per beam (GPU-made series)",
           "h2d_bytes_first_block": int(sum(h.numel() for h in first)),
           "h2d_GBps_alone": ss.copy_rate(chunks[0]) / 1e9,
           "assemble_ms_alone": ss.assemble_time() * 1e3}
    legs = [("plain", None)]
    if not args.no_ranker and all(pd["nchans"] % 64 == 0 for pd in pds):
        r = spl.Ranker(max_batch=256)
        r.set_weights(np.load(args.ranker_weights) if os.path.exists(args.ranker_weights)
                      else ranking.initial_weights(0))
        legs.append(("ranker", r))
    for name, ranker in legs:
        ss.ranker = ranker
        tm = {}
        wall, res = ss.run(first, chunks, n_blocks, warmup, timing=tm, on_block=on_block)
        steady = tm["steady_s"]
        out["h2d_bytes_per_block"] = tm["h2d_bytes_per_block"]
        out[name] = {"ms_per_block": steady * 1e3, "real_time_beams_per_gpu": len(pds) * block_s / steady,
                     "wall_ms_per_block_with_drain": wall * 1e3, "drain_ms": tm["drain_s"] * 1e3,
                     "recall": float(np.mean([q["recall"] for q in res])),
                     "false_alarms_per_beam_block": float(np.mean([q["false_alarms"] for q in res])) / len(pds),
                     "side_lobes_per_beam_block": float(np.mean([q["side_lobes"] for q in res])) / len(pds)}
    out["h2d_bytes_whole_blocks"] = int(sum(p.info["nchans"] * p.info["n_in"] for p in ss.plans))
    del ss
    return out


def cpu_baseline(pd, plan, W, target_s=12.0):
    """The oracle on the host cores on a bounded sample: the first k DM trials of the
    workload's first block over all its samples (dedispersion + boxcar search + peak
    filter), k chosen for about target_s seconds of CPU work.  When the block has a
    channel count the snippets accept, also the oracle's snippets of a few of its
    candidates and its float64 CNN forward pass on a few snippets."""
    import numpy as np

    import oracle
    # the oracle's own DM trials and delay table, from the plan's parameters
    dms = oracle.dm_trials(pd["dm_ranges"])
    D, _ = oracle.delay_table(pd["nchans"], pd["fch1"], pd["foff"], pd["tsamp"], dms)
    i = dict(oracle.sizes(D, pd["n_out"], pd["widths"]), ndm=int(dms.size), nchans=int(pd["nchans"]),
             n_out=int(pd["n_out"]), norm_window=int(pd.get("norm_window") or pd["n_out"]))
    _, x = W.c2_like_block(pd, i["n_in"], 99, 0, 4) if i["nchans"] > 256 else W.c1_block(i["n_in"], seed=99)
    x = np.ascontiguousarray(x[:, :i["n_in"]])
    last = {}

    def run(k):
        t = time.perf_counter()
        last["r"] = oracle.search_beam(x, D[:k], dms[:k], i["n_out"], i["norm_window"], pd["widths"],
                                       pd["threshold"])
        return time.perf_counter() - t

    k = min(i["ndm"], 16)
    t = run(k)
    k2 = int(min(i["ndm"], max(k, k * target_s / max(t, 1e-3))))
    t2 = run(k2)
    r = last["r"]
    x0 = x
    blocks = 1
    if k2 == i["ndm"] and i["nchans"] > 256:
        # the whole block took less than target_s: search further blocks of the workload
        # (other beams, same plan) until about target_s of CPU work is timed
        while t2 < target_s and blocks < 8:
            _, x = W.c2_like_block(pd, i["n_in"], 99, blocks, 4)
            x = np.ascontiguousarray(x[:, :i["n_in"]])
            t2 += run(k2)
            blocks += 1
        x = x0
    out = {"value": blocks * k2 * i["n_out"] / t2, "unit": "DM-trial·samples/s", "cores": oracle.num_threads(),
           "kind": "oracle", "seconds": round(t2, 3),
           "sample": (f"first {k2} of {i['ndm']} DM trials x {i['n_out']} samples of one "
                      f"{i['nchans']}-channel block" if blocks == 1 else
                      f"all {k2} DM trials x {i['n_out']} samples of {blocks} {i['nchans']}-channel blocks "
                      f"(beams of the workload)") + ": dedispersion + boxcar search + peak filters"}
    # the same oracle on one core: the first k trials of the first block, about 8 s
    n_all = oracle.num_threads()
    oracle.set_threads(1)
    try:
        k1 = max(1, int(k2 * 8.0 / max(t2 / blocks, 1e-3) / n_all))
        k1 = min(k1, i["ndm"])
        t1 = run(k1)
        if t1 < 2.0 and k1 < i["ndm"]:
            k1 = min(i["ndm"], int(k1 * 8.0 / max(t1, 1e-3)))
            t1 = run(k1)
    finally:
        oracle.set_threads(n_all)
    out["one_core"] = {"value": k1 * i["n_out"] / t1, "cores": 1, "seconds": round(t1, 3),
                       "sample": f"first {k1} of {i['ndm']} DM trials x {i['n_out']} samples of one "
                                 f"{i['nchans']}-channel block: dedispersion + boxcar search + peak filters"}
    if i["nchans"] % 64 == 0 and r["cands"].size and k2 == i["ndm"]:
        from oracle import cnn
        cs = r["cands"][:8]
        t = time.perf_counter()
        snips = [oracle.snippets(x, D, r["X"], i["n_out"], i["norm_window"], int(c["dm_index"]), int(c["t_sample"]))
                 for c in cs]
        ts = time.perf_counter() - t
        p = cnn.init_params(0)
        xin = oracle.bf16_bits_to_f32(np.stack(snips[:2])).astype(np.float64)
        t = time.perf_counter()
        cnn.forward(p, xin)
        tf = time.perf_counter() - t
        out["ranker"] = {"snippets_per_s": len(cs) / ts, "cnn_forward_candidates_per_s": xin.shape[0] / tf,
                         "sample": f"oracle snippets of {len(cs)} candidates of that block; float64 CNN "
                                   f"forward of {xin.shape[0]} snippets (numpy, single process)"}
    return out


def dedisp_source_hash():
    """SHA-256 over what the dedispersion kernel is compiled from, in a fixed order: its
    section of kernels.hip (from the dedispersion banner to the next kernel's), the
    staging-depth constant of kernels.h, and the headers that define its descriptors
    and device helpers.  Edits to the other kernels leave it unchanged."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2606_27262_amd", "csrc")
    src = open(os.path.join(csrc, "kernels.hip")).read()
    i = src.index("// ------------------------------------------------------------- dedispersion")
    j = src.index("// ------------------------------------------------------- moments + thresholds")
    h = hashlib.sha256()
    h.update(src[i:j].encode())
    h.update("\n".join(re.findall(r"^constexpr int dedisp_stage_rows.*$", open(os.path.join(csrc, "kernels.h")).read(),
                                   re.M)).encode())
    for f in ("spl_internal.h", "spl_device.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def counter_traffic(workload, tiles):
    """HBM bytes per dedispersion launch from the committed rocprofv3 counter summary of
    this workload (FETCH_SIZE and WRITE_SIZE, scaled by a 1 GiB copy), or None when
    there is none, or the kernel source or the tile shape differ from those the counters
    were taken with."""
    import re
    path = os.path.join(ROOT, "profiles", f"dedisp_{workload}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"^counters: workload=(\S+) kernel=k_dedisp tiles=(\d+),(\d+),(\d+),(\d+),(\d+) grid=\d+ "
                  r"fetch_bytes=(\d+) write_bytes=(\d+) dedisp_src_sha256=([0-9a-f]{64})$", open(path).read(), re.M)
    if not m or m.group(1) != workload or dedisp_source_hash() != m.group(9):
        return None
    shape = tuple(int(m.group(i)) for i in range(2, 7))   # trials/wave, groups, waves, chan_chunk, buffers
    if any((t["dm_per_wave"], t["time_groups"], t["waves"], t["chan_chunk"], t.get("buffers", 1)) != shape
           for t in tiles):
        return None
    return {"fetch_bytes": int(m.group(7)), "write_bytes": int(m.group(8))}


def corner_turn_leg(spl, plan, reps=12, nbuf=4):
    """Corner turn of blocks of the workload's first plan (time-major spectra in,
    channel-major rows out): HIP-event time per launch and the achieved bytes/s, with
    2 bytes per sample (one read, one write) as the algorithmic traffic.  The launches
    rotate over nbuf block pairs (0.86 GB for 4096 x 26305 samples), more than the
    256 MB last-level cache, so the figure is an HBM rate."""
    import torch
    n_t, nch = plan.info["n_in"], plan.info["nchans"]
    src = [torch.randint(0, 256, (n_t, nch), dtype=torch.uint8, device="cuda") for _ in range(nbuf)]
    dst = [torch.empty((nch, (n_t + 255) // 256 * 256), dtype=torch.uint8, device="cuda") for _ in range(nbuf)]
    s = torch.cuda.current_stream()
    for i in range(nbuf):
        spl.corner_turn(src[i], out=dst[i])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for r in range(reps):
        spl.corner_turn(src[r % nbuf], out=dst[r % nbuf])
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbps = 2.0 * n_t * nch / (ms / 1e3) / 1e9
    del src, dst
    return {"samples": n_t * nch, "launch_ms": ms, "achieved_GBps": gbps, "peak_GBps": 8000.0,
            "frac": gbps / 8000.0}


def injector_leg(spl, W, pds, plans, blocks, pulses, ms_step, reps=5):
    """Quantised-domain injection of the workload's bursts (the same pulses its blocks
    carry, each a window of the dispersed template over every channel) into copies of
    the beams' blocks: HIP-event time per block of all beams (one call per beam), with
    10 bytes per injected value (signal, random word, sample read and written) as the
    algorithmic traffic."""
    import numpy as np
    import torch
    from paper_2606_27262_amd import synth
    work = []
    for b, (pd, p) in enumerate(zip(pds, plans)):
        n_in = p.info["n_in"]
        if not pulses[b]:
            continue
        t_start, sig = synth.burst_windows(W.block_spec(pd, n_in, pulses[b]), pulses[b], pd["widths"])
        words = synth.random_words(1000 + b, sig.shape).view(np.int32)
        work.append((blocks[b].clone(), n_in, torch.from_numpy(t_start).cuda(), torch.from_numpy(sig).cuda(),
                     torch.from_numpy(words).cuda()))
    if not work:
        return None
    values = sum(int(s.numel()) for _, _, _, s, _ in work)
    s = torch.cuda.current_stream()

    def one_block():
        for blk, n_in, ts, sg, rw in work:
            spl.inject_quantised(blk, ts, sg, rw, n_t=n_in, stream=s)

    one_block()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        one_block()
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del work
    return {"bursts": sum(len(x) for x in pulses), "values": values, "ms_per_block": ms,
            "values_per_s": values / (ms / 1e3), "algorithmic_GBps": 10.0 * values / (ms / 1e3) / 1e9,
            "frac_of_step": ms / ms_step, "mode": "sample"}


def per_beam_comparison(spl, plans, blocks, args, cands, stats):
    """The same blocks searched beam by beam (plain mode: one launch sequence per beam),
    for the comparison of the batched form with the per-beam pipeline."""
    import torch
    b2 = spl.Batch(plans, mode=spl.MODE_PLAIN_PER_BEAM)
    b2.attach()
    if not args.no_autotune:
        import tempfile
        b2.autotune(blocks, cache_path=args.tile_cache or os.path.join(tempfile.gettempdir(), "spotlight_tiles.txt"))
    steps = max(2, args.steps // 4)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b2.run(blocks, cands, stats, stream=s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        for _ in range(steps):
            b2.run(blocks, cands, stats, stream=s)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    del b2
    return {"ms_per_step": ms, "steps": steps}


def ranker_leg(spl, pds, plans, batch, blocks, pulses, cands, stats, stream, args, ms_step, block_s):
    """Candidate stage on the last run's candidates: the plain optimisation path (host)
    against the ranker path (optimisation with the CNN in place of the density test and
    the S/N cut, the CNN on device),
    recall and false alarms on the injected pulses; then the CNN's own throughput in
    training and inference on batches of 256 snippets."""
    import numpy as np
    import torch

    from paper_2606_27262_amd import ranking

    nb = len(plans)
    with torch.cuda.stream(stream):
        batch.run(blocks, cands, stats, stream=stream)
    torch.cuda.synchronize()
    recs = spl.candidates_to_numpy(cands, stats)
    tsamp = np.array([pd["tsamp"] for pd in pds], np.float64)
    ranker = spl.Ranker(max_batch=256)
    trained = os.path.exists(args.ranker_weights)
    ranker.set_weights(np.load(args.ranker_weights) if trained else ranking.initial_weights(0))
    t0 = time.perf_counter()
    fp = spl.optimise_plain(recs, tsamp, nb)
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()

    def score(r):
        dev = torch.from_numpy(np.ascontiguousarray(r).view(np.int32).reshape(-1, 8).copy()).cuda()
        return ranker.score(spl.snippets(batch, dev)).cpu().numpy()

    op = ranking.load_operating_point(args.operating_point)
    thr = ranking.beam_thresholds(pds, op)
    kept, surv, lg = ranking.ranker_path(spl, recs, tsamp, nb, score, threshold=thr)
    n_scored = surv.size
    t_rank = time.perf_counter() - t0
    snip_leg = None
    if surv.size:
        # the snippet kernel alone on the scored records: bytes it must move per candidate
        # = 64 DM-transform rows x 256 int32 + nch x 256 block bytes read, 64 KiB written
        dev = torch.from_numpy(np.ascontiguousarray(surv).view(np.int32).reshape(-1, 8).copy()).cuda()
        buf = torch.empty((surv.size, 2, 64, 256), dtype=torch.int16, device="cuda")
        spl.snippets(batch, dev, out=buf)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            spl.snippets(batch, dev, out=buf)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        nch = [p.info["nchans"] for p in plans]
        per_cand = [64 * 256 * 4 + nch[int(b)] * 256 + 2 * 64 * 256 * 2 for b in surv["beam"]]
        snip_leg = {"candidates": int(surv.size), "launch_ms": ms, "bytes": int(sum(per_cand)),
                    "achieved_GBps": sum(per_cand) / (ms / 1e3) / 1e9, "peak_GBps": 8000.0}
        # fine-DM plane 0 (64 DMs around each candidate's DM, dedispersed from the block)
        spl.snippets(batch, dev, out=buf, fine_keep=0.1)
        e0.record()
        for _ in range(3):
            spl.snippets(batch, dev, out=buf, fine_keep=0.1)
        e1.record()
        torch.cuda.synchronize()
        ms_f = e0.elapsed_time(e1) / 3
        adds = sum(64 * 256 * nch[int(b)] for b in surv["beam"])
        # block bytes the plane must read: per channel the 256 samples plus the spread of
        # its 64 delays (2 dDM x the channel's delay per unit DM), at most 64 x 256
        touched = 0
        for b in np.unique(surv["beam"]):
            pd = pds[int(b)]
            f = pd["fch1"] + np.arange(pd["nchans"]) * pd["foff"]
            per_dm = 4148.8064239 * (1.0 / f ** 2 - 1.0 / f.max() ** 2) / pd["tsamp"]
            nu, bw = (f.max() + f.min()) / 2e3, pd["nchans"] * abs(pd["foff"])
            w = surv["width"][surv["beam"] == b].astype(np.float64)
            half = (np.sqrt(np.pi) / 2 / 0.1) * (w * pd["tsamp"] * 1e3) * nu ** 3 / (6.91e-3 * bw)
            touched += int(np.minimum(64 * 256, 256 + 2 * half[:, None] * per_dm[None, :]).sum())
        sel_w = surv["width"].astype(np.int64)
        snip_leg["fine_dm"] = {"launch_ms_both_planes": ms_f, "plane0_ms": ms_f - ms, "adds": adds,
                               "Tadds_per_s": adds / ((ms_f - ms) / 1e3) / 1e12 if ms_f > ms else None,
                               "block_bytes_touched": touched,
                               "touched_GBps": touched / ((ms_f - ms) / 1e3) / 1e9 if ms_f > ms else None,
                               "widths_p50_p90_max": [int(np.percentile(sel_w, 50)), int(np.percentile(sel_w, 90)),
                                                      int(sel_w.max())]}
    pr = ranking.recall_and_false_alarms(fp, pulses, pds)
    rr = ranking.recall_and_false_alarms(kept, pulses, pds)
    matched = ranking.at_false_alarms(spl, surv, lg, pulses, pds, pr["false_alarms"], nb)

    # throughput of the network itself
    rng = np.random.default_rng(0)
    n = 256
    x = torch.from_numpy(rng.normal(0, 1, size=(n, 2, 64, 256)).astype(np.float32)).cuda()
    snip = (x.view(torch.int32) >> 16).to(torch.int16)   # truncated BF16 patterns are enough here
    lab = torch.from_numpy((rng.random(n) < 0.5).astype(np.float32)).cuda()
    probe = spl.Ranker(max_batch=n)
    probe.set_weights(ranking.initial_weights(1))
    flop_fwd = 2.0 * (9 * (2 * 32 * 64 * 256 + 32 * 32 * (32 * 128 + 16 * 64 + 8 * 32))) + 2.0 * (2048 * 64 + 64)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    t_inf = timed(lambda: probe.score(snip), 10)
    t_trn = timed(lambda: probe.train_step(snip, lab, 1e-4), 10)
    del probe
    return {
        "weights": "trained" if trained else "untrained (initial weights)",
        "plain_path": {**pr, "host_ms": t_plain * 1e3},
        "ranker_path": {**rr, "scored": int(n_scored), "stage_ms": t_rank * 1e3,
                        "logit_thresholds": sorted(set(float(v) for v in thr))},
        "ranker_path_p05": ranking.recall_and_false_alarms(
            spl.anti_coincidence(surv[lg >= 0.0], tsamp, nb), pulses, pds) if surv.size else None,
        "ranker_at_plain_false_alarms": matched,
        "snippets": snip_leg,
        # the candidate stage after the search of the same block (serial), or overlapped
        # with the search of the next block (the stage runs on the host and the GPU's
        # snippets and CNN take a few ms)
        "real_time_beams_per_gpu": {
            "plain_serial": nb / ((ms_step + t_plain * 1e3) / 1e3 / block_s),
            "plain_overlapped": nb / (max(ms_step, t_plain * 1e3) / 1e3 / block_s),
            "ranker_serial": nb / ((ms_step + t_rank * 1e3) / 1e3 / block_s),
            "ranker_overlapped": nb / (max(ms_step, t_rank * 1e3) / 1e3 / block_s)},
        "cnn": {"batch": n, "flop_forward_per_candidate": flop_fwd,
                "inference_ms": t_inf * 1e3, "inference_candidates_per_s": n / t_inf,
                "inference_tflops": n * flop_fwd / t_inf / 1e12,
                "train_step_ms": t_trn * 1e3, "train_candidates_per_s": n / t_trn,
                "train_tflops": 3 * n * flop_fwd / t_trn / 1e12,
                "mfma_peak_tflops_bf16": 2500.0},
    }


def growth_leg(spl, W, pd, tiles, block_s, sizes=(96, 384, 768), steps=2, seed=77):
    """Real-time beams measured by growing the batch of the 24-beam shape: batches of
    `sizes` beams of the same plan, blocks made on the GPU (the same recipe as the
    workload's: ten pulses and 2 % RFI channels per beam, torch's noise), one persistent
    launch captured in a hipGraph with the tiles the autotuner chose for the plan.  A size
    is skipped when its blocks and workspace do not fit the free device memory."""
    import torch
    plan = spl.Plan.from_dict(pd)
    n_in = plan.info["n_in"]
    rows = []
    for nb in sizes:
        probe = spl.Batch([plan] * nb, mode=spl.MODE_PERSISTENT_GRAPH)
        need = probe.workspace_bytes() + nb * pd["nchans"] * ((n_in + 255) // 256 * 256) + (4 << 30)
        free, _ = torch.cuda.mem_get_info()
        if need > free:
            rows.append({"beams": nb, "skipped": f"needs {need / 2**30:.1f} GiB, {free / 2**30:.1f} GiB free"})
            del probe
            continue
        blocks = [W.c2_like_block_torch(pd, n_in, seed, b, 10)[1] for b in range(nb)]
        probe.set_tiles(0, tiles["dm_per_wave"], tiles["time_groups"], tiles["chan_chunk"], waves=tiles["waves"],
                        buffers=tiles.get("buffers", 1))
        probe.attach()
        cands = spl.new_candidates(1 << 20)
        stats = torch.zeros(spl.STATS_WORDS, dtype=torch.int64, device="cuda")
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            probe.run(blocks, cands, stats, stream=s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(s):
            for _ in range(steps):
                probe.run(blocks, cands, stats, stream=s)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        st = spl.stats_dict(stats)
        rtf = ms / 1e3 / block_s
        rows.append({"beams": nb, "ms_per_step": ms, "ms_per_beam": ms / nb, "real_time_factor": rtf,
                     "dm_trial_samples_per_s": nb * plan.info["ndm"] * plan.info["n_out"] / (ms / 1e3),
                     "hit_overflow": st["hit_overflow"]})
        log(f"growth: {nb} beams {ms:.1f} ms per step (real-time factor {rtf:.4f})")
        del probe, blocks, cands, stats
        torch.cuda.empty_cache()
    done = [r for r in rows if "ms_per_step" in r and r["real_time_factor"] <= 1.0]
    out = {"sizes": rows}
    if done:
        big = max(done, key=lambda r: r["beams"])
        out["largest_measured_beams"] = big["beams"]
        out["real_time_beams_measured_at_least"] = big["beams"]
        out["real_time_beams_extrapolated"] = big["beams"] / big["real_time_factor"]
        out["extrapolation"] = (f"linear from the largest measured batch ({big['beams']} beams, real-time factor "
                                f"{big['real_time_factor']:.4f}); the blocks and workspace of that many beams "
                                f"exceed one GPU's memory, so they would run as successive batches")
    return out


def uneven_leg(spl, W, args, steps=5, warmup=2, seed=4):
    """The 32-beam uneven batch (16 beams of the 2048-channel 300-500 MHz plan, 16 of the
    4096-channel 550-750 MHz plan with 3072 trials), blocks made on the GPU with the
    workload's recipe (ten pulses, 2 % RFI channels, zero-DM bursts; torch's noise), one
    persistent graph launch with autotuned tiles: ms per step, throughput, the
    dedispersion launch against the add peak, and per band the plain path against the
    ranker path on the step's candidates (recall and false alarms of the injected pulses,
    at the ranker's own operating point and at the plain path's false-alarm count)."""
    import tempfile

    import numpy as np
    import torch

    from paper_2606_27262_amd import ranking
    pds = W.batch_c4_plans()
    cache = {}
    plans = []
    for pd in pds:
        key = json.dumps(pd, sort_keys=True, default=str)
        if key not in cache:
            cache[key] = spl.Plan.from_dict(pd)
        plans.append(cache[key])
    blocks, pulses = [], []
    for b, (pd, p) in enumerate(zip(pds, plans)):
        spec, x = W.c2_like_block_torch(pd, p.info["n_in"], seed, b, 10, dm_max_pulse=0.9 * W.dm_max(pd),
                                        zero_dm_rate=0.2)
        blocks.append(x)
        pulses.append(list(spec.pulses))
    # the zero-DM bursts light up every trial near their time: 1.6e8 hits per block
    batch = spl.Batch(plans, mode=spl.MODE_PERSISTENT_GRAPH, hit_capacity=1 << 28)
    batch.attach()
    if not args.no_autotune:
        batch.autotune(blocks, cache_path=args.tile_cache or os.path.join(tempfile.gettempdir(), "spotlight_tiles.txt"))
    cands = spl.new_candidates(1 << 22)
    stats = torch.zeros(spl.STATS_WORDS, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for _ in range(warmup):
            batch.run(blocks, cands, stats, stream=s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        for _ in range(steps):
            batch.run(blocks, cands, stats, stream=s)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    st = spl.stats_dict(stats)
    batch.set_profiling(True)
    with torch.cuda.stream(s):
        for _ in range(steps):
            batch.run(blocks, cands, stats, stream=s)
    torch.cuda.synchronize()
    stages = batch.stage_times(reset=True)
    batch.set_profiling(False)
    dd_ms, dd_n = stages["dedisp"]
    adds = sum(p.info["ndm"] * p.info["nchans"] * p.info["n_out"] for p in plans)
    block_s = max(pd["n_out"] * pd["tsamp"] for pd in pds)
    out = {"workload": "c4", "beams": len(pds), "ms_per_step": ms,
           "value": sum(p.info["ndm"] * p.info["n_out"] for p in plans) / (ms / 1e3),
           "unit": "DM-trial·samples/s", "real_time_factor": ms / 1e3 / block_s,
           "dedisp_ms_per_step": dd_ms / steps, "dedisp_adds_per_s": adds / (dd_ms / steps / 1e3),
           "dedisp_frac_add_peak": adds / (dd_ms / steps / 1e3) / PEAK_ADDS,
           "tiles": {f"{p.info['nchans']}ch": batch.tiles(b) for b, p in ((0, plans[0]), (1, plans[1]))},
           "candidates": st["n_candidates"], "hits": st["n_hits"], "hit_overflow": st["hit_overflow"],
           "cand_overflow": st["cand_overflow"]}
    assert not (st["hit_overflow"] or st["cand_overflow"]), st
    if not args.no_ranker:
        with torch.cuda.stream(s):
            batch.run(blocks, cands, stats, stream=s)
        torch.cuda.synchronize()
        recs = spl.candidates_to_numpy(cands, stats)
        tsamp = np.array([pd["tsamp"] for pd in pds], np.float64)
        ranker = spl.Ranker(max_batch=256)
        ranker.set_weights(np.load(args.ranker_weights) if os.path.exists(args.ranker_weights)
                           else ranking.initial_weights(0))

        def score(r):
            dev = torch.from_numpy(np.ascontiguousarray(r).view(np.int32).reshape(-1, 8).copy()).cuda()
            return ranker.score(spl.snippets(batch, dev)).cpu().numpy()

        fp = spl.optimise_plain(recs, tsamp, len(pds))
        thr = ranking.beam_thresholds(pds, ranking.load_operating_point(args.operating_point))
        fr, scored, lg = ranking.ranker_path(spl, recs, tsamp, len(pds), score, threshold=thr)
        out["ranker"] = per_band_comparison(spl, pds, pulses, fp, fr, scored, lg)
    del batch, blocks
    torch.cuda.empty_cache()
    return out


def per_band_comparison(spl, pds, pulses, fp, fr, scored, lg):
    """Per band (beams sharing channel count and band): recall and false alarms of the
    plain path and the ranker path, and the ranker at the plain path's false-alarm count
    (thresholds on its logits, anti-coincidence among that band's beams)."""
    import numpy as np

    from paper_2606_27262_amd import ranking
    bands = {}
    for b, pd in enumerate(pds):
        bands.setdefault(f"{pd['nchans']}ch/{pd['fch1'] + (pd['nchans'] - 1) * pd['foff']:.0f}-{pd['fch1']:.0f}MHz",
                         []).append(b)
    out = {}
    for name, beams in bands.items():
        remap = np.full(len(pds), -1, np.int64)
        remap[beams] = np.arange(len(beams))

        def sub(c):
            c = c[np.isin(c["beam"], beams)].copy()
            c["beam"] = remap[c["beam"]]
            return c

        ps = [pulses[b] for b in beams]
        pdb = [pds[b] for b in beams]
        p_ = ranking.recall_and_false_alarms(sub(fp), ps, pdb)
        r_ = ranking.recall_and_false_alarms(sub(fr), ps, pdb)
        sel = np.isin(scored["beam"], beams)
        m = ranking.at_false_alarms(spl, sub(scored), lg[sel], ps, pdb, p_["false_alarms"], len(beams))
        nbb = len(beams)
        out[name] = {"beams": nbb,
                     "plain": {**p_, "false_alarms_per_beam_block": p_["false_alarms"] / nbb},
                     "ranker": {**r_, "false_alarms_per_beam_block": r_["false_alarms"] / nbb},
                     "ranker_at_plain_false_alarms": m}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c2s", "c3s"])
    ap.add_argument("--mode", default="auto", choices=["auto", "plain", "graph"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default dedispersion tiles")
    ap.add_argument("--tile-cache", default=None, help="autotuner cache file (default: a file in $TMPDIR)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this size first (calibrates HBM byte counters)")
    ap.add_argument("--no-ranker", action="store_true", help="skip the candidate-ranker leg")
    ap.add_argument("--e2e-blocks", type=int, default=8,
                    help="blocks of the end-to-end stream leg of a multi-beam workload (0: skip)")
    ap.add_argument("--no-per-beam", action="store_true",
                    help="skip the comparison run of a multi-beam workload in plain per-beam mode")
    ap.add_argument("--no-uneven", action="store_true", help="skip the 32-beam uneven-batch leg of the c3 run")
    ap.add_argument("--growth", default="96,384,768",
                    help="beam counts of the growing-batch leg of the c3 run (comma-separated; empty: skip)")
    ap.add_argument("--ranker-weights", default=os.path.join(ROOT, "paper_2606_27262_amd", "data",
                                                             "ranker_weights.npy"))
    ap.add_argument("--operating-point", default=os.path.join(ROOT, "paper_2606_27262_amd", "data",
                                                              "ranker_weights_operating_point.json"),
                    help="per-band logit thresholds of the ranker path (JSON written by train_ranker)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: each GPU searches its own share of beams "
              "independently and there is no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_27262_amd import spotlight as spl
    from paper_2606_27262_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    e2e = args.e2e_blocks > 0 and args.workload in ("c3", "c4", "c3s")
    pds, plans, blocks, pulses, _ = make_workload(args.workload, spl, W)
    nb = len(plans)
    mode = args.mode
    if mode == "auto":
        mode = "plain" if nb == 1 else "graph"
    # the uneven batch's zero-DM bursts light up every trial near their time (1.6e8 hits
    # per block): its hit list is sized for them
    batch = spl.Batch(plans, mode=spl.MODE_PERSISTENT_GRAPH if mode == "graph" else spl.MODE_PLAIN_PER_BEAM,
                      hit_capacity=(1 << 28) if args.workload == "c4" else 0)
    batch.attach()
    if not args.no_autotune:
        import tempfile
        cache = args.tile_cache or os.path.join(tempfile.gettempdir(), "spotlight_tiles.txt")
        t_tune = time.perf_counter()
        batch.autotune(blocks, cache_path=cache)
        log(f"autotune {time.perf_counter() - t_tune:.1f}s -> {batch.tiles(0)}")
    cands = spl.new_candidates(1 << 20)
    stats = torch.zeros(spl.STATS_WORDS, dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()

    # profiling (per-stage HIP events) is live in the timed region for eager runs; a
    # graph-mode run is timed as a whole and its stages are timed in a second,
    # eager pass of the same launches
    eager_profile = mode == "plain"
    batch.set_profiling(eager_profile)
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            batch.run(blocks, cands, stats, stream=stream)
    torch.cuda.synchronize()
    st0 = spl.stats_dict(stats)
    if st0["hit_overflow"] or st0["cand_overflow"]:
        raise SystemExit(f"capacity exceeded in the warm-up runs: {st0}")
    batch.stage_times(reset=True)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(args.steps):
            batch.run(blocks, cands, stats, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = spl.stats_dict(stats)
    if eager_profile:
        stages = batch.stage_times(reset=True)
    else:
        batch.set_profiling(True)
        with torch.cuda.stream(stream):
            for _ in range(args.steps):
                batch.run(blocks, cands, stats, stream=stream)
        torch.cuda.synchronize()
        stages = batch.stage_times(reset=True)

    trial_samples = sum(p.info["ndm"] * p.info["n_out"] for p in plans)
    adds = sum(p.info["ndm"] * p.info["nchans"] * p.info["n_out"] for p in plans)
    ms_step = elapsed / args.steps * 1e3
    value = trial_samples * args.steps / elapsed
    block_s = max(pd["n_out"] * pd["tsamp"] for pd in pds)
    rtf = (ms_step / 1e3) / block_s
    dd_ms, dd_n = stages["dedisp"]
    launches_per_step = dd_n / args.steps
    avg_launch_s = dd_ms / 1e3 / dd_n
    adds_per_launch = adds / launches_per_step
    achieved = adds_per_launch / avg_launch_s
    stage_ms = {k: round(v[0] / args.steps, 4) for k, v in stages.items()}
    out = {
        "metric": "DM-trial·samples/s and real-time beams per MI355X",
        "value": value,
        "unit": "DM-trial·samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "beams": nb, "mode": mode, "autotuned": not args.no_autotune,
                   "plans": sorted(set(W.describe(pd) for pd in pds)),
                   "tiles": [batch.tiles(b) for b in sorted(set(range(nb)) & {0, nb - 1})]},
        "real_time_factor": rtf,
        "real_time_beams_per_gpu": nb / rtf,
        "stage_ms_per_step": stage_ms,
        "candidates_per_step": st["n_candidates"],
        "hits_per_step": st["n_hits"],
        "roofline": {"bound": "alu", "kernel": "k_dedisp", "achieved": achieved / 1e12,
                     "peak": PEAK_ADDS / 1e12, "unit": "Tadd/s (int32)", "frac": achieved / PEAK_ADDS,
                     "traffic": None, "launch_ms": avg_launch_s * 1e3,
                     "adds_per_launch": adds_per_launch,
                     # two exact adds per lane and clock (v_add3_u32, or two 16-bit lanes of a
                     # 32-bit add): the kernel's instruction mix reaches for this one
                     "peak_two_adds_per_lane": 2 * PEAK_ADDS / 1e12,
                     "frac_two_adds_per_lane": achieved / (2 * PEAK_ADDS)},
    }
    tr = counter_traffic(args.workload, [batch.tiles(b) for b in range(nb)])
    if tr is not None and launches_per_step == 1:
        out["roofline"]["traffic"] = tr["fetch_bytes"] + tr["write_bytes"]
        out["roofline"]["traffic_detail"] = {
            "unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)", **tr,
            "algorithmic_bytes": sum(p.info["nchans"] * p.info["n_in"] + 4 * p.info["ndm"] * p.info["n_dd"]
                                     for p in plans),
            "achieved_GBps": (tr["fetch_bytes"] + tr["write_bytes"]) / avg_launch_s / 1e9}
    if nb > 1 and not args.no_per_beam and mode == "graph":
        out["plain_per_beam"] = per_beam_comparison(spl, plans, blocks, args, cands, stats)
        out["plain_per_beam"]["real_time_beams_per_gpu"] = nb / (out["plain_per_beam"]["ms_per_step"] / 1e3 / block_s)
    if all(pd["nchans"] % 16 == 0 for pd in pds):
        out["corner_turn"] = corner_turn_leg(spl, plans[0])
    if any(pulses):
        log("injector leg")
        out["injector"] = injector_leg(spl, W, pds, plans, blocks, pulses, ms_step)
    if not args.no_ranker and all(pd["nchans"] % 64 == 0 for pd in pds):
        log("ranker leg")
        out["ranker"] = ranker_leg(spl, pds, plans, batch, blocks, pulses, cands, stats, stream, args, ms_step,
                                   block_s)
    tiles0 = batch.tiles(0)
    del batch, blocks
    torch.cuda.empty_cache()
    if e2e:
        log("end-to-end stream")
        out["end_to_end"] = end_to_end_leg(spl, W, pds, args, n_blocks=args.e2e_blocks)
        torch.cuda.empty_cache()
    if args.workload == "c3" and not args.no_uneven:
        log("uneven 32-beam batch")
        out["uneven_batch"] = uneven_leg(spl, W, args)
    if args.workload == "c3" and args.growth:
        log("growing the batch")
        out["real_time_beams"] = growth_leg(spl, W, pds[0], tiles0, block_s,
                                            sizes=tuple(int(v) for v in args.growth.split(",")))
        out["real_time_beams"]["sizes"].insert(0, {"beams": nb, "ms_per_step": ms_step, "ms_per_beam": ms_step / nb,
                                                   "real_time_factor": rtf, "dm_trial_samples_per_s": value})
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(pds[0], plans[0], W)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
