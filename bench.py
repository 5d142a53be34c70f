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
    else:
        raise SystemExit(f"unknown workload {name}")
    plans, cache = [], {}
    for pd in pds:
        key = json.dumps(pd, sort_keys=True, default=str)
        if key not in cache:
            cache[key] = spl.Plan.from_dict(pd)
        plans.append(cache[key])
    blocks, pulses = [], []
    seed = {"c1": 1, "c2": 2, "c3": 3, "c4": 4}[name]
    for b, (pd, p) in enumerate(zip(pds, plans)):
        n_in = p.info["n_in"]
        if name == "c1":
            spec, x = W.c1_block(n_in, seed=seed)
        elif name == "c2":
            spec, x = W.c2_like_block(pd, n_in, seed, b, 20)
        elif name == "c3":
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


def end_to_end_leg(spl, pds, host, pulses, args, n_blocks=8, warmup=2):
    """Sustained stream of blocks (paper_2606_27262_amd.streaming): pinned host-to-device
    copy of the next block and the candidate stage of the previous block overlap the
    search of the current one.  The stream repeats the workload's blocks."""
    import tempfile

    import numpy as np

    from paper_2606_27262_amd import ranking, streaming
    block_s = max(pd["n_out"] * pd["tsamp"] for pd in pds)
    ss = streaming.StreamingSearch(spl, pds)
    ss.attach(tile_cache=None if args.no_autotune else
              (args.tile_cache or os.path.join(tempfile.gettempdir(), "spotlight_tiles.txt")))
    out = {"blocks": n_blocks, "warmup": warmup,
           "h2d_bytes_per_block": int(sum(h.numel() for h in host)),
           "h2d_GBps_alone": ss.copy_rate(host) / 1e9}
    legs = [("plain", None)]
    if not args.no_ranker and all(pd["nchans"] % 64 == 0 for pd in pds):
        r = spl.Ranker(max_batch=256)
        r.set_weights(np.load(args.ranker_weights) if os.path.exists(args.ranker_weights)
                      else ranking.initial_weights(0))
        legs.append(("ranker", r))
    for name, ranker in legs:
        ss.ranker = ranker
        wall, res = ss.run([host], n_blocks, warmup,
                           on_block=lambda k, f, nc: ranking.recall_and_false_alarms(f, pulses, pds))
        out[name] = {"ms_per_block": wall * 1e3, "real_time_beams_per_gpu": len(pds) * block_s / wall,
                     "recall": float(np.mean([q["recall"] for q in res])),
                     "false_alarms_per_beam_block": float(np.mean([q["false_alarms"] for q in res])) / len(pds)}
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
    D = plan.delays().astype(np.int64)
    dms = plan.dms()
    i = plan.info
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
    out = {"value": k2 * i["n_out"] / t2, "unit": "DM-trial·samples/s", "cores": oracle.num_threads(),
           "kind": "oracle", "seconds": round(t2, 3),
           "sample": f"first {k2} of {i['ndm']} DM trials x {i['n_out']} samples of one "
                     f"{i['nchans']}-channel block: dedispersion + boxcar search + peak filters"}
    r = last["r"]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4"])
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
    ap.add_argument("--ranker-weights", default=os.path.join(ROOT, "paper_2606_27262_amd", "data",
                                                             "ranker_weights.npy"))
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build runs each GPU's share of beams "
              "independently and has no multi-GPU path; run with --gpus 1", file=sys.stderr)
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
    e2e = args.e2e_blocks > 0 and args.workload in ("c3", "c4")
    pds, plans, blocks, pulses, host = make_workload(args.workload, spl, W, keep_host=e2e)
    nb = len(plans)
    mode = args.mode
    if mode == "auto":
        mode = "plain" if nb == 1 else "graph"
    batch = spl.Batch(plans, mode=spl.MODE_PERSISTENT_GRAPH if mode == "graph" else spl.MODE_PLAIN_PER_BEAM)
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
                     "adds_per_launch": adds_per_launch},
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
    if not args.no_ranker and all(pd["nchans"] % 64 == 0 for pd in pds):
        log("ranker leg")
        out["ranker"] = ranker_leg(spl, pds, plans, batch, blocks, pulses, cands, stats, stream, args, ms_step,
                                   block_s)
    if e2e:
        log("end-to-end stream")
        del batch
        out["end_to_end"] = end_to_end_leg(spl, pds, host, pulses, args, n_blocks=args.e2e_blocks)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(pds[0], plans[0], W)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
