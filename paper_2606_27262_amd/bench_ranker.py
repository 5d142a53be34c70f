"""Throughput of the ranker's CNN kernels on one GPU: inference (forward pass and
logits) and training steps (forward, backward, Adam) on batches of synthetic snippets,
timed with HIP events on the launch stream; prints one JSON line.

    python -m paper_2606_27262_amd.bench_ranker --batch 256 --reps 20

The work per candidate is the network's multiply-adds x 2 (118.2 MFLOP forward, three
times that for a training step), against the 2.5 PFLOP/s dense BF16 matrix-core peak.
Under rocprofv3 --kernel-trace the per-kernel durations of the same launches appear.
"""
from __future__ import annotations

import argparse
import json
import sys


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="both", choices=["both", "infer", "train"])
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this size first (calibrates HBM byte counters)")
    a = ap.parse_args(argv)

    import numpy as np
    import torch

    from . import ranking
    from . import spotlight as spl

    assert torch.cuda.is_available(), "the ranker benchmark needs a GPU"
    if a.copy_probe_mib:
        src = torch.ones(a.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    rng = np.random.default_rng(0)
    n = a.batch
    x = torch.from_numpy(rng.normal(0, 1, size=(n, 2, 64, 256)).astype(np.float32)).cuda()
    snip = (x.view(torch.int32) >> 16).to(torch.int16)
    lab = torch.from_numpy((rng.random(n) < 0.5).astype(np.float32)).cuda()
    r = spl.Ranker(max_batch=n)
    r.set_weights(ranking.initial_weights(1))
    s = torch.cuda.current_stream()
    # multiply-adds x 2 of one forward pass: four 3x3 convolutions (2 -> 32 channels at
    # 64 x 256, then 32 -> 32 at 32 x 128, 16 x 64, 8 x 32) and the two dense layers
    flop_fwd = 2.0 * 9 * (2 * 32 * 64 * 256 + 32 * 32 * (32 * 128 + 16 * 64 + 8 * 32)) + 2.0 * (2048 * 64 + 64)
    out = {"batch": n, "flop_forward_per_candidate": flop_fwd, "peak_tflops_bf16": 2500.0}

    def timed(fn):
        for _ in range(a.warmup):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        for _ in range(a.reps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / a.reps / 1e3

    if a.mode in ("both", "infer"):
        t = timed(lambda: r.score(snip))
        out["inference"] = {"ms": t * 1e3, "candidates_per_s": n / t, "tflops": n * flop_fwd / t / 1e12,
                            "frac_peak": n * flop_fwd / t / 2.5e15}
    if a.mode in ("both", "train"):
        t = timed(lambda: r.train_step(snip, lab, 1e-4))
        out["train_step"] = {"ms": t * 1e3, "candidates_per_s": n / t, "tflops": 3 * n * flop_fwd / t / 1e12,
                             "frac_peak": 3 * n * flop_fwd / t / 2.5e15}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
