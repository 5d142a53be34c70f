"""Train the CNN candidate ranker on synthetic bursts in searched blocks of both bands and
compare the ranker path with the plain optimisation path on fresh blocks of each band.

    python -m paper_2606_27262_amd.train_ranker --bursts 100000 --out weights.npy

Training set, per band (the 4096-channel 550-750 MHz plan with 2048 trials to DM 2000,
and the 2048-channel 300-500 MHz plan at 0.65536 ms with 1024 trials to DM 1000):
blocks with injected bursts (DM U(20, min(2000, 0.98 of the plan's last DM)), FWHM
log-U(1, 128) samples, S/N U(6, 30)), 2 % RFI channels and zero-DM bursts common to the
beams, made on the GPU (synth.make_block_torch) and searched by the library; of the NMS
candidates matching a burst the strongest and one other per burst are positives, an
equal number of unmatched candidates negatives.  Every burst is distinct.  Prints one
JSON line with the training history and the per-band evaluation.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time


def log(*a):
    print(*a, file=sys.stderr, flush=True)


BANDS = {
    "550-750MHz/4096ch": {"plan": "plan_c2", "pulses": 10},
    "300-500MHz/2048ch": {"plan": "plan_band3_c4", "pulses": 20},
}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--bursts", type=int, default=100000, help="distinct injected bursts per band")
    ap.add_argument("--bands", default=",".join(BANDS), help="comma-separated band names")
    ap.add_argument("--beams", type=int, default=8, help="beams per training batch")
    ap.add_argument("--per-burst", type=int, default=2, help="positive snippets kept per burst")
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--max-batch", type=int, default=256)
    ap.add_argument("--eval-batches", type=int, default=4)
    ap.add_argument("--eval-beams", type=int, default=24)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--eval-seed", type=int, default=7000)
    ap.add_argument("--init", default=None, metavar="WEIGHTS", help="start from these weights (.npy)")
    ap.add_argument("--out", default="ranker_weights.npy")
    ap.add_argument("--fine-keep", type=float, default=None,
                    help="train and evaluate on fine-DM planes (DM* +- the offset keeping this S/N fraction)")
    ap.add_argument("--json", default=None)
    ap.add_argument("--op-out", default=None, metavar="JSON",
                    help="write the per-band operating point (the logit threshold at the plain path's false-alarm "
                         "count on the evaluation blocks); default: next to --out")
    ap.add_argument("--eval-only", default=None, metavar="WEIGHTS",
                    help="skip training: evaluate these weights (.npy) against the plain path")
    a = ap.parse_args(argv)

    import numpy as np
    import torch

    from . import ranking
    from . import spotlight as spl
    from . import workloads as W

    assert torch.cuda.is_available(), "training runs on the GPU"
    t_start = time.time()
    bands = [b for b in a.bands.split(",") if b]
    ranker = spl.Ranker(max_batch=a.max_batch)
    out = {"fine_keep": a.fine_keep, "bands": {}}
    if a.eval_only:
        ranker.set_weights(np.load(a.eval_only))
        out["weights"] = os.path.abspath(a.eval_only)
    else:
        ranker.set_weights(np.load(a.init) if a.init else ranking.initial_weights(a.seed))
        xs, ys = [], []
        for bi, name in enumerate(bands):
            cfg = BANDS[name]
            pd = getattr(W, cfg["plan"])()
            pds = [pd for _ in range(a.beams)]
            n_batches = int(math.ceil(a.bursts / (a.beams * cfg["pulses"])))
            t0 = time.time()
            x, y, n_b, n_f = ranking.mine(spl, pds, n_batches, (a.seed * 10 + bi) * 1_000_000, log=log,
                                          n_pulses=cfg["pulses"], fine_keep=a.fine_keep, per_burst=a.per_burst,
                                          device="cuda", mode=spl.MODE_PERSISTENT_GRAPH)
            out["bands"][name] = {"train": {"bursts": n_b, "bursts_detected": n_f, "snippets": int(y.size),
                                            "positives": int(y.sum()), "blocks": n_batches * a.beams,
                                            "mining_s": round(time.time() - t0, 1)}}
            log(f"{name}: {n_b} bursts, {n_f} with a candidate, {y.size} snippets ({int(y.sum())} positive) "
                f"in {time.time() - t0:.0f} s")
            xs.append(x)
            ys.append(y)
            torch.cuda.empty_cache()
        x = torch.cat(xs)
        y = np.concatenate(ys)
        del xs
        t_train = time.time()
        hist = ranking.train(ranker, x, y, epochs=a.epochs, batch=a.max_batch, lr=a.lr, seed=a.seed, log=log)
        torch.cuda.synchronize()
        out["train"] = {"snippets": int(y.size), "positives": int(y.sum()), "epochs": a.epochs, "lr": a.lr,
                        "batch": a.max_batch, "seconds": round(time.time() - t_train, 1),
                        "history": [[e, round(l_, 5), round(v, 4)] for e, l_, v in hist]}
        np.save(a.out, ranker.get_weights())
        out["weights"] = os.path.abspath(a.out)
        del x
        torch.cuda.empty_cache()
    for bi, name in enumerate(bands):
        cfg = BANDS[name]
        pd = getattr(W, cfg["plan"])()
        pde = [pd for _ in range(a.eval_beams)]
        res = ranking.evaluate(spl, pde, ranker, a.eval_batches, a.eval_seed + 1000 * bi, log=log,
                               n_pulses=cfg["pulses"], fine_keep=a.fine_keep, device="cuda",
                               mode=spl.MODE_PERSISTENT_GRAPH)
        out["bands"].setdefault(name, {})["eval"] = res
        m = res["ranker_at_plain_false_alarms"]
        log(f"{name}: plain recall {res['plain']['recall']:.3f} ({res['plain']['false_alarms']} false alarms), "
            f"ranker recall {res['ranker']['recall']:.3f} ({res['ranker']['false_alarms']}), at the plain "
            f"path's false alarms {m['recall'] if m else float('nan'):.3f}")
    if not a.eval_only:
        op_path = a.op_out or os.path.splitext(a.out)[0] + "_operating_point.json"
        op = {"source": "held-out evaluation of train_ranker (fresh seeds): the lowest logit threshold whose final "
                        "list holds no more unmatched candidates than the plain path's",
              "logit_threshold": {name: b["eval"]["ranker_at_plain_false_alarms"]["threshold_logit"]
                                  for name, b in out["bands"].items()
                                  if b.get("eval", {}).get("ranker_at_plain_false_alarms")}}
        with open(op_path, "w") as f:
            f.write(json.dumps(op, indent=1) + "\n")
        out["operating_point"] = op_path
    out["wall_s"] = round(time.time() - t_start, 1)
    line = json.dumps(out)
    print(line, flush=True)
    if a.json:
        with open(a.json, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
