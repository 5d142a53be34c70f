"""Train the CNN candidate ranker on synthetic bursts in searched 4096-channel blocks and
compare the ranker path with the plain optimisation path on fresh blocks.

    python -m paper_2606_27262_amd.train_ranker --train-batches 30 --out weights.npy

Training set: NMS candidates of blocks with injected bursts (DM 20-2000, FWHM 1-128
samples, S/N 6-30), 2% RFI channels and zero-DM bursts common to the beams; positives
are candidates matching a burst, negatives an equal number of the others.  Prints one
JSON line with the training history and the evaluation.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train-batches", type=int, default=30)
    ap.add_argument("--beams", type=int, default=8, help="beams per training batch")
    ap.add_argument("--pulses", type=int, default=8, help="bursts per beam and block")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--max-batch", type=int, default=256)
    ap.add_argument("--eval-batches", type=int, default=2)
    ap.add_argument("--eval-beams", type=int, default=24)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--eval-seed", type=int, default=7000)
    ap.add_argument("--out", default="ranker_weights.npy")
    ap.add_argument("--fine-keep", type=float, default=None,
                    help="train and evaluate on fine-DM planes (DM* +- the offset keeping this S/N fraction)")
    ap.add_argument("--json", default=None)
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
    ranker = spl.Ranker(max_batch=a.max_batch)
    if a.eval_only:
        ranker.set_weights(np.load(a.eval_only))
        pde = [W.plan_c2() for _ in range(a.eval_beams)]
        res = ranking.evaluate(spl, pde, ranker, a.eval_batches, a.eval_seed, log=log, n_pulses=a.pulses,
                               fine_keep=a.fine_keep)
        line = json.dumps({"eval": res, "fine_keep": a.fine_keep, "weights": os.path.abspath(a.eval_only),
                           "wall_s": time.time() - t_start})
        print(line, flush=True)
        if a.json:
            with open(a.json, "w") as f:
                f.write(line + "\n")
        return
    ranker.set_weights(ranking.initial_weights(a.seed))
    pds = [W.plan_c2() for _ in range(a.beams)]
    x, y = ranking.mine(spl, pds, a.train_batches, a.seed * 100000, log=log, n_pulses=a.pulses,
                        fine_keep=a.fine_keep)
    log(f"training set: {x.shape[0]} snippets, {int(y.sum())} positive")
    t_train = time.time()
    hist = ranking.train(ranker, x, y, epochs=a.epochs, batch=a.max_batch, lr=a.lr, seed=a.seed, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t_train
    w = ranker.get_weights()
    np.save(a.out, w)
    del x
    pde = [W.plan_c2() for _ in range(a.eval_beams)]
    res = ranking.evaluate(spl, pde, ranker, a.eval_batches, a.eval_seed, log=log, n_pulses=a.pulses,
                           fine_keep=a.fine_keep)
    out = {"fine_keep": a.fine_keep, "train": {"snippets": int(y.size), "positives": int(y.sum()), "epochs": a.epochs, "lr": a.lr,
                     "batch": a.max_batch, "seconds": t_train,
                     "history": [[e, round(l, 5), round(v, 4)] for e, l, v in hist]},
           "eval": res, "weights": os.path.abspath(a.out), "wall_s": time.time() - t_start}
    line = json.dumps(out)
    print(line, flush=True)
    if a.json:
        with open(a.json, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
