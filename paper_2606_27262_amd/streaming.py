"""Sustained search of a stream of blocks (the paper's real-time loop: each block of
every beam is searched while the next one is read in, and the candidates of a block
are optimised and classified while the next block is searched).

Three batches, each with its own workspace and its own device block set, rotate (a
batch always sees the same block pointers, so a run uploads nothing that could queue
behind the big copy).  For block k, slot k % 3:
  compute stream search of block k in its slot (persistent launch, hipGraph), after
                 its copy
  copy stream    pinned host blocks of k+1 -> slot (k+1) % 3, enqueued right after the
                 search of k: that slot last held block k-2, done in the previous step
  host           candidate stage of block k-1: plain optimisation path, or the ranker
                 path (grouping, snippets and CNN on a third stream, anti-coincidence)
So the copy of the next block and the candidate stage of the previous one both overlap
the search of the current one.  Every copy between host and device goes through pinned
buffers on a stream: a copy into pageable host memory would wait for the whole device,
i.e. for the search of the next block.  The run statistics and a prefix of the
candidate records (a power of two above the largest count seen) follow the search on
the compute stream; records beyond the prefix, if a block has more, are fetched after
the statistics arrive.  Copying the whole 1M-record buffer there instead queued it
behind the next block's 2.6 GB upload and held back the next search by ~7 ms.  All
device memory and streams come from torch; every step of the search runs in
libspotlight.
"""
from __future__ import annotations

import time

import numpy as np

from . import ranking


class StreamingSearch:
    def __init__(self, spl, pds, ranker=None, mode=None, cand_capacity=1 << 20, max_scored=16384):
        import torch
        self.spl, self.pds, self.ranker = spl, pds, ranker
        self.nb = len(pds)
        plans, cache = [], {}
        for pd in pds:
            key = repr(sorted(pd.items()))
            if key not in cache:
                cache[key] = spl.Plan.from_dict(pd)
            plans.append(cache[key])
        self.plans = plans
        mode = spl.MODE_PERSISTENT_GRAPH if mode is None else mode
        self.batches = [spl.Batch(plans, mode=mode) for _ in range(3)]
        self.cands = [spl.new_candidates(cand_capacity) for _ in range(3)]
        self.stats = [torch.zeros(spl.STATS_WORDS, dtype=torch.int64, device="cuda") for _ in range(3)]
        self.dev = [[torch.empty((p.info["nchans"], (p.info["n_in"] + 255) // 256 * 256), dtype=torch.uint8,
                                 device="cuda") for p in plans] for _ in range(3)]
        self.h_cands = [torch.empty((cand_capacity, 8), dtype=torch.int32, pin_memory=True) for _ in range(3)]
        self.h_stats = [torch.empty(spl.STATS_WORDS, dtype=torch.int64, pin_memory=True) for _ in range(3)]
        # ranker stage buffers
        self.max_scored = max_scored
        self.h_recs = torch.empty((max_scored, 8), dtype=torch.int32, pin_memory=True)
        self.d_recs = torch.empty((max_scored, 8), dtype=torch.int32, device="cuda")
        self.d_snip = torch.empty((max_scored, 2, spl.SNIPPET_ROWS, spl.SNIPPET_COLS), dtype=torch.int16, device="cuda")
        self.d_logits = torch.empty(max_scored, dtype=torch.float32, device="cuda")
        self.h_logits = torch.empty(max_scored, dtype=torch.float32, pin_memory=True)
        self.copy_stream = torch.cuda.Stream()
        self.compute_stream = torch.cuda.Stream()
        self.rank_stream = torch.cuda.Stream()
        # records copied back right behind each search: a power of two above the largest
        # count seen (the whole 1M-record buffer queued behind the next block's upload on
        # the copy engine and held back the next search by ~7 ms)
        self.copy_hint = min(cand_capacity, 1 << 17)
        self.copied = [0, 0, 0]
        self.tsamp = np.array([pd["tsamp"] for pd in pds], np.float64)

    def attach(self, tile_cache=None):
        for b, dev in zip(self.batches, self.dev):
            b.attach()
            if tile_cache:
                b.autotune(dev, cache_path=tile_cache)

    def copy_rate(self, host_set, reps=3):
        """Bytes/s of one pinned host -> device copy of a block set on the copy stream."""
        import torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(self.copy_stream):
            e0.record(self.copy_stream)
            for _ in range(reps):
                for d, h in zip(self.dev[0], host_set):
                    d.copy_(h, non_blocking=True)
            e1.record(self.copy_stream)
        torch.cuda.synchronize()
        return reps * sum(h.numel() for h in host_set) / (e0.elapsed_time(e1) / 1e3)

    def _fetch(self, slot, searched):
        """Complete the block's candidate records on the host: the prefix copied behind
        the search already holds the first `copied` of them; any beyond it are copied now
        (and the prefix grows for later blocks).  Returns their number and the search's
        total."""
        import torch
        n = int(self.h_stats[slot][1])
        cap = self.h_cands[slot].shape[0]
        m = min(n, cap)
        c = self.copied[slot]
        if m > c:   # rare: more records than the prefix; the common path touches no stream
            self.rank_stream.wait_event(searched)
            with torch.cuda.stream(self.rank_stream):
                self.h_cands[slot][c:m].copy_(self.cands[slot][c:m], non_blocking=True)
            self.rank_stream.synchronize()
        while self.copy_hint < cap and self.copy_hint < m + (m >> 2):
            self.copy_hint = min(cap, 2 * self.copy_hint)
        return m, n

    def _stage(self, slot, m, n):
        """Candidate stage of the block searched in batch `slot`: its m records are in
        pinned host memory."""
        import torch
        spl = self.spl
        recs = self.h_cands[slot][:m].numpy().view(spl.CAND_DTYPE).reshape(-1).copy()
        if self.ranker is None:
            return spl.optimise_plain(recs, self.tsamp, self.nb), n
        batch = self.batches[slot]

        def score(r):
            k = min(r.size, self.max_scored)   # beyond max_scored records are kept unscored (logit +inf)
            out = np.full(r.size, np.inf, np.float32)
            if k == 0:
                return out
            self.h_recs[:k].numpy()[:] = np.ascontiguousarray(r[:k]).view(np.int32).reshape(-1, 8)
            with torch.cuda.stream(self.rank_stream):
                self.d_recs[:k].copy_(self.h_recs[:k], non_blocking=True)
                spl.snippets(batch, self.d_recs, n=k, out=self.d_snip[:k], stream=self.rank_stream)
                self.ranker.score(self.d_snip[:k], logits=self.d_logits[:k], stream=self.rank_stream)
                self.h_logits[:k].copy_(self.d_logits[:k], non_blocking=True)
            self.rank_stream.synchronize()
            out[:k] = self.h_logits[:k].numpy()
            return out

        final, _, _ = ranking.ranker_path(spl, recs, self.tsamp, self.nb, score)
        return final, n

    def run(self, host_sets, n_blocks, warmup=2, on_block=None, timing=None):
        """Stream n_blocks blocks, block k taken from host_sets[k % len(host_sets)] (lists of
        pinned uint8 tensors [nch][pitch], one per beam).  Returns the wall time per block
        over the blocks after `warmup` (the last block's candidate stage, which nothing
        overlaps, included) and the per-block results of on_block(k, final,
        n_candidates).  With a dict `timing`, also fills in the steady-state period: the
        device time from the first measured block's start to the end of the last block's
        search and its copies back, per block ("steady_s"), and the candidate stage of the
        last block alone ("drain_s")."""
        import torch
        copied = [torch.cuda.Event() for _ in range(3)]
        searched = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        t_ev0 = torch.cuda.Event(enable_timing=True)
        results = []

        def enqueue_copy(k):
            s = k % 3
            src = host_sets[k % len(host_sets)]
            with torch.cuda.stream(self.copy_stream):
                for d, h in zip(self.dev[s], src):
                    d.copy_(h, non_blocking=True)
                copied[s].record(self.copy_stream)

        def enqueue_search(k):
            s = k % 3
            self.compute_stream.wait_event(copied[s])
            self.batches[s].run(self.dev[s], self.cands[s], self.stats[s], stream=self.compute_stream)
            c = self.copy_hint
            with torch.cuda.stream(self.compute_stream):
                self.h_stats[s].copy_(self.stats[s], non_blocking=True)
                self.h_cands[s][:c].copy_(self.cands[s][:c], non_blocking=True)
            self.copied[s] = c
            searched[s].record(self.compute_stream)

        torch.cuda.synchronize()
        enqueue_copy(0)
        t_start = None
        for k in range(n_blocks + 1):
            if k == warmup:
                torch.cuda.synchronize()
                t_start = time.perf_counter()
                t_ev0.record(self.compute_stream)
            if k < n_blocks:
                enqueue_search(k)
            if k + 1 < n_blocks:
                enqueue_copy(k + 1)   # set (k+1) % 3 last held block k-2, done in the previous iteration
            if k >= 1:
                searched[(k - 1) % 3].synchronize()
                t_stage = time.perf_counter()
                m, ncand = self._fetch((k - 1) % 3, searched[(k - 1) % 3])
                final, ncand = self._stage((k - 1) % 3, m, ncand)
                if on_block is not None:
                    results.append(on_block(k - 1, final, ncand))
        torch.cuda.synchronize()
        t_end = time.perf_counter()
        wall = t_end - t_start
        m = max(1, n_blocks - warmup)
        if timing is not None:
            timing["steady_s"] = t_ev0.elapsed_time(searched[(n_blocks - 1) % 3]) / 1e3 / m
            timing["drain_s"] = t_end - t_stage
        return wall / m, results
