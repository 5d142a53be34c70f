"""Sustained search of continuous beam streams (the paper's real-time loop: blocks are
read with an overlap so that every sweep and boxcar of the owned samples is complete;
each block of every beam is searched while the next one is read in, and the candidates
of a block are optimised and classified while the next block is searched).

Device ring.  Block k of a beam owns stream samples [k n_out, (k+1) n_out) and reads
[k n_out, k n_out + n_in): consecutive blocks share n_in - n_out = s_max + w_max - 1
samples.  Three device block slots per beam rotate; for block k >= 1 only its n_out new
samples cross the host link, as one contiguous copy from pinned host memory into a
device staging buffer on the copy stream; on the same stream spl_stream_assemble then
writes slot k % 3 from the previous block's tail (slot (k-1) % 3) and the staged samples,
while block k-1 is searched.  The first block of a stream is uploaded whole.
The normaliser is not carried: each block's mean and sigma come from its own owned
samples (a search of block k is a function of block k alone, equal to the oracle's
search of the same samples).

Three batches, one per slot, each with its own workspace, rotate with the slots (a batch
always sees the same block pointers, so a run uploads nothing that could queue behind
the big copy).  For block k, slot k % 3:
  compute stream search of block k (after its assembly; persistent launch, hipGraph),
                 then the run statistics and a prefix of the records to pinned host
                 memory
  copy stream    new samples of block k+1 -> staging buffer (k+1) % 3 and the assembly
                 of slot (k+1) % 3 from them and the tail of slot k % 3, enqueued right
                 after the search of k: that buffer and that slot last fed block k-2,
                 whose search the host has waited for
  host           candidate stage of block k-1: plain optimisation path, or the ranker
                 path (grouping, snippets and CNN on a third stream, anti-coincidence)
So the copy of the next block and the candidate stage of the previous one both overlap
the search of the current one.  Every copy between host and device goes through pinned
buffers on a stream: a copy into pageable host memory would wait for the whole device,
i.e. for the search of the next block.  The record prefix copied back is a power of two
above the largest count seen; records beyond it, if a block has more, are fetched after
the statistics arrive (copying the whole 1M-record buffer there instead queued it behind
the next block's upload and held back the next search by ~7 ms).  All device memory and
streams come from torch; every step of the search runs in libspotlight.
"""
from __future__ import annotations

import time

import numpy as np

from . import ranking


class StreamingSearch:
    def __init__(self, spl, pds, ranker=None, mode=None, cand_capacity=1 << 20, max_scored=16384, hit_capacity=0,
                 thresholds=0.0):
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
        self.batches = [spl.Batch(plans, mode=mode, hit_capacity=hit_capacity) for _ in range(3)]
        self.cands = [spl.new_candidates(cand_capacity) for _ in range(3)]
        self.stats = [torch.zeros(spl.STATS_WORDS, dtype=torch.int64, device="cuda") for _ in range(3)]
        self.dev = [[torch.empty((p.info["nchans"], (p.info["n_in"] + 255) // 256 * 256), dtype=torch.uint8,
                                 device="cuda") for p in plans] for _ in range(3)]
        self.stage = [[spl.new_stage(p.info["nchans"], p.info["n_out"]) for p in plans] for _ in range(3)]
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
        self.thresholds = thresholds   # the ranker path's logit threshold (a number or one per beam)

    def attach(self, tile_cache=None):
        for b, dev in zip(self.batches, self.dev):
            b.attach()
            if tile_cache:
                b.autotune(dev, cache_path=tile_cache)

    def copy_rate(self, chunk_set, reps=3):
        """Bytes/s of the new samples of one block of every beam (pinned host memory ->
        staging buffers) on the copy stream, alone."""
        import torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(self.copy_stream):
            e0.record(self.copy_stream)
            for _ in range(reps):
                for d, h in zip(self.stage[0], chunk_set):
                    d.copy_(h, non_blocking=True)
            e1.record(self.copy_stream)
        torch.cuda.synchronize()
        return reps * sum(h.numel() for h in chunk_set) / (e0.elapsed_time(e1) / 1e3)

    def assemble_time(self, reps=3):
        """Seconds of spl_stream_assemble for every beam (slot 0 and staging buffer 1 ->
        slot 1) on the compute stream, alone."""
        import torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(self.compute_stream):
            e0.record(self.compute_stream)
            for _ in range(reps):
                for p, dn, dp, st in zip(self.plans, self.dev[1], self.dev[0], self.stage[1]):
                    self.spl.stream_assemble(dn, dp, st, p.info["n_out"], p.info["n_in"], stream=self.compute_stream)
            e1.record(self.compute_stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    def _fetch(self, slot, searched):
        """Complete the block's candidate records on the host: the prefix copied behind
        the search already holds the first `copied` of them; any beyond it are copied now
        (and the prefix grows for later blocks).  Returns their number and the search's
        total."""
        import torch
        n = int(self.h_stats[slot][1])
        ov = int(self.h_stats[slot][6])
        if ov & 0xFFFFFFFF:
            raise RuntimeError(f"a block had {int(self.h_stats[slot][0])} boxcar hits, more than the batch's hit "
                               "capacity: create the stream with a larger hit_capacity")
        if ov >> 32:
            raise RuntimeError(f"a block had {n} candidates, more than the candidate capacity: create the stream "
                               "with a larger cand_capacity")
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

    def _stage(self, slot, recs, n):
        """Candidate stage of the block searched in batch `slot` (its records `recs`)."""
        import torch
        spl = self.spl
        if self.ranker is None:
            return spl.optimise_plain(recs, self.tsamp, self.nb), n
        batch = self.batches[slot]

        def score(r):
            k = r.size   # at most max_scored: ranker_path routes the rest to the plain path
            self.h_recs[:k].numpy()[:] = np.ascontiguousarray(r).view(np.int32).reshape(-1, 8)
            with torch.cuda.stream(self.rank_stream):
                self.d_recs[:k].copy_(self.h_recs[:k], non_blocking=True)
                spl.snippets(batch, self.d_recs, n=k, out=self.d_snip[:k], stream=self.rank_stream)
                self.ranker.score(self.d_snip[:k], logits=self.d_logits[:k], stream=self.rank_stream)
                self.h_logits[:k].copy_(self.d_logits[:k], non_blocking=True)
            self.rank_stream.synchronize()
            return self.h_logits[:k].numpy().copy()

        final, _, _ = ranking.ranker_path(spl, recs, self.tsamp, self.nb, score, threshold=self.thresholds,
                                          max_scored=self.max_scored)
        return final, n

    def run(self, first_set, chunk_sets, n_blocks, warmup=2, on_block=None, timing=None):
        """Stream n_blocks consecutive blocks of every beam's continuous stream.
        first_set: per beam a pinned uint8 tensor [nch][pitch] (pitch = the slot pitch,
        n_in rounded up to 256) holding block 0.  chunk_sets: a list of sets, each per
        beam a pinned contiguous uint8 tensor [nch][n_out] of new samples; block k >= 1 is
        the last n_in - n_out samples of block k-1 followed by
        chunk_sets[(k - 1) % len(chunk_sets)].
        Returns the wall time per block over the blocks after `warmup` (the last block's
        candidate stage, which nothing overlaps, included) and the per-block results of
        on_block(k, final, n_candidates, records).  With a dict `timing`, also fills in
        the steady-state period: the device time from the first measured block's start
        to the end of the last block's search and its copies back, per block
        ("steady_s"), the candidate stage of the last block alone ("drain_s") and the
        host-to-device bytes per block after the first ("h2d_bytes_per_block")."""
        import torch
        spl = self.spl
        copied = [torch.cuda.Event() for _ in range(3)]
        searched = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        t_ev0 = torch.cuda.Event(enable_timing=True)
        results = []
        n_out = [p.info["n_out"] for p in self.plans]
        n_in = [p.info["n_in"] for p in self.plans]
        for h, d in zip(first_set, self.dev[0]):
            assert h.shape == d.shape and h.is_pinned()
        for cs in chunk_sets:
            for b, h in enumerate(cs):
                assert h.is_pinned() and h.is_contiguous() and h.shape == (self.plans[b].info["nchans"], n_out[b])

        def enqueue_copy(k):
            s = k % 3
            with torch.cuda.stream(self.copy_stream):
                if k == 0:
                    for d, h in zip(self.dev[s], first_set):
                        d.copy_(h, non_blocking=True)
                else:
                    for d, h in zip(self.stage[s], chunk_sets[(k - 1) % len(chunk_sets)]):
                        d.copy_(h, non_blocking=True)
                    # slot s last held block k-3, whose search the host has waited for; the
                    # previous slot holds block k-1, assembled earlier on this stream and
                    # only read (by its search) meanwhile
                    for b, (dn, dp, st) in enumerate(zip(self.dev[s], self.dev[(k - 1) % 3], self.stage[s])):
                        spl.stream_assemble(dn, dp, st, n_out[b], n_in[b], stream=self.copy_stream)
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
                # staging buffer and slot (k+1) % 3 last fed block k-2, whose search the
                # host waited for in the previous iteration
                enqueue_copy(k + 1)
            if k >= 1:
                searched[(k - 1) % 3].synchronize()
                t_stage = time.perf_counter()
                m, ncand = self._fetch((k - 1) % 3, searched[(k - 1) % 3])
                recs = self.h_cands[(k - 1) % 3][:m].numpy().view(self.spl.CAND_DTYPE).reshape(-1).copy()
                final, ncand = self._stage((k - 1) % 3, recs, ncand)
                if on_block is not None:
                    results.append(on_block(k - 1, final, ncand, recs))
        torch.cuda.synchronize()
        t_end = time.perf_counter()
        wall = t_end - t_start
        m = max(1, n_blocks - warmup)
        if timing is not None:
            timing["steady_s"] = t_ev0.elapsed_time(searched[(n_blocks - 1) % 3]) / 1e3 / m
            timing["drain_s"] = t_end - t_stage
            timing["h2d_bytes_per_block"] = int(sum(p.info["nchans"] * n for p, n in zip(self.plans, n_out)))
        return wall / m, results
