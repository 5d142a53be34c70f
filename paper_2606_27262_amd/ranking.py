"""Candidate classification stage on the library's kernels (classification section of
the paper): matching of candidates to injected bursts (labels), mining of labelled
snippets from searched blocks, the training loop of the CNN ranker, and the inline
ranking of the candidates that survive the plain optimisation path.

Every numerical step runs in libspotlight (search, snippets, CNN); this module only
moves records between host and device and draws the synthetic bursts.

Labels.  A candidate (t, w, DM) of beam b matches an injected burst (t0, FWHM W, DM0)
of the same beam when |t - t0| <= max(w, W) + 4 samples and
|DM - DM0| <= (max(w, W) + 4) / k + dm_step, with k the dispersion delay across the
band per unit DM in samples (Eq. (1) between the outer channel centres): beyond that
DM offset the burst is smeared over more than its own width plus the margin.

A candidate that matches no burst but lies on a burst's dispersion track is a side
lobe of that burst, not a false alarm: dedispersed at DM0 - D, the burst is smeared
from t0 over k*D samples (towards later t for D > 0, earlier for D < 0, the highest
channel staying at t0), so the candidate's window [t, t + w) must reach that span
widened by W + 4 samples, and its S/N must not exceed what the smeared burst can give
there: 1.2 * S/N0 * sqrt(W / sqrt(W^2 + (k*D)^2)) + 2 (smearing adds in quadrature to
the width; the margin covers the noise).  Recall counts matches; false alarms count every
candidate that matches no burst, and are split into side lobes and the rest (off track).
The side-lobe allowance is a hand-set choice, parity unpinned: it only splits the count.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import synth
from . import workloads as W

DISPERSION_CONSTANT = 4148.8064239   # MHz^2 pc^-1 cm^3 s, Eq. (1)

# Optimisation parameters of the ranker path before the CNN: every NMS candidate is its
# own core point (min_pts 1), so DBSCAN only merges neighbours into one representative;
# no S/N cut; the DM and width cuts stay; the anti-coincidence filter is left for after
# the CNN (it must count only the candidates the CNN keeps: noise peaks in every beam
# would otherwise make every arrival time look coincident).
RANKER_OPT = {"min_pts": 1, "snr_min": 0.0, "coinc_min_beams": 1 << 30}


def band_key(pd) -> str:
    """Name of a plan's band: its edge frequencies and channel count, e.g. 550-750MHz/4096ch."""
    half = abs(pd["foff"]) / 2.0
    f = [pd["fch1"], pd["fch1"] + (pd["nchans"] - 1) * pd["foff"]]
    return f"{min(f) - half:.0f}-{max(f) + half:.0f}MHz/{pd['nchans']}ch"


def load_operating_point(path):
    """Per-band logit thresholds of the ranker path ({band_key: threshold}), or {}."""
    import json
    import os
    if not path or not os.path.exists(path):
        return {}
    return {k: float(v) for k, v in json.load(open(path))["logit_threshold"].items()}


def beam_thresholds(pds, operating_point, default=0.0):
    """Logit threshold of each beam: its band's operating point, else `default` (0: the
    probability 0.5 the paper's classifier keeps)."""
    return np.array([operating_point.get(band_key(pd), default) for pd in pds], np.float32)


def _by_key(c: np.ndarray) -> np.ndarray:
    return c[np.lexsort((c["t_sample"], c["dm_index"], c["beam"]))] if c.size else c


def ranker_path(spl, cands, tsamp, n_beams, score_fn, threshold=0.0, max_scored=None):
    """Optimisation with RANKER_OPT, the CNN (score_fn: records -> logits), then the
    anti-coincidence filter on the records whose logit is >= threshold (a number, or one
    per beam).  Returns (final records, scored records, their logits).

    The plain path is the fallback: when the ranker has no weights (score_fn raises
    SPL_E_NO_WEIGHTS) every beam takes it; when the representatives number more than
    max_scored, beams are scored in beam order while their representatives fit, and each
    beam that does not fit takes the plain path on its own candidates (density test and
    every cut), its survivors joining the CNN's before the anti-coincidence filter."""
    surv = spl.optimise_plain(cands, tsamp, n_beams, **RANKER_OPT)
    plain_beams = np.zeros(n_beams, bool)
    if max_scored is not None and surv.size > max_scored:
        counts = np.bincount(surv["beam"], minlength=n_beams)
        budget = int(max_scored)
        for b in range(n_beams):
            if counts[b] <= budget:
                budget -= int(counts[b])
            else:
                plain_beams[b] = True
    scored = surv[~plain_beams[surv["beam"]]] if surv.size else surv
    lg = np.zeros(0, np.float32)
    if scored.size:
        try:
            lg = np.asarray(score_fn(scored), np.float32)
        except spl.SplError as e:
            if e.status != spl.SPL_E_NO_WEIGHTS:
                raise
            return spl.optimise_plain(cands, tsamp, n_beams), scored[:0], lg
    thr = np.asarray(threshold, np.float32)
    if scored.size:
        kept = scored[lg >= (thr[scored["beam"]] if thr.ndim else thr)]
    else:
        kept = scored
    if plain_beams.any():
        raw = cands[plain_beams[cands["beam"]]]
        pf = spl.optimise_plain(raw, tsamp, n_beams, coinc_min_beams=1 << 30)
        kept = _by_key(np.concatenate([kept, pf]))
    final = spl.anti_coincidence(kept, tsamp, n_beams)
    return final, scored, lg


def band_delay_per_dm(pd) -> float:
    """Delay in samples across the band (outer channel centres) per unit DM."""
    f = [pd["fch1"], pd["fch1"] + (pd["nchans"] - 1) * pd["foff"]]
    f_lo, f_hi = min(f), max(f)
    return DISPERSION_CONSTANT * (1.0 / (f_lo * f_lo) - 1.0 / (f_hi * f_hi)) / pd["tsamp"]


def _pulse_arrays(pulses):
    return (np.array([p.t0 for p in pulses], np.float64), np.array([p.dm for p in pulses], np.float64),
            np.array([p.fwhm for p in pulses], np.float64), np.array([p.snr for p in pulses], np.float64))


def match(cands: np.ndarray, pulses_by_beam, pds) -> np.ndarray:
    """Index (within its beam's list) of the burst each candidate matches, or -1; the
    closest burst in time wins when several qualify (the earlier in the list on a tie)."""
    out = np.full(cands.size, -1, np.int64)
    if cands.size == 0:
        return out
    beams = cands["beam"].astype(np.int64)
    for b in np.unique(beams):
        ps = pulses_by_beam[b]
        if not ps:
            continue
        sel = np.nonzero(beams == b)[0]
        c = cands[sel]
        pd = pds[b]
        k = band_delay_per_dm(pd)
        dm_step = pd["dm_ranges"][0][1]
        t0, dm0, fw, _ = _pulse_arrays(ps)
        tol = np.maximum(c["width"].astype(np.float64)[:, None], fw[None, :]) + 4.0
        dt = np.abs(c["t_sample"].astype(np.float64)[:, None] - t0[None, :])
        ok = (dt <= tol) & (np.abs(c["dm"].astype(np.float64)[:, None] - dm0[None, :]) <= tol / k + dm_step)
        dt = np.where(ok, dt, np.inf)
        j = np.argmin(dt, axis=1)
        out[sel] = np.where(np.isfinite(dt[np.arange(sel.size), j]), j, -1)
    return out


def on_track(cands: np.ndarray, pulses_by_beam, pds) -> np.ndarray:
    """True for candidates on the dispersion track of an injected burst of their beam."""
    out = np.zeros(cands.size, bool)
    if cands.size == 0:
        return out
    beams = cands["beam"].astype(np.int64)
    for b in np.unique(beams):
        ps = pulses_by_beam[b]
        if not ps:
            continue
        sel = np.nonzero(beams == b)[0]
        c = cands[sel]
        k = band_delay_per_dm(pds[b])
        t0, dm0, fw, snr0 = _pulse_arrays(ps)
        t = c["t_sample"].astype(np.float64)[:, None]
        w = c["width"].astype(np.float64)[:, None]
        span = k * (dm0[None, :] - c["dm"].astype(np.float64)[:, None])
        lo = t0[None, :] + np.minimum(0.0, span) - fw[None, :] - 4.0
        hi = t0[None, :] + np.maximum(0.0, span) + fw[None, :] + 4.0
        snr_max = 1.2 * snr0[None, :] * np.sqrt(fw[None, :] / np.hypot(fw[None, :], span)) + 2.0
        hit = (t + w >= lo) & (t <= hi) & (c["snr"].astype(np.float64)[:, None] <= snr_max)
        out[sel] = hit.any(axis=1)
    return out


def recall_and_false_alarms(final: np.ndarray, pulses_by_beam, pds, context_by_beam=None) -> dict:
    """Recall of the injected bursts of the block and its false alarms.  false_alarms =
    final candidates matching no burst (the measurement's definition); it splits into
    side_lobes (on a burst's dispersion track, see on_track) and off_track.
    context_by_beam (optional): bursts of neighbouring blocks of a stream (t0 relative
    to this block): a candidate matching one is not a false alarm, and they count
    neither as injected nor as recovered."""
    m = match(final, pulses_by_beam, pds)
    unmatched = m < 0
    every = pulses_by_beam
    if context_by_beam is not None:
        unmatched &= match(final, context_by_beam, pds) < 0
        every = [list(a) + list(b) for a, b in zip(pulses_by_beam, context_by_beam)]
    tr = on_track(final, every, pds)
    n_inj = sum(len(p) for p in pulses_by_beam)
    found = set()
    for i, j in enumerate(m):
        if j >= 0:
            found.add((int(final[i]["beam"]), int(j)))
    return {"injected": n_inj, "recovered": len(found), "recall": len(found) / max(1, n_inj),
            "false_alarms": int(np.sum(unmatched)), "side_lobes": int(np.sum(unmatched & tr)),
            "off_track": int(np.sum(unmatched & ~tr)), "kept": int(final.size)}


def burst_batch(pds, seed: int, n_pulses: int = 8, dm_lo: float = 20.0, dm_hi: float = 2000.0,
                fwhm_hi: float = 128.0, snr_lo: float = 6.0, snr_hi: float = 30.0, rfi_frac: float = 0.02,
                zero_dm_rate: float = 0.2, n_in=None, device=None):
    """Blocks of a batch of beams with injected bursts (DM uniform, FWHM log-uniform,
    S/N uniform), 2% RFI channels per beam, and zero-DM impulsive RFI common to every
    beam of the batch (terrestrial interference enters all beams at once).  With a
    torch device the blocks are made there (synth.make_block_torch: same recipe, torch's
    noise) as uint8 tensors [nch][pitch]; else numpy arrays [nch][n_in]."""
    rng_common = np.random.default_rng([seed, 777])
    n_in = n_in or [None] * len(pds)
    zd = synth.zero_dm_bursts(rng_common, max(n_in), pds[0]["tsamp"], zero_dm_rate) if zero_dm_rate > 0 else ()
    blocks, pulses = [], []
    for b, pd in enumerate(pds):
        rng = np.random.default_rng([seed, b, 4242])
        hi = min(dm_hi, W.dm_max(pd) * 0.98)
        ps = synth.pulses_evenly(rng, n_pulses, pd["n_out"], dm_lo, hi, 1.0, fwhm_hi, snr_lo, snr_hi)
        rfi = synth.rfi_channels(rng, pd["nchans"], rfi_frac) if rfi_frac > 0 else None
        zd_b = [z for z in zd if z[0] < n_in[b]]
        spec = W.block_spec(pd, n_in[b], ps, rfi, zd_b)
        if device is not None:
            blocks.append(synth.make_block_torch(spec, seed, b, pd["widths"], device=device))
        else:
            blocks.append(synth.make_block(spec, seed, b, pd["widths"])[:, :n_in[b]])
        pulses.append(ps)
    return blocks, pulses


class Stage:
    """Search + optimisation + optional ranker for a fixed batch of plans."""

    def __init__(self, spl, pds, cand_capacity=1 << 20, mode=0, fine_keep=None, hit_capacity=0):
        import torch
        self.spl, self.pds = spl, pds
        self.fine_keep = fine_keep   # None: DM-time plane on the search grid; else fine-DM plane
        self.plans = [spl.Plan.from_dict(pd) for pd in pds]
        self.n_in = [p.info["n_in"] for p in self.plans]
        self.mode = mode
        self.batch = spl.Batch(self.plans, mode=mode, hit_capacity=hit_capacity)
        self.cands = spl.new_candidates(cand_capacity)
        self.stats = torch.zeros(spl.STATS_WORDS, dtype=torch.int64, device="cuda")
        self.tsamp = np.array([pd["tsamp"] for pd in pds], np.float64)
        self.regrown = 0

    def search(self, blocks):
        """Search numpy blocks [nch][n_in] (uploaded) or device blocks [nch][pitch].  A run
        whose hits or candidates exceed the capacities (the statistics carry the true
        counts) is searched again with capacities that hold them."""
        import torch
        dev = [x if isinstance(x, torch.Tensor) else self.spl.upload_block(x) for x in blocks]
        self.batch.run(dev, self.cands, self.stats)
        torch.cuda.synchronize()
        st = self.spl.stats_dict(self.stats)
        if st["hit_overflow"] or st["cand_overflow"]:
            def room(n):
                return 1 << max(20, int(math.ceil(math.log2(max(2, 1.25 * n)))))
            self.batch = self.spl.Batch(self.plans, mode=self.mode, hit_capacity=room(st["n_hits"]))
            if st["cand_overflow"]:
                self.cands = self.spl.new_candidates(room(st["n_candidates"]))
            self.regrown += 1
            self.batch.run(dev, self.cands, self.stats)
            torch.cuda.synchronize()
            st = self.spl.stats_dict(self.stats)
            assert not (st["hit_overflow"] or st["cand_overflow"]), st
        self._dev_blocks = dev   # the snippets read these blocks
        return self.spl.candidates_to_numpy(self.cands, self.stats)

    def snippets(self, recs: np.ndarray):
        import torch
        dev = torch.from_numpy(np.ascontiguousarray(recs).view(np.int32).reshape(-1, 8).copy()).cuda()
        return self.spl.snippets(self.batch, dev, fine_keep=self.fine_keep)

    def plain(self, cands, **kw):
        return self.spl.optimise_plain(cands, self.tsamp, len(self.pds), **kw)

    def ranked(self, cands, ranker):
        """The ranker path: the optimisation stage with the CNN in place of the density
        test and the S/N cut, the CNN keeping probability >= 0.5 before the
        anti-coincidence filter.  Returns (final, scored records, logits)."""
        return ranker_path(self.spl, cands, self.tsamp, len(self.pds),
                           lambda recs: ranker.score(self.snippets(recs)).cpu().numpy())


def mine(spl, pds, n_batches, seed0, neg_ratio=1.0, log=print, fine_keep=None, per_burst=0, device=None,
         mode=0, **burst_kw):
    """Labelled snippets (device int16 [n][2][64][256], float32 labels) from the NMS
    candidates of searched blocks: candidates matching a burst are positives (all of
    them, or per_burst > 0: the strongest and per_burst - 1 others drawn at random per
    burst), a random subset of the unmatched ones (neg_ratio per positive) negatives.
    device: make the blocks there (see burst_batch).  Also returns the number of bursts
    injected and of bursts with at least one positive."""
    import torch
    st = Stage(spl, pds, fine_keep=fine_keep, mode=mode, hit_capacity=1 << 26)
    xs, ys = [], []
    n_bursts = n_found = 0
    t_log = time.time()
    for i in range(n_batches):
        t0 = time.time()
        blocks, pulses = burst_batch(pds, seed0 + i, n_in=st.n_in, device=device, **burst_kw)
        t1 = time.time()
        cands = st.search(blocks)
        m = match(cands, pulses, pds)
        rng = np.random.default_rng(seed0 + i)
        n_bursts += sum(len(p) for p in pulses)
        pos = np.nonzero(m >= 0)[0]
        if per_burst > 0 and pos.size:
            key = cands["beam"][pos].astype(np.int64) * 1_000_003 + m[pos]
            keep = []
            for k_ in np.unique(key):
                grp = pos[key == k_]
                best = grp[np.argmax(cands["snr"][grp])]
                rest = grp[grp != best]
                keep.append(best)
                if per_burst > 1 and rest.size:
                    keep.extend(rng.choice(rest, size=min(rest.size, per_burst - 1), replace=False))
            pos = np.sort(np.array(keep, np.int64))
        n_found += int(np.unique(cands["beam"][pos].astype(np.int64) * 1_000_003 + m[pos]).size) if pos.size else 0
        neg = np.nonzero(m < 0)[0]
        k = min(neg.size, int(math.ceil(neg_ratio * max(1, pos.size))))
        neg = rng.choice(neg, size=k, replace=False) if k else neg[:0]
        sel = np.concatenate([pos, neg])
        if sel.size:
            xs.append(st.snippets(cands[sel]).clone())
            ys.append(np.concatenate([np.ones(pos.size, np.float32), np.zeros(neg.size, np.float32)]))
        del blocks
        if i + 1 == n_batches or time.time() - t_log > 20:
            t_log = time.time()
            log(f"mine batch {i + 1}/{n_batches}: {cands.size} candidates, {pos.size} positive, "
                f"{neg.size} negative; bursts {n_found}/{n_bursts} found so far "
                f"(gen {t1 - t0:.2f}s, search+snip {time.time() - t1:.2f}s)")
    x = torch.cat(xs) if xs else torch.zeros((0, 2, 64, 256), dtype=torch.int16, device="cuda")
    y = np.concatenate(ys) if ys else np.zeros(0, np.float32)
    if st.regrown:
        log(f"capacities regrown {st.regrown} times")
    return x, y, n_bursts, n_found


def train(ranker, x, y, epochs=20, batch=256, lr=1e-3, val_frac=0.1, seed=0, log=print):
    """Adam on shuffled minibatches; the weights of the epoch with the best validation
    accuracy are kept.  Returns the history of (epoch, train loss, val acc)."""
    import torch
    n = x.shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    n_val = int(round(val_frac * n))
    val, tr = perm[:n_val], perm[n_val:]
    yd = torch.from_numpy(y).cuda()
    hist = []
    best_acc, best_w = -1.0, None
    for ep in range(epochs):
        order = rng.permutation(tr)
        tot, cnt = 0.0, 0
        for i in range(0, order.size, batch):
            idx = torch.from_numpy(order[i:i + batch]).cuda()
            loss = ranker.train_step(x.index_select(0, idx), yd.index_select(0, idx), lr)
            tot += float(loss.item()) * idx.numel()
            cnt += idx.numel()
        acc = float("nan")
        if n_val:
            vi = torch.from_numpy(val).cuda()
            lg = ranker.score(x.index_select(0, vi)).cpu().numpy()
            acc = float(np.mean((lg >= 0) == (y[val] >= 0.5)))
        hist.append((ep, tot / max(1, cnt), acc))
        log(f"epoch {ep + 1}/{epochs}: train loss {tot / max(1, cnt):.4f}, val acc {acc:.4f}")
        if n_val and acc > best_acc:
            best_acc, best_w = acc, ranker.get_weights()
    if best_w is not None:
        ranker.set_weights(best_w)
    return hist


def evaluate(spl, pds, ranker, n_batches, seed0, log=print, fine_keep=None, device=None, mode=0, **burst_kw):
    """Recall and false alarms of the plain path and of the ranker path on fresh blocks
    (made on `device` when given, see burst_batch)."""
    import torch
    st = Stage(spl, pds, fine_keep=fine_keep, mode=mode, hit_capacity=1 << 26)
    plain_all, rank_all, pulses_all, cand_all, scored_all, logit_all = [], [], [], 0, [], []
    t_rank = 0.0
    for i in range(n_batches):
        blocks, pulses = burst_batch(pds, seed0 + i, n_in=st.n_in, device=device, **burst_kw)
        cands = st.search(blocks)
        del blocks
        cand_all += cands.size
        fp = st.plain(cands)
        t0 = time.time()
        if ranker is not None:
            fr, surv, lg = st.ranked(cands, ranker)
        else:
            surv, lg, fr = fp.copy(), np.zeros(fp.size, np.float32), fp.copy()
        torch.cuda.synchronize()
        t_rank += time.time() - t0
        off = len(pulses_all)
        for arr in (fp, fr, surv):
            arr["beam"] += off
        plain_all.append(fp)
        rank_all.append(fr)
        scored_all.append(surv)
        logit_all.append(lg)
        pulses_all.extend(pulses)
        log(f"eval batch {i + 1}/{n_batches}: {cands.size} candidates, plain keeps {fp.size}, ranker keeps {fr.size}")
    pds_all = [pds[b % len(pds)] for b in range(len(pulses_all))]
    plain = np.concatenate(plain_all)
    rank = np.concatenate(rank_all)
    res = {"beam_blocks": len(pulses_all), "candidates": cand_all,
           "plain": recall_and_false_alarms(plain, pulses_all, pds_all),
           "ranker": recall_and_false_alarms(rank, pulses_all, pds_all),
           "ranker_stage_s": t_rank}
    for k in ("plain", "ranker"):
        res[k]["false_alarms_per_beam_block"] = res[k]["false_alarms"] / max(1, len(pulses_all))
    scored = np.concatenate(scored_all)
    logits = np.concatenate(logit_all)
    res["ranker_at_plain_false_alarms"] = at_false_alarms(spl, scored, logits, pulses_all, pds_all,
                                                          res["plain"]["false_alarms"], len(pds))
    return res


def at_false_alarms(spl, scored, logits, pulses_by_beam, pds, target, beams_per_batch):
    """The ranker path at a false-alarm budget: the lowest logit threshold whose final
    list (records with logit >= threshold, then the anti-coincidence filter within each
    batch of beams_per_batch beams) holds at most `target` candidates matching no burst.
    Returns its recall, false alarms and threshold (None if no threshold qualifies)."""
    m = match(scored, pulses_by_beam, pds)
    fa_mask = m < 0
    key = {(int(r["beam"]), int(r["dm_index"]), int(r["t_sample"])): i for i, r in enumerate(scored)}
    tsamp_all = np.array([pd["tsamp"] for pd in pds], np.float64)
    n_beams = len(pulses_by_beam)
    n_inj = sum(len(p) for p in pulses_by_beam)
    taus = np.unique(np.concatenate([np.quantile(logits, np.linspace(0.0, 1.0, 401)) if logits.size else [],
                                     [np.inf]]))
    nbb = beams_per_batch

    def filtered(sel):
        out = []
        for b0 in range(0, n_beams, nbb):
            part = sel[(sel["beam"] >= b0) & (sel["beam"] < b0 + nbb)].copy()
            part["beam"] -= b0
            f = spl.anti_coincidence(part, tsamp_all[b0:b0 + nbb], min(nbb, n_beams - b0))
            f["beam"] += b0
            out.append(f)
        return np.concatenate(out) if out else sel[:0]

    for tau in taus:
        fin = filtered(scored[logits >= tau]) if np.isfinite(tau) else scored[:0]
        idx = np.array([key[(int(r["beam"]), int(r["dm_index"]), int(r["t_sample"]))] for r in fin], np.int64)
        fa = int(np.sum(fa_mask[idx])) if idx.size else 0
        if fa <= target:
            found = {(int(scored[i]["beam"]), int(m[i])) for i in idx if m[i] >= 0}
            return {"threshold_logit": float(tau), "recall": len(found) / max(1, n_inj), "recovered": len(found),
                    "false_alarms": fa, "false_alarms_per_beam_block": fa / max(1, n_beams),
                    "kept": int(idx.size)}
    return None


def initial_weights(seed: int = 0) -> np.ndarray:
    """He-uniform weights (limit sqrt(6 / fan_in)), zero biases, in the parameter order
    of the ranker ABI, float32."""
    rng = np.random.default_rng(seed)
    parts = []
    cin = (2, 32, 32, 32)
    for k in range(4):
        fan = cin[k] * 9
        parts.append(rng.uniform(-math.sqrt(6.0 / fan), math.sqrt(6.0 / fan), size=32 * cin[k] * 9))
        parts.append(np.zeros(32))
    parts.append(rng.uniform(-math.sqrt(6.0 / 2048), math.sqrt(6.0 / 2048), size=64 * 2048))
    parts.append(np.zeros(64))
    parts.append(rng.uniform(-math.sqrt(6.0 / 64), math.sqrt(6.0 / 64), size=64))
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float32)
