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
the width; the margin covers the noise).  Recall counts matches; false alarms count
candidates that neither match nor lie on a track.
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


def ranker_path(spl, cands, tsamp, n_beams, score_fn, threshold=0.0):
    """Optimisation with RANKER_OPT, the CNN (score_fn: records -> logits), then the
    anti-coincidence filter on the records whose logit is >= threshold.  Returns
    (final records, scored records, their logits)."""
    surv = spl.optimise_plain(cands, tsamp, n_beams, **RANKER_OPT)
    if surv.size == 0:
        return surv, surv, np.zeros(0, np.float32)
    lg = score_fn(surv)
    final = spl.anti_coincidence(surv[lg >= threshold], tsamp, n_beams)
    return final, surv, lg


def band_delay_per_dm(pd) -> float:
    """Delay in samples across the band (outer channel centres) per unit DM."""
    f = [pd["fch1"], pd["fch1"] + (pd["nchans"] - 1) * pd["foff"]]
    f_lo, f_hi = min(f), max(f)
    return DISPERSION_CONSTANT * (1.0 / (f_lo * f_lo) - 1.0 / (f_hi * f_hi)) / pd["tsamp"]


def match(cands: np.ndarray, pulses_by_beam, pds) -> np.ndarray:
    """Index (within its beam's list) of the burst each candidate matches, or -1; the
    closest burst in time wins when several qualify."""
    out = np.full(cands.size, -1, np.int64)
    for i, c in enumerate(cands):
        b = int(c["beam"])
        pd = pds[b]
        k = band_delay_per_dm(pd)
        dm_step = pd["dm_ranges"][0][1]
        best, best_dt = -1, None
        for j, p in enumerate(pulses_by_beam[b]):
            tol = max(float(c["width"]), p.fwhm) + 4.0
            dt = abs(float(c["t_sample"]) - p.t0)
            if dt <= tol and abs(float(c["dm"]) - p.dm) <= tol / k + dm_step:
                if best_dt is None or dt < best_dt:
                    best, best_dt = j, dt
        out[i] = best
    return out


def on_track(cands: np.ndarray, pulses_by_beam, pds) -> np.ndarray:
    """True for candidates on the dispersion track of an injected burst of their beam."""
    out = np.zeros(cands.size, bool)
    for i, c in enumerate(cands):
        b = int(c["beam"])
        k = band_delay_per_dm(pds[b])
        t, w = float(c["t_sample"]), float(c["width"])
        for p in pulses_by_beam[b]:
            span = k * (p.dm - float(c["dm"]))
            lo = p.t0 + min(0.0, span) - p.fwhm - 4.0
            hi = p.t0 + max(0.0, span) + p.fwhm + 4.0
            snr_max = 1.2 * p.snr * math.sqrt(p.fwhm / math.hypot(p.fwhm, span)) + 2.0
            if t + w >= lo and t <= hi and float(c["snr"]) <= snr_max:
                out[i] = True
                break
    return out


def recall_and_false_alarms(final: np.ndarray, pulses_by_beam, pds) -> dict:
    m = match(final, pulses_by_beam, pds)
    tr = on_track(final, pulses_by_beam, pds)
    n_inj = sum(len(p) for p in pulses_by_beam)
    found = set()
    for i, j in enumerate(m):
        if j >= 0:
            found.add((int(final[i]["beam"]), int(j)))
    return {"injected": n_inj, "recovered": len(found), "recall": len(found) / max(1, n_inj),
            "false_alarms": int(np.sum((m < 0) & ~tr)), "side_lobes": int(np.sum((m < 0) & tr)),
            "kept": int(final.size)}


def burst_batch(pds, seed: int, n_pulses: int = 8, dm_lo: float = 20.0, dm_hi: float = 2000.0,
                fwhm_hi: float = 128.0, snr_lo: float = 6.0, snr_hi: float = 30.0, rfi_frac: float = 0.02,
                zero_dm_rate: float = 0.2, n_in=None):
    """Blocks of a batch of beams with injected bursts (DM uniform, FWHM log-uniform,
    S/N uniform), 2% RFI channels per beam, and zero-DM impulsive RFI common to every
    beam of the batch (terrestrial interference enters all beams at once)."""
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
        blocks.append(synth.make_block(spec, seed, b, pd["widths"])[:, :n_in[b]])
        pulses.append(ps)
    return blocks, pulses


class Stage:
    """Search + optimisation + optional ranker for a fixed batch of plans."""

    def __init__(self, spl, pds, cand_capacity=1 << 20, mode=0, fine_keep=None):
        import torch
        self.spl, self.pds = spl, pds
        self.fine_keep = fine_keep   # None: DM-time plane on the search grid; else fine-DM plane
        self.plans = [spl.Plan.from_dict(pd) for pd in pds]
        self.n_in = [p.info["n_in"] for p in self.plans]
        self.batch = spl.Batch(self.plans, mode=mode)
        self.cands = spl.new_candidates(cand_capacity)
        self.stats = torch.zeros(spl.STATS_WORDS, dtype=torch.int64, device="cuda")
        self.tsamp = np.array([pd["tsamp"] for pd in pds], np.float64)

    def search(self, blocks_np):
        import torch
        dev = [self.spl.upload_block(x) for x in blocks_np]
        self.batch.run(dev, self.cands, self.stats)
        torch.cuda.synchronize()
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


def mine(spl, pds, n_batches, seed0, neg_ratio=1.0, log=print, fine_keep=None, **burst_kw):
    """Labelled snippets (device int16 [n][2][64][256], float32 labels) from the NMS
    candidates of searched blocks: matched candidates are positives, a random subset
    of the unmatched ones (neg_ratio per positive) negatives."""
    import torch
    st = Stage(spl, pds, fine_keep=fine_keep)
    xs, ys = [], []
    for i in range(n_batches):
        t0 = time.time()
        blocks, pulses = burst_batch(pds, seed0 + i, n_in=st.n_in, **burst_kw)
        t1 = time.time()
        cands = st.search(blocks)
        del blocks
        m = match(cands, pulses, pds)
        pos = np.nonzero(m >= 0)[0]
        neg = np.nonzero(m < 0)[0]
        rng = np.random.default_rng(seed0 + i)
        k = min(neg.size, int(math.ceil(neg_ratio * max(1, pos.size))))
        neg = rng.choice(neg, size=k, replace=False) if k else neg[:0]
        sel = np.concatenate([pos, neg])
        if sel.size:
            xs.append(st.snippets(cands[sel]).clone())
            ys.append(np.concatenate([np.ones(pos.size, np.float32), np.zeros(neg.size, np.float32)]))
        log(f"mine batch {i + 1}/{n_batches}: {cands.size} candidates, {pos.size} positive, "
            f"{neg.size} negative (gen {t1 - t0:.1f}s, search+snip {time.time() - t1:.1f}s)")
    x = torch.cat(xs) if xs else torch.zeros((0, 2, 64, 256), dtype=torch.int16, device="cuda")
    y = np.concatenate(ys) if ys else np.zeros(0, np.float32)
    return x, y


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


def evaluate(spl, pds, ranker, n_batches, seed0, log=print, fine_keep=None, **burst_kw):
    """Recall and false alarms of the plain path and of the ranker path on fresh blocks."""
    import torch
    st = Stage(spl, pds, fine_keep=fine_keep)
    plain_all, rank_all, pulses_all, cand_all, scored_all, logit_all = [], [], [], 0, [], []
    t_rank = 0.0
    for i in range(n_batches):
        blocks, pulses = burst_batch(pds, seed0 + i, n_in=st.n_in, **burst_kw)
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
    # the ranker at the plain path's false-alarm rate: the lowest logit threshold whose
    # false alarms do not exceed the plain path's
    scored = np.concatenate(scored_all)
    logits = np.concatenate(logit_all)
    target = res["plain"]["false_alarms"]
    m = match(scored, pulses_all, pds_all)
    fa_mask = (m < 0) & ~on_track(scored, pulses_all, pds_all)
    key = {(int(r["beam"]), int(r["dm_index"]), int(r["t_sample"])): i for i, r in enumerate(scored)}
    tsamp_all = np.array([pd["tsamp"] for pd in pds_all], np.float64)
    n_inj = res["plain"]["injected"]
    best = None
    taus = np.unique(np.concatenate([np.quantile(logits, np.linspace(0.0, 1.0, 401)) if logits.size else [],
                                     [np.inf]]))
    nbb = len(pds)   # beams per batch: the filter runs within each batch

    def filtered(sel):
        out = []
        for b0 in range(0, len(pulses_all), nbb):
            part = sel[(sel["beam"] >= b0) & (sel["beam"] < b0 + nbb)].copy()
            part["beam"] -= b0
            f = spl.anti_coincidence(part, tsamp_all[b0:b0 + nbb], nbb)
            f["beam"] += b0
            out.append(f)
        return np.concatenate(out) if out else sel[:0]

    for tau in taus:
        fin = filtered(scored[logits >= tau]) if np.isfinite(tau) else scored[:0]
        idx = np.array([key[(int(r["beam"]), int(r["dm_index"]), int(r["t_sample"]))] for r in fin], np.int64)
        fa = int(np.sum(fa_mask[idx])) if idx.size else 0
        if fa <= target:
            found = {(int(scored[i]["beam"]), int(m[i])) for i in idx if m[i] >= 0}
            best = {"threshold_logit": float(tau), "recall": len(found) / max(1, n_inj), "recovered": len(found),
                    "false_alarms": fa, "false_alarms_per_beam_block": fa / max(1, len(pulses_all)),
                    "kept": int(idx.size)}
            break
    res["ranker_at_plain_false_alarms"] = best
    return res


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
