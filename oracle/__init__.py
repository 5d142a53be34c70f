"""CPU oracle for the SPOTLIGHT single-pulse search hot path.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product path (the HIP library and its
Python binding) never imports, calls or links anything in this directory.

The arithmetic lives in ``oracle.c`` (plain loops, IEEE binary64, no FMA
contraction) and in the numpy code below (candidate assembly, the plain
candidate-optimisation path, snippet extraction and the CNN ranker in float64).
Nothing here is shared with the HIP path.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# SPL_ORACLE_LIBRARY names another build of oracle.c (the sanitizer test's)
_LIB_PATH = os.environ.get("SPL_ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
_lib = None

# Candidate record, field for field the 32-byte record of the search output.
CAND_DTYPE = np.dtype([("beam", "<i4"), ("dm_index", "<i4"), ("t_sample", "<i4"),
                       ("width", "<i4"), ("boxcar_sum", "<i4"), ("snr", "<f4"),
                       ("dm", "<f4"), ("flags", "<u4")])


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain -O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_sanitized(out: str) -> str:
    """Compile oracle.c with clang's AddressSanitizer and UndefinedBehaviorSanitizer
    (no OpenMP) into `out`, for runs with clang's ASan runtime preloaded."""
    subprocess.check_call(["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", _SRC, "-o", out, "-lm"])
    return out


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.orc_delay_table.argtypes = [i32, f64, f64, f64, i32, P, P]
        lib.orc_delay_table.restype = i64
        lib.orc_dedisperse.argtypes = [P, i64, i32, P, i32, i32, P]
        lib.orc_dedisperse.restype = None
        lib.orc_moments.argtypes = [P, i32, i32, i32, i32, P, P, P]
        lib.orc_moments.restype = None
        lib.orc_mu_sigma.argtypes = [i64, i64, i64, P, P]
        lib.orc_mu_sigma.restype = None
        lib.orc_snr.argtypes = [i64, i32, f64, f64]
        lib.orc_snr.restype = f64
        lib.orc_search.argtypes = [P, i32, i32, i32, i32, P, i32, f64, P, P, P, P, P]
        lib.orc_search.restype = i64
        lib.orc_nms.argtypes = [P, P, P, i64, i32, i32, i32, i32, P, P]
        lib.orc_nms.restype = i32
        lib.orc_dbscan.argtypes = [P, P, i64, f64, i32, P]
        lib.orc_dbscan.restype = i32
        lib.orc_num_threads.argtypes = []
        lib.orc_num_threads.restype = i32
        lib.orc_set_threads.argtypes = [i32]
        lib.orc_set_threads.restype = None
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    _load().orc_set_threads(int(n))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


DISPERSION_CONSTANT = 4148.8064239  # MHz^2 pc^-1 cm^3 s, Eq. (1)


# --------------------------------------------------------------------------
# Plan quantities
# --------------------------------------------------------------------------
def dm_trials(ranges) -> np.ndarray:
    """DM_d = dm_start + d*dm_step per sub-range, sub-ranges concatenated
    (the dedispersion plan of the dedispersion section)."""
    out = []
    for start, step, n in ranges:
        out.extend(float(start) + float(d) * float(step) for d in range(int(n)))
    return np.asarray(out, dtype=np.float64)


def snr_kept(ddm: float, width_ms: float, bw_mhz: float, nu_ghz: float) -> float:
    """S/N fraction kept by a Gaussian pulse of FWHM width_ms dedispersed ddm off its DM:
    (sqrt(pi)/2) erf(z)/z with z = 6.91e-3 ddm B / (W nu^3) (Eq. snrloss, Eq. zetadef)."""
    z = 6.91e-3 * ddm * bw_mhz / (width_ms * (nu_ghz * nu_ghz * nu_ghz))
    if z == 0.0:
        return 1.0
    return (math.sqrt(math.pi) / 2.0) * math.erf(z) / z


def smearing_ranges(nch: int, fch1: float, foff: float, tsamp: float, dm_min: float, dm_max: float,
                    max_loss: float, w_min_s: float = 0.0) -> list:
    """DM sub-ranges (start, step, n) whose step keeps a pulse half a step off above
    1 - max_loss of its S/N, for the narrowest pulse a trial at DM can see: FWHM
    sqrt(w_min^2 + tsamp^2 + t_chan(DM)^2), t_chan = 8.3e-3 DM |foff| / nu_lo^3 ms (the
    smearing within one channel at the lowest channel centre; Cordes & McLaughlin).
    The plan is the dedispersion section's: sub-ranges of growing spacing.  Steps are
    powers of two; a sub-range ends at the first of its trials (not its first) where
    twice its step is allowed, and trials run to the first one >= dm_max."""
    edge = [fch1, fch1 + (nch - 1) * foff]
    lo, hi = min(edge), max(edge)
    tsamp_ms, w_ms, chan = tsamp * 1e3, w_min_s * 1e3, abs(foff)
    nu_lo = lo / 1e3
    nu_c = (0.5 * (lo + hi)) / 1e3
    bw = nch * abs(foff)

    def ok(step, dm):
        tc = 8.3e-3 * dm * chan / (nu_lo * nu_lo * nu_lo)
        width = math.sqrt(w_ms * w_ms + tsamp_ms * tsamp_ms + tc * tc)
        return snr_kept(0.5 * step, width, bw, nu_c) >= 1.0 - max_loss

    e = 20
    while not ok(math.ldexp(1.0, e), dm_min):
        e -= 1
    ranges = []
    start, step, i = dm_min, math.ldexp(1.0, e), 0
    while True:
        dm = start + i * step
        if dm >= dm_max:
            ranges.append((start, step, i + 1))
            return ranges
        if i >= 1 and ok(2.0 * step, dm):
            ranges.append((start, step, i))
            start, step, i = dm, 2.0 * step, 0
            if start >= dm_max:
                ranges.append((start, step, 1))
                return ranges
        i += 1


def delay_table(nch: int, fch1: float, foff: float, tsamp: float, dms) -> tuple[np.ndarray, int]:
    """Integer delays [ndm][nch] (Eq. (1), nearest, ties away from zero) and the
    count of half-integer tie risks."""
    dms = np.ascontiguousarray(dms, dtype=np.float64)
    out = np.empty((dms.size, nch), dtype=np.int64)
    ties = _load().orc_delay_table(nch, fch1, foff, tsamp, dms.size, _p(dms), _p(out))
    return out, int(ties)


def sizes(delays: np.ndarray, n_out: int, widths) -> dict:
    """n_dd = n_out + w_max - 1 dedispersed samples; n_in = n_dd + s_max input
    samples per block (the overlap tail carried by the block)."""
    s_max = int(delays.max()) if delays.size else 0
    n_dd = int(n_out) + int(max(widths)) - 1
    return {"s_max": s_max, "n_dd": n_dd, "n_in": n_dd + s_max}


# --------------------------------------------------------------------------
# Search stages
# --------------------------------------------------------------------------
def corner_turn(x_tc: np.ndarray) -> np.ndarray:
    """Channel-major copy of a time-major block: out[c][t] = x_tc[t][c] (the search
    reads one row per channel; filterbank data arrive one spectrum per sample)."""
    x_tc = np.asarray(x_tc, dtype=np.uint8)
    n_t, nch = x_tc.shape
    out = np.empty((nch, n_t), dtype=np.uint8)
    for c in range(nch):
        out[c, :] = x_tc[:, c]
    return out


def dedisperse(x: np.ndarray, delays: np.ndarray, n_dd: int) -> np.ndarray:
    """X[d][t] = sum_c x[c][t + delay[d][c]], t < n_dd (int64)."""
    x = np.ascontiguousarray(x, dtype=np.uint8)
    nch, n_in = x.shape
    delays = np.ascontiguousarray(delays, dtype=np.int64)
    ndm = delays.shape[0]
    assert delays.shape[1] == nch
    if ndm and nch:
        assert int(delays.max()) + n_dd <= n_in and int(delays.min()) >= 0
    X = np.empty((ndm, n_dd), dtype=np.int64)
    _load().orc_dedisperse(_p(x), n_in, nch, _p(delays), ndm, n_dd, _p(X))
    return X


def moments(X: np.ndarray, n_out: int, L: int):
    X = np.ascontiguousarray(X, dtype=np.int64)
    ndm, n_dd = X.shape
    nseg = (n_out + L - 1) // L
    n = np.empty((ndm, nseg), np.int64)
    s1 = np.empty((ndm, nseg), np.int64)
    s2 = np.empty((ndm, nseg), np.int64)
    _load().orc_moments(_p(X), ndm, n_dd, n_out, L, _p(n), _p(s1), _p(s2))
    return n, s1, s2


def mu_sigma(n: int, s1: int, s2: int) -> tuple[float, float]:
    mu = ctypes.c_double()
    sg = ctypes.c_double()
    _load().orc_mu_sigma(int(n), int(s1), int(s2), ctypes.byref(mu), ctypes.byref(sg))
    return mu.value, sg.value


def snr(B: int, w: int, mu: float, sigma: float) -> float:
    return _load().orc_snr(int(B), int(w), float(mu), float(sigma))


def search(X: np.ndarray, n_out: int, L: int, widths, theta: float) -> dict:
    """Boxcar hits: one per (d, t) above threshold, with the best width."""
    X = np.ascontiguousarray(X, dtype=np.int64)
    ndm, n_dd = X.shape
    w = np.ascontiguousarray(widths, dtype=np.int32)
    assert n_dd >= n_out + int(w.max()) - 1
    lib = _load()
    n = lib.orc_search(_p(X), ndm, n_dd, n_out, L, _p(w), w.size, theta,
                       None, None, None, None, None)
    out = {k: np.empty(n, dt) for k, dt in
           (("d", np.int32), ("t", np.int32), ("w", np.int32), ("B", np.int64), ("snr", np.float64))}
    if n:
        m = lib.orc_search(_p(X), ndm, n_dd, n_out, L, _p(w), w.size, theta,
                           _p(out["d"]), _p(out["t"]), _p(out["w"]), _p(out["B"]), _p(out["snr"]))
        assert m == n
    return out


def nms(hits: dict, ndm: int, ntime: int, stencils=((1, 1), (5, 5))) -> np.ndarray:
    """Sequential peak filters; returns the survivor mask."""
    n = hits["d"].size
    alive = np.ones(n, np.uint8)
    lib = _load()
    d = np.ascontiguousarray(hits["d"], np.int32)
    t = np.ascontiguousarray(hits["t"], np.int32)
    s = np.ascontiguousarray(hits["snr"], np.float64)
    for rd, rt in stencils:
        nxt = np.empty(n, np.uint8)
        if n:
            rc = lib.orc_nms(_p(d), _p(t), _p(s), n, ndm, ntime, rd, rt, _p(alive), _p(nxt))
            assert rc == 0
        alive = nxt
    return alive.astype(bool)


def candidates(beam: int, hits: dict, alive: np.ndarray, dms: np.ndarray) -> np.ndarray:
    """Candidate records (beam, d, t, w, B, float32(snr), float32(DM), 0) in (d, t) order."""
    idx = np.nonzero(alive)[0]
    out = np.zeros(idx.size, CAND_DTYPE)
    out["beam"] = beam
    out["dm_index"] = hits["d"][idx]
    out["t_sample"] = hits["t"][idx]
    out["width"] = hits["w"][idx]
    out["boxcar_sum"] = hits["B"][idx]
    out["snr"] = hits["snr"][idx].astype(np.float32)
    out["dm"] = dms[hits["d"][idx]].astype(np.float32)
    return out


def search_beam(x: np.ndarray, delays: np.ndarray, dms: np.ndarray, n_out: int, L: int,
                widths, theta: float, stencils=((1, 1), (5, 5)), beam: int = 0):
    """The whole per-beam search: dedisperse, boxcar search, peak filter."""
    sz = sizes(delays, n_out, widths)
    X = dedisperse(x, delays, sz["n_dd"])
    hits = search(X, n_out, L, widths, theta)
    alive = nms(hits, delays.shape[0], n_out, stencils)
    return {"X": X, "hits": hits, "alive": alive,
            "cands": candidates(beam, hits, alive, np.asarray(dms, np.float64))}


# --------------------------------------------------------------------------
# Plain candidate-optimisation path (candidate optimisation section)
# --------------------------------------------------------------------------
DEFAULT_OPT = dict(eps=0.5, min_pts=5, t_scale_s=0.05, dm_scale=20.0,
                   snr_min=10.0, dm_min=10.0, width_max_s=0.100,
                   coinc_dt_s=0.05, coinc_frac=0.5, coinc_min_beams=3)


def dbscan(x: np.ndarray, y: np.ndarray, eps: float, min_pts: int) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    lab = np.empty(x.size, np.int32)
    _load().orc_dbscan(_p(x), _p(y), x.size, eps, min_pts, _p(lab))
    return lab


def plain_optimise(cands: np.ndarray, tsamp_of_beam, n_beams: int, **kw) -> np.ndarray:
    """Per beam: DBSCAN on (t*tsamp/t_scale, DM/dm_scale), keep the highest-S/N
    member of each cluster (equal S/N: earlier in (d, t) order), drop noise;
    then S/N >= snr_min, DM >= dm_min, width*tsamp <= width_max_s; then, with
    at least coinc_min_beams beams, drop a candidate when more than coinc_frac
    of the beams hold a survivor within coinc_dt_s of its arrival time."""
    p = dict(DEFAULT_OPT)
    p.update(kw)
    tsamp_of_beam = np.asarray(tsamp_of_beam, np.float64)
    kept = []
    for b in range(n_beams):
        cb = cands[cands["beam"] == b]
        order = np.lexsort((cb["t_sample"], cb["dm_index"]))
        cb = cb[order]
        if cb.size == 0:
            continue
        ts = tsamp_of_beam[b]
        x = cb["t_sample"].astype(np.float64) * ts / p["t_scale_s"]
        y = cb["dm"].astype(np.float64) / p["dm_scale"]
        lab = dbscan(x, y, p["eps"], p["min_pts"])
        for k in range(int(lab.max()) + 1 if lab.size else 0):
            members = np.nonzero(lab == k)[0]
            if members.size == 0:
                continue
            best = members[0]
            for m in members[1:]:
                if cb["snr"][m] > cb["snr"][best]:
                    best = m
            kept.append(cb[best])
    if not kept:
        return np.zeros(0, CAND_DTYPE)
    c = np.array(kept, dtype=CAND_DTYPE)
    ts = tsamp_of_beam[c["beam"]]
    ok = ((c["snr"] >= np.float32(p["snr_min"])) & (c["dm"].astype(np.float64) >= p["dm_min"]) &
          (c["width"].astype(np.float64) * ts <= p["width_max_s"]))
    c = c[ok]
    return anti_coincidence(c, tsamp_of_beam, n_beams, **{k: p[k] for k in
                                                          ("coinc_dt_s", "coinc_frac", "coinc_min_beams")})


def anti_coincidence(c: np.ndarray, tsamp_of_beam, n_beams: int, coinc_dt_s=0.05, coinc_frac=0.5,
                     coinc_min_beams=3) -> np.ndarray:
    """Anti-coincidence across the batch's beams (candidate optimisation section): with
    at least coinc_min_beams beams, drop a candidate when more than coinc_frac of the
    beams hold a candidate within coinc_dt_s of its arrival time.  Sorted by (beam, d, t)."""
    tsamp_of_beam = np.asarray(tsamp_of_beam, np.float64)
    c = np.asarray(c, CAND_DTYPE)
    if n_beams >= coinc_min_beams and c.size:
        tabs = c["t_sample"].astype(np.float64) * tsamp_of_beam[c["beam"]]
        drop = np.zeros(c.size, bool)
        for i in range(c.size):
            near = np.abs(tabs - tabs[i]) <= coinc_dt_s
            nb = np.unique(c["beam"][near]).size
            drop[i] = nb > coinc_frac * n_beams
        c = c[~drop]
    order = np.lexsort((c["t_sample"], c["dm_index"], c["beam"]))
    return c[order]


# --------------------------------------------------------------------------
# Snippets for the candidate ranker (classification section features)
# --------------------------------------------------------------------------
SNIP_ROWS, SNIP_COLS = 64, 256


def f32_to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even of float32 to bfloat16, returned as uint16 bits."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) >> 16
    return r.astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, np.uint16).astype(np.uint32) << 16).view(np.float32)


def _mu_sigma_exact(vals: np.ndarray):
    """mu = S1/n, sigma = sqrt(n*S2 - S1^2)/n from exact integer moments
    (the normaliser of the search); sigma = 0 when the variance is 0."""
    n = int(vals.size)
    if n == 0:
        return 0.0, 0.0
    s1 = int(vals.astype(np.int64).sum())
    s2 = sum(int(a) * int(a) for a in vals.astype(np.int64)) if n < 64 else int(
        (vals.astype(np.int64) * vals.astype(np.int64)).sum())
    V = n * s2 - s1 * s1
    mu = float(s1) / float(n)
    return mu, (float(np.sqrt(float(V))) / float(n) if V > 0 else 0.0)


def snippets(x: np.ndarray, delays: np.ndarray, X: np.ndarray, n_out: int, L: int,
             d_star: int, t_star: int) -> np.ndarray:
    """Two 64x256 BF16 planes around a candidate (d*, t*):
    [0] DM-time: rows d*-32..d*+31 of the DM transform over t*-128..t*+127,
        each row standardised by its own (mu, sigma) over the segment of t*;
    [1] frequency-time: 64 sub-bands of nch/64 adjacent channels, each summed
        after the delays of trial d*, over the same samples, each sub-band
        standardised over its valid samples.
    Entries outside the DM range or outside [0, n_dd) are 0.  Values are
    float32((v - mu)/sigma) evaluated in float64, then rounded to BF16."""
    ndm, n_dd = X.shape
    nch = x.shape[0]
    R, C = SNIP_ROWS, SNIP_COLS
    out = np.zeros((2, R, C), np.float32)
    ts = np.arange(t_star - C // 2, t_star + C // 2)
    tvalid = (ts >= 0) & (ts < n_dd)
    tv = ts[tvalid]
    seg = t_star // L
    lo, hi = seg * L, min((seg + 1) * L, n_out)
    for r in range(R):
        d = d_star - R // 2 + r
        if d < 0 or d >= ndm:
            continue
        mu, sg = _mu_sigma_exact(X[d, lo:hi])
        if sg > 0.0:
            out[0, r, tvalid] = ((X[d, tv].astype(np.float64) - mu) / sg).astype(np.float32)
    per = nch // R
    for k in range(R):
        v = np.zeros(tv.size, np.int64)
        for c in range(k * per, (k + 1) * per):
            v += x[c, tv + int(delays[d_star, c])]
        mu, sg = _mu_sigma_exact(v)
        if sg > 0.0:
            out[1, k, tvalid] = ((v.astype(np.float64) - mu) / sg).astype(np.float32)
    return f32_to_bf16_bits(out)


FINE_KEEP = 0.1   # S/N kept at the edges of the fine-DM plane (a 90 % loss)


def fine_dm_half_range(width: int, tsamp: float, fch1: float, foff: float, nch: int,
                       keep: float = FINE_KEEP) -> float:
    """Half-width dDM (pc cm^-3) of the fine-DM plane of a candidate of `width` samples:
    the DM offset at which a Gaussian pulse that wide keeps `keep` of its S/N, from the
    large-zeta form of Eq. snrloss, (S(dDM)/S) = sqrt(pi)/(2 zeta), with zeta of
    Eq. zetadef.  This is Eq. deltadm with its unit conversion redone: with W in seconds
    and nu in MHz the constant is sqrt(pi)/13820, not the printed sqrt(pi)/1382.  nu is
    the band centre (midway between the outer channel centres), the bandwidth
    nch*|foff|."""
    f = fch1 + np.arange(nch, dtype=np.float64) * foff
    fref, flo = float(f.max()), float(f.min())
    w_ms = (float(width) * tsamp) * 1000.0
    nu = ((fref + flo) * 0.5) / 1000.0
    bw = float(nch) * abs(foff)
    zeta = 0.88622692545275801365 / keep          # sqrt(pi)/2 over the S/N kept
    return ((zeta * w_ms) * ((nu * nu) * nu)) / (6.91e-3 * bw)


def fine_dm_snippet(x: np.ndarray, n_in: int, fch1: float, foff: float, tsamp: float, dm_star: float,
                    width: int, t_star: int, keep: float = FINE_KEEP) -> np.ndarray:
    """Fine-DM DM-time plane (64x256 BF16 bits) of a candidate (trial DM dm_star, boxcar
    width, sample t_star): row r is the brute-force dedispersion at DM
    dm_star + (r - 32) * dDM/32 (dDM from fine_dm_half_range; delays by Eq. (1) as for a
    plan), over samples t_star-128 .. t_star+127.  An entry is valid when every
    channel's sample lies in [0, n_in).  All valid entries are standardised by one
    mu, sigma from their exact integer moments; values float32((v - mu)/sigma) in
    float64, then BF16 (RNE); invalid entries 0."""
    nch = x.shape[0]
    R, C = SNIP_ROWS, SNIP_COLS
    step = fine_dm_half_range(width, tsamp, fch1, foff, nch, keep) / 32.0
    dms = np.array([dm_star + float(r - 32) * step for r in range(R)], dtype=np.float64)
    D, _ = delay_table(nch, fch1, foff, tsamp, dms)
    ts = np.arange(t_star - C // 2, t_star + C // 2, dtype=np.int64)
    X = np.zeros((R, C), np.int64)
    valid = np.zeros((R, C), bool)
    for r in range(R):
        ok = (ts + D[r].min() >= 0) & (ts + D[r].max() < n_in)
        valid[r] = ok
        tv = ts[ok]
        for c in range(nch):
            X[r, ok] += x[c, tv + D[r, c]]
    mu, sg = _mu_sigma_exact(X[valid])
    out = np.zeros((R, C), np.float32)
    if sg > 0.0:
        out[valid] = ((X[valid].astype(np.float64) - mu) / sg).astype(np.float32)
    return f32_to_bf16_bits(out)
