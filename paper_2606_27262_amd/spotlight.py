"""ctypes binding of libspotlight.so (argument marshalling only).

Device memory and streams come from PyTorch; every step of the search runs in
the library's HIP kernels.  Importing this module fails if the library is not
built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SPL_LIBRARY names another build of the library (the host-sanitizer test's)
LIB_PATH = os.environ.get("SPL_LIBRARY") or os.path.join(_HERE, "libspotlight.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2606_27262_amd.build.build() "
                      "(or __graft_entry__.build()) before using the search")
# torch is loaded first so that the library's libamdhip64.so.7 resolves to the HIP runtime
# torch already holds: device memory and streams come from torch, and a second HIP/HSA
# runtime in the same process would not see the device.
import torch  # noqa: E402,F401
_lib = ctypes.CDLL(LIB_PATH)

STAGES = ("dedisp", "thresholds", "boxcar", "peaks")
SPL_OK, SPL_E_INVALID_ARG, SPL_E_HIP, SPL_E_OOM, SPL_E_CAPACITY, SPL_E_UNSUPPORTED, \
    SPL_E_NO_WEIGHTS, SPL_E_INTERNAL = range(8)
MODE_PLAIN_PER_BEAM, MODE_PERSISTENT_GRAPH = 0, 1
MAX_STENCILS = 4

CAND_DTYPE = np.dtype([("beam", "<i4"), ("dm_index", "<i4"), ("t_sample", "<i4"),
                       ("width", "<i4"), ("boxcar_sum", "<i4"), ("snr", "<f4"),
                       ("dm", "<f4"), ("flags", "<u4")])


class SplError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"spotlight error {status}: {msg}")
        self.status = status


class _Band(ctypes.Structure):
    _fields_ = [("nchans", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("norm_window", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("fch1_mhz", ctypes.c_double), ("foff_mhz", ctypes.c_double),
                ("tsamp_s", ctypes.c_double)]


class _DMRange(ctypes.Structure):
    _fields_ = [("dm_start", ctypes.c_double), ("dm_step", ctypes.c_double),
                ("n_trials", ctypes.c_int32), ("reserved0", ctypes.c_int32)]


class _SearchOpts(ctypes.Structure):
    _fields_ = [("n_stencils", ctypes.c_int32), ("stencil_rd", ctypes.c_int32 * MAX_STENCILS),
                ("stencil_rt", ctypes.c_int32 * MAX_STENCILS)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("nchans", "ndm", "n_out", "n_dd", "n_in", "s_max",
                                               "n_widths", "w_max", "norm_window", "n_segments",
                                               "n_stencils", "reserved0")] + [("threshold", ctypes.c_double)]


class _BatchOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("hit_capacity", ctypes.c_int64)]


class _Tiles(ctypes.Structure):
    _fields_ = [("dm_per_wave", ctypes.c_int32), ("time_groups", ctypes.c_int32),
                ("chan_chunk", ctypes.c_int32), ("waves", ctypes.c_int32), ("buffers", ctypes.c_int32)]


class _SmearingOpts(ctypes.Structure):
    _fields_ = [("dm_min", ctypes.c_double), ("dm_max", ctypes.c_double), ("max_loss", ctypes.c_double),
                ("w_min_s", ctypes.c_double)]


class _OptParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("min_pts", ctypes.c_int32), ("coinc_min_beams", ctypes.c_int32),
                ("t_scale_s", ctypes.c_double), ("dm_scale", ctypes.c_double), ("snr_min", ctypes.c_double),
                ("dm_min", ctypes.c_double), ("width_max_s", ctypes.c_double), ("coinc_dt_s", ctypes.c_double),
                ("coinc_frac", ctypes.c_double)]


STATS_FIELDS = ("n_hits", "n_candidates", "n_after_stencil0", "n_after_stencil1",
                "n_after_stencil2", "n_after_stencil3", "overflow")
STATS_WORDS = 7   # int64 words of spl_run_stats

_P = ctypes.c_void_p
_I32, _I64, _F64, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t


def _sig(name, args, res=ctypes.c_int32):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("spl_last_error", [], ctypes.c_char_p)
_sig("spl_version", [], ctypes.c_int32)
_sig("spl_plan_create", [ctypes.POINTER(_Band), ctypes.POINTER(_DMRange), _I32, _P, _I32, _F64,
                         ctypes.POINTER(_SearchOpts), ctypes.POINTER(_P)])
_sig("spl_plan_create_from_delays", [ctypes.POINTER(_Band), _P, _P, _I32, _P, _I32, _F64,
                                     ctypes.POINTER(_SearchOpts), ctypes.POINTER(_P)])
_sig("spl_plan_query", [_P, ctypes.POINTER(_PlanInfo)])
_sig("spl_plan_delays", [_P, _P])
_sig("spl_plan_dms", [_P, _P])
_sig("spl_plan_destroy", [_P], None)
_sig("spl_plan_smearing_ranges", [ctypes.POINTER(_Band), ctypes.POINTER(_SmearingOpts), _P, _I32,
                                  ctypes.POINTER(_I32)])
_sig("spl_batch_create", [ctypes.POINTER(_P), _I32, ctypes.POINTER(_BatchOpts), ctypes.POINTER(_P)])
_sig("spl_batch_workspace_size", [_P, ctypes.POINTER(_SZ), ctypes.POINTER(_SZ)])
_sig("spl_batch_set_workspace", [_P, _P, _SZ])
_sig("spl_batch_run", [_P, ctypes.POINTER(_P), ctypes.POINTER(_I64), _P, _I64, _P, _P])
_sig("spl_batch_dm_transform", [_P, _I32, ctypes.POINTER(_P), ctypes.POINTER(_I64)])
_sig("spl_batch_moments", [_P, _I32, ctypes.POINTER(_P), ctypes.POINTER(_P)])
_sig("spl_batch_get_tiles", [_P, _I32, ctypes.POINTER(_Tiles)])
_sig("spl_batch_set_tiles", [_P, _I32, ctypes.POINTER(_Tiles)])
_sig("spl_batch_destroy", [_P], None)
_sig("spl_batch_run_static", [_P, ctypes.POINTER(_P), ctypes.POINTER(_I64), _P, _I64, _P, _P])
STATIC_SCRATCH_BYTES = 64 << 20   # SPL_STATIC_SCRATCH_BYTES
_sig("spl_batch_set_profiling", [_P, _I32])
_sig("spl_autotune", [_P, ctypes.POINTER(_P), ctypes.POINTER(_I64), ctypes.c_char_p, _I32, _P])
_sig("spl_batch_stage_times", [_P, _P, _P, _I32])
_sig("spl_debug_mu_sigma", [_P, _P, _P, _I64, _P, _P, _P])
_sig("spl_opt_defaults", [ctypes.POINTER(_OptParams)], None)
_sig("spl_optimise_plain", [_P, _I64, _P, _I32, ctypes.POINTER(_OptParams), _P, _I64, ctypes.POINTER(_I64)])
_sig("spl_anti_coincidence", [_P, _I64, _P, _I32, ctypes.POINTER(_OptParams), _P, _I64, ctypes.POINTER(_I64)])


class _RankerOpts(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("reserved1", ctypes.c_float)]


class _Quantiser(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_int32), ("reserved", ctypes.c_int32), ("mu", ctypes.c_double),
                ("sigma", ctypes.c_double), ("level", ctypes.c_double), ("offset", ctypes.c_double)]


INJECT_SAMPLE, INJECT_ARGMAX = 0, 1

_F32 = ctypes.c_float
_sig("spl_corner_turn", [_P, _I64, _I32, _I64, _P, _I64, _P])
_sig("spl_stream_assemble", [_P, _I64, _P, _I64, _P, _I64, _I32, _I64, _I64, _P])
_sig("spl_inject_quantised", [_P, _I64, _I64, _I32, _P, _P, _P, _I32, _I32, ctypes.POINTER(_Quantiser), _I32, _P])
_sig("spl_ranker_snippets", [_P, _P, _I64, _P, _P])
_sig("spl_ranker_snippets_fine", [_P, _P, _I64, _F64, _P, _P])
_sig("spl_ranker_create", [ctypes.POINTER(_RankerOpts), ctypes.POINTER(_P)])
_sig("spl_ranker_workspace_size", [_P, ctypes.POINTER(_SZ)])
_sig("spl_ranker_set_workspace", [_P, _P, _SZ])
_sig("spl_ranker_set_weights", [_P, _P])
_sig("spl_ranker_get_weights", [_P, _P, _P])
_sig("spl_ranker_score", [_P, _P, _I64, _P, _P])
_sig("spl_ranker_backward", [_P, _P, _P, _I64, _P, _P])
_sig("spl_ranker_train_step", [_P, _P, _P, _I64, _F32, _P, _P])
_sig("spl_ranker_grads", [_P, ctypes.POINTER(_P)])
_sig("spl_ranker_destroy", [_P], None)
_sig("spl_debug_gemm_bf16", [_P, _I64, _P, _I64, _P, _I64, _I32, _I32, _I32, _P])
_sig("spl_ranker_debug_pool_args", [_P, _I32, ctypes.POINTER(_P)])
_sig("spl_ranker_debug_fc_preact", [_P, ctypes.POINTER(_P)])

SNIPPET_ROWS, SNIPPET_COLS = 64, 256
SNIPPET_ELEMS = 2 * SNIPPET_ROWS * SNIPPET_COLS
RANKER_PARAMS = 159553


def _check(st):
    if st != SPL_OK:
        raise SplError(st, _lib.spl_last_error().decode())


def version() -> int:
    return int(_lib.spl_version())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def smearing_ranges(nchans, fch1, foff, tsamp, dm_min, dm_max, max_loss=0.1, w_min_s=0.0):
    """DM sub-ranges [(dm_start, dm_step, n_trials)] with smearing-limited spacing
    (see spl_plan_smearing_ranges)."""
    band = _Band(int(nchans), 1, 0, 0, float(fch1), float(foff), float(tsamp))
    o = _SmearingOpts(float(dm_min), float(dm_max), float(max_loss), float(w_min_s))
    cap = 64
    out = (_DMRange * cap)()
    n = _I32()
    _check(_lib.spl_plan_smearing_ranges(ctypes.byref(band), ctypes.byref(o), out, cap, ctypes.byref(n)))
    return [(out[k].dm_start, out[k].dm_step, out[k].n_trials) for k in range(n.value)]


class Plan:
    """Search plan of one beam (see spl_plan_create)."""

    def __init__(self, nchans, fch1, foff, tsamp, n_out, dm_ranges=None, widths=(1,), threshold=6.0,
                 norm_window=0, stencils=((1, 1), (5, 5)), delays=None, dms=None):
        band = _Band(int(nchans), int(n_out), int(norm_window), 0, float(fch1), float(foff), float(tsamp))
        w = np.ascontiguousarray(widths, np.int32)
        opts = _SearchOpts()
        opts.n_stencils = len(stencils)
        for k, (rd, rt) in enumerate(stencils):
            opts.stencil_rd[k] = int(rd)
            opts.stencil_rt[k] = int(rt)
        h = _P()
        if delays is None:
            rr = (_DMRange * len(dm_ranges))(*[_DMRange(float(a), float(b), int(n), 0) for a, b, n in dm_ranges])
            _check(_lib.spl_plan_create(ctypes.byref(band), rr, len(dm_ranges), w.ctypes.data, w.size,
                                        float(threshold), ctypes.byref(opts), ctypes.byref(h)))
        else:
            dl = np.ascontiguousarray(delays, np.int32)
            dv = None if dms is None else np.ascontiguousarray(dms, np.float64)
            _check(_lib.spl_plan_create_from_delays(ctypes.byref(band), dl.ctypes.data,
                                                    None if dv is None else dv.ctypes.data, dl.shape[0],
                                                    w.ctypes.data, w.size, float(threshold), ctypes.byref(opts),
                                                    ctypes.byref(h)))
        self._h = h
        self.tsamp = float(tsamp)
        # the caller's own arguments, kept so that a checker can rebuild the plan's tables
        # independently of the library
        self.args = {"nchans": int(nchans), "fch1": float(fch1), "foff": float(foff), "tsamp": float(tsamp),
                     "n_out": int(n_out), "dm_ranges": None if dm_ranges is None else [tuple(r) for r in dm_ranges],
                     "widths": tuple(int(v) for v in widths), "threshold": float(threshold),
                     "norm_window": int(norm_window), "stencils": tuple(tuple(s) for s in stencils),
                     "delays": None if delays is None else np.array(delays, np.int64),
                     "dms": None if dms is None else np.array(dms, np.float64)}
        self.info = self.query()

    @classmethod
    def from_dict(cls, p, **kw):
        return cls(p["nchans"], p["fch1"], p["foff"], p["tsamp"], p["n_out"], p["dm_ranges"], p["widths"],
                   p["threshold"], norm_window=p.get("norm_window", 0), **kw)

    def query(self) -> dict:
        i = _PlanInfo()
        _check(_lib.spl_plan_query(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in _PlanInfo._fields_}

    def delays(self) -> np.ndarray:
        out = np.empty((self.info["ndm"], self.info["nchans"]), np.int32)
        _check(_lib.spl_plan_delays(self._h, out.ctypes.data))
        return out

    def dms(self) -> np.ndarray:
        out = np.empty(self.info["ndm"], np.float64)
        _check(_lib.spl_plan_dms(self._h, out.ctypes.data))
        return out

    def __del__(self, _destroy=_lib.spl_plan_destroy):
        # the destroy function is bound when the class is made: at interpreter exit the
        # module's globals may already be gone when the last handle is collected
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _destroy(h)


class Batch:
    """A batch of beams searched per run.  Device memory (workspace, candidates,
    statistics) is allocated here with torch and owned by this object."""

    def __init__(self, plans, mode=MODE_PLAIN_PER_BEAM, hit_capacity=0, device="cuda"):
        self.plans = list(plans)
        arr = (_P * len(self.plans))(*[p._h for p in self.plans])
        opts = _BatchOpts(int(mode), 0, int(hit_capacity))
        h = _P()
        _check(_lib.spl_batch_create(arr, len(self.plans), ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self.mode = mode
        self.device = device
        self.ws = None
        self._stream = None

    def workspace_parts(self) -> tuple:
        """(persistent, scratch) bytes of the device workspace (see spl_batch_workspace_size)."""
        p, s = _SZ(), _SZ()
        _check(_lib.spl_batch_workspace_size(self._h, ctypes.byref(p), ctypes.byref(s)))
        return int(p.value), int(s.value)

    def workspace_bytes(self) -> int:
        return sum(self.workspace_parts())

    def tiles(self, beam=0) -> dict:
        t = _Tiles()
        _check(_lib.spl_batch_get_tiles(self._h, beam, ctypes.byref(t)))
        return {"dm_per_wave": t.dm_per_wave, "time_groups": t.time_groups, "chan_chunk": t.chan_chunk,
                "waves": t.waves, "buffers": t.buffers}

    def set_tiles(self, beam, dm_per_wave, time_groups, chan_chunk=0, waves=4, buffers=1):
        t = _Tiles(int(dm_per_wave), int(time_groups), int(chan_chunk), int(waves), int(buffers))
        _check(_lib.spl_batch_set_tiles(self._h, beam, ctypes.byref(t)))
        if self.ws is not None:
            self.attach()

    def attach(self):
        """Allocate (or grow) the workspace with torch and upload the plan tables."""
        import torch
        nbytes = self.workspace_bytes()
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = None
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_off = (-base) % 256
        _check(_lib.spl_batch_set_workspace(self._h, ctypes.c_void_p(base + self._ws_off), nbytes))

    def run(self, blocks, cands=None, stats=None, stream=None):
        """Enqueue one search.  blocks: list of uint8 CUDA tensors [nch][pitch] (pitch a
        multiple of 16).  cands: int32 tensor [capacity, 8]; stats: int64 tensor [7]."""
        import torch
        if self.ws is None:
            self.attach()
        nb = len(self.plans)
        assert len(blocks) == nb
        ptrs = (_P * nb)(*[b.data_ptr() for b in blocks])
        pitches = (_I64 * nb)(*[b.stride(0) for b in blocks])
        for b in blocks:
            assert b.dtype == torch.uint8 and b.is_cuda and b.dim() == 2 and b.stride(1) == 1
        if stats is None:
            stats = torch.zeros(STATS_WORDS, dtype=torch.int64, device=self.device)
        cap = 0 if cands is None else cands.shape[0]
        cptr = None if cands is None else ctypes.c_void_p(cands.data_ptr())
        if self.mode == MODE_PERSISTENT_GRAPH and stream is None:
            # graph capture needs a stream other than the default one
            if self._stream is None:
                self._stream = torch.cuda.Stream(device=self.device)
            cur = torch.cuda.current_stream()
            self._stream.wait_stream(cur)
            _check(_lib.spl_batch_run(self._h, ptrs, pitches, cptr, cap, ctypes.c_void_p(stats.data_ptr()),
                                      _stream_handle(self._stream)))
            cur.wait_stream(self._stream)
        else:
            _check(_lib.spl_batch_run(self._h, ptrs, pitches, cptr, cap, ctypes.c_void_p(stats.data_ptr()),
                                      _stream_handle(stream)))
        return cands, stats

    def run_static(self, blocks, cands, stats, stream=None):
        """spl_batch_run_static: one search with the library's static device scratch as
        the workspace (no device allocation by the library; the caller passes the
        candidate and statistics tensors).  The batch needs no attached workspace."""
        import torch
        nb = len(self.plans)
        assert len(blocks) == nb
        for b in blocks:
            assert b.dtype == torch.uint8 and b.is_cuda and b.dim() == 2 and b.stride(1) == 1
        ptrs = (_P * nb)(*[b.data_ptr() for b in blocks])
        pitches = (_I64 * nb)(*[b.stride(0) for b in blocks])
        _check(_lib.spl_batch_run_static(self._h, ptrs, pitches, ctypes.c_void_p(cands.data_ptr()), cands.shape[0],
                                         ctypes.c_void_p(stats.data_ptr()), _stream_handle(stream)))
        return cands, stats

    def autotune(self, blocks, cache_path=None, force=False, stream=None):
        """Choose the dedispersion tiling of every plan by timing the compiled shapes
        on `blocks` (see spl_autotune).  Returns the chosen tiles per beam."""
        if self.ws is None:
            self.attach()
        nb = len(self.plans)
        ptrs = (_P * nb)(*[b.data_ptr() for b in blocks])
        pitches = (_I64 * nb)(*[b.stride(0) for b in blocks])
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(_lib.spl_autotune(self._h, ptrs, pitches, path, 1 if force else 0, _stream_handle(stream)))
        return [self.tiles(b) for b in range(nb)]

    def set_profiling(self, enable=True):
        _check(_lib.spl_batch_set_profiling(self._h, 1 if enable else 0))

    def stage_times(self, reset=True) -> dict:
        """Summed HIP-event times (ms) and counts of the profiled stages since the last reset."""
        ms = np.zeros(len(STAGES), np.float64)
        cnt = np.zeros(len(STAGES), np.int64)
        _check(_lib.spl_batch_stage_times(self._h, ms.ctypes.data, cnt.ctypes.data, 1 if reset else 0))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(STAGES)}

    def _view(self, ptr, nbytes, dtype):
        off = ptr - self.ws.data_ptr()
        assert 0 <= off and off + nbytes <= self.ws.numel()
        return self.ws[off:off + nbytes].view(dtype)

    def dm_transform(self, beam):
        """Device view int32 [ndm][pitch] of the last run's DM transform of `beam`."""
        import torch
        p = _P()
        pitch = _I64()
        _check(_lib.spl_batch_dm_transform(self._h, beam, ctypes.byref(p), ctypes.byref(pitch)))
        ndm = self.plans[beam].info["ndm"]
        return self._view(p.value, ndm * pitch.value * 4, torch.int32).view(ndm, pitch.value)

    def moments(self, beam):
        import torch
        a, b = _P(), _P()
        _check(_lib.spl_batch_moments(self._h, beam, ctypes.byref(a), ctypes.byref(b)))
        info = self.plans[beam].info
        n = info["ndm"] * info["n_segments"]
        s1 = self._view(a.value, n * 8, torch.int64).view(info["ndm"], info["n_segments"])
        s2 = self._view(b.value, n * 8, torch.int64).view(info["ndm"], info["n_segments"])
        return s1, s2

    def __del__(self, _destroy=_lib.spl_batch_destroy):
        # the destroy function is bound when the class is made: at interpreter exit the
        # module's globals may already be gone when the last handle is collected
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _destroy(h)


def new_candidates(capacity, device="cuda"):
    import torch
    return torch.empty((int(capacity), 8), dtype=torch.int32, device=device)


def candidates_to_numpy(cands, stats) -> np.ndarray:
    """Copy the written candidate records to a numpy structured array."""
    n = int(stats[1].item())
    cap = cands.shape[0]
    m = min(n, cap)
    raw = cands[:m].cpu().numpy()
    return raw.view(CAND_DTYPE).reshape(-1)


def stats_dict(stats) -> dict:
    s = stats.cpu().numpy()
    ov = int(s[6])
    return {"n_hits": int(s[0]), "n_candidates": int(s[1]),
            "n_after_stencil": [int(v) for v in s[2:6]],
            "hit_overflow": ov & 0xFFFFFFFF, "cand_overflow": (ov >> 32) & 0xFFFFFFFF}


def opt_params(**kw) -> _OptParams:
    p = _OptParams()
    _lib.spl_opt_defaults(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def optimise_plain(cands: np.ndarray, tsamp_of_beam, n_beams: int, **kw) -> np.ndarray:
    """Plain candidate-optimisation path on host records (numpy CAND_DTYPE)."""
    c = np.ascontiguousarray(cands, dtype=CAND_DTYPE)
    ts = np.ascontiguousarray(tsamp_of_beam, np.float64)
    out = np.zeros(max(1, c.size), CAND_DTYPE)
    n_out = _I64()
    p = opt_params(**kw)
    _check(_lib.spl_optimise_plain(c.ctypes.data if c.size else None, c.size, ts.ctypes.data, int(n_beams),
                                   ctypes.byref(p), out.ctypes.data, out.size, ctypes.byref(n_out)))
    return out[:n_out.value].copy()


def anti_coincidence(cands: np.ndarray, tsamp_of_beam, n_beams: int, **kw) -> np.ndarray:
    """The plain path's anti-coincidence filter alone, on host records."""
    c = np.ascontiguousarray(cands, dtype=CAND_DTYPE)
    ts = np.ascontiguousarray(tsamp_of_beam, np.float64)
    out = np.zeros(max(1, c.size), CAND_DTYPE)
    n_out = _I64()
    p = opt_params(**kw)
    _check(_lib.spl_anti_coincidence(c.ctypes.data if c.size else None, c.size, ts.ctypes.data, int(n_beams),
                                     ctypes.byref(p), out.ctypes.data, out.size, ctypes.byref(n_out)))
    return out[:n_out.value].copy()


def debug_mu_sigma(n, s1, s2, stream=None):
    """Normaliser on device (test hook): int64 CUDA tensors -> (mu, sigma) float64."""
    import torch
    mu = torch.empty(n.shape, dtype=torch.float64, device=n.device)
    sg = torch.empty(n.shape, dtype=torch.float64, device=n.device)
    _check(_lib.spl_debug_mu_sigma(ctypes.c_void_p(n.data_ptr()), ctypes.c_void_p(s1.data_ptr()),
                                   ctypes.c_void_p(s2.data_ptr()), n.numel(), ctypes.c_void_p(mu.data_ptr()),
                                   ctypes.c_void_p(sg.data_ptr()), _stream_handle(stream)))
    return mu, sg


def upload_block(x_np, device="cuda", pitch=None):
    """uint8 numpy block [nch][>= n_in] -> CUDA tensor with a 256-multiple pitch."""
    import torch
    nch, n = x_np.shape
    p = pitch or (n + 255) // 256 * 256
    t = torch.zeros((nch, p), dtype=torch.uint8, device=device)
    t[:, :n] = torch.from_numpy(np.ascontiguousarray(x_np)).to(device)
    return t


def stream_assemble(d_next, d_prev, d_stage, n_out, n_in, stream=None):
    """spl_stream_assemble: device block d_next (uint8 CUDA tensor [nch][pitch]) = the last
    n_in - n_out samples of device block d_prev, then the n_out new samples of d_stage
    (uint8 CUDA tensor [nch][stage_pitch], stage_pitch >= n_out, whose storage extends at
    least 16 bytes past its last row's n_out-th byte)."""
    nch = d_next.shape[0]
    assert d_prev.shape[0] == nch and d_stage.shape[0] == nch
    assert d_next.stride(1) == 1 and d_prev.stride(1) == 1 and d_stage.stride(1) == 1
    end = d_stage.storage_offset() + (nch - 1) * d_stage.stride(0) + int(n_out) + 16
    assert end <= d_stage.untyped_storage().nbytes(), "the staging buffer needs 16 bytes of slack after its last row"
    _check(_lib.spl_stream_assemble(ctypes.c_void_p(d_next.data_ptr()), d_next.stride(0),
                                    ctypes.c_void_p(d_prev.data_ptr()), d_prev.stride(0),
                                    ctypes.c_void_p(d_stage.data_ptr()), d_stage.stride(0), nch, int(n_out),
                                    int(n_in), _stream_handle(stream)))


def new_stage(nch, n_out, device="cuda"):
    """Device staging buffer [nch][n_out] for stream_assemble, with the 16 bytes of slack
    its last row needs (an allocation of nch * n_out + 256 bytes)."""
    import torch
    flat = torch.empty(nch * n_out + 256, dtype=torch.uint8, device=device)
    return flat[:nch * n_out].view(nch, n_out)


def corner_turn(x_tc, out=None, pitch=None, stream=None):
    """Time-major uint8 CUDA tensor [n_t][nch] (row stride a multiple of 16) ->
    channel-major [nch][pitch] (pitch a multiple of 256 by default)."""
    import torch
    n_t, nch = x_tc.shape
    assert x_tc.dtype == torch.uint8 and x_tc.stride(1) == 1
    if out is None:
        p = pitch or (n_t + 255) // 256 * 256
        out = torch.empty((nch, p), dtype=torch.uint8, device=x_tc.device)
    _check(_lib.spl_corner_turn(ctypes.c_void_p(x_tc.data_ptr()), n_t, nch, x_tc.stride(0),
                                ctypes.c_void_p(out.data_ptr()), out.stride(0), _stream_handle(stream)))
    return out


def inject_quantised(block, t_start, signal, random_words=None, *, bits=8, mu=128.0, sigma=16.0,
                     level=1.0 / 16.0, offset=-0.5, mode=INJECT_SAMPLE, n_t=None, stream=None):
    """Add signal windows to a quantised uint8 CUDA block [nch][pitch] in place.

    t_start int32 [n_win][nch], signal float32 [n_win][nch][n_sig] and random_words
    uint32 (int32 storage) of the signal's shape, all on the block's device; samples
    outside [0, n_t) (n_t defaults to the pitch) are skipped.  The default quantiser is
    the synthetic blocks' clip(round(128 + 16 n)).  Windows of one call must not
    overlap."""
    import torch
    nch, pitch = block.shape
    assert block.dtype == torch.uint8 and block.stride(1) == 1
    n_win, nch_s, n_sig = signal.shape
    assert nch_s == nch and tuple(t_start.shape) == (n_win, nch)
    assert signal.dtype == torch.float32 and signal.is_contiguous()
    assert t_start.dtype == torch.int32 and t_start.is_contiguous()
    rw = None
    if random_words is not None:
        assert random_words.shape == signal.shape and random_words.is_contiguous()
        assert random_words.dtype in (torch.int32, torch.uint32)
        rw = ctypes.c_void_p(random_words.data_ptr())
    q = _Quantiser(bits=bits, reserved=0, mu=mu, sigma=sigma, level=level, offset=offset)
    _check(_lib.spl_inject_quantised(ctypes.c_void_p(block.data_ptr()), block.stride(0),
                                     pitch if n_t is None else int(n_t), nch, ctypes.c_void_p(t_start.data_ptr()),
                                     ctypes.c_void_p(signal.data_ptr()), rw, n_win, n_sig, ctypes.byref(q), mode,
                                     _stream_handle(stream)))
    return block


def snippets(batch: Batch, cands, n=None, out=None, stream=None, fine_keep=None):
    """Feature snippets of device candidate records (int32 [>= n, 8]) of the batch's
    last run -> int16 tensor [n][2][64][256] holding BF16 bit patterns.  With fine_keep
    (e.g. 0.1) plane 0 is the fine-DM plane around each candidate's DM."""
    import torch
    n = cands.shape[0] if n is None else int(n)
    if out is None:
        out = torch.empty((n, 2, SNIPPET_ROWS, SNIPPET_COLS), dtype=torch.int16, device=cands.device)
    if fine_keep is None:
        _check(_lib.spl_ranker_snippets(batch._h, ctypes.c_void_p(cands.data_ptr()), n,
                                        ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    else:
        _check(_lib.spl_ranker_snippets_fine(batch._h, ctypes.c_void_p(cands.data_ptr()), n, float(fine_keep),
                                             ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


class Ranker:
    """CNN candidate ranker on the library's kernels; the workspace (weights, Adam
    state, activations) is a torch allocation owned by this object."""

    def __init__(self, max_batch=256, beta1=0.9, beta2=0.999, eps=1e-8, device="cuda"):
        import torch
        o = _RankerOpts(int(max_batch), 0, beta1, beta2, eps, 0.0)
        h = _P()
        _check(_lib.spl_ranker_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.max_batch = int(max_batch)
        self.device = device
        nb = _SZ()
        _check(_lib.spl_ranker_workspace_size(self._h, ctypes.byref(nb)))
        self.ws_bytes = int(nb.value)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        self._off = (-base) % 256
        _check(_lib.spl_ranker_set_workspace(self._h, ctypes.c_void_p(base + self._off), self.ws_bytes))
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)

    def set_weights(self, params: np.ndarray):
        v = np.ascontiguousarray(params, np.float32).ravel()
        assert v.size == RANKER_PARAMS
        _check(_lib.spl_ranker_set_weights(self._h, v.ctypes.data))

    def get_weights(self, stream=None) -> np.ndarray:
        v = np.zeros(RANKER_PARAMS, np.float32)
        _check(_lib.spl_ranker_get_weights(self._h, v.ctypes.data, _stream_handle(stream)))
        return v

    def score(self, snip, logits=None, stream=None):
        """Logits float32 [n] of snippets int16 [n][2][64][256] (BF16 bit patterns)."""
        import torch
        n = snip.shape[0]
        if logits is None:
            logits = torch.empty(n, dtype=torch.float32, device=snip.device)
        _check(_lib.spl_ranker_score(self._h, ctypes.c_void_p(snip.data_ptr()), n, ctypes.c_void_p(logits.data_ptr()),
                                     _stream_handle(stream)))
        return logits

    def backward(self, snip, labels, stream=None):
        """Loss tensor [1]; gradients stay in the ranker (grads())."""
        _check(_lib.spl_ranker_backward(self._h, ctypes.c_void_p(snip.data_ptr()), ctypes.c_void_p(labels.data_ptr()),
                                        snip.shape[0], ctypes.c_void_p(self.loss.data_ptr()), _stream_handle(stream)))
        return self.loss

    def train_step(self, snip, labels, lr, stream=None):
        _check(_lib.spl_ranker_train_step(self._h, ctypes.c_void_p(snip.data_ptr()),
                                          ctypes.c_void_p(labels.data_ptr()), snip.shape[0], float(lr),
                                          ctypes.c_void_p(self.loss.data_ptr()), _stream_handle(stream)))
        return self.loss

    def grads(self):
        """Device view float32 [RANKER_PARAMS] of the last gradients."""
        import torch
        p = _P()
        _check(_lib.spl_ranker_grads(self._h, ctypes.byref(p)))
        off = p.value - self.ws.data_ptr()
        assert 0 <= off and off + RANKER_PARAMS * 4 <= self.ws.numel()
        return self.ws[off:off + RANKER_PARAMS * 4].view(torch.float32)

    def pool_args(self, layer):
        """Device view uint8 [Nb][H/2][W/2][32] of conv layer `layer`'s pooling decisions."""
        import torch
        p = _P()
        _check(_lib.spl_ranker_debug_pool_args(self._h, int(layer), ctypes.byref(p)))
        nb = (self.max_batch + 31) // 32 * 32
        h, w = (32, 16, 8, 4)[layer], (128, 64, 32, 16)[layer]
        n = nb * h * w * 32
        off = p.value - self.ws.data_ptr()
        assert 0 <= off and off + n <= self.ws.numel()
        return self.ws[off:off + n].view(nb, h, w, 32)

    def fc_preact(self):
        """Device view float32 [Nb][64] of FC1's output before its bias (last pass)."""
        import torch
        p = _P()
        _check(_lib.spl_ranker_debug_fc_preact(self._h, ctypes.byref(p)))
        nb = (self.max_batch + 31) // 32 * 32
        off = p.value - self.ws.data_ptr()
        assert 0 <= off and off + nb * 64 * 4 <= self.ws.numel()
        return self.ws[off:off + nb * 64 * 4].view(torch.float32).view(nb, 64)

    def __del__(self, _destroy=_lib.spl_ranker_destroy):
        # the destroy function is bound when the class is made: at interpreter exit the
        # module's globals may already be gone when the last handle is collected
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _destroy(h)


def debug_gemm_bf16(a, b, stream=None):
    """C = A * B^T on the ranker's matrix-core kernel (test hook): int16 CUDA tensors
    A [M][K], B [N][K] of BF16 bit patterns (K a multiple of 32) -> float32 [M][N]."""
    import torch
    m, k = a.shape
    n = b.shape[0]
    c = torch.empty((m, n), dtype=torch.float32, device=a.device)
    _check(_lib.spl_debug_gemm_bf16(ctypes.c_void_p(a.data_ptr()), a.stride(0), ctypes.c_void_p(b.data_ptr()),
                                    b.stride(0), ctypes.c_void_p(c.data_ptr()), n, m, n, k, _stream_handle(stream)))
    return c
