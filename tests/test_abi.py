"""Host-side checks of the C ABI (no GPU): every declared symbol is exported, the
library's own delay table equals the oracle's bit for bit, plan sizes, argument
validation and batch layout."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2606_27262_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spotlight.h")

spl = pytest.importorskip("paper_2606_27262_amd.spotlight",
                          reason="libspotlight.so not built")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(spl_[a-z0-9_]+)\s*\(", src)
    return sorted(set(n for n in names if not n.startswith("spl_status")))


def test_every_declared_function_is_exported():
    lib = ctypes.CDLL(spl.LIB_PATH)
    names = _declared()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version():
    assert spl.version() >= 100


@pytest.mark.parametrize("mk", [W.plan_c1, W.plan_c2, W.plan_band3_c4, W.plan_band4_c4])
def test_library_delay_table_equals_oracle(mk):
    p = mk()
    plan = spl.Plan.from_dict(p)
    dms = oracle.dm_trials(p["dm_ranges"])
    D, ties = oracle.delay_table(p["nchans"], p["fch1"], p["foff"], p["tsamp"], dms)
    assert ties == 0
    assert np.array_equal(plan.dms(), dms)
    assert np.array_equal(plan.delays().astype(np.int64), D)
    sz = oracle.sizes(D, p["n_out"], p["widths"])
    info = plan.info
    assert (info["s_max"], info["n_dd"], info["n_in"]) == (sz["s_max"], sz["n_dd"], sz["n_in"])
    assert info["ndm"] == dms.size and info["n_segments"] == 1


def test_reversed_band_and_multi_range_plan():
    p = W.plan_c1()
    ranges = [(0.0, 2.0, 10), (20.0, 5.0, 7)]
    nch = p["nchans"]
    f_last = p["fch1"] + (nch - 1) * p["foff"]
    plan = spl.Plan(nch, f_last, -p["foff"], p["tsamp"], 1000, ranges, (1, 2), 6.0)
    dms = oracle.dm_trials(ranges)
    D, _ = oracle.delay_table(nch, f_last, -p["foff"], p["tsamp"], dms)
    assert np.array_equal(plan.delays(), D)
    assert np.all(plan.delays()[:, -1] == 0)


@pytest.mark.parametrize("bad", [
    dict(widths=(2, 1)), dict(widths=()), dict(threshold=0.0), dict(tsamp=0.0), dict(nchans=0),
    dict(n_out=0), dict(widths=(1, 20000)), dict(norm_window=-1),
])
def test_plan_validation(bad):
    args = dict(nchans=16, fch1=500.0, foff=-1.0, tsamp=1e-3, n_out=100, dm_ranges=[(0.0, 1.0, 4)],
                widths=(1, 2), threshold=6.0)
    args.update(bad)
    with pytest.raises(spl.SplError):
        spl.Plan(**args)


def test_int32_overflow_is_refused():
    with pytest.raises(spl.SplError) as e:
        spl.Plan(65536, 500.0, -0.001, 1e-3, 1000, [(0.0, 1.0, 2)], (1, 256), 6.0)
    assert e.value.status == spl.SPL_E_UNSUPPORTED


def test_from_delays_rejects_negative():
    with pytest.raises(spl.SplError):
        spl.Plan(2, 500.0, -1.0, 1e-3, 10, widths=(1,), delays=np.array([[0, -1]], np.int32))


def test_batch_layout_host_only():
    plans = [spl.Plan.from_dict(W.plan_band3_c4()), spl.Plan.from_dict(W.plan_band4_c4())]
    b = spl.Batch([plans[0], plans[1], plans[0]], mode=spl.MODE_PERSISTENT_GRAPH, hit_capacity=1 << 20)
    n = b.workspace_bytes()
    # at least the three DM transforms, all of them in the per-run scratch part; the
    # persistent part holds at least both plans' delay tables
    need = sum(p.info["ndm"] * p.info["n_dd"] * 4 for p in (plans[0], plans[1], plans[0]))
    assert n > need
    persistent, scratch = b.workspace_parts()
    assert persistent + scratch == n and scratch > need and persistent % 256 == 0
    assert persistent >= sum(p.info["ndm"] * p.info["nchans"] * 4 for p in plans)
    t = b.tiles(1)
    assert t["chan_chunk"] >= 4 and t["dm_per_wave"] in (2, 4, 8, 16) and t["buffers"] == 1
    with pytest.raises(spl.SplError):
        b.set_tiles(0, 3, 1)
    # two LDS buffers: 16-wavefront shapes only, at most one staged row per wavefront
    b.set_tiles(1, 4, 2, 16, waves=16, buffers=2)
    assert b.tiles(1) == {"dm_per_wave": 4, "time_groups": 2, "chan_chunk": 16, "waves": 16, "buffers": 2}
    b.set_tiles(0, 2, 2, 8, waves=16, buffers=2)
    assert b.tiles(2) == b.tiles(0) == {"dm_per_wave": 2, "time_groups": 2, "chan_chunk": 8, "waves": 16,
                                        "buffers": 2}   # beams of one plan share its tiling
    for bad in (dict(waves=8, buffers=2), dict(waves=16, buffers=3), dict(waves=16, buffers=-1)):
        with pytest.raises(spl.SplError):
            b.set_tiles(1, 4, 2, 16, **bad)
    with pytest.raises(spl.SplError):
        b.set_tiles(1, 4, 2, 32, waves=16, buffers=2)
    with pytest.raises(spl.SplError):   # two buffers of 16 rows of ~1.9 KB exceed the LDS
        b.set_tiles(0, 2, 2, 16, waves=16, buffers=2)
    assert b.tiles(1)["buffers"] == 2 and b.tiles(0)["chan_chunk"] == 8   # refusals keep the tiling
    b.set_tiles(1, 4, 2, 32, waves=16)
    assert b.tiles(1)["buffers"] == 1 and b.tiles(1)["chan_chunk"] == 32
    # chan_chunk 0: the largest that fits; a 16-wavefront workgroup has the whole LDS
    b.set_tiles(1, 4, 2, 0, waves=16)
    assert b.tiles(1)["chan_chunk"] == 32
    b.set_tiles(1, 4, 2, 0, waves=16, buffers=2)
    assert b.tiles(1)["chan_chunk"] == 16
    b.set_tiles(0, 2, 2, 0, waves=16, buffers=2)   # rows of ~1.9 KB: two buffers of 8 channels
    assert b.tiles(0)["chan_chunk"] == 8


def _rand_cands(rng, n_beams, per_beam, clustered=True):
    parts = []
    for b in range(n_beams):
        n = int(rng.integers(0, per_beam))
        c = np.zeros(n, oracle.CAND_DTYPE)
        c["beam"] = b
        if clustered and n:
            centres = rng.integers(0, 2000, size=(4, 2))
            k = rng.integers(0, 4, n)
            c["dm_index"] = np.clip(centres[k, 0] + rng.integers(-15, 16, n), 0, 2047)
            c["t_sample"] = np.clip(centres[k, 1] * 8 + rng.integers(-30, 31, n), 0, 16383)
        else:
            c["dm_index"] = rng.integers(0, 2048, n)
            c["t_sample"] = rng.integers(0, 16384, n)
        c["width"] = rng.choice([1, 2, 4, 8, 16, 32, 64, 128], n)
        c["snr"] = rng.uniform(6, 30, n).astype(np.float32).round(1)
        c["dm"] = (c["dm_index"] * 0.9765625).astype(np.float32)
        parts.append(c)
    c = np.concatenate(parts) if parts else np.zeros(0, oracle.CAND_DTYPE)
    # unique (beam, d, t), sorted like the search output
    _, u = np.unique(c[["beam", "dm_index", "t_sample"]], return_index=True)
    c = c[np.sort(u)]
    return c[np.lexsort((c["t_sample"], c["dm_index"], c["beam"]))]


@pytest.mark.parametrize("n_beams", [1, 2, 5, 24])
def test_plain_path_library_equals_oracle(n_beams):
    rng = np.random.default_rng(100 + n_beams)
    for trial in range(6):
        c = _rand_cands(rng, n_beams, 400, clustered=trial % 2 == 0)
        ts = np.full(n_beams, 1.31072e-3)
        ts[::2] = 0.65536e-3
        ref = oracle.plain_optimise(c, ts, n_beams)
        got = spl.optimise_plain(c, ts, n_beams)
        assert np.array_equal(got, ref), (trial, got.size, ref.size)
    # a coincident burst in every beam is removed
    if n_beams >= 3:
        parts = [c]
        for b in range(n_beams):
            for k in range(6):
                x = np.zeros(1, oracle.CAND_DTYPE)
                x["beam"], x["dm_index"], x["t_sample"], x["width"] = b, 300 + k, 9000 + k, 4
                x["snr"], x["dm"] = 25.0 + k, 300.0 + k
                parts.append(x)
        c2 = np.concatenate(parts)
        ts = np.full(n_beams, 1.31072e-3)   # same arrival time in seconds in every beam
        ref = oracle.plain_optimise(c2, ts, n_beams)
        got = spl.optimise_plain(c2, ts, n_beams)
        assert np.array_equal(got, ref)
        assert not np.any((got["t_sample"] >= 9000) & (got["t_sample"] < 9006))


def test_ranker_handle_validation():
    """Host-only paths of the ranker ABI: option checks and workspace sizing."""
    lib = ctypes.CDLL(spl.LIB_PATH)
    h = ctypes.c_void_p()
    bad = spl._RankerOpts(2000, 0, 0.9, 0.999, 1e-8, 0.0)
    assert lib.spl_ranker_create(ctypes.byref(bad), ctypes.byref(h)) == spl.SPL_E_INVALID_ARG
    bad = spl._RankerOpts(32, 0, 1.5, 0.999, 1e-8, 0.0)
    assert lib.spl_ranker_create(ctypes.byref(bad), ctypes.byref(h)) == spl.SPL_E_INVALID_ARG
    sizes = []
    for mb in (1, 32, 33, 64):
        o = spl._RankerOpts(mb, 0, 0.0, 0.0, 0.0, 0.0)
        assert spl._lib.spl_ranker_create(ctypes.byref(o), ctypes.byref(h)) == spl.SPL_OK
        n = ctypes.c_size_t()
        assert spl._lib.spl_ranker_workspace_size(h, ctypes.byref(n)) == spl.SPL_OK
        sizes.append(n.value)
        # no workspace: every device call is refused before touching the GPU
        assert spl._lib.spl_ranker_score(h, None, 0, None, None) == spl.SPL_E_INVALID_ARG
        spl._lib.spl_ranker_destroy(h)
    # batches are padded to 32 candidates
    assert sizes[0] == sizes[1] and sizes[2] == sizes[3] and sizes[2] > sizes[1]
    assert sizes[1] % 256 == 0
    # about 2.1 MB of activations and gradients per candidate (pooled BF16 outputs and
    # decisions of the four layers, the widest dZ and dX) plus weights, moments and tables;
    # the convolutions' FP32 results never reach memory in the forward pass
    per = (sizes[2] - sizes[1]) / 32
    assert 1.8e6 < per < 2.5e6, per


def test_anti_coincidence_equals_oracle():
    """The library's anti-coincidence step alone equals the oracle's on random records
    crowded in time, across the beam-count threshold and the 50% rule."""
    rng = np.random.default_rng(17)
    for n_beams, n in ((2, 40), (3, 60), (8, 200), (24, 500)):
        c = np.zeros(n, oracle.CAND_DTYPE)
        c["beam"] = rng.integers(0, n_beams, n)
        c["dm_index"] = rng.integers(0, 100, n)
        c["t_sample"] = rng.integers(0, 16384, n)
        # interference events: records in about 70% of the beams at nearly the same time
        for e in range(5):
            T = int(rng.integers(100, 16000))
            idx = rng.choice(n, size=n // 10, replace=False)
            c["t_sample"][idx] = T + rng.integers(-10, 11, idx.size)
            c["beam"][idx] = rng.choice(n_beams, size=idx.size, replace=True) if n_beams > 3 else c["beam"][idx]
        c["dm"] = c["dm_index"] * 1.0
        c["snr"] = rng.uniform(6, 20, n).astype(np.float32)
        c["width"] = 1
        ts = np.full(n_beams, 1.31072e-3)
        ref = oracle.anti_coincidence(c, ts, n_beams)
        got = spl.anti_coincidence(c.astype(spl.CAND_DTYPE), ts, n_beams)
        assert np.array_equal(got.view(np.int32), ref.view(np.int32)), n_beams
        if n_beams >= 3:
            assert 0 < ref.size < c.size   # the filter acted


@pytest.mark.parametrize("band", [W.plan_c1, W.plan_c2, W.plan_band3_c4, W.plan_band4_c4])
def test_smearing_ranges_equal_oracle(band):
    p = band()
    for loss, wmin, lo, hi in ((0.1, 0.0, 0.0, 2000.0), (0.05, 0.0, 3.0, 500.0), (0.2, 1e-3, 0.0, 3000.0)):
        got = spl.smearing_ranges(p["nchans"], p["fch1"], p["foff"], p["tsamp"], lo, hi, loss, wmin)
        ref = oracle.smearing_ranges(p["nchans"], p["fch1"], p["foff"], p["tsamp"], lo, hi, loss, wmin)
        assert got == ref
        plan = spl.Plan(p["nchans"], p["fch1"], p["foff"], p["tsamp"], 1024, got, (1, 2), 6.0)
        dms = oracle.dm_trials(got)
        D, ties = oracle.delay_table(p["nchans"], p["fch1"], p["foff"], p["tsamp"], dms)
        assert ties == 0 and np.array_equal(plan.delays().astype(np.int64), D)


def test_injector_argument_checks_before_any_device_work():
    """spl_inject_quantised refuses bad quantisers, modes, shapes and missing buffers on
    the host; empty work returns SPL_OK without touching a device."""
    lib = spl._lib
    Q = spl._Quantiser
    P = ctypes.c_void_p
    fake = P(16)   # never dereferenced: every call below fails or returns before a launch

    def call(q, mode=spl.INJECT_ARGMAX, nch=4, n_t=64, pitch=64, n_win=1, n_sig=8, block=fake, ts=fake,
             sig=fake, words=None):
        return lib.spl_inject_quantised(block, pitch, n_t, nch, ts, sig, words, n_win, n_sig,
                                        None if q is None else ctypes.byref(q), mode, None)

    good = Q(bits=8, reserved=0, mu=128.0, sigma=16.0, level=1.0 / 16, offset=-0.5)
    assert call(None) == spl.SPL_E_INVALID_ARG
    for bad in (Q(0, 0, 0.0, 1.0, 1.0, 0.0), Q(9, 0, 0.0, 1.0, 1.0, 0.0), Q(8, 0, 0.0, 0.0, 1.0, 0.0),
                Q(8, 0, 0.0, 1.0, -1.0, 0.0), Q(8, 0, float("nan"), 1.0, 1.0, 0.0),
                Q(8, 0, 0.0, 1.0, 1.0, float("inf"))):
        assert call(bad) == spl.SPL_E_INVALID_ARG
    assert call(good, mode=2) == spl.SPL_E_INVALID_ARG
    assert call(good, nch=0) == spl.SPL_E_INVALID_ARG
    assert call(good, pitch=32) == spl.SPL_E_INVALID_ARG        # pitch < n_t
    assert call(good, n_sig=-1) == spl.SPL_E_INVALID_ARG
    assert call(good, block=None) == spl.SPL_E_INVALID_ARG
    assert call(good, mode=spl.INJECT_SAMPLE) == spl.SPL_E_INVALID_ARG   # SAMPLE needs random words
    # nothing to do: no launch, no error
    assert call(good, n_t=0, block=None) == spl.SPL_OK
    assert call(good, n_win=0, block=None) == spl.SPL_OK
    assert call(good, n_sig=0, block=None) == spl.SPL_OK


def test_fine_snippets_argument_checks():
    lib = spl._lib
    assert lib.spl_ranker_snippets_fine(None, None, 0, 1.5, None, None) == spl.SPL_E_INVALID_ARG
    assert lib.spl_ranker_snippets_fine(None, None, 0, 0.0, None, None) == spl.SPL_E_INVALID_ARG
    assert lib.spl_ranker_snippets_fine(None, None, 0, 0.1, None, None) == spl.SPL_E_INVALID_ARG   # no batch


def test_static_entry_point_rejects_a_batch_beyond_its_scratch():
    """spl_batch_run_static refuses, before any device work, a batch whose workspace
    exceeds the static scratch (the 24-beam 4096-channel batch needs gigabytes)."""
    plan = spl.Plan.from_dict(W.plan_c2())
    batch = spl.Batch([plan] * 2)
    assert batch.workspace_bytes() > spl.STATIC_SCRATCH_BYTES
    nb = 2
    fake = 1 << 40    # aligned stand-ins: the size check comes before any device access
    ptrs = (ctypes.c_void_p * nb)(fake, fake)
    pitches = (ctypes.c_int64 * nb)(*[(plan.info["n_in"] + 15) // 16 * 16] * nb)
    st = spl._lib.spl_batch_run_static(batch._h, ptrs, pitches, ctypes.c_void_p(fake), 16,
                                       ctypes.c_void_p(fake), None)
    assert st == spl.SPL_E_UNSUPPORTED
    assert b"static scratch" in spl._lib.spl_last_error()


def test_stream_assemble_argument_checks():
    """spl_stream_assemble refuses, before any device work, pitches below the row
    lengths, n_out outside [1, n_in], misaligned sizes and overlapping buffers."""
    lib = spl._lib
    f = 1 << 40   # stand-in addresses: every check here comes before a device access
    g, h = f + (1 << 30), f + (2 << 30)
    E = spl.SPL_E_INVALID_ARG
    assert lib.spl_stream_assemble(f, 128, g, 256, h, 64, 4, 48, 150, None) == E     # next pitch < n_in
    assert lib.spl_stream_assemble(f, 256, g, 256, h, 32, 4, 48, 150, None) == E     # stage pitch < n_out
    assert lib.spl_stream_assemble(f, 256, f + 512, 256, h, 64, 4, 48, 150, None) == E   # blocks overlap
    assert lib.spl_stream_assemble(f, 256, g, 256, f + 600, 64, 4, 48, 150, None) == E   # stage overlaps next
    assert lib.spl_stream_assemble(f, 256, g, 256, h, 64, 4, 200, 150, None) == E    # n_out > n_in
    assert lib.spl_stream_assemble(f, 256, g, 256, h, 64, 4, 40, 150, None) == E     # n_out not a multiple of 16
    assert lib.spl_stream_assemble(f + 8, 256, g, 256, h, 64, 4, 48, 150, None) == E  # misaligned block
    assert lib.spl_stream_assemble(f, 256, g, 256, h, 66, 4, 48, 150, None) == E     # stage pitch % 4
    assert lib.spl_stream_assemble(f, 256, None, 256, h, 64, 4, 48, 150, None) == E  # no previous block
    assert lib.spl_stream_assemble(f, 256, g, 256, h, 64, 0, 48, 150, None) == E     # no channels
