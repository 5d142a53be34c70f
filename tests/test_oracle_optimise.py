"""Pins of the oracle's plain candidate-optimisation path and snippet extraction.

DBSCAN is checked against scikit-learn's implementation of the same textbook
algorithm (Ester et al. 1996); the plain path against a hand-built candidate set
whose outcome follows from the stated rules; the snippets against numpy's mean
and standard deviation.
"""
import numpy as np
import pytest

import oracle


def test_dbscan_matches_sklearn_core_and_noise():
    sk = pytest.importorskip("sklearn.cluster")
    rng = np.random.default_rng(5)
    for trial in range(25):
        n = int(rng.integers(1, 200))
        centres = rng.uniform(0, 10, size=(4, 2))
        pts = np.concatenate([centres[rng.integers(0, 4, n // 2)] + rng.normal(0, 0.3, (n // 2, 2)),
                              rng.uniform(0, 10, size=(n - n // 2, 2))])
        lab = oracle.dbscan(pts[:, 0], pts[:, 1], 0.5, 5)
        ref = sk.DBSCAN(eps=0.5, min_samples=5).fit(pts)
        core = np.zeros(n, bool)
        core[ref.core_sample_indices_] = True
        assert np.array_equal(lab < 0, ref.labels_ < 0)
        # the partition of core points into clusters is the same
        for i in np.nonzero(core)[0]:
            same_me = (lab == lab[i]) & core
            same_ref = (ref.labels_ == ref.labels_[i]) & core
            assert np.array_equal(same_me, same_ref)
        # cluster numbers follow the lowest-index core point
        firsts = [int(np.nonzero((lab == k) & core)[0][0]) for k in range(lab.max() + 1)]
        assert firsts == sorted(firsts)


def _cand(beam, d, t, w, snr, dm):
    c = np.zeros(1, oracle.CAND_DTYPE)
    c["beam"], c["dm_index"], c["t_sample"], c["width"] = beam, d, t, w
    c["snr"], c["dm"] = snr, dm
    return c


def test_plain_path_rules():
    ts = 1.31072e-3
    parts = []
    # beam 0: a cluster of 6 points near (t=1000, DM 100), best S/N 15 -> kept
    for k in range(6):
        parts.append(_cand(0, 100 + k, 1000 + k, 4, 11.0 + k * 0.8, 100.0 + k))
    # beam 0: a lone point (noise for DBSCAN) -> dropped
    parts.append(_cand(0, 300, 5000, 4, 40.0, 300.0))
    # beam 1: a cluster whose best S/N is 9 -> below 10 -> dropped
    for k in range(5):
        parts.append(_cand(1, 50 + k, 2000 + k, 2, 7.0 + k * 0.5, 50.0 + k))
    # beam 2: a cluster at DM 5 -> below DM 10 -> dropped
    for k in range(5):
        parts.append(_cand(2, 1 + k, 3000 + k, 2, 20.0 + k, 5.0))
    # beam 3: a cluster with width 128 samples (168 ms) -> too wide -> dropped
    for k in range(5):
        parts.append(_cand(3, 80 + k, 4000 + k, 128, 20.0 + k, 80.0 + k))
    c = np.concatenate(parts)
    out = oracle.plain_optimise(c, [ts] * 6, 6)
    assert out.size == 1
    assert out["beam"][0] == 0 and out["dm_index"][0] == 105 and out["snr"][0] == np.float32(15.0)


def test_plain_path_anti_coincidence():
    ts = 1.31072e-3
    parts = []
    # the same arrival time in 4 of 6 beams (a majority) -> all removed
    for b in range(4):
        for k in range(5):
            parts.append(_cand(b, 200 + k, 7000 + k, 4, 20.0 + k, 200.0 + k))
    # another time in 2 of 6 beams -> kept
    for b in (4, 5):
        for k in range(5):
            parts.append(_cand(b, 400 + k, 9000 + k, 4, 20.0 + k, 400.0 + k))
    out = oracle.plain_optimise(np.concatenate(parts), [ts] * 6, 6)
    assert sorted(out["beam"].tolist()) == [4, 5]
    # with fewer than 3 beams the filter does not apply
    out2 = oracle.plain_optimise(np.concatenate(parts[:10]), [ts] * 2, 2)
    assert out2.size == 2


def test_bf16_rounding_definition():
    f = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -8, -3.5, 1.0 + 2 ** -8 + 2 ** -20,
                  3.0e38], np.float32)
    b = oracle.f32_to_bf16_bits(f)
    back = oracle.bf16_bits_to_f32(b)
    # halfway cases go to the even neighbour; above-halfway rounds up
    assert back[0] == 1.0 and back[1] == 1.0
    assert back[2] == np.float32(1.0 + 2 ** -6)
    assert back[3] == -3.5
    assert back[4] == np.float32(1.0 + 2 ** -7)
    assert np.isfinite(back[5])


def test_snippets_against_numpy_statistics():
    rng = np.random.default_rng(9)
    nch, n_in, ndm, n_out = 128, 700, 80, 400
    x = rng.integers(0, 256, size=(nch, n_in), dtype=np.uint8)
    delays = np.sort(rng.integers(0, 150, size=(ndm, nch)), axis=1)
    delays = np.sort(delays, axis=0)
    X = oracle.dedisperse(x, delays, 420)
    for (d0, t0) in ((40, 200), (3, 10), (78, 399)):
        s = oracle.snippets(x, delays, X, n_out, n_out, d0, t0)
        v = oracle.bf16_bits_to_f32(s)
        ts = np.arange(t0 - 128, t0 + 128)
        ok = (ts >= 0) & (ts < 420)
        for r in range(64):
            d = d0 - 32 + r
            if not 0 <= d < ndm:
                assert np.all(v[0, r] == 0)
                continue
            seg = X[d, :n_out].astype(np.float64)
            ref = (X[d, ts[ok]] - seg.mean()) / seg.std()
            assert np.allclose(v[0, r, ok], ref, rtol=2 ** -7, atol=1e-6)
            assert np.all(v[0, r, ~ok] == 0)
        for k in range(64):
            sub = sum(x[c, ts[ok] + delays[d0, c]].astype(np.int64) for c in range(2 * k, 2 * k + 2))
            ref = (sub - sub.mean()) / sub.std()
            assert np.allclose(v[1, k, ok], ref, rtol=2 ** -7, atol=1e-6)
