"""Pins of the float64 ranker oracle: torch's float64 convolution, pooling, linear
layers, loss and autograd (library routines), and central finite differences."""
import numpy as np
import pytest

from oracle import cnn

torch = pytest.importorskip("torch")
F = torch.nn.functional


def _torch_forward(p, x):
    t = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    a = torch.tensor(x, dtype=torch.float64)
    for k in range(1, 5):
        a = F.max_pool2d(F.relu(F.conv2d(a, t[f"c{k}w"], t[f"c{k}b"], padding=1)), 2)
    h = F.relu(F.linear(a.reshape(a.shape[0], -1), t["f1w"], t["f1b"]))
    return F.linear(h, t["f2w"], t["f2b"])[:, 0], t


def test_param_count_and_flops():
    assert cnn.n_params() == (2 * 32 * 9 + 32) + 3 * (32 * 32 * 9 + 32) + (2048 * 64 + 64) + (64 + 1)
    # about 118 MFLOP per forward pass
    assert 1.15e8 < cnn.flops_forward_per_sample() < 1.21e8


def test_forward_and_backward_match_torch_float64():
    rng = np.random.default_rng(0)
    p = cnn.init_params(1)
    for k in p:
        if k.endswith("b"):
            p[k] = rng.normal(0, 0.1, p[k].shape)
    x = rng.normal(0, 1, size=(3, 2, 64, 256))
    y = np.array([1.0, 0.0, 1.0])
    logit, cache = cnn.forward(p, x)
    tl, tp = _torch_forward(p, x)
    assert np.allclose(logit, tl.detach().numpy(), rtol=1e-12, atol=1e-12)
    loss, g = cnn.backward(p, cache, y)
    tloss = F.binary_cross_entropy_with_logits(tl, torch.tensor(y))
    assert abs(loss - tloss.item()) < 1e-12
    tloss.backward()
    for k in p:
        ref = tp[k].grad.numpy()
        assert np.allclose(g[k], ref, rtol=1e-9, atol=1e-13), k


def test_central_finite_differences():
    rng = np.random.default_rng(2)
    p = cnn.init_params(3)
    x = rng.normal(0, 1, size=(1, 2, 64, 256))
    y = np.array([1.0])
    logit, cache = cnn.forward(p, x)
    _, g = cnn.backward(p, cache, y)
    eps = 1e-7   # small enough that no ReLU or pooling kink is crossed
    for name in cnn.PARAM_ORDER:
        flat = p[name].ravel()
        for idx in rng.choice(flat.size, size=min(2, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = cnn.bce_with_logits(cnn.forward(p, x)[0], y)
            flat[idx] = old - eps
            lm = cnn.bce_with_logits(cnn.forward(p, x)[0], y)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = g[name].ravel()[idx]
            assert abs(fd - an) <= 1e-6 * max(1e-2, abs(an)), (name, idx, fd, an)


def test_maxpool_tie_goes_to_first():
    x = np.zeros((1, 1, 2, 2))
    out, arg = cnn.maxpool2(x)
    assert arg[0, 0, 0, 0] == 0
    g = cnn.maxpool2_backward(np.ones((1, 1, 1, 1)), arg, x.shape)
    assert g[0, 0, 0, 0] == 1 and g.sum() == 1


def test_given_pool_decisions_reproduce_own_pass():
    """Feeding the forward pass its own arg-max decisions changes nothing; marking a
    window 255 zeroes its pooled value and its gradient."""
    rng = np.random.default_rng(4)
    p = cnn.init_params(4)
    for k in p:
        if k.endswith("b"):
            p[k] = rng.normal(0, 0.1, p[k].shape)
    x = rng.normal(0, 1, size=(2, 2, 64, 256))
    y = np.array([1.0, 0.0])
    l0, c0 = cnn.forward(p, x)
    args = []
    for k in range(1, 5):   # the given convention: 255 where no element is positive
        a = c0[f"arg{k}"].copy()
        a[c0[f"x{k}"] <= 0] = 255
        args.append(a)
    assert any(np.any(a == 255) for a in args)
    l1, c1 = cnn.forward(p, x, pool_args=args, fc_gate=c0["h"] > 0)
    assert np.array_equal(l0, l1)
    _, g0 = cnn.backward(p, c0, y)
    _, g1 = cnn.backward(p, c1, y)
    for k in g0:
        assert np.array_equal(g0[k], g1[k]), k
    # one window of layer 4 marked as having no positive element
    a4 = args[3].copy()
    a4[0, 5, 1, 2] = 255
    l2, c2 = cnn.forward(p, x, pool_args=args[:3] + [a4])
    assert c2["x4"][0, 5, 1, 2] == 0.0
    _, g2 = cnn.backward(p, c2, y)
    z4 = c2["z4"]
    gr = cnn.maxpool2_backward(np.ones_like(c2["x4"]), a4, z4.shape)
    assert gr[0, 5, 2:4, 4:6].sum() == 0.0 and gr.sum() == np.sum(a4 != 255)


def test_given_fc_gate_closes_a_unit():
    rng = np.random.default_rng(6)
    p = cnn.init_params(6)
    x = rng.normal(0, 1, size=(1, 2, 64, 256))
    y = np.array([1.0])
    l0, c0 = cnn.forward(p, x)
    gate = c0["h"] > 0
    j = int(np.argmax(c0["h"][0]))
    gate[0, j] = False
    l1, c1 = cnn.forward(p, x, fc_gate=gate)
    assert np.isclose(l0[0] - l1[0], c0["h"][0, j] * p["f2w"][0, j], rtol=1e-12, atol=1e-12)
    _, g1 = cnn.backward(p, c1, y)
    assert g1["f1b"][j] == 0.0 and np.all(g1["f1w"][j] == 0.0)


def _bf16_emulation(p, x):
    """The float32/bfloat16 evaluation of the stated arithmetic (oracle.cnn.forward_bf16):
    conv pre-activations z1..z4 and FC1 pre-activations without the bias."""
    _, zs, h = cnn.forward_bf16(p, x)
    return zs, h - np.asarray(p["f1b"]).astype(np.float32).astype(np.float64)


def test_bf16_deviation_model_covers_an_emulation():
    """Pin of the deviation model the GPU ranker's parity bounds come from: the
    pre-activations of an independent float32/bfloat16 emulation of the stated arithmetic
    lie within 6 model standard deviations of the float64 network's at every element of
    every layer, the model is not loose (root-mean-square deviation between 0.2 and 1.5
    standard deviations per layer), and dropping its weight-rounding term fails the first
    layer (whose input is exact)."""
    rng = np.random.default_rng(12)
    p = cnn.init_params(5)
    for k in p:
        if k.endswith("b"):
            p[k] = rng.normal(0, 0.05, p[k].shape)
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    x = cnn.round_bf16(rng.normal(0, 1, size=(3, 2, 64, 256)))
    _, cache = cnn.forward(p, x)
    V = cnn.deviation_model(p, cache)
    zs, h = _bf16_emulation(p, x)
    for k in range(1, 5):
        d = (zs[k - 1] - cache[f"z{k}"]) / np.sqrt(V[f"z{k}"])
        rms = float(np.sqrt(np.mean(d * d)))
        assert np.max(np.abs(d)) <= 6.0, (k, np.max(np.abs(d)))
        assert 0.2 <= rms <= 1.5, (k, rms)
    dh = (h - (cache["h"] - p["f1b"])) / np.sqrt(V["h"])
    assert np.max(np.abs(dh)) <= 6.0 and 0.2 <= float(np.sqrt(np.mean(dh * dh))) <= 1.5
    V0 = cnn.deviation_model(p, cache, weight_rounding=False)
    d1 = (zs[0] - cache["z1"]) / np.sqrt(V0["z1"] + 1e-300)
    assert np.max(np.abs(d1)) > 6.0


def test_round_bf16_matches_bit_rounding():
    """round_bf16 equals the snippets' float32 -> bfloat16 bit rounding (ties to even)."""
    import oracle
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 1000), [0.0, 1.0, -1.0]]).astype(np.float32)
    ties = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8)], np.float32)
    v = np.concatenate([v, ties])
    want = oracle.bf16_bits_to_f32(oracle.f32_to_bf16_bits(v)).astype(np.float64)
    assert np.array_equal(cnn.round_bf16(v.astype(np.float64)), want)
    h = cnn.half_ulp_bf16(v.astype(np.float64))
    assert np.all(np.abs(want - v) <= h)


def test_decision_check_accepts_an_emulation_and_rejects_planted_choices():
    """The GPU parity test's decision check (near-tie bound from the deviation model):
    every pooling choice and hidden-layer gate of the float32/bfloat16 emulation passes it,
    some differ from the float64 network's own (so the check is exercised), and choosing
    the smallest element of every window, or flipping a clearly open gate, fails it."""
    from cnn_decisions import NEAR_TIE_SIGMAS, check_pool_decisions, _windows
    rng = np.random.default_rng(40)
    p = cnn.init_params(40)
    for k in p:
        if k.endswith("b"):
            p[k] = rng.normal(0, 0.05, p[k].shape)
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    x = cnn.round_bf16(rng.normal(0, 1, size=(2, 2, 64, 256)))
    _, cache = cnn.forward(p, x)
    V = cnn.deviation_model(p, cache)
    zs, h = _bf16_emulation(p, x)
    n_diff_total = 0
    for k in range(1, 5):
        zw = _windows(zs[k - 1])
        emu = np.where(zw.max(-1) > 0, np.argmax(zw, -1), 255)
        n_diff, n_bad = check_pool_decisions(cache[f"z{k}"], V[f"z{k}"], emu)
        assert n_bad == 0, (k, n_bad)
        n_diff_total += n_diff
        _, n_bad = check_pool_decisions(cache[f"z{k}"], V[f"z{k}"], np.argmin(zw, -1))
        assert n_bad > 0.5 * zw[..., 0].size, (k, n_bad)
    assert n_diff_total > 0
    hv = cache["h"]
    gate = (h + p["f1b"]) > 0
    ok = (gate == (hv > 0)) | (np.abs(hv) <= NEAR_TIE_SIGMAS * np.sqrt(V["h"]))
    assert ok.all()
    j = np.unravel_index(np.argmax(hv), hv.shape)
    flipped = gate.copy()
    flipped[j] = False
    ok = (flipped == (hv > 0)) | (np.abs(hv) <= NEAR_TIE_SIGMAS * np.sqrt(V["h"]))
    assert not ok[j]
