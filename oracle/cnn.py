"""Float64 reference of the candidate ranker (test infrastructure only).

A small CNN stands in for the paper's FETCH classifier (classification section):
its input is the two 64x256 feature planes of a candidate (DM-time and
frequency-time), and it outputs one logit; a probability >= 0.5 keeps the
candidate.  Layers, in order:
  4 x [3x3 convolution, stride 1, zero padding 1, bias -> ReLU -> 2x2 max pool]
      with channels 2 -> 32 -> 32 -> 32 -> 32   (64x256 -> 4x16)
  flatten (channel, row, column) -> 2048
  fully connected 2048 -> 64, bias -> ReLU -> fully connected 64 -> 1, bias
Loss: binary cross-entropy on the logit, averaged over the batch.
Max-pool ties go to the first element of the window in row-major order.
Parameters are a dict of float64 arrays:
  c{k}w [32][Cin][3][3], c{k}b [32] (k = 1..4), f1w [64][2048], f1b [64],
  f2w [1][64], f2b [1].
Plain numpy: convolution as a sum of 9 shifted products, no fusion or blocking.
"""
from __future__ import annotations

import numpy as np

CONV_CHANNELS = (2, 32, 32, 32, 32)
IN_H, IN_W = 64, 256
FC_IN, FC_HIDDEN = 2048, 64
PARAM_ORDER = ("c1w", "c1b", "c2w", "c2b", "c3w", "c3b", "c4w", "c4b", "f1w", "f1b", "f2w", "f2b")


def param_shapes() -> dict:
    s = {}
    for k in range(4):
        cin, cout = CONV_CHANNELS[k], CONV_CHANNELS[k + 1]
        s[f"c{k + 1}w"] = (cout, cin, 3, 3)
        s[f"c{k + 1}b"] = (cout,)
    s["f1w"] = (FC_HIDDEN, FC_IN)
    s["f1b"] = (FC_HIDDEN,)
    s["f2w"] = (1, FC_HIDDEN)
    s["f2b"] = (1,)
    return s


def init_params(seed: int = 0) -> dict:
    """He-uniform weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in param_shapes().items():
        if name.endswith("b"):
            p[name] = np.zeros(shp)
        else:
            fan_in = int(np.prod(shp[1:]))
            lim = np.sqrt(6.0 / fan_in)
            p[name] = rng.uniform(-lim, lim, size=shp)
    return p


def flatten_params(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], np.float64).ravel() for k in PARAM_ORDER])


def unflatten_params(v: np.ndarray) -> dict:
    out, o = {}, 0
    for k in PARAM_ORDER:
        shp = param_shapes()[k]
        n = int(np.prod(shp))
        out[k] = np.asarray(v[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def n_params() -> int:
    return sum(int(np.prod(s)) for s in param_shapes().values())


def conv3x3(x, w, b):
    n, c, h, wd = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.zeros((n, w.shape[0], h, wd))
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("nchw,oc->nohw", xp[:, :, ky:ky + h, kx:kx + wd], w[:, :, ky, kx])
    return out + b[None, :, None, None]


def conv3x3_backward(x, w, gout):
    """Gradients of conv3x3 with respect to input, weight and bias."""
    n, c, h, wd = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            gw[:, :, ky, kx] = np.einsum("nohw,nchw->oc", gout, xp[:, :, ky:ky + h, kx:kx + wd])
            gxp[:, :, ky:ky + h, kx:kx + wd] += np.einsum("nohw,oc->nchw", gout, w[:, :, ky, kx])
    return gxp[:, :, 1:-1, 1:-1], gw, gout.sum(axis=(0, 2, 3))


def maxpool2(x):
    """2x2 max pool and the window position (0..3, row-major) of each maximum."""
    n, c, h, w = x.shape
    win = x.reshape(n, c, h // 2, 2, w // 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(n, c, h // 2, w // 2, 4)
    arg = np.argmax(win, axis=-1)          # first maximum on ties
    return np.take_along_axis(win, arg[..., None], axis=-1)[..., 0], arg


def maxpool2_backward(gout, arg, shape):
    n, c, h, w = shape
    g = np.zeros((n, c, h // 2, w // 2, 5))   # slot 4 collects windows marked 255
    a = np.where(np.asarray(arg) == 255, 4, arg).astype(np.int64)
    np.put_along_axis(g, a[..., None], gout[..., None], axis=-1)
    g = g[..., :4]
    return g.reshape(n, c, h // 2, w // 2, 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(n, c, h, w)


def pool_given(r, arg):
    """2x2 max pool whose window choices are given: arg (0..3, row-major) picks the
    element, 255 gives 0 and marks a window through which no gradient flows.  A given
    choice 0..3 also decides the ReLU gate: the gradient passes to that element."""
    n, c, h, w = r.shape
    win = r.reshape(n, c, h // 2, 2, w // 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(n, c, h // 2, w // 2, 4)
    a = np.asarray(arg).astype(np.int64)
    out = np.take_along_axis(win, np.minimum(a, 3)[..., None], axis=-1)[..., 0]
    out[a == 255] = 0.0
    return out


def forward(p: dict, x: np.ndarray, pool_args=None, fc_gate=None):
    """x [N][2][64][256] -> logits [N] and the saved activations.

    pool_args (optional): the max-pool window choices of each layer, [N][32][H/2][W/2]
    (0..3, or 255 for a window without a positive element), for comparing with an
    implementation that decided near-tied maxima, or the sign of a near-zero
    pre-activation, in another precision: the arg-max and the ReLU gate are discrete
    decisions, so both sides must take the same ones.  With given choices the gradient
    passes to the chosen element of every window not marked 255.
    fc_gate (optional): bool [N][64], the given ReLU gates of the hidden layer (open:
    the unit's value and gradient pass; closed: both are 0)."""
    cache = {"x0": np.asarray(x, np.float64), "given": pool_args is not None}
    a = cache["x0"]
    for k in range(1, 5):
        z = conv3x3(a, p[f"c{k}w"], p[f"c{k}b"])
        r = np.maximum(z, 0.0)
        if pool_args is None:
            a, arg = maxpool2(r)
        else:
            arg = np.asarray(pool_args[k - 1])
            a = pool_given(r, arg)
        cache[f"z{k}"], cache[f"arg{k}"], cache[f"x{k}"] = z, arg, a
    f = a.reshape(a.shape[0], -1)
    h = f @ p["f1w"].T + p["f1b"]
    gate = (h > 0) if fc_gate is None else np.asarray(fc_gate, bool)
    hr = np.where(gate, np.maximum(h, 0.0), 0.0)
    cache["gate"] = gate
    logit = (hr @ p["f2w"].T + p["f2b"])[:, 0]
    cache.update(f=f, h=h, hr=hr)
    return logit, cache


def bce_with_logits(logit, y):
    """Mean of max(z, 0) - z*y + log(1 + exp(-|z|))."""
    z = np.asarray(logit, np.float64)
    return float(np.mean(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def backward(p: dict, cache: dict, y: np.ndarray) -> tuple[float, dict]:
    """Loss and gradients of the mean BCE loss with respect to every parameter."""
    x0 = cache["x0"]
    n = x0.shape[0]
    hr, h, f = cache["hr"], cache["h"], cache["f"]
    logit = (hr @ p["f2w"].T + p["f2b"])[:, 0]
    loss = bce_with_logits(logit, y)
    g = {}
    gz = (1.0 / (1.0 + np.exp(-logit)) - y) / n          # d loss / d logit
    g["f2w"] = gz[None, :] @ hr
    g["f2b"] = np.array([gz.sum()])
    ghr = gz[:, None] * p["f2w"]
    gh = ghr * cache.get("gate", h > 0)
    g["f1w"] = gh.T @ f
    g["f1b"] = gh.sum(axis=0)
    gf = gh @ p["f1w"]
    ga = gf.reshape(cache["x4"].shape)
    for k in range(4, 0, -1):
        z = cache[f"z{k}"]
        gr = maxpool2_backward(ga, cache[f"arg{k}"], z.shape)
        gzk = gr if cache.get("given") else gr * (z > 0)
        xin = cache[f"x{k - 1}"]
        ga, g[f"c{k}w"], g[f"c{k}b"] = conv3x3_backward(xin, p[f"c{k}w"], gzk)
    return loss, g


def flops_forward_per_sample() -> int:
    """Multiply-adds x 2 of one forward pass (convolutions and fully connected layers)."""
    tot, h, w = 0, IN_H, IN_W
    for k in range(4):
        tot += 2 * 9 * CONV_CHANNELS[k] * CONV_CHANNELS[k + 1] * h * w
        h, w = h // 2, w // 2
    return tot + 2 * FC_IN * FC_HIDDEN + 2 * FC_HIDDEN


# --------------------------------------------------------------------------
# How far an evaluation with BF16 operands may lie from this float64 network
# --------------------------------------------------------------------------
BF16_SIGNIFICAND_BITS = 8      # bfloat16: 7 stored bits + the implicit one
FP32_UNIT_ROUNDOFF = 2.0 ** -24


def round_bf16(a):
    """float64 values rounded to the nearest bfloat16 (ties to even), as float64."""
    a = np.asarray(a, np.float64)
    m, e = np.frexp(a)                              # a = m 2^e, 0.5 <= |m| < 1
    scale = np.ldexp(1.0, BF16_SIGNIFICAND_BITS - e)
    with np.errstate(invalid="ignore", over="ignore"):
        r = np.rint(a * scale) / scale              # rint: ties to even
    return np.where(a == 0.0, 0.0, r)


def half_ulp_bf16(a):
    """Half the spacing of bfloat16 numbers at |a|: the largest error of rounding a to
    the nearest bfloat16 (0 at 0)."""
    a = np.asarray(a, np.float64)
    _, e = np.frexp(a)                              # 2^(e-1) <= |a| < 2^e
    return np.where(a == 0.0, 0.0, np.ldexp(1.0, e - 1 - BF16_SIGNIFICAND_BITS))


def deviation_model(p: dict, cache: dict, weight_rounding: bool = True) -> dict:
    """Variance of the difference between this network's pre-activations and those of an
    evaluation that rounds every convolution and FC1 weight to bfloat16, rounds every
    pooled activation to bfloat16 and accumulates in float32 (the ranker ABI's stated
    arithmetic), given this network's forward cache.

    Model: each rounding error is independent, with variance (the rounding error of that
    weight)^2 for the weights (known exactly) and h^2/3 (uniform within half an ulp h of
    the oracle's value) for the pooled activations; errors propagate linearly through each
    layer (Var dz = sum w^2 Var da + sum a^2 dw^2); max pooling passes on the largest
    variance of its window; float32 accumulation adds at most K 2^-24 sum |a w| for K
    products, counted as a variance term of that size squared.  Returns the variances
    "z1".."z4" (conv pre-activations [N][32][H][W]), "h" (FC1 pre-activations [N][64])
    and "logit" [N]."""
    out = {}
    Va = np.zeros_like(cache["x0"])
    zero_b = np.zeros(CONV_CHANNELS[1])
    for k in range(1, 5):
        w = p[f"c{k}w"]
        dw = (round_bf16(w) - w) if weight_rounding else np.zeros_like(w)
        xin = cache[f"x{k - 1}"]
        K = 9 * w.shape[1]
        acc = K * FP32_UNIT_ROUNDOFF * conv3x3(np.abs(xin), np.abs(w), zero_b)
        Vz = conv3x3(Va, w * w, zero_b) + conv3x3(xin * xin, dw * dw, zero_b) + acc * acc
        out[f"z{k}"] = Vz
        n, c, hgt, wid = Vz.shape
        win = Vz.reshape(n, c, hgt // 2, 2, wid // 2, 2).max(axis=(3, 5))
        Va = win + half_ulp_bf16(cache[f"x{k}"]) ** 2 / 3.0
    f = cache["f"]
    Vf = Va.reshape(Va.shape[0], -1)
    w1 = p["f1w"]
    dw1 = (round_bf16(w1) - w1) if weight_rounding else np.zeros_like(w1)
    acc = FC_IN * FP32_UNIT_ROUNDOFF * (np.abs(f) @ np.abs(w1).T)
    Vh = Vf @ (w1 * w1).T + (f * f) @ (dw1 * dw1).T + acc * acc
    out["h"] = Vh
    out["logit"] = Vh @ (p["f2w"][0] ** 2)
    return out


def forward_bf16(p: dict, x: np.ndarray):
    """The network evaluated with the ranker ABI's stated arithmetic, in numpy float32:
    convolution and FC1 weights rounded to bfloat16, products summed in float32, biases
    added in float32, pooled activations rounded to bfloat16, FC2 in float32.  Returns
    the logits [N] (float64), the conv pre-activations z1..z4 and the FC1
    pre-activations h (float64 copies of the float32 values).  Written independently of
    deviation_model, which is pinned against it."""
    wb = {k: round_bf16(v).astype(np.float32) for k, v in p.items()}
    a = np.asarray(x).astype(np.float32)
    zs = []
    for k in range(1, 5):
        w, b = wb[f"c{k}w"], np.asarray(p[f"c{k}b"]).astype(np.float32)
        n, c, h, wd = a.shape
        ap = np.pad(a, ((0, 0), (0, 0), (1, 1), (1, 1)))
        z = np.zeros((n, w.shape[0], h, wd), np.float32)
        for ky in range(3):
            for kx in range(3):
                z += np.einsum("nchw,oc->nohw", ap[:, :, ky:ky + h, kx:kx + wd], w[:, :, ky, kx]).astype(np.float32)
        z += b[None, :, None, None]
        zs.append(z.astype(np.float64))
        r = np.maximum(z, np.float32(0))
        pooled = r.reshape(n, w.shape[0], h // 2, 2, wd // 2, 2).max(axis=(3, 5))
        a = round_bf16(pooled).astype(np.float32)
    f = a.reshape(a.shape[0], -1)
    h = (f @ wb["f1w"].T).astype(np.float32) + np.asarray(p["f1b"]).astype(np.float32)
    hr = np.maximum(h, np.float32(0))
    logit = (hr @ np.asarray(p["f2w"]).astype(np.float32).T)[:, 0] + np.float32(np.asarray(p["f2b"])[0])
    return logit.astype(np.float64), zs, h.astype(np.float64)

