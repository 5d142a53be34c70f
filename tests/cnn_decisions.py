"""Validity check of a BF16 evaluation's discrete decisions against the float64 ranker
network (test helper).

Max pooling and ReLU are discrete decisions: an evaluation in another precision may take
a different one wherever the float64 values are nearly tied.  Such a decision is
accepted only inside the bound the BF16 deviation model gives
(oracle.cnn.deviation_model)."""
import numpy as np

# A kernel decision (pool window choice, ReLU gate) may differ from the float64 network's
# own only where the float64 values are tied within this many standard deviations of the
# BF16 deviation model (oracle.cnn.deviation_model, pinned to lie within 6 deviations of
# an emulation of the stated arithmetic at every element).
NEAR_TIE_SIGMAS = 6.0


def _windows(a):
    n, c, h, w = a.shape
    return a.reshape(n, c, h // 2, 2, w // 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(n, c, h // 2, w // 2, 4)


def check_pool_decisions(z, var, karg):
    """Every kernel window choice must be one the float64 values allow within the bound.
    A choice j (0..3) needs z_j + S s_j > 0 and z_m - z_j <= S (s_m + s_j) for every m of
    the window; 255 (no positive element) needs z_m <= S s_m for every m.  Returns the
    number of windows whose choice differs from the float64 network's own and the number
    of choices outside the bound."""
    S = NEAR_TIE_SIGMAS
    zw, sw = _windows(z), np.sqrt(_windows(var))
    own = np.where(zw.max(-1) > 0, np.argmax(zw, -1), 255)
    ka = np.asarray(karg).astype(np.int64)
    none = ka == 255
    j = np.minimum(ka, 3)[..., None]
    zj = np.take_along_axis(zw, j, -1)
    sj = np.take_along_axis(sw, j, -1)
    ok_pick = ((zj + S * sj)[..., 0] > 0) & np.all(zw - zj <= S * (sw + sj), axis=-1)
    ok_none = np.all(zw <= S * sw, axis=-1)
    ok = np.where(none, ok_none, ok_pick)
    return int(np.count_nonzero(ka != own)), int(np.count_nonzero(~ok))
