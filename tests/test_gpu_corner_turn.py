"""GPU parity of the corner turn: bit for bit against the oracle, at tile-ragged
sizes and at the 4096-channel, 26,305-sample block of the 24-beam workload."""
import sys

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_27262_amd import spotlight
    return spotlight


@pytest.mark.parametrize("n_t,nch,extra_stride", [(1, 16, 0), (63, 16, 0), (64, 256, 0), (130, 272, 16),
                                                  (1000, 4096, 0), (26305, 4096, 0)])
def test_corner_turn_matches_oracle(spl, n_t, nch, extra_stride):
    print(f"corner turn n_t={n_t} nch={nch}", flush=True)
    rng = np.random.default_rng(n_t + nch)
    x_tc = rng.integers(0, 256, size=(n_t, nch + extra_stride), dtype=np.uint8)
    dev = torch.from_numpy(x_tc).cuda()[:, :nch]
    pitch = (n_t + 255) // 256 * 256
    out = torch.full((nch, pitch), 7, dtype=torch.uint8, device="cuda")
    spl.corner_turn(dev, out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    if n_t * nch <= 1 << 22:
        ref = oracle.corner_turn(x_tc[:, :nch])
    else:
        ref = np.ascontiguousarray(x_tc[:, :nch].T)   # same definition, vectorised for the full block
    assert np.array_equal(got[:, :n_t], ref)
    assert np.all(got[:, n_t:] == 7)    # bytes past n_t untouched


def test_corner_turn_rejects_bad_shapes(spl):
    x = torch.zeros((10, 24), dtype=torch.uint8, device="cuda")
    with pytest.raises(spl.SplError) as ei:
        spl.corner_turn(x)
    assert ei.value.status == spl.SPL_E_UNSUPPORTED
