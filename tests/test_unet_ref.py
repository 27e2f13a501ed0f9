"""Pins of the FP64 U-Net reference: central finite differences of its
hand-derived backward pass, BF16 rounding against torch, and the loss."""
import numpy as np
import pytest

from oracle import unet_ref as U


def test_param_count_matches_library():
    import paper_2510_11508_amd as ni
    assert ni.lib().ni_unet_param_count() == U.param_count()


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e-3, 1000), rng.normal(0, 1e4, 1000)])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.bf16(x), ref)


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_matches_finite_differences(seed):
    rng = np.random.default_rng(seed)
    prm = U.init_params(seed)
    prm[:] += rng.normal(0, 0.01, prm.size)          # non-zero biases too
    feat = rng.normal(0, 1, (1, 16, 16, 6))
    dout = rng.normal(0, 1, (1, 16, 16))
    out, cache = U.forward(prm, feat)
    g = U.backward(prm, cache, dout)
    # probe coordinates in every layer's weights and biases and the head
    offs, o = [], 0
    for ci, co in U.SPECS:
        offs.append((o, 9 * ci * co))
        o += 9 * ci * co
        offs.append((o, co))
        o += co
    offs.append((o, U.HEAD_C + 1))
    eps = 1e-6
    for start, n in offs:
        for idx in rng.integers(start, start + n, size=2):
            p1 = prm.copy(); p1[idx] += eps
            p2 = prm.copy(); p2[idx] -= eps
            f1 = np.sum(U.forward(p1, feat)[0] * dout)
            f2 = np.sum(U.forward(p2, feat)[0] * dout)
            fd = (f1 - f2) / (2 * eps)
            assert abs(fd - g[idx]) <= 1e-5 * max(1.0, abs(fd)), (idx, fd, g[idx])


def test_centred_mse_gradient_and_offset_invariance():
    rng = np.random.default_rng(3)
    pred = rng.normal(0, 1, (2, 8, 8))
    tgt = rng.normal(0, 1, (2, 8, 8))
    lab = rng.integers(-1, 5, (2, 8, 8))
    l0, g = U.centred_mse(pred, tgt, lab)
    # adding a constant per component leaves the loss unchanged
    off = rng.normal(0, 3, 5)
    p2 = pred + np.where(lab >= 0, off[np.maximum(lab, 0)], 0.0)
    assert abs(U.centred_mse(p2, tgt, lab)[0] - l0) < 1e-12
    eps = 1e-6
    for idx in [(0, 1, 2), (1, 7, 7), (0, 4, 0)]:
        p = pred.copy(); p[idx] += eps
        q = pred.copy(); q[idx] -= eps
        fd = (U.centred_mse(p, tgt, lab)[0] - U.centred_mse(q, tgt, lab)[0]) / (2 * eps)
        assert abs(fd - g[idx]) < 1e-7
