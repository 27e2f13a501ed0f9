"""FP64 CPU reference of the warm-start U-Net (forward and backward).

TEST INFRASTRUCTURE ONLY (see oracle/ni_oracle.py).  Plain NumPy: each 3x3
convolution is a sum over its nine taps of shifted matrix products; the
backward pass is derived by hand (chain rule per layer) and pinned by finite
differences in tests/test_unet_ref.py.

With bf16=True the reference rounds exactly where the HIP kernels store in
BF16 (input features, weights, every conv output, data gradients), so the
two implementations can be compared far tighter than the BF16 unit
roundoff: what remains are FP32 accumulation-order effects.

Parameter vector layout (FP32 on the device, FP64 here): for each of the
14 convolutions W[tap][ci][co] (tap = 3*dy + dx over the 3x3 window, ci
over the real input channels) then b[co]; then the 1x1 head w[16], b.
"""
from __future__ import annotations

import numpy as np

SPECS = [(6, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128),
         (192, 64), (64, 64), (96, 32), (32, 32), (48, 16), (16, 16)]
HEAD_C = 16


def param_count():
    return sum(9 * ci * co + co for ci, co in SPECS) + HEAD_C + 1


def unpack(prm):
    prm = np.asarray(prm, np.float64)
    out, o = [], 0
    for ci, co in SPECS:
        w = prm[o:o + 9 * ci * co].reshape(9, ci, co)
        o += 9 * ci * co
        b = prm[o:o + co]
        o += co
        out.append((w, b))
    hw = prm[o:o + HEAD_C]
    hb = prm[o + HEAD_C]
    return out, hw, hb


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.asarray(x, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(x, w, b):
    """x [B,H,W,Ci], w [9,Ci,Co], zero padding 1."""
    B, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.broadcast_to(b, (B, H, W, w.shape[2])).copy() if b is not None else np.zeros((B, H, W, w.shape[2]))
    for tap in range(9):
        dy, dx = divmod(tap, 3)
        out += xp[:, dy:dy + H, dx:dx + W, :] @ w[tap]
    return out


def conv3x3_bwd(x, w, g):
    """Gradients of sum(g * conv3x3(x, w, b)): (dx, dw, db)."""
    B, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    g2 = g.reshape(-1, g.shape[3])
    for tap in range(9):
        dy, dx = divmod(tap, 3)
        win = xp[:, dy:dy + H, dx:dx + W, :]
        dw[tap] = win.reshape(-1, win.shape[3]).T @ g2
        dxp[:, dy:dy + H, dx:dx + W, :] += g @ w[tap].T
    return dxp[:, 1:-1, 1:-1, :], dw, g2.sum(0)


def pool(x):
    """2x2 max pool; argmax = first maximum in the order (0,0),(0,1),(1,0),(1,1)."""
    B, H, W, C = x.shape
    q = x.reshape(B, H // 2, 2, W // 2, 2, C).transpose(0, 1, 3, 2, 4, 5).reshape(B, H // 2, W // 2, 4, C)
    idx = np.argmax(q, axis=3)
    return np.take_along_axis(q, idx[:, :, :, None, :], 3)[:, :, :, 0, :], idx


def pool_bwd(g, idx, shape):
    B, H, W, C = shape
    d = np.zeros((B, H // 2, W // 2, 4, C))
    np.put_along_axis(d, idx[:, :, :, None, :], g[:, :, :, None, :], 3)
    return d.reshape(B, H // 2, W // 2, 2, 2, C).transpose(0, 1, 3, 2, 4, 5).reshape(B, H, W, C)


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_bwd(g):
    B, H, W, C = g.shape
    return g.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def forward(prm, feat, bf=False):
    """feat [B,H,W,6] -> (out [B,H,W], cache)."""
    layers, hw, hb = unpack(prm)
    R = bf16 if bf else (lambda a: np.asarray(a, np.float64))
    if bf:
        layers = [(bf16(w), np.asarray(b, np.float32).astype(np.float64)) for w, b in layers]
    c = {"layers": layers, "hw": hw, "bf": bf}

    def cv(l, x):
        w, b = layers[l]
        return R(np.maximum(conv3x3(x, w, b), 0.0))

    x = R(feat)
    c["x"] = x
    c["e0a"] = cv(0, x)
    c["e0b"] = cv(1, c["e0a"])
    c["p0"], c["i0"] = pool(c["e0b"])
    c["e1a"] = cv(2, c["p0"])
    c["e1b"] = cv(3, c["e1a"])
    c["p1"], c["i1"] = pool(c["e1b"])
    c["e2a"] = cv(4, c["p1"])
    c["e2b"] = cv(5, c["e2a"])
    c["p2"], c["i2"] = pool(c["e2b"])
    c["e3a"] = cv(6, c["p2"])
    c["e3b"] = cv(7, c["e3a"])
    c["cat2"] = np.concatenate([up(c["e3b"]), c["e2b"]], axis=3)
    c["d2a"] = cv(8, c["cat2"])
    c["d2b"] = cv(9, c["d2a"])
    c["cat1"] = np.concatenate([up(c["d2b"]), c["e1b"]], axis=3)
    c["d1a"] = cv(10, c["cat1"])
    c["d1b"] = cv(11, c["d1a"])
    c["cat0"] = np.concatenate([up(c["d1b"]), c["e0b"]], axis=3)
    c["d0a"] = cv(12, c["cat0"])
    c["d0b"] = cv(13, c["d0a"])
    out = c["d0b"] @ hw + hb
    c["hb"] = hb
    return out, c


def output_magnitude(c):
    """Per pixel, the sum of the magnitudes of the head's terms:
    |d0b| . |w_head| + |b_head| (the scale of the rounding error a sum of
    those terms can carry)."""
    hw = c["hw"]
    return np.abs(c["d0b"]) @ np.abs(hw) + abs(c.get("hb", 0.0))


def backward(prm, c, dout, magnitudes=False):
    """Gradient of sum(dout * out) w.r.t. the parameter vector.  With
    magnitudes=True, also the same contractions over absolute values
    (sum_pixels |x| |delta| per weight, sum |delta| per bias), the scale of
    each gradient entry's rounding error."""
    layers, hw = c["layers"], c["hw"]
    R = bf16 if c["bf"] else (lambda a: np.asarray(a, np.float64))
    grads = [None] * len(SPECS)
    mags = [None] * len(SPECS)

    def cb(l, x, y, dy, need_dx=True):
        g = dy * (y > 0)
        dx, dw, db = conv3x3_bwd(x, layers[l][0], g)
        grads[l] = (dw, db)
        if magnitudes:
            _, mw, mb = conv3x3_bwd(np.abs(x), np.abs(layers[l][0]), np.abs(g))
            mags[l] = (mw, mb)
        return R(dx) if need_dx else None

    dhw = np.einsum("bhwc,bhw->c", c["d0b"], dout)
    dhb = dout.sum()
    d = R(dout[..., None] * hw)
    d = cb(13, c["d0a"], c["d0b"], d)
    dcat0 = cb(12, c["cat0"], c["d0a"], d)
    d = R(up_bwd(dcat0[..., :32]))
    d = cb(11, c["d1a"], c["d1b"], d)
    dcat1 = cb(10, c["cat1"], c["d1a"], d)
    d = R(up_bwd(dcat1[..., :64]))
    d = cb(9, c["d2a"], c["d2b"], d)
    dcat2 = cb(8, c["cat2"], c["d2a"], d)
    d = R(up_bwd(dcat2[..., :128]))
    d = cb(7, c["e3a"], c["e3b"], d)
    d = cb(6, c["p2"], c["e3a"], d)
    d = R(dcat2[..., 128:] + pool_bwd(d, c["i2"], c["e2b"].shape))
    d = cb(5, c["e2a"], c["e2b"], d)
    d = cb(4, c["p1"], c["e2a"], d)
    d = R(dcat1[..., 64:] + pool_bwd(d, c["i1"], c["e1b"].shape))
    d = cb(3, c["e1a"], c["e1b"], d)
    d = cb(2, c["p0"], c["e1a"], d)
    d = R(dcat0[..., 32:] + pool_bwd(d, c["i0"], c["e0b"].shape))
    d = cb(1, c["e0a"], c["e0b"], d)
    cb(0, c["x"], c["e0a"], d, need_dx=False)
    out = []
    for dw, db in grads:
        out.append(dw.ravel())
        out.append(db)
    out.append(dhw)
    out.append(np.array([dhb]))
    if not magnitudes:
        return np.concatenate(out)
    mag = []
    for mw, mb in mags:
        mag.append(mw.ravel())
        mag.append(mb)
    mag.append(np.einsum("bhwc,bhw->c", np.abs(c["d0b"]), np.abs(dout)))
    mag.append(np.array([np.abs(dout).sum()]))
    return np.concatenate(out), np.concatenate(mag)


def init_params(seed):
    """He-normal weights, zero biases (CPU-side helper for tests)."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in SPECS:
        parts.append(rng.normal(0, np.sqrt(2.0 / (9 * ci)), 9 * ci * co))
        parts.append(np.zeros(co))
    parts.append(rng.normal(0, np.sqrt(1.0 / HEAD_C), HEAD_C))
    parts.append(np.zeros(1))
    return np.concatenate(parts)


def centred_mse(pred, target, labels):
    """Loss of the warm-start training: per-component centred squared error
    over valid pixels, and its gradient w.r.t. pred."""
    v = labels >= 0
    lab = labels[v]
    e = (pred - target)[v]
    K = int(lab.max()) + 1 if lab.size else 0
    s = np.bincount(lab, weights=e, minlength=K)
    n = np.bincount(lab, minlength=K)
    ec = e - (s / np.maximum(n, 1))[lab]
    loss = float(np.sum(ec * ec) / max(v.sum(), 1))
    g = np.zeros_like(pred)
    g[v] = 2.0 * ec / max(v.sum(), 1)
    return loss, g
