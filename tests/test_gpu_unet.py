"""Warm-start U-Net on the GPU (through the C ABI) against the FP64 reference.

Forward / backward are compared with the reference in its BF16-emulating
mode (it rounds where the kernels store BF16), so what remains is FP32
accumulation order plus the rare BF16 rounding flip it causes: relative L2
error bounds 1e-2 (output) and 3e-2 (per-layer gradients)."""
import sys

import numpy as np
import pytest

from oracle import unet_ref as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def log(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2510_11508_amd as ni
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ni.Context(0)
    c.ni_unet_init(1234)
    yield c
    c.close()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def test_forward_backward_match_reference(ctx):
    rng = np.random.default_rng(0)
    prm = ctx.ni_unet_get_params().astype(np.float64)
    prm[:] += rng.normal(0, 0.01, prm.size)  # non-zero biases
    ctx.ni_unet_set_params(prm.astype(np.float32))
    prm = ctx.ni_unet_get_params().astype(np.float64)
    feat = rng.normal(0, 1, (2, 16, 24, 6)).astype(np.float32)
    log("[unet] forward 2x16x24")
    out = ctx.ni_unet_forward(torch.from_numpy(feat).cuda()).cpu().numpy()
    ref, cache = U.forward(prm, feat.astype(np.float64), bf=True)
    assert rel(out, ref) < 1e-2, rel(out, ref)
    dout = rng.normal(0, 1, out.shape).astype(np.float32)
    log("[unet] backward")
    g = ctx.ni_unet_backward(torch.from_numpy(dout).cuda()).cpu().numpy().astype(np.float64)
    gr = U.backward(prm, cache, dout.astype(np.float64))
    o, errs = 0, []
    for l, (ci, co) in enumerate(U.SPECS):
        nw = 9 * ci * co
        errs.append((l, round(rel(g[o:o + nw], gr[o:o + nw]), 4), round(rel(g[o + nw:o + nw + co], gr[o + nw:o + nw + co]), 4)))
        o += nw + co
    errs.append(("head", round(rel(g[o:], gr[o:]), 4), 0.0))
    log(f"[unet] grad rel err (layer, weights, bias): {errs}")
    assert all(ew < 3e-2 and eb < 3e-2 for _, ew, eb in errs), errs


def test_train_step_reduces_loss(ctx):
    import paper_2510_11508_amd as ni
    import synth
    rng = np.random.default_rng(1)
    ctx.ni_unet_init(7)
    B, S = 2, 32
    samples = [synth.make_patch(i, S) for i in range(B)]
    n = np.stack([s.normals for s in samples])
    m = np.stack([s.mask for s in samples])
    # target: smooth log-depth; labels: one component per patch
    t = np.stack([np.where(s.mask > 0, np.log(s.depth_gt), 0.0) for s in samples]).astype(np.float32)
    lab = np.stack([np.where(s.mask > 0, i, -1) for i, s in enumerate(samples)]).astype(np.int32)
    args = [torch.from_numpy(a).cuda() for a in (n, m)]
    tt, ll = torch.from_numpy(t).cuda(), torch.from_numpy(lab).cuda()
    cams = [s.cam.as_dict() for s in samples]
    losses = []
    for k in range(30):
        losses.append(ctx.ni_unet_train_step(args[0], args[1], cams, tt, ll, B, 1e-3))
    log(f"[unet] loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert np.isfinite(losses).all() and losses[-1] < 0.5 * losses[0]


def test_save_load_roundtrip_and_predict(ctx):
    import paper_2510_11508_amd as ni
    import synth
    s = synth.make("c2", 0)
    ctx.ni_unet_init(99)
    blob = ctx.ni_unet_save()
    assert len(blob) == ni.lib().ni_unet_blob_size() and blob[:8] == b"NIUNET01"
    n, m = torch.from_numpy(s.normals).cuda(), torch.from_numpy(s.mask).cuda()
    a = ctx.ni_unet_predict(n, m, s.cam.as_dict()).cpu().numpy()
    ctx.ni_unet_init(5)
    ctx.ni_unet_load(blob)
    b = ctx.ni_unet_predict(n, m, s.cam.as_dict()).cpu().numpy()
    assert a.shape == s.mask.shape and np.all(np.isfinite(a)) and np.array_equal(a, b)
    with pytest.raises(ni.NIError):
        ctx.ni_unet_load(b"NIUNET01" + b"\x00" * 10)


def test_warm_start_reaches_the_same_solution(ctx):
    """Any start (here an untrained model) must converge to the same fill."""
    import paper_2510_11508_amd as ni
    import synth
    from oracle import ni_oracle as O
    s = synth.make("c2", 1)
    ctx.ni_unet_init(3)
    n, m = torch.from_numpy(s.normals).cuda(), torch.from_numpy(s.mask).cuda()
    e = O.edges(s.normals, s.mask, s.cam, 2.0)
    lab, K = O.labels(e)
    zref = O.fill(e, lab, K)
    log("[unet] warm fill")
    z, rep = ctx.ni_fill(n, m, s.cam.as_dict(), torch.from_numpy(lab).cuda(), K, ni.ni_params_default(warm_start=1))
    v = s.mask > 0
    assert np.max(np.abs(z.cpu().numpy()[v] - zref[v])) <= 1e-6 + 1e-4
