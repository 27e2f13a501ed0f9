"""What the trained warm-start network gains over the plain method.

The committed weights (trained on 20k seeded 256x256 patches of c3-style
scenes, targets = the plain method's fill) are loaded through the C ABI.
On held-out maps the test measures:

- the per-component-centred mean squared error of the network's log-depth
  against the plain fill, next to that of the zero start;
- the fill work (pixel-iterations) and the final depth with warm_start = 1
  and 0.

What is asserted: the prediction is closer to the fill than the zero start
(the network learned something); the warm start never changes the answer
beyond the parity bound; it does not cost more than 5% extra fill work.
The measured gains are printed.  A start that is worse than zero for a
component is dropped by the library, so the warm start cannot slow a
component down.
"""
import os
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2510_11508_amd",
                       "weights", "unet_warmstart.niunet")


def log(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2510_11508_amd as ni
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained weights")
    c = ni.Context(0)
    c.ni_unet_load(open(WEIGHTS, "rb").read())
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def centred_mse(pred, target, labels):
    v = labels >= 0
    lab = labels[v]
    e = (pred - target)[v].astype(np.float64)
    K = int(lab.max()) + 1
    m = np.bincount(lab, weights=e, minlength=K) / np.maximum(np.bincount(lab, minlength=K), 1)
    return float(np.mean((e - m[lab]) ** 2))


@pytest.mark.parametrize("seed", [50001, 50002, 50003])
def test_prediction_beats_zero_start_on_held_out_patches(ctx, seed):
    import paper_2510_11508_amd as ni
    s = synth.make_patch(seed, 256)
    p = ni.ni_params_default(theta_c_deg=2.0)
    n, m, cam = dev(s.normals), dev(s.mask), s.cam.as_dict()
    log(f"[warm start] patch seed {seed}")
    lab, K, _ = ctx.ni_label(n, m, cam, p)
    z, _ = ctx.ni_fill(n, m, cam, lab, K, p)
    pred = ctx.ni_unet_predict(n, m, cam).cpu().numpy()
    lab = lab.cpu().numpy()
    z = z.cpu().numpy()
    l_net = centred_mse(pred, z, lab)
    l_zero = centred_mse(np.zeros_like(z), z, lab)
    log(f"  centred MSE vs plain fill: network {l_net:.3e}, zero start {l_zero:.3e} "
        f"(ratio {l_net / l_zero:.3f})")
    assert l_net < l_zero


def test_warm_start_gain_on_c2(ctx):
    import paper_2510_11508_amd as ni
    s = synth.make("c2", 3)
    n, m, cam = dev(s.normals), dev(s.mask), s.cam.as_dict()
    out = {}
    for warm in (0, 1):
        p = ni.ni_params_default(theta_c_deg=2.0, irls_iters=15, warm_start=warm)
        log(f"[warm start] c2 seed 3 warm_start={warm}")
        out[warm] = ctx.ni_integrate(n, m, cam, p)
    r0, r1 = out[0]["report"], out[1]["report"]
    v = s.mask > 0
    d0, d1 = out[0]["depth"].cpu().numpy()[v], out[1]["depth"].cpu().numpy()[v]
    log(f"  fill pixel-iterations: zero {r0['fill_px_iters']}, warm {r1['fill_px_iters']} "
        f"({r1['fill_px_iters'] / max(r0['fill_px_iters'], 1):.3f}x); largest component iterations "
        f"{r0['fill_iters_max']} -> {r1['fill_iters_max']}; starts dropped {r1['warm_fallbacks']}")
    log(f"  fill time: zero {r0['ms_fill_small'] + r0['ms_fill_large']:.2f} ms, warm "
        f"{r1['ms_warm'] + r1['ms_fill_small'] + r1['ms_fill_large']:.2f} ms (incl. network {r1['ms_warm']:.2f} ms)")
    assert np.max(np.abs(d1 - d0) / np.abs(d0)) <= 1e-4
    assert r1["fill_px_iters"] <= 1.05 * r0["fill_px_iters"]
