"""The allocation-free labelling entry point (ni_label_noalloc) against
ni_label, through the C ABI: bit-identical labels and K on two calls in a
row (the second on a smaller map, so stale scratch contents from the first
would show), maps at the size limit, the size check, and a non-finite
normal inside the mask."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    import paper_2510_11508_amd as ni
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ni.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def both(ctx, s, theta, conn=4):
    import paper_2510_11508_amd as ni
    p = ni.ni_params_default(theta_c_deg=theta, connectivity=conn)
    n, m = dev(s.normals), dev(s.mask)
    ref, Kr, _ = ctx.ni_label(n, m, s.cam.as_dict(), p)
    lab = torch.full(tuple(s.mask.shape), 12345, dtype=torch.int32, device="cuda")
    K = ctx.ni_label_noalloc(n, m, s.cam.as_dict(), lab, p)
    torch.cuda.synchronize()
    return K, lab.cpu().numpy(), Kr, ref.cpu().numpy()


def test_noalloc_labels_equal_ni_label(ctx):
    for name, seed, theta in [("c2", 0, 2.0), ("c1", 1, 2.0), ("c2", 3, 0.5), ("c1", 2, 0.0)]:
        s = synth.make(name, seed)
        print(f"[noalloc] {name} seed {seed} theta {theta}", flush=True)
        K, lab, Kr, ref = both(ctx, s, theta)
        assert K == Kr and np.array_equal(lab, ref)


def test_noalloc_labels_8_connectivity(ctx):
    """8-connectivity: the diagonal edge bits take one more byte per pixel
    of the scratch; at the pixel limit too."""
    for s, theta in [(synth.make("c2", 0), 2.0), (synth.make("c1", 0), 180.0), (synth.tiny(6, 1024, 1024), 2.0)]:
        print(f"[noalloc] 8-connectivity {s.mask.shape} theta {theta}", flush=True)
        K, lab, Kr, ref = both(ctx, s, theta, 8)
        assert K == Kr and np.array_equal(lab, ref)


def test_noalloc_at_the_size_limit(ctx):
    # 1024 x 1024 = 2^20 px and a 4096 x 256 strip (the side limit)
    for H, W in [(1024, 1024), (256, 4096)]:
        s = synth.tiny(5, H, W, "persp")
        print(f"[noalloc] {H}x{W}", flush=True)
        K, lab, Kr, ref = both(ctx, s, 2.0)
        assert K == Kr and np.array_equal(lab, ref)


def test_noalloc_rejects_oversize_and_nonfinite(ctx):
    import paper_2510_11508_amd as ni
    for H, W in [(1025, 1024), (16, 4097)]:
        s = synth.tiny(1, H, W, "ortho")
        lab = torch.empty((H, W), dtype=torch.int32, device="cuda")
        print(f"[noalloc] oversize {H}x{W}", flush=True)
        with pytest.raises(ni.NIError) as ex:
            ctx.ni_label_noalloc(dev(s.normals), dev(s.mask), s.cam.as_dict(), lab)
        assert ex.value.status == ni.NI_E_SHAPE
    s = synth.tiny(2)
    n = s.normals.copy()
    v = np.argwhere(s.mask > 0)[3]
    n[v[0], v[1], 0] = np.nan
    lab = torch.empty(s.mask.shape, dtype=torch.int32, device="cuda")
    print("[noalloc] nan inside the mask", flush=True)
    with pytest.raises(ni.NIError) as ex:
        ctx.ni_label_noalloc(dev(n), dev(s.mask), s.cam.as_dict(), lab)
    assert ex.value.status == ni.NI_E_NONFINITE
    # and a clean call right after (the flag is cleared per call)
    s = synth.make("c1", 0)
    K, lab, Kr, ref = both(ctx, s, 2.0)
    assert K == Kr and np.array_equal(lab, ref)
