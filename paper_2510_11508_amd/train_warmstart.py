"""Train the warm-start U-Net on fills produced by the plain method.

Data: seeded 256x256 crops of 2048x2048 perspective scenes (f = 2400,
40 depth steps, 60 bumps, blob masks; synth.make_patch).  For every patch
the library labels the continuous components and fills them (zero-start
CG at 1e-6); the fill's per-component-centred log-depth is the target.  The
network sees the normals, the mask and the ray directions and is trained
with the per-component centred MSE (it only has to be right up to one
offset per component, which the CG start centring removes anyway).

Every step runs in the HIP library (ni_label, ni_fill, ni_unet_train_step);
this script only batches patches.

  python -m paper_2510_11508_amd.train_warmstart --patches 20000 --epochs 2 \\
      --out paper_2510_11508_amd/weights/unet_warmstart.niunet
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _gen(seed):
    import synth
    s = synth.make_patch(seed, 256)
    return s.normals, s.mask, s.cam.as_dict()


def make_dataset(ctx, pool, n, seed0, log):
    """Patches plus their plain-method fills (targets) and labels."""
    import torch

    import paper_2510_11508_amd as ni
    p = ni.ni_params_default(theta_c_deg=2.0)
    N = np.empty((n, 256, 256, 3), np.float32)
    M = np.empty((n, 256, 256), np.uint8)
    T = np.empty((n, 256, 256), np.float32)
    L = np.empty((n, 256, 256), np.int32)
    K = np.empty(n, np.int32)
    cams = []
    t0 = time.time()
    for i, (nn, mm, cam) in enumerate(pool.imap(_gen, range(seed0, seed0 + n), chunksize=16)):
        dn, dm = torch.from_numpy(nn).cuda(), torch.from_numpy(mm).cuda()
        lab, k, _ = ctx.ni_label(dn, dm, cam, p)
        z, _ = ctx.ni_fill(dn, dm, cam, lab, k, p)
        N[i], M[i], T[i], L[i], K[i] = nn, mm, z.cpu().numpy(), lab.cpu().numpy(), k
        cams.append(cam)
        if (i + 1) % 1000 == 0:
            log(f"data {i + 1}/{n} patches ({time.time() - t0:.0f} s)")
    return N, M, T, L, K, cams


def train(args, log=print):
    import torch

    # the generator workers are forked before this process loads the library
    # or touches the GPU
    with Pool(args.workers) as pool:
        import paper_2510_11508_amd as ni
        ctx = ni.Context(0)
        N, M, T, L, K, cams = make_dataset(ctx, pool, args.patches, args.seed, log)
    ctx.ni_unet_init(args.seed)
    rng = np.random.default_rng(args.seed)
    B = args.batch
    steps = 0
    total = args.epochs * (len(N) // B)
    t0 = time.time()
    hist = []
    for ep in range(args.epochs):
        order = rng.permutation(len(N))
        for bi in range(len(N) // B):
            idx = order[bi * B:(bi + 1) * B]
            lab = L[idx].copy()
            off = np.concatenate([[0], np.cumsum(K[idx])[:-1]]).astype(np.int32)
            lab = np.where(lab >= 0, lab + off[:, None, None], -1).astype(np.int32)
            ncomp = int(K[idx].sum())
            # cosine learning-rate decay
            lr = args.lr * 0.5 * (1.0 + np.cos(np.pi * steps / max(total, 1)))
            loss = ctx.ni_unet_train_step(torch.from_numpy(N[idx]).cuda(), torch.from_numpy(M[idx]).cuda(),
                                          [cams[i] for i in idx], torch.from_numpy(T[idx]).cuda(),
                                          torch.from_numpy(lab).cuda(), ncomp, float(lr))
            hist.append(loss)
            steps += 1
            if steps % 100 == 0:
                log(f"epoch {ep} step {steps}/{total} loss {np.mean(hist[-100:]):.4e} "
                    f"({time.time() - t0:.0f} s)")
    blob = ctx.ni_unet_save()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "wb") as f:
        f.write(blob)
    log(f"saved {args.out} ({len(blob)} bytes); final loss {np.mean(hist[-100:]):.4e}")
    ctx.close()
    return hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--patches", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2510_11508_amd", "weights", "unet_warmstart.niunet"))
    args = ap.parse_args()
    train(args, log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    main()
