"""Benchmark: valid Mpixels/s integrated at a 1e-6 relative CG residual.

One step = one ni_integrate call on one synthetic normal map already
resident in HBM (labels, fill, relative-scale IRLS, output), every fill
system stopped at ||r_c|| <= 1e-6 ||b_c||.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c3|c5]

The roofline object describes one PCG iteration of the large fill
components.  By default they are solved together by one PCG preconditioned
by a multigrid V-cycle (aggregates of 2x2 pixel blocks per component); one
iteration is the cycle's launches on every level plus the (p, q) and
(x, r) updates on level 0.  Its algorithmic bytes come from the library
(ni_report.fill_mg_bytes: per level, the CSR rows, entries and FP64
vectors each kernel must read or write once; neighbour re-reads are cache
hits).  achieved = those bytes / the event-timed duration of one iteration
(the solve's launches, batched, divided by the iterations).  With the
Jacobi preconditioner (fill_precond = 0) the unit is the two- or
three-launch chunked iteration (k_lg_*) at 64 B per active pixel.
traffic = calibrated FETCH_SIZE + WRITE_SIZE per iteration from committed
counter runs (profiles/fill_mg_traffic_<workload>.json), while they match
the kernel sources.  The CPU baseline is the FP64 oracle on this host.

With a trained warm-start model (paper_2510_11508_amd/weights/, or
--model) the same map is also integrated with warm_start = 1 and the
report compares the two at the same 1e-6 residual (relative to ||b||):
speedup = wall(zero start) / wall(warm start incl. network inference).
"""
import os

# the oracle's CPU baseline is timed single-threaded: pin BLAS pools before numpy loads
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import argparse
import hashlib
import json
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "valid Mpixels/s integrated at 1e-6 residual; warm-start vs plain CG speedup"
HBM_PEAK_GBS = 8000.0
CG_BYTES_PER_PX_ITER = 64
DEFAULT_MODEL = os.path.join(ROOT, "paper_2510_11508_amd", "weights", "unet_warmstart.niunet")
# forward multiply-adds per input pixel of the warm-start U-Net: 3x3
# convolutions (cin -> cout) at full, 1/4, 1/16 and 1/64 resolution, plus
# the 1x1 head
UNET_LEVELS = [(1, [(6, 16), (16, 16), (48, 16), (16, 16)]), (4, [(16, 32), (32, 32), (96, 32), (32, 32)]),
               (16, [(32, 64), (64, 64), (192, 64), (64, 64)]), (64, [(64, 128), (128, 128)])]
UNET_FLOP_PER_PX = 2 * (sum(9 * ci * co / div for div, convs in UNET_LEVELS for ci, co in convs) + 16)
BF16_PEAK_TFLOPS = 2500.0
WORKLOADS = {
    "c2": "512x512 perspective (f=600), 5 depth steps, 6 bumps, 45% blob mask, noise 0.005, theta_c 2 deg, T=15",
    "c3": "2048x2048 perspective (f=2400), 40 steps, 60 bumps, 70% blob mask, noise 0.005, theta_c 2 deg, T=15",
    "c5": "4096x4096 perspective (f=4800), 150 steps, 240 bumps, 72% blob mask, noise 0.01, theta_c 2 deg, T=15",
}


def kernel_hash():
    h = hashlib.sha256()
    for f in ("ni_fill.hip", "ni_amg.hip"):
        h.update(open(os.path.join(ROOT, "paper_2510_11508_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_record(workload, key):
    """HBM bytes per fill CG iteration from committed rocprofv3 counter
    runs, if they were taken on the current kernel sources with the same
    preconditioner and schedule (key: "multigrid" or "CHUNK:SPLIT")."""
    path = os.path.join(ROOT, "profiles", f"fill_mg_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("schedules", {}).get(key, {}).get("bytes_per_launch")


def cpu_baseline(sample, params, budget_s=12.0):
    """The FP64 oracle as it stands, on this host, single-threaded."""
    from oracle import ni_oracle as O
    n_valid = int((sample.mask > 0).sum())
    runs, t0 = 0, time.perf_counter()
    while True:
        O.integrate(sample.normals, sample.mask, sample.cam, params)
        runs += 1
        el = time.perf_counter() - t0
        if el >= budget_s or runs >= 50:
            break
    return dict(value=n_valid * runs / el / 1e6, unit="Mpx/s", cores=1, kind="oracle",
                sample=f"{runs} full oracle integration(s) of the same {sample.name} map "
                       f"({n_valid} valid px), FP64 sparse-direct solves, {el:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--model", default=DEFAULT_MODEL, help="warm-start weights (skipped if absent)")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-start comparison")
    ap.add_argument("--no-pixel-level", action="store_true",
                    help="skip the pixel-level comparison (theta_c = 0: every pixel its own component)")
    ap.add_argument("--fill-schedule", default=None, metavar="CHUNK:SPLIT",
                    help="fix the large-path fill schedule (e.g. 4096:1) instead of autotuning it")
    ap.add_argument("--fill-precond", type=int, default=None, choices=[0, 1],
                    help="preconditioner of the large fill components (default: the library's, multigrid)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}); there is no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2510_11508_amd as ni
    import synth

    s = synth.make(a.workload, a.seed)
    T = int(s.params["irls_iters"])
    sched = {}
    if a.fill_schedule:
        ch, sp = a.fill_schedule.split(":")
        sched = dict(fill_chunk=int(ch), fill_split=int(sp))
    if a.fill_precond is not None:
        sched["fill_precond"] = a.fill_precond
    p = ni.ni_params_default(theta_c_deg=2.0, irls_iters=T, **sched)
    dev = torch.device("cuda:0")
    normals = torch.from_numpy(s.normals).to(dev)
    mask = torch.from_numpy(s.mask).to(dev)
    n_valid = int((s.mask > 0).sum())
    ctx = ni.Context(0)
    cam = s.cam.as_dict()

    if a.copy_calibration:
        # a plain 1 GiB device copy: the same counters read on it give the
        # bytes-per-count factor of the fill kernels' counter readings
        src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def timed(prm):
        for _ in range(a.warmup):
            ctx.ni_integrate(normals, mask, cam, prm)
        torch.cuda.synchronize()
        reps = []
        t0 = time.perf_counter()
        for _ in range(a.steps):
            out = ctx.ni_integrate(normals, mask, cam, prm)
            reps.append(out["report"])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / a.steps
        return ms, reps, out

    ms, reps, out = timed(p)
    value = n_valid / (ms / 1000.0) / 1e6

    def stage_ms(rs):
        return {k[3:]: round(float(np.mean([r[k] for r in rs])), 3) for k in rs[-1] if k.startswith("ms_")}

    warm = None
    if not a.no_warm and os.path.exists(a.model):
        ctx.ni_unet_load(open(a.model, "rb").read())
        pw = ni.ni_params_default(theta_c_deg=2.0, irls_iters=T, warm_start=1)
        ms_w, reps_w, out_w = timed(pw)
        rw = reps_w[-1]
        z_ref, z_w = out["depth"], out_w["depth"]
        v = torch.isfinite(z_ref)
        dz = float(((z_w[v] - z_ref[v]).abs() / z_ref[v].abs().clamp_min(1e-30)).max()) if bool(v.any()) else 0.0
        warm = dict(model=os.path.relpath(a.model, ROOT), ms_per_step=round(ms_w, 3),
                    value=round(n_valid / (ms_w / 1000.0) / 1e6, 3),
                    speedup=round(ms / ms_w, 3),
                    fill_speedup=round((reps[-1]["ms_fill_small"] + reps[-1]["ms_fill_large"]) /
                                       max(rw["ms_warm"] + rw["ms_fill_small"] + rw["ms_fill_large"], 1e-9), 3),
                    stages_ms=stage_ms(reps_w),
                    fill_iters_max=dict(zero=reps[-1]["fill_iters_max"], warm=rw["fill_iters_max"]),
                    fill_px_iters=dict(zero=reps[-1]["fill_px_iters"], warm=rw["fill_px_iters"]),
                    fallbacks=rw["warm_fallbacks"], max_relres=rw["fill_max_relres"],
                    max_rel_depth_diff_vs_zero_start=dz)
        # network inference alone (features, forward, crop) on this map
        hw = int(s.mask.shape[0]) * int(s.mask.shape[1])
        for _ in range(2):
            ctx.ni_unet_predict(normals, mask, cam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            ctx.ni_unet_predict(normals, mask, cam)
        torch.cuda.synchronize()
        ms_u = (time.perf_counter() - t0) * 1000.0 / 5
        tfl = UNET_FLOP_PER_PX * hw / (ms_u / 1000.0) / 1e12
        warm["unet_forward"] = dict(ms_per_map=round(ms_u, 3), flop_per_px=round(UNET_FLOP_PER_PX),
                                    tflops=round(tfl, 2), peak_tflops=BF16_PEAK_TFLOPS,
                                    frac=round(tfl / BF16_PEAK_TFLOPS, 4), dtype="bf16 mfma, fp32 accumulate")

    pixel = None
    if not a.no_pixel_level:
        # the paper's plain form: no continuous components, the relative
        # scales of all pixels by the same IRLS (one warm-up, one timed call)
        pp = ni.ni_params_default(theta_c_deg=0.0, irls_iters=T)
        ctx.ni_integrate(normals, mask, cam, pp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op = ctx.ni_integrate(normals, mask, cam, pp)
        torch.cuda.synchronize()
        ms_p = (time.perf_counter() - t0) * 1000.0
        pixel = dict(ms_per_step=round(ms_p, 3), value=round(n_valid / (ms_p / 1000.0) / 1e6, 3), K=op["K"],
                     component_speedup=round(ms_p / ms, 2), quot_iters=op["report"]["quot_iters"])

    rep = reps[-1]
    k_ms = float(np.mean([r["ms_large_kernel"] for r in reps]))
    launches = max(rep["fill_large_launches"], 1)
    launch_ms = k_ms / launches
    mg = rep["fill_mg_levels"] > 0 and not rep["fill_mg_fallback"]
    if mg:
        launch_bytes = rep["fill_mg_bytes"]
        key = "multigrid"
        kernel = ("one multigrid-preconditioned PCG iteration of the large fill components: k_cy_down, "
                  "k_cy_restrict, k_cy_up on every level, k_cy_coarsest, k_fs_scal1, k_cg_pq, k_cg_scal, k_fs_xr")
    else:
        px_iters = rep["fill_large_px_iters"]
        launch_bytes = CG_BYTES_PER_PX_ITER * px_iters / launches
        key = f"{rep['fill_chunk']}:{rep['fill_split']}"
        kernel = (("k_lg_p + k_lg_q + k_lg_b" if rep["fill_split"] else "k_lg_a + k_lg_b")
                  + " (one Jacobi-PCG iteration of the large components)")
    achieved = launch_bytes / (launch_ms / 1000.0) / 1e9 if k_ms > 0 else 0.0
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic_record(a.workload, key),
                kernel=kernel, bytes_per_iteration=round(launch_bytes), iterations=launches,
                ms_per_iteration=round(launch_ms, 5))
    if mg:
        roof["levels"] = rep["fill_mg_levels"]
    else:
        roof["bytes_per_px_iter"] = CG_BYTES_PER_PX_ITER

    line = dict(metric=METRIC, value=round(value, 3), unit="Mpx/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
                ms_per_step=round(ms, 3), higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f32 stencil and small-component CG, f64 multigrid CG and reductions", data="synthetic",
                config=dict(workload=f"{a.workload}: {WORKLOADS[a.workload]}", seed=a.seed, n_valid=n_valid,
                            K=out["K"], H=int(s.mask.shape[0]), W=int(s.mask.shape[1])),
                stages_ms=stage_ms(reps),
                fill=dict(iters_max=rep["fill_iters_max"], n_small=rep["n_small"], n_large=rep["n_large"],
                          px_iters=rep["fill_px_iters"], max_relres=rep["fill_max_relres"],
                          preconditioner="multigrid" if mg else "jacobi",
                          mg_fallback=rep["fill_mg_fallback"],
                          **(dict(mg_levels=rep["fill_mg_levels"], mg_iterations=launches)
                             if mg else dict(tuned_schedule=dict(chunk_px=rep["fill_chunk"],
                                                                 launches_per_iteration=3 if rep["fill_split"] else 2)))),
                quot_iters=rep["quot_iters"],
                roofline=roof)
    if warm is not None:
        line["warm_start"] = warm
    if pixel is not None:
        line["pixel_level"] = pixel
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(s, dict(theta_c_deg=2.0, irls_iters=T))
    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
