"""Benchmark: valid Mpixels/s integrated at a 1e-6 relative CG residual.

One step = one ni_integrate call on one synthetic normal map already
resident in HBM (labels, fill, relative-scale IRLS, output), every fill
system stopped at ||r_c|| <= 1e-6 ||b_c||.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c3|c5]

The default workload is c5 (4096^2, the largest single-GPU configuration).
Beside the zero-start rate (`value`) the line carries, on the same map: the
learned warm start at the same residual, optional merging every 5
iterations, 8-connectivity, the pixel-level form (every pixel its own
component), the pixel-level log-depth baseline without discontinuity term
(ND), and the FP64 oracle on this host.

roofline: one PCG iteration of the batched fill of the large components
(the multigrid-preconditioned CG over all of them at once).  Algorithmic
bytes = 32 B per active pixel per CG iteration (FP32 right and down
weights, 8 B, plus x, r, p read and written, 24 B) times the pixels of the
large components, all of which take part in every iteration.  achieved =
those bytes / the HIP-event-timed duration of one iteration (the solve's
launches divided by its iterations), measured inside this run.  The bytes
the multigrid iteration itself moves by its own model (every level's CSR
and FP64 vectors, ni_report.fill_mg_bytes) are reported beside it.
traffic = calibrated FETCH_SIZE + WRITE_SIZE per iteration from committed
counter runs (profiles/fill_mg_traffic_<workload>.json, written by
--digest-counters), while they match the kernel sources.
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
CG_BYTES_PER_PX_ITER = 32   # algorithmic bytes per active pixel per CG iteration
JACOBI_BYTES_PER_PX_ITER = 64
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


def cpu_baseline(name, seed, params):
    """The FP64 oracle as it stands, on this host, single-threaded: one full
    integration of the named map (c3 when the workload is c5: the oracle's
    direct solves on a 4096^2 map take minutes)."""
    import synth
    from oracle import ni_oracle as O
    sample = synth.make(name, seed)
    n_valid = int((sample.mask > 0).sum())
    runs, t0 = 0, time.perf_counter()
    while True:
        O.integrate(sample.normals, sample.mask, sample.cam, params)
        runs += 1
        el = time.perf_counter() - t0
        if el >= 10.0 or runs >= 50:
            break
    return dict(value=round(n_valid * runs / el / 1e6, 4), unit="Mpx/s", cores=1, kind="oracle",
                sample=f"{runs} full oracle integration(s) of the {name} map, seed {seed} "
                       f"({n_valid} valid px), FP64 sparse-direct solves, {el:.1f} s")


FILL_KERNELS = r"(k_cy_\w+<1>|k_fs_rz|k_fs_scal1|k_fs_pq|k_fs_alpha|k_fs_xr|k_runsum_\w+<1>)"


def _csv_rows(d, suffix):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _short(name):
    import re
    n = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*", "", n).strip()


def _kname(row):
    return row.get("Kernel_Name") or row.get("Name") or ""


def digest_counters(workload, fetch_dir, write_dir):
    """profiles/fill_mg_traffic_<workload>.{json,md} from two counter runs of
    `bench.py --workload W --steps 1 --warmup 0 --no-cpu-baseline --no-warm
    --no-pixel-level --copy-calibration` (one integration), FETCH_SIZE then
    WRITE_SIZE, each with its JSON line in <dir>/bench.json.  Counter values
    (KiB per dispatch) are scaled by what the same counter reads on the
    plain 1 GiB copy of the calibration, summed over the dispatches of the
    fill solve's kernels and divided by its iterations."""
    import re
    line = json.load(open(os.path.join(fetch_dir, "bench.json")))
    its = line["roofline"]["iterations"]
    out = {}
    for cname, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _csv_rows(d, "counter_collection.csv") if r.get("Counter_Name") == cname]
        cal = max((float(r["Counter_Value"]) for r in rows if "copy" in _kname(r).lower()), default=0.0)
        if cal <= 0:
            raise SystemExit(f"no copy-calibration dispatch in {d}")
        factor = (1 << 30) / (cal * 1024.0)
        per_kernel = {}
        for r in rows:
            k = _kname(r)
            if re.search(FILL_KERNELS, k):
                short = _short(k)
                per_kernel[short] = per_kernel.get(short, 0.0) + float(r["Counter_Value"])
        tot = sum(per_kernel.values())
        out[cname] = dict(calibration_KiB=cal, factor=factor, fill_KiB=tot, per_kernel_KiB=per_kernel,
                          bytes_per_iteration=tot * 1024.0 * factor / its)
    traffic = out["FETCH_SIZE"]["bytes_per_iteration"] + out["WRITE_SIZE"]["bytes_per_iteration"]
    alg = line["roofline"]["bytes_per_iteration"]
    rec = dict(workload=workload, kernel_hash=kernel_hash(),
               unit="bytes per PCG iteration of the large fill components",
               schedules={"multigrid": dict(bytes_per_launch=round(traffic),
                                            fetch_bytes=round(out["FETCH_SIZE"]["bytes_per_iteration"]),
                                            write_bytes=round(out["WRITE_SIZE"]["bytes_per_iteration"]),
                                            algorithmic_bytes=alg, ratio_to_algorithmic=round(traffic / alg, 3),
                                            multigrid_model_bytes=line["roofline"].get("multigrid_model", {})
                                            .get("bytes_per_iteration"),
                                            iterations=its, counters=out)})
    base = os.path.join(ROOT, "profiles", f"fill_mg_traffic_{workload}")
    json.dump(rec, open(base + ".json", "w"), indent=1)
    mm = rec["schedules"]["multigrid"]["multigrid_model_bytes"]
    with open(base + ".md", "w") as f:
        f.write(f"# HBM-side traffic of one PCG iteration of the large fill components, workload {workload}\n\n")
        f.write("Two counter runs of one integration each (FETCH_SIZE, then WRITE_SIZE); the same process also\n"
                "runs a plain 1 GiB device copy, whose reading gives the bytes-per-count factor:\n\n")
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            f.write(f"    cd /tmp && timeout -s KILL 300 rocprofv3 --pmc {c} --output-format csv -d <dir_{c}> -o run -- "
                    f"python3 <repo>/bench.py --workload {workload} --steps 1 --warmup 0 --no-cpu-baseline "
                    f"--no-warm --no-pixel-level --no-merging --no-baseline --no-conn8 --copy-calibration > <dir_{c}>/bench.json\n")
        f.write(f"    python3 <repo>/bench.py --workload {workload} --digest-counters <dir_FETCH_SIZE> <dir_WRITE_SIZE>\n\n")
        f.write(f"Fill-solve kernels (`{FILL_KERNELS}`), {its} iterations.\n\n")
        f.write("| counter | copy reading (KiB) | factor | fill solve (KiB) | per iteration (MB) |\n|---|---|---|---|---|\n")
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            o = out[c]
            f.write(f"| {c} | {o['calibration_KiB']:,.1f} | {o['factor']:.4f} | {o['fill_KiB']:,.0f} | "
                    f"{o['bytes_per_iteration'] / 1e6:,.1f} |\n")
        f.write(f"\n- Measured traffic per iteration: {traffic / 1e6:,.1f} MB.\n")
        f.write(f"- Algorithmic bytes per iteration (32 B x {line['roofline']['active_px']:,} active px): "
                f"{alg / 1e6:,.1f} MB (ratio {traffic / alg:.2f}).\n")
        if mm:
            f.write(f"- The multigrid iteration's own model (every level, FP64): {mm / 1e6:,.1f} MB "
                    f"(ratio {traffic / mm:.2f}).\n")
        f.write("\nFETCH_SIZE by kernel over the solve (KiB, uncalibrated):\n\n| kernel | KiB |\n|---|---|\n")
        for k, v in sorted(out["FETCH_SIZE"]["per_kernel_KiB"].items(), key=lambda kv: -kv[1]):
            f.write(f"| {k} | {v:,.0f} |\n")
        f.write(f"\n`{os.path.basename(base)}.json` holds these figures with a hash of `ni_fill.hip` and "
                "`ni_amg.hip`; `bench.py` reports them as `roofline.traffic` only while the hash matches.\n")
    print(json.dumps(rec["schedules"]["multigrid"]["bytes_per_launch"]))


def digest_trace(workload, d):
    """profiles/integrate_<workload>_kernel_stats.md from a rocprofv3
    --kernel-trace --stats run of this script (its JSON line in d/bench.json):
    the top kernels, and the fill solve's kernel time per iteration beside
    the bench's own event-timed figure."""
    import re
    line = json.load(open(os.path.join(d, "bench.json")))
    rows = _csv_rows(d, "kernel_stats.csv")
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    calls = line["steps"] + line["warmup"]
    fill_ns = sum(float(r["TotalDurationNs"]) for r in rows if re.search(FILL_KERNELS, r["Name"]))
    quot_ns = sum(float(r["TotalDurationNs"]) for r in rows if re.search(r"k_cy_\w+<0>|k_cg_\w+<0>|k_cg_\w+_f\b", r["Name"]))
    its = line["roofline"]["iterations"]
    base = os.path.join(ROOT, "profiles", f"integrate_{workload}_kernel_stats.md")
    with open(base, "w") as f:
        f.write(f"# Kernel time, whole integration, workload {workload} "
                f"({line['config']['n_valid']:,} valid px, K = {line['config']['K']:,})\n\n")
        f.write("Command (from the repository root, on the GPU):\n\n")
        f.write(f"    cd /tmp && rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- python3 "
                f"<repo>/bench.py --workload {workload} --steps {line['steps']} --warmup {line['warmup']} "
                "--no-cpu-baseline --no-warm --no-pixel-level --no-merging --no-baseline --no-conn8 > <dir>/bench.json\n")
        f.write(f"    python3 <repo>/bench.py --workload {workload} --digest-trace <dir>\n\n")
        f.write(f"{calls} ni_integrate calls. Kernel time {tot / 1e6 / calls:,.2f} ms per call; "
                f"bench ms_per_step {line['ms_per_step']} (event-timed stages: {line['stages_ms']}).\n\n")
        f.write(f"- Fill solve of the large components (`{FILL_KERNELS}`): "
                f"{fill_ns / 1e6 / calls:,.2f} ms per call, {fill_ns / 1e3 / calls / max(its, 1):,.1f} us per "
                f"iteration over {its} iterations; the bench's HIP-event figure for the same iteration: "
                f"{line['roofline']['ms_per_iteration'] * 1e3:,.1f} us (it also spans the gaps between launches).\n")
        f.write(f"- Relative-scale solves (quotient multigrid PCG, `<0>` kernels): {quot_ns / 1e6 / calls:,.2f} ms "
                "per call.\n\n")
        # kernel time by part of the path (first matching pattern)
        parts = [("fill: multigrid PCG of the large components", FILL_KERNELS),
                 ("fill: small-component tiers", r"k_fill_small"),
                 ("relative scales: quotient PCG (V-cycle, scalars, updates)",
                  r"k_cy_\w+<0>|k_cg_\w+<0>|k_cg_\w+_f\b|k_cg_xr\b|k_cg_init"),
                 ("hierarchy builds (aggregation, Galerkin sums, sorts, scans)", r"k_am_|k_gm_|k_rs_|k_scan_"),
                 ("relative scales: weights, pieces, flow residual, energy",
                  r"k_irls_|k_flow_|k_piece_|k_uf_union_list|k_scale_add|k_add_f64|k_q_matrix|k_sum_parts"),
                 ("other", r".")]
        share = {}
        for r in rows:
            for nm, pat in parts:
                if re.search(pat, r["Name"]):
                    share[nm] = share.get(nm, 0.0) + float(r["TotalDurationNs"])
                    break
        f.write("| part | ms per call | share |\n|---|---|---|\n")
        for nm, _ in parts:
            v = share.get(nm, 0.0)
            f.write(f"| {nm} | {v / 1e6 / calls:,.2f} | {100 * v / tot:.1f}% |\n")
        f.write("\n")
        f.write("| kernel | calls | total ms | avg us | min us | max us | share |\n|---|---|---|---|---|---|---|\n")
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:24]:
            nm = _short(r["Name"])
            f.write(f"| {nm} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:,.2f} | "
                    f"{float(r['AverageNs']) / 1e3:,.2f} | {float(r['MinNs']) / 1e3:,.2f} | "
                    f"{float(r['MaxNs']) / 1e3:,.2f} | {100 * float(r['TotalDurationNs']) / tot:.1f}% |\n")
        f.write("\nbench.py line of the same run:\n\n    " + json.dumps({k: line[k] for k in (
            "value", "unit", "ms_per_step", "stages_ms", "quot_iters", "quot_iters_refine", "roofline") if k in line}) + "\n")
    print(base)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--model", default=DEFAULT_MODEL, help="warm-start weights (skipped if absent)")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-start comparison")
    ap.add_argument("--no-merging", action="store_true",
                    help="skip the optional-merging leg (freq_merging = 5, the paper's large-map setting)")
    ap.add_argument("--no-baseline", action="store_true",
                    help="skip the pixel-level log-depth baseline leg (variant 1, ND form)")
    ap.add_argument("--no-conn8", action="store_true", help="skip the 8-connectivity leg")
    ap.add_argument("--no-pixel-level", action="store_true",
                    help="skip the pixel-level comparison (theta_c = 0: every pixel its own component)")
    ap.add_argument("--fill-schedule", default=None, metavar="CHUNK:SPLIT",
                    help="fix the large-path fill schedule (e.g. 4096:1) instead of autotuning it")
    ap.add_argument("--fill-precond", type=int, default=None, choices=[0, 1],
                    help="preconditioner of the large fill components (default: the library's, multigrid)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--unet-only", type=int, default=0, metavar="N",
                    help="only run the warm-start network's inference N times on the workload's map "
                         "(for counter runs of its MFMA kernels) and print its timing")
    ap.add_argument("--digest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/fill_mg_traffic_<workload>.{json,md} from two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) of this script with --steps 1 --warmup 0 --copy-calibration")
    ap.add_argument("--digest-trace", metavar="DIR",
                    help="write profiles/integrate_<workload>_kernel_stats.md from a rocprofv3 --kernel-trace "
                         "--stats run of this script (CSV output) and its JSON line (DIR/bench.json)")
    a = ap.parse_args()
    if a.digest_counters:
        digest_counters(a.workload, *a.digest_counters)
        return
    if a.digest_trace:
        digest_trace(a.workload, a.digest_trace)
        return
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

    if a.unet_only:
        ctx.ni_unet_load(open(a.model, "rb").read())
        hw = int(s.mask.shape[0]) * int(s.mask.shape[1])
        ctx.ni_unet_predict(normals, mask, cam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.unet_only):
            ctx.ni_unet_predict(normals, mask, cam)
        torch.cuda.synchronize()
        ms_u = (time.perf_counter() - t0) * 1000.0 / a.unet_only
        tfl = UNET_FLOP_PER_PX * hw / (ms_u / 1000.0) / 1e12
        print(json.dumps(dict(workload=a.workload, calls=a.unet_only + 1, ms_per_map=round(ms_u, 3),
                              flop_per_px=round(UNET_FLOP_PER_PX), tflops=round(tfl, 2),
                              frac_bf16_peak=round(tfl / BF16_PEAK_TFLOPS, 4))))
        ctx.close()
        return

    ms, reps, out = timed(p)
    value = n_valid / (ms / 1000.0) / 1e6

    def stage_ms(rs):
        return {k[3:]: round(float(np.mean([r[k] for r in rs])), 3) for k in rs[-1] if k.startswith("ms_")}

    def depth_diff(z_ref, z_x):
        """Relative depth difference to the main leg's output: its maximum
        and the share of valid pixels beyond the parity bound (1e-4) and
        beyond 1e-2 (where the relative scale of a weakly linked piece moved)."""
        v = torch.isfinite(z_ref)
        if not bool(v.any()):
            return dict(max=0.0, frac_px_over_1e_4=0.0, frac_px_over_1e_2=0.0)
        d = (z_x[v] - z_ref[v]).abs() / z_ref[v].abs().clamp_min(1e-30)
        return dict(max=float(d.max()), frac_px_over_1e_4=float((d > 1e-4).float().mean()),
                    frac_px_over_1e_2=float((d > 1e-2).float().mean()))

    warm = None
    if not a.no_warm and os.path.exists(a.model):
        ctx.ni_unet_load(open(a.model, "rb").read())
        pw = ni.ni_params_default(theta_c_deg=2.0, irls_iters=T, warm_start=1)
        ms_w, reps_w, out_w = timed(pw)
        rw = reps_w[-1]
        dz = depth_diff(out["depth"], out_w["depth"])
        warm = dict(model=os.path.relpath(a.model, ROOT), ms_per_step=round(ms_w, 3),
                    value=round(n_valid / (ms_w / 1000.0) / 1e6, 3),
                    speedup=round(ms / ms_w, 3),
                    fill_speedup=round((reps[-1]["ms_fill_small"] + reps[-1]["ms_fill_large"]) /
                                       max(rw["ms_warm"] + rw["ms_fill_small"] + rw["ms_fill_large"], 1e-9), 3),
                    stages_ms=stage_ms(reps_w),
                    fill_iters_max=dict(zero=reps[-1]["fill_iters_max"], warm=rw["fill_iters_max"]),
                    fill_px_iters=dict(zero=reps[-1]["fill_px_iters"], warm=rw["fill_px_iters"]),
                    fallbacks=rw["warm_fallbacks"], max_relres=rw["fill_max_relres"],
                    rel_depth_diff_vs_zero_start=dz)
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

    merging = None
    if not a.no_merging:
        # Alg. 1 with the optional merge step every 5 iterations (Sec. 3.5)
        pm = ni.ni_params_default(theta_c_deg=2.0, irls_iters=T, freq_merging=5, **sched)
        ms_m, reps_m, out_m = timed(pm)
        rm = reps_m[-1]
        dz = depth_diff(out["depth"], out_m["depth"])
        merging = dict(freq_merging=5, ms_per_step=round(ms_m, 3), value=round(n_valid / (ms_m / 1000.0) / 1e6, 3),
                       speedup_vs_no_merging=round(ms / ms_m, 3), merges=rm["merges"],
                       nodes_final=rm["nodes_final"], stages_ms=stage_ms(reps_m), quot_iters=rm["quot_iters"],
                       rel_depth_diff_vs_no_merging=dz)

    conn8 = None
    if not a.no_conn8:
        # 8-connectivity on the same map (diagonal edges in the pixel graph,
        # the 8-connected fill systems on the multigrid path)
        p8 = ni.ni_params_default(theta_c_deg=2.0, irls_iters=T, connectivity=8, **sched)
        ms_8, reps_8, out_8 = timed(p8)
        r8 = reps_8[-1]
        conn8 = dict(ms_per_step=round(ms_8, 3), value=round(n_valid / (ms_8 / 1000.0) / 1e6, 3), K=out_8["K"],
                     n_inter_edges=r8["n_inter_edges"], stages_ms=stage_ms(reps_8),
                     fill=dict(iters_max=r8["fill_iters_max"], px_iters=r8["fill_px_iters"],
                               mg_levels=r8["fill_mg_levels"], mg_iterations=r8["fill_large_launches"],
                               max_relres=r8["fill_max_relres"]),
                     quot_iters=r8["quot_iters"])

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

    baseline = None
    if not a.no_baseline:
        # the pixel-level log-depth baseline without discontinuity term (ND):
        # one warm-up, one timed call, the same T and tolerances
        pb = ni.ni_params_default(irls_iters=T, variant=1)
        ctx.ni_integrate(normals, mask, cam, pb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ob = ctx.ni_integrate(normals, mask, cam, pb)
        torch.cuda.synchronize()
        ms_b = (time.perf_counter() - t0) * 1000.0
        baseline = dict(ms_per_step=round(ms_b, 3), value=round(n_valid / (ms_b / 1000.0) / 1e6, 3),
                        component_speedup=round(ms_b / ms, 2), quot_iters=ob["report"]["quot_iters"])

    rep = reps[-1]
    k_ms = float(np.mean([r["ms_large_kernel"] for r in reps]))
    launches = max(rep["fill_large_launches"], 1)
    launch_ms = k_ms / launches
    mg = rep["fill_mg_levels"] > 0 and not rep["fill_mg_fallback"]
    large_px = int(rep["fill_large_px"])
    launch_bytes = CG_BYTES_PER_PX_ITER * large_px
    if mg:
        key = "multigrid"
        kernel = ("one multigrid-preconditioned PCG iteration of the large fill components (all of them at "
                  "once, each with its own scalars): k_cy_down<1>, k_cy_restrict<1>, k_cy_up<1> on the levels above "
                  "the tail, k_cy_tail<1> (the coarse levels and the exact coarsest solve in one workgroup, from "
                  "LDS), k_fs_rz, k_fs_scal1, k_fs_pq, k_fs_alpha, k_fs_xr, k_runsum_tile<1> and "
                  "k_runsum_top<1> (three per-component sums)")
    else:
        key = f"{rep['fill_chunk']}:{rep['fill_split']}"
        kernel = (("k_lg_p + k_lg_q + k_lg_b" if rep["fill_split"] else "k_lg_a + k_lg_b")
                  + " (one Jacobi-PCG iteration of the large components)")
    achieved = launch_bytes / (launch_ms / 1000.0) / 1e9 if k_ms > 0 else 0.0
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic_record(a.workload, key),
                kernel=kernel, bytes_per_iteration=launch_bytes, bytes_per_px_iter=CG_BYTES_PER_PX_ITER,
                active_px=large_px, iterations=launches, ms_per_iteration=round(launch_ms, 5))
    if mg:
        mb = rep["fill_mg_bytes"]
        ma = mb / (launch_ms / 1000.0) / 1e9 if k_ms > 0 else 0.0
        roof["multigrid_model"] = dict(levels=rep["fill_mg_levels"], bytes_per_iteration=round(mb),
                                       achieved=round(ma, 1), frac=round(ma / HBM_PEAK_GBS, 4))
    else:
        ja = JACOBI_BYTES_PER_PX_ITER * rep["fill_large_px_iters"] / launches / (launch_ms / 1000.0) / 1e9
        roof["jacobi_model"] = dict(bytes_per_px_iter=JACOBI_BYTES_PER_PX_ITER, achieved=round(ja, 1),
                                    frac=round(ja / HBM_PEAK_GBS, 4))

    line = dict(metric=METRIC, value=round(value, 3), unit="Mpx/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
                ms_per_step=round(ms, 3), higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f32 stencil and small-component CG; f64 multigrid fill CG, reductions and relative-scale solve",
                data="synthetic",
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
                quot_iters_refine=rep["quot_iters_refine"],
                roofline=roof)
    if warm is not None:
        line["warm_start"] = warm
    if merging is not None:
        line["merging"] = merging
    if conn8 is not None:
        line["connectivity8"] = conn8
    if pixel is not None:
        line["pixel_level"] = pixel
    if baseline is not None:
        line["logdepth_baseline_nd"] = baseline
    if not a.no_cpu_baseline:
        cname = "c3" if a.workload == "c5" else a.workload
        line["cpu_baseline"] = cpu_baseline(cname, a.seed, dict(theta_c_deg=2.0, irls_iters=T))
    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
