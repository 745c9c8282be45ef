#!/usr/bin/env python3
"""Throughput of the sDEM total viewshed on one MI355X.

One step = one tvs_total_viewshed call (all sectors: relocation of every skewed row, sweep,
back-projection) on a device-resident synthetic DEM shaped like the paper's 2000x2000, 10 m
workload. Prints one JSON line: LoS cell-evaluations/s (whole job), total-viewshed cells/s, the
sweep kernel against its ALU roofline (kernel durations from HIP events recorded by the library
on the call's stream inside the timed region), the relocation kernel variant against HBM, the CPU
oracle's rate on a bounded sample of the same workload, and (default run) a batch pass over 64
tiles of uneven size and a served Poisson request stream as sub-objects.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload tvs2000] [--flags 0]
                    [--no-batch] [--no-serve] [--no-cpu-baseline] [--mode single|batch|serve|multiple]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs at a 2.4 GHz peak engine clock. The published FP32 vector peak, 157.3 TFLOP/s,
# is 128 FP32 lane-operations per CU per clock with an FMA counted as 2 flops; plain (non-packed)
# FP32 VALU instructions reach that issue rate on gfx950 (VALU counters of the sweep show more
# than 64 lanes/clk/CU). The FP64 vector peak, 78.6 TFLOP/s, is 64 FP64 lane-operations per CU
# per clock. One line-of-sight evaluation is 5 algorithmic operations: subtract, divide, compare,
# max, conditional integer add; the peak counts each lane-operation once, at the rate of the
# precision the decision is taken in.
CU, CLOCK_HZ = 256, 2.4e9
ALU_PEAK_OPS_F32 = CU * 128 * CLOCK_HZ        # 7.86e13 lane-ops/s = 157.3 TFLOP/s / 2
ALU_PEAK_OPS_F64 = CU * 64 * CLOCK_HZ         # 3.93e13 lane-ops/s = 78.6 TFLOP/s / 2
OPS_PER_EVAL = 5
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_digest():
    """Hash of the code of every library source the single-grid step runs (kernels, launch plan and
    host code all change the bytes a launch moves; the request server's file is not on that path),
    without its // comments and blank lines, so that edits to comments keep a traffic summary valid.
    The sources hold no "//" inside string literals."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "paper_2003_02200_amd", "csrc", "*.h")) +
                       glob.glob(os.path.join(ROOT, "paper_2003_02200_amd", "csrc", "*.hip"))):
        if os.path.basename(path) == "tvs_server.hip":
            continue
        h.update(os.path.basename(path).encode())
        for line in open(path, encoding="utf-8"):
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()


def read_traffic(path, workload, flags):
    """HBM bytes per sweep launch from a committed counter summary (FETCH_SIZE + WRITE_SIZE,
    scaled by a copy kernel of known size). None unless it was taken on this kernel source,
    workload and flags."""
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    try:
        if (fields.get("library_source_sha256") != kernel_source_digest() or fields.get("workload") != workload
                or int(fields.get("flags", "-1")) != flags):
            return None
        return int(fields["hbm_read_bytes_per_launch"]) + int(fields["hbm_write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_counters(path, workload, flags):
    """VALU figures of the sweep from a committed counter summary (SQ_INSTS_VALU etc. over the launches
    of one step): None unless it was taken on this library source, workload and flags."""
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    try:
        if (fields.get("library_source_sha256") != kernel_source_digest() or fields.get("workload") != workload
                or int(fields.get("flags", "-1")) != flags):
            return None
        return {"valu_lanes_per_clk_per_cu": float(fields["sweep_valu_lanes_per_clk_per_cu"]),
                "valu_issue_frac_of_fp64_rate": float(fields["sweep_valu_lanes_per_clk_per_cu"]) / 64.0,
                "valu_lane_insts_per_eval_done": float(fields["sweep_valu_lane_insts_per_eval_done"]),
                "sweep_clock_ghz": float(fields["sweep_clock_ghz"]),
                "source": os.path.relpath(path, ROOT)}
    except (KeyError, ValueError):
        return None


def sub_bench(name, fn):
    """A sub-measurement of the line: its failure is reported in the line (with the error) instead of
    losing the headline measurement already taken."""
    try:
        return fn()
    except Exception as e:  # noqa: BLE001 - any failure of a sub-measurement is reported, not raised
        log(f"{name}: failed: {type(e).__name__}: {e}")
        return {"error": f"{type(e).__name__}: {e}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tvs2000")
    ap.add_argument("--flags", type=int, default=0, help="TVS_FLAG_* bits (0: double elevations, reciprocal-product slope, early exit)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="single mode: leave out the batch sub-object")
    ap.add_argument("--no-serve", action="store_true", help="single mode: leave out the serve sub-object")
    ap.add_argument("--traffic-summary", default=os.path.join(ROOT, "profiles", "sweep_tvs2000_traffic.md"))
    ap.add_argument("--counter-summary", default=os.path.join(ROOT, "profiles", "tvs2000_counters.md"))
    ap.add_argument("--mode", choices=("single", "batch", "serve", "multiple"), default="single",
                    help="single: the 2000x2000 workload (the headline), with batch and serve passes as sub-objects; "
                         "batch: 64 independent tiles of uneven size through the batched path, against the plain "
                         "per-tile loop; serve: a Poisson stream of singular and total requests through the request "
                         "server; multiple: the count map of 10 random POVs on the 2000x2000 workload, against 10 "
                         "singular calls")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--batch-tiles", type=int, default=64)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before timing, copy this many MiB device-to-device (a plain copy kernel of known size "
                         "that scales the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        log("bench.py measures one GPU only: the library has no multi-GPU path "
            "(sectors would shard across GPUs with one final reduce; see the design notes). Run with --gpus 1.")
        sys.exit(2)

    if args.mode == "batch":
        print(json.dumps(bench_batch(args, args.batch_tiles, args.steps, args.warmup, standalone=True)), flush=True)
        return
    if args.mode == "serve":
        print(json.dumps(bench_serve(args, args.serve_seconds, cold=True, standalone=True)), flush=True)
        return
    if args.mode == "multiple":
        return bench_multiple(args)
    line = bench_single(args)
    if not args.no_serve and args.workload == "tvs2000" and args.flags == 0:
        line["serve"] = sub_bench("serve", lambda: bench_serve(args, 8.0, cold=False))
    if not args.no_batch and args.workload == "tvs2000" and args.flags == 0:
        line["batch"] = sub_bench("batch", lambda: bench_batch(args, args.batch_tiles, 2, 1))
    print(json.dumps(line), flush=True)


def bench_single(args):
    import numpy as np
    import torch

    import paper_2003_02200_amd as tvs
    from synth import WORKLOADS, workload_dem

    w = WORKLOADS[args.workload]
    dem = workload_dem(args.workload)
    H, W = dem.shape
    call = (w["spacing"], w["obs_height"], w["n_sectors"], w["max_dist"])
    evals, pairs = tvs.los_evals(H, W, *[call[0], call[2], call[3]])
    torch.cuda.set_device(0)
    d = torch.from_numpy(dem).cuda()
    torch.cuda.synchronize()
    log(f"workload {args.workload}: {H}x{W}, {w['n_sectors']} sectors, {evals:.3e} LoS evals/step")

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.copy_calibration_mib} MiB done")
        del src, dst

    for i in range(args.warmup):
        out = tvs.total_viewshed(d, *call, flags=args.flags)
        torch.cuda.synchronize()
        log(f"warmup {i} done")

    # evaluations the sweep carries out (its exact early exit skips targets that provably stay
    # hidden); deterministic for a given input, so counted once outside the timed region
    _, st0 = tvs.total_viewshed(d, *call, flags=args.flags | tvs.FLAG_COUNT_EVALS, stats=True)
    torch.cuda.synchronize()
    evals_done = st0.sweep_evals_done
    log(f"sweep carries out {evals_done:.3e} of {evals:.3e} evaluations ({evals_done / evals:.3f})")

    sweep_ms = reloc_ms = back_ms = 0.0
    sweep_n = reloc_n = back_n = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out, st = tvs.total_viewshed(d, *call, flags=args.flags, stats=True)
        sweep_ms += st.sweep_ms
        reloc_ms += st.reloc_ms
        back_ms += st.backproj_ms
        sweep_n += st.sweep_launches
        reloc_n += st.reloc_launches
        back_n += st.backproj_launches
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_s = elapsed / args.steps
    log(f"timed {args.steps} steps: {step_s * 1e3:.2f} ms/step")
    res = out.cpu().numpy()
    if not np.all(np.isfinite(res)):
        log("non-finite output")
        sys.exit(1)

    # dominant kernel: the sweep (ALU bound), priced at the peak of the decision's precision
    f32 = bool(args.flags & tvs.FLAG_SLOPE_F32)
    ALU_PEAK_OPS = ALU_PEAK_OPS_F32 if f32 else ALU_PEAK_OPS_F64
    avg_sweep_s = sweep_ms / 1e3 / max(sweep_n, 1)
    ops_done_per_launch = OPS_PER_EVAL * evals_done * args.steps / max(sweep_n, 1)
    ops_closed_per_launch = OPS_PER_EVAL * evals * args.steps / max(sweep_n, 1)
    achieved = ops_done_per_launch / avg_sweep_s if sweep_n else None
    traffic = read_traffic(args.traffic_summary, args.workload, args.flags)
    roofline = {
        "bound": "alu",
        "achieved": achieved / 1e12 if achieved else None,
        "peak": ALU_PEAK_OPS / 1e12,
        "unit": "TFLOP/s",
        "frac": (achieved / ALU_PEAK_OPS) if achieved else None,
        "traffic": traffic,
        "kernel": "k_sweep",
        "basis": "lane-operations of the line-of-sight evaluations the sweep carries out (5 per evaluation: "
                 "subtract, divide, compare, max, conditional add) per launch, over the launch's average "
                 "duration from HIP events on the call's stream",
        "frac_closed_form": (ops_closed_per_launch / avg_sweep_s / ALU_PEAK_OPS) if sweep_n else None,
        "frac_closed_form_note": "the same launches priced on every evaluation the workload defines (closed "
                                 "form, 5 ops each): above 1 because the exact early exit and block skip rule "
                                 "most of them hidden without evaluating them, so it is not a roofline fraction",
        "ops_per_eval": OPS_PER_EVAL,
        "avg_launch_ms": avg_sweep_s * 1e3,
        "launches": sweep_n,
        "evals_done_per_step": evals_done,
        "evals_done_frac": evals_done / evals,
        "counters": read_counters(args.counter_summary, args.workload, args.flags),
    }
    kernels = {
        "sweep_ms_per_step": sweep_ms / args.steps,
        "backproj_ms_per_step": back_ms / args.steps,
        "transpose_ms_per_step": reloc_ms / args.steps,
        "evals_per_s_sweep_only": evals * args.steps / (sweep_ms / 1e3) if sweep_ms > 0 else None,
        "chunks_per_step": st.chunks,
        "scratch_bytes": st.scratch_bytes,
        "note": "the sweep gathers each skewed row from the grid (Alg. 6's interpolation), so the step has no "
                "relocation launch; the transposed grid serves the 45-135 deg axes",
    }

    # the relocation as its own kernel (TVS_FLAG_RELOCATE), measured outside the timed region: its
    # algorithmic bytes per existing sample are 4 read + 4 written for a float skwDEM (the paper's), and
    # 4 + 8 as the library writes it (double elevations)
    relocation = None
    if args.flags == 0:
        tvs.total_viewshed(d, *call, flags=tvs.FLAG_RELOCATE)
        torch.cuda.synchronize()  # the warm call ends before the first timed one starts
        rms = rn = rsteps = 0
        rstep_ms = 0.0
        for _ in range(2):
            t1 = time.perf_counter()
            _, rst = tvs.total_viewshed(d, *call, flags=tvs.FLAG_RELOCATE, stats=True)
            torch.cuda.synchronize()
            rstep_ms += (time.perf_counter() - t1) * 1e3
            rms += rst.reloc_ms
            rn += rst.reloc_launches
            rsteps += 1
        per_step_s = rms / 1e3 / rsteps
        relocation = {
            "kernel": "k_relocate (TVS_FLAG_RELOCATE variant)",
            "ms_per_step": rms / rsteps,
            "launches_per_step": rn // rsteps,
            "variant_ms_per_step": rstep_ms / rsteps,
            "alg_GBps_8B_per_sample": pairs * 8 / per_step_s / 1e9,
            "frac_hbm_8B_per_sample": pairs * 8 / per_step_s / 1e9 / HBM_PEAK_GBS,
            "alg_GBps_12B_per_sample": pairs * 12 / per_step_s / 1e9,
            "frac_hbm_12B_per_sample": pairs * 12 / per_step_s / 1e9 / HBM_PEAK_GBS,
        }
        log(f"relocation kernel: {rms / rsteps:.3f} ms per step, {relocation['frac_hbm_8B_per_sample']:.3f} "
            f"of HBM on 8 B/sample ({relocation['frac_hbm_12B_per_sample']:.3f} on 12 B)")

    # the host entry point (DEM in host memory, map back to host memory): PCIe transfers, host-side
    # validation and device scratch included; reported beside `value`, never as it
    host_ms = None
    if args.flags == 0:
        tvs.total_viewshed(dem, *call)
        t1 = time.perf_counter()
        for _ in range(2):
            tvs.total_viewshed(dem, *call)
        host_ms = (time.perf_counter() - t1) / 2 * 1e3
        log(f"host entry point: {host_ms:.2f} ms per call")

    cpu = None if args.no_cpu_baseline else sub_bench("cpu baseline", lambda: cpu_baseline(args.workload, dem, call))

    return {
        "metric": "LoS cell-evals/s + total-viewshed cells/s at 2000² DEM; p50/p99 serve latency",
        "value": evals * args.steps / elapsed,
        "unit": "LoS cell-evals/s",
        "value_basis": "line-of-sight evaluations the workload defines (every POV-target pair in range, "
                       "closed form); the sweep decides all of them, carrying out evals_done_frac of them "
                       "and ruling the rest hidden by an exact bound",
        "evals_carried_out_per_s": evals_done * args.steps / elapsed,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if f32 else "f64",
        "slope": (("correctly rounded float quotient" if args.flags & tvs.FLAG_SLOPE_EXACT else
                   "float difference x float reciprocal") if f32 else
                  "correctly rounded double quotient" if args.flags & (tvs.FLAG_SLOPE_F64 | tvs.FLAG_SLOPE_EXACT) else
                  "double difference x double reciprocal"),
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {H}x{W} diamond-square DEM (seed {w['seed']}, roughness {w['roughness']}, "
                        f"0-{w['zmax']:.0f} m), spacing {w['spacing']} m, observer {w['obs_height']} m, "
                        f"{w['n_sectors']} sectors, max distance {w['max_dist']:.0f} m",
            "rows": H, "cols": W, "n_sectors": w["n_sectors"], "max_dist_m": w["max_dist"],
            "flags": args.flags, "los_evals_per_step": evals, "pov_sector_pairs_per_step": pairs,
        },
        "total_viewshed_cells_per_s": H * W / step_s,
        "host_api": None if host_ms is None else {
            "ms_per_call": host_ms, "total_viewshed_cells_per_s": H * W / (host_ms / 1e3),
            "note": "tvs_total_viewshed with the DEM and map in host memory: PCIe copies and host-side "
                    "validation included"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "relocation": relocation,
    }


def cpu_baseline(workload, dem, call):
    """The oracle as it stands on the host cores: the centred 256 x 256 crop of the 2000 x 2000 workload
    (every POV of the crop walks the whole DEM in every sector), the full 128 x 128 workload, and the
    centred 64 x 64 crop of the 4000 x 4000 precision-study workload (5 m, 360 sectors, 10 km)."""
    import oracle
    from synth import WORKLOADS, workload_dem

    H, W = dem.shape
    cw = min(256, H, W)
    r0, c0 = (H - cw) // 2, (W - cw) // 2
    log(f"cpu baseline: oracle on the {cw}x{cw} centre crop ...")
    t1 = time.perf_counter()
    _, ev_cpu = oracle.total(dem, *call, prec=64, window=(r0, c0, cw, cw), count=True)
    cpu_s = time.perf_counter() - t1
    w1 = WORKLOADS["tvs128"]
    d1 = workload_dem("tvs128")
    t2 = time.perf_counter()
    _, ev1 = oracle.total(d1, w1["spacing"], w1["obs_height"], w1["n_sectors"], w1["max_dist"], prec=64, count=True)
    s1 = time.perf_counter() - t2
    w4 = WORKLOADS["tvs4000"]
    d4 = workload_dem("tvs4000")
    c4 = 64
    r4, q4 = (d4.shape[0] - c4) // 2, (d4.shape[1] - c4) // 2
    t3 = time.perf_counter()
    _, ev4 = oracle.total(d4, w4["spacing"], w4["obs_height"], w4["n_sectors"], w4["max_dist"], prec=64,
                          window=(r4, q4, c4, c4), count=True)
    s4 = time.perf_counter() - t3
    log(f"cpu baseline: {ev_cpu / cpu_s:.3e} evals/s on {oracle.threads()} threads")
    return {
        "value": ev_cpu / cpu_s,
        "unit": "LoS cell-evals/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": f"centred {cw}x{cw} crop (rows/cols {r0}..{r0 + cw - 1}) of the {H}x{W} {workload} workload, all "
                  f"{call[2]} sectors, double oracle walking both skewed samples of every cell and sector: "
                  f"{ev_cpu:.3e} evals in {cpu_s:.1f} s",
        "cells_per_s": cw * cw / cpu_s,
        "full_128x128_workload": {"evals": ev1, "seconds": s1, "evals_per_s": ev1 / s1,
                                  "cells_per_s": 128 * 128 / s1},
        "crop_64x64_of_4000x4000": {"evals": ev4, "seconds": s4, "evals_per_s": ev4 / s4,
                                      "cells_per_s": c4 * c4 / s4},
    }


def bench_batch(args, ntiles, steps, warmup, standalone=False):
    """Batched total viewsheds of independent tiles (sides uniform in 256..2048, observer
    1.5..30 m, max distance = tile extent, 180 sectors): the captured batch graph against the
    plain per-tile loop, both timed over whole passes on the same GPU."""
    import torch

    import paper_2003_02200_amd as tvs
    from synth import BATCH64, batch_workload

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    spec = batch_workload(ntiles, BATCH64["seed"], workers=8)
    log(f"batch: generated {len(spec)} tiles in {time.perf_counter() - t0:.1f} s")
    n = BATCH64["n_sectors"]
    flags = args.flags
    dems = [torch.from_numpy(t["dem"]).cuda() for t in spec]
    out_b = [torch.zeros(d.shape, dtype=torch.float64, device="cuda") for d in dems]
    out_t = [torch.zeros(d.shape, dtype=torch.float64, device="cuda") for d in dems]
    tiles_b = [(dems[i], out_b[i], t["spacing"], t["obs_height"], t["max_dist"]) for i, t in enumerate(spec)]
    tiles_t = [(dems[i], out_t[i], t["spacing"], t["obs_height"], t["max_dist"]) for i, t in enumerate(spec)]
    torch.cuda.synchronize()

    def timed(fn, k):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) / k

    for _ in range(warmup):
        tvs.total_viewshed_tiles(tiles_t, n, flags)
    loop_s = timed(lambda: tvs.total_viewshed_tiles(tiles_t, n, flags), steps)
    log(f"batch: per-tile loop {loop_s * 1e3:.1f} ms per pass")
    t1 = time.perf_counter()
    batch = tvs.Batch(tiles_b, n, flags=flags | tvs.FLAG_AUTOTUNE)
    create_s = time.perf_counter() - t1
    for _ in range(warmup):
        batch.run()
    batch_s = timed(batch.run, steps)
    info = batch.info()
    log(f"batch: {batch_s * 1e3:.1f} ms per pass, created in {create_s:.1f} s (tuning {info.tune_ms:.0f} ms)")
    worst = max(float((ob - ot).abs().max() / ot.abs().max()) for ob, ot in zip(out_b, out_t))
    evals = info.los_evals
    cells = sum(d.numel() for d in dems)
    res = {
        "metric": "LoS cell-evals/s, batch of independent tiles",
        "value": evals / batch_s,
        "unit": "LoS cell-evals/s",
        "ms_per_pass": batch_s * 1e3,
        "steps": steps, "warmup": warmup,
        "config": {"workload": f"batch of {len(spec)} square fractal tiles, sides {min(t['dem'].shape[0] for t in spec)}"
                               f"..{max(t['dem'].shape[0] for t in spec)}, 10 m, observer 1.5..30 m, {n} sectors, "
                               "max distance = tile extent", "tiles": len(spec), "cells": cells,
                   "los_evals_per_pass": evals, "flags": flags},
        "per_tile_loop": {"ms_per_pass": loop_s * 1e3, "value": evals / loop_s},
        "speedup_vs_per_tile_loop": loop_s / batch_s,
        "plan": {"chunks": info.chunks, "graph_kernels": info.kernel_launches, "tuned": bool(info.tuned),
                 "tune_ms": info.tune_ms, "create_s": create_s, "scratch_bytes": info.scratch_bytes,
                 "buckets": batch.buckets()},
        "max_rel_diff_vs_per_tile_loop": worst,
    }
    batch.close()
    if standalone:
        res.update({"n_gpus": 1, "ms_per_step": batch_s * 1e3, "higher_is_better": True, "scaling": "weak",
                    "vs_baseline": None, "dtype": "f32" if flags & tvs.FLAG_SLOPE_F32 else "f64",
                    "data": "synthetic"})
    return res


def bench_multiple(args):
    """Multiple viewshed (Section 5.3's GIS comparison shape): per cell, how many of 10 random POVs
    see it, on the 2000x2000 workload, in one call; timed against 10 singular viewshed calls."""
    import numpy as np
    import torch

    import paper_2003_02200_amd as tvs
    from synth import WORKLOADS, workload_dem

    w = WORKLOADS["tvs2000"]
    torch.cuda.set_device(0)
    d = torch.from_numpy(workload_dem("tvs2000")).cuda()
    rng = np.random.default_rng(2020)
    povs = [(int(rng.integers(0, 2000)), int(rng.integers(0, 2000))) for _ in range(10)]
    call = (w["spacing"], w["obs_height"], w["n_sectors"], w["max_dist"])

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    mult_s = timed(lambda: tvs.multiple_viewshed(d, *call, povs), args.steps)

    def singles():
        for (i, j) in povs:
            tvs.singular_viewshed(d, *call, i, j)

    sing_s = timed(singles, args.steps)
    cnt = tvs.multiple_viewshed(d, *call, povs)
    torch.cuda.synchronize()
    seen = int((cnt.cpu().numpy().view(np.uint32) > 0).sum())
    log(f"multiple viewshed of 10 POVs: {mult_s * 1e3:.2f} ms; 10 singular areas: {sing_s * 1e3:.2f} ms")
    print(json.dumps({
        "metric": "multiple viewshed latency (count map of 10 POVs)", "value": mult_s * 1e3, "unit": "ms",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": mult_s * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "tvs2000 grid, 10 random POVs (seed 2020), 180 sectors, 10 km"},
        "ten_singular_areas_ms": sing_s * 1e3, "cells_seen_by_any": seen,
    }), flush=True)


def bench_serve(args, seconds, cold=False, standalone=False):
    """Request serving: resident fractal grids (singular pool 512..4096, total pool 256..1024,
    10 m), a Poisson stream (seed 5) of 80 % singular requests (random POV, max distance = grid
    extent) and 20 % total requests (max distance = grid extent), observer 1.5 m, 180 sectors.
    Reports latency percentiles under the stream (overall and per kind), then the capacity with every
    request queued at once against the plain path that runs the same requests one by one."""
    import numpy as np
    import torch

    import paper_2003_02200_amd as tvs
    from synth import fractal_dem

    torch.cuda.set_device(0)
    n, h0, dx = 180, 1.5, 10.0
    sing_sides = [512, 1024, 1536, 2048, 3072, 4096]
    tot_sides = [256, 384, 512, 640, 768, 1024]
    t0 = time.perf_counter()
    grids = [fractal_dem(sd, 500 + x, 0.55, 2500.0) for x, sd in enumerate(sing_sides + tot_sides)]
    log(f"serve: generated {len(grids)} grids in {time.perf_counter() - t0:.1f} s")
    rng = np.random.default_rng(5)
    reqs = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / args.serve_rate)
        if t >= seconds:
            break
        if rng.uniform() < 0.8:
            g = int(rng.integers(0, len(sing_sides)))
            sd = sing_sides[g]
            reqs.append((t, "s", g, int(rng.integers(0, sd)), int(rng.integers(0, sd))))
        else:
            g = len(sing_sides) + int(rng.integers(0, len(tot_sides)))
            reqs.append((t, "t", g, 0, 0))
    R = [grids[r[2]].shape[0] * dx for r in reqs]
    ev_total = sum(tvs.los_evals(grids[r[2]].shape[0], grids[r[2]].shape[1], dx, n, R[x])[0]
                   for x, r in enumerate(reqs) if r[1] == "t")
    log(f"serve: {len(reqs)} requests over {seconds} s ({sum(r[1] == 't' for r in reqs)} total)")

    def run_server(paced):
        srv = tvs.Server(streams=4, max_singular_batch=64)
        ids = [srv.add_grid(g, dx) for g in grids]
        tickets = [None] * len(reqs)
        # warm the kernels
        srv.wait(srv.submit_singular(ids[0], h0, n, R[0], 0, 0))
        srv.wait(srv.submit_total(ids[-1], h0, n, grids[-1].shape[0] * dx))
        torch.cuda.synchronize()
        start = time.perf_counter()
        for x, (ta, kind, g, i, j) in enumerate(reqs):
            if paced:
                delay = start + ta - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            tickets[x] = (srv.submit_singular(ids[g], h0, n, R[x], i, j) if kind == "s"
                          else srv.submit_total(ids[g], h0, n, R[x]))
        res = [srv.wait(tk) for tk in tickets]
        wall = time.perf_counter() - start
        st = srv.stats().as_dict()
        for tk in tickets:
            srv.release(tk)
        srv.close()
        return res, wall, st

    def pct(res, kind=None, field="latency_ms"):
        v = np.array([getattr(r, field) for r, q in zip(res, reqs) if kind is None or q[1] == kind])
        return (float(np.percentile(v, 50)), float(np.percentile(v, 99))) if len(v) else (None, None)

    res_c = st_c = None
    if cold:
        # The first server of a process grows the device memory pool and the pinned staging while it
        # serves; the headline pass runs after a flood pass has done that, the cold pass is reported.
        log("serve: paced stream, cold process ...")
        res_c, _, st_c = run_server(True)
        assert all(r.status == 0 for r in res_c)
        log(f"serve: cold p99 {pct(res_c)[1]:.2f} ms, singular p99 {pct(res_c, 's')[1]:.2f} ms")
    log("serve: flood (every request queued at once) ...")
    res_f, wall_f, st_f = run_server(False)
    assert all(r.status == 0 for r in res_f)
    log(f"serve: flood {len(reqs) / wall_f:.1f} req/s")
    log("serve: paced stream ...")
    res, wall, st = run_server(True)
    assert all(r.status == 0 for r in res)
    log(f"serve: paced p50 {pct(res)[0]:.2f} ms p99 {pct(res)[1]:.2f} ms, singular p99 {pct(res, 's')[1]:.2f} ms, "
        f"total p99 {pct(res, 't')[1]:.2f} ms over {wall:.1f} s")
    log("serve: plain path, one request at a time ...")
    dg = [torch.from_numpy(g).cuda() for g in grids]
    tvs.singular_viewshed(dg[0], dx, h0, n, R[0], 0, 0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for x, (ta, kind, g, i, j) in enumerate(reqs):
        if kind == "s":
            tvs.singular_viewshed(dg[g], dx, h0, n, R[x], i, j)
        else:
            tvs.total_viewshed(dg[g], dx, h0, n, R[x])
            torch.cuda.synchronize()
    plain = time.perf_counter() - t1
    log(f"serve: plain {len(reqs) / plain:.1f} req/s")

    def per_launch(stt):
        return {"singular_queries_per_launch": stt["singular_batched"] / max(stt["singular_batches"], 1),
                "total_queries_per_launch": (stt["total_batched"] / max(stt["total_batches"], 1))
                if "total_batches" in stt else 1.0}

    out = {
        "metric": "p50/p99 serve latency (ms), Poisson request stream",
        "value": pct(res)[1],
        "unit": "ms (p99)",
        "config": {"workload": f"{len(reqs)} requests, Poisson {args.serve_rate:g}/s for {seconds:g} s: "
                               "80% singular on grids 512..4096, 20% total on grids 256..1024, 10 m, observer 1.5 m, "
                               "180 sectors, max distance = grid extent", "requests": len(reqs)},
        "latency_ms": {"p50": pct(res)[0], "p99": pct(res)[1], "singular_p50": pct(res, "s")[0],
                       "singular_p99": pct(res, "s")[1], "total_p50": pct(res, "t")[0], "total_p99": pct(res, "t")[1],
                       "singular_queue_p99": pct(res, "s", "queue_ms")[1]},
        "served_req_per_s": len(reqs) / wall,
        "capacity_req_per_s": len(reqs) / wall_f,
        "plain_one_at_a_time_req_per_s": len(reqs) / plain,
        "capacity_vs_plain": plain / wall_f,
        "total_los_evals_per_s_at_capacity": ev_total / wall_f,
        "batching_paced": per_launch(st),
        "batching_flood": per_launch(st_f),
        "server_paced": st, "server_flood": st_f,
    }
    if cold:
        out["latency_ms_cold_process"] = {"p50": pct(res_c)[0], "p99": pct(res_c)[1],
                                          "singular_p99": pct(res_c, "s")[1], "total_p99": pct(res_c, "t")[1]}
    if standalone:
        out.update({"n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": wall * 1e3, "higher_is_better": False,
                    "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic"})
    return out


if __name__ == "__main__":
    main()
