#!/usr/bin/env python3
"""Throughput of the fused fluctuating D2Q9 step on one MI355X.

Workload (default): 8192 x 8192 periodic single phase (rho0 = 1, A = 0.05, B = 0.04,
kappa = 0.02, c0sq = 1/3, tau_s = tau_b = 0.8, kT = 1e-5), populations stored in FP32 as
deviations from the rest state (w_i rho0 here), every step with noise.  A "step" is one pass of the whole
update (pull-stream, density halo, stencils, equilibrium, Philox noise, MRT relaxation,
store) over the lattice.  The same workload is also timed with FP64 storage.

Prints one JSON line.  The CPU baseline is the FP64 oracle (test infrastructure) timed on
a bounded sample of the same workload; the same leg reports the FP32-shifted moment error
of the GPU against that oracle run.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % HBM roofline, FP32-shifted vs FP64, at stated S(k)/moment error"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {"fp32s": 72, "fp32": 72, "fp64": 144}   # read + write of 9 populations
COUNTERS = os.path.join(ROOT, "profiles", "k_step2_fp32s_8192_counters.json")
# VALU issue peak: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles, 2.4 GHz
VALU_PEAK_WAVE_INSTS = 256 * 4 / 4 * 2.4e9
# the byte counters depend on the step kernel (its source, RNG and shared structs) and on the
# tile list that lb_init builds
KERNEL_SRCS = [os.path.join(ROOT, "paper_1009_0254_amd", "csrc", f)
               for f in ("lb_kernels.hip", "lb_step2.hip", "lb_collide.h", "lb_rng.h", "lb_internal.h", "lb_tiles.hip")]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    """Hash of the step kernel's code: its sources without comments and whitespace, so that
    an edit of a comment does not disown the profiled byte counters."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        src = open(f).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update("".join(src.split()).encode())
    return h.hexdigest()[:16]


def time_precision(torch, L, cfg, precision, steps, warmup):
    lat = L.Lattice(cfg, precision=precision)
    lat.step(warmup)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    lat.step(steps)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    flags, t = lat.lb_status_flags()
    tune = lat.lb_tuning()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return wall, ev_ms, flags, tune


def counters_for(workload, tile):
    """The committed rocprofv3 counters of this kernel source, workload and launch
    configuration (strip width, rows, steps per launch), or None when the kernel source has
    changed since they were taken or this configuration is not one profiled."""
    try:
        c = json.load(open(COUNTERS))
    except (OSError, ValueError):
        return None
    if c.get("kernel_src_sha") != kernel_sha() or c.get("workload_key") != workload:
        return None
    return c.get("per_tile", {}).get("%d,%d,%d" % tile)


def traffic_from_counters(workload, tile):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE counters, each scaled by
    the same counter's reading of a plain copy of known size; null as in counters_for."""
    t = counters_for(workload, tile)
    return t.get("hbm_bytes_per_launch") if t else None


def kernel_name(tune, reps):
    """The step kernel that ran: two steps per launch (k_step2), or one (k_step, whose
    whole-row-strip variant runs when some replica fits one strip)."""
    if tune[3] == 2:
        return "k_step2<float,float,false>"
    return "k_step<float,float,false,false,%s>" % ("true" if any(r["nx"] <= tune[0] for r in reps) else "false")


def cpu_baseline(torch, L, cfg, steps):
    import numpy as np
    from oracle import oracle as O

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = cfg["nx"] * cfg["ny"]
    log("cpu baseline: oracle", cfg["nx"], "x", cfg["ny"], steps, "steps,", threads, "threads")
    ora = O.Oracle(cfg)
    t0 = time.perf_counter()
    ora.step(steps)
    dt = time.perf_counter() - t0
    mo = ora.moments()
    # the GPU on the same steps, FP32-shifted storage
    lat = L.Lattice(cfg, precision="fp32s")
    lat.step(steps)
    mg = lat.moments()
    lat.close()
    err = []
    for a in range(9):
        scale = np.abs(mo[a] - mo[a].mean()).max()
        err.append(float(np.abs(mg[a] - mo[a]).max() / scale))
    del mo, mg, ora
    out = {"value": n * steps / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{cfg['nx']}x{cfg['ny']} lattice of the same workload, {steps} steps, FP64 "
                     f"({dt:.1f} s)"}
    one = cpu_baseline_one_core(cfg)
    if one:
        out["one_core"] = one
    return out, err


def cpu_baseline_one_core(cfg, side=2048, steps=4):
    """The oracle on one host core (a child process with OMP_NUM_THREADS=1) on a side x side
    crop of the same workload."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r)\n"
            "from oracle import oracle as O\n"
            "cfg = dict(%r, nx=%d, ny=%d)\n"
            "o = O.Oracle(cfg); t0 = time.perf_counter(); o.step(%d); print(time.perf_counter() - t0)\n"
            % (ROOT, {k: v for k, v in cfg.items()}, side, side, steps))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        dt = float(r.stdout.strip().splitlines()[-1])
    except (subprocess.SubprocessError, ValueError, IndexError):
        return None
    log(f"cpu baseline, one core: {side}^2 x {steps} steps in {dt:.1f} s")
    return {"value": side * side * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{side}x{side} crop of the same workload, {steps} steps, FP64 ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--workload", default="single_phase_8192", choices=["slab_2048", "single_phase_8192", "ensemble_336", "quench_16384"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--no-sk", action="store_true", help="skip timing one S(k) sample")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip timing the 336-replica ensemble beside a single-lattice workload")
    ap.add_argument("--no-correlated", action="store_true",
                    help="skip timing the same lattice with spatially correlated noise")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after timing, copy this many bytes once with a plain device copy "
                         "(calibrates profiler byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the lattice would shard as y-slabs with a 2-row halo exchange per step; not built).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1009_0254_amd import lbfluct as L
    from paper_1009_0254_amd import workloads as W

    cfg = {"slab_2048": W.slab_2048, "single_phase_8192": W.single_phase_8192, "ensemble_336": W.ensemble_336, "quench_16384": W.quench_16384}[args.workload]()
    prec = "fp32s"
    reps = cfg if isinstance(cfg, list) else [cfg]
    n = sum(r["nx"] * r["ny"] for r in reps)
    if isinstance(cfg, list):
        sizes = sorted({r["nx"] for r in reps})
        mix = ", ".join("%d x %d^2" % (sum(1 for r in reps if r["nx"] == z), z) for z in sizes)
        desc = (f"d2q9 fluctuating Swift model, ensemble of {len(reps)} replicas ({mix}), "
                "kT log-uniform in [1e-6, 1e-4], FP32-shifted populations")
        cfg = dict(nx=n, ny=1, kT=None)          # for the report only
    else:
        desc = (f"d2q9 fluctuating Swift model, {cfg['nx']}x{cfg['ny']} periodic "
                f"{'two-phase' if cfg['c0sq'] == 0 else 'single phase'}, kT={cfg['kT']}, FP32-shifted populations")
    log("workload", args.workload, desc)

    wall, ev_ms, flags, tune = time_precision(torch, L, reps, prec, args.steps, args.warmup)
    ms = wall * 1e3 / args.steps
    kern_ms = ev_ms / args.steps
    mlups = n * args.steps / wall / 1e6
    achieved = BYTES_PER_UPDATE[prec] * n / (kern_ms * 1e-3) / 1e9
    log(f"fp32s: {ms:.4f} ms/step wall, {kern_ms:.4f} ms/step events, {mlups:.0f} MLUPS, {achieved:.0f} GB/s")

    out = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "nodes": n, "replicas": len(reps),
                   "nx": reps[0]["nx"], "ny": reps[0]["ny"], "precision": prec, "parallelism": "single GPU",
                   "tile": {"strip_width": tune[0], "rows": tune[1], "workgroups": tune[2],
                            "steps_per_launch": tune[3]}},
        # achieved: the algorithmic bytes of the lattice updates (one read and one write of the
        # nine populations per node and step) over the measured time per step; the two-step
        # kernel moves about half of them through HBM (see traffic)
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_from_counters(args.workload, (tune[0], tune[1], tune[3])),
                     "kernel": kernel_name(tune, reps),
                     "tile": "%d,%d" % (tune[0], tune[1]),
                     "steps_per_launch": tune[3],
                     "bytes_per_update": BYTES_PER_UPDATE[prec],
                     "algorithmic_bytes_per_launch": BYTES_PER_UPDATE[prec] * n * tune[3],
                     "launch_ms": kern_ms * tune[3]},
        "status_flags": flags,
    }
    ctr = counters_for(args.workload, (tune[0], tune[1], tune[3]))
    if ctr and ctr.get("valu_wave_insts_per_launch"):
        # the kernel's own bound: VALU instructions per launch (SQ_INSTS_VALU of the committed
        # counters, fixed by the code and the launch shape) over the measured launch time
        a = ctr["valu_wave_insts_per_launch"] / (kern_ms * tune[3] * 1e-3)
        out["roofline"]["alu"] = {"bound": "alu", "achieved": a, "peak": VALU_PEAK_WAVE_INSTS,
                                  "unit": "wave64 VALU instructions/s", "frac": a / VALU_PEAK_WAVE_INSTS}
    if not args.no_ensemble and args.workload != "ensemble_336":
        # the batched workload: 256 x 128^2 + 64 x 256^2 + 16 x 512^2 replicas in one launch,
        # timed over at least 64 steps (graph replay)
        ens = W.ensemble_336()
        ne = sum(r["nx"] * r["ny"] for r in ens)
        se = max(args.steps, 64)
        we, ee, fe, te = time_precision(torch, L, ens, prec, se, max(args.warmup, 32))
        ke = ee / se
        out["ensemble_336"] = {"MLUPS": ne * se / we / 1e6, "ms_per_step": we * 1e3 / se, "steps": se,
                               "nodes": ne, "replicas": len(ens),
                               "achieved_GBs": BYTES_PER_UPDATE[prec] * ne / (ke * 1e-3) / 1e9,
                               "frac": BYTES_PER_UPDATE[prec] * ne / (ke * 1e-3) / 1e9 / HBM_PEAK_GBS,
                               "kernel": kernel_name(te, ens),
                               "tile": {"strip_width": te[0], "rows": te[1], "workgroups": te[2],
                                        "steps_per_launch": te[3]},
                               "status_flags": fe}
        log(f"ensemble_336: {we * 1e3 / se:.4f} ms/step, {ne * se / we / 1e6:.0f} MLUPS, "
            f"frac {out['ensemble_336']['frac']:.3f}")
    if not args.no_fp64:
        w64, e64, f64, tune64 = time_precision(torch, L, reps, "fp64", max(args.steps // 2, 10), args.warmup // 2 + 1)
        s64 = max(args.steps // 2, 10)
        k64 = e64 / s64
        out["fp64"] = {"value": n * s64 / w64 / 1e6, "unit": "MLUPS", "ms_per_step": w64 * 1e3 / s64,
                       "achieved_GBs": BYTES_PER_UPDATE["fp64"] * n / (k64 * 1e-3) / 1e9,
                       "frac": BYTES_PER_UPDATE["fp64"] * n / (k64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "tile": {"strip_width": tune64[0], "rows": tune64[1], "steps_per_launch": tune64[3]}}
        out["fp32s_over_fp64"] = out["value"] / out["fp64"]["value"]
        log(f"fp64: {out['fp64']['ms_per_step']:.4f} ms/step, {out['fp64']['value']:.0f} MLUPS")
    if (not args.no_correlated and len(reps) == 1 and max(cfg["nx"], cfg["ny"]) <= 8192
            and cfg["nx"] & (cfg["nx"] - 1) == 0 and cfg["ny"] & (cfg["ny"] - 1) == 0 and cfg["kT"] > 0):
        # the same lattice with the exact Xi(k) noise: per step the FFT noise filter + the step
        sc = max(args.steps // 3, 10)
        wc, ec, fc, tc = time_precision(torch, L, [dict(cfg, noise="correlated")], prec, sc, args.warmup // 3 + 1)
        out["correlated_noise"] = {"ms_per_step": wc * 1e3 / sc, "MLUPS": n * sc / wc / 1e6,
                                   "time_over_k0_noise": (wc * 1e3 / sc) / ms, "status_flags": fc}
        log(f"correlated noise: {wc * 1e3 / sc:.4f} ms/step ({(wc * 1e3 / sc) / ms:.2f}x the k=0 noise step)")
    if not args.no_sk:
        # one S(k) sample of all nine modes of every replica (one batched pass), and one
        # radially binned density snapshot of replica 0
        lat = L.Lattice(reps, precision=prec, structure_factor=True)
        lat.step(2)
        lat.lb_structure_factor(L.LB_SK_SAMPLE, -1)       # first touch
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(3):
            lat.lb_structure_factor(L.LB_SK_SAMPLE, -1)
        e1.record(st)
        torch.cuda.synchronize()
        sk_ms = e0.elapsed_time(e1) / 3
        t0 = time.perf_counter()
        lat.lb_structure_factor(L.LB_SK_SNAPSHOT, 0)
        snap_ms = (time.perf_counter() - t0) * 1e3
        lat.close()
        del lat
        torch.cuda.empty_cache()
        out["structure_factor"] = {"sample_ms": sk_ms, "modes": 9, "replicas": len(reps),
                                   "overhead_sampling_every_20_steps": sk_ms / (20 * ms),
                                   "snapshot_rho_radial_ms": snap_ms}
        log(f"S(k) sample of all 9 modes, {len(reps)} replica(s): {sk_ms:.2f} ms "
            f"({100 * sk_ms / (20 * ms):.1f}% of 20 steps); radial rho snapshot {snap_ms:.2f} ms")
    if args.copy_probe:
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = args.copy_probe
        del src, dst
    if not args.no_cpu_baseline and len(reps) == 1:
        cb, err = cpu_baseline(torch, L, cfg, args.cpu_steps)
        out["cpu_baseline"] = cb
        out["accuracy"] = {"moment_rel_err_fp32s_vs_oracle": max(err[:3]), "all_modes": err,
                           "steps": args.cpu_steps, "tolerance": 1e-5}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
