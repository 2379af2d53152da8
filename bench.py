"""Benchmark of the gfx950 solver: cell-RK-stage updates per second.

Default workload: the 2D shock-helium-bubble case, 1024 x 256 cells, FP64 and
mixed (FP32 storage and fluxes, FP64 closure) paths, `--steps` time steps of
four stages each, state resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 2000] [--warmup 50] [--workload shock_bubble_2d]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="shock_bubble_2d",
                    choices=["shock_bubble_2d", "drop_2d", "bubble_collapse_batch", "liquid_jet_3d",
                             "interface_advection_1d"])
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed"])
    ap.add_argument("--tile", type=int, default=-1, help="stage-kernel tile index (-1: autotune)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=4)
    ap.add_argument("--timing-steps", type=int, default=20, help="steps of per-stage event timing")
    return ap.parse_args()


def make_workload(name, steps):
    from paper_2304_00140_amd import workloads as W
    if name == "shock_bubble_2d":
        return [W.shock_bubble_2d(1024, 256, steps)], dict(workload=name, nx=1024, ny=256)
    if name == "drop_2d":
        return [W.drop_2d(256, steps)], dict(workload=name, nx=256, ny=256, sigma=0.07)
    if name == "interface_advection_1d":
        return [W.interface_advection_1d(200)], dict(workload=name, nx=200)
    if name == "bubble_collapse_batch":
        cases = W.bubble_collapse_batch(256, steps=steps)
        return cases, dict(workload=name, cases=256, n_min=64, n_max=256)
    if name == "liquid_jet_3d":
        return [W.liquid_jet_3d(512, 256, 256, steps)], dict(workload=name, nx=512, ny=256, nz=256)
    raise ValueError(name)


def run_path(cases, prec, args, stream, torch):
    from paper_2304_00140_amd import fvm
    batch = len(cases) > 1
    if batch:
        h = fvm.Batch(cases, prec, stream=stream.cuda_stream)
        for i in range(len(cases)):
            h.init_primitive(i)
        ncell = h.cells()
    else:
        h = fvm.Context(cases[0], prec, stream=stream.cuda_stream)
        h.init_primitive()
        ncell = h.ncell
    if args.tile >= 0:
        h.set_tile(args.tile)
        tile, tune = args.tile, None
    else:
        from paper_2304_00140_amd import tune as tuner
        tile, tune = tuner.autotune(h, prec, verbose=True)
    h.n_steps(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    h.n_steps(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    stage_ms = h.time_stages(args.timing_steps)
    nq = cases[0]["grid"]["dim"] + 3
    return dict(handle=h, ncell=ncell, ms=ms, stage_ms=stage_ms, nq=nq, tile=tile,
                tune={str(k): round(v * 1e3, 3) for k, v in (tune or {}).items()})


def l1_errors(a, b, uref):
    """relative L1 of the mixed-path primitives a against FP64-path b"""
    n = a.shape[1]
    return {
        "rho": float(np.abs(a[0] - b[0]).sum() / np.abs(b[0]).sum()),
        "u": float(np.abs(a[1:4] - b[1:4]).sum() / (n * uref)),
        "p": float(np.abs(a[4] - b[4]).sum() / np.abs(b[4]).sum()),
        "Y": float(np.abs(a[6] - b[6]).sum() / n),
    }


def cpu_baseline(cases, steps):
    from oracle.oracle import Oracle
    case = cases[0]
    o = Oracle(case)
    q = o.cons_from_prim()
    t0 = time.perf_counter()
    t = 0.0
    for k in range(steps):
        t, _ = o.step(q, k, t)
    sec = time.perf_counter() - t0
    ncell = int(np.prod(case["grid"]["n"]))
    return dict(value=ncell * 4 * steps / sec, unit="cell-RK-stage updates/s", cores=int(o.L.og_nthreads()),
                kind="oracle", sample=f"{case['name']} {ncell} cells x {steps} steps (first case only)",
                seconds=round(sec, 3))


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("this build runs on one GPU; the multi-GPU decomposition is described in DESIGN.md, "
              "not launched", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2304_00140_amd import build, fvm
    if not os.path.exists(fvm.LIB_PATH):
        build.build()
    fvm.lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    cases, cfg = make_workload(args.workload, args.steps)
    paths = {"both": [fvm.FVM_FP64, fvm.FVM_MIXED], "fp64": [fvm.FVM_FP64], "mixed": [fvm.FVM_MIXED]}[args.precision]
    res = {}
    for prec in paths:
        res[prec] = run_path(cases, prec, args, stream, torch)
        print(f"# {'fp64' if prec == 0 else 'mixed'}: {res[prec]['ms']:.2f} ms for {args.steps} steps, "
              f"stage ms {[round(x, 4) for x in res[prec]['stage_ms']]}", file=sys.stderr, flush=True)
    main_prec = paths[0]
    r = res[main_prec]
    cell_stages = r["ncell"] * 4 * args.steps
    value = cell_stages / (r["ms"] * 1e-3)
    word = 8 if main_prec == fvm.FVM_FP64 else 4
    bytes_per_cell_stage = 2.75 * r["nq"] * word
    stage_avg_ms = float(np.mean(r["stage_ms"]))
    achieved = r["ncell"] * bytes_per_cell_stage / (stage_avg_ms * 1e-3) / 1e9
    out = {
        "metric": "cell-RK-stage updates/s + HBM GB/s frac, FP64 vs mixed FP32 at stated L1 err",
        "value": value,
        "unit": "cell-RK-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == fvm.FVM_FP64 else "f32+f64-closure",
        "data": "synthetic",
        "config": dict(cfg, cells=r["ncell"], steps=args.steps, parallelism="single-gpu"),
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "k_stage12" if cases[0]["grid"]["dim"] < 3 else "k_stage3",
            "algorithmic_bytes_per_cell_stage": bytes_per_cell_stage,
            "stage_ms": r["stage_ms"],
            "tile": r["tile"],
            "tune_us_per_stage": r["tune"],
        },
    }
    if fvm.FVM_MIXED in res and len(paths) == 2:
        m = res[fvm.FVM_MIXED]
        mv = m["ncell"] * 4 * args.steps / (m["ms"] * 1e-3)
        mavg = float(np.mean(m["stage_ms"]))
        mach = m["ncell"] * 2.75 * m["nq"] * 4 / (mavg * 1e-3) / 1e9
        entry = {"value": mv, "ms_per_step": m["ms"] / args.steps, "dtype": "f32+f64-closure",
                 "stage_ms": m["stage_ms"], "achieved_GBs": mach, "frac": mach / HBM_PEAK_GBS,
                 "tile": m["tile"], "tune_us_per_stage": m["tune"]}
        if len(cases) == 1:
            uref = {"shock_bubble_2d": 113.5, "drop_2d": 0.53, "liquid_jet_3d": 300.0,
                    "interface_advection_1d": 100.0}.get(args.workload, 1.0)
            entry["l1_vs_fp64"] = l1_errors(m["handle"].get_primitive(), r["handle"].get_primitive(), uref)
        out["mixed"] = entry
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cases, args.cpu_sample_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
