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
# VALU issue ceiling of MI355X for unpacked FP32 and FP64 vector instructions:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-instructions per second
VALU_PEAK_TINSTR = 256 * 4 * 16 * 2.4e9 / 1e12

# Per-unit figures of the dominant kernel measured with rocprofv3 on these
# workloads and launch shapes (profiles/k_stage12_shock_bubble_2d_counters.md,
# profiles/k_stage12_dual_gas_layer_2d_counters.md,
# profiles/k_baro12_vapour_bubble_wall_2d_counters.md,
# profiles/k_bface3_cube_to_sphere_3d_counters.md,
# profiles/k_face3_liquid_jet_3d_counters.md): executed VALU lane-instructions
# per cell-stage (SQ_INSTS_VALU x 64 / cells; in 3D the closure and face kernels
# of a stage together) and HBM bytes per stage (FETCH_SIZE x 2.0 + WRITE_SIZE x
# 1.0 in KiB, factors from a 1 GiB device copy).  Keyed by (workload,
# precision, tile, kernel build).
KERNEL_BUILD = "k_stage12-v13"
MEASURED = {
    ("shock_bubble_2d", 0, 10, "k_stage12-v13"): dict(valu_per_cell_stage=3526591.4 * 64 / 262144,
                                             traffic_bytes=(9771.0 * 2 + 10242.1) * 1024),
    ("shock_bubble_2d", 1, 10, "k_stage12-v13"): dict(valu_per_cell_stage=3373269.2 * 64 / 262144,
                                             traffic_bytes=(4965.6 * 2 + 5122.1) * 1024),
    ("dual_gas_layer_2d", 0, 10, "k_stage12-v13"): dict(valu_per_cell_stage=8795769.9 * 64 / 524288,
                                               traffic_bytes=(22478.6 * 2 + 24580.1) * 1024),
    ("dual_gas_layer_2d", 1, 9, "k_stage12-v13"): dict(valu_per_cell_stage=8557505.1 * 64 / 524288,
                                               traffic_bytes=(11345.9 * 2 + 12296.1) * 1024),
    ("vapour_bubble_wall_2d", 0, 9, "k_stage12-v13"): dict(valu_per_cell_stage=8114414.4 * 64 / 524288,
                                                   traffic_bytes=(15062.4 * 2 + 16392.1) * 1024),
    ("vapour_bubble_wall_2d", 1, 10, "k_stage12-v13"): dict(valu_per_cell_stage=6842057.9 * 64 / 524288,
                                                   traffic_bytes=(7599.0 * 2 + 8196.1) * 1024),
    ("liquid_jet_3d", 0, 4, "k_stage12-v13"): dict(valu_per_cell_stage=(333992682.4 + 1326082430.9) * 64 / 33554432,
                                           traffic_bytes=((928041.1 + 3522144.5) * 2 +
                                                          (2547827.9 + 1673987.5)) * 1024),
    ("liquid_jet_3d", 1, 0, "k_stage12-v13"): dict(valu_per_cell_stage=(376349584.9 + 1422188568.0) * 64 / 33554432,
                                           traffic_bytes=((462805.9 + 1687499.4) * 2 +
                                                          (1215968.9 + 814903.5)) * 1024),
    ("cube_to_sphere_3d", 0, 4, "k_stage12-v13"): dict(valu_per_cell_stage=(51613794.0 + 412734614.7) * 64 / 16777216,
                                               traffic_bytes=((339514.1 + 1350660.6) * 2 +
                                                              (1230793.9 + 682506.0)) * 1024),
    ("cube_to_sphere_3d", 1, 4, "k_stage12-v13"): dict(valu_per_cell_stage=(55545824.0 + 360647183.0) * 64 / 16777216,
                                               traffic_bytes=((164659.7 + 629517.9) * 2 +
                                                              (674552.5 + 358678.3)) * 1024),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's own step count: 200 in 3D, 500 for the batch, 1e4 for the drop, else 2000)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="shock_bubble_2d",
                    choices=["shock_bubble_2d", "drop_2d", "bubble_collapse_batch", "liquid_jet_3d",
                             "liquid_jet_3d_viscous", "dual_gas_layer_2d", "vapour_bubble_wall_2d",
                             "cube_to_sphere_3d", "interface_advection_1d"])
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed"])
    ap.add_argument("--tile", type=int, default=-1, help="stage-kernel tile index (-1: autotune)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU-baseline sample length")
    ap.add_argument("--retune", action="store_true", help="re-run the tile autotuner and store its choice")
    ap.add_argument("--timing-steps", type=int, default=20, help="steps of per-stage event timing")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 5 times (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = DEFAULT_STEPS.get(args.workload, 2000)
    return args


# step counts the workloads are specified with (the 3D cases 200 steps, the
# batch of bubble collapses 500 steps each, the drop 10^4 steps)
DEFAULT_STEPS = {"bubble_collapse_batch": 500, "liquid_jet_3d": 200, "liquid_jet_3d_viscous": 200,
                 "cube_to_sphere_3d": 200, "drop_2d": 10000}


def copy_probe(mib):
    """device-to-device copy of a known size: read mib MiB, write mib MiB per copy"""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    print(json.dumps({"copy_probe_mib": mib, "ms_per_copy": ms, "GBs": 2 * mib * (1 << 20) / (ms * 1e-3) / 1e9}))


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
    if name == "dual_gas_layer_2d":
        return [W.dual_gas_layer_2d(1024, 512, steps)], dict(workload=name, nx=1024, ny=512, components=3,
                                                             sigma=0.028)
    if name == "vapour_bubble_wall_2d":
        return [W.vapour_bubble_wall_2d(1024, 512, steps)], dict(workload=name, nx=1024, ny=512, dx=4e-6,
                                                                 model="barotropic")
    if name == "cube_to_sphere_3d":
        return [W.cube_to_sphere_3d(256, steps)], dict(workload=name, nx=256, ny=256, nz=256, sigma=800.0,
                                                       model="barotropic")
    if name == "liquid_jet_3d_viscous":
        return [W.liquid_jet_3d(512, 256, 256, steps, viscous=True)], dict(workload=name, nx=512, ny=256, nz=256)
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
        tile, tune = tuner.autotune(h, prec, verbose=True, retune=args.retune, save=args.retune)
        # the tuner advances the state: start the measured run from the initial state again
        if batch:
            for i in range(len(cases)):
                h.init_primitive(i)
        else:
            h.init_primitive()
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
    nq = h.nq
    return dict(handle=h, ncell=ncell, ms=ms, stage_ms=stage_ms, nq=nq, tile=tile,
                tune={str(k): round(v, 5) for k, v in (tune or {}).items()})


def kernel_name(case):
    baro = int(case["eos"].get("model", 0)) == 1
    if case["grid"]["dim"] == 3:
        return "k_bprim3+k_bface3" if baro else "k_prim3+k_face3"
    return "k_baro12" if baro else "k_stage12"


def l1_errors(a, b, uref):
    """relative L1 of the mixed-path primitives a against FP64-path b"""
    n = a.shape[1]
    out = {
        "rho": float(np.abs(a[0] - b[0]).sum() / np.abs(b[0]).sum()),
        "u": float(np.abs(a[1:4] - b[1:4]).sum() / (n * uref)),
        "p": float(np.abs(a[4] - b[4]).sum() / np.abs(b[4]).sum()),
        "Y": float(np.abs(a[6] - b[6]).sum() / n),
    }
    if a.shape[0] > 9:
        out["Y2"] = float(np.abs(a[9] - b[9]).sum() / n)
    return out


def cpu_baseline(cases, seconds):
    """the oracle on the host cores, on a bounded sample of the workload: whole
    steps of the first case (for the large 3D cases a reduced grid of the same case)
    until about `seconds` of CPU work"""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import workloads as W
    case = cases[0]
    if case["grid"]["dim"] == 3 and np.prod(case["grid"]["n"]) > 2_000_000:
        if case["name"] == "cube_to_sphere_3d":
            case = W.cube_to_sphere_3d(64, 1)
        else:
            case = W.liquid_jet_3d(128, 64, 64, steps=1, viscous=case.get("viscous", False))
    o = Oracle(case)
    q = o.cons_from_prim()
    t0 = time.perf_counter()
    t, k = 0.0, 0
    while k < 2 or time.perf_counter() - t0 < seconds:
        t, _ = o.step(q, k, t)
        k += 1
    sec = time.perf_counter() - t0
    ncell = int(np.prod(case["grid"]["n"]))
    return dict(value=ncell * 4 * k / sec, unit="cell-RK-stage updates/s", cores=int(o.L.og_nthreads()),
                kind="oracle", sample=f"{case['name']} {'x'.join(str(n) for n in case['grid']['n'][:case['grid']['dim']])}"
                f" cells, {k} steps from the initial state", seconds=round(sec, 2))


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("fvm runs on one GPU: the decomposition over several GPUs is a design that is not "
              "built, so --gpus must be 1", file=sys.stderr)
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
    # average duration of one stage launch: the HIP-event-timed region on the
    # solver's stream holds 4 stage launches per step (and one tiny step-counter
    # kernel per 50 steps)
    stage_avg_ms = r["ms"] / (4 * args.steps)
    hbm_alg = r["ncell"] * bytes_per_cell_stage / (stage_avg_ms * 1e-3) / 1e9
    meas = MEASURED.get((args.workload, main_prec, r["tile"], KERNEL_BUILD))
    if meas:
        achieved = meas["valu_per_cell_stage"] * r["ncell"] / (stage_avg_ms * 1e-3) / 1e12
        traffic = meas["traffic_bytes"]
    else:
        achieved, traffic = None, None
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
            "bound": "alu",
            "achieved": achieved,
            "peak": VALU_PEAK_TINSTR,
            "unit": "T VALU lane-instr/s",
            "frac": None if achieved is None else achieved / VALU_PEAK_TINSTR,
            "traffic": traffic,
            "kernel": kernel_name(cases[0]),
            "kernel_build": KERNEL_BUILD,
            "valu_per_cell_stage": None if meas is None else meas["valu_per_cell_stage"],
            "stage_launch_ms": stage_avg_ms,
            "stage_ms": r["stage_ms"],
            "hbm": {"algorithmic_bytes_per_cell_stage": bytes_per_cell_stage, "achieved_GBs": hbm_alg,
                    "peak_GBs": HBM_PEAK_GBS, "frac": hbm_alg / HBM_PEAK_GBS,
                    "counter_GBs": None if traffic is None else traffic / (stage_avg_ms * 1e-3) / 1e9},
            "tile": r["tile"],
            "tune_ms_per_stage": r["tune"],
        },
    }
    if fvm.FVM_MIXED in res and len(paths) == 2:
        m = res[fvm.FVM_MIXED]
        mv = m["ncell"] * 4 * args.steps / (m["ms"] * 1e-3)
        mavg = m["ms"] / (4 * args.steps)
        mach = m["ncell"] * 2.75 * m["nq"] * 4 / (mavg * 1e-3) / 1e9
        entry = {"value": mv, "ms_per_step": m["ms"] / args.steps, "dtype": "f32+f64-closure",
                 "stage_ms": m["stage_ms"], "achieved_GBs": mach, "frac": mach / HBM_PEAK_GBS,
                 "tile": m["tile"], "tune_ms_per_stage": m["tune"]}
        mm = MEASURED.get((args.workload, fvm.FVM_MIXED, m["tile"], KERNEL_BUILD))
        if mm:
            entry["valu_frac"] = mm["valu_per_cell_stage"] * m["ncell"] / (mavg * 1e-3) / 1e12 / VALU_PEAK_TINSTR
        if len(cases) == 1:
            uref = {"shock_bubble_2d": 113.5, "drop_2d": 0.53, "liquid_jet_3d": 300.0, "liquid_jet_3d_viscous": 300.0,
                    "dual_gas_layer_2d": 25.0, "vapour_bubble_wall_2d": 31.6, "cube_to_sphere_3d": 3.0,
                    "interface_advection_1d": 100.0}.get(args.workload, 1.0)
            entry["l1_vs_fp64"] = l1_errors(m["handle"].get_primitive(), r["handle"].get_primitive(), uref)
        out["mixed"] = entry
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cases, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
