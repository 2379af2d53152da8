"""Benchmark of the gfx950 solver: cell-RK-stage updates per second.

Default workload: the 3D liquid jet (Section 4.7 shape), 512 x 256 x 256
cells, Peng-Robinson gas, CSF, sensor switching; the headline is the path its
configuration names (mixed: FP32 storage and fluxes, FP64 closure), with the
FP64 path measured beside it.  `--steps` time steps of four stages each, the
state resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 200] [--warmup 50] [--workload liquid_jet_3d]
"""
import argparse
import glob
import hashlib
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

# the precision each workload's configuration names for its headline
MAIN_PRECISION = {"liquid_jet_3d": "mixed", "liquid_jet_3d_viscous": "mixed", "drop_2d": "mixed",
                  "bubble_collapse_batch": "mixed", "shock_bubble_2d": "fp64", "dual_gas_layer_2d": "fp64",
                  "vapour_bubble_wall_2d": "fp64", "cube_to_sphere_3d": "fp64", "interface_advection_1d": "fp64"}


def kernel_source_hash():
    """hash of the HIP/C++ sources the library is built from: rocprofv3 counter
    figures below are valid only for the build they were taken on"""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2304_00140_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:12]


# rocprofv3 --pmc figures of the stage kernels on these workloads and launch
# shapes (files under profiles/ named for kernel and workload give the
# commands; a 3D stage sums its closure and face kernels): executed VALU
# lane-instructions per cell-stage (SQ_INSTS_VALU x 64 / cells) and HBM bytes
# per stage launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 in KiB, the factors
# read off a 1 GiB device copy).  Keyed by (workload,
# precision, tile, hash of the kernel sources); a key that does not match the
# built sources reports null instead of stale numbers.
MEASURED = {
    ("liquid_jet_3d", "mixed", 4, "1194ec10b665"): {"valu_per_cell_stage": 1809.2, "traffic_bytes": 8254990131},
    ("liquid_jet_3d", "fp64", 15, "1194ec10b665"): {"valu_per_cell_stage": 2268.1, "traffic_bytes": 14588750395},
    ("liquid_jet_3d", "mixed", 7, "1194ec10b665"): {"valu_per_cell_stage": 1968.1, "traffic_bytes": 3098237986},
    ("liquid_jet_3d", "fp64", 7, "1194ec10b665"): {"valu_per_cell_stage": 2320.7, "traffic_bytes": 5786164187},
    ("shock_bubble_2d", "fp64", 10, "1194ec10b665"): {"valu_per_cell_stage": 821.6, "traffic_bytes": 30496587},
    ("shock_bubble_2d", "mixed", 10, "1194ec10b665"): {"valu_per_cell_stage": 783.0, "traffic_bytes": 15420247},
    ("drop_2d", "mixed", 1, "1194ec10b665"): {"valu_per_cell_stage": 1399.0, "traffic_bytes": 4050920},
    ("drop_2d", "fp64", 1, "1194ec10b665"): {"valu_per_cell_stage": 1497.5, "traffic_bytes": 7879764},
    ("bubble_collapse_batch", "mixed", 3, "1194ec10b665"): {"valu_per_cell_stage": 1049.7, "traffic_bytes": 432785685},
    ("bubble_collapse_batch", "fp64", 3, "1194ec10b665"): {"valu_per_cell_stage": 1117.8, "traffic_bytes": 862843361},
    ("vapour_bubble_wall_2d", "fp64", 9, "1194ec10b665"): {"valu_per_cell_stage": 926.5, "traffic_bytes": 47624930},
    ("vapour_bubble_wall_2d", "mixed", 10, "1194ec10b665"): {"valu_per_cell_stage": 796.3, "traffic_bytes": 23957217},
    ("cube_to_sphere_3d", "fp64", 16, "1194ec10b665"): {"valu_per_cell_stage": 1445.4, "traffic_bytes": 5560591824},
    ("cube_to_sphere_3d", "mixed", 15, "1194ec10b665"): {"valu_per_cell_stage": 1248.8, "traffic_bytes": 3249863504},
    ("dual_gas_layer_2d", "fp64", 10, "1194ec10b665"): {"valu_per_cell_stage": 1023.5, "traffic_bytes": 71383045},
    ("dual_gas_layer_2d", "mixed", 10, "1194ec10b665"): {"valu_per_cell_stage": 907.9, "traffic_bytes": 35798626},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's own step count: 200 in 3D, 500 for the batch, 1e4 for the drop, else 2000)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="liquid_jet_3d",
                    choices=["shock_bubble_2d", "drop_2d", "bubble_collapse_batch", "liquid_jet_3d",
                             "liquid_jet_3d_viscous", "dual_gas_layer_2d", "vapour_bubble_wall_2d",
                             "cube_to_sphere_3d", "interface_advection_1d"])
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed"])
    ap.add_argument("--tile", type=int, default=-1, help="stage-kernel tile index (-1: autotune)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU-baseline sample length")
    ap.add_argument("--retune", action="store_true", help="re-run the tile autotuner and store its choice")
    ap.add_argument("--timing-steps", type=int, default=20, help="steps of per-stage event timing")
    ap.add_argument("--drop-diag-steps", type=int, default=None,
                    help="drop_2d: steps of the Laplace-jump / spurious-current diagnostics after the timed "
                         "region (default: the configured 1e4; 0 skips them)")
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


def kernel_name(case, tile):
    from paper_2304_00140_amd import fvm
    baro = int(case["eos"].get("model", 0)) == 1
    dim = case["grid"]["dim"]
    if dim == 3:
        if baro:
            return "k_bprim3+k_csf_zero+k_bface3" if float(case["scheme"].get("sigma", 0.0)) > 0.0 else "k_bprim3+k_bface3"
        pair = "k_prim3+k_csf_zero+k_face3" if float(case["scheme"].get("sigma", 0.0)) > 0.0 else "k_prim3+k_face3"
        return {1: pair, 2: "k_march3", 3: "k_prim3+k_march3"}[fvm.lib().fvm_tile_kernels(dim, tile)]
    return "k_baro12" if baro else "k_stage12"


def linf_errors(a, b, uref):
    """largest difference of the mixed-path primitives a against FP64-path b:
    rho and p over the field's largest magnitude, u over U_ref, xi as is"""
    out = {
        "rho": float(np.abs(a[0] - b[0]).max() / np.abs(b[0]).max()),
        "u": float(np.abs(a[1:4] - b[1:4]).max() / uref),
        "p": float(np.abs(a[4] - b[4]).max() / np.abs(b[4]).max()),
        "Y": float(np.abs(a[6] - b[6]).max()),
    }
    if a.shape[0] in (11,):
        out["Y2"] = float(np.abs(a[9] - b[9]).max())
    return out


def l1_errors(a, b, uref):
    """relative L1 of the mixed-path primitives a against FP64-path b: rho and
    p over the field's L1 norm, u over N U_ref, xi (and xi_2) over N"""
    n = a.shape[1]
    out = {
        "rho": float(np.abs(a[0] - b[0]).sum() / np.abs(b[0]).sum()),
        "u": float(np.abs(a[1:4] - b[1:4]).sum() / (n * uref)),
        "p": float(np.abs(a[4] - b[4]).sum() / np.abs(b[4]).sum()),
        "Y": float(np.abs(a[6] - b[6]).sum() / n),
    }
    if a.shape[0] in (11,):
        out["Y2"] = float(np.abs(a[9] - b[9]).sum() / n)
    return out


def drop_physics(case, prec, stream, steps, every, tile):
    """Section 4.4 / Appendix C diagnostics of the static drop: the Laplace
    jump <p>_{r < R/2} - <p>_{r > 3R/2} against sigma / R, and the largest
    spurious speed max |u| against the step"""
    from paper_2304_00140_amd import fvm, workloads as W
    ctx = fvm.Context(case, prec, stream=stream.cuda_stream)
    ctx.set_tile(tile)
    ctx.init_primitive()
    x, y = W.cell_centres(case["grid"])
    Lx = case["grid"]["n"][0] * case["grid"]["dx"][0]
    r = np.hypot(x - 0.5 * Lx, y - 0.5 * Lx)
    R = case["radius"]
    sig = case["scheme"]["sigma"]
    inner, outer = r < 0.5 * R, r > 1.5 * R
    umax, done = [], 0
    while done < steps:
        k = min(every, steps - done)
        ctx.n_steps(k)
        done += k
        w = ctx.get_primitive()
        umax.append([done, float(np.hypot(w[1], w[2]).max())])
    dp = float(w[4][inner].mean() - w[4][outer].mean())
    ctx.close()
    return dict(steps=steps, laplace_dp_Pa=dp, sigma_over_R_Pa=sig / R, laplace_ratio=dp * R / sig,
                max_u_vs_step=umax), w


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
    ncell = int(np.prod(case["grid"]["n"]))

    def timed(budget):
        q = o.cons_from_prim()
        t0 = time.perf_counter()
        t, k = 0.0, 0
        while k < 2 or time.perf_counter() - t0 < budget:
            t, _ = o.step(q, k, t)
            k += 1
        return k, time.perf_counter() - t0

    cores = int(o.L.og_nthreads())
    k, sec = timed(seconds)
    # the same sample on one thread, over a third of the time
    o.L.og_set_nthreads(1)
    k1, sec1 = timed(seconds / 3.0)
    o.L.og_set_nthreads(cores)
    return dict(value=ncell * 4 * k / sec, unit="cell-RK-stage updates/s", cores=cores,
                kind="oracle", sample=f"{case['name']} {'x'.join(str(n) for n in case['grid']['n'][:case['grid']['dim']])}"
                f" cells, {k} steps from the initial state", seconds=round(sec, 2),
                one_thread=dict(value=ncell * 4 * k1 / sec1, steps=k1, seconds=round(sec1, 2)))


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
    main_name = MAIN_PRECISION.get(args.workload, "fp64") if args.precision == "both" else args.precision
    other = {"fp64": "mixed", "mixed": "fp64"}[main_name]
    names = [main_name] + ([other] if args.precision == "both" else [])
    code = {"fp64": fvm.FVM_FP64, "mixed": fvm.FVM_MIXED}
    res = {}
    for name in names:
        res[name] = run_path(cases, code[name], args, stream, torch)
        print(f"# {name}: {res[name]['ms']:.2f} ms for {args.steps} steps, "
              f"stage ms {[round(x, 4) for x in res[name]['stage_ms']]}", file=sys.stderr, flush=True)
    src_hash = kernel_source_hash()

    def path_entry(name):
        r = res[name]
        word = 8 if name == "fp64" else 4
        bpcs = 2.75 * r["nq"] * word           # algorithmic bytes per cell-stage
        # one stage launch on average: the HIP-event-timed region on the
        # solver's stream holds 4 stage launches per step (and one tiny
        # step-counter kernel per 50 steps)
        stage_ms = r["ms"] / (4 * args.steps)
        alg_bytes = r["ncell"] * bpcs
        achieved = alg_bytes / (stage_ms * 1e-3) / 1e9
        meas = MEASURED.get((args.workload, name, r["tile"], src_hash))
        valu = None
        if meas:
            vps = meas["valu_per_cell_stage"]
            valu = {"per_cell_stage": vps, "achieved_T_lane_instr_s": vps * r["ncell"] / (stage_ms * 1e-3) / 1e12,
                    "peak": VALU_PEAK_TINSTR,
                    "frac": vps * r["ncell"] / (stage_ms * 1e-3) / 1e12 / VALU_PEAK_TINSTR}
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": meas["traffic_bytes"] if meas else None,
                "kernel": kernel_name(cases[0], r["tile"]), "kernel_src": src_hash,
                "algorithmic_bytes_per_cell_stage": bpcs, "algorithmic_bytes_per_launch": alg_bytes,
                "stage_launch_ms": stage_ms, "stage_ms": r["stage_ms"], "tile": r["tile"],
                "tune_ms_per_stage": r["tune"], "valu": valu}
        return dict(value=r["ncell"] * 4 * args.steps / (r["ms"] * 1e-3), ms_per_step=r["ms"] / args.steps,
                    dtype="f64" if name == "fp64" else "f32+f64-closure", roofline=roof)

    main_e = path_entry(main_name)
    out = {
        "metric": "cell-RK-stage updates/s + HBM GB/s frac, FP64 vs mixed FP32 at stated L1 err",
        "value": main_e["value"],
        "unit": "cell-RK-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_e["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_e["dtype"],
        "data": "synthetic",
        "config": dict(cfg, cells=res[main_name]["ncell"], steps=args.steps, precision=main_name,
                       parallelism="single-gpu"),
        "roofline": main_e["roofline"],
    }
    if len(names) == 2:
        e = path_entry(other)
        if len(cases) == 1:
            uref = {"shock_bubble_2d": 113.5, "drop_2d": 0.53, "liquid_jet_3d": 300.0, "liquid_jet_3d_viscous": 300.0,
                    "dual_gas_layer_2d": 25.0, "vapour_bubble_wall_2d": 31.6, "cube_to_sphere_3d": 3.0,
                    "interface_advection_1d": 100.0}.get(args.workload, 1.0)
            wm, wf = res["mixed"]["handle"].get_primitive(), res["fp64"]["handle"].get_primitive()
            out["l1_mixed_vs_fp64"] = l1_errors(wm, wf, uref)
            out["linf_mixed_vs_fp64"] = linf_errors(wm, wf, uref)
        out[other] = e
    diag = DEFAULT_STEPS["drop_2d"] if args.drop_diag_steps is None else args.drop_diag_steps
    if args.workload == "drop_2d" and diag > 0:
        # the static drop over its configured 10^4 steps (by default), both paths, outside the timed region
        phys = {}
        ws = {}
        for name in names:
            phys[name], ws[name] = drop_physics(cases[0], code[name], stream, diag, min(1000, diag),
                                                   res[name]["tile"])
        if len(names) == 2:
            R, sig = cases[0]["radius"], cases[0]["scheme"]["sigma"]
            phys["mixed_vs_fp64_p_max_over_sigma_R"] = float(np.abs(ws["mixed"][4] - ws["fp64"][4]).max() * R / sig)
            phys["l1_mixed_vs_fp64"] = l1_errors(ws["mixed"], ws["fp64"], 0.53)
        out["drop_physics"] = phys
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cases, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
