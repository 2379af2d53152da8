"""Launch-shape autotuner for the fused stage kernels.

Times every tile shape of the context's dimension on the path that production
runs take (fvm_n_steps: HIP-graph replays of whole steps; the state advances)
and keeps the fastest.  Choices are cached per (dimension, precision,
switching, CSF on, closure kinds or the barotropic model, stress terms on, cell count): in memory for the process and in
tune_cache.json beside this file, which the tuner writes when asked
(`save=True`) and every later run reads, so that a benchmark or a profile
uses the same launch shape as the run that chose it.
"""
import ctypes as C
import json
import os
import time

CACHE_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def _load_file():
    try:
        with open(CACHE_FILE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}

_cache = {}


def key_of(handle, precision):
    case = handle.case if hasattr(handle, "case") else handle.cases[0]
    ncell = handle.ncell if hasattr(handle, "ncell") else handle.cells()
    s = case["scheme"]
    e = case["eos"]
    diff = any(v > 0 for v in list(e.get("mu", [])) + list(e.get("kc", [])))
    kinds = (("barotropic", "gas2") if len(e["kind"]) == 3 else ("barotropic",)) \
        if int(e.get("model", 0)) == 1 else tuple(e["kind"])
    return (case["grid"]["dim"], precision, int(s["switching"]), s["sigma"] > 0, kinds, diff, int(ncell))


def _restart(handle):
    if hasattr(handle, "cases"):
        for i in range(len(handle.cases)):
            handle.init_primitive(i)
    else:
        handle.init_primitive()


def autotune(handle, precision, steps=50, warm=50, verbose=False, retune=False, save=False):
    """handle: fvm.Context or fvm.Batch; returns (best tile, {tile: ms per stage}).  A sweep
    (no cached choice) leaves the handle's state at its case's initial primitives advanced by
    the last tile's timed steps: set the state again before a measured run."""
    from . import fvm
    k = key_of(handle, precision)
    if k in _cache and not retune:
        handle.set_tile(_cache[k][0])
        return _cache[k]
    stored = _load_file().get(repr(k))
    if stored is not None and not retune:
        _cache[k] = (int(stored["tile"]), {int(t): v for t, v in stored["ms_per_stage"].items()})
        handle.set_tile(_cache[k][0])
        return _cache[k]
    L = fvm.lib()
    dim = k[0]
    times = {}
    for t in range(L.fvm_tile_count(dim)):
        try:
            handle.set_tile(t)
        except fvm.FvmError:
            continue   # a tile whose kernels do not fit this closure and precision
        # every tile is timed on the same steps from the initial state (a case
        # is not advanced through all tiles' steps, which may outlast its
        # physical time span)
        _restart(handle)
        handle.n_steps(warm)
        t0 = time.perf_counter()
        handle.n_steps(steps)
        times[t] = (time.perf_counter() - t0) / (4 * steps) * 1e3   # ms per stage
        if verbose:
            tx, ty, nt = C.c_int(), C.c_int(), C.c_int()
            L.fvm_tile_shape(dim, t, C.byref(tx), C.byref(ty), C.byref(nt))
            print(f"# tile {t} ({tx.value}x{ty.value}, {nt.value} threads): {times[t] * 1e3:.2f} us/stage", flush=True)
    best = min(times, key=times.get)
    handle.set_tile(best)
    _cache[k] = (best, times)
    if save:
        data = _load_file()
        data[repr(k)] = {"tile": best, "ms_per_stage": {str(t): v for t, v in times.items()}}
        with open(CACHE_FILE, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    return best, times
