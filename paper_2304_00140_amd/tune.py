"""Launch-shape autotuner for the fused stage kernels.

Times every tile shape of the context's dimension with HIP events around the
stage launches (fvm_time_stages, which advances the state) and keeps the
fastest.  Results are cached per (dimension, precision, switching, CSF on,
closure kind, cell count) for the process.
"""
import ctypes as C

import numpy as np

_cache = {}


def key_of(handle, precision):
    case = handle.case if hasattr(handle, "case") else handle.cases[0]
    ncell = handle.ncell if hasattr(handle, "ncell") else handle.cells()
    s = case["scheme"]
    return (case["grid"]["dim"], precision, int(s["switching"]), s["sigma"] > 0, tuple(case["eos"]["kind"]),
            int(ncell))


def autotune(handle, precision, steps=6, warm=2, verbose=False):
    """handle: fvm.Context or fvm.Batch with a state set; returns (best tile, {tile: ms per stage})"""
    from . import fvm
    k = key_of(handle, precision)
    if k in _cache:
        handle.set_tile(_cache[k][0])
        return _cache[k]
    L = fvm.lib()
    dim = k[0]
    times = {}
    for t in range(L.fvm_tile_count(dim)):
        handle.set_tile(t)
        handle.time_stages(warm)
        times[t] = float(np.mean(handle.time_stages(steps)))
        if verbose:
            tx, ty, nt = C.c_int(), C.c_int(), C.c_int()
            L.fvm_tile_shape(dim, t, C.byref(tx), C.byref(ty), C.byref(nt))
            print(f"# tile {t} ({tx.value}x{ty.value}, {nt.value} threads): {times[t] * 1e3:.2f} us/stage", flush=True)
    best = min(times, key=times.get)
    handle.set_tile(best)
    _cache[k] = (best, times)
    return best, times
