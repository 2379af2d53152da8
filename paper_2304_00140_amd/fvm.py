"""Python binding of the gfx950 solver library (include/fvm.h).

Argument marshalling only: every step of the right-hand side and of the time
integration runs in the HIP kernels of libfvm.so.  The C functions are
exposed under their own names (fvm_create, fvm_rhs, ...); `Context` and
`Batch` wrap a context with numpy / torch arrays and the case dicts of
`workloads`.  There is no fallback: if libfvm.so is missing or cannot be
loaded, importing the library raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfvm.so")
MAXSPEC = 4

FVM_OK, FVM_EINVAL, FVM_EHIP, FVM_ENOMEM, FVM_ENONPHYS, FVM_ENAN, FVM_ESTATE = 0, -1, -2, -3, -4, -5, -6
FVM_FP64, FVM_MIXED = 0, 1
FVM_TK_STAGE, FVM_TK_PAIR, FVM_TK_MARCH, FVM_TK_PRIM_MARCH = 0, 1, 2, 3
ERRNAMES = {-1: "EINVAL", -2: "EHIP", -3: "ENOMEM", -4: "ENONPHYS", -5: "ENAN", -6: "ESTATE"}


class fvm_grid_desc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("dx", C.c_double * 3), ("bc", (C.c_int * 2) * 3),
                ("in_p", C.c_double), ("in_T", C.c_double), ("in_alpha", C.c_double), ("in_u", C.c_double),
                ("in_radius", C.c_double), ("in_center", C.c_double * 2), ("in_noise", C.c_double),
                ("in_seed", C.c_uint64), ("ff_p", C.c_double), ("ff_T", C.c_double), ("ff_alpha", C.c_double)]


class fvm_eos_desc(C.Structure):
    _fields_ = [("kind", C.c_int * 3), ("gamma", C.c_double * 3), ("pinf", C.c_double * 3),
                ("cv", C.c_double * 3), ("q", C.c_double * 3), ("pr_ns", C.c_int * 2),
                ("pr_X", (C.c_double * MAXSPEC) * 2), ("pr_Tc", (C.c_double * MAXSPEC) * 2),
                ("pr_pc", (C.c_double * MAXSPEC) * 2), ("pr_omega", (C.c_double * MAXSPEC) * 2),
                ("pr_M", (C.c_double * MAXSPEC) * 2), ("pr_Zc", (C.c_double * MAXSPEC) * 2),
                ("pr_vc", (C.c_double * MAXSPEC) * 2), ("pr_kij", ((C.c_double * MAXSPEC) * MAXSPEC) * 2),
                ("p_ref", C.c_double), ("T_ref", C.c_double), ("mu", C.c_double * 3), ("kc", C.c_double * 3),
                ("ncomp", C.c_int), ("model", C.c_int), ("bt_rho_sat", C.c_double), ("bt_p_sat", C.c_double),
                ("bt_c_liq", C.c_double), ("bt_rho_vap", C.c_double), ("bt_RT", C.c_double),
                ("bt_mu_vap", C.c_double), ("bt_RT2", C.c_double)]


class fvm_scheme_desc(C.Structure):
    _fields_ = [("switching", C.c_int), ("lim_u", C.c_int), ("lim_s", C.c_int), ("thinc", C.c_int),
                ("beta", C.c_double), ("thinc_gamma", C.c_double), ("eps_interface", C.c_double),
                ("theta_ducros", C.c_double), ("theta_gas", C.c_double), ("eps_ducros", C.c_double),
                ("kappa3", C.c_double), ("rk", C.c_double * 4), ("cfl", C.c_double), ("sigma", C.c_double),
                ("eps_normal", C.c_double), ("gravity", C.c_double * 3), ("thermal", C.c_int)]


_P = C.c_void_p
_DP = C.POINTER(C.c_double)
_I64P = C.POINTER(C.c_int64)
_IP = C.POINTER(C.c_int)
_GP, _EP, _SP = C.POINTER(fvm_grid_desc), C.POINTER(fvm_eos_desc), C.POINTER(fvm_scheme_desc)

# name -> (restype, argtypes); the same set as include/fvm.h
SIGNATURES = {
    "fvm_version": (C.c_int, []),
    "fvm_create": (C.c_int, [C.POINTER(_P), _GP, _EP, _SP, C.c_int, _P]),
    "fvm_destroy": (None, [_P]),
    "fvm_init_primitive": (C.c_int, [_P, _DP]),
    "fvm_set_state": (C.c_int, [_P, _DP]),
    "fvm_set_state_device": (C.c_int, [_P, _P]),
    "fvm_get_state": (C.c_int, [_P, _DP]),
    "fvm_get_state_device": (C.c_int, [_P, _P]),
    "fvm_get_primitive": (C.c_int, [_P, _DP]),
    "fvm_rhs": (C.c_int, [_P, _P, _P, C.c_int64]),
    "fvm_rhs_noalloc": (C.c_int, [_GP, _EP, _SP, _P, _P, C.c_int64, _P]),
    "fvm_step": (C.c_int, [_P, _DP, _DP]),
    "fvm_n_steps": (C.c_int, [_P, C.c_int, C.c_double, _DP]),
    "fvm_clock": (C.c_int, [_P, _DP, _DP, _I64P]),
    "fvm_totals": (C.c_int, [_P, _DP]),
    "fvm_error_info": (C.c_int, [_P, _IP, _I64P, _I64P]),
    "fvm_tile_count": (C.c_int, [C.c_int]),
    "fvm_tile_shape": (C.c_int, [C.c_int, C.c_int, _IP, _IP, _IP]),
    "fvm_tile_kernels": (C.c_int, [C.c_int, C.c_int]),
    "fvm_set_tile": (C.c_int, [_P, C.c_int]),
    "fvm_time_stages": (C.c_int, [_P, C.c_int, _DP]),
    "fvm_batch_create": (C.c_int, [C.POINTER(_P), C.c_int, _GP, _EP, _SP, C.c_int, _P]),
    "fvm_batch_destroy": (None, [_P]),
    "fvm_batch_init_primitive": (C.c_int, [_P, C.c_int, _DP]),
    "fvm_batch_set_state": (C.c_int, [_P, C.c_int, _DP]),
    "fvm_batch_get_state": (C.c_int, [_P, C.c_int, _DP]),
    "fvm_batch_n_steps": (C.c_int, [_P, C.c_int, _DP]),
    "fvm_batch_totals": (C.c_int, [_P, C.c_int, _DP]),
    "fvm_batch_error_info": (C.c_int, [_P, _IP, _IP, _I64P, _I64P]),
    "fvm_batch_time_stages": (C.c_int, [_P, C.c_int, _DP]),
    "fvm_batch_cells": (C.c_int64, [_P]),
    "fvm_batch_set_tile": (C.c_int, [_P, C.c_int]),
    "fvm_last_error": (C.c_char_p, [_P]),
    "fvm_batch_last_error": (C.c_char_p, [_P]),
}

_lib = None


def lib():
    """load libfvm.so (raises if it is not built)"""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run paper_2304_00140_amd/build.py "
                               "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def __getattr__(name):
    if name in SIGNATURES:
        return getattr(lib(), name)
    raise AttributeError(name)


class FvmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRNAMES.get(code, code)}: {msg}")
        self.code = code


# ---------------------------------------------------------------- descriptors
def grid_desc(gd):
    g = fvm_grid_desc()
    g.dim = gd["dim"]
    for d in range(3):
        g.n[d] = int(gd["n"][d])
        g.dx[d] = float(gd["dx"][d])
        for s in range(2):
            g.bc[d][s] = int(gd["bc"][d][s])
    inf = gd.get("inflow", {})
    g.in_p, g.in_T, g.in_alpha = inf.get("p", 0.0), inf.get("T", 0.0), inf.get("alpha", 0.0)
    g.in_u, g.in_radius, g.in_noise = inf.get("u", 0.0), inf.get("radius", 0.0), inf.get("noise", 0.0)
    c = inf.get("center", [0.0, 0.0])
    g.in_center[0], g.in_center[1] = c[0], c[1]
    g.in_seed = int(inf.get("seed", 0))
    ff = gd.get("farfield", {})
    g.ff_p, g.ff_T, g.ff_alpha = ff.get("p", 0.0), ff.get("T", 0.0), ff.get("alpha", 0.0)
    return g


def eos_desc(ed, storage=None):
    e = fvm_eos_desc()
    nc = len(ed["kind"])
    e.ncomp = nc
    e.model = int(ed.get("model", 0))
    if e.model == 1:
        b = ed["baro"]
        e.bt_rho_sat, e.bt_p_sat, e.bt_c_liq = b["rho_sat"], b["p_sat"], b["c_liq"]
        e.bt_rho_vap, e.bt_RT = b["rho_vap"], b["RT"]
        e.bt_mu_vap = b.get("mu_vap", 0.0)
        e.bt_RT2 = b.get("RT2", 0.0)
    for k in range(nc):
        e.kind[k] = int(ed["kind"][k])
        e.gamma[k], e.pinf[k], e.cv[k], e.q[k] = ed["gamma"][k], ed["pinf"][k], ed["cv"][k], ed["q"][k]
        e.mu[k], e.kc[k] = (ed.get("mu") or [0.0] * nc)[k], (ed.get("kc") or [0.0] * nc)[k]
        pr = ed["pr"][k]
        if pr is not None:
            if k > 1:
                raise ValueError("a Peng-Robinson fluid is supported as component 0 or 1 of two")
            e.pr_ns[k] = len(pr["species"])
            for a, s in enumerate(pr["species"]):
                e.pr_X[k][a] = pr["X"][a]
                e.pr_Tc[k][a], e.pr_pc[k][a], e.pr_omega[k][a] = s["Tc"], s["pc"], s["omega"]
                e.pr_M[k][a], e.pr_Zc[k][a], e.pr_vc[k][a] = s["M"], s["Zc"], s["vc"]
                for b in range(len(pr["species"])):
                    e.pr_kij[k][a][b] = pr["kij"][a][b]
    if storage:
        e.p_ref, e.T_ref = storage.get("p_ref", 0.0), storage.get("T_ref", 0.0)
    return e


def scheme_desc(sd):
    s = fvm_scheme_desc()
    for name in ("switching", "lim_u", "lim_s", "thinc"):
        setattr(s, name, int(sd[name]))
    for name in ("beta", "thinc_gamma", "eps_interface", "theta_ducros", "theta_gas", "eps_ducros",
                 "kappa3", "cfl", "sigma", "eps_normal"):
        setattr(s, name, float(sd[name]))
    for i in range(4):
        s.rk[i] = sd["rk"][i]
    for i, gi in enumerate(sd.get("gravity", [0.0, 0.0, 0.0])):
        s.gravity[i] = gi
    s.thermal = int(sd.get("thermal", 0))
    return s


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def _stream_ptr(stream):
    if stream is None:
        return None
    return C.c_void_p(int(stream))


def rhs_noalloc(case, q_in_ptr, r_out_ptr, step=0, stream=None):
    """fvm_rhs_noalloc: one FP64 right-hand side of `case` from device array
    q_in_ptr into r_out_ptr ([N_q, ncell] FP64 device pointers), no context and
    no device allocation; launched on `stream` without waiting"""
    L = lib()
    g, e, s = grid_desc(case["grid"]), eos_desc(case["eos"], None), scheme_desc(case["scheme"])
    rc = L.fvm_rhs_noalloc(C.byref(g), C.byref(e), C.byref(s), C.c_void_p(q_in_ptr), C.c_void_p(r_out_ptr),
                           step, _stream_ptr(stream))
    if rc:
        raise FvmError(rc, L.fvm_last_error(None).decode())


# ---------------------------------------------------------------- wrappers
class Context:
    """one case on the GPU; `stream` is a hipStream_t handle (e.g.
    torch.cuda.Stream().cuda_stream) or None for the default stream"""

    def __init__(self, case, precision=FVM_FP64, stream=None, shifts=True):
        self.L = lib()
        self.case = case
        self.dim = case["grid"]["dim"]
        self.ncomp = len(case["eos"]["kind"])
        self.barotropic = int(case["eos"].get("model", 0)) == 1
        self.nq = self.dim + self.ncomp if self.barotropic else self.dim + self.ncomp + 1
        self.ncell = int(np.prod(case["grid"]["n"]))
        self._g = grid_desc(case["grid"])
        self._e = eos_desc(case["eos"], case.get("storage") if shifts else None)
        self._s = scheme_desc(case["scheme"])
        self._h = C.c_void_p()
        self.stream = stream
        rc = self.L.fvm_create(C.byref(self._h), C.byref(self._g), C.byref(self._e), C.byref(self._s),
                               precision, _stream_ptr(stream))
        if rc:
            raise FvmError(rc, self.L.fvm_last_error(None).decode())

    def _chk(self, rc):
        if rc:
            raise FvmError(rc, self.L.fvm_last_error(self._h).decode())

    def close(self):
        if self._h:
            self.L.fvm_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_primitive(self, prim=None):
        prim = np.ascontiguousarray(self.case["prim"] if prim is None else prim, dtype=np.float64)
        self._chk(self.L.fvm_init_primitive(self._h, _dp(prim)))

    def set_state(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        self._chk(self.L.fvm_set_state(self._h, _dp(q)))

    def set_state_device(self, q_ptr):
        self._chk(self.L.fvm_set_state_device(self._h, C.c_void_p(q_ptr)))

    def get_state(self):
        q = np.empty((self.nq, self.ncell))
        self._chk(self.L.fvm_get_state(self._h, _dp(q)))
        return q

    def get_state_device(self, q_ptr):
        self._chk(self.L.fvm_get_state_device(self._h, C.c_void_p(q_ptr)))

    def get_primitive(self):
        w = np.empty((12 if self.barotropic else (11 if self.ncomp == 3 else 9), self.ncell))
        self._chk(self.L.fvm_get_primitive(self._h, _dp(w)))
        return w

    def rhs(self, q_in_ptr, r_out_ptr, step=0):
        """device pointers (e.g. tensor.data_ptr()) of [N_q, ncell] FP64 arrays"""
        self._chk(self.L.fvm_rhs(self._h, C.c_void_p(q_in_ptr), C.c_void_p(r_out_ptr), step))

    def step(self):
        dt, t = C.c_double(), C.c_double()
        self._chk(self.L.fvm_step(self._h, C.byref(dt), C.byref(t)))
        return t.value, dt.value

    def n_steps(self, n, t_end=0.0):
        t = C.c_double()
        self._chk(self.L.fvm_n_steps(self._h, n, t_end, C.byref(t)))
        return t.value

    def clock(self):
        t, dt, n = C.c_double(), C.c_double(), C.c_int64()
        self._chk(self.L.fvm_clock(self._h, C.byref(t), C.byref(dt), C.byref(n)))
        return t.value, dt.value, n.value

    def totals(self):
        out = np.empty(self.nq)
        self._chk(self.L.fvm_totals(self._h, _dp(out)))
        return out

    def error_info(self):
        code, cell, step = C.c_int(), C.c_int64(), C.c_int64()
        self._chk(self.L.fvm_error_info(self._h, C.byref(code), C.byref(cell), C.byref(step)))
        return code.value, cell.value, step.value

    def set_tile(self, tile):
        self._chk(self.L.fvm_set_tile(self._h, tile))

    def time_stages(self, steps):
        ms = (C.c_double * 4)()
        self._chk(self.L.fvm_time_stages(self._h, steps, ms))
        return list(ms)


class Batch:
    """many independent cases (same dimension, scheme and precision)"""

    def __init__(self, cases, precision=FVM_MIXED, stream=None, shifts=True):
        self.L = lib()
        self.cases = cases
        n = len(cases)
        self.dim = cases[0]["grid"]["dim"]
        if int(cases[0]["eos"].get("model", 0)) == 1:
            self.nq = self.dim + len(cases[0]["eos"]["kind"])
        else:
            self.nq = self.dim + len(cases[0]["eos"]["kind"]) + 1
        self._g = (fvm_grid_desc * n)(*[grid_desc(c["grid"]) for c in cases])
        self._e = (fvm_eos_desc * n)(*[eos_desc(c["eos"], c.get("storage") if shifts else None) for c in cases])
        self._s = scheme_desc(cases[0]["scheme"])
        self._h = C.c_void_p()
        rc = self.L.fvm_batch_create(C.byref(self._h), n, self._g, self._e, C.byref(self._s), precision,
                                     _stream_ptr(stream))
        if rc:
            raise FvmError(rc, self.L.fvm_batch_last_error(None).decode())

    def _chk(self, rc):
        if rc:
            raise FvmError(rc, self.L.fvm_batch_last_error(self._h).decode())

    def close(self):
        if self._h:
            self.L.fvm_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_primitive(self, i, prim=None):
        prim = np.ascontiguousarray(self.cases[i]["prim"] if prim is None else prim, dtype=np.float64)
        self._chk(self.L.fvm_batch_init_primitive(self._h, i, _dp(prim)))

    def set_state(self, i, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        self._chk(self.L.fvm_batch_set_state(self._h, i, _dp(q)))

    def get_state(self, i):
        n = int(np.prod(self.cases[i]["grid"]["n"]))
        q = np.empty((self.nq, n))
        self._chk(self.L.fvm_batch_get_state(self._h, i, _dp(q)))
        return q

    def n_steps(self, n):
        t = np.empty(len(self.cases))
        self._chk(self.L.fvm_batch_n_steps(self._h, n, _dp(t)))
        return t

    def totals(self, i):
        out = np.empty(self.nq)
        self._chk(self.L.fvm_batch_totals(self._h, i, _dp(out)))
        return out

    def cells(self):
        return int(self.L.fvm_batch_cells(self._h))

    def set_tile(self, tile):
        self._chk(self.L.fvm_batch_set_tile(self._h, tile))

    def time_stages(self, steps):
        ms = (C.c_double * 4)()
        self._chk(self.L.fvm_batch_time_stages(self._h, steps, ms))
        return list(ms)
