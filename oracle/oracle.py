"""ctypes view of the CPU FP64 oracle (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this module.  It mirrors oracle.h and takes the case dicts produced by the
seeded workload generators.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
MAXSPEC = 4
# rows of a cell's primitive vector in oracle.h (the last, OW_E, is the
# specific internal energy)
OW_N = 13


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("dx", C.c_double * 3),
                ("bc", (C.c_int * 2) * 3),
                ("in_p", C.c_double), ("in_T", C.c_double), ("in_alpha", C.c_double),
                ("in_u", C.c_double), ("in_radius", C.c_double), ("in_center", C.c_double * 2),
                ("in_noise", C.c_double), ("in_seed", C.c_uint64),
                ("ff_p", C.c_double), ("ff_T", C.c_double), ("ff_alpha", C.c_double)]


MAXCOMP = 3


class Eos(C.Structure):
    _fields_ = [("kind", C.c_int * MAXCOMP), ("gamma", C.c_double * MAXCOMP), ("pinf", C.c_double * MAXCOMP),
                ("cv", C.c_double * MAXCOMP), ("q", C.c_double * MAXCOMP),
                ("pr_ns", C.c_int * 2),
                ("pr_X", (C.c_double * MAXSPEC) * 2), ("pr_Tc", (C.c_double * MAXSPEC) * 2),
                ("pr_pc", (C.c_double * MAXSPEC) * 2), ("pr_omega", (C.c_double * MAXSPEC) * 2),
                ("pr_M", (C.c_double * MAXSPEC) * 2), ("pr_Zc", (C.c_double * MAXSPEC) * 2),
                ("pr_vc", (C.c_double * MAXSPEC) * 2),
                ("pr_kij", ((C.c_double * MAXSPEC) * MAXSPEC) * 2),
                ("mu", C.c_double * MAXCOMP), ("kc", C.c_double * MAXCOMP), ("ncomp", C.c_int),
                ("model", C.c_int), ("bt_rho_sat", C.c_double), ("bt_p_sat", C.c_double),
                ("bt_c_liq", C.c_double), ("bt_rho_vap", C.c_double), ("bt_RT", C.c_double),
                ("bt_mu_vap", C.c_double), ("bt_RT2", C.c_double)]


class Scheme(C.Structure):
    _fields_ = [("switching", C.c_int), ("lim_u", C.c_int), ("lim_s", C.c_int), ("thinc", C.c_int),
                ("beta", C.c_double), ("thinc_gamma", C.c_double), ("eps_interface", C.c_double),
                ("theta_ducros", C.c_double), ("theta_gas", C.c_double), ("eps_ducros", C.c_double),
                ("kappa3", C.c_double), ("rk", C.c_double * 4), ("cfl", C.c_double),
                ("sigma", C.c_double), ("eps_normal", C.c_double), ("gravity", C.c_double * 3),
                ("thermal", C.c_int)]


RHS_FN = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int, C.c_void_p)

_lib = None


def lib():
    global _lib
    if _lib is None:
        from . import build as _b   # noqa: F401  (package-relative when imported as oracle.oracle)
        if _b.needs_build():
            _b.build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        pg, pe, ps = C.POINTER(Grid), C.POINTER(Eos), C.POINTER(Scheme)
        sig = {
            "og_eos_forward": (C.c_int, [pe, C.c_double, C.c_double, C.c_double, dp, dp]),
            "og_eos_forward_e": (C.c_int, [pe, C.c_double, C.c_double, C.c_double, dp, dp]),
            "og_eos_inverse": (C.c_int, [pe, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]),
            "og_eos_forward2": (C.c_int, [pe, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]),
            "og_eos_inverse2": (C.c_int, [pe, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                          dp, dp]),
            "og_mix_sound2": (C.c_double, [pe, C.c_double, C.c_double, C.c_double, C.c_double]),
            "og_ncomp": (C.c_int, [pe]),
            "og_is_barotropic": (C.c_int, [pe]),
            "og_baro_liquid_density": (C.c_double, [pe, C.c_double]),
            "og_baro_density": (C.c_double, [pe, C.c_double, C.c_double]),
            "og_baro_pressure": (C.c_int, [pe, C.c_double, C.c_double, dp]),
            "og_baro_sound": (C.c_double, [pe, C.c_double]),
            "og_baro_fractions": (None, [pe, C.c_double, C.c_double, C.c_double, dp, dp]),
            "og_baro_viscosity": (C.c_double, [pe, C.c_double, C.c_double]),
            "og_baro_density2": (C.c_double, [pe, C.c_double, C.c_double, C.c_double]),
            "og_baro_pressure2": (C.c_int, [pe, C.c_double, C.c_double, C.c_double, dp]),
            "og_baro_fractions2": (None, [pe, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp, dp]),
            "og_face_flux_baro": (C.c_int, [pe, ps, C.c_int, C.c_int, dp, C.c_int, C.c_int, C.c_int,
                                            dp, dp, dp]),
            "og_sound": (C.c_double, [pe, C.c_int, C.c_double, C.c_double]),
            "og_mix_sound": (C.c_double, [pe, C.c_double, C.c_double, C.c_double]),
            "og_clip_fraction": (C.c_double, [C.c_double]),
            "og_spec_volume": (C.c_double, [pe, C.c_int, C.c_double, C.c_double]),
            "og_spec_energy": (C.c_double, [pe, C.c_int, C.c_double, C.c_double]),
            "og_pr_coeffs": (C.c_int, [pe, C.c_int, C.c_double, dp, dp, dp, dp, dp]),
            "og_pr_pressure": (C.c_double, [pe, C.c_int, C.c_double, C.c_double]),
            "og_pr_energy_tv": (C.c_double, [pe, C.c_int, C.c_double, C.c_double]),
            "og_limiter_table": (C.c_double, [C.c_int, C.c_double]),
            "og_slope": (C.c_double, [C.c_int, C.c_double, C.c_double]),
            "og_thinc_left": (C.c_double, [C.c_double] * 5),
            "og_thinc_right": (C.c_double, [C.c_double] * 5),
            "og_central4": (C.c_double, [C.c_double] * 4),
            "og_face_flux": (C.c_int, [pe, ps, C.c_int, C.c_int, dp, C.c_int, C.c_int, C.c_int,
                                       dp, dp, dp]),
            "og_cons_from_prim": (C.c_int, [pg, pe, dp, dp]),
            "og_prim_from_cons": (C.c_int, [pg, pe, dp, dp]),
            "og_rhs": (C.c_int, [pg, pe, ps, dp, C.c_int64, dp]),
            "og_curvature": (C.c_int, [pg, pe, ps, dp, dp]),
            "og_dt": (C.c_double, [pg, pe, ps, dp]),
            "og_sensor_flags": (C.c_int, [pg, pe, ps, dp, C.POINTER(C.c_ubyte)]),
            "og_step": (C.c_int, [pg, pe, ps, dp, C.c_int64, dp, C.c_double, dp]),
            "og_run": (C.c_int, [pg, pe, ps, dp, C.c_int64, C.c_int, dp, C.c_double]),
            "og_totals": (None, [pg, pe, dp, dp]),
            "og_lsrk": (None, [ps, dp, C.c_int, C.c_double, RHS_FN, C.c_void_p]),
            "og_splitmix64": (C.c_uint64, [C.c_uint64]),
            "og_noise01": (C.c_double, [C.c_uint64] * 5),
            "og_nthreads": (C.c_int, []),
            "og_set_nthreads": (None, [C.c_int]),
            "og_last_error": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_grid(gd):
    g = Grid()
    g.dim = gd["dim"]
    for d in range(3):
        g.n[d] = int(gd["n"][d])
        g.dx[d] = float(gd["dx"][d])
        for s in range(2):
            g.bc[d][s] = int(gd["bc"][d][s])
    inf = gd.get("inflow", {})
    g.in_p, g.in_T, g.in_alpha = inf.get("p", 0.0), inf.get("T", 0.0), inf.get("alpha", 0.0)
    g.in_u, g.in_radius = inf.get("u", 0.0), inf.get("radius", 0.0)
    c = inf.get("center", [0.0, 0.0])
    g.in_center[0], g.in_center[1] = c[0], c[1]
    g.in_noise, g.in_seed = inf.get("noise", 0.0), int(inf.get("seed", 0))
    ff = gd.get("farfield", {})
    g.ff_p, g.ff_T, g.ff_alpha = ff.get("p", 0.0), ff.get("T", 0.0), ff.get("alpha", 0.0)
    return g


def make_eos(ed):
    e = Eos()
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
            sp = pr["species"]
            e.pr_ns[k] = len(sp)
            for a, s in enumerate(sp):
                e.pr_X[k][a] = pr["X"][a]
                e.pr_Tc[k][a], e.pr_pc[k][a], e.pr_omega[k][a] = s["Tc"], s["pc"], s["omega"]
                e.pr_M[k][a], e.pr_Zc[k][a], e.pr_vc[k][a] = s["M"], s["Zc"], s["vc"]
                for b in range(len(sp)):
                    e.pr_kij[k][a][b] = pr["kij"][a][b]
    return e


def make_scheme(sd):
    s = Scheme()
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


class Oracle:
    """Oracle bound to one case dict."""

    def __init__(self, case):
        self.case = case
        self.L = lib()
        self.g = make_grid(case["grid"])
        self.e = make_eos(case["eos"])
        self.s = make_scheme(case["scheme"])
        self.dim = case["grid"]["dim"]
        self.ncomp = len(case["eos"]["kind"])
        self.barotropic = int(case["eos"].get("model", 0)) == 1
        self.nq = self.dim + self.ncomp if self.barotropic else self.dim + self.ncomp + 1
        self.ncell = int(np.prod(case["grid"]["n"]))

    def _err(self, rc, what):
        if rc:
            raise RuntimeError(f"oracle {what} failed ({rc}): {self.L.og_last_error().decode()}")

    def cons_from_prim(self, prim=None):
        prim = np.ascontiguousarray(self.case["prim"] if prim is None else prim, dtype=np.float64)
        q = np.empty((self.nq, self.ncell))
        self._err(self.L.og_cons_from_prim(C.byref(self.g), C.byref(self.e), _dp(prim), _dp(q)), "cons_from_prim")
        return q

    def prim_from_cons(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        W = np.empty((OW_N, self.ncell))
        self._err(self.L.og_prim_from_cons(C.byref(self.g), C.byref(self.e), _dp(q), _dp(W)), "prim_from_cons")
        # rows: rho, u, v, w, p, T, xi_1, c, alpha_1 (+ xi_2, alpha_2 with three components;
        # + xi_2 = 0, alpha_2 = 0, alpha_V in the barotropic model)
        if self.barotropic:
            return W[:12]
        return W[:11] if self.ncomp == 3 else W[:9]

    def rhs(self, q, step=0):
        q = np.ascontiguousarray(q, dtype=np.float64)
        r = np.empty_like(q)
        self._err(self.L.og_rhs(C.byref(self.g), C.byref(self.e), C.byref(self.s), _dp(q), step, _dp(r)), "rhs")
        return r

    def curvature(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        k = np.empty(self.ncell)
        self._err(self.L.og_curvature(C.byref(self.g), C.byref(self.e), C.byref(self.s), _dp(q), _dp(k)), "curvature")
        return k

    def sensor_flags(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        fl = np.zeros(self.ncell, dtype=np.uint8)
        self._err(self.L.og_sensor_flags(C.byref(self.g), C.byref(self.e), C.byref(self.s), _dp(q),
                                         fl.ctypes.data_as(C.POINTER(C.c_ubyte))), "sensor_flags")
        return fl

    def dt(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        return self.L.og_dt(C.byref(self.g), C.byref(self.e), C.byref(self.s), _dp(q))

    def step(self, q, step=0, t=0.0, t_end=0.0):
        """advance q in place by one step; returns (t, dt)"""
        assert q.flags.c_contiguous and q.dtype == np.float64
        tt = C.c_double(t)
        dt = C.c_double(0.0)
        self._err(self.L.og_step(C.byref(self.g), C.byref(self.e), C.byref(self.s), _dp(q), step,
                                 C.byref(tt), t_end, C.byref(dt)), "step")
        return tt.value, dt.value

    def run(self, q, nsteps, step0=0, t=0.0, t_end=0.0):
        assert q.flags.c_contiguous and q.dtype == np.float64
        tt = C.c_double(t)
        self._err(self.L.og_run(C.byref(self.g), C.byref(self.e), C.byref(self.s), _dp(q), step0,
                                nsteps, C.byref(tt), t_end), "run")
        return tt.value

    def totals(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        out = np.empty(self.nq)
        self.L.og_totals(C.byref(self.g), C.byref(self.e), _dp(q), _dp(out))
        return out
