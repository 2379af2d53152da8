"""Pins of the oracle's reconstruction, Riemann solver, TDU and face flux
(Section 3.2, 3.3, Table 4.2, Appendix D) against closed forms."""
import ctypes as C
import math

import numpy as np
import pytest

from oracle.oracle import lib, make_eos, make_scheme
from paper_2304_00140_amd import workloads as W

L = lambda: lib()  # noqa: E731
LIMS = ["minmod", "koren", "vanalbada", "vanleer", "chakravarthy", "mc", "superbee"]


def test_limiters_consistent_at_r1_and_zero_at_extrema():
    """f(1) = 1 for every entry of Table 4.2 (second order on linear data) and no
    slope at a local extremum (TVD)."""
    for name in LIMS:
        k = W.LIM[name]
        assert abs(L().og_limiter_table(k, 1.0) - 1.0) < 1e-15, name
        assert L().og_slope(k, 1.0, -2.0) == 0.0
        assert L().og_slope(k, -0.5, 0.3) == 0.0


def test_limiter_symmetry():
    """f(r)/r = f(1/r) for the symmetric limiters of Table 4.2; Koren is not symmetric"""
    for name in ["minmod", "vanalbada", "vanleer", "mc", "superbee"]:
        k = W.LIM[name]
        for r in [0.1, 0.37, 0.8, 1.7, 4.2]:
            a = L().og_limiter_table(k, r) / r
            b = L().og_limiter_table(k, 1.0 / r)
            assert abs(a - b) < 1e-14, name
    k = W.LIM["koren"]
    assert abs(L().og_limiter_table(k, 0.5) / 0.5 - L().og_limiter_table(k, 2.0)) > 0.1


def cell_avgs(poly, x0, h, n):
    """exact cell averages of a polynomial (coefficients low->high) on cells [x0+i h, x0+(i+1) h]"""
    P = np.polynomial.polynomial.Polynomial(poly).integ()
    edges = x0 + h * np.arange(n + 1)
    return np.diff(P(edges)) / h


def test_koren_third_order_on_quadratics():
    """'Koren ... 3rd-order accurate for smooth data' (Section 3.3): on cell
    averages of a monotone quadratic the left and right face values are exact."""
    k = W.LIM["koren"]
    rng = np.random.default_rng(5)
    for _ in range(50):
        c = rng.uniform(-1, 1, 3)
        c[1] = 3.0 * abs(c[1]) + 1.0          # monotone on [0, 4]
        c[2] = 0.2 * c[2]
        a = cell_avgs(c, 0.0, 1.0, 4)
        exact = np.polynomial.polynomial.polyval(2.0, c)
        fl = a[1] + 0.5 * L().og_slope(k, a[1] - a[0], a[2] - a[1])
        fr = a[2] - 0.5 * L().og_slope(k, a[3] - a[2], a[2] - a[1])
        # the limiter is inactive when the ratio of differences stays in its linear range
        r_l = (a[2] - a[1]) / (a[1] - a[0])
        r_r = (a[2] - a[1]) / (a[3] - a[2])
        if 0.25 < r_l < 2.5:
            assert abs(fl - exact) < 1e-13
        if 0.25 < r_r < 2.5:
            assert abs(fr - exact) < 1e-13


def test_minmod_tvd_bounds():
    rng = np.random.default_rng(6)
    k = W.LIM["minmod"]
    for _ in range(200):
        a = rng.normal(size=4)
        fl = a[1] + 0.5 * L().og_slope(k, a[1] - a[0], a[2] - a[1])
        assert min(a[1], a[2]) - 1e-15 <= fl <= max(a[1], a[2]) + 1e-15


def tanh_profile_avgs(xc, theta, beta, lo, hi):
    """exact cell averages of m + (M-m)/2 (1 + theta tanh(beta (x - xc))) on the
    unit cells [-1,0], [0,1], [1,2] and the profile's face values"""
    def prim(x):   # antiderivative of tanh(beta (x - xc))
        return math.log(math.cosh(beta * (x - xc))) / beta
    avgs = []
    for a in (-1.0, 0.0, 1.0):
        avg_tanh = prim(a + 1) - prim(a)
        avgs.append(lo + 0.5 * (hi - lo) * (1 + theta * avg_tanh))
    f0 = lo + 0.5 * (hi - lo) * (1 + theta * math.tanh(beta * (0.0 - xc)))
    f1 = lo + 0.5 * (hi - lo) * (1 + theta * math.tanh(beta * (1.0 - xc)))
    return avgs, f0, f1


@pytest.mark.parametrize("xc", [0.2, 0.5, 0.77])
@pytest.mark.parametrize("theta", [1.0, -1.0])
def test_thinc_reproduces_its_tanh_profile(xc, theta):
    """eq. (3-3)/(3-4): when the middle cell's average comes from a tanh profile
    spanning the neighbours' range, the face values are that profile's values
    at the cell's faces (closed form of THINC).  A non-zero minimum checks the
    range reading of the F denominator."""
    beta = 1.6
    lo, hi = 0.1, 0.85
    # the middle cell holds the jump; the neighbours hold the profile's limits
    avgs, f0, f1 = tanh_profile_avgs(xc, theta, beta, lo, hi)
    a = lo if theta > 0 else hi
    c = hi if theta > 0 else lo
    left = L().og_thinc_left(a, avgs[1], c, beta, 1e-20)    # value at x = 1 (right face of the cell)
    right = L().og_thinc_right(a, avgs[1], c, beta, 1e-20)  # value at x = 0 (left face of the cell)
    assert abs(left - f1) < 1e-12
    assert abs(right - f0) < 1e-12


def test_thinc_symmetric_at_half():
    """F = 1/2: face values symmetric about the mid value"""
    l = L().og_thinc_left(0.0, 0.5, 1.0, 1.6, 0.0)
    r = L().og_thinc_right(0.0, 0.5, 1.0, 1.6, 0.0)
    assert abs((l + r) - 1.0) < 1e-14


def test_central4_exact_on_cubics():
    """eq. (D.1): the fourth-order central face value is exact for cell averages of cubics"""
    rng = np.random.default_rng(7)
    for _ in range(20):
        c = rng.normal(size=4)
        a = cell_avgs(c, -2.0, 1.0, 4)   # cells i-1 .. i+2 around the face x = 0
        assert abs(L().og_central4(*a) - np.polynomial.polynomial.polyval(0.0, c)) < 1e-13


# ------------------------------------------------------------- face flux

EOSD = W.make_eos(W.sg(4.4, 6e8, 607.866), W.sg(1.4, 0.0, 717.5))


def face(W4, f=1, sl=0, sr=0, dim=2, d=0, scheme=None):
    e = make_eos(EOSD)
    s = make_scheme(scheme or W.default_scheme())
    arr = np.ascontiguousarray(W4, dtype=np.float64)
    F = np.zeros(7)
    us, ps = C.c_double(), C.c_double()
    rc = L().og_face_flux(C.byref(e), C.byref(s), dim, d, arr.ctypes.data_as(C.POINTER(C.c_double)),
                          f, sl, sr, F.ctypes.data_as(C.POINTER(C.c_double)), C.byref(us), C.byref(ps))
    assert rc == 0
    return F[:dim + 3], us.value, ps.value


def prim_row(e, p, T, Y, u):
    r, en = C.c_double(), C.c_double()
    L().og_eos_forward(C.byref(e), p, T, Y, C.byref(r), C.byref(en))
    c = L().og_mix_sound(C.byref(e), p, T, Y)
    v_g = L().og_spec_volume(C.byref(e), 1, p, T)
    return [r.value, u[0], u[1], u[2], p, T, Y, c, Y * r.value * v_g, 0.0, 0.0, 0.0, en.value], en.value


@pytest.mark.parametrize("f", [1, 0])
@pytest.mark.parametrize("Y", [0.0, 0.3, 1.0])
def test_uniform_state_gives_euler_flux(f, Y):
    """a uniform state: u* = u_n, p* = p and the face flux is the exact flux of
    eq. (2-2): (rho u, rho u u + p n, rho u H, rho u xi)"""
    e = make_eos(EOSD)
    p, T, u = 2e5, 310.0, (12.0, -3.0, 0.0)
    row, en = prim_row(e, p, T, Y, u)
    W4 = [row] * 4
    for d in (0, 1):
        F, us, ps = face(W4, f=f, d=d)
        rho = row[0]
        un = u[d]
        H = en + 0.5 * (u[0] ** 2 + u[1] ** 2) + p / rho
        exact = [rho * un, rho * un * u[0] + (p if d == 0 else 0), rho * un * u[1] + (p if d == 1 else 0),
                 rho * un * H, rho * un * Y]
        assert abs(us - un) < 1e-12 * 20
        assert abs(ps - p) < 1e-9
        np.testing.assert_allclose(F, exact, rtol=1e-12, atol=1e-9)


def test_mirror_symmetry_of_the_face():
    """reversing the stencil and the normal velocity mirrors the face flux"""
    e = make_eos(EOSD)
    rng = np.random.default_rng(9)
    for f in (1, 0):
        rows = []
        for _ in range(4):
            r, _ = prim_row(e, 1e5 * rng.uniform(0.8, 1.2), rng.uniform(280, 320), rng.uniform(0, 1),
                            (rng.uniform(-50, 50), rng.uniform(-50, 50), 0.0))
            rows.append(r)
        F, us, ps = face(rows, f=f)
        mir = [list(r) for r in rows[::-1]]
        for r in mir:
            r[1] = -r[1]
        Fm, usm, psm = face(mir, f=f)
        assert abs(us + usm) < 1e-12 * (abs(us) + 1)
        assert abs(ps - psm) < 1e-9
        assert abs(F[0] + Fm[0]) < 1e-10 * (abs(F[0]) + 1)
        assert abs(F[1] - Fm[1]) < 1e-9 * abs(F[1])
        assert abs(F[2] + Fm[2]) < 1e-9 * (abs(F[2]) + 1)


def test_third_difference_pressure_term_is_dissipative():
    """smooth branch (D.5): a pressure higher on the left of the face pushes u*
    to the right of the central velocity"""
    e = make_eos(EOSD)
    rows = [prim_row(e, p, 300.0, 1.0, (0.0, 0.0, 0.0))[0] for p in (0.99e5, 1.01e5, 0.99e5, 1.01e5)]
    _, us, _ = face(rows, f=0)
    assert us > 0.0


def test_tdu_ideal_gas_density():
    """TDU (eq. 3-5): the face density of an ideal gas is p*/(R T_f)"""
    e = make_eos(EOSD)
    rows = [prim_row(e, 1e5 * (1 + 0.01 * i), 300.0 + i, 1.0, (10.0, 0.0, 0.0))[0] for i in range(4)]
    F, us, ps = face(rows, f=1)
    # upwind (u* > 0): left state; T_L by Minmod from cells 0..2
    T = [300.0 + i for i in range(4)]
    TL = T[1] + 0.5 * L().og_slope(0, T[1] - T[0], T[2] - T[1])
    assert abs(F[0] / us - ps / (287.0 * TL)) < 1e-12 * F[0] / us
