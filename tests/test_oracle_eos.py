"""Pins of the oracle's thermodynamic closure (Appendix A) against what the
paper and thermodynamics fix independently of the oracle's own formulas."""
import ctypes as C
import math

import numpy as np
import pytest

from oracle.oracle import lib, make_eos
from paper_2304_00140_amd import workloads as W


def _eos(c0, c1):
    return make_eos(W.make_eos(c0, c1))


WATER = W.sg(4.4, 6e8, 607.866)
AIR = W.sg(1.4, 0.0, 717.5)
GAS_T41_1 = W.sg(5.0, 0.0, 1875.18)
GAS_T41_2 = W.sg(1.6, 0.0, 472.22)
PRMIX = W.pr_mixture([W.NITROGEN, W.METHANE], [0.8, 0.2], 900.0)


def fwd(e, p, T, Y):
    r, en = C.c_double(), C.c_double()
    assert lib().og_eos_forward(C.byref(e), p, T, Y, C.byref(r), C.byref(en)) == 0
    return r.value, en.value


def inv(e, rho, en, Y, Tg=0.0):
    p, T = C.c_double(), C.c_double()
    rc = lib().og_eos_inverse(C.byref(e), rho, en, Y, Tg, C.byref(p), C.byref(T))
    assert rc == 0
    return p.value, T.value


def test_table_41_densities():
    """Table 4.1: rho = p / (R T) with R = (gamma - 1) cv gives the printed
    4.444 and 117.647 kg/m^3 at 1e7 Pa, 300 K (R read in J/(kg K))."""
    e = _eos(GAS_T41_1, GAS_T41_2)
    r1, _ = fwd(e, 1e7, 300.0, 0.0)
    r2, _ = fwd(e, 1e7, 300.0, 1.0)
    assert abs(r1 - 4.444) < 5e-4
    assert abs(r2 - 117.647) < 5e-3


def test_pure_stiffened_gas_law():
    """eq. (A.1.1): p = (gamma - 1) rho (e - q) - gamma p_inf for each pure component,
    and the ideal-gas forms rho = p / (R T), e = cv T (Appendix A.1 text)."""
    e = _eos(W.sg(4.4, 6e8, 607.866, q=-1.2e6), AIR)
    for p, T in [(1e5, 290.0), (3e7, 400.0), (-2e7, 280.0)]:
        rho, en = fwd(e, p, T, 0.0)
        assert abs((4.4 - 1) * rho * (en + 1.2e6) - 4.4 * 6e8 - p) < 1e-6 * (p + 6e8) * 1e-3
        rho, en = fwd(e, abs(p), T, 1.0)
        assert abs(rho - abs(p) / (287.0 * T)) < 1e-12 * rho
        assert abs(en - 717.5 * T) < 1e-12 * en


def test_sound_speed_matches_appendix_a():
    """c_k = sqrt(gamma (p + p_inf) / rho_k) as printed in Appendix A.1."""
    e = _eos(WATER, AIR)
    for p, T in [(1e5, 290.0), (5e7, 350.0)]:
        for k in (0, 1):
            rho, _ = fwd(e, p, T, float(k))
            g, pinf = (4.4, 6e8) if k == 0 else (1.4, 0.0)
            c_ref = math.sqrt(g * (p + pinf) / rho)
            assert abs(lib().og_sound(C.byref(e), k, p, T) - c_ref) < 1e-12 * c_ref


def test_water_sound_speed_value():
    """water-like stiffened gas at 1 bar: c = 1624.9 m/s for rho = 1000"""
    T = 1e5 / (1.2 * 287.0)
    cv = (1e5 + 6e8) / (3.4 * 1000 * T)
    e = _eos(W.sg(4.4, 6e8, cv), AIR)
    c = lib().og_sound(C.byref(e), 0, 1e5, T)
    assert abs(c - 1624.94) < 0.01


@pytest.mark.parametrize("pair", [(WATER, AIR), (GAS_T41_1, GAS_T41_2), (AIR, WATER)])
def test_round_trip_and_mixing(pair):
    """(p, T, xi) -> (rho, e) -> (p, T): the inverse (a quadratic) and the
    forward law are independent formulas; a volume-weighted mixture of the two
    pure fluids at one (p, T) must invert to that (p, T) (Table A.1)."""
    e = _eos(*pair)
    rng = np.random.default_rng(1)
    worst_p = worst_T = 0.0
    for _ in range(400):
        p = 10 ** rng.uniform(3.5, 8)
        T = rng.uniform(200, 900)
        al = rng.choice([0.0, 1.0, rng.uniform(0, 1), 10 ** rng.uniform(-12, -1)])
        rL, eL = fwd(e, p, T, 0.0)
        rG, eG = fwd(e, p, T, 1.0)
        rho = al * rG + (1 - al) * rL
        rhoe = al * rG * eG + (1 - al) * rL * eL
        Y = al * rG / rho
        pp, TT = inv(e, rho, rhoe / rho, Y)
        scale = p + max(pair[0]["pinf"], pair[1]["pinf"])
        worst_p = max(worst_p, abs(pp - p) / scale)
        worst_T = max(worst_T, abs(TT - T) / T)
    assert worst_p < 1e-11
    assert worst_T < 1e-10


def test_liquid_in_tension_pure_cell():
    """a pure liquid cell below zero pressure (p > -p_inf) is a valid state"""
    e = _eos(WATER, AIR)
    rho, en = fwd(e, -5e7, 300.0, 0.0)
    p, T = inv(e, rho, en, 0.0)
    assert abs(p + 5e7) < 1e-6 * 6e8 and abs(T - 300) < 1e-9


def test_fraction_outside_unit_interval_closes_as_pure_component():
    """A mass fraction just below 0 (above 1) is closed as the pure liquid
    (gas): the result is eq. (A.1.1) solved for p and T by hand, for an SG and
    a Peng-Robinson partner."""
    gl, pl, cl = 2.5, 3.338e8, 806.7
    for partner in (AIR, PRMIX):
        e = _eos(W.sg(gl, pl, cl), partner)
        rho, en = 704.0, 7.98e5
        p_hand = (gl - 1) * rho * en - gl * pl
        T_hand = (en - pl / rho) / cl
        for Y in (-2.4e-4, -1e-12):
            p, T = inv(e, rho, en, Y)
            assert abs(p - p_hand) < 1e-12 * (abs(p_hand) + pl)
            assert abs(T - T_hand) < 1e-12 * T_hand
    e = _eos(WATER, AIR)
    rho = 1.2
    en = 717.5 * 300.0
    p, T = inv(e, rho, en, 1.0 + 3e-7)
    assert abs(p - 0.4 * rho * en) < 1e-12 * p and abs(T - 300.0) < 1e-12 * 300.0
    assert lib().og_clip_fraction(float("nan")) != lib().og_clip_fraction(float("nan"))


def test_sound_speed_of_pure_liquid_in_tension_with_pr_partner():
    """a pure liquid cell below zero pressure keeps the liquid's
    c = sqrt(gamma (gamma - 1) cv T) (Appendix A.1): the absent Peng-Robinson
    gas, which has no state at p < 0, does not enter the maximum"""
    gl, pl, cl = 2.5, 3.338e8, 806.7
    e = _eos(W.sg(gl, pl, cl), PRMIX)
    for p, T in [(-3.9e7, 366.8), (5e6, 400.0)]:
        c = lib().og_mix_sound(C.byref(e), p, T, -1e-11)
        assert abs(c - math.sqrt(gl * (gl - 1) * cl * T)) < 1e-12 * c
    # with the gas present at positive pressure both enter: the liquid's is larger
    c = lib().og_mix_sound(C.byref(e), 5e6, 400.0, 0.5)
    assert c >= math.sqrt(gl * (gl - 1) * cl * 400.0) * (1 - 1e-15)


# ---------------------------------------------------------------- Peng-Robinson

def test_pr_ideal_gas_limit():
    """a, b -> 0 relative to RT v at low pressure: Z -> 1 and the departure energy
    vanishes (A.2.1 reduces to the ideal gas)."""
    e = _eos(WATER, PRMIX)
    M = 0.8 * W.NITROGEN["M"] + 0.2 * W.METHANE["M"]
    for T in (300.0, 800.0):
        p = 10.0
        v = lib().og_spec_volume(C.byref(e), 1, p, T)
        Z = p * v * M / (W.R_UNIV * T)
        assert abs(Z - 1) < 1e-5
        en = lib().og_spec_energy(C.byref(e), 1, p, T)
        assert abs(en - 900.0 * T) < 1e-4 * en


def test_pr_cubic_root_and_pressure():
    """v(p, T) from the cubic satisfies eq. (A.2.1) p = RT/(V-b) - a/(V^2+2bV-b^2)"""
    e = _eos(WATER, PRMIX)
    for p in (1e5, 5e6, 6e7):
        for T in (250.0, 400.0, 900.0):
            v = lib().og_spec_volume(C.byref(e), 1, p, T)
            assert abs(lib().og_pr_pressure(C.byref(e), 1, T, v) - p) < 1e-10 * p


def test_pr_departure_energy_is_the_integral():
    """e(T, v) - e_ideal(T) = integral_inf^V (T dp/dT|_V - p) dV' (textbook
    identity), evaluated by quadrature with dp/dT from finite differences of the
    pressure law only."""
    e = _eos(WATER, PRMIX)
    L = lib()
    M = 0.8 * W.NITROGEN["M"] + 0.2 * W.METHANE["M"]
    for T, v in [(400.0, 1.0 / 40.0), (300.0, 1.0 / 200.0)]:
        def integrand(vm):
            h = 1e-4 * T
            dpdT = (L.og_pr_pressure(C.byref(e), 1, T + h, vm) - L.og_pr_pressure(C.byref(e), 1, T - h, vm)) / (2 * h)
            return T * dpdT - L.og_pr_pressure(C.byref(e), 1, T, vm)
        # substitute v = v0 / s, s in (0, 1]: dv = -v0/s^2 ds
        s = np.linspace(1e-6, 1.0, 200001)
        f = np.array([integrand(v / si) * v / si ** 2 for si in s])
        integral = -np.trapezoid(f, s)          # from infinity down to v
        dep = L.og_pr_energy_tv(C.byref(e), 1, T, v) - 900.0 * T
        assert abs(dep - integral) < 2e-4 * abs(dep)


def test_pr_round_trip_pure_and_mixed():
    e = _eos(W.sg(2.5, 3.338e8, 806.7), PRMIX)
    rng = np.random.default_rng(3)
    for _ in range(60):
        p = 10 ** rng.uniform(5, 7.5)
        T = rng.uniform(250, 700)
        al = rng.choice([1.0, rng.uniform(0, 1), 1 - 10 ** rng.uniform(-10, -2)])
        rL, eL = fwd(e, p, T, 0.0)
        rG, eG = fwd(e, p, T, 1.0)
        rho = al * rG + (1 - al) * rL
        Y = al * rG / rho
        en = (al * rG * eG + (1 - al) * rL * eL) / rho
        pp, TT = inv(e, rho, en, Y)
        assert abs(pp - p) < 1e-9 * (p + 3.338e8)
        assert abs(TT - T) < 1e-9 * T


def test_pr_sound_speed_from_thermodynamics():
    """c^2 = (dp/drho)_e + p / rho^2 (dp/de)_rho, finite differences of the
    oracle's pressure as a function of (rho, e) (the inverse), against the
    closed-form speed of sound."""
    e = _eos(WATER, PRMIX)
    for p, T in [(5e6, 400.0), (2e7, 300.0)]:
        rho, en = fwd(e, p, T, 1.0)

        def P(r, ee):
            return inv(e, r, ee, 1.0)[0]
        hr, he = 1e-5 * rho, 1e-5 * en
        dpdr = (P(rho + hr, en) - P(rho - hr, en)) / (2 * hr)
        dpde = (P(rho, en + he) - P(rho, en - he)) / (2 * he)
        c2 = dpdr + p / rho ** 2 * dpde
        c = lib().og_sound(C.byref(e), 1, p, T)
        assert abs(math.sqrt(c2) - c) < 1e-5 * c
