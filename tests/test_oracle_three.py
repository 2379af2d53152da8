"""Pins of the oracle's second gas species (three components: a liquid and two
ideal gases, Table A.1 and eqs. A.1.2-A.1.5 in pressure-temperature
equilibrium; both gas mass fractions transported, reconstructed and used by
the TDU) against what the mathematics fixes: closure round trips, reduction to
two components, invariance under splitting one gas into two identical ones,
stationarity, pressure/velocity equilibrium across moving interfaces and
conservation."""
import ctypes as C

import numpy as np
import pytest

from oracle.oracle import Oracle, lib, make_eos
from paper_2304_00140_amd import workloads as W

WATER = W.sg(4.4, 6e8, 607.866)
AIR = W.sg(1.4, 0.0, 717.5)
HEL = W.sg(1.67, 0.0, 3110.0)


def fwd2(e, p, T, Y1, Y2):
    r, en = C.c_double(), C.c_double()
    assert lib().og_eos_forward2(C.byref(e), p, T, Y1, Y2, C.byref(r), C.byref(en)) == 0
    return r.value, en.value


def inv2(e, rho, en, Y1, Y2):
    p, T = C.c_double(), C.c_double()
    assert lib().og_eos_inverse2(C.byref(e), rho, en, Y1, Y2, 0.0, C.byref(p), C.byref(T)) == 0
    return p.value, T.value


def test_three_component_round_trip():
    """(p, T, alpha_1, alpha_2) -> (rho, e, xi_1, xi_2) by Table A.1 with each
    component's own law, back to (p, T) by the closure"""
    e = make_eos(W.make_eos(WATER, AIR, HEL))
    L = lib()
    rng = np.random.default_rng(21)
    for _ in range(200):
        p = 10 ** rng.uniform(4, 8)
        T = rng.uniform(250, 900)
        a1, a2 = rng.dirichlet([1, 1, 1])[:2] * rng.choice([1.0, 1e-3, 1 - 1e-9])
        r = [1.0 / L.og_spec_volume(C.byref(e), k, p, T) for k in range(3)]
        en_k = [L.og_spec_energy(C.byref(e), k, p, T) for k in range(3)]
        al = [1 - a1 - a2, a1, a2]
        rho = sum(al[k] * r[k] for k in range(3))
        Y = [al[k] * r[k] / rho for k in range(3)]
        en = sum(Y[k] * en_k[k] for k in range(3))
        rr, ee = fwd2(e, p, T, Y[1], Y[2])
        assert abs(rr / rho - 1) < 1e-12 and abs(ee / en - 1) < 1e-12
        pp, TT = inv2(e, rho, en, Y[1], Y[2])
        assert abs(pp - p) < 1e-9 * (p + 6e8) and abs(TT - T) < 1e-9 * T


def test_reduces_to_two_components_without_the_second_gas():
    e3 = make_eos(W.make_eos(WATER, AIR, HEL))
    e2 = make_eos(W.make_eos(WATER, AIR))
    L = lib()
    for p, T, Y in [(1e5, 300.0, 1e-3), (3e6, 500.0, 0.5), (1e7, 350.0, 0.999)]:
        r2, en2 = C.c_double(), C.c_double()
        L.og_eos_forward(C.byref(e2), p, T, Y, C.byref(r2), C.byref(en2))
        r3, en3 = fwd2(e3, p, T, Y, 0.0)
        assert r3 == r2.value and en3 == en2.value
        pa, Ta = C.c_double(), C.c_double()
        L.og_eos_inverse(C.byref(e2), r2.value, en2.value, Y, 0.0, C.byref(pa), C.byref(Ta))
        pb, Tb = inv2(e3, r2.value, en2.value, Y, 0.0)
        assert abs(pb - pa.value) < 1e-12 * (p + 6e8) and abs(Tb - Ta.value) < 1e-12 * T


def test_splitting_a_gas_into_two_identical_gases():
    """gas 2 identical to gas 1: any split of the gas mass fraction gives the
    two-component state (the closure sees one gas)"""
    e3 = make_eos(W.make_eos(WATER, AIR, AIR))
    e2 = make_eos(W.make_eos(WATER, AIR))
    L = lib()
    for p, T, Y in [(1e5, 300.0, 0.2), (5e6, 420.0, 0.7)]:
        r2, en2 = C.c_double(), C.c_double()
        L.og_eos_forward(C.byref(e2), p, T, Y, C.byref(r2), C.byref(en2))
        for f in (0.0, 0.3, 0.5, 1.0):
            r3, en3 = fwd2(e3, p, T, f * Y, (1 - f) * Y)
            assert abs(r3 / r2.value - 1) < 1e-14 and abs(en3 / en2.value - 1) < 1e-14
            pp, TT = inv2(e3, r2.value, en2.value, f * Y, (1 - f) * Y)
            assert abs(pp - p) < 1e-9 * (p + 6e8) and abs(TT - T) < 1e-10 * T


SPLIT = 0.3


def split_case(dim, n, seed, thinc, switching=0, sigma=0.0):
    """a two-component random state and the same state with its gas split
    0.3 : 0.7 between two identical gases"""
    c2 = W.random_state(dim, n, seed, switching=switching, sigma=sigma)
    c2["scheme"]["thinc"] = thinc
    c3 = dict(c2)
    c3["eos"] = W.make_eos(_comp(c2, 0), _comp(c2, 1), _comp(c2, 1))
    p, T, a = c2["prim"][0], c2["prim"][1], c2["prim"][2]
    u = list(c2["prim"][3:3 + dim])
    c3["prim"] = W.pack_prim(p, T, SPLIT * a, u + [(1.0 - SPLIT) * a])
    return c2, c3


def _comp(case, k):
    e = case["eos"]
    return W.sg(e["gamma"][k], e["pinf"][k], e["cv"][k], e["q"][k])


@pytest.mark.parametrize("dim,switching,sigma", [(1, 0, 0.0), (2, 0, 0.0), (2, 1, 0.05), (3, 1, 0.0)])
def test_rhs_invariant_under_gas_splitting(dim, switching, sigma):
    """the limiters are homogeneous of degree one, so scaling a gas fraction
    scales its reconstruction; with gas 2 = gas 1 and xi_1 : xi_2 = 0.3 : 0.7
    the three-component RHS of mass, momentum and energy equals the
    two-component RHS and the two fraction RHS are 0.3 and 0.7 of its xi RHS
    (THINC off: its eligibility band eps < xi < 1 - eps is not scale-free)"""
    n = {1: [61], 2: [23, 17], 3: [11, 9, 8]}[dim]
    c2, c3 = split_case(dim, n, 30 + dim, thinc=0, switching=switching, sigma=sigma)
    o2, o3 = Oracle(c2), Oracle(c3)
    q2, q3 = o2.cons_from_prim(), o3.cons_from_prim()
    np.testing.assert_allclose(q3[:2 + dim], q2[:2 + dim], rtol=1e-13, atol=1e-13 * np.abs(q2).max())
    r2, r3 = o2.rhs(q2), o3.rhs(q3)
    scale = np.abs(r2).max(axis=1)
    for f in range(2 + dim):
        assert np.abs(r3[f] - r2[f]).max() < 1e-10 * scale[f]
    assert np.abs(r3[2 + dim] - SPLIT * r2[2 + dim]).max() < 1e-10 * scale[2 + dim]
    assert np.abs(r3[3 + dim] - (1.0 - SPLIT) * r2[2 + dim]).max() < 1e-10 * scale[2 + dim]


def test_uniform_three_component_state_is_stationary():
    c = W.random_state(2, [12, 10], 5, second_gas=True)
    x, y = W.cell_centres(c["grid"])
    c["prim"] = W.pack_prim(np.full_like(x, 2e5), np.full_like(x, 320.0), np.full_like(x, 0.3),
                            [np.full_like(x, 7.0), np.full_like(x, -3.0), np.full_like(x, 0.25)])
    o = Oracle(c)
    q = o.cons_from_prim()
    assert q.shape[0] == 6
    r = o.rhs(q)
    scale = np.abs(q).max(axis=1, keepdims=True) / c["grid"]["dx"][0] * 1e-13 * 200
    assert np.all(np.abs(r) <= scale)


def test_three_component_advection_keeps_pressure_and_velocity():
    """a liquid slab between the two gases, uniform p, T and u, periodic: the
    interfaces move without disturbing p and u (the TDU's equilibrium
    property with two transported gas fractions)"""
    n = 100
    g = W.make_grid(1, [n], [1.0], [[W.BC_PERIODIC, W.BC_PERIODIC]])
    x = W.cell_centres(g)[0]
    liq = (1.0 - W.smeared(x - 0.6, 0.01)) * W.smeared(x - 0.3, 0.01)
    gas2 = W.smeared(x - 0.6, 0.01) * (1.0 - W.smeared(x - 0.85, 0.01))
    a1 = np.clip(1.0 - liq - gas2, 0.0, 1.0)
    prim = W.pack_prim(np.full(n, 1e5), np.full(n, 300.0), a1, [np.full(n, 50.0), gas2])
    case = dict(name="adv3", grid=g, eos=W.make_eos(WATER, AIR, HEL), scheme=W.default_scheme(),
                prim=prim, steps=None, t_end=0.0, storage=dict(p_ref=1e5, T_ref=300.0))
    o = Oracle(case)
    q = o.cons_from_prim()
    tot0 = o.totals(q)
    t = 0.0
    for k in range(150):
        t, _ = o.step(q, k, t)
    w = o.prim_from_cons(q)
    assert np.abs(w[4] - 1e5).max() < 1e-12 * 6e8
    assert np.abs(w[1] - 50.0).max() < 1e-12 * 50.0
    assert w[9].max() > 0.9 and w[6].max() > 0.9      # both gases still there
    tot = o.totals(q)
    np.testing.assert_allclose(tot, tot0, rtol=1e-13, atol=1e-13 * np.abs(tot0).max())


def test_field_round_trip_recovers_both_volume_fractions():
    """primitives (p, T, alpha_1, u, alpha_2) -> conserved -> primitives gives
    back both gas volume fractions (A.1.4) and the volume fractions of the
    three components sum to one (A.1.5)"""
    c = W.random_state(2, [17, 13], 8, second_gas=True)
    o = Oracle(c)
    q = o.cons_from_prim()
    w = o.prim_from_cons(q)
    pr = c["prim"]
    np.testing.assert_allclose(w[4], pr[0], rtol=1e-10)
    np.testing.assert_allclose(w[5], pr[1], rtol=1e-11)
    np.testing.assert_allclose(w[8], pr[2], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(w[10], pr[5], rtol=1e-9, atol=1e-12)
    L = lib()
    vL = np.array([L.og_spec_volume(C.byref(o.e), 0, p, T) for p, T in zip(w[4], w[5])])
    aL = (1.0 - w[6] - w[9]) * w[0] * vL
    np.testing.assert_allclose(aL + w[8] + w[10], 1.0, atol=1e-10)
