"""Seeded synthetic workloads shaped like the paper's cases.

This module only builds inputs: grid, material and scheme parameters and the
initial primitive fields (p, T, alpha_G, u).  It holds none of the method's
arithmetic; conversion of primitives to conserved variables is done by the
consumer (the GPU library or the CPU oracle), each with its own closure.

Component 0 ("L") is the liquid or ambient fluid, component 1 ("G") the gas or
bubble fluid; xi is the mass fraction of G.

Every case dict has:
  name, grid{dim, n[3], dx[3], bc[3][2], inflow{...}}, eos{kind[2], gamma[2],
  pinf[2], cv[2], q[2], pr[2]}, scheme{...}, prim[(3+D), ncell] (p, T, alpha_G,
  u_1..u_D; x fastest), steps, t_end, storage{p_ref, T_ref}.
A barotropic-model case (eos["model"] = MODEL_BAROTROPIC) carries the
parameters of Section 2.2 in eos["baro"]; its T row is not used.
"""
import math

import numpy as np

BC_PERIODIC, BC_WALL, BC_ZEROGRAD, BC_INFLOW, BC_FARFIELD = 0, 1, 2, 3, 4
EOS_SG, EOS_PR = 0, 1
MODEL_FOUR_EQ, MODEL_BAROTROPIC = 0, 1
LIM = {"minmod": 0, "koren": 1, "vanalbada": 2, "vanleer": 3, "chakravarthy": 4,
       "mc": 5, "superbee": 6, "none": 7}
R_UNIV = 8.314462618

# public critical constants (NIST Chemistry WebBook / Poling, Prausnitz &
# O'Connell tables): Tc [K], pc [Pa], acentric factor, molar mass [kg/mol], Zc
NITROGEN = dict(Tc=126.19, pc=3.3958e6, omega=0.0372, M=28.0134e-3, Zc=0.2894)
METHANE = dict(Tc=190.56, pc=4.5992e6, omega=0.0114, M=16.0428e-3, Zc=0.2863)


def default_scheme(**kw):
    s = dict(switching=0, lim_u=LIM["koren"], lim_s=LIM["minmod"], thinc=1,
             beta=1.6, thinc_gamma=1e-20, eps_interface=1e-4,
             theta_ducros=0.95, theta_gas=0.4, eps_ducros=1e-20, kappa3=0.25,
             rk=[0.25, 1.0 / 3.0, 0.5, 1.0], cfl=0.5, sigma=0.0, eps_normal=1e-12,
             gravity=[0.0, 0.0, 0.0])
    s.update(kw)
    return s


def sg(gamma, pinf, cv, q=0.0, mu=0.0, kc=0.0):
    """stiffened-gas component; mu [Pa s] and kc [W/(m K)] are its viscosity
    and thermal conductivity (0: inviscid, adiabatic)"""
    return dict(kind=EOS_SG, gamma=gamma, pinf=pinf, cv=cv, q=q, mu=mu, kc=kc)


def pr_mixture(species, X, cv, q=0.0, mu=0.0, kc=0.0):
    """Peng-Robinson pseudo-mixture of fixed composition X (mole fractions)."""
    sp = [dict(s) for s in species]
    for s in sp:
        s["vc"] = s["Zc"] * R_UNIV * s["Tc"] / s["pc"]
    return dict(kind=EOS_PR, gamma=0.0, pinf=0.0, cv=cv, q=q, species=sp, X=list(X),
                kij=[[0.0] * len(sp) for _ in sp], mu=mu, kc=kc)


def make_eos(c0, c1, c2=None):
    """closure of two components, or of three (liquid c0 and two ideal gases
    c1, c2 whose mass fractions are both transported)"""
    comps = [c0, c1] if c2 is None else [c0, c1, c2]
    return dict(kind=[c["kind"] for c in comps], gamma=[c["gamma"] for c in comps],
                pinf=[c["pinf"] for c in comps], cv=[c["cv"] for c in comps],
                q=[c["q"] for c in comps], pr=[c if c["kind"] == EOS_PR else None for c in comps],
                mu=[c.get("mu", 0.0) for c in comps], kc=[c.get("kc", 0.0) for c in comps])


def baro_eos(rho_sat=1000.0, p_sat=2340.0, c_liq=1500.0, rho_vap=0.0173, R_gas=296.8, T_gas=336.9,
             mu_liq=0.0, mu_gas=0.0, mu_vap=0.0, RT2=None, mu_gas2=0.0):
    """barotropic equilibrium model (Section 2.2): a liquid that becomes a
    liquid-vapour mixture below p_sat, and one isothermal ideal gas (two with
    RT2 = R_Gas2 T_ref2 given, eqs. 2-5, 2-6).  Defaults: Section 4.5's liquid
    and gas values; the saturated vapour density is that of water vapour at
    2340 Pa, 293 K (p / (R_v T), R_v = 461.5 J/(kg K)).  mu_liq, mu_gas,
    mu_vap, mu_gas2 [Pa s]: the viscosities of eq. (2-8) (0: inviscid)."""
    n = 2 if RT2 is None else 3
    baro = dict(rho_sat=rho_sat, p_sat=p_sat, c_liq=c_liq, rho_vap=rho_vap, RT=R_gas * T_gas, mu_vap=mu_vap)
    if RT2 is not None:
        baro["RT2"] = RT2
    return dict(model=MODEL_BAROTROPIC, kind=[EOS_SG] * n, gamma=[0.0] * n, pinf=[0.0] * n,
                cv=[0.0] * n, q=[0.0] * n, pr=[None] * n, mu=[mu_liq, mu_gas, mu_gas2][:n], kc=[0.0] * n,
                baro=baro)


def cv_for_density(gamma, pinf, rho, p, T):
    """Specific heat that puts a stiffened gas at density rho at (p, T); the
    paper's cases give (gamma, p_inf, rho) and one temperature for all fluids."""
    return (p + pinf) / ((gamma - 1.0) * rho * T)


def make_grid(dim, n, L, bc):
    n3 = list(n) + [1] * (3 - len(n))
    L3 = list(L) + [1.0] * (3 - len(L))
    dx = [L3[d] / n3[d] if d < dim else 1.0 for d in range(3)]
    bc3 = [list(b) for b in bc] + [[BC_PERIODIC, BC_PERIODIC]] * (3 - len(bc))
    return dict(dim=dim, n=n3, dx=dx, bc=bc3,
                inflow=dict(p=0.0, T=0.0, alpha=0.0, u=0.0, radius=0.0, center=[0.0, 0.0],
                            noise=0.0, seed=0),
                farfield=dict(p=0.0, T=0.0, alpha=0.0))


def cell_centres(grid):
    dim = grid["dim"]
    axes = [(np.arange(grid["n"][d]) + 0.5) * grid["dx"][d] for d in range(dim)]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")[::-1]   # x fastest in C order
    return [m.reshape(-1) for m in mesh]


def smeared(dist, width):
    """0 inside (dist < 0), 1 outside, tanh profile of the given width"""
    return 0.5 * (1.0 + np.tanh(dist / width))


def pack_prim(p, T, alpha, u):
    return np.ascontiguousarray(np.stack([p, T, alpha] + list(u)).astype(np.float64))


# ---------------------------------------------------------------- the cases

def interface_advection_1d(n=200, periods=1.0):
    """Water slab in air, periodic, uniform p, u, T (interface-only problem,
    Section 4.1 shape with a stiff liquid)."""
    p0, u0 = 1e5, 100.0
    T0 = p0 / (1.2 * 287.0)
    water = sg(4.4, 6e8, cv_for_density(4.4, 6e8, 1000.0, p0, T0))
    air = sg(1.4, 0.0, 287.0 / 0.4)
    g = make_grid(1, [n], [1.0], [[BC_PERIODIC, BC_PERIODIC]])
    (x,) = cell_centres(g)
    alpha = np.where((x > 0.25) & (x < 0.75), 0.0, 1.0)
    prim = pack_prim(np.full(n, p0), np.full(n, T0), alpha, [np.full(n, u0)])
    return dict(name="interface_advection_1d", grid=g, eos=make_eos(water, air),
                scheme=default_scheme(), prim=prim, steps=None, t_end=periods * 1.0 / u0,
                storage=dict(p_ref=p0, T_ref=T0))


def interface_advection_1d_paper(n=100, periods=4.0):
    """Section 4.1 with Table 4.1's two ideal gases, 0.2 m, p = 1e7, u = 5."""
    p0, u0, T0 = 1e7, 5.0, 300.0
    c1 = sg(5.0, 0.0, 1875.18)
    c2 = sg(1.6, 0.0, 472.22)
    g = make_grid(1, [n], [0.2], [[BC_PERIODIC, BC_PERIODIC]])
    (x,) = cell_centres(g)
    alpha = np.where((x > 0.05) & (x < 0.15), 1.0, 0.0)
    prim = pack_prim(np.full(n, p0), np.full(n, T0), alpha, [np.full(n, u0)])
    return dict(name="interface_advection_1d_paper", grid=g, eos=make_eos(c1, c2),
                scheme=default_scheme(), prim=prim, steps=None, t_end=periods * 0.2 / u0,
                storage=dict(p_ref=p0, T_ref=T0))


def normal_shock(gamma, M):
    """textbook normal-shock ratios: p2/p1, rho2/rho1, T2/T1"""
    pr = 1.0 + 2.0 * gamma / (gamma + 1.0) * (M * M - 1.0)
    rr = (gamma + 1.0) * M * M / ((gamma - 1.0) * M * M + 2.0)
    return pr, rr, pr / rr


def shock_bubble_2d(nx=1024, ny=256, steps=2000):
    """Mach 1.22 shock in air hitting a helium-like cylinder (Section 4.2 shape)."""
    Lx, Ly = 0.2, 0.05
    R_air, g_air = 287.0, 1.4
    R_he, g_he = 2080.0, 1.67
    p1 = 1e5
    T1 = p1 / (0.166 * R_he)
    air = sg(g_air, 0.0, R_air / (g_air - 1.0))
    he = sg(g_he, 0.0, R_he / (g_he - 1.0))
    g = make_grid(2, [nx, ny], [Lx, Ly], [[BC_ZEROGRAD, BC_ZEROGRAD], [BC_WALL, BC_WALL]])
    x, y = cell_centres(g)
    dx = g["dx"][0]
    xc, yc, rb = 0.125, 0.025, 0.0125
    r = np.hypot(x - xc, y - yc)
    alpha = 1.0 - smeared(r - rb, dx)
    M = 1.22
    pr, rr, tr = normal_shock(g_air, M)
    c1 = math.sqrt(g_air * R_air * T1)
    u2 = -M * c1 * (1.0 - 1.0 / rr)
    post = x > 0.145
    p = np.where(post, p1 * pr, p1)
    T = np.where(post, T1 * tr, T1)
    u = np.where(post, u2, 0.0)
    v = np.zeros_like(u)
    prim = pack_prim(p, T, alpha, [u, v])
    return dict(name="shock_bubble_2d", grid=g, eos=make_eos(air, he), scheme=default_scheme(),
                prim=prim, steps=steps, t_end=0.0, storage=dict(p_ref=p1, T_ref=T1))


def drop_2d(n=256, steps=10000, mode2=0.0, sigma=0.07, L=1e-3, rel_radius=0.25):
    """Water drop in air with CSF surface tension (Section 4.4 / Appendix C shape);
    mode2 > 0 gives r_s = R (1 + mode2 cos 2 phi)."""
    T0, p_out = 293.15, 1e5
    Rd = rel_radius * L
    p_in = p_out + sigma / Rd
    water = sg(4.4, 6e8, cv_for_density(4.4, 6e8, 1000.0, p_in, T0))
    air = sg(1.4, 0.0, 287.0 / 0.4)
    g = make_grid(2, [n, n], [L, L], [[BC_PERIODIC, BC_PERIODIC], [BC_PERIODIC, BC_PERIODIC]])
    x, y = cell_centres(g)
    dx = g["dx"][0]
    phi = np.arctan2(y - 0.5 * L, x - 0.5 * L)
    rs = Rd * (1.0 + mode2 * np.cos(2.0 * phi))
    alpha = smeared(np.hypot(x - 0.5 * L, y - 0.5 * L) - rs, dx)
    p = p_out + (p_in - p_out) * (1.0 - alpha)
    prim = pack_prim(p, np.full_like(p, T0), alpha, [np.zeros_like(p), np.zeros_like(p)])
    return dict(name="drop_2d", grid=g, eos=make_eos(water, air),
                scheme=default_scheme(sigma=sigma), prim=prim, steps=steps, t_end=0.0,
                storage=dict(p_ref=p_out, T_ref=T0), radius=Rd)


def bubble_collapse_batch(ncases=256, seed=230400140, nmin=64, nmax=256, steps=500):
    """Independent 2D gas-bubble collapses of uneven size (Section 4.9 shape):
    N ~ U{nmin..nmax}, bubble radius 0.1-0.3 of the domain, liquid/gas pressure
    ratio 10-1000 log-uniform.  The liquid starts from the Rayleigh-collapse
    pressure profile p = p_L + (p_g - p_L) R / r (no jump at the bubble wall)
    and the box is surrounded by a far-field reservoir at (p_L, T) standing in
    for the paper's non-reflective boundaries."""
    rng = np.random.default_rng(seed)
    L, T0, pg = 2e-3, 293.15, 1e4
    water = sg(4.4, 6e8, cv_for_density(4.4, 6e8, 1000.0, 1e5, T0))
    air = sg(1.4, 0.0, 287.0 / 0.4)
    cases = []
    for c in range(ncases):
        N = int(rng.integers(nmin, nmax + 1))
        fR = float(rng.uniform(0.1, 0.3))
        ratio = float(10.0 ** rng.uniform(1.0, 3.0))
        g = make_grid(2, [N, N], [L, L], [[BC_FARFIELD, BC_FARFIELD], [BC_FARFIELD, BC_FARFIELD]])
        pL = ratio * pg
        g["farfield"] = dict(p=pL, T=T0, alpha=0.0)
        x, y = cell_centres(g)
        r = np.hypot(x - 0.5 * L, y - 0.5 * L)
        R = fR * L
        alpha = 1.0 - smeared(r - R, g["dx"][0])
        p_liq = pL + (pg - pL) * np.minimum(1.0, R / np.maximum(r, 1e-300))
        p = pg * alpha + p_liq * (1.0 - alpha)
        prim = pack_prim(p, np.full_like(p, T0), alpha, [np.zeros_like(p), np.zeros_like(p)])
        cases.append(dict(name=f"bubble_collapse_{c}", grid=g, eos=make_eos(water, air),
                          scheme=default_scheme(), prim=prim, steps=steps, t_end=0.0,
                          storage=dict(p_ref=pL, T_ref=T0), ratio=ratio, radius=R))
    return cases


def liquid_jet_3d(nx=512, ny=256, nz=256, steps=200, D=89.4e-6, cells_per_D=32, seed=7,
                  gas="pr", core_length=None, viscous=False):
    """n-dodecane-like jet into an 80/20 N2/CH4 ambient at 5 MPa (Section 4.7/4.8
    shape), uniform Cartesian grid, inflow at x = 0 with 5 % velocity noise.

    The liquid core starts as a cylinder of diameter D along the whole domain
    (core_length=None), the stand-in for a jet that has already left the
    nozzle.  A finite core (core_length in m) has a flat head that hits the gas
    at rest; the lateral relief of that impact focuses on the axis, puts the
    liquid into tension and empties cells that hold trace gas to near vacuum,
    where the mixture has no state within a few hundred steps.

    viscous=True adds the stress and conduction terms of eq. (2-2) as in
    Section 4.8, with n-dodecane-like liquid mu = 4.5e-4 Pa s, kc = 0.11 W/(m K)
    and N2/CH4-like gas mu = 2.3e-5 Pa s, kc = 0.032 W/(m K) near 400 K
    (public property tables)."""
    p0, T0, uj = 5e6, 400.0, 300.0
    rho_l, c_l, g_l = 700.0, 1100.0, 2.5
    pinf_l = rho_l * c_l * c_l / g_l - p0
    mu_l, kc_l, mu_g, kc_g = (4.5e-4, 0.11, 2.3e-5, 0.032) if viscous else (0.0, 0.0, 0.0, 0.0)
    liquid = sg(g_l, pinf_l, cv_for_density(g_l, pinf_l, rho_l, p0, T0), mu=mu_l, kc=kc_l)
    X = [0.8, 0.2]
    Mmix = X[0] * NITROGEN["M"] + X[1] * METHANE["M"]
    cv_g = (X[0] * 2.5 + X[1] * 3.9) * R_UNIV / Mmix
    if gas == "pr":
        gasc = pr_mixture([NITROGEN, METHANE], X, cv_g, mu=mu_g, kc=kc_g)
    else:   # ideal-gas stand-in of the same molar mass and cv
        gasc = sg(1.0 + R_UNIV / (Mmix * cv_g), 0.0, cv_g, mu=mu_g, kc=kc_g)
    dx = D / cells_per_D
    g = make_grid(3, [nx, ny, nz], [nx * dx, ny * dx, nz * dx],
                  [[BC_INFLOW, BC_ZEROGRAD], [BC_ZEROGRAD, BC_ZEROGRAD], [BC_ZEROGRAD, BC_ZEROGRAD]])
    yc, zc = 0.5 * ny * dx, 0.5 * nz * dx
    g["inflow"] = dict(p=p0, T=T0, alpha=0.0, u=uj, radius=0.5 * D, center=[yc, zc],
                       noise=0.05, seed=seed)
    x, y, z = cell_centres(g)
    r = np.hypot(y - yc, z - zc)
    liq = 1.0 - smeared(r - 0.5 * D, dx)
    if core_length is not None:
        liq = liq * (1.0 - smeared(x - core_length, dx))
    alpha = 1.0 - liq
    del r
    u = uj * liq
    zero = np.zeros_like(u)
    prim = pack_prim(np.full_like(u, p0), np.full_like(u, T0), alpha, [u, zero, zero])
    return dict(name="liquid_jet_3d_viscous" if viscous else "liquid_jet_3d", grid=g, eos=make_eos(liquid, gasc),
                scheme=default_scheme(switching=1, sigma=0.02), prim=prim, steps=steps,
                t_end=0.0, storage=dict(p_ref=p0, T_ref=T0), viscous=viscous)


def dual_gas_layer_2d(nx=1024, ny=512, steps=1000, seed=2304, L=1e-3):
    """Temporal liquid layer between two different gases (the second gas
    species: three components), shaped like Section 4.6's dual-fuel shear layer:
    an n-dodecane-like stiffened-gas layer at +25 m/s between nitrogen-like
    (above) and methane-like (below) ideal gases at -25 m/s, 6 MPa, 400 K;
    periodic in x, slip walls in y; both interfaces carry seeded sinusoidal
    perturbations; sigma = 0.028 N/m (Section 4.8), sensor switching on."""
    rng = np.random.default_rng(seed)
    p0, T0, du = 6e6, 400.0, 25.0
    rho_l, c_l, g_l = 700.0, 1100.0, 2.5
    pinf_l = rho_l * c_l * c_l / g_l - p0
    liquid = sg(g_l, pinf_l, cv_for_density(g_l, pinf_l, rho_l, p0, T0))
    n2 = sg(1.4, 0.0, 2.5 * R_UNIV / NITROGEN["M"])
    ch4 = sg(1.0 + 1.0 / 3.3, 0.0, 3.3 * R_UNIV / METHANE["M"])
    g = make_grid(2, [nx, ny], [L, L * ny / nx], [[BC_PERIODIC, BC_PERIODIC], [BC_WALL, BC_WALL]])
    dx = g["dx"][0]
    x, y = cell_centres(g)
    Ly = ny * dx
    h = 0.0625 * Ly * 2.0                       # layer half-thickness
    def wave():
        f = np.zeros_like(x)
        for _ in range(4):
            k = int(rng.integers(1, 9))
            f += rng.uniform(-1, 1) * np.sin(2 * np.pi * k * x / L + rng.uniform(0, 2 * np.pi))
        return 2.0 * dx * f
    top = 0.5 * Ly + h + wave()
    bot = 0.5 * Ly - h + wave()
    liq = (1.0 - smeared(y - top, dx)) * smeared(y - bot, dx)
    a_n2 = (1.0 - liq) * smeared(y - 0.5 * Ly, 4 * dx)
    a_ch4 = np.clip(1.0 - liq - a_n2, 0.0, 1.0)
    u = du * (2.0 * liq - 1.0)
    v = np.zeros_like(u)
    prim = pack_prim(np.full_like(x, p0), np.full_like(x, T0), a_n2, [u, v, a_ch4])
    return dict(name="dual_gas_layer_2d", grid=g, eos=make_eos(liquid, n2, ch4),
                scheme=default_scheme(switching=1, sigma=0.028), prim=prim, steps=steps, t_end=0.0,
                storage=dict(p_ref=p0, T_ref=T0))


def square_to_circle_2d(n=150, steps=2000, L=0.75, side=0.2, sigma=800.0):
    """Section 4.5's 2D shape recovery: a square liquid body (rho 1000) of side
    0.2 m centred in a 0.75 m box of gas (rho 1 at 1 bar), sigma = 800 N/m,
    barotropic model with the section's values; zero-gradient sides stand in
    for its non-reflective boundaries; uniform 1 bar, at rest."""
    g = make_grid(2, [n, n], [L, L], [[BC_ZEROGRAD, BC_ZEROGRAD], [BC_ZEROGRAD, BC_ZEROGRAD]])
    x, y = cell_centres(g)
    dist = np.maximum(np.abs(x - 0.5 * L), np.abs(y - 0.5 * L)) - 0.5 * side
    alpha = smeared(dist, g["dx"][0])
    z = np.zeros_like(x)
    prim = pack_prim(np.full_like(x, 1e5), z, alpha, [z, z])
    return dict(name="square_to_circle_2d", grid=g, eos=baro_eos(),
                scheme=default_scheme(sigma=sigma, switching=1), prim=prim, steps=steps, t_end=0.0,
                storage=dict(p_ref=1e5, T_ref=0.0))


def cube_to_sphere_3d(n=64, steps=2000, L=0.75, side=0.2, sigma=800.0):
    """Section 4.5's 3D shape recovery: a cubic liquid body (rho 1000) of side
    0.2 m centred in a 0.75 m box of gas (rho 1 at 1 bar), sigma = 800 N/m,
    barotropic model with the section's values, zero-gradient sides, at rest."""
    g = make_grid(3, [n, n, n], [L, L, L], [[BC_ZEROGRAD, BC_ZEROGRAD]] * 3)
    x, y, z = cell_centres(g)
    dist = np.maximum(np.maximum(np.abs(x - 0.5 * L), np.abs(y - 0.5 * L)), np.abs(z - 0.5 * L)) - 0.5 * side
    alpha = smeared(dist, g["dx"][0])
    zero = np.zeros_like(x)
    prim = pack_prim(np.full_like(x, 1e5), zero, alpha, [zero, zero, zero])
    return dict(name="cube_to_sphere_3d", grid=g, eos=baro_eos(),
                scheme=default_scheme(sigma=sigma, switching=1), prim=prim, steps=steps, t_end=0.0,
                storage=dict(p_ref=1e5, T_ref=0.0))


def vapour_bubble_wall_2d(nx=1024, ny=512, steps=2000, dx=4e-6, R=400e-6, H=440e-6, p_b=1342.0,
                          p_inf=1e6):
    """Section 4.9's vapour bubble near a wall on a uniform 4 um grid: radius
    400 um, centre 440 um above a slip wall (y = 0), interior a liquid-vapour
    mixture at 1342 Pa (barotropic model, water-like liquid with p_sat = 2340
    Pa), liquid at p_inf = 1 MPa far away with the Rayleigh-collapse profile
    p = p_inf + (p_b - p_inf) R / r in between; the other sides are a far-field
    reservoir at p_inf."""
    g = make_grid(2, [nx, ny], [nx * dx, ny * dx], [[BC_FARFIELD, BC_FARFIELD], [BC_WALL, BC_FARFIELD]])
    g["farfield"] = dict(p=p_inf, T=0.0, alpha=0.0)   # the barotropic model has no temperature
    x, y = cell_centres(g)
    r = np.hypot(x - 0.5 * nx * dx, y - H)
    inside = 1.0 - smeared(r - R, dx)
    p_liq = p_inf + (p_b - p_inf) * np.minimum(1.0, R / np.maximum(r, 1e-300))
    p = p_b * inside + p_liq * (1.0 - inside)
    z = np.zeros_like(x)
    prim = pack_prim(p, z, z, [z, z])
    return dict(name="vapour_bubble_wall_2d", grid=g, eos=baro_eos(), scheme=default_scheme(),
                prim=prim, steps=steps, t_end=0.0, storage=dict(p_ref=p_inf, T_ref=0.0))


def cavitation_tube_1d(n=400, u0=10.0, p0=1e5, L=1.0):
    """1D expansion: water at p0 with u = -u0 left of the middle and +u0 right of
    it between two slip walls; the rarefaction drops the pressure below p_sat
    and a liquid-vapour mixture forms in the middle (barotropic model)."""
    g = make_grid(1, [n], [L], [[BC_WALL, BC_WALL]])
    x = cell_centres(g)[0]
    u = np.where(x < 0.5 * L, -u0, u0)
    z = np.zeros_like(x)
    prim = pack_prim(np.full_like(x, p0), z, z, [u])
    return dict(name="cavitation_tube_1d", grid=g, eos=baro_eos(), scheme=default_scheme(),
                prim=prim, steps=None, t_end=0.0, storage=dict(p_ref=p0, T_ref=0.0))


# ------------------------------------------------------- test-state generators

def random_state(dim, n, seed, L=1e-3, interface=True, liquid=True, velocity=30.0,
                 bc=None, sigma=0.0, switching=0, gas="sg", second_gas=False, barotropic=False):
    """Seeded smooth random fields with a wavy interface: used for one-RHS and
    few-step comparisons.  Periodic by default.  second_gas=True makes a
    three-component case: the gas side is shared between an air-like and a
    helium-like ideal gas by a smooth random split.  barotropic=True makes a
    barotropic-model case whose pressure spans about 0.2 .. 2 p_sat, so
    that liquid, liquid-vapour mixture and gas all occur (with second_gas,
    two gases in the barotropic model)."""
    rng = np.random.default_rng(seed)
    n3 = list(n) + [1] * (3 - len(n))
    if bc is None:
        bc = [[BC_PERIODIC, BC_PERIODIC]] * dim
    g = make_grid(dim, n3[:dim], [L * n3[d] / n3[0] for d in range(dim)], bc)
    xs = cell_centres(g)
    T0, p0 = 300.0, 1e5 if liquid else 1e5
    if liquid:
        c0 = sg(4.4, 6e8, cv_for_density(4.4, 6e8, 1000.0, p0, T0))
    else:
        c0 = sg(1.6, 0.0, 472.22)
    if gas == "pr":
        Mmix = 0.8 * NITROGEN["M"] + 0.2 * METHANE["M"]
        c1 = pr_mixture([NITROGEN, METHANE], [0.8, 0.2], (0.8 * 2.5 + 0.2 * 3.9) * R_UNIV / Mmix)
    else:
        c1 = sg(1.4, 0.0, 717.5)

    def smooth(amp):
        f = np.zeros_like(xs[0])
        for _ in range(3):
            kv = rng.integers(1, 3, size=dim)
            ph = rng.uniform(0, 2 * np.pi, size=dim)
            term = np.ones_like(f)
            for d in range(dim):
                Ld = g["n"][d] * g["dx"][d]
                term = term * np.sin(2 * np.pi * kv[d] * xs[d] / Ld + ph[d])
            f += rng.uniform(-1, 1) * term
        return amp * f / 3.0

    p = p0 * (1.0 + smooth(0.05))
    T = T0 * (1.0 + smooth(0.02))
    u = [velocity * (0.5 + smooth(1.0)) if d == 0 else velocity * smooth(1.0) for d in range(dim)]
    if interface:
        centre = [0.5 * g["n"][d] * g["dx"][d] for d in range(dim)]
        rad = 0.3 * g["n"][0] * g["dx"][0]
        r = np.sqrt(sum((xs[d] - centre[d]) ** 2 for d in range(dim)))
        r = r * (1.0 + 0.1 * smooth(1.0))
        alpha = smeared(r - rad, 1.5 * g["dx"][0])
        alpha = np.clip(alpha + rng.uniform(-1, 1, size=alpha.shape) * 1e-3 * alpha * (1 - alpha), 0, 1)
    else:
        alpha = 0.5 + smooth(0.3)
    if barotropic:
        eos = baro_eos()
        pb = eos["baro"]["p_sat"] * np.maximum(0.2, 1.0 + 1.6 * smooth(1.0))
        # a tenth of the velocity: near p_sat the mixture is soft (c_M ~ 1.5 m/s)
        # and a stronger random compression drives cells across the kink of the
        # law at p_sat within a few steps
        ub = [0.1 * ud for ud in u]
        if second_gas:
            # the gas shared between the model's gas and a helium-like second
            # gas (R 2077.1 J/(kg K) at the same temperature)
            eos = baro_eos(RT2=2077.1 * 336.9)
            share = 0.5 + 0.45 * np.tanh(3.0 * smooth(1.0))
            prim = pack_prim(pb, np.zeros_like(pb), alpha * share, ub + [alpha * (1.0 - share)])
        else:
            prim = pack_prim(pb, np.zeros_like(pb), alpha, ub)
        return dict(name=f"random_baro_{dim}d_{seed}", grid=g, eos=eos,
                    scheme=default_scheme(sigma=sigma, switching=switching), prim=prim, steps=None,
                    t_end=0.0, storage=dict(p_ref=eos["baro"]["p_sat"], T_ref=0.0))
    if second_gas:
        share = 0.5 + 0.45 * np.tanh(3.0 * smooth(1.0))
        prim = pack_prim(p, T, alpha * share, list(u) + [alpha * (1.0 - share)])
        eos = make_eos(c0, c1, sg(1.67, 0.0, 3110.0))
    else:
        prim = pack_prim(p, T, alpha, u)
        eos = make_eos(c0, c1)
    return dict(name=f"random_{dim}d_{seed}", grid=g, eos=eos,
                scheme=default_scheme(sigma=sigma, switching=switching), prim=prim, steps=None,
                t_end=0.0, storage=dict(p_ref=p0, T_ref=T0))
