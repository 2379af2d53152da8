"""GPU (gfx950) barotropic cavitation model (Section 2.2; liquid-vapour density
THINC of Section 3.4) against the CPU FP64 oracle through the C ABI: one RHS
on every tile in 1D, 2D and 3D (walls, far field, switching, CSF, gravity,
viscous stress with the mixture viscosity of eq. 2-8), primitives, steps, totals, the mixed path against FP64, a moving gas-liquid
interface in equilibrium, a cavitating expansion, the vapour bubble near a
wall and the square-to-circle case, and the rejected configurations."""
import numpy as np
import pytest

from paper_2304_00140_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_00140_amd import fvm
    fvm.lib()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def stream(dev):
    return torch.cuda.Stream(device=dev)


def field_err(a, b):
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return (np.abs(a - b).max(axis=1) / scale).max()


EPS = 2.0 ** -52


def p_noise(case):
    """rounding noise of the barotropic pressure: in the liquid branch
    p = p_sat + c_L^2 (rho_L - rho_sat), so one ulp of density (rho_sat 2^-52)
    is c_L^2 rho_sat 2^-52 of pressure (5e-7 Pa for water), far above 1e-10 of
    a pressure near p_sat; the two sides form rho from partial densities in
    different orders, and the oracle's own right-hand side moves by that much
    when its input density moves by one ulp"""
    b = case["eos"]["baro"]
    return b["c_liq"] ** 2 * b["rho_sat"] * EPS


def rhs_ok(a, b, case, k=16):
    """per field: |a - b| <= 1e-10 of the field's scale, plus for the momentum
    rows k pressure-noise units per face over the cell size"""
    dim = case["grid"]["dim"]
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    extra = np.zeros(b.shape[0])
    extra[1:1 + dim] = k * p_noise(case) / min(case["grid"]["dx"][:dim])
    d = np.abs(a - b).max(axis=1)
    return bool(np.all(d <= 1e-10 * scale + extra)), d / scale


def gpu_rhs(ctx, q, dev):
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    rd = torch.zeros_like(qd)
    torch.cuda.synchronize()
    ctx.rhs(qd.data_ptr(), rd.data_ptr(), 0)
    return rd.cpu().numpy()


SPECS = [
    dict(dim=1, n=[131], seed=61),
    dict(dim=1, n=[77], seed=62, bc=[[W.BC_WALL, W.BC_ZEROGRAD]], sigma=0.05),
    dict(dim=2, n=[45, 37], seed=63),
    dict(dim=2, n=[41, 29], seed=64, switching=1, sigma=0.05,
         bc=[[W.BC_WALL, W.BC_ZEROGRAD], [W.BC_ZEROGRAD, W.BC_WALL]]),
    dict(dim=2, n=[38, 33], seed=65, switching=1, gravity=[3.0, -9.81, 0.0]),
    dict(dim=1, n=[90], seed=66, viscous=True),
    dict(dim=2, n=[40, 35], seed=67, switching=1, sigma=0.05, viscous=True,
         bc=[[W.BC_WALL, W.BC_ZEROGRAD], [W.BC_PERIODIC, W.BC_PERIODIC]]),
]

# viscosities of liquid, gas and vapour (eq. 2-8) large enough that the stress
# part is of the order of the inviscid momentum right-hand side on these grids
VISC = (5e-3, 1e-3, 2e-3)


def viscous(c):
    b = dict(c["eos"]["baro"], mu_vap=VISC[2])
    c["eos"] = dict(c["eos"], mu=[VISC[0], VISC[1]], baro=b)
    return c


def make(spec):
    spec = dict(spec)
    dim, n, seed = spec.pop("dim"), spec.pop("n"), spec.pop("seed")
    grav = spec.pop("gravity", None)
    visc = spec.pop("viscous", False)
    c = W.random_state(dim, n, seed, barotropic=True, **spec)
    if grav is not None:
        c["scheme"] = dict(c["scheme"], gravity=grav)
    return viscous(c) if visc else c


@pytest.mark.parametrize("spec", SPECS, ids=lambda s: f"{s['dim']}d-{s['seed']}")
def test_barotropic_rhs_every_tile(dev, stream, spec):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = make(spec)
    o = Oracle(case)
    q = o.cons_from_prim()
    assert q.shape[0] == case["grid"]["dim"] + 2
    r_ref = o.rhs(q)
    fl = o.sensor_flags(q)
    for tile in range(fvm.lib().fvm_tile_count(case["grid"]["dim"])):
        ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
        ctx.set_tile(tile)
        ok, rel = rhs_ok(gpu_rhs(ctx, q, dev), r_ref, case)
        print(f"barotropic {spec} tile {tile}: {np.array2string(rel, precision=2)} "
              f"(liquid-vapour THINC cells {int(((fl >> 4) & 3).astype(bool).sum())})", flush=True)
        assert ok
        ctx.close()


def test_barotropic_primitives_steps_totals_and_mixed(dev, stream):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = make(dict(dim=2, n=[47, 31], seed=66, sigma=0.05))
    o = Oracle(case)
    q = o.cons_from_prim()
    ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    ctx.init_primitive()
    np.testing.assert_allclose(ctx.get_state(), q, rtol=1e-12, atol=1e-12 * np.abs(q).max())
    w, w_ref = ctx.get_primitive(), o.prim_from_cons(q)
    assert w.shape == w_ref.shape == (12, q.shape[1])
    for f in (0, 1, 2, 6, 7, 8, 11):
        np.testing.assert_allclose(w[f], w_ref[f], rtol=1e-10, atol=1e-12 * max(np.abs(w_ref[f]).max(), 1e-300))
    np.testing.assert_allclose(w[4], w_ref[4], rtol=1e-10, atol=16 * p_noise(case))
    np.testing.assert_allclose(ctx.totals(), o.totals(q), rtol=1e-12)
    t = 0.0
    for k in range(4):
        t, _ = o.step(q, k, t)
    t_gpu = ctx.n_steps(4)
    err = field_err(ctx.get_state(), q)
    print(f"barotropic 4 steps: {err:.3e}", flush=True)
    assert abs(t_gpu / t - 1) < 1e-12
    assert err < 1e-10
    m = fvm.Context(case, fvm.FVM_MIXED, stream=stream.cuda_stream)
    m.init_primitive()
    m.n_steps(4)
    a, b = m.get_primitive(), ctx.get_primitive()
    l1 = {f: np.abs(a[i] - b[i]).sum() / np.abs(b[i]).sum() for f, i in (("rho", 0), ("p", 4))}
    l1["Y"] = np.abs(a[6] - b[6]).sum() / a.shape[1]
    print(f"barotropic mixed vs fp64 L1: {l1}", flush=True)
    assert max(l1.values()) < 1e-4


def test_moving_gas_liquid_interface_keeps_pressure_and_velocity(dev, stream):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    n = 100
    g = W.make_grid(1, [n], [1.0], [[W.BC_PERIODIC, W.BC_PERIODIC]])
    x = W.cell_centres(g)[0]
    alpha = 1.0 - (1.0 - W.smeared(x - 0.7, 0.01)) * W.smeared(x - 0.3, 0.01)
    prim = W.pack_prim(np.full(n, 1e5), np.zeros(n), alpha, [np.full(n, 20.0)])
    case = dict(name="adv_baro", grid=g, eos=W.baro_eos(), scheme=W.default_scheme(), prim=prim,
                steps=None, t_end=0.0, storage=dict(p_ref=1e5, T_ref=0.0))
    ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    ctx.init_primitive()
    ctx.n_steps(200)
    w = ctx.get_primitive()
    assert np.abs(w[4] - 1e5).max() < 1e-12 * 1500.0 ** 2 * 1000.0 * 1e-3
    assert np.abs(w[1] - 20.0).max() < 1e-11 * 20.0
    o = Oracle(case)
    q = o.cons_from_prim()
    o.run(q, 200)
    assert field_err(ctx.get_state(), q) < 1e-10


@pytest.mark.parametrize("name", ["cavitation_tube_1d", "vapour_bubble_wall_2d", "square_to_circle_2d"])
def test_barotropic_workloads_steps(dev, stream, name):
    """the cavitating expansion (liquid-vapour THINC active), the vapour bubble
    near a wall on a coarse grid and Section 4.5's square (sigma = 800) over
    20-40 steps, FP64 against the oracle; mixed within L1 1e-4 of FP64"""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    if name == "cavitation_tube_1d":
        case, steps = W.cavitation_tube_1d(200, 1.0), 40
    elif name == "vapour_bubble_wall_2d":
        case, steps = W.vapour_bubble_wall_2d(128, 64, 20, dx=32e-6), 20
    else:
        case, steps = W.square_to_circle_2d(150, 20), 20
    ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    ctx.init_primitive()
    t_gpu = ctx.n_steps(steps)
    o = Oracle(case)
    q0 = o.cons_from_prim()
    q = q0.copy()
    t = o.run(q, steps)
    # the oracle's own sensitivity: the same run from a start density one ulp
    # higher (the stiff liquid turns that ulp into c_L^2 rho 2^-52 of pressure)
    qs = q0.copy()
    qs[0] *= 1.0 + EPS
    o.run(qs, steps)
    scale = np.maximum(np.abs(q).max(axis=1), 1e-300)
    sens = np.abs(qs - q).max(axis=1) / scale
    rel = np.abs(ctx.get_state() - q).max(axis=1) / scale
    w = o.prim_from_cons(q)
    print(f"{name}: {steps} steps {np.array2string(rel, precision=2)} (oracle one-ulp sensitivity "
          f"{np.array2string(sens, precision=2)}), vapour cells {(w[11] > 0).sum()}, liquid-vapour THINC cells "
          f"{int(((o.sensor_flags(q) >> 4) & 3).astype(bool).sum())}", flush=True)
    assert abs(t_gpu / t - 1) < 1e-12
    assert np.all(rel <= np.maximum(1e-10, 4.0 * sens))
    m = fvm.Context(case, fvm.FVM_MIXED, stream=stream.cuda_stream)
    m.init_primitive()
    m.n_steps(steps)
    a, b = m.get_primitive(), ctx.get_primitive()
    l1 = max(np.abs(a[f] - b[f]).sum() / np.abs(b[f]).sum() for f in (0, 4))
    print(f"{name} mixed vs fp64 L1 rho/p: {l1:.2e}", flush=True)
    assert l1 < 1e-4


SPECS3 = [dict(n=[19, 13, 11], seed=81), dict(n=[17, 14, 12], seed=82, switching=1, sigma=0.05),
          dict(n=[13, 12, 18], seed=83, switching=1, bc=[[W.BC_WALL, W.BC_ZEROGRAD], [W.BC_PERIODIC, W.BC_PERIODIC],
                                                        [W.BC_ZEROGRAD, W.BC_WALL]], gravity=[0.0, 0.0, -9.81]),
          dict(n=[14, 12, 11], seed=85, switching=1, viscous=True)]


@pytest.mark.parametrize("spec", SPECS3, ids=lambda s: f"3d-{s['seed']}")
def test_barotropic_rhs_3d_every_tile(dev, stream, spec):
    """the 3D closure + face kernels of the barotropic model, one RHS on every
    3D tile (periodic, walls, zero gradient, switching, CSF, gravity)"""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    spec = dict(spec)
    n, seed = spec.pop("n"), spec.pop("seed")
    grav = spec.pop("gravity", None)
    visc = spec.pop("viscous", False)
    case = W.random_state(3, n, seed, barotropic=True, **spec)
    if grav is not None:
        case["scheme"] = dict(case["scheme"], gravity=grav)
    if visc:
        case = viscous(case)
    o = Oracle(case)
    q = o.cons_from_prim()
    assert q.shape[0] == 5
    r_ref = o.rhs(q)
    fl = o.sensor_flags(q)
    for tile in range(fvm.lib().fvm_tile_count(3)):
        ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
        try:
            ctx.set_tile(tile)
        except fvm.FvmError as e:
            # the z-marching tiles take the four-equation model only
            assert "z-marching" in str(e)
            ctx.close()
            continue
        ok, rel = rhs_ok(gpu_rhs(ctx, q, dev), r_ref, case)
        print(f"barotropic 3D {n} seed {seed} tile {tile}: {np.array2string(rel, precision=2)} "
              f"(liquid-vapour THINC cells {int(((fl >> 4) & 7).astype(bool).sum())})", flush=True)
        assert ok
        ctx.close()


def test_barotropic_3d_steps_mixed_and_cube_to_sphere(dev, stream):
    """a 3D random barotropic state over 4 steps (FP64 against the oracle,
    mixed within L1 1e-4), and Section 4.5's cube (40^3, sigma = 800) over
    10 steps against the oracle"""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    for case, steps in ((W.random_state(3, [18, 15, 13], 84, barotropic=True, sigma=0.05), 4),
                        (W.cube_to_sphere_3d(40, 10), 10)):
        ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
        ctx.init_primitive()
        t_gpu = ctx.n_steps(steps)
        o = Oracle(case)
        q0 = o.cons_from_prim()
        q = q0.copy()
        t = o.run(q, steps)
        qs = q0.copy()
        qs[0] *= 1.0 + EPS
        o.run(qs, steps)
        scale = np.maximum(np.abs(q).max(axis=1), 1e-300)
        sens = np.abs(qs - q).max(axis=1) / scale
        rel = np.abs(ctx.get_state() - q).max(axis=1) / scale
        print(f"{case['name']} 3D {steps} steps: {np.array2string(rel, precision=2)} "
              f"(oracle one-ulp sensitivity {np.array2string(sens, precision=2)})", flush=True)
        assert abs(t_gpu / t - 1) < 1e-12
        assert np.all(rel <= np.maximum(1e-10, 4.0 * sens))
        m = fvm.Context(case, fvm.FVM_MIXED, stream=stream.cuda_stream)
        m.init_primitive()
        m.n_steps(steps)
        a, b = m.get_primitive(), ctx.get_primitive()
        l1 = max(np.abs(a[f] - b[f]).sum() / np.abs(b[f]).sum() for f in (0, 4))
        print(f"{case['name']} 3D mixed vs fp64 L1 rho/p: {l1:.2e}", flush=True)
        assert l1 < 1e-4


@pytest.mark.parametrize("dim", [2, 3])
def test_barotropic_viscous_steps_and_mixed(dev, stream, dim):
    """the stress terms with the mixture viscosity of eq. 2-8 (liquid, vapour
    and gas cells) over four steps: FP64 against the oracle (the time step
    includes the viscous limit), the mixed path within L1 1e-4 of FP64"""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    n = [36, 30] if dim == 2 else [14, 13, 12]
    case = viscous(W.random_state(dim, n, 70 + dim, barotropic=True, switching=1))
    o = Oracle(case)
    q0 = o.cons_from_prim()
    q = q0.copy()
    t = o.run(q, 4)
    ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    ctx.init_primitive()
    t_gpu = ctx.n_steps(4)
    # the oracle's own sensitivity: the same run from a start density one ulp higher
    qs = q0.copy()
    qs[0] *= 1.0 + EPS
    o.run(qs, 4)
    scale = np.maximum(np.abs(q).max(axis=1), 1e-300)
    sens = np.abs(qs - q).max(axis=1) / scale
    rel = np.abs(ctx.get_state() - q).max(axis=1) / scale
    print(f"barotropic viscous {dim}D 4 steps: {np.array2string(rel, precision=2)} "
          f"(oracle one-ulp sensitivity {np.array2string(sens, precision=2)})", flush=True)
    assert abs(t_gpu / t - 1) < 1e-12
    assert np.all(rel <= np.maximum(1e-10, 4.0 * sens))
    m = fvm.Context(case, fvm.FVM_MIXED, stream=stream.cuda_stream)
    m.init_primitive()
    m.n_steps(4)
    a, b = m.get_primitive(), ctx.get_primitive()
    l1 = max(np.abs(a[f] - b[f]).sum() / np.abs(b[f]).sum() for f in (0, 4))
    print(f"barotropic viscous {dim}D mixed vs fp64 L1 {l1:.2e}", flush=True)
    assert l1 < 1e-4


def test_barotropic_viscous_time_step(dev, stream):
    """a shear wave in the liquid-vapour mixture with gas (uniform p < p_sat,
    alpha_G = 0.3) viscous enough that the diffusive limit 2 mu / rho sum 1/dx^2
    sets the time step: 50 FP64 steps against the oracle, times equal"""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    n, L = 32, 1e-3
    g = W.make_grid(2, [n, 4], [L, L / 8], [[W.BC_PERIODIC] * 2] * 2)
    case = dict(name="bshear", grid=g, eos=W.baro_eos(mu_liq=10.0, mu_gas=2.0, mu_vap=1.0),
                scheme=W.default_scheme(), steps=None, t_end=0.0, storage=dict(p_ref=1e5, T_ref=0.0))
    x, y = W.cell_centres(g)
    p = 0.5 * case["eos"]["baro"]["p_sat"]
    case["prim"] = W.pack_prim(np.full_like(x, p), np.zeros_like(x), np.full_like(x, 0.3),
                               [0 * x, 0.01 * np.sin(2 * np.pi * x / L)])
    o = Oracle(case)
    q = o.cons_from_prim()
    w = o.prim_from_cons(q)
    dx = L / n
    conv = (np.abs(w[1]) + w[7]).max() / dx + (np.abs(w[2]) + w[7]).max() / (L / 8 / 4)
    assert o.dt(q) < 0.9 * case["scheme"]["cfl"] / conv   # the viscous limit is the binding one
    t = o.run(q, 50)
    ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    ctx.init_primitive()
    t_gpu = ctx.n_steps(50)
    err = field_err(ctx.get_state(), q)
    print(f"barotropic viscous shear wave 50 steps: {err:.3e}, t {t_gpu:.6e} vs {t:.6e}", flush=True)
    assert abs(t_gpu / t - 1) < 1e-12
    assert err < 1e-10


def test_barotropic_rejections(dev, stream):
    from paper_2304_00140_amd import fvm
    # no energy equation: no heat conduction; viscosities finite and >= 0
    for key, val in (("kc", [1e-3, 0.0]), ("mu", [-1e-3, 0.0])):
        c2 = W.random_state(2, [16, 16], 68, barotropic=True)
        c2["eos"] = dict(c2["eos"], **{key: val})
        with pytest.raises(fvm.FvmError):
            fvm.Context(c2, fvm.FVM_FP64, stream=stream.cuda_stream)
    c2 = W.random_state(2, [16, 16], 68, barotropic=True)
    c2["eos"] = dict(c2["eos"], baro=dict(c2["eos"]["baro"], mu_vap=float("nan")))
    with pytest.raises(fvm.FvmError):
        fvm.Context(c2, fvm.FVM_FP64, stream=stream.cuda_stream)
    c3 = W.random_state(2, [16, 16], 69, barotropic=True)
    c3["eos"] = dict(c3["eos"], baro=dict(c3["eos"]["baro"], rho_vap=2000.0))
    with pytest.raises(fvm.FvmError):
        fvm.Context(c3, fvm.FVM_FP64, stream=stream.cuda_stream)
    # a far-field reservoir needs a positive pressure (no temperature in the model)
    c4 = W.vapour_bubble_wall_2d(32, 24, 1, dx=40e-6)
    c4["grid"] = dict(c4["grid"], farfield=dict(p=0.0, T=300.0, alpha=0.0))
    with pytest.raises(fvm.FvmError):
        fvm.Context(c4, fvm.FVM_FP64, stream=stream.cuda_stream)


def test_vapour_bubble_full_size_in_the_benchmark_launch(dev, stream):
    """the benchmark's 1024 x 512 vapour bubble near a wall with the tile the
    benchmark uses, 10 FP64 steps against the oracle (same tolerance as
    above), and the mixed path within L1 1e-4 of FP64"""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm, tune
    case = W.vapour_bubble_wall_2d(1024, 512, 10)
    h = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    h.init_primitive()
    tile, _ = tune.autotune(h, fvm.FVM_FP64)
    h.init_primitive()
    t_gpu = h.n_steps(10)
    o = Oracle(case)
    q0 = o.cons_from_prim()
    q = q0.copy()
    t = o.run(q, 10)
    qs = q0.copy()
    qs[0] *= 1.0 + EPS
    o.run(qs, 10)
    scale = np.maximum(np.abs(q).max(axis=1), 1e-300)
    sens = np.abs(qs - q).max(axis=1) / scale
    rel = np.abs(h.get_state() - q).max(axis=1) / scale
    print(f"vapour bubble 1024 x 512, tile {tile}, 10 steps: {np.array2string(rel, precision=2)} "
          f"(oracle one-ulp sensitivity {np.array2string(sens, precision=2)})", flush=True)
    assert abs(t_gpu / t - 1) < 1e-12
    assert np.all(rel <= np.maximum(1e-10, 4.0 * sens))
    m = fvm.Context(case, fvm.FVM_MIXED, stream=stream.cuda_stream)
    m.init_primitive()
    mtile, _ = tune.autotune(m, fvm.FVM_MIXED)
    m.init_primitive()
    m.n_steps(10)
    a, b = m.get_primitive(), h.get_primitive()
    l1 = max(np.abs(a[f] - b[f]).sum() / np.abs(b[f]).sum() for f in (0, 4))
    print(f"vapour bubble mixed (tile {mtile}) vs fp64 L1 rho/p: {l1:.2e}", flush=True)
    assert l1 < 1e-4
