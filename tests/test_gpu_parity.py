"""GPU (gfx950) path against the CPU FP64 oracle, through the C ABI.

FP64 path: element-wise agreement to 1e-10 relative to each field's largest
magnitude.  Mixed path (FP32 storage/fluxes, FP64 closure): 1e-4 relative
L1 per field.  Sizes span several tiles with ragged tails."""
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


def ctx_for(case, prec, stream, tile=None):
    from paper_2304_00140_amd import fvm
    c = fvm.Context(case, prec, stream=stream.cuda_stream)
    if tile is not None:
        c.set_tile(tile)
    return c


def field_err(a, b):
    """max |a - b| per field over max |b| per field"""
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return (np.abs(a - b).max(axis=1) / scale).max()


def field_errs(a, b):
    """max |a - b| per field over max |b| per field, one value per field"""
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return np.abs(a - b).max(axis=1) / scale


def gpu_rhs(ctx, q, dev, step=0):
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    rd = torch.zeros_like(qd)
    torch.cuda.synchronize()
    ctx.rhs(qd.data_ptr(), rd.data_ptr(), step)
    return rd.cpu().numpy()


RHS_CASES = [
    dict(dim=1, n=[203], seed=1),
    dict(dim=1, n=[77], seed=2, bc=[[W.BC_WALL, W.BC_ZEROGRAD]], sigma=0.05),
    dict(dim=2, n=[70, 37], seed=3),
    dict(dim=2, n=[70, 37], seed=4, switching=1),
    dict(dim=2, n=[45, 52], seed=5, sigma=0.07),
    dict(dim=2, n=[45, 52], seed=6, sigma=0.07, switching=1,
         bc=[[W.BC_WALL, W.BC_ZEROGRAD], [W.BC_ZEROGRAD, W.BC_WALL]]),
    dict(dim=2, n=[33, 9], seed=7, liquid=False),
]


def make_case(spec):
    spec = dict(spec)
    dim, n, seed = spec.pop("dim"), spec.pop("n"), spec.pop("seed")
    return W.random_state(dim, n, seed, **spec)


@pytest.mark.parametrize("spec", RHS_CASES, ids=lambda s: f"{s['dim']}d-{s['seed']}")
def test_rhs_fp64_matches_oracle(dev, stream, spec):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = make_case(spec)
    o = Oracle(case)
    q = o.cons_from_prim()
    r_ref = o.rhs(q)
    for tile in range(fvm.lib().fvm_tile_count(case["grid"]["dim"])):
        ctx = ctx_for(case, fvm.FVM_FP64, stream, tile)
        r = gpu_rhs(ctx, q, dev)
        err = field_err(r, r_ref)
        print(f"rhs {spec} tile {tile}: {err:.3e}", flush=True)
        assert err < 1e-10


def test_rhs_inflow_noise_matches_oracle(dev, stream):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = W.random_state(2, [40, 30], 9, bc=[[W.BC_INFLOW, W.BC_ZEROGRAD], [W.BC_WALL, W.BC_PERIODIC]])
    case["grid"]["bc"][1] = [W.BC_PERIODIC, W.BC_PERIODIC]
    case["grid"]["inflow"] = dict(p=1.05e5, T=300.0, alpha=0.0, u=40.0, radius=0.3 * 40 * case["grid"]["dx"][0],
                                  center=[0.5 * 30 * case["grid"]["dx"][1], 0.0], noise=0.05, seed=11)
    o = Oracle(case)
    q = o.cons_from_prim()
    ctx = ctx_for(case, fvm.FVM_FP64, stream)
    for step in (0, 3):
        assert field_err(gpu_rhs(ctx, q, dev, step), o.rhs(q, step)) < 1e-10


def test_rhs_farfield_matches_oracle(dev, stream):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = W.random_state(2, [37, 29], 19, bc=[[W.BC_FARFIELD, W.BC_ZEROGRAD], [W.BC_WALL, W.BC_FARFIELD]])
    case["grid"]["farfield"] = dict(p=1.3e5, T=305.0, alpha=0.0)
    o = Oracle(case)
    q = o.cons_from_prim()
    for prec_tile in range(fvm.lib().fvm_tile_count(2)):
        ctx = ctx_for(case, fvm.FVM_FP64, stream, prec_tile)
        assert field_err(gpu_rhs(ctx, q, dev), o.rhs(q)) < 1e-10
    case3 = W.random_state(3, [11, 9, 10], 20, bc=[[W.BC_FARFIELD, W.BC_ZEROGRAD], [W.BC_WALL, W.BC_FARFIELD],
                                                   [W.BC_PERIODIC, W.BC_PERIODIC]])
    case3["grid"]["farfield"] = dict(p=1.3e5, T=305.0, alpha=0.0)
    o3 = Oracle(case3)
    q3 = o3.cons_from_prim()
    ctx = ctx_for(case3, fvm.FVM_FP64, stream)
    assert field_err(gpu_rhs(ctx, q3, dev), o3.rhs(q3)) < 1e-10


def test_primitives_match_oracle(dev, stream):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = W.random_state(2, [37, 21], 12)
    o = Oracle(case)
    q = o.cons_from_prim()
    ctx = ctx_for(case, fvm.FVM_FP64, stream)
    ctx.set_state(q)
    w = ctx.get_primitive()
    w_ref = o.prim_from_cons(q)
    np.testing.assert_allclose(w[4], w_ref[4], rtol=1e-12, atol=1e-12 * 6e8)
    np.testing.assert_allclose(w[5], w_ref[5], rtol=1e-12)
    np.testing.assert_allclose(w[[0, 6, 7, 8]], w_ref[[0, 6, 7, 8]], rtol=1e-12, atol=1e-14)
    # init from primitives on the device equals the oracle's conversion
    ctx.init_primitive()
    np.testing.assert_allclose(ctx.get_state(), q, rtol=1e-13, atol=1e-13 * np.abs(q).max())


@pytest.mark.parametrize("spec", [RHS_CASES[0], RHS_CASES[3], RHS_CASES[5]],
                         ids=lambda s: f"{s['dim']}d-{s['seed']}")
def test_steps_fp64_match_oracle(dev, stream, spec):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = make_case(spec)
    o = Oracle(case)
    q = o.cons_from_prim()
    ctx = ctx_for(case, fvm.FVM_FP64, stream)
    ctx.set_state(q)
    t_ref = 0.0
    for k in range(5):
        t_ref, _ = o.step(q, k, t_ref)
    t = ctx.n_steps(5)
    assert abs(t - t_ref) < 1e-12 * t_ref
    err = field_err(ctx.get_state(), q)
    print(f"5 steps {spec}: {err:.3e}", flush=True)
    assert err < 1e-10


def test_interface_advection_period_fp64(dev, stream):
    """one advection period of the stiff water slab (FP64): the kernel keeps p
    and u at their initial values and matches the oracle's interface"""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = W.interface_advection_1d(200, periods=1.0)
    ctx = ctx_for(case, fvm.FVM_FP64, stream)
    ctx.init_primitive()
    t_end = case["t_end"]
    t = ctx.n_steps(7000, t_end)
    assert abs(t - t_end) < 1e-15
    w = ctx.get_primitive()
    assert np.abs(w[4] - 1e5).max() / (1e5 + 6e8) < 1e-12
    assert np.abs(w[1] - 100.0).max() / 100.0 < 1e-11
    o = Oracle(case)
    q = o.cons_from_prim()
    tt, n = 0.0, 0
    while tt < t_end * (1 - 1e-14):
        tt, _ = o.step(q, n, tt, t_end)
        n += 1
    w_ref = o.prim_from_cons(q)
    assert np.abs(w[6] - w_ref[6]).max() < 1e-9


def test_conservation_fp64_and_mixed(dev, stream):
    from paper_2304_00140_amd import fvm
    case = W.random_state(2, [64, 48], 21)
    for prec, tol in ((fvm.FVM_FP64, 1e-13), (fvm.FVM_MIXED, 1e-6)):
        ctx = ctx_for(case, prec, stream)
        ctx.init_primitive()
        t0 = ctx.totals()
        ctx.n_steps(60)
        t1 = ctx.totals()
        rel = np.abs(t1 - t0) / np.maximum(np.abs(t0), 1e-30)
        print("conservation", prec, rel, flush=True)
        assert rel[0] < tol and rel[-1] < tol and rel[-2] < tol


def test_tile_shapes_bitwise_identical_and_deterministic(dev, stream):
    from paper_2304_00140_amd import fvm
    case = W.random_state(2, [70, 37], 31, sigma=0.05, switching=1,
                          bc=[[W.BC_WALL, W.BC_ZEROGRAD], [W.BC_PERIODIC, W.BC_PERIODIC]])
    for prec in (fvm.FVM_FP64, fvm.FVM_MIXED):
        outs = []
        for tile in list(range(fvm.lib().fvm_tile_count(2))) + [0]:
            ctx = ctx_for(case, prec, stream, tile)
            ctx.init_primitive()
            ctx.n_steps(7)
            outs.append(ctx.get_state())
        for o in outs[1:]:
            np.testing.assert_array_equal(o, outs[0])


def test_graph_replay_equals_single_steps(dev, stream):
    from paper_2304_00140_amd import fvm
    case = W.random_state(2, [40, 36], 41)
    a = ctx_for(case, fvm.FVM_MIXED, stream)
    a.init_primitive()
    a.n_steps(120)          # 2 graph replays of 50 steps + 20 single launches
    b = ctx_for(case, fvm.FVM_MIXED, stream)
    b.init_primitive()
    for _ in range(120):
        b.step()
    np.testing.assert_array_equal(a.get_state(), b.get_state())
    assert a.clock() == b.clock()


def test_batch_equals_single_cases(dev, stream):
    from paper_2304_00140_amd import fvm
    cases = fvm_cases = W.bubble_collapse_batch(ncases=3, nmin=20, nmax=50, steps=5)
    b = fvm.Batch(cases, fvm.FVM_MIXED, stream=stream.cuda_stream)
    for i in range(len(cases)):
        b.init_primitive(i)
    b.n_steps(6)
    for i, c in enumerate(fvm_cases):
        s = ctx_for(c, fvm.FVM_MIXED, stream)
        s.init_primitive()
        s.n_steps(6)
        np.testing.assert_array_equal(b.get_state(i), s.get_state())


def test_mixed_precision_against_fp64(dev, stream):
    """mixed path vs FP64 path after 100 steps of a small shock-bubble case:
    relative L1 per field (rho, u, p, xi) below 1e-4"""
    from paper_2304_00140_amd import fvm
    case = W.shock_bubble_2d(nx=128, ny=32, steps=100)
    res = {}
    for prec in (fvm.FVM_FP64, fvm.FVM_MIXED):
        ctx = ctx_for(case, prec, stream)
        ctx.init_primitive()
        ctx.n_steps(100)
        res[prec] = ctx.get_primitive()
    a, b = res[fvm.FVM_MIXED], res[fvm.FVM_FP64]
    l1 = {
        "rho": np.abs(a[0] - b[0]).sum() / np.abs(b[0]).sum(),
        "u": np.abs(a[1:3] - b[1:3]).sum() / (a.shape[1] * 113.5),
        "p": np.abs(a[4] - b[4]).sum() / np.abs(b[4]).sum(),
        "Y": np.abs(a[6] - b[6]).sum() / a.shape[1],
    }
    print("mixed vs fp64 L1", l1, flush=True)
    assert max(l1.values()) < 1e-4


def test_nonphysical_state_is_reported(dev, stream):
    from paper_2304_00140_amd import fvm
    from oracle.oracle import Oracle
    case = W.random_state(2, [20, 20], 51)
    q = Oracle(case).cons_from_prim()
    q[0, 37] = -1.0
    ctx = ctx_for(case, fvm.FVM_FP64, stream)
    with pytest.raises(fvm.FvmError) as ei:
        ctx.set_state(q)
    assert ei.value.code in (fvm.FVM_ENONPHYS, fvm.FVM_ENAN)
    with pytest.raises(fvm.FvmError):
        ctx.n_steps(1)


RHS3_CASES = [
    dict(dim=3, n=[19, 14, 11], seed=61),
    dict(dim=3, n=[13, 17, 9], seed=62, switching=1, sigma=0.05),
    dict(dim=3, n=[12, 10, 10], seed=63, sigma=0.07, bc=[[W.BC_WALL, W.BC_ZEROGRAD], [W.BC_ZEROGRAD, W.BC_WALL],
                                                        [W.BC_PERIODIC, W.BC_PERIODIC]]),
]


@pytest.mark.parametrize("spec", RHS3_CASES, ids=lambda s: f"3d-{s['seed']}")
def test_rhs3d_fp64_matches_oracle(dev, stream, spec):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = make_case(spec)
    o = Oracle(case)
    q = o.cons_from_prim()
    r_ref = o.rhs(q)
    for tile in range(fvm.lib().fvm_tile_count(3)):
        ctx = ctx_for(case, fvm.FVM_FP64, stream, tile)
        err = field_err(gpu_rhs(ctx, q, dev), r_ref)
        print(f"rhs3d {spec} tile {tile}: {err:.3e}", flush=True)
        assert err < 1e-10


@pytest.mark.parametrize("dim", [2, 3])
def test_peng_robinson_gas_matches_oracle(dev, stream, dim):
    """stiffened liquid + Peng-Robinson N2/CH4 gas: closure, one RHS and three steps"""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    n = [33, 21] if dim == 2 else [14, 11, 9]
    case = W.random_state(dim, n, 70 + dim, gas="pr", velocity=10.0)
    o = Oracle(case)
    q = o.cons_from_prim()
    ctx = ctx_for(case, fvm.FVM_FP64, stream)
    ctx.set_state(q)
    w, w_ref = ctx.get_primitive(), o.prim_from_cons(q)
    np.testing.assert_allclose(w[4], w_ref[4], rtol=1e-10, atol=1e-10 * 1e5)
    np.testing.assert_allclose(w[5], w_ref[5], rtol=1e-10)
    print(f"PR {dim}d sound speed: {np.abs(w[7] / w_ref[7] - 1).max():.3e}", flush=True)
    np.testing.assert_allclose(w[7], w_ref[7], rtol=1e-9)
    r_ref = o.rhs(q)
    err = field_errs(gpu_rhs(ctx, q, dev), r_ref)
    # the bar per field: 1e-10, or four times the oracle's own change under a
    # one-ulp perturbation of its input where that is larger (the stiff
    # liquid's pressure, and with it the momentum rows, is fixed only to
    # rounding of p + p_inf ~ 6e8 Pa)
    sens = ulp_sensitivity(o, q, r_ref)
    print(f"PR {dim}d rhs: {err} one-ulp sensitivity {sens}", flush=True)
    assert np.all(err < np.maximum(1e-10, 4.0 * sens))
    t = 0.0
    for k in range(3):
        t, _ = o.step(q, k, t)
    ctx.n_steps(3)
    err = field_err(ctx.get_state(), q)
    print(f"PR {dim}d 3 steps: {err:.3e}", flush=True)
    assert err < 1e-10


def test_liquid_jet_small_fp64_and_mixed(dev, stream):
    """3D jet with inflow noise, Peng-Robinson gas, CSF and sensor switching, at
    a small size: FP64 GPU steps against the oracle, mixed against FP64"""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = W.liquid_jet_3d(nx=40, ny=20, nz=20, cells_per_D=8, steps=3)
    o = Oracle(case)
    q = o.cons_from_prim()
    ctx = ctx_for(case, fvm.FVM_FP64, stream)
    ctx.init_primitive()
    np.testing.assert_allclose(ctx.get_state(), q, rtol=1e-12, atol=1e-12 * np.abs(q).max())
    err = field_err(gpu_rhs(ctx, q, dev, 0), o.rhs(q, 0))
    print(f"jet rhs: {err:.3e}", flush=True)
    assert err < 1e-10
    t = 0.0
    for k in range(3):
        t, _ = o.step(q, k, t)
    ctx.n_steps(3)
    err = field_err(ctx.get_state(), q)
    print(f"jet 3 steps fp64: {err:.3e}", flush=True)
    assert err < 1e-10
    m = ctx_for(case, fvm.FVM_MIXED, stream)
    m.init_primitive()
    m.n_steps(3)
    a, b = m.get_primitive(), ctx.get_primitive()
    l1p = np.abs(a[4] - b[4]).sum() / np.abs(b[4]).sum()
    l1u = np.abs(a[1:4] - b[1:4]).sum() / (a.shape[1] * 300.0)
    print(f"jet mixed vs fp64 L1 p {l1p:.2e} u {l1u:.2e}", flush=True)
    assert l1p < 1e-4 and l1u < 1e-4


@pytest.mark.parametrize("gas,dim", [("sg", 2), ("pr", 3)])
def test_mass_fraction_outside_unit_interval(dev, stream, gas, dim):
    """cells whose mass fraction sits a little below 0 or above 1 (what an
    unbounded central reconstruction leaves behind) close as the nearer pure
    component on both sides: primitives and one RHS"""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    n = [37, 29] if dim == 2 else [15, 12, 10]
    case = W.random_state(dim, n, 90 + dim, gas=gas, velocity=10.0, switching=1, sigma=0.05)
    al = case["prim"][2]
    lo, hi = al < 0.05, al > 0.95
    assert lo.any() and hi.any()
    al[lo], al[hi] = 0.0, 1.0              # pure cells, then nudged just outside [0, 1]
    o = Oracle(case)
    q = o.cons_from_prim()
    q[2 + dim, lo] = -1e-8 * q[0, lo]
    q[2 + dim, hi] = (1.0 + 1e-9) * q[0, hi]
    ctx = ctx_for(case, fvm.FVM_FP64, stream)
    ctx.set_state(q)
    w, w_ref = ctx.get_primitive(), o.prim_from_cons(q)
    for f in (4, 5, 7, 8):
        np.testing.assert_allclose(w[f], w_ref[f], rtol=1e-10, atol=1e-10 * np.abs(w_ref[f]).max())
    err = field_err(gpu_rhs(ctx, q, dev), o.rhs(q))
    print(f"outside [0, 1] {gas} {dim}d rhs: {err:.3e}", flush=True)
    assert err < 1e-10


def test_liquid_jet_nozzle_lip_fp64(dev, stream):
    """jet at its full resolution (32 cells across) through the first 60 steps,
    where the flow round the nozzle lip drives the mass fraction below zero and
    the pressure there down: FP64 GPU steps against the oracle"""
    from oracle.oracle import Oracle
    case = W.liquid_jet_3d(nx=40, ny=40, nz=40, steps=60)
    from paper_2304_00140_amd import fvm
    o = Oracle(case)
    q = o.cons_from_prim()
    ctx = ctx_for(case, fvm.FVM_FP64, stream)
    ctx.init_primitive()
    t = 0.0
    done = 0
    for chunk in (10, 30, 60):
        for k in range(done, chunk):
            t, _ = o.step(q, k, t)
        ctx.n_steps(chunk - done)
        done = chunk
        err = field_err(ctx.get_state(), q)
        print(f"jet lip {done} steps: {err:.3e}", flush=True)
        assert err < 1e-10
    assert (q[5] / q[0]).min() < 0.0


MINIMAL = [(1, [2]), (2, [2, 2]), (2, [2, 3]), (3, [2, 2, 2]), (3, [3, 2, 2])]


def ulp_sensitivity(o, q, r, trials=8):
    """per field: the largest change of the oracle's own RHS when every input
    word moves by one ulp in a random direction, over the field's largest
    |RHS| (how far rounding alone moves a right-hand side that is a small
    difference of large fluxes)"""
    rng = np.random.default_rng(0)
    scale = np.maximum(np.abs(r).max(axis=1), 1e-300)
    worst = np.zeros(q.shape[0])
    for _ in range(trials):
        rp = o.rhs(q * (1.0 + rng.choice([-1.0, 1.0], size=q.shape) * 2.0 ** -52))
        worst = np.maximum(worst, np.abs(rp - r).max(axis=1) / scale)
    return worst


@pytest.mark.parametrize("dim,n", MINIMAL, ids=lambda v: str(v))
def test_minimal_grids_match_oracle(dev, stream, dim, n):
    """the smallest grids the ABI accepts (two cells in a direction: the
    two-cell halo on either side reaches across the whole domain) with
    periodic, wall and zero-gradient ends, CSF and switching on: one RHS on
    every tile and three steps against the oracle, the mixed path finite.
    With two periodic cells the two faces of a cell see the same pair of cells
    in mirrored order, so a right-hand side can be a difference of nearly equal
    fluxes; per field the bar is then 1e-10 or 16 times the oracle's own
    one-ulp input sensitivity of that field, whichever is larger."""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    for bc in (W.BC_PERIODIC, W.BC_WALL, W.BC_ZEROGRAD):
        case = W.random_state(dim, n, 5, bc=[[bc, bc]] * dim, sigma=0.05, switching=1)
        o = Oracle(case)
        q = o.cons_from_prim()
        r_ref = o.rhs(q)
        bar = np.maximum(1e-10, 16.0 * ulp_sensitivity(o, q, r_ref))
        scale = np.maximum(np.abs(r_ref).max(axis=1), 1e-300)
        for tile in range(fvm.lib().fvm_tile_count(dim)):
            ctx = ctx_for(case, fvm.FVM_FP64, stream, tile)
            err = np.abs(gpu_rhs(ctx, q, dev) - r_ref).max(axis=1) / scale
            print(f"minimal grid {dim}D {n} bc {bc} tile {tile}: rhs {np.array2string(err, precision=1)} "
                  f"bar {np.array2string(bar, precision=1)}", flush=True)
            assert np.all(err <= bar), (bc, tile)
            ctx.close()
        ctx = ctx_for(case, fvm.FVM_FP64, stream)
        ctx.init_primitive()
        t = 0.0
        for k in range(3):
            t, _ = o.step(q, k, t)
        t_gpu = ctx.n_steps(3)
        err = field_err(ctx.get_state(), q)
        print(f"minimal grid {dim}D {n} bc {bc}: 3 steps {err:.2e}", flush=True)
        assert err < 1e-10 and abs(t_gpu / t - 1) < 1e-12
        m = ctx_for(case, fvm.FVM_MIXED, stream)
        m.init_primitive()
        m.n_steps(3)
        assert np.isfinite(m.get_state()).all()
        m.close()
        ctx.close()


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_grids_below_two_cells_are_rejected(dev, stream, dim):
    from paper_2304_00140_amd import fvm
    for bad in (1, 0, -3):
        case = W.random_state(dim, [4] * dim, 6)
        case["grid"] = dict(case["grid"], n=[bad] + [4] * (dim - 1) + [1] * (3 - dim))
        with pytest.raises(fvm.FvmError) as e:
            fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
        assert "EINVAL" in str(e.value)
