"""GPU (gfx950) viscous stress, heat conduction and gravity (eq. 2-2) against
the CPU FP64 oracle, through the C ABI: the stress part alone (RHS with minus
RHS without the transport coefficients, on both sides), whole RHS, steps, and
the mixed path against FP64."""
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


def gpu_rhs(case, q, dev, stream, tile, prec=None):
    from paper_2304_00140_amd import fvm
    ctx = fvm.Context(case, fvm.FVM_FP64 if prec is None else prec, stream=stream.cuda_stream)
    ctx.set_tile(tile)
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    rd = torch.zeros_like(qd)
    torch.cuda.synchronize()
    ctx.rhs(qd.data_ptr(), rd.data_ptr(), 0)
    out = rd.cpu().numpy()
    ctx.close()
    return out


def viscous(case, mu=(4.0, 0.5), kc=(600.0, 30.0), gravity=(0.0, 0.0, 0.0)):
    """the case with (strong) transport coefficients, so that the stress terms
    are of the size of the convective ones on these small grids"""
    c = dict(case)
    c["eos"] = dict(case["eos"], mu=list(mu), kc=list(kc))
    c["scheme"] = dict(case["scheme"], gravity=list(gravity))
    return c


def inviscid(case):
    return viscous(case, (0.0, 0.0), (0.0, 0.0))


SPECS = [
    dict(dim=1, n=[97], seed=11),
    dict(dim=2, n=[45, 37], seed=12, switching=1),
    dict(dim=2, n=[41, 29], seed=13, sigma=0.05, bc=[[W.BC_WALL, W.BC_ZEROGRAD], [W.BC_ZEROGRAD, W.BC_WALL]]),
    dict(dim=3, n=[14, 11, 9], seed=14, switching=1),
    dict(dim=3, n=[12, 10, 9], seed=15, gas="pr", velocity=10.0,
         bc=[[W.BC_WALL, W.BC_ZEROGRAD], [W.BC_PERIODIC, W.BC_PERIODIC], [W.BC_ZEROGRAD, W.BC_WALL]]),
]


def make(spec):
    spec = dict(spec)
    dim, n, seed = spec.pop("dim"), spec.pop("n"), spec.pop("seed")
    return W.random_state(dim, n, seed, **spec)


@pytest.mark.parametrize("spec", SPECS, ids=lambda s: f"{s['dim']}d-{s['seed']}")
def test_stress_terms_match_oracle_every_tile(dev, stream, spec):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    base = make(spec)
    dim = base["grid"]["dim"]
    g = [30.0, -9.81e3, 5e3][:dim] + [0.0] * (3 - dim)
    cv, ci = viscous(base, gravity=g), inviscid(base)
    o = Oracle(cv)
    q = o.cons_from_prim()
    rv, ri = o.rhs(q), Oracle(ci).rhs(q)
    dref = rv - ri
    assert np.abs(dref[1:1 + dim]).max() > 1e-3 * np.abs(rv[1:1 + dim]).max()   # the terms matter
    for tile in range(fvm.lib().fvm_tile_count(dim)):
        try:
            gv = gpu_rhs(cv, q, dev, stream, tile)
        except fvm.FvmError as e:
            # the z-marching 3D tiles take inviscid cases only
            assert dim == 3 and "z-marching" in str(e)
            continue
        gi = gpu_rhs(ci, q, dev, stream, tile)
        e_all = field_err(gv, rv)
        e_diff = field_err((gv - gi)[1:2 + dim], dref[1:2 + dim])
        print(f"viscous {spec} tile {tile}: rhs {e_all:.3e} stress part {e_diff:.3e}", flush=True)
        assert e_all < 1e-10
        assert e_diff < 1e-9


@pytest.mark.parametrize("dim", [2, 3])
def test_viscous_steps_match_oracle(dev, stream, dim):
    """FP64 steps with stress terms, gravity and the diffusive time-step bound"""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    n = [33, 27] if dim == 2 else [13, 11, 10]
    base = W.random_state(dim, n, 40 + dim, sigma=0.05, switching=1)
    case = viscous(base, mu=(0.3, 0.05), kc=(60.0, 3.0), gravity=[0.0, -9.81e4, 0.0])
    o = Oracle(case)
    q = o.cons_from_prim()
    ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    ctx.set_state(q)
    dt_ref = o.dt(q)
    t = 0.0
    for k in range(5):
        t, _ = o.step(q, k, t)
    t_gpu = ctx.n_steps(5)
    err = field_err(ctx.get_state(), q)
    print(f"viscous {dim}d 5 steps: {err:.3e}, dt0 {dt_ref:.4e}, t {t:.6e} / {t_gpu:.6e}", flush=True)
    assert abs(t_gpu / t - 1) < 1e-12
    assert err < 1e-10
    # the mixed path stays within the stated L1 of the FP64 path
    m = fvm.Context(case, fvm.FVM_MIXED, stream=stream.cuda_stream)
    m.set_state(o.cons_from_prim())
    m.n_steps(5)
    a, b = m.get_primitive(), ctx.get_primitive()
    l1p = np.abs(a[4] - b[4]).sum() / np.abs(b[4]).sum()
    l1r = np.abs(a[0] - b[0]).sum() / np.abs(b[0]).sum()
    print(f"viscous {dim}d mixed vs fp64 L1 p {l1p:.2e} rho {l1r:.2e}", flush=True)
    assert l1p < 1e-4 and l1r < 1e-4


def test_free_fall_on_the_gpu(dev, stream):
    """uniform state in a periodic box under gravity: v = g t to rounding"""
    from paper_2304_00140_amd import fvm
    case = W.random_state(2, [40, 24], 3)
    x, y = W.cell_centres(case["grid"])
    case["prim"] = W.pack_prim(np.full_like(x, 1e5), np.full_like(x, 300.0), np.full_like(x, 0.2),
                               [0 * x, 0 * x])
    case["scheme"] = dict(case["scheme"], gravity=[0.0, -9.81e3, 0.0])
    ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    ctx.init_primitive()
    t = ctx.n_steps(60)
    w = ctx.get_primitive()
    np.testing.assert_allclose(w[2], -9.81e3 * t, rtol=1e-11)
    assert np.abs(w[1]).max() < 1e-12 * 9.81e3 * t
