"""The internal-energy face closure (Appendix B: e* reconstructed where T is
otherwise, rho* = f(p*, xi*, e*); scheme thermal = 1) on the GPU against the
CPU FP64 oracle through the C ABI: one right-hand side and three steps on
every 1D and 2D tile, with walls, zero-gradient and periodic sides, sensor
switching, CSF, stress terms and gravity; the mixed path against the FP64
path; the allocation-free entry point; and the closures and dimensions it
refuses."""
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


def field_errs(a, b):
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return np.abs(a - b).max(axis=1) / scale


def gpu_rhs(ctx, q, dev, step=0):
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    rd = torch.zeros_like(qd)
    torch.cuda.synchronize()
    ctx.rhs(qd.data_ptr(), rd.data_ptr(), step)
    return rd.cpu().numpy()


def viscous(c):
    """the random state's stiffened-gas pair with water- and air-like
    viscosities and conductivities (stress and conduction terms of eq. 2-2)"""
    cv_w = W.cv_for_density(4.4, 6e8, 1000.0, 1e5, 300.0)
    c["eos"] = W.make_eos(W.sg(4.4, 6e8, cv_w, mu=1e-3, kc=0.6), W.sg(1.4, 0.0, 717.5, mu=1.8e-5, kc=0.026))
    return c


def cases():
    c1 = W.random_state(1, [157], 91, switching=1, sigma=0.05, bc=[[W.BC_WALL, W.BC_ZEROGRAD]])
    c2 = W.random_state(2, [45, 37], 92, switching=1, sigma=0.05)
    c3 = W.random_state(2, [41, 29], 93, sigma=0.05, bc=[[W.BC_WALL, W.BC_ZEROGRAD], [W.BC_ZEROGRAD, W.BC_WALL]])
    c3["scheme"]["gravity"] = [30.0, -9.81e3, 0.0]
    c4 = viscous(W.random_state(2, [38, 33], 94, switching=1))
    out = {"1d-walls": c1, "2d-periodic": c2, "2d-walls-gravity": c3, "2d-viscous": c4}
    for c in out.values():
        c["scheme"]["thermal"] = 1
    return out


NAMES = ["1d-walls", "2d-periodic", "2d-walls-gravity", "2d-viscous"]


@pytest.mark.parametrize("name", NAMES)
def test_energy_faces_rhs_and_steps_every_tile(dev, stream, name):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = cases()[name]
    dim = case["grid"]["dim"]
    o = Oracle(case)
    q = o.cons_from_prim()
    r_ref = o.rhs(q)
    qs = q.copy()
    t_ref = 0.0
    for k in range(3):
        t_ref, _ = o.step(qs, k, t_ref)
    # the energy faces change the right-hand side against the temperature faces
    c0 = dict(case, scheme=dict(case["scheme"], thermal=0))
    assert field_errs(Oracle(c0).rhs(q), r_ref).max() > 1e-6
    for tile in range(fvm.lib().fvm_tile_count(dim)):
        ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
        ctx.set_tile(tile)
        err = field_errs(gpu_rhs(ctx, q, dev), r_ref)
        ctx.init_primitive()
        t = ctx.n_steps(3)
        serr = field_errs(ctx.get_state(), qs).max()
        print(f"energy faces {name} tile {tile}: rhs {np.array2string(err, precision=2)}, 3 steps {serr:.2e}",
              flush=True)
        assert np.all(err < 1e-10)
        assert serr < 1e-10 and abs(t / t_ref - 1) < 1e-12
        ctx.close()


def l1(a, b):
    n = a.shape[1]
    return {"rho": np.abs(a[0] - b[0]).sum() / np.abs(b[0]).sum(), "u": np.abs(a[1:4] - b[1:4]).sum() / (n * 30.0),
            "p": np.abs(a[4] - b[4]).sum() / np.abs(b[4]).sum(), "Y": np.abs(a[6] - b[6]).sum() / n}


@pytest.mark.parametrize("name", NAMES[1:])
def test_energy_faces_mixed_against_fp64(dev, stream, name):
    """five steps of the 2D states: the mixed path against the FP64 path per
    field, beside the FP64 path from its own start rounded to FP32.  (The 1D
    random states drive their gas to near vacuum within a few steps, p down
    to 1e-42 Pa, which FP32 storage does not resolve with either thermal
    variable.)"""
    from paper_2304_00140_amd import fvm
    case = cases()[name]
    h = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    m = fvm.Context(case, fvm.FVM_MIXED, stream=stream.cuda_stream)
    g = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    h.init_primitive()
    m.init_primitive()
    g.set_state(h.get_state().astype(np.float32).astype(np.float64))
    for c in (h, m, g):
        c.n_steps(5)
    b = h.get_primitive()
    e, es = l1(m.get_primitive(), b), l1(g.get_primitive(), b)
    print(f"energy faces {name} mixed vs fp64 L1 {e}; fp64 from FP32-rounded start {es}", flush=True)
    for f in e:
        assert e[f] <= max(1e-4, 2.0 * es[f]), f
    for c in (h, m, g):
        c.close()


def test_energy_faces_allocation_free_entry(dev, stream):
    from paper_2304_00140_amd import fvm
    case = cases()["2d-periodic"]
    ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    ctx.init_primitive()
    q = torch.from_numpy(ctx.get_state()).to(dev)
    r1, r2 = torch.zeros_like(q), torch.zeros_like(q)
    torch.cuda.synchronize()
    ctx.rhs(q.data_ptr(), r1.data_ptr(), 0)
    fvm.rhs_noalloc(case, q.data_ptr(), r2.data_ptr(), 0, stream.cuda_stream)
    stream.synchronize()
    assert field_errs(r2.cpu().numpy(), r1.cpu().numpy()).max() < 1e-12
    ctx.close()


def test_energy_faces_refused_where_not_built(dev, stream):
    from paper_2304_00140_amd import fvm
    refused = [W.random_state(3, [9, 8, 7], 95), W.random_state(2, [12, 10], 96, gas="pr"),
               W.random_state(2, [12, 10], 97, second_gas=True), W.random_state(2, [12, 10], 98, barotropic=True)]
    for c in refused:
        c["scheme"]["thermal"] = 1
        with pytest.raises(fvm.FvmError, match="internal-energy"):
            fvm.Context(c, fvm.FVM_FP64, stream=stream.cuda_stream)
    bad = W.random_state(2, [12, 10], 99)
    bad["scheme"]["thermal"] = 2
    with pytest.raises(fvm.FvmError, match="thermal"):
        fvm.Context(bad, fvm.FVM_FP64, stream=stream.cuda_stream)
