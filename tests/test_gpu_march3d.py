"""The z-marching 3D stage kernel against the CPU FP64 oracle through the C
ABI: one right-hand side and a few steps on every z-marching tile, with z
extents that span several plane chunks and ragged x-y tiles, for the
stiffened-gas pair and the Peng-Robinson gas, with walls, zero-gradient,
far-field and noisy inflow ghosts, sensor switching, CSF and gravity; the
mixed path against the FP64 path."""
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


def march_tiles():
    """3D tile indices of the z-marching kernel: those a barotropic case
    refuses as z-marching tiles"""
    from paper_2304_00140_amd import fvm
    ctx = fvm.Context(W.random_state(3, [9, 8, 7], 86, barotropic=True), fvm.FVM_FP64)
    tiles = []
    for tile in range(fvm.lib().fvm_tile_count(3)):
        try:
            ctx.set_tile(tile)
        except fvm.FvmError as e:
            if "z-marching" in str(e):
                tiles.append(tile)
    ctx.close()
    assert len(tiles) == 10
    return tiles


def field_err(a, b):
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return np.abs(a - b).max(axis=1) / scale


def gpu_rhs(ctx, q, dev, step=0):
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    rd = torch.zeros_like(qd)
    torch.cuda.synchronize()
    ctx.rhs(qd.data_ptr(), rd.data_ptr(), step)
    return rd.cpu().numpy()


def ulp_sensitivity(o, q, r, trials=4):
    """the oracle's own per-field RHS change under a one-ulp change of every
    input word (seeded random signs), over the field's largest |RHS|"""
    rng = np.random.default_rng(0)
    scale = np.maximum(np.abs(r).max(axis=1), 1e-300)
    worst = np.zeros(q.shape[0])
    for _ in range(trials):
        rp = o.rhs(q * (1.0 + rng.choice([-1.0, 1.0], size=q.shape) * 2.0 ** -52))
        worst = np.maximum(worst, np.abs(rp - r).max(axis=1) / scale)
    return worst


def cases():
    c1 = W.random_state(3, [37, 19, 70], 81, switching=1, sigma=0.05)
    c2 = W.random_state(3, [21, 26, 45], 82, sigma=0.07,
                        bc=[[W.BC_WALL, W.BC_ZEROGRAD], [W.BC_ZEROGRAD, W.BC_WALL], [W.BC_WALL, W.BC_ZEROGRAD]])
    c2["scheme"]["gravity"] = [30.0, -9.81e3, 5e3]
    c3 = W.random_state(3, [18, 17, 40], 83, switching=1, sigma=0.05,
                        bc=[[W.BC_FARFIELD, W.BC_ZEROGRAD], [W.BC_PERIODIC, W.BC_PERIODIC],
                            [W.BC_ZEROGRAD, W.BC_FARFIELD]])
    c3["grid"]["farfield"] = dict(p=1.3e5, T=305.0, alpha=0.0)
    c4 = W.random_state(3, [23, 15, 38], 84, gas="pr", velocity=10.0, switching=1, sigma=0.05)
    c5 = W.liquid_jet_3d(nx=40, ny=20, nz=36, cells_per_D=8, steps=3)
    return {"sg-periodic": c1, "sg-walls-gravity": c2, "sg-farfield": c3, "pr": c4, "jet": c5}


CASE_NAMES = ["sg-periodic", "sg-walls-gravity", "sg-farfield", "pr", "jet"]


@pytest.mark.parametrize("name", CASE_NAMES)
def test_march_rhs_every_tile(dev, stream, name):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = cases()[name]
    o = Oracle(case)
    q = o.cons_from_prim()
    steps = (0, 3) if name == "jet" else (0,)
    for step in steps:
        r_ref = o.rhs(q, step)
        # PR: 1e-10, or four times the oracle's own one-ulp sensitivity where larger
        bar = np.maximum(1e-10, 4.0 * ulp_sensitivity(o, q, r_ref)) if name == "pr" else np.full(q.shape[0], 1e-10)
        for tile in march_tiles():
            ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
            ctx.set_tile(tile)
            err = field_err(gpu_rhs(ctx, q, dev, step), r_ref)
            print(f"march {name} step {step} tile {tile}: {np.array2string(err, precision=2)}", flush=True)
            assert np.all(err < bar)
            ctx.close()


@pytest.mark.parametrize("name", CASE_NAMES)
def test_march_steps_every_tile(dev, stream, name):
    """three steps on every z-marching tile (the CFL bound of each new state
    comes from the last stage of the step before) and the mixed path within
    1e-4 relative L1 of the FP64 path"""
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = cases()[name]
    o = Oracle(case)
    q = o.cons_from_prim()
    t_ref = 0.0
    for k in range(3):
        t_ref, _ = o.step(q, k, t_ref)
    for tile in march_tiles():
        ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
        ctx.set_tile(tile)
        ctx.init_primitive()
        t = ctx.n_steps(3)
        err = field_err(ctx.get_state(), q).max()
        print(f"march {name} tile {tile}: 3 steps {err:.3e}, t {t:.6e} / {t_ref:.6e}", flush=True)
        assert abs(t / t_ref - 1) < 1e-12
        assert err < 1e-10
        m = fvm.Context(case, fvm.FVM_MIXED, stream=stream.cuda_stream)
        m.set_tile(tile)
        m.init_primitive()
        m.n_steps(3)
        a, b = m.get_primitive(), ctx.get_primitive()
        n = a.shape[1]
        uref = 300.0 if name == "jet" else 30.0
        l1 = {"rho": np.abs(a[0] - b[0]).sum() / np.abs(b[0]).sum(), "p": np.abs(a[4] - b[4]).sum() / np.abs(b[4]).sum(),
              "u": np.abs(a[1:4] - b[1:4]).sum() / (n * uref), "Y": np.abs(a[6] - b[6]).sum() / n}
        print(f"march {name} tile {tile}: mixed vs fp64 {l1}", flush=True)
        assert max(l1.values()) < 1e-4
        ctx.close()
        m.close()


def test_march_tiles_equal_the_face_kernel_tiles(dev, stream):
    """50 steps of the small jet: every z-marching tile against the closure +
    face kernel pair (tile 0), FP64, to rounding of the whole run"""
    from paper_2304_00140_amd import fvm
    case = W.liquid_jet_3d(nx=40, ny=20, nz=36, cells_per_D=8, steps=50)
    ref = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    ref.init_primitive()
    ref.n_steps(50)
    qr = ref.get_state()
    for tile in march_tiles():
        ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
        ctx.set_tile(tile)
        ctx.init_primitive()
        ctx.n_steps(50)
        err = field_err(ctx.get_state(), qr).max()
        print(f"march tile {tile} vs tile 0 after 50 jet steps: {err:.3e}", flush=True)
        assert err < 1e-9
        ctx.close()


def test_march_tiles_refused_where_not_supported(dev, stream):
    from paper_2304_00140_amd import fvm
    for case in (W.random_state(3, [9, 8, 7], 85, second_gas=True), W.random_state(3, [9, 8, 7], 86, barotropic=True)):
        ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
        for tile in march_tiles():
            with pytest.raises(fvm.FvmError, match="z-marching"):
                ctx.set_tile(tile)
        ctx.close()
