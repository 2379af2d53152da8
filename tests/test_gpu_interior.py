"""GPU (gfx950) stage kernels on grids large enough that every tile shape has
tiles whose two-cell halo lies inside the domain (those stage their halo
without the boundary logic, at 32-bit offsets) next to boundary tiles (the
per-cell ghost path), and tiles whose 27-tile neighbourhood is uniform in the
gas fractions (the 3D face kernels skip the CSF term there, which is exactly
zero, after the closure kernel's extremes and the mark kernel) next to
interface tiles.  One FP64 right-hand side on every tile against the oracle,
and a 3D batch against its cases alone in both precisions.

Sizes: a 3D tile of TX x TY x TZ cells at x0 has an inside halo when
x0 >= 2 and x0 + TX + 2 <= n (likewise y, z); the widest 3D tile row is
16 cells in x and 8 in y and z, so 40 x 20 x 20 holds such tiles for every
row; the 2D tiles need 132 cells in x (64 x 4) and 68 in y (32 x 32)."""
import numpy as np
import pytest

from paper_2304_00140_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS = 2.0 ** -52


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


def gpu_rhs(ctx, q, dev, step=0):
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    rd = torch.zeros_like(qd)
    torch.cuda.synchronize()
    ctx.rhs(qd.data_ptr(), rd.data_ptr(), step)
    return rd.cpu().numpy()


def field_errs(a, b):
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return np.abs(a - b).max(axis=1) / scale


def inside_tiles(n, t):
    """number of tiles of shape t whose two-cell halo lies inside a grid n"""
    count = 1
    for nd, td in zip(n, t):
        count *= sum(1 for x0 in range(0, nd, td) if x0 >= 2 and x0 + td + 2 <= nd)
    return count


def one_ulp_sensitivity(o, q, r_ref):
    """the oracle's own change of each RHS field under a one-ulp change of its
    liquid partial density, over each field's scale"""
    qs = q.copy()
    qs[0] *= 1.0 + EPS
    return field_errs(o.rhs(qs), r_ref)


def every_tile(case, dim, dev, stream, sens=None):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    o = Oracle(case)
    q = o.cons_from_prim()
    r_ref = o.rhs(q)
    bar = np.full(q.shape[0], 1e-10)
    if sens:
        bar = np.maximum(bar, 4.0 * one_ulp_sensitivity(o, q, r_ref))
    n = case["grid"]["n"][:dim]
    tested = 0
    for tile in range(fvm.lib().fvm_tile_count(dim)):
        ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
        try:
            ctx.set_tile(tile)
        except fvm.FvmError as e:
            # the z-marching tiles take the four-equation model only
            assert "z-marching" in str(e)
            ctx.close()
            continue
        err = field_errs(gpu_rhs(ctx, q, dev), r_ref)
        print(f"{case['name']} {n} tile {tile}: {np.array2string(err, precision=2)}", flush=True)
        assert np.all(err < bar)
        ctx.close()
        tested += 1
    assert tested > 0


def test_tile_shapes_have_inside_tiles_here():
    """the grids below hold inside-halo tiles for every tile shape of the
    library (a check of the sizes, not of the GPU; the 3D tiles are at most 8
    cells deep in z)"""
    import ctypes as C
    from paper_2304_00140_amd import fvm
    L = fvm.lib()
    for dim, n in ((2, [136, 72]), (3, [40, 20, 20])):
        for tile in range(L.fvm_tile_count(dim)):
            if dim == 3 and L.fvm_tile_kernels(3, tile) != fvm.FVM_TK_PAIR:
                continue
            tx, ty, nt = C.c_int(), C.c_int(), C.c_int()
            assert L.fvm_tile_shape(dim, tile, C.byref(tx), C.byref(ty), C.byref(nt)) == 0
            t = [tx.value, ty.value, 8][:dim]
            assert inside_tiles(n, t) > 0, (dim, tile, t)


def test_jet_every_3d_tile(dev, stream):
    """Peng-Robinson jet (core of 8 cells across, CSF and switching on, inflow
    noise): gas-only tiles surround the core"""
    case = W.liquid_jet_3d(nx=40, ny=20, nz=20, cells_per_D=8, steps=3)
    every_tile(case, 3, dev, stream)


def test_cube_every_3d_tile(dev, stream):
    """barotropic cube of liquid in gas (sigma = 800), 40^3: most tiles hold
    gas only.  At rest the momentum rows carry the CSF force (they agree to
    about 3e-13); the two mass rows are rounding noise of the uniform
    pressure (1e-9 and 1e-12 against densities of 1000 and 1), so the bar is
    1e-10 or four times the oracle's own one-ulp sensitivity, whichever is
    larger"""
    case = W.cube_to_sphere_3d(40, 10)
    every_tile(case, 3, dev, stream, sens=True)


def test_two_phase_2d_every_tile(dev, stream):
    """2D random state with switching and CSF"""
    case = W.random_state(2, [136, 72], 97, switching=1, sigma=0.05)
    every_tile(case, 2, dev, stream)


def test_barotropic_2d_every_tile(dev, stream):
    case = W.random_state(2, [136, 72], 98, barotropic=True, switching=1, sigma=0.05)
    every_tile(case, 2, dev, stream, sens=True)


def test_batch3d_equals_single_cases(dev, stream):
    """two 3D jets of different sizes in one batch (one tile table, the CSF
    marks built per case from its own tiles) against each case alone: the
    same bits after three steps, on an 8 x 8 x 8 tile with inside tiles in
    both cases"""
    from paper_2304_00140_amd import fvm
    cases = [W.liquid_jet_3d(nx=40, ny=20, nz=20, cells_per_D=8, steps=3),
             W.liquid_jet_3d(nx=36, ny=28, nz=20, cells_per_D=8, steps=3)]
    for prec in (fvm.FVM_FP64, fvm.FVM_MIXED):
        b = fvm.Batch(cases, prec, stream=stream.cuda_stream)
        b.set_tile(15)
        for i in range(len(cases)):
            b.init_primitive(i)
        b.n_steps(3)
        for i, c in enumerate(cases):
            s = fvm.Context(c, prec, stream=stream.cuda_stream)
            s.set_tile(15)
            s.init_primitive()
            s.n_steps(3)
            np.testing.assert_array_equal(b.get_state(i), s.get_state())
            s.close()


def test_walls_and_periodic_sides_every_3d_tile(dev, stream):
    """the cube with slip walls on some sides and a periodic pair on another:
    tiles at a wall are marked from their neighbours (mirror ghosts), tiles
    at the periodic sides keep the CSF term; one RHS on every 3D tile"""
    case = W.cube_to_sphere_3d(40, 10)
    case["grid"] = dict(case["grid"], bc=[[W.BC_WALL, W.BC_ZEROGRAD], [W.BC_PERIODIC, W.BC_PERIODIC],
                                          [W.BC_WALL, W.BC_WALL]])
    every_tile(case, 3, dev, stream, sens=True)


def test_jet_walls_every_3d_tile(dev, stream):
    """the four-equation jet with slip walls on the y and z sides"""
    case = W.liquid_jet_3d(nx=40, ny=20, nz=20, cells_per_D=8, steps=3)
    bc = case["grid"]["bc"]
    case["grid"] = dict(case["grid"], bc=[bc[0], [W.BC_WALL, W.BC_WALL], [W.BC_WALL, W.BC_ZEROGRAD]])
    every_tile(case, 3, dev, stream)
