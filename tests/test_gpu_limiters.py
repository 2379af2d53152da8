"""GPU (gfx950) stage kernels with limiters other than the default pair
(Koren for velocities, Minmod for p, T, xi), which run the kernels that read
the limiter kind at run time, against the CPU FP64 oracle: one RHS per
limiter pair (Table 4.2) in 1D, 2D, 3D and the barotropic model, and the
default pair through the same test for comparison."""
import numpy as np
import pytest

from paper_2304_00140_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PAIRS = [("koren", "minmod"), ("vanleer", "superbee"), ("mc", "vanalbada"), ("chakravarthy", "koren"),
         ("minmod", "mc")]


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


def gpu_rhs(ctx, q, dev):
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    rd = torch.zeros_like(qd)
    torch.cuda.synchronize()
    ctx.rhs(qd.data_ptr(), rd.data_ptr(), 0)
    return rd.cpu().numpy()


def case_for(kind, lu, ls):
    if kind == "1d":
        c = W.random_state(1, [97], 71)
    elif kind == "2d":
        c = W.random_state(2, [37, 29], 72, switching=1, sigma=0.05)
    elif kind == "3d":
        c = W.random_state(3, [14, 11, 10], 73, switching=1)
    else:
        c = W.random_state(2, [37, 29], 74, barotropic=True)
    c["scheme"] = dict(c["scheme"], lim_u=W.LIM[lu], lim_s=W.LIM[ls])
    return c


@pytest.mark.parametrize("kind", ["1d", "2d", "3d", "baro"])
@pytest.mark.parametrize("pair", PAIRS, ids=lambda p: f"{p[0]}-{p[1]}")
def test_limiter_pair_rhs(dev, stream, kind, pair):
    from oracle.oracle import Oracle
    from paper_2304_00140_amd import fvm
    case = case_for(kind, *pair)
    o = Oracle(case)
    q = o.cons_from_prim()
    r_ref = o.rhs(q)
    ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    r = gpu_rhs(ctx, q, dev)
    scale = np.maximum(np.abs(r_ref).max(axis=1), 1e-300)
    rel = np.abs(r - r_ref).max(axis=1) / scale
    tol = np.full(rel.shape, 1e-10)
    if kind == "baro":
        # the stiff barotropic liquid's pressure rounding (c_L^2 rho_sat 2^-52
        # per face) on the momentum rows, as in the barotropic parity tests
        b = case["eos"]["baro"]
        tol[1:3] += 16 * b["c_liq"] ** 2 * b["rho_sat"] * 2.0 ** -52 / case["grid"]["dx"][0] / scale[1:3]
    print(f"{kind} limiters {pair}: {np.array2string(rel, precision=2)}", flush=True)
    assert np.all(rel <= tol)
    ctx.close()
