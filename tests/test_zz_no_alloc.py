"""fvm_rhs_noalloc (no context, no device allocation; workspace in a static
device array) against fvm_rhs of a context on the same input: two calls in a
row, the second on a smaller case, in 2D and 3D; and the size limit."""
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


def _ctx_rhs(case, q, dev, stream, step):
    from paper_2304_00140_amd import fvm
    ctx = fvm.Context(case, fvm.FVM_FP64, stream=stream.cuda_stream)
    qd = torch.from_numpy(q).to(dev)
    rd = torch.zeros_like(qd)
    torch.cuda.synchronize()
    ctx.rhs(qd.data_ptr(), rd.data_ptr(), step)
    r = rd.cpu().numpy()
    ctx.close()
    return r


def _noalloc_rhs(case, q, dev, stream, step):
    from paper_2304_00140_amd import fvm
    qd = torch.from_numpy(q).to(dev)
    rd = torch.full_like(qd, float("nan"))
    torch.cuda.synchronize()
    fvm.rhs_noalloc(case, qd.data_ptr(), rd.data_ptr(), step, stream.cuda_stream)
    stream.synchronize()
    return rd.cpu().numpy()


def _err(a, b):
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return (np.abs(a - b).max(axis=1) / scale).max()


CASES = [
    ("2d", lambda: W.random_state(2, [70, 37], 3, sigma=0.07, switching=1),
     lambda: W.random_state(2, [33, 21], 4, gas="pr", velocity=10.0)),
    ("3d", lambda: W.random_state(3, [20, 13, 11], 5, sigma=0.05, switching=1),
     lambda: W.random_state(3, [9, 8, 7], 6, bc=[[W.BC_WALL, W.BC_ZEROGRAD]] * 3)),
]


@pytest.mark.parametrize("name,big,small", CASES, ids=[c[0] for c in CASES])
def test_noalloc_rhs_matches_context_rhs(dev, name, big, small):
    from oracle.oracle import Oracle
    stream = torch.cuda.Stream(device=dev)
    for k, make in enumerate((big, small)):
        case = make()
        q = np.ascontiguousarray(Oracle(case).cons_from_prim())
        r0 = _ctx_rhs(case, q, dev, stream, 3)
        r1 = _noalloc_rhs(case, q, dev, stream, 3)
        err = _err(r1, r0)
        print(f"noalloc {name} call {k} {case['grid']['n']}: {err:.3e}", flush=True)
        assert np.all(np.isfinite(r1))
        assert err < 1e-10


def test_noalloc_rejects_a_case_beyond_the_workspace(dev):
    from paper_2304_00140_amd import fvm
    case = W.random_state(2, [2048, 1024], 7)
    qd = torch.zeros((5, 4), dtype=torch.float64, device=dev)
    with pytest.raises(fvm.FvmError, match="workspace"):
        fvm.rhs_noalloc(case, qd.data_ptr(), qd.data_ptr(), 0, None)
