"""Batches (many independent cases of uneven size advanced together through
the tile table) of the barotropic model in 2D and 3D and of the
three-component model in 2D and 3D: every case of the batch bit-identical to the
same case advanced on its own, in both precisions; mixing models in one batch
is rejected."""
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


def model_cases(kind):
    if kind == "baro2d":
        return [W.vapour_bubble_wall_2d(nx, ny, 10, dx=dx, p_inf=pi)
                for nx, ny, dx, pi in ((48, 24, 40e-6, 1e6), (61, 37, 30e-6, 3e6), (33, 50, 35e-6, 5e5))]
    if kind == "baro3d":
        return [W.random_state(3, n, seed, barotropic=True, bc=[[W.BC_WALL, W.BC_ZEROGRAD]] * 3)
                for n, seed in (([12, 10, 9], 91), ([17, 9, 11], 92))]
    if kind == "three3d":
        return [W.random_state(3, n, seed, second_gas=True, switching=1, sigma=0.05,
                               bc=[[W.BC_WALL, W.BC_ZEROGRAD], [W.BC_PERIODIC, W.BC_PERIODIC],
                                   [W.BC_ZEROGRAD, W.BC_WALL]])
                for n, seed in (([13, 10, 9], 98), ([9, 14, 11], 99))]
    return [W.random_state(2, n, seed, second_gas=True, bc=[[W.BC_WALL, W.BC_WALL]] * 2)
            for n, seed in (([30, 22], 93), ([41, 19], 94), ([25, 33], 95))]


@pytest.mark.parametrize("kind", ["baro2d", "baro3d", "three2d", "three3d"])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_batch_equals_single_cases(dev, stream, kind, prec):
    from paper_2304_00140_amd import fvm
    cases = model_cases(kind)
    b = fvm.Batch(cases, prec, stream=stream.cuda_stream)
    for i in range(len(cases)):
        b.init_primitive(i)
    b.n_steps(6)
    for i, c in enumerate(cases):
        s = fvm.Context(c, prec, stream=stream.cuda_stream)
        s.init_primitive()
        s.n_steps(6)
        np.testing.assert_array_equal(b.get_state(i), s.get_state())
        s.close()
    print(f"{kind} batch of {len(cases)} ({'fp64' if prec == 0 else 'mixed'}): bit-identical", flush=True)


def test_batch_of_mixed_models_is_rejected(dev, stream):
    from paper_2304_00140_amd import fvm
    cases = [W.random_state(2, [20, 16], 96), W.random_state(2, [20, 16], 97, barotropic=True)]
    with pytest.raises(fvm.FvmError):
        fvm.Batch(cases, fvm.FVM_FP64, stream=stream.cuda_stream)
