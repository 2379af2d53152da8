"""Host logic of the tile autotuner: cases whose kernels differ (closure
kinds, the barotropic model with one or two gases, precision, stress terms)
never share a cache entry, so a tile tuned for one is never applied to a case
whose kernels refuse it."""
from types import SimpleNamespace

from paper_2304_00140_amd import tune, workloads as W


def handle(case):
    n = 1
    for d in range(case["grid"]["dim"]):
        n *= case["grid"]["n"][d]
    return SimpleNamespace(case=case, ncell=n)


def test_cache_keys_separate_models_gases_and_precisions():
    one = W.random_state(3, [10, 9, 8], 1, barotropic=True)
    two = W.random_state(3, [10, 9, 8], 1, barotropic=True, second_gas=True)
    four = W.random_state(3, [10, 9, 8], 1)
    three = W.random_state(3, [10, 9, 8], 1, second_gas=True)
    keys = [tune.key_of(handle(c), p) for c in (one, two, four, three) for p in (0, 1)]
    assert len(set(keys)) == len(keys)
    visc = dict(two, eos=W.baro_eos(mu_liq=1e-3, RT2=two["eos"]["baro"]["RT2"]))
    assert tune.key_of(handle(visc), 0) != tune.key_of(handle(two), 0)
    assert tune.key_of(handle(two), 0) == tune.key_of(handle(dict(two)), 0)
