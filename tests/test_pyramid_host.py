"""Host logic of the multilevel scheme: the library's pyramid plan (a host-only C-ABI call,
no device needed) equals the oracle's plan, and bad arguments give the documented codes."""
import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def disco():
    from paper_1807_00467_amd import disco as d
    return d


def test_library_plan_equals_oracle_plan(disco):
    rng = np.random.default_rng(11)
    cases = [((512, 512, 128), (0.7, 0.7, 2.5)), ((64, 64, 48), (1.5, 1.5, 1.5)), ((512, 512, 256), (0.7, 0.7, 1.25)),
             ((192, 192, 160), (1.0, 1.0, 1.0)), ((48, 32, 24), (1.2, 1.4, 2.2))]
    for _ in range(300):
        shape = tuple(int(x) for x in rng.choice([4, 8, 12, 16, 24, 32, 40, 48, 64, 96, 128, 256], 3))
        spacing = tuple(float(x) for x in rng.uniform(0.3, 4.0, 3))
        cases.append((shape, spacing))
    for shape, spacing in cases:
        for levels in (1, 2, 4, 8):
            lib = disco.pyramid_plan(shape, spacing, levels)
            ref = oracle.pyramid_plan(shape, spacing, levels)
            assert len(lib) == len(ref), (shape, spacing, levels)
            for (n, h, hv), r in zip(lib, ref):
                assert n == r["shape"] and hv == r["halve"]
                assert h == r["spacing"]  # doubling is exact


def test_plan_argument_errors(disco):
    with pytest.raises(disco.DiscoError) as e:
        disco.pyramid_plan((30, 32, 32), (1.0, 1.0, 1.0), 4)
    assert e.value.code == disco.ERR_SHAPE
    with pytest.raises(disco.DiscoError) as e:
        disco.pyramid_plan((32, 32, 32), (1.0, -1.0, 1.0), 4)
    assert e.value.code == disco.ERR_NONFINITE
    with pytest.raises(disco.DiscoError) as e:
        disco.pyramid_plan((32, 32, 32), (1.0, 1.0, 1.0), 9)
    assert e.value.code == disco.ERR_ARG
