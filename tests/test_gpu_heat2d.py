"""GPU tests of the multi-step 2D heat kernels (variants tb2d_*): T steps per
launch in LDS must equal T plain sweeps bit for bit, for ragged tiles, grids
smaller than a tile or one point wide, step counts that mix multi-step
passes with plain sweeps, and radius 1 and 2; and the 256^2 x 100 workload
meets the FP64 oracle's tolerance."""
import numpy as np
import pytest

import oracle
import paper_2404_02218_amd as S
import workloads as W
from _helpers import gpu_heat, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,radius", [((256, 256), 1), ((50, 77), 1), ((5, 7), 1), ((1, 100), 1),
                                          ((100, 1), 1), ((33, 300), 2), ((70, 45), 2)])
def test_multistep_equals_plain_sweeps_bitwise(device, shape, radius):
    rng = np.random.default_rng(sum(shape) + radius)
    u0 = W.round_to_storage(rng.uniform(0, 1, shape), "f32")
    alpha = 0.2 if radius == 1 else 0.1
    plan = S.Plan(S.HEAT, shape, radius, S.heat_weights(2 * radius, alpha), halo=radius)
    names = [plan.variant_name(v) for v in range(plan.variant_count())]
    assert len(names) == 5 and all(n.startswith("tb2d_") for n in names[1:])
    for nsteps in (1, 3, 8, 16, 17, 33, 100):
        base = gpu_heat(plan, u0, nsteps, variant=0)
        for v in range(1, len(names)):
            got = gpu_heat(plan, u0, nsteps, variant=v)
            assert np.array_equal(got, base), (names[v], nsteps)


def test_multistep_heat2d_workload_meets_oracle_tolerance(device):
    H = W.heat2d_c1()
    u0 = W.round_to_storage(H.u0, "f32")
    plan = S.Plan(S.HEAT, H.shape, 1, S.heat_weights(2, H.alpha), halo=1)
    assert plan.variant_name(plan.variant) == "tb2d_t8_16x16"
    got = gpu_heat(plan, u0, H.nsteps)
    c = [H.alpha * x for x in oracle.fd_weights_float(2)]
    ref = W.interior_of(oracle.heat_run(W.embed(u0, 1), 1, 1, c, H.nsteps), 1)
    assert rel_err(got, ref) <= 1e-5


def test_tuned_2d_heat_plan_equals_plain_sweeps(device):
    """stencil_tune picks among the point kernel and the multi-step kernels;
    whatever it picks, a run equals the point kernel's bits."""
    shape = (96, 130)
    u0 = W.round_to_storage(np.random.default_rng(5).uniform(0, 1, shape), "f32")
    plan = S.Plan(S.HEAT, shape, 1, S.heat_weights(2, 0.2), halo=1)
    f = [plan.field() for _ in range(2)]
    f[0].load(W.embed(u0, 1))
    plan.tune(f, reps=3)
    assert 0 <= plan.variant < plan.variant_count()
    got = gpu_heat(plan, u0, 37)
    assert np.array_equal(got, gpu_heat(plan, u0, 37, variant=0))
