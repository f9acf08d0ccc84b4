"""GPU tests of the depth-2 temporally blocked wave sweep (variants named
tb2_*): its results must equal the plain z-marching sweep bit for bit, for
every storage type, ragged tile edges, several z-chunks, sources next to tile
corners (whose extended regions overlap up to four tiles), receivers, and
step counts that mix two-step passes with plain steps; and it must meet the
FP64 oracle's tolerance on its own."""
import numpy as np
import pytest

import paper_2404_02218_amd as S
from _helpers import gpu_wave, oracle_wave, rel_err, wave_inputs

pytestmark = pytest.mark.gpu


def _tb_variants(plan):
    return [v for v in range(plan.variant_count()) if plan.variant_name(v).startswith("tb2_")]


@pytest.mark.parametrize("dtype", [S.F32, S.BF16, S.F16])
@pytest.mark.parametrize("shape", [(45, 38, 97), (13, 70, 130)])
def test_temporal_blocking_equals_plain_sweep_bitwise(device, dtype, shape):
    u0, um1, beta = wave_inputs(shape, seed=61, dtype=dtype)
    nz, ny, nx = shape
    # next to tile corners (tiles are 64 x 32), on the first and last planes
    src = np.array([[nz // 2, 31, 63], [0, 32, 64], [nz - 1, ny - 1, nx - 1], [3, 29, 67], [nz // 3, 0, 0]])
    rec = np.array([[nz // 2, 31, 64], [1, 33, 62], [nz - 1, 0, nx - 1]])
    plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4, dtype=dtype)
    tbs = _tb_variants(plan)
    assert len(tbs) == 3
    for nsteps in (2, 4, 5, 6, 11):
        amp = np.random.default_rng(62 + nsteps).standard_normal((nsteps, len(src)))
        base = gpu_wave(plan, u0, um1, beta, nsteps, src=src, amp=amp, rec=rec, variant=1)
        for v in tbs:
            got = gpu_wave(plan, u0, um1, beta, nsteps, src=src, amp=amp, rec=rec, variant=v)
            for x, y in zip(got, base):
                assert np.array_equal(x, y), (plan.variant_name(v), nsteps)


def test_temporal_blocking_meets_oracle_tolerance(device):
    shape = (40, 52, 75)
    u0, um1, beta = wave_inputs(shape, seed=71)
    src = np.array([[20, 26, 37]])
    rec = np.array([[20, 26, 45], [5, 5, 5]])
    amp = np.random.default_rng(72).standard_normal((24, 1))
    plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4)
    v = _tb_variants(plan)[-1]
    a, b, tr = gpu_wave(plan, u0, um1, beta, 24, src=src, amp=amp, rec=rec, variant=v)
    ra, rb, rtr = oracle_wave(u0, um1, beta, 4, 4, 24, src=src, amp=amp, rec=rec)
    assert rel_err(a, ra) <= 1e-5
    assert rel_err(b, rb) <= 1e-5
    assert rel_err(tr, rtr) <= 1e-5


def test_temporal_blocking_split_runs_and_tiny_grids(device):
    # run(a) + run(b) == run(a + b) across pass boundaries; grids smaller than a tile
    for shape in [(30, 41, 66), (3, 5, 7), (1, 1, 1)]:
        u0, um1, beta = wave_inputs(shape, seed=81)
        plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4)
        plan.variant = _tb_variants(plan)[0]
        whole = gpu_wave(plan, u0, um1, beta, 17)
        parts = gpu_wave(plan, u0, um1, beta, 17, split=[5, 8, 4])
        plain = gpu_wave(plan, u0, um1, beta, 17, variant=2)
        for x, y, z in zip(whole, parts, plain):
            assert np.array_equal(x, y) and np.array_equal(x, z), shape
