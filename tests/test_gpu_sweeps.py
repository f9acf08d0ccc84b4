"""GPU parity of the heat and wave sweeps against the FP64 oracle, through
the C ABI, plus the bit-exact invariants that need no oracle (every kernel
variant computes the same bits; run(a)+run(b) == run(a+b); the light cone;
the halo is never written)."""
import math

import numpy as np
import pytest

import oracle
import paper_2404_02218_amd as S
import workloads as W
from _helpers import DT_NAMES, gpu_heat, gpu_wave, oracle_wave, rel_err, torch_f64, wave_inputs

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


def test_c1_heat2d_so2_full_size(device):
    P = W.heat2d_c1()
    u0 = W.round_to_storage(P.u0, "f32")
    plan = S.Plan(S.HEAT, P.shape, 1, S.heat_weights(2, P.alpha), halo=1)
    got = gpu_heat(plan, u0, P.nsteps)
    c = [P.alpha * x for x in oracle.fd_weights_float(2)]
    ref = W.interior_of(oracle.heat_run(W.embed(u0, 1), 1, 1, c, P.nsteps), 1)
    assert rel_err(got, ref) <= TOL_F32


def test_heat2d_dirichlet_sine_mode_closed_form(device):
    n, alpha, steps, p, q = 61, 0.2, 50, 2, 7
    i = np.arange(1, n + 1)
    mode = np.outer(np.sin(math.pi * p * i / (n + 1)), np.sin(math.pi * q * i / (n + 1)))
    g = 1 - 4 * alpha * (math.sin(math.pi * p / (2 * (n + 1))) ** 2
                         + math.sin(math.pi * q / (2 * (n + 1))) ** 2)
    plan = S.Plan(S.HEAT, (n, n), 1, S.heat_weights(2, alpha), halo=1)
    got = gpu_heat(plan, W.round_to_storage(mode, "f32"), steps)
    assert np.max(np.abs(got - g ** steps * mode)) <= 1e-5


@pytest.mark.parametrize("shape", [(37, 45, 83), (70, 33, 130), (1, 1, 1), (5, 64, 64)])
def test_heat3d_so4_all_variants_bitwise_and_parity(device, shape):
    rng = np.random.default_rng(21)
    u0 = W.round_to_storage(rng.random(shape) + W.gaussian_bump(shape, 6.0), "f32")
    plan = S.Plan(S.HEAT, shape, 2, S.heat_weights(4, 0.05), halo=2)
    base = gpu_heat(plan, u0, 12, variant=0)
    c = [0.05 * x for x in oracle.fd_weights_float(4)]
    ref = W.interior_of(oracle.heat_run(W.embed(u0, 2), 2, 2, c, 12), 2)
    assert rel_err(base, ref) <= TOL_F32
    for v in range(1, plan.variant_count()):
        got = gpu_heat(plan, u0, 12, variant=v)
        assert np.array_equal(got, base), plan.variant_name(v)


@pytest.mark.parametrize("dtype", [S.BF16, S.F16])
@pytest.mark.parametrize("radius", [2, 4])
def test_heat3d_16bit_all_variants_bitwise(device, dtype, radius):
    # every z-marching variant of a 16-bit heat plan equals the
    # one-point-per-thread kernel bit for bit (ragged tiles in x and y)
    shape = (37, 45, 83)
    rng = np.random.default_rng(23)
    u0 = W.round_to_storage(rng.random(shape) + W.gaussian_bump(shape, 6.0), DT_NAMES[dtype])
    plan = S.Plan(S.HEAT, shape, radius, S.heat_weights(2 * radius, 0.05), halo=radius, dtype=dtype)
    base = gpu_heat(plan, u0, 12, variant=0)
    assert np.all(np.isfinite(base)) and np.abs(base).max() > 0
    for v in range(1, plan.variant_count()):
        got = gpu_heat(plan, u0, 12, variant=v)
        assert np.array_equal(got, base), plan.variant_name(v)


@pytest.mark.parametrize("radius", [1, 3, 4])
def test_heat3d_other_radii_all_variants_bitwise_and_parity(device, radius):
    """The z-marching and temporally blocked heat kernels are built for
    radius 1..4 and the tuner may pick any of them: every variant gives
    variant 0's bits on grids with ragged tiles, and variant 0 meets the
    oracle."""
    shape = (29, 37, 71)
    rng = np.random.default_rng(22 + radius)
    u0 = W.round_to_storage(rng.random(shape) + W.gaussian_bump(shape, 5.0), "f32")
    alpha = 0.1 / radius
    plan = S.Plan(S.HEAT, shape, radius, S.heat_weights(2 * radius, alpha), halo=radius)
    base = gpu_heat(plan, u0, 10, variant=0)
    c = [alpha * x for x in oracle.fd_weights_float(2 * radius)]
    ref = W.interior_of(oracle.heat_run(W.embed(u0, radius), radius, radius, c, 10), radius)
    assert rel_err(base, ref) <= TOL_F32
    names = [plan.variant_name(v) for v in range(plan.variant_count())]
    assert any(n.startswith("tb2_") for n in names)
    for v in range(1, plan.variant_count()):
        got = gpu_heat(plan, u0, 10, variant=v)
        assert np.array_equal(got, base), names[v]


def test_heat3d_periodic_fourier_mode(device):
    shape, alpha, steps = (24, 20, 36), 0.05, 30
    m = (1, 2, 3)
    k = [2 * math.pi * m[d] / shape[d] for d in range(3)]
    z, y, x = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    mode = W.round_to_storage(np.cos(k[0] * z + k[1] * y + k[2] * x + 0.3), "f32")
    c4 = oracle.fd_weights(4)
    g = 1 - alpha * sum(oracle.symbol(c4, kd) for kd in k)
    plan = S.Plan(S.HEAT, shape, 2, S.heat_weights(4, alpha), halo=2, bc=S.BC_PERIODIC)
    got = gpu_heat(plan, mode, steps)
    assert np.max(np.abs(got - g ** steps * mode)) <= 2e-6
    ref = W.interior_of(oracle.heat_run(W.embed(mode, 2), 2, 2,
                                        [alpha * float(v) for v in c4], steps, periodic=True), 2)
    assert rel_err(got, ref) <= TOL_F32


@pytest.mark.parametrize("shape", [(40, 52, 75), (33, 17, 140)])
def test_wave3d_so8_parity_with_source_and_receivers(device, shape):
    u0, um1, beta = wave_inputs(shape, seed=31)
    src = np.array([[shape[0] // 2, shape[1] // 3, shape[2] - 3], [4, 5, 6]])
    rec = np.array([[1, 1, 1], [shape[0] - 1, shape[1] - 1, shape[2] - 1], [10, 7, 64 % shape[2]],
                    [shape[0] // 2, shape[1] // 3, shape[2] - 3]])
    steps = 60
    amp = np.random.default_rng(32).standard_normal((steps, 2))
    plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4)
    a, b, tr = gpu_wave(plan, u0, um1, beta, steps, src=src, amp=amp, rec=rec)
    ra, rb, rtr = oracle_wave(u0, um1, beta, 4, 4, steps, src=src, amp=amp, rec=rec)
    assert rel_err(a, ra) <= TOL_F32
    assert rel_err(b, rb) <= TOL_F32
    assert rel_err(tr, rtr) <= TOL_F32


@pytest.mark.parametrize("dtype", [S.F32, S.BF16, S.F16])
def test_wave3d_all_variants_bitwise(device, dtype):
    # variant 0 is the one-point-per-thread kernel, which widens every operand
    # and computes in FP32; the z-marching variants (FP16: operands read as
    # FP16 by the mixed-precision FMA) and the temporally blocked ones must
    # give the same bits, with ragged tile edges and sources on the faces
    shape = (45, 38, 97)
    u0, um1, beta = wave_inputs(shape, seed=41, dtype=dtype)
    src = np.array([[20, 30, 90], [44, 0, 0]])
    rec = np.array([[20, 30, 90], [3, 3, 3]])
    amp = np.random.default_rng(42).standard_normal((9, 2))
    plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4, dtype=dtype)
    base = gpu_wave(plan, u0, um1, beta, 9, src=src, amp=amp, rec=rec, variant=0)
    for v in range(1, plan.variant_count()):
        got = gpu_wave(plan, u0, um1, beta, 9, src=src, amp=amp, rec=rec, variant=v)
        for x, y in zip(got, base):
            assert np.array_equal(x, y), plan.variant_name(v)


def test_wave_split_runs_are_bitwise_equal(device):
    shape = (30, 41, 66)
    u0, um1, beta = wave_inputs(shape, seed=51)
    src = np.array([[15, 20, 33]])
    rec = np.array([[15, 20, 40], [2, 2, 2]])
    amp = np.random.default_rng(52).standard_normal((23, 1))
    plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4)
    whole = gpu_wave(plan, u0, um1, beta, 23, src=src, amp=amp, rec=rec)
    parts = gpu_wave(plan, u0, um1, beta, 23, src=src, amp=amp, rec=rec, split=[7, 1, 15])
    for x, y in zip(whole, parts):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("steps", [1, 4, 9])
def test_wave_light_cone_exact_on_gpu(device, steps):
    shape, r = (40, 36, 70), 4
    s = np.array([19, 17, 20])
    beta = W.round_to_storage(np.random.default_rng(3).uniform(0.01, 0.05, shape), "f32")
    amp = np.ones((steps, 1))
    plan = S.Plan(S.WAVE2, shape, r, S.second_derivative_weights(8), halo=r)
    z0 = np.zeros(shape)
    a, _, _ = gpu_wave(plan, z0, z0, beta, steps, src=[s], amp=amp)
    zz, yy, xx = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    hops = (np.ceil(np.abs(zz - s[0]) / r) + np.ceil(np.abs(yy - s[1]) / r)
            + np.ceil(np.abs(xx - s[2]) / r))
    assert np.all(a[hops > steps - 1] == 0.0)
    tip = s.copy()
    tip[2] += r * (steps - 1)
    assert a[tuple(tip)] != 0.0


def test_halo_is_never_written(device):
    import torch
    shape = (20, 24, 40)
    u0, um1, beta = wave_inputs(shape, seed=61)
    plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4)
    f = [plan.field() for _ in range(3)]
    for fld, arr in zip(f, (u0, um1, beta)):
        full = np.full(tuple(n + 8 for n in shape), np.nan)
        full[4:-4, 4:-4, 4:-4] = arr
        # NaN everywhere outside the star's reach: corners and edges of the halo
        ring = W.embed(np.ones(shape), 4)
        for d in range(3):
            sl = [slice(4, -4)] * 3
            sl[d] = slice(None)
            ring[tuple(sl)] = 1
        full[ring == 0] = np.nan
        # the face halo itself is zero (Dirichlet)
        face = (ring == 1) & np.isnan(full)
        full[face] = 0.0
        fld.load(full)
    for v in range(plan.variant_count()):
        plan.variant = v
        g = [plan.field() for _ in range(3)]
        for src_f, dst_f in zip(f, g):
            dst_f.storage.copy_(src_f.storage)
        before = g[1].to_numpy()
        plan.run(g, 3)
        torch.cuda.synchronize()
        out = g[0].to_numpy()
        assert np.all(np.isfinite(out[4:-4, 4:-4, 4:-4])), plan.variant_name(v)
        halo_mask = np.ones(out.shape, bool)
        halo_mask[4:-4, 4:-4, 4:-4] = False
        np.testing.assert_array_equal(out[halo_mask], before[halo_mask])


@pytest.mark.parametrize("shape,so", [((300,), 8), ((57, 91), 4), ((64, 129), 8)])
def test_wave_1d_2d_parity(device, shape, so):
    r = so // 2
    u0, um1, beta = wave_inputs(shape, seed=71, halo=r)
    src = np.array([[s // 2 for s in shape]])
    rec = np.array([[s // 3 for s in shape]])
    amp = np.random.default_rng(72).standard_normal((40, 1))
    plan = S.Plan(S.WAVE2, shape, r, S.second_derivative_weights(so), halo=r)
    a, b, tr = gpu_wave(plan, u0, um1, beta, 40, src=src, amp=amp, rec=rec)
    ra, rb, rtr = oracle_wave(u0, um1, beta, r, r, 40, src=src, amp=amp, rec=rec)
    assert rel_err(a, ra) <= TOL_F32 and rel_err(tr, rtr) <= TOL_F32


def test_apply_on_sub_box(device):
    import torch
    shape = (21, 30, 45)
    u0, um1, beta = wave_inputs(shape, seed=81)
    plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4)
    f = [plan.field() for _ in range(3)]
    f[0].load(W.embed(u0, 4))
    f[1].load(W.embed(um1, 4))
    f[2].load(W.embed(beta, 4))
    out = plan.field()
    out.load(np.full(plan.layout.extents, 7.0))
    lo, hi = [3, 0, 10], [20, 30, 44]
    plan.apply(out, f, lo, hi)
    torch.cuda.synchronize()
    got = out.interior(4)
    ra, _, _ = oracle_wave(u0, um1, beta, 4, 4, 1)
    box = tuple(slice(a, b) for a, b in zip(lo, hi))
    assert rel_err(got[box], ra[box]) <= TOL_F32
    mask = np.ones(shape, bool)
    mask[box] = False
    assert np.all(got[mask] == 7.0)


def test_empty_interior_is_a_no_op(device):
    plan = S.Plan(S.WAVE2, (0, 10, 10), 4, S.second_derivative_weights(8), halo=4)
    f = [plan.field() for _ in range(3)]
    plan.run(f, 5)
    plan2 = S.Plan(S.HEAT, (0,), 1, S.heat_weights(2, 0.1))
    g = [plan2.field() for _ in range(2)]
    plan2.run(g, 3)


def test_tune_cache_separates_boundary_conditions(device):
    """A tuned Dirichlet plan's choice must not carry over to a periodic plan
    of the same shape (the periodic halo refresh and the zero-halo kernels
    differ): tune both, in that order, and check each run against the
    oracle."""
    shape3, alpha = (26, 34, 70), 0.05
    rng = np.random.default_rng(91)
    u3 = W.round_to_storage(rng.random(shape3), "f32")
    c4 = [alpha * x for x in oracle.fd_weights_float(4)]
    for bc, periodic in ((S.BC_DIRICHLET0, False), (S.BC_PERIODIC, True)):
        plan = S.Plan(S.HEAT, shape3, 2, S.heat_weights(4, alpha), halo=2, bc=bc)
        f = [plan.field() for _ in range(2)]
        f[0].load(W.embed(u3, 2))
        plan.tune(f, reps=1)
        if periodic:
            assert not plan.variant_name(plan.variant).startswith("tb2_")
        got = gpu_heat(plan, u3, 8)
        ref = W.interior_of(oracle.heat_run(W.embed(u3, 2), 2, 2, c4, 8, periodic=periodic), 2)
        assert rel_err(got, ref) <= TOL_F32, (bc, plan.variant_name(plan.variant))
    # 2D heat: the multi-step variants exist only with the zero halo
    shape2 = (40, 56)
    u2 = W.round_to_storage(rng.random(shape2), "f32")
    c2 = [0.2 * x for x in oracle.fd_weights_float(2)]
    for bc, periodic in ((S.BC_DIRICHLET0, False), (S.BC_PERIODIC, True)):
        plan = S.Plan(S.HEAT, shape2, 1, S.heat_weights(2, 0.2), halo=1, bc=bc)
        f = [plan.field() for _ in range(2)]
        f[0].load(W.embed(u2, 1))
        plan.tune(f, reps=1)
        got = gpu_heat(plan, u2, 20)
        ref = W.interior_of(oracle.heat_run(W.embed(u2, 1), 1, 1, c2, 20, periodic=periodic), 1)
        assert rel_err(got, ref) <= TOL_F32, (bc, plan.variant_name(plan.variant))


def test_rerun_with_coincident_sources_matches_oracle(device):
    """A 2D wave run twice on the same fields, source table and amplitude
    buffers, with the same number of sources: first at distinct positions,
    then with several at one point (fewer position groups).  The second run
    must not replay the first run's graph with the old group count."""
    import torch
    shape = (48, 70)
    u0, um1, beta = wave_inputs(shape, seed=93, halo=4)
    plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4)
    steps = 12
    amp = torch_f64(np.random.default_rng(94).standard_normal((steps, 4)), device)
    tr = torch.zeros((steps, 2), dtype=torch.float64, device=device)
    rec = np.array([[24, 35], [10, 60]])
    f = [plan.field() for _ in range(3)]
    for src in (np.array([[10, 10], [20, 30], [30, 50], [40, 65]]),
                np.array([[24, 35], [24, 35], [24, 35], [5, 5]]),
                np.array([[10, 10], [20, 30], [30, 50], [40, 65]])):
        f[0].load(W.embed(u0, 4))
        f[1].load(W.embed(um1, 4))
        f[2].load(W.embed(beta, 4))
        tr.zero_()
        plan.run(f, steps, src=src, src_amp=amp, rec=rec, rec_trace=tr)
        torch.cuda.synchronize()
        ra, rb, rtr = oracle_wave(u0, um1, beta, 4, 4, steps, src=src, amp=amp.cpu().numpy(), rec=rec)
        assert rel_err(f[0].interior(4), ra) <= TOL_F32, src.tolist()
        assert rel_err(tr.cpu().numpy(), rtr) <= TOL_F32, src.tolist()
