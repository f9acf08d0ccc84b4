"""GPU tests of point sources that share a grid point, of interpolated
(off-grid) sources and receivers, and of the absorbing layer: every kernel
variant gives the same bits, and the results meet the FP64 oracle's
tolerance (oracle: its own multilinear weights, on-grid sources of amount
w * q at the corners, traces as the weighted corner sums; the damped
leapfrog with the full damping field)."""
import ctypes as C

import numpy as np
import pytest

import oracle
import paper_2404_02218_amd as S
import workloads as W
from _helpers import gpu_wave, oracle_wave, rel_err, torch_f64, wave_inputs

pytestmark = pytest.mark.gpu


def _plan(shape, radius):
    return S.Plan(S.WAVE2, shape, radius, S.second_derivative_weights(2 * radius), halo=radius)


def _all_variants_equal(plan, run):
    base = run(0)
    for v in range(1, plan.variant_count()):
        got = run(v)
        for x, y in zip(got, base):
            assert np.array_equal(x, y), plan.variant_name(v)
    return base


@pytest.mark.parametrize("shape,radius", [((20, 40, 70), 4), ((50, 77), 2)])
def test_point_sources_at_one_grid_point(device, shape, radius):
    """Several sources at one point are applied one after another in index
    order by every kernel (the point kernel's injection groups them)."""
    u0, um1, beta = wave_inputs(shape, seed=101)
    hi = [n - 1 for n in shape]
    a, b = [n // 2 for n in shape], [3] * len(shape)
    src = np.array([a, a, b, hi, a, b])
    rec = np.array([a, b])
    amp = np.random.default_rng(102).standard_normal((9, len(src)))
    plan = _plan(shape, radius)
    base = _all_variants_equal(plan, lambda v: gpu_wave(plan, u0, um1, beta, 9, src=src, amp=amp, rec=rec,
                                                        variant=v))
    ref = oracle_wave(u0, um1, beta, radius, radius, 9, src=src, amp=amp, rec=rec)
    for x, y in zip(base, ref):
        assert rel_err(x, y) <= 1e-5


def _gpu_interp(plan, u0, um1, beta, nsteps, src, amp, rec, variant, device):
    import torch
    h = plan.halo
    f = [plan.field(device) for _ in range(3)]
    for fi, a in zip(f, (u0, um1, beta)):
        fi.load(W.embed(a, h))
    plan.variant = variant
    tr = torch.zeros((nsteps, len(rec)), dtype=torch.float64, device=device)
    plan.run_interp(f, nsteps, src=src, src_amp=torch_f64(amp, device), rec=rec, rec_trace=tr)
    torch.cuda.synchronize()
    return f[0].interior(h), f[1].interior(h), tr.cpu().numpy()


def _oracle_interp(u0, um1, beta, radius, nsteps, src, amp, rec):
    shape = u0.shape
    nd, nc = len(shape), 1 << len(shape)
    cs, ws = oracle.interp(shape, src)
    cr, wr = oracle.interp(shape, rec)
    amp8 = (np.asarray(amp)[:, :, None] * ws[None]).reshape(nsteps, -1)
    a, b, tr8 = oracle_wave(u0, um1, beta, radius, radius, nsteps, src=cs.reshape(-1, nd), amp=amp8,
                            rec=cr.reshape(-1, nd))
    return a, b, (tr8.reshape(nsteps, len(rec), nc) * wr[None]).sum(-1)


@pytest.mark.parametrize("shape,radius", [((30, 41, 66), 4), ((45, 70), 2), ((2, 9, 70), 1)])
def test_interpolated_sources_and_receivers(device, shape, radius):
    rng = np.random.default_rng(111 + len(shape))
    nd = len(shape)
    u0, um1, beta = wave_inputs(shape, seed=112)
    hi = np.array(shape, dtype=np.float64) - 1
    src = rng.uniform(0, 1, (5, nd)) * hi
    src[0] = hi                        # the upper corner of the grid
    src[1] = np.floor(src[1])          # a grid point
    src[3] = src[2]                    # two sources at one position
    rec = rng.uniform(0, 1, (4, nd)) * hi
    rec[0] = src[0]
    rec[1] = 0
    amp = rng.standard_normal((12, len(src)))
    plan = _plan(shape, radius)
    base = _all_variants_equal(plan, lambda v: _gpu_interp(plan, u0, um1, beta, 12, src, amp, rec, v, device))
    ref = _oracle_interp(u0, um1, beta, radius, 12, src, amp, rec)
    for x, y in zip(base, ref):
        assert rel_err(x, y) <= 1e-5
    assert np.abs(base[2]).max() > 0


def test_interpolation_at_grid_points_equals_point_sources(device):
    shape = (20, 33, 40)
    u0, um1, beta = wave_inputs(shape, seed=121)
    src = np.array([[10, 16, 20], [19, 32, 39], [0, 0, 0], [10, 16, 20]])
    rec = np.array([[10, 16, 21], [19, 32, 39]])
    amp = np.random.default_rng(122).standard_normal((7, len(src)))
    plan = _plan(shape, 4)
    pts = gpu_wave(plan, u0, um1, beta, 7, src=src, amp=amp, rec=rec, variant=1)
    itp = _gpu_interp(plan, u0, um1, beta, 7, src.astype(np.float64), amp, rec.astype(np.float64), 1, device)
    for x, y in zip(pts, itp):
        assert np.array_equal(x, y)


def _gamma(shape, prof):
    g = np.zeros(shape)
    for a, p in enumerate(prof):
        g = g + p.reshape([-1 if b == a else 1 for b in range(len(shape))])
    return g


@pytest.mark.parametrize("shape,radius", [((30, 44, 70), 4), ((60, 90), 2)])
def test_absorbing_layer(device, shape, radius):
    u0, um1, beta = wave_inputs(shape, seed=131)
    prof = W.damping_profiles(shape, 6, 0.25)
    nd = len(shape)
    src = np.array([[n // 2 for n in shape], [1] * nd])
    rec = np.array([[n // 3 for n in shape], [n - 2 for n in shape]])
    amp = np.random.default_rng(132).standard_normal((10, 2))
    plan = _plan(shape, radius)
    undamped = gpu_wave(plan, u0, um1, beta, 10, src=src, amp=amp, rec=rec, variant=plan.variant_count() - 1)
    nvar = plan.variant_count()
    plan.set_damping(prof)
    # 3D: the temporally blocked variants take the layer too (both stages)
    assert any(plan.variant_name(v).startswith("tb2_") for v in range(plan.variant_count())) == (nd == 3)
    assert plan.variant_count() == nvar
    base = _all_variants_equal(plan, lambda v: gpu_wave(plan, u0, um1, beta, 10, src=src, amp=amp, rec=rec,
                                                        variant=v))
    c = oracle.fd_weights_float(2 * radius)
    h = radius
    a, b, tr = oracle.wave_run_damped(W.embed(u0, h), W.embed(um1, h), W.embed(beta, h),
                                      W.embed(_gamma(shape, prof), h), h, radius, c, 10, src=src, src_amp=amp,
                                      rec=rec)
    for x, y in zip(base, (W.interior_of(a, h), W.interior_of(b, h), tr)):
        assert rel_err(x, y) <= 1e-5
    assert not np.array_equal(base[0], undamped[0])
    # the adjoint path refuses a damped plan
    nb = C.c_size_t()
    assert S.lib().stencil_adjoint_workspace(plan.handle, 10, 2, C.byref(nb)) == -2
    # a zero profile is the undamped sweep bit for bit, and so is removing
    # the layer
    plan.set_damping([np.zeros(n) for n in shape])
    v1 = min(1, plan.variant_count() - 1)
    zero = gpu_wave(plan, u0, um1, beta, 10, src=src, amp=amp, rec=rec, variant=v1)
    plan.set_damping(None)
    assert plan.variant_count() == nvar
    plain = gpu_wave(plan, u0, um1, beta, 10, src=src, amp=amp, rec=rec, variant=v1)
    for x, y in zip(zero, plain):
        assert np.array_equal(x, y)
    for x, y in zip(plain, undamped):
        assert np.array_equal(x, y)
