"""Parity at the full workload sizes, in the tuned launch configuration the
benchmark times.  A whole multi-step run at 512^3 is beyond what the FP64
oracle finishes in seconds, so these check what holds at any size:
  * one sweep from random levels (plus a source) over the whole 512^3 field
    against the oracle's one-step update computed everywhere;
  * the exact light cone after many steps from a zero start;
  * the 512^3 x 50-step heat in its tuned variant against the whole oracle
    run (the 13-point heat is cheap enough for the oracle at full size);
  * batched == sequential (bitwise) for the 32 uneven shots;
  * the 256^3 x 500-step checkpointed gradient against central differences of
    the GPU misfit, with observed data from the FP64 oracle, and the traces
    against the oracle's."""
import numpy as np
import pytest

import oracle
import paper_2404_02218_amd as S
import workloads as W
from _helpers import gpu_heat, rel_err, torch_f64

pytestmark = pytest.mark.gpu


def _tuned_wave(P, dtype=S.F32, dn="f32"):
    plan = S.Plan(S.WAVE2, P.shape, 4, S.second_derivative_weights(8), halo=4, dtype=dtype)
    f = [plan.field() for _ in range(3)]
    f[2].load(W.embed(W.round_to_storage(P.beta, dn), 4))
    plan.tune(f, reps=2)
    return plan, f


# One sweep rounds the new level once to storage, and the source point once
# more after the FP64 addition: each point is off by at most two unit
# roundoffs of the largest level value (2^-8 BF16, 2^-11 FP16), plus FP32
# arithmetic (well below 1e-5 of it).
ONE_SWEEP_BOUND = {"f32": 1e-6, "bf16": 2 * 2.0 ** -8 + 1e-5, "f16": 2 * 2.0 ** -11 + 1e-5}


@pytest.mark.parametrize("dn", ["f32", "bf16", "f16"])
def test_c3_full_size_one_sweep_everywhere(device, dn):
    import torch
    dtype = S.DTYPES[dn]
    P = W.wave3d_c3(nsteps=1)
    plan, f = _tuned_wave(P, dtype, dn)
    rng = np.random.default_rng(2024)
    u = W.round_to_storage(rng.standard_normal(P.shape).astype(np.float32), dn)
    up = W.round_to_storage(rng.standard_normal(P.shape).astype(np.float32), dn)
    f[0].load(W.embed(u, 4))
    f[1].load(W.embed(up, 4))
    amp = np.array([[3.5]])
    plan.run(f, 1, src=P.src, src_amp=torch_f64(amp, device))
    torch.cuda.synchronize()
    got = f[0].interior(4)
    beta = W.embed(W.round_to_storage(P.beta, dn), 4)
    ub = W.embed(u, 4)
    Lu = W.interior_of(oracle.star(ub, 4, 4, oracle.fd_weights_float(8)), 4)
    ref = 2 * u - up + W.interior_of(beta, 4) * Lu
    ref[tuple(P.src[0])] += 3.5
    err = rel_err(got, ref)
    print(f"{dn}: one sweep at 512^3, variant {plan.variant_name(plan.variant)}: {err:.2e}")
    assert err <= ONE_SWEEP_BOUND[dn]


def test_c3_full_size_light_cone_after_40_steps(device):
    import torch
    P = W.wave3d_c3(nsteps=40)
    plan, f = _tuned_wave(P)
    plan.run(f, 40, src=P.src, src_amp=torch_f64(P.src_amp, device))
    torch.cuda.synchronize()
    a = f[0].interior(4)
    s = P.src[0]
    n = P.shape[0]
    ax = np.arange(n)
    hz = np.ceil(np.abs(ax - s[0]) / 4)
    hy = np.ceil(np.abs(ax - s[1]) / 4)
    hx = np.ceil(np.abs(ax - s[2]) / 4)
    hops = hz[:, None, None] + hy[None, :, None] + hx[None, None, :]
    assert np.all(a[hops > 39] == 0.0)
    assert np.count_nonzero(a) > 0


def test_c3_full_size_multi_step_matches_oracle_on_a_slab(device):
    """60 steps at 512^3 with the source at z = 8.  The stencil moves
    information at most 4 cells per step, so every level stays exactly zero
    beyond z = 8 + 4*59; the full-grid run therefore equals a run on the slab
    z < 256 with a zero halo above it, which the oracle finishes in seconds."""
    import torch
    steps = 60
    P = W.wave3d_c3(nsteps=steps)
    plan, f = _tuned_wave(P)
    src = np.array([[8, 256, 256]])
    amp = W.source_amplitudes(W.ricker(np.arange(steps) * P.dt), P.dt,
                              float(P.velocity[8, 256, 256])).reshape(-1, 1)
    plan.run(f, steps, src=src, src_amp=torch_f64(amp, device))
    torch.cuda.synchronize()
    full = f[0].interior(4)
    reach = 8 + 4 * (steps - 1)
    assert np.all(full[reach + 1:] == 0.0)
    got = full[:256]
    b = W.embed(W.round_to_storage(P.beta, "f32")[:256], 4)
    z = np.zeros_like(b)
    a, _, _ = oracle.wave_run(z, z, b, 4, 4, oracle.fd_weights_float(8), steps, src=src, src_amp=amp)
    err = rel_err(got, W.interior_of(a, 4))
    print(f"{steps} steps at 512^3 vs oracle on z < 256: {err:.2e}")
    assert err <= 1e-5


def test_c2_full_size_tuned_run_matches_oracle(device):
    """The 512^3 so-4 heat, 50 steps, in the variant the tuner picks (the
    configuration the benchmark times), against the whole FP64 oracle run;
    the tuned run also gives the plain sweep's bits."""
    import torch
    P = W.heat3d_c2()
    u0 = W.round_to_storage(P.u0, "f32")
    plan = S.Plan(S.HEAT, P.shape, 2, S.heat_weights(4, P.alpha), halo=2)
    f = [plan.field() for _ in range(2)]
    f[0].load(W.embed(u0, 2))
    plan.tune(f, reps=2)
    tuned = plan.variant_name(plan.variant)
    got = gpu_heat(plan, u0, P.nsteps)
    plain = gpu_heat(plan, u0, P.nsteps, variant=2)
    assert np.array_equal(got, plain), tuned
    del f, plain
    torch.cuda.empty_cache()
    c = [P.alpha * x for x in oracle.fd_weights_float(4)]
    ref = W.interior_of(oracle.heat_run(W.embed(u0, 2), 2, 2, c, P.nsteps), 2)
    err = rel_err(got, ref)
    print(f"C2 512^3 x {P.nsteps}, {tuned}: {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("dn", ["f32", "bf16", "f16"])
def test_c3_full_size_temporal_blocking_equals_plain_sweep(device, dn):
    """Six steps over the whole 512^3 field from random levels with the
    Ricker source: every temporally blocked variant (two-step passes, plus
    plain steps for the remainder) gives the plain sweep's bits."""
    import torch
    dtype = S.DTYPES[dn]
    P = W.wave3d_c3(nsteps=6)
    plan = S.Plan(S.WAVE2, P.shape, 4, S.second_derivative_weights(8), halo=4, dtype=dtype)
    rng = np.random.default_rng(2025)
    levels = [W.embed(W.round_to_storage(rng.standard_normal(P.shape).astype(np.float32), dn), 4)
              for _ in range(2)]
    beta = W.embed(W.round_to_storage(P.beta, dn), 4)
    amp = torch_f64(P.src_amp[:6], device)

    def run(variant):
        f = [plan.field() for _ in range(3)]
        f[0].load(levels[0])
        f[1].load(levels[1])
        f[2].load(beta)
        plan.variant = variant
        plan.run(f, 6, src=P.src, src_amp=amp)
        torch.cuda.synchronize()
        return f
    base = run(2)
    for v in range(plan.variant_count()):
        if not plan.variant_name(v).startswith("tb2_"):
            continue
        got = run(v)
        for a, b in zip(got[:2], base[:2]):
            assert torch.equal(a.storage, b.storage), plan.variant_name(v)
        del got


@pytest.mark.parametrize("variant", [None, "persistent_zmarch_64x16_t256_zc32_nt"])
def test_c4_full_size_batched_equals_sequential(device, variant):
    # the tuned batch variant from zero levels, and the persistent launch
    # (grid barriers between steps) from random levels, so that every halo
    # row a tile reads from a neighbour processed elsewhere carries data
    import torch
    B = W.batch_c4(nsteps=6)
    shapes = [s.shape for s in B.shots]
    bp = S.BatchPlan(shapes, 4, S.second_derivative_weights(8))
    fields, amps, recs, trs = [], [], [], []
    gen = torch.Generator(device=device).manual_seed(7)
    for i, sh in enumerate(B.shots):
        g = [bp.field(i) for _ in range(3)]
        g[2].load(W.embed(W.round_to_storage(sh.beta, "f32"), 4))
        if variant is not None:
            for k in (0, 1):
                g[k].view[4:-4, 4:-4, 4:-4] = torch.rand(sh.shape, generator=gen, device=device) - 0.5
        fields.append(g)
        amps.append(torch_f64(sh.src_amp, device))
        recs.append(np.array([[8, sh.shape[1] // 2, sh.shape[2] // 2]]))
        trs.append(torch.zeros((6, 1), dtype=torch.float64, device=device))
    init = [[f[k].storage.clone() for k in (0, 1)] for f in fields]
    if variant is None:
        bp.tune(fields, reps=1)
    else:
        bp.variant = next(v for v in range(bp.variant_count()) if bp.variant_name(v) == variant)
    bp.run(fields, 6, [sh.src for sh in B.shots], amps, recs, trs)
    torch.cuda.synchronize()
    for i, sh in enumerate(B.shots):
        p = S.Plan(S.WAVE2, sh.shape, 4, S.second_derivative_weights(8), halo=4)
        g = [p.field() for _ in range(3)]
        g[0].storage.copy_(init[i][0])
        g[1].storage.copy_(init[i][1])
        g[2].storage.copy_(fields[i][2].storage)
        t = torch.zeros((6, 1), dtype=torch.float64, device=device)
        p.run(g, 6, src=sh.src, src_amp=amps[i], rec=recs[i], rec_trace=t)
        torch.cuda.synchronize()
        assert torch.equal(g[0].storage, fields[i][0].storage), i
        assert torch.equal(g[1].storage, fields[i][1].storage), i
        assert torch.equal(t, trs[i]), i


def test_c5_full_size_gradient(device):
    import torch
    P = W.inversion_c5()
    N, k = P.nsteps, P.checkpoint_every
    dt, h = P.dt, P.h
    nrec = len(P.rec)
    c8 = oracle.fd_weights_float(8)

    def oracle_traces(m):
        beta = W.embed(W.round_to_storage(dt * dt / (h * h * m), "f32"), 4)
        amp = (dt * dt / m[tuple(P.src[0])] * P.wavelet).reshape(-1, 1)
        z = np.zeros_like(beta)
        return oracle.wave_run(z, z, beta, 4, 4, c8, N, src=P.src, src_amp=amp, rec=P.rec)[2]

    dobs = oracle_traces(P.m_true)
    plan = S.Plan(S.WAVE2, P.shape, 4, S.second_derivative_weights(8), halo=4)
    ws = torch.empty(plan.adjoint_workspace_bytes(N, k), dtype=torch.uint8, device=device)

    def gpu(m, grad=True):
        f = [plan.field() for _ in range(3)]
        f[2].load(W.embed(W.round_to_storage(dt * dt / (h * h * m), "f32"), 4))
        amp = torch_f64((dt * dt / m[tuple(P.src[0])] * P.wavelet).reshape(-1, 1), device)
        tr = torch.zeros((N, nrec), dtype=torch.float64, device=device)
        plan.forward_ckpt(f, N, k, ws, src=P.src, src_amp=amp, rec=P.rec, rec_trace=tr)
        d = tr.cpu().numpy()
        J = 0.5 * float(np.sum((d - dobs) ** 2))
        if not grad:
            return d, J, None
        g = torch.zeros(P.shape, dtype=torch.float64, device=device)
        scale = torch_f64(np.array([dt * dt / m[tuple(p)] for p in P.rec]), device)
        plan.adjoint(f[2], N, k, ws, torch_f64(d - dobs, device), P.rec, scale, dt, g,
                     src=P.src, src_amp=amp)
        torch.cuda.synchronize()
        return d, J, g.cpu().numpy()

    m0 = P.m0
    d0, J0, g = gpu(m0)
    ref0 = oracle_traces(m0)
    e_tr = rel_err(d0, ref0)
    dm = P.m_true - m0
    gdm = float(np.sum(g * dm))
    eps = 0.05
    _, Jp, _ = gpu(m0 + eps * dm, grad=False)
    _, Jm, _ = gpu(m0 - eps * dm, grad=False)
    fd = (Jp - Jm) / (2 * eps)
    print(f"C5 256^3 x 500: traces vs oracle {e_tr:.2e}; J0 {J0:.6e}; FD {fd:.6e}; <g,dm> {gdm:.6e}; "
          f"rel {abs(fd - gdm) / abs(gdm):.2e}")
    assert e_tr <= 1e-5
    # the data must see the perturbation: a misfit far above FP32 noise
    assert J0 >= 1e-4 * 0.5 * float(np.sum(ref0 ** 2))
    assert abs(gdm) > 0 and abs(fd) > 0
    assert abs(fd - gdm) <= 1e-3 * abs(gdm)
