"""Every workload configuration at its specified size and step count against
the FP64 oracle, in the launch configuration the benchmark times (the tuned
variant), with the error metric of the method's precision study: the largest
|gpu - oracle| over the compared levels divided by the largest |oracle| over
the same levels (levels every 25 steps and the last one).

  * so-8 wave 512^3 x 400 steps for FP32, BF16 and FP16 storage (the oracle
    is fed the storage-rounded velocity term, so the error isolates the
    kernel's arithmetic and its storage of the levels);
  * 32 batched shots of uneven sizes, 200 steps each, every shot against its
    own oracle run (levels and receiver traces);
  * the checkpointed misfit gradient, 500 steps, a checkpoint every 25 steps,
    64 receivers, against the oracle's gradient of the same discrete
    recurrence (relative L2), at 256^3 as configured (the oracle keeps every
    forward level in FP64: 74 GB of host memory) and at 128^3 with the
    oracle's own gradient pinned to central differences of its misfit.

The oracle needs about 40 s per 512^3 x 400-step run on 16 host threads."""
import numpy as np
import pytest

import oracle
import paper_2404_02218_amd as S
import workloads as W
from _helpers import rel_err, torch_f64

pytestmark = pytest.mark.gpu

C8 = None


def _c8():
    global C8
    if C8 is None:
        C8 = oracle.fd_weights_float(8)
    return C8


# Bounds over the whole 400-step run.  FP32: the configured 1e-5.  16-bit
# storage rounds every new level (unit roundoff 2^-8 for BF16, 2^-11 for
# FP16), and that rounding accumulates over the run; the bounds are about 3x
# the errors measured at this size (BF16 1.9e-2, FP16 1.4e-3).
C3_BOUND = {"f32": 1e-5, "f16": 5e-3, "bf16": 6e-2}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dn", ["f32", "f16", "bf16"])
def test_c3_whole_run_matches_oracle(device, dn):
    import torch
    P = W.wave3d_c3()
    every = 25
    plan = S.Plan(S.WAVE2, P.shape, 4, S.second_derivative_weights(8), halo=4, dtype=S.DTYPES[dn])
    f = [plan.field() for _ in range(3)]
    beta = W.round_to_storage(P.beta, dn)
    f[2].load(W.embed(beta, 4))
    plan.tune(f, reps=2)
    vname = plan.variant_name(plan.variant)
    amp_all = torch_f64(P.src_amp, device)
    # the run the benchmark times: all 400 steps in one call
    plan.run(f, P.nsteps, src=P.src, src_amp=amp_all)
    torch.cuda.synchronize()
    whole = [f[0].storage.clone(), f[1].storage.clone()]
    f[0].zero()
    f[1].zero()
    bb = W.embed(beta, 4)
    a = np.zeros_like(bb)
    b = np.zeros_like(bb)
    num = den = 0.0
    for t0 in range(0, P.nsteps, every):
        k = min(every, P.nsteps - t0)
        amp = P.src_amp[t0:t0 + k]
        plan.run(f, k, src=P.src, src_amp=torch_f64(amp, device))
        torch.cuda.synchronize()
        got = f[0].interior(4)
        a, b, _ = oracle.wave_run(a, b, bb, 4, 4, _c8(), k, src=P.src, src_amp=amp)
        ref = W.interior_of(a, 4)
        num = max(num, float(np.max(np.abs(got - ref))))
        den = max(den, float(np.max(np.abs(ref))))
        del got, ref
    final = rel_err(f[0].interior(4), W.interior_of(a, 4))
    err = num / den
    print(f"C3 {dn} 512^3 x {P.nsteps}, {vname}: {err:.3e} over the run, final level alone {final:.3e}")
    # segmented runs give the single run's bits (the tested split invariant)
    assert torch.equal(f[0].storage, whole[0]) and torch.equal(f[1].storage, whole[1])
    assert den > 0
    assert err <= C3_BOUND[dn]


@pytest.fixture(scope="module")
def c4_run(device):
    """The 32 shots, tuned and run for 200 steps in one batched call, with a
    receiver above each source."""
    import torch
    B = W.batch_c4()
    bp = S.BatchPlan([s.shape for s in B.shots], 4, S.second_derivative_weights(8))
    fields, amps, recs, trs = [], [], [], []
    for i, sh in enumerate(B.shots):
        g = [bp.field(i) for _ in range(3)]
        g[2].load(W.embed(W.round_to_storage(sh.beta, "f32"), 4))
        fields.append(g)
        amps.append(torch_f64(sh.src_amp, device))
        s = sh.src[0]
        recs.append(np.array([[max(0, s[0] - 6), s[1], s[2]], [s[0], s[1], s[2]]]))
        trs.append(torch.zeros((B.nsteps, 2), dtype=torch.float64, device=device))
    bp.tune(fields, reps=1)
    bp.run(fields, B.nsteps, [sh.src for sh in B.shots], amps, recs, trs)
    torch.cuda.synchronize()
    yield B, bp, fields, recs, trs
    del fields, trs
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("group", range(4))
def test_c4_batched_200_steps_match_oracle(c4_run, group):
    """Shots 8g .. 8g+7 of the batched run against their own oracle runs:
    the last two levels and the receiver traces, each within 1e-5."""
    B, bp, fields, recs, trs = c4_run
    for i in range(8 * group, 8 * group + 8):
        sh = B.shots[i]
        beta = W.embed(W.round_to_storage(sh.beta, "f32"), 4)
        z = np.zeros_like(beta)
        a, b, rtr = oracle.wave_run(z, z, beta, 4, 4, _c8(), B.nsteps, src=sh.src, src_amp=sh.src_amp,
                                    rec=recs[i])
        e0 = rel_err(fields[i][0].interior(4), W.interior_of(a, 4))
        e1 = rel_err(fields[i][1].interior(4), W.interior_of(b, 4))
        et = rel_err(trs[i].cpu().numpy(), rtr)
        print(f"C4 shot {i} {sh.shape[0]}^3, {bp.variant_name(bp.variant)}: "
              f"u^N {e0:.2e}, u^(N-1) {e1:.2e}, traces {et:.2e}")
        assert e0 <= 1e-5 and e1 <= 1e-5 and et <= 1e-5, i


@pytest.mark.timeout(900)
def test_c5_full_config_gradient_matches_oracle_gradient(device):
    """The gradient configuration as specified: 256^3, 500 steps, a
    checkpoint every 25, 64 receivers, through the single-call misfit
    gradient, against the oracle's gradient (which keeps all 502 FP64
    levels: 74 GB of host memory), fed the beta the GPU formed."""
    import torch
    P = W.inversion_c5()
    N, k, dt, h = P.nsteps, P.checkpoint_every, P.dt, P.h
    nrec = len(P.rec)
    assert P.shape == (256, 256, 256) and nrec == 64 and k == 25 and N == 500
    amp = lambda m: (dt * dt / m[tuple(P.src[0])] * P.wavelet).reshape(-1, 1)  # noqa: E731
    bt = W.embed(W.round_to_storage(dt * dt / (h * h * P.m_true), "f32"), 4)
    z = np.zeros_like(bt)
    dobs = oracle.wave_run(z, z, bt, 4, 4, _c8(), N, src=P.src, src_amp=amp(P.m_true), rec=P.rec)[2]
    del bt, z
    m0 = P.m0
    plan = S.Plan(S.WAVE2, P.shape, 4, S.second_derivative_weights(8), halo=4)
    f = [plan.field() for _ in range(3)]
    ws = torch.empty(plan.adjoint_workspace_bytes(N, k), dtype=torch.uint8, device=device)
    tr = torch.zeros((N, nrec), dtype=torch.float64, device=device)
    misfit = torch.zeros(1, dtype=torch.float64, device=device)
    g = torch.empty(P.shape, dtype=torch.float64, device=device)
    plan.gradient(f, torch_f64(m0, device), dt, h, N, k, ws, P.src, torch_f64(P.wavelet.reshape(-1, 1), device),
                  P.rec, tr, torch_f64(dobs, device), misfit, g)
    torch.cuda.synchronize()
    beta_gpu = W.embed(f[2].interior(4), 4)
    del f, ws
    torch.cuda.empty_cache()
    rtr, rJ, rg = oracle.wave_gradient(beta_gpu, 4, 4, _c8(), N, P.src, amp(m0), P.rec, dobs,
                                       np.array([dt * dt / m0[tuple(p)] for p in P.rec]), -1.0 / (dt * dt))
    d = tr.cpu().numpy()
    e_d = rel_err(d, rtr)
    e_J = abs(float(misfit.item()) - rJ) / rJ
    gg = g.cpu().numpy()
    e_g = float(np.linalg.norm(gg - rg) / np.linalg.norm(rg))
    print(f"C5 256^3 x {N}, checkpoint {k}: traces {e_d:.2e}, misfit {e_J:.2e} (J {rJ:.6e}), "
          f"gradient rel L2 {e_g:.2e}")
    assert rJ >= 1e-4 * 0.5 * float(np.sum(rtr ** 2))   # the data see the anomaly
    assert e_d <= 1e-5
    assert e_J <= 1e-4
    assert e_g <= 1e-4


@pytest.mark.timeout(900)
def test_c5_gradient_500_steps_matches_oracle_gradient(device):
    """500 steps, a checkpoint every 25, 64 receivers, the gradient workload's
    geometry on a 128^3 grid, through the single-call misfit gradient (the
    library forms beta, the source amounts and the receiver weights from m):
    traces, misfit and gradient against the oracle's (which keeps every
    level), fed the beta the GPU stored; and the FP64 oracle gradient against
    central differences of the oracle misfit."""
    import torch
    P = W.inversion_c5(n=128)
    N, k, dt, h = P.nsteps, P.checkpoint_every, P.dt, P.h
    nrec = len(P.rec)
    assert nrec == 64 and len({tuple(r) for r in P.rec}) == 64

    def src_amp(m):
        return (dt * dt / m[tuple(P.src[0])] * P.wavelet).reshape(-1, 1)

    rec_w = lambda m: np.array([dt * dt / m[tuple(p)] for p in P.rec])  # noqa: E731

    def oracle_grad(beta, m, dobs):
        return oracle.wave_gradient(W.embed(beta, 4), 4, 4, _c8(), N, P.src, src_amp(m), P.rec, dobs, rec_w(m),
                                    -1.0 / (dt * dt))

    zero = np.zeros((N, nrec))
    dobs, _, _ = oracle_grad(W.round_to_storage(dt * dt / (h * h * P.m_true), "f32"), P.m_true, zero)
    m0 = P.m0

    plan = S.Plan(S.WAVE2, P.shape, 4, S.second_derivative_weights(8), halo=4)
    f = [plan.field() for _ in range(3)]
    m_dev = torch_f64(m0, device)
    plan.wave_beta(m_dev, dt, h, f[2])
    plan.tune(f, reps=2)
    ws = torch.empty(plan.adjoint_workspace_bytes(N, k), dtype=torch.uint8, device=device)
    tr = torch.zeros((N, nrec), dtype=torch.float64, device=device)
    misfit = torch.zeros(1, dtype=torch.float64, device=device)
    g = torch.empty(P.shape, dtype=torch.float64, device=device)
    plan.gradient(f, m_dev, dt, h, N, k, ws, P.src, torch_f64(P.wavelet.reshape(-1, 1), device), P.rec, tr,
                  torch_f64(dobs, device), misfit, g)
    torch.cuda.synchronize()
    beta_gpu = f[2].interior(4)
    rtr, rJ, rg = oracle_grad(beta_gpu, m0, dobs)
    d = tr.cpu().numpy()
    J = float(misfit.item())
    g = g.cpu().numpy()
    e_d = rel_err(d, rtr)
    e_J = abs(J - rJ) / rJ
    e_g = float(np.linalg.norm(g - rg) / np.linalg.norm(rg))
    # the oracle gradient against central differences of the oracle misfit,
    # all in FP64 (beta unrounded: FP32 rounding of beta would put noise of
    # relative size 2^-24 / eps into the differences)
    dm = P.m_true - m0
    eps = 1e-3
    b64 = lambda m: dt * dt / (h * h * m)  # noqa: E731
    _, _, g64 = oracle_grad(b64(m0), m0, dobs)
    _, Jp, _ = oracle_grad(b64(m0 + eps * dm), m0 + eps * dm, dobs)
    _, Jm, _ = oracle_grad(b64(m0 - eps * dm), m0 - eps * dm, dobs)
    fd = (Jp - Jm) / (2 * eps)
    gdm64 = float(np.sum(g64 * dm))
    del g64
    print(f"C5 128^3 x {N}, checkpoint {k}, {plan.variant_name(plan.variant)}: traces {e_d:.2e}, "
          f"misfit {e_J:.2e}, gradient rel L2 {e_g:.2e}; FP64 oracle: FD {fd:.8e} vs <g, dm> {gdm64:.8e}")
    assert rJ >= 1e-4 * 0.5 * float(np.sum(rtr ** 2))   # the data see the anomaly
    assert e_d <= 1e-5
    assert e_J <= 1e-4
    assert e_g <= 1e-4
    assert abs(fd - gdm64) <= 1e-5 * abs(gdm64)
