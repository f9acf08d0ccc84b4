"""GPU parity of the checkpointed adjoint: traces, misfit gradient against
the FP64 oracle's gradient, and the gradient against central differences of
the GPU misfit."""
import numpy as np
import pytest

import oracle
import paper_2404_02218_amd as S
import workloads as W
from _helpers import torch_f64

pytestmark = pytest.mark.gpu


def _problem(shape=(34, 30, 38), steps=110, seed=131):
    rng = np.random.default_rng(seed)
    h = 10.0
    v0 = W.layered_velocity(rng, shape)
    vt = v0 * (1 + 0.2 * W.gaussian_bump(shape, 6.0))
    dt = W.wave_dt(max(v0.max(), vt.max()), h)
    src = np.array([[4, shape[1] // 2, shape[2] // 2]])
    rec = np.array([[3, shape[1] // 2, x] for x in range(3, shape[2] - 3, 4)])
    w = W.ricker(np.arange(steps) * dt, f0=40.0)
    return dict(shape=shape, h=h, dt=dt, v0=v0, vt=vt, src=src, rec=rec, w=w, steps=steps)


def _oracle(P, m, dobs):
    dt, h = P["dt"], P["h"]
    beta = W.round_to_storage(dt * dt / (h * h * m), "f32")
    amp = (dt * dt / m[tuple(P["src"][0])] * P["w"]).reshape(-1, 1)
    rec_w = np.array([dt * dt / m[tuple(p)] for p in P["rec"]])
    return oracle.wave_gradient(W.embed(beta, 4), 4, 4, oracle.fd_weights_float(8), P["steps"],
                                P["src"], amp, P["rec"], dobs, rec_w, -1.0 / (dt * dt))


def _gpu(P, m, dobs, every, device, want_grad=True):
    import torch
    dt, h, steps = P["dt"], P["h"], P["steps"]
    plan = S.Plan(S.WAVE2, P["shape"], 4, S.second_derivative_weights(8), halo=4)
    f = [plan.field() for _ in range(3)]
    beta = W.round_to_storage(dt * dt / (h * h * m), "f32")
    f[2].load(W.embed(beta, 4))
    amp = torch_f64((dt * dt / m[tuple(P["src"][0])] * P["w"]).reshape(-1, 1), device)
    nrec = len(P["rec"])
    tr = torch.zeros((steps, nrec), dtype=torch.float64, device=device)
    ws = torch.empty(plan.adjoint_workspace_bytes(steps, every), dtype=torch.uint8, device=device)
    plan.forward_ckpt(f, steps, every, ws, src=P["src"], src_amp=amp, rec=P["rec"], rec_trace=tr)
    d = tr.cpu().numpy()
    J = 0.5 * float(np.sum((d - dobs) ** 2))
    if not want_grad:
        return d, J, None
    resid = torch_f64(d - dobs, device)
    scale = torch_f64(np.array([dt * dt / m[tuple(p)] for p in P["rec"]]), device)
    grad = torch.zeros(P["shape"], dtype=torch.float64, device=device)
    beta_f = plan.field().load(W.embed(beta, 4))
    plan.adjoint(beta_f, steps, every, ws, resid, P["rec"], scale, dt, grad,
                 src=P["src"], src_amp=amp)
    torch.cuda.synchronize()
    return d, J, grad.cpu().numpy()


@pytest.mark.parametrize("every", [25, 7, 110])
def test_gradient_matches_oracle(device, every):
    P = _problem()
    nrec = len(P["rec"])
    dobs, _, _ = _oracle(P, 1 / P["vt"] ** 2, np.zeros((P["steps"], nrec)))
    m0 = 1 / P["v0"] ** 2
    rtr, rJ, rg = _oracle(P, m0, dobs)
    d, J, g = _gpu(P, m0, dobs, every, device)
    e_d = np.max(np.abs(d - rtr)) / np.max(np.abs(rtr))
    e_J = abs(J - rJ) / rJ
    e_g = np.linalg.norm(g - rg) / np.linalg.norm(rg)
    print(f"checkpoint every {every}: traces {e_d:.2e}, misfit {e_J:.2e}, gradient rel L2 {e_g:.2e}")
    assert e_d <= 1e-5
    # J and g are driven by residuals d - d_obs, smaller than d itself, so the
    # FP32 trace error is amplified by max|d| / |d - d_obs|; measured about
    # 1e-5 (misfit) and 5e-6 (gradient)
    assert e_J <= 1e-4
    assert e_g <= 1e-4


def test_gradient_matches_gpu_central_differences(device):
    P = _problem(shape=(30, 28, 32), steps=90, seed=137)
    nrec = len(P["rec"])
    dobs, _, _ = _oracle(P, 1 / P["vt"] ** 2, np.zeros((P["steps"], nrec)))
    m0 = 1 / P["v0"] ** 2
    _, J0, g = _gpu(P, m0, dobs, 25, device)
    dm = (1 / P["vt"] ** 2 - m0)
    gdm = float(np.sum(g * dm))
    eps = 1e-2
    _, Jp, _ = _gpu(P, m0 + eps * dm, dobs, 25, device, want_grad=False)
    _, Jm, _ = _gpu(P, m0 - eps * dm, dobs, 25, device, want_grad=False)
    fd = (Jp - Jm) / (2 * eps)
    print(f"J0 {J0:.6e}  FD {fd:.6e}  <g,dm> {gdm:.6e}  rel {abs(fd - gdm) / abs(gdm):.2e}")
    assert abs(fd - gdm) <= 1e-3 * abs(gdm)


def test_recompute_equals_forward_bitwise(device):
    """Checkpointed forward + adjoint with lambda driven by zero residuals
    leaves the gradient exactly zero, and splitting the forward into
    checkpoints does not change its traces."""
    import torch
    P = _problem(shape=(24, 20, 36), steps=40, seed=139)
    m0 = 1 / P["v0"] ** 2
    nrec = len(P["rec"])
    d1, _, _ = _gpu(P, m0, np.zeros((P["steps"], nrec)), 40, device, want_grad=False)
    d2, _, _ = _gpu(P, m0, np.zeros((P["steps"], nrec)), 3, device, want_grad=False)
    assert np.array_equal(d1, d2)
    _, _, g = _gpu(P, m0, d1, 6, device)
    assert np.all(g == 0.0)
    del torch


def test_autograd_function_matches_direct_calls_and_fd(device):
    import torch
    from paper_2404_02218_amd.wave import WaveModel
    P = _problem(shape=(30, 26, 34), steps=80, seed=141)
    nrec = len(P["rec"])
    dobs, _, _ = _oracle(P, 1 / P["vt"] ** 2, np.zeros((P["steps"], nrec)))
    model = WaveModel(P["shape"], P["h"], P["dt"], P["src"], P["w"], P["rec"], P["steps"], 20)
    m0 = torch_f64(1 / P["v0"] ** 2, device).requires_grad_(True)
    d_obs = torch_f64(dobs, device)
    d = model(m0)
    J = 0.5 * ((d - d_obs) ** 2).sum()
    J.backward()
    g = m0.grad.cpu().numpy()
    # the same computation through the direct ABI calls
    d2, J2, g2 = _gpu(P, 1 / P["v0"] ** 2, dobs, 20, device)
    # beta is rounded from FP64 on the host there and on the device here
    assert abs(float(J) - J2) <= 1e-6 * J2
    assert np.linalg.norm(g - g2) <= 1e-5 * np.linalg.norm(g2)
    dm = torch_f64(1 / P["vt"] ** 2 - 1 / P["v0"] ** 2, device)
    eps = 1e-2
    with torch.no_grad():
        Jp = 0.5 * ((model(m0 + eps * dm) - d_obs) ** 2).sum().item()
        Jm = 0.5 * ((model(m0 - eps * dm) - d_obs) ** 2).sum().item()
    gdm = float((m0.grad * dm).sum())
    fd = (Jp - Jm) / (2 * eps)
    print(f"autograd: FD {fd:.6e}  <g,dm> {gdm:.6e}  rel {abs(fd - gdm) / abs(gdm):.2e}")
    assert abs(fd - gdm) <= 1e-3 * abs(gdm)
    # a backward after a newer forward is refused
    d3 = model(m0)
    model(m0.detach())
    with pytest.raises(RuntimeError):
        (0.5 * (d3 ** 2).sum()).backward()


@pytest.mark.parametrize("steps,every", [(40, 1), (41, 1), (41, 41), (41, 7), (40, 6), (40, 39)])
def test_checkpointed_forward_equals_run_and_adjoint_repeats(device, steps, every):
    """The checkpointed forward sweeps from checkpoint to checkpoint in the
    workspace and into the caller's fields at the end: its final two levels
    and traces equal the plain run's bit for bit, also when the workspace
    starts filled with NaN bytes (only its interiors are ever written by the
    sweeps), and a second adjoint call on the same checkpoints gives the same
    gradient bits."""
    import torch
    P = _problem(shape=(26, 22, 34), steps=steps, seed=151)
    dt, h = P["dt"], P["h"]
    m0 = 1 / P["v0"] ** 2
    plan = S.Plan(S.WAVE2, P["shape"], 4, S.second_derivative_weights(8), halo=4)
    beta = W.round_to_storage(dt * dt / (h * h * m0), "f32")
    amp = torch_f64((dt * dt / m0[tuple(P["src"][0])] * P["w"]).reshape(-1, 1), device)
    nrec = len(P["rec"])

    def fields():
        f = [plan.field() for _ in range(3)]
        f[2].load(W.embed(beta, 4))
        return f

    fr = fields()
    tr_run = torch.zeros((steps, nrec), dtype=torch.float64, device=device)
    plan.run(fr, steps, src=P["src"], src_amp=amp, rec=P["rec"], rec_trace=tr_run)
    fc = fields()
    tr = torch.zeros((steps, nrec), dtype=torch.float64, device=device)
    ws = torch.full((plan.adjoint_workspace_bytes(steps, every),), 0xFF, dtype=torch.uint8, device=device)
    plan.forward_ckpt(fc, steps, every, ws, src=P["src"], src_amp=amp, rec=P["rec"], rec_trace=tr)
    torch.cuda.synchronize()
    for i in (0, 1):
        assert np.array_equal(fc[i].to_numpy().view(np.uint32), fr[i].to_numpy().view(np.uint32)), i
    assert np.array_equal(tr.cpu().numpy(), tr_run.cpu().numpy())

    resid = tr.clone()
    scale = torch_f64(np.array([dt * dt / m0[tuple(p)] for p in P["rec"]]), device)
    grads = []
    for _ in range(2):
        g = torch.zeros(P["shape"], dtype=torch.float64, device=device)
        plan.adjoint(fc[2], steps, every, ws, resid, P["rec"], scale, dt, g, src=P["src"], src_amp=amp)
        torch.cuda.synchronize()
        grads.append(g.cpu().numpy())
    assert np.all(np.isfinite(grads[0])) and np.any(grads[0] != 0)
    assert np.array_equal(grads[0], grads[1])
