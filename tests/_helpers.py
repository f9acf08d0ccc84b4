"""Shared helpers of the GPU parity tests: run the same seeded inputs through
the library (C ABI) and through the FP64 oracle, and compare."""
from __future__ import annotations

import numpy as np

import oracle
import paper_2404_02218_amd as S
import workloads as W

DT_NAMES = {S.F32: "f32", S.BF16: "bf16", S.F16: "f16"}


def rel_err(gpu, ref) -> float:
    """max |gpu - ref| / max |ref| (the normwise reading of a max-relative error)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref))
    if den == 0:
        return float(np.max(np.abs(gpu)))
    return float(np.max(np.abs(gpu - ref)) / den)


def torch_f64(a, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)


def wave_inputs(shape, seed, dtype=S.F32, halo=4, random_state=True, beta_range=(0.005, 0.05)):
    """Storage-rounded (u0, um1, beta) interiors for a wave test."""
    rng = np.random.default_rng(seed)
    dn = DT_NAMES[dtype]
    beta = W.round_to_storage(rng.uniform(*beta_range, shape), dn)
    if random_state:
        u0 = W.round_to_storage(rng.standard_normal(shape), dn)
        um1 = W.round_to_storage(u0 + 0.01 * rng.standard_normal(shape), dn)
    else:
        u0 = np.zeros(shape)
        um1 = np.zeros(shape)
    return u0, um1, beta


def gpu_wave(plan, u0, um1, beta, nsteps, src=None, amp=None, rec=None, variant=None,
             device="cuda", split=None):
    """Run the wave on the GPU; returns (u^N, u^{N-1}, traces) interiors."""
    import torch
    h = plan.halo
    f = [plan.field(device) for _ in range(3)]
    f[0].load(W.embed(u0, h))
    f[1].load(W.embed(um1, h))
    f[2].load(W.embed(beta, h))
    if variant is not None:
        plan.variant = variant
    nrec = 0 if rec is None else len(rec)
    tr = torch.zeros((nsteps, nrec), dtype=torch.float64, device=device) if nrec else None
    amp_t = torch_f64(amp, device) if src is not None else None
    if split is None:
        plan.run(f, nsteps, src=src, src_amp=amp_t, rec=rec, rec_trace=tr)
    else:
        done = 0
        for part in split:
            a_t = amp_t[done:done + part].contiguous() if amp_t is not None else None
            t_t = (torch.zeros((part, nrec), dtype=torch.float64, device=device) if nrec else None)
            plan.run(f, part, src=src, src_amp=a_t, rec=rec, rec_trace=t_t)
            if nrec:
                tr[done:done + part] = t_t
            done += part
    torch.cuda.synchronize()
    return f[0].interior(h), f[1].interior(h), (tr.cpu().numpy() if nrec else None)


def oracle_wave(u0, um1, beta, halo, radius, nsteps, src=None, amp=None, rec=None, periodic=False):
    c = oracle.fd_weights_float(2 * radius)
    a, b, tr = oracle.wave_run(W.embed(u0, halo), W.embed(um1, halo), W.embed(beta, halo), halo,
                               radius, c, nsteps, src=src, src_amp=amp, rec=rec, periodic=periodic)
    return W.interior_of(a, halo), W.interior_of(b, halo), tr


def gpu_heat(plan, u0, nsteps, device="cuda", variant=None):
    import torch
    h = plan.halo
    f = [plan.field(device) for _ in range(2)]
    f[0].load(W.embed(u0, h))
    if variant is not None:
        plan.variant = variant
    plan.run(f, nsteps)
    torch.cuda.synchronize()
    return f[0].interior(h)
