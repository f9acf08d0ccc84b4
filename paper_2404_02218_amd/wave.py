"""The so-8 acoustic wave forward model m -> receiver traces as a
torch.autograd.Function.

forward: beta = dt^2 / (h^2 m) is written by the library's kernel, the
source amount dt^2 / m_s * w(t_n) is formed on the device, and the
checkpointed forward run records the traces.  backward: the library's
checkpointed adjoint sweep with fused imaging returns dJ/dm for the incoming
trace gradient (for J = 1/2 |d - d_obs|^2 that gradient is d - d_obs).  The
gradient is exact for the discrete recurrence in m-form, which already
accounts for the source amount's dependence on m.
"""
from __future__ import annotations

import numpy as np

from . import WAVE2, Plan, second_derivative_weights


class WaveModel:
    """Plan, fields and checkpoint workspace of one forward model.

    The workspace holds the checkpoints of the latest forward call; a
    backward after a newer forward of the same model raises instead of
    using the wrong checkpoints.
    """

    def __init__(self, shape, h: float, dt: float, src, wavelet, rec, nsteps: int,
                 checkpoint_every: int, device="cuda"):
        import torch
        self.shape = tuple(int(s) for s in shape)
        self.h, self.dt = float(h), float(dt)
        self.nsteps, self.every = int(nsteps), int(checkpoint_every)
        self.src = np.asarray(src, dtype=np.int64).reshape(-1, 3)
        self.rec = np.asarray(rec, dtype=np.int64).reshape(-1, 3)
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.wavelet = torch.as_tensor(np.asarray(wavelet, dtype=np.float64), device=self.device)
        if self.wavelet.shape[0] != self.nsteps:
            raise ValueError("wavelet must hold one sample per step")
        self.plan = Plan(WAVE2, self.shape, 4, second_derivative_weights(8), halo=4)
        self.fields = [self.plan.field(self.device) for _ in range(3)]
        nbytes = self.plan.adjoint_workspace_bytes(self.nsteps, self.every)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.generation = 0
        self._src_idx = self._flat(self.src)
        self._rec_idx = self._flat(self.rec)

    def _flat(self, pos):
        import torch
        nz, ny, nx = self.shape
        idx = [(int(p[0]) * ny + int(p[1])) * nx + int(p[2]) for p in pos]
        return torch.tensor(idx, dtype=torch.int64, device=self.device)

    def __call__(self, m):
        return WaveTraces.apply(m, self)


def _autograd_function():
    import torch

    class _WaveTraces(torch.autograd.Function):
        @staticmethod
        def forward(ctx, m, model: WaveModel):
            if m.dtype != torch.float64 or tuple(m.shape) != model.shape or m.device != model.device:
                raise ValueError("m must be an FP64 tensor of the model's interior shape on its device")
            m = m.contiguous()
            plan, f, dt = model.plan, model.fields, model.dt
            plan.wave_beta(m, dt, model.h, f[2])
            ms = m.reshape(-1).index_select(0, model._src_idx)
            amp = ((dt * dt) / ms).reshape(1, -1) * model.wavelet.reshape(-1, 1)
            amp = amp.contiguous()
            tr = torch.zeros((model.nsteps, len(model.rec)), dtype=torch.float64, device=model.device)
            f[0].storage.zero_()
            f[1].storage.zero_()
            plan.forward_ckpt(f, model.nsteps, model.every, model.workspace, src=model.src,
                              src_amp=amp, rec=model.rec, rec_trace=tr)
            model.generation += 1
            ctx.model = model
            ctx.generation = model.generation
            ctx.save_for_backward(m, amp)
            return tr

        @staticmethod
        def backward(ctx, grad_traces):
            model = ctx.model
            if ctx.generation != model.generation:
                raise RuntimeError("the model ran another forward since this one; its checkpoints "
                                   "are gone (one backward per forward)")
            m, amp = ctx.saved_tensors
            dt = model.dt
            mr = m.reshape(-1).index_select(0, model._rec_idx)
            scale = ((dt * dt) / mr).contiguous()
            grad = torch.zeros_like(m)
            model.plan.adjoint(model.fields[2], model.nsteps, model.every, model.workspace,
                               grad_traces.contiguous(), model.rec, scale, -1.0 / (dt * dt), grad,
                               src=model.src, src_amp=amp)
            return grad, None

    return _WaveTraces


class _Lazy:
    _fn = None

    def apply(self, *args):
        if _Lazy._fn is None:
            _Lazy._fn = _autograd_function()
        return _Lazy._fn.apply(*args)


WaveTraces = _Lazy()
