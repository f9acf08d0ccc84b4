"""The so-8 acoustic wave forward model m -> receiver traces as a
torch.autograd.Function.

forward: the library writes beta = dt^2 / (h^2 m) and the point scales
dt^2 / m at the sources and receivers, injects the wavelet times the source
scale, and records the traces in its checkpointed forward run.  backward: the
library's checkpointed adjoint sweep with fused imaging returns dJ/dm for the
incoming trace gradient (for J = 1/2 |d - d_obs|^2 that gradient is
d - d_obs), with the receiver scales as residual weights.  The gradient is
exact for the discrete recurrence in m-form, which already accounts for the
source amount's dependence on m.  This module only marshals arguments.
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
        w = np.asarray(wavelet, dtype=np.float64)
        if w.ndim == 1:
            w = np.repeat(w.reshape(-1, 1), len(self.src), axis=1)
        if w.shape != (self.nsteps, len(self.src)):
            raise ValueError("wavelet must hold one sample per step (per source, or shared)")
        self.wavelet = torch.as_tensor(np.ascontiguousarray(w), device=self.device)
        self.plan = Plan(WAVE2, self.shape, 4, second_derivative_weights(8), halo=4)
        self.fields = [self.plan.field(self.device) for _ in range(3)]
        nbytes = self.plan.adjoint_workspace_bytes(self.nsteps, self.every)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.generation = 0

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
            src_scale = plan.point_scale(m, dt, model.src)
            tr = torch.zeros((model.nsteps, len(model.rec)), dtype=torch.float64, device=model.device)
            f[0].storage.zero_()
            f[1].storage.zero_()
            plan.forward_ckpt(f, model.nsteps, model.every, model.workspace, src=model.src,
                              src_amp=model.wavelet, rec=model.rec, rec_trace=tr, src_scale=src_scale)
            model.generation += 1
            ctx.model = model
            ctx.generation = model.generation
            ctx.save_for_backward(m, src_scale)
            return tr

        @staticmethod
        def backward(ctx, grad_traces):
            model = ctx.model
            if ctx.generation != model.generation:
                raise RuntimeError("the model ran another forward since this one; its checkpoints "
                                   "are gone (one backward per forward)")
            m, src_scale = ctx.saved_tensors
            rec_scale = model.plan.point_scale(m, model.dt, model.rec)
            grad = torch.zeros_like(m)
            model.plan.adjoint(model.fields[2], model.nsteps, model.every, model.workspace,
                               grad_traces.contiguous(), model.rec, rec_scale, model.dt, grad,
                               src=model.src, src_amp=model.wavelet, src_scale=src_scale)
            return grad, None

    return _WaveTraces


class _Lazy:
    _fn = None

    def apply(self, *args):
        if _Lazy._fn is None:
            _Lazy._fn = _autograd_function()
        return _Lazy._fn.apply(*args)


WaveTraces = _Lazy()
