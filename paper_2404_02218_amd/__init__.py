"""MI355X (gfx950) star-stencil sweeps: heat / Jacobi and the second-order
acoustic wave, halo exchange declarations with pack/unpack, batched shots and
the checkpointed adjoint, behind the C ABI of libstencil.so.

This module marshals arguments only.  PyTorch supplies device memory and
streams; every sweep, copy, injection and reduction runs in the library's HIP
kernels.  Importing it does not load the library; the first call does, and
fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _abi
from ._abi import (BC_DIRICHLET0, BC_PERIODIC, BF16, CHECK_BAD_BETA, CHECK_NONFINITE,  # noqa: F401
                   CHECK_OVERFLOW, CHECK_UNSTABLE, F16, F32, HEAT, WAVE2, CheckReport, Exchange, Receivers,
                   ReceiversInterp, Source, SourceInterp, StencilError, call, lib)
from .coeffs import damping_profile, heat_weights, second_derivative_weights  # noqa: F401

DTYPES = {"f32": F32, "bf16": BF16, "f16": F16}
_ESIZE = {F32: 4, BF16: 2, F16: 2}


def _torch():
    import torch
    return torch


def _tdtype(dt):
    torch = _torch()
    return {F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16}[dt]


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _i64(vals, n=3):
    arr = (C.c_int64 * n)()
    for i, v in enumerate(vals):
        arr[i] = int(v)
    return arr


def _positions(pos):
    """Host [n][3] int64 array (first ndim slots used)."""
    if pos is None:
        return None, 0
    p = np.asarray(pos, dtype=np.int64)
    if p.ndim == 1:
        p = p.reshape(1, -1)
    out = np.zeros((p.shape[0], 3), dtype=np.int64)
    out[:, :p.shape[1]] = p
    return np.ascontiguousarray(out), p.shape[0]


@dataclass
class Layout:
    extents: tuple
    strides: tuple
    offset: int
    bytes: int


class Field:
    """One field (stencil.field): padded device storage plus a strided view
    of the buffer extents (halo included)."""

    def __init__(self, layout: Layout, dtype: int, device="cuda"):
        torch = _torch()
        self.layout = layout
        self.dtype = dtype
        n = layout.bytes // _ESIZE[dtype]
        self.storage = torch.zeros(n, dtype=_tdtype(dtype), device=device)
        self.view = self.storage.as_strided(layout.extents, layout.strides, layout.offset)

    @property
    def ptr(self) -> int:
        return self.storage.data_ptr()

    def to_numpy(self) -> np.ndarray:
        """Dense FP64 copy of the buffer (halo included)."""
        return self.view.to(_torch().float64).cpu().numpy()

    def interior(self, halo: int) -> np.ndarray:
        a = self.to_numpy()
        return a[tuple(slice(halo, s - halo) for s in a.shape)]

    def load(self, arr: np.ndarray) -> "Field":
        """Write a dense buffer (FP64, rounded to the storage dtype)."""
        torch = _torch()
        t = torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float64))
        self.view.copy_(t.to(self.view.device).to(self.view.dtype))
        return self

    def zero(self) -> "Field":
        self.storage.zero_()
        return self


class _Points:
    """Keeps the ctypes structs and the host arrays they point to alive."""

    def __init__(self, pos, dev, scale=None):
        self.pos, self.n = _positions(pos)
        self.dev = dev
        self.scale = scale

    def source(self):
        if self.n == 0:
            return None
        sc = C.c_void_p(self.scale.data_ptr()) if self.scale is not None else None
        return Source(self.n, self.pos.ctypes.data_as(C.c_void_p), C.c_void_p(self.dev.data_ptr()), sc)

    def receivers(self):
        if self.n == 0:
            return None
        return Receivers(self.n, self.pos.ctypes.data_as(C.c_void_p), C.c_void_p(self.dev.data_ptr()))


def _real_positions(pos, ndim):
    """[n, ndim] real positions as a C-contiguous [n, 3] float64 array."""
    p = np.asarray(pos, dtype=np.float64).reshape(-1, ndim)
    out = np.zeros((p.shape[0], 3), dtype=np.float64)
    out[:, :ndim] = p
    return np.ascontiguousarray(out)


class _Workspace:
    """Caller memory for a plan's run workspace (stencil_run_workspace /
    stencil_set_workspace), grown when the plan's variant needs more."""

    def __init__(self):
        self.buf = None

    def ensure(self, handle, stream=None):
        b = C.c_size_t()
        call("stencil_run_workspace", handle, C.byref(b))
        need = b.value
        if need == 0 or (self.buf is not None and self.buf.numel() >= need):
            return
        torch = _torch()
        self.buf = torch.empty(need, dtype=torch.uint8, device=torch.cuda.current_device())
        call("stencil_set_workspace", handle, C.c_void_p(self.buf.data_ptr()), need, _stream_ptr(stream))


def _check_f64_device(t, shape, what):
    torch = _torch()
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous FP64 device tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Plan:
    """A stencil plan (stencil_create)."""

    def __init__(self, kind: int, shape, radius: int, coeffs, halo: int | None = None,
                 dtype: int = F32, bc: int = BC_DIRICHLET0):
        self.kind, self.radius, self.dtype, self.bc = kind, radius, dtype, bc
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        self.halo = radius if halo is None else halo
        self.coeffs = [float(c) for c in coeffs]
        h = C.c_void_p()
        c = (C.c_double * 5)(*(self.coeffs + [0.0] * (5 - len(self.coeffs))))
        call("stencil_create", C.byref(h), kind, self.ndim, _i64(self.shape), radius, c, self.halo,
             dtype, bc)
        self._h = h
        self.layout = self._layout()
        self._ws = _Workspace()

    def _layout(self) -> Layout:
        e, s, o, b = (C.c_int64 * 3)(), (C.c_int64 * 3)(), C.c_int64(), C.c_int64()
        call("stencil_layout", self._h, e, s, C.byref(o), C.byref(b))
        return Layout(tuple(e[:self.ndim]), tuple(s[:self.ndim]), o.value, b.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().stencil_destroy(h)
            except Exception:
                pass

    @property
    def handle(self):
        return self._h

    def field(self, device="cuda") -> Field:
        return Field(self.layout, self.dtype, device)

    # one load/apply/store on [lo, hi)
    def apply(self, out: Field, inputs, lo=None, hi=None, stream=None):
        lo = lo if lo is not None else [0] * self.ndim
        hi = hi if hi is not None else list(self.shape)
        ptrs = (C.c_void_p * 3)(*[f.ptr for f in inputs] + [0] * (3 - len(inputs)))
        call("stencil_apply", self._h, C.c_void_p(out.ptr), ptrs, _i64(lo), _i64(hi),
             _stream_ptr(stream))

    def run_workspace_bytes(self) -> int:
        b = C.c_size_t()
        call("stencil_run_workspace", self._h, C.byref(b))
        return b.value

    def run(self, fields: list, nsteps: int, src=None, src_amp=None, rec=None, rec_trace=None,
            stream=None, src_scale=None):
        """nsteps sweeps; `fields` is permuted in place like the pointer array.
        src_amp[t, s] is added at source s after step t, times src_scale[s]
        when given (device FP64).  A variant that needs a run workspace gets
        one allocated here (caller memory kept with the plan)."""
        ptrs = (C.c_void_p * 3)(*[f.ptr for f in fields] + [0] * (3 - len(fields)))
        sp = _Points(src, src_amp, src_scale)
        rp = _Points(rec, rec_trace)
        if sp.n:
            _check_f64_device(src_amp, (nsteps, sp.n), "src_amp")
            if src_scale is not None:
                _check_f64_device(src_scale, (sp.n,), "src_scale")
        if rp.n:
            _check_f64_device(rec_trace, (nsteps, rp.n), "rec_trace")
        self._ws.ensure(self._h, stream)
        s, r = sp.source(), rp.receivers()
        call("stencil_run", self._h, ptrs, int(nsteps), C.byref(s) if s else None,
             C.byref(r) if r else None, _stream_ptr(stream))
        if ptrs[0] != fields[0].ptr:
            fields[0], fields[1] = fields[1], fields[0]
        return fields

    def set_damping(self, profiles):
        """Absorbing layer (stencil_wave_damping): one 1D array of damping
        per axis (extent entries each), or None to remove it."""
        if profiles is None:
            call("stencil_wave_damping", self._h, None)
            return
        if len(profiles) != self.ndim:
            raise ValueError(f"expected {self.ndim} per-axis profiles")
        flat = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in profiles]))
        if flat.size != sum(self.shape):
            raise ValueError("each profile needs one entry per interior point of its axis")
        call("stencil_wave_damping", self._h, flat.ctypes.data_as(C.c_void_p))

    def interp_weights(self, pos):
        """Corners [n, 2^ndim, ndim] and weights [n, 2^ndim] of real interior
        positions [n, ndim] (stencil_interp_weights)."""
        p = _real_positions(pos, self.ndim)
        n, nc = p.shape[0], 1 << self.ndim
        corners = np.zeros((max(n, 1), nc, 3), dtype=np.int64)
        w = np.zeros((max(n, 1), nc), dtype=np.float64)
        call("stencil_interp_weights", self._h, n, p.ctypes.data_as(C.c_void_p),
             corners.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p))
        return corners[:n, :, :self.ndim], w[:n]

    def run_interp(self, fields: list, nsteps: int, src=None, src_amp=None, rec=None, rec_trace=None,
                   stream=None):
        """run() with sources and receivers at real positions [n, ndim]
        (stencil_run_interp)."""
        ptrs = (C.c_void_p * 3)(*[f.ptr for f in fields] + [0] * (3 - len(fields)))
        sp = _real_positions(src, self.ndim) if src is not None else np.zeros((0, 3))
        rp = _real_positions(rec, self.ndim) if rec is not None else np.zeros((0, 3))
        s = r = None
        if len(sp):
            _check_f64_device(src_amp, (nsteps, len(sp)), "src_amp")
            s = SourceInterp(len(sp), sp.ctypes.data_as(C.c_void_p), C.c_void_p(src_amp.data_ptr()))
        if len(rp):
            _check_f64_device(rec_trace, (nsteps, len(rp)), "rec_trace")
            r = ReceiversInterp(len(rp), rp.ctypes.data_as(C.c_void_p), C.c_void_p(rec_trace.data_ptr()))
        self._ws.ensure(self._h, stream)
        call("stencil_run_interp", self._h, ptrs, int(nsteps), C.byref(s) if s else None,
             C.byref(r) if r else None, _stream_ptr(stream))
        if ptrs[0] != fields[0].ptr:
            fields[0], fields[1] = fields[1], fields[0]
        return fields

    # exchanges
    def exchanges(self, grid, coord, periodic=False, box=False):
        """Exchange declarations of the rank at `coord`: faces, or with
        box=True faces, edges and corners (stencil_exchanges_box)."""
        arr = (Exchange * 26)()
        n = C.c_int(26)
        g = (C.c_int32 * 3)(*[int(x) for x in grid] + [1] * (3 - len(grid)))
        cc = (C.c_int32 * 3)(*[int(x) for x in coord] + [0] * (3 - len(coord)))
        call("stencil_exchanges_box" if box else "stencil_exchanges", self._h, g, cc, int(periodic),
             C.cast(arr, C.c_void_p), C.byref(n))
        return [arr[i] for i in range(n.value)]

    def exchange_elems(self, ex) -> int:
        return int(sum(int(np.prod(e.size[:self.ndim])) for e in ex))

    def _ex_arr(self, ex):
        arr = (Exchange * max(1, len(ex)))()
        for i, e in enumerate(ex):
            arr[i] = e
        return arr

    def pack(self, field: Field, ex, buf, stream=None):
        call("stencil_halo_pack", self._h, C.c_void_p(field.ptr),
             C.cast(self._ex_arr(ex), C.c_void_p), len(ex), C.c_void_p(buf.data_ptr()),
             _stream_ptr(stream))

    def unpack(self, field: Field, ex, buf, stream=None):
        call("stencil_halo_unpack", self._h, C.c_void_p(field.ptr),
             C.cast(self._ex_arr(ex), C.c_void_p), len(ex), C.c_void_p(buf.data_ptr()),
             _stream_ptr(stream))

    # variants
    def variant_count(self) -> int:
        n = C.c_int()
        call("stencil_variant_count", self._h, C.byref(n))
        return n.value

    def variant_name(self, v: int) -> str:
        buf = C.create_string_buffer(64)
        call("stencil_variant_name", self._h, int(v), buf, 64)
        return buf.value.decode()

    @property
    def variant(self) -> int:
        v = C.c_int()
        call("stencil_get_variant", self._h, C.byref(v))
        return v.value

    @variant.setter
    def variant(self, v: int):
        call("stencil_set_variant", self._h, int(v))

    def tune(self, fields: list, reps: int = 3, stream=None) -> int:
        ptrs = (C.c_void_p * max(3, len(fields)))(*[f.ptr for f in fields])
        call("stencil_tune", self._h, ptrs, int(reps), _stream_ptr(stream))
        return self.variant

    # adjoint
    def adjoint_workspace_bytes(self, nsteps: int, every: int) -> int:
        b = C.c_size_t()
        call("stencil_adjoint_workspace", self._h, int(nsteps), int(every), C.byref(b))
        return b.value

    def forward_ckpt(self, fields, nsteps, every, workspace, src=None, src_amp=None, rec=None,
                     rec_trace=None, stream=None, src_scale=None):
        ptrs = (C.c_void_p * 3)(*[f.ptr for f in fields])
        sp, rp = _Points(src, src_amp, src_scale), _Points(rec, rec_trace)
        if sp.n:
            _check_f64_device(src_amp, (nsteps, sp.n), "src_amp")
            if src_scale is not None:
                _check_f64_device(src_scale, (sp.n,), "src_scale")
        if rp.n:
            _check_f64_device(rec_trace, (nsteps, rp.n), "rec_trace")
        s, r = sp.source(), rp.receivers()
        call("stencil_forward_ckpt", self._h, ptrs, int(nsteps), int(every),
             C.byref(s) if s else None, C.byref(r) if r else None,
             C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
             _stream_ptr(stream))
        if ptrs[0] != fields[0].ptr:
            fields[0], fields[1] = fields[1], fields[0]
        return fields

    def adjoint(self, beta: Field, nsteps, every, workspace, resid, rec, rec_scale, dt,
                grad, src=None, src_amp=None, stream=None, src_scale=None):
        """grad += dJ/dm for the trace gradient `resid` (stencil_adjoint)."""
        sp, rp = _Points(src, src_amp, src_scale), _Points(rec, None)
        if sp.n:
            _check_f64_device(src_amp, (nsteps, sp.n), "src_amp")
            if src_scale is not None:
                _check_f64_device(src_scale, (sp.n,), "src_scale")
        _check_f64_device(resid, (nsteps, rp.n), "resid")
        _check_f64_device(rec_scale, (rp.n,), "rec_scale")
        _check_f64_device(grad, self.shape, "grad")
        s = sp.source()
        r = Receivers(rp.n, rp.pos.ctypes.data_as(C.c_void_p), None) if rp.n else None
        call("stencil_adjoint", self._h, C.c_void_p(beta.ptr), int(nsteps), int(every),
             C.byref(s) if s else None, C.byref(r) if r else None,
             C.c_void_p(resid.data_ptr()), C.c_void_p(rec_scale.data_ptr()), float(dt),
             C.c_void_p(grad.data_ptr()), C.c_void_p(workspace.data_ptr()),
             workspace.numel() * workspace.element_size(), _stream_ptr(stream))

    def gradient(self, fields, m, dt: float, h: float, nsteps: int, every: int, workspace, src, wavelet,
                 rec, rec_trace, d_obs, misfit, grad, stream=None):
        """Misfit and its gradient with respect to m in one call
        (stencil_gradient): wavelet [nsteps, nsrc] FP64, d_obs and rec_trace
        [nsteps, nrec], misfit a one-element FP64 tensor, grad the interior
        shape; all device tensors.  `fields` is permuted like run()."""
        ptrs = (C.c_void_p * 3)(*[f.ptr for f in fields])
        sp, rp = _Points(src, wavelet), _Points(rec, rec_trace)
        _check_f64_device(m, self.shape, "m")
        if sp.n:
            _check_f64_device(wavelet, (nsteps, sp.n), "wavelet")
        _check_f64_device(rec_trace, (nsteps, rp.n), "rec_trace")
        _check_f64_device(d_obs, (nsteps, rp.n), "d_obs")
        _check_f64_device(misfit, (1,), "misfit")
        _check_f64_device(grad, self.shape, "grad")
        s, r = sp.source(), rp.receivers()
        call("stencil_gradient", self._h, ptrs, C.c_void_p(m.data_ptr()), float(dt), float(h), int(nsteps),
             int(every), C.byref(s) if s else None, C.byref(r) if r else None, C.c_void_p(d_obs.data_ptr()),
             C.c_void_p(misfit.data_ptr()), C.c_void_p(grad.data_ptr()), C.c_void_p(workspace.data_ptr()),
             workspace.numel() * workspace.element_size(), _stream_ptr(stream))
        if ptrs[0] != fields[0].ptr:
            fields[0], fields[1] = fields[1], fields[0]
        return fields

    def point_scale(self, m, dt: float, pos, stream=None):
        """dt^2 / m at interior positions [n, ndim] (stencil_wave_point_scale):
        a device FP64 tensor [n]."""
        torch = _torch()
        _check_f64_device(m, self.shape, "m")
        p, n = _positions(pos)
        out = torch.empty(max(n, 1), dtype=torch.float64, device=m.device)[:n]
        call("stencil_wave_point_scale", self._h, C.c_void_p(m.data_ptr()), float(dt), n,
             p.ctypes.data_as(C.c_void_p) if n else None, C.c_void_p(out.data_ptr()) if n else None,
             _stream_ptr(stream))
        return out

    def stability(self) -> float:
        """D times the largest symbol value of the weights (stencil_stability)."""
        d = C.c_double()
        call("stencil_stability", self._h, C.byref(d))
        return d.value

    def check(self, fields, stream=None) -> dict:
        """Scan of the levels (and beta) for non-finite values, overflow and
        the stability condition (stencil_check; synchronises the stream)."""
        ptrs = (C.c_void_p * 3)(*[f.ptr for f in fields] + [0] * (3 - len(fields)))
        rep = CheckReport()
        call("stencil_check", self._h, ptrs, C.byref(rep), _stream_ptr(stream))
        out = {k: getattr(rep, k) for k, _ in CheckReport._fields_ if k != "reserved"}
        out["nonfinite"] = bool(rep.flags & CHECK_NONFINITE)
        out["overflow"] = bool(rep.flags & CHECK_OVERFLOW)
        out["unstable"] = bool(rep.flags & CHECK_UNSTABLE)
        out["bad_beta"] = bool(rep.flags & CHECK_BAD_BETA)
        return out

    def wave_beta(self, m, dt: float, h: float, beta: Field, stream=None):
        _check_f64_device(m, self.shape, "m")
        call("stencil_wave_beta", self._h, C.c_void_p(m.data_ptr()), float(dt), float(h),
             C.c_void_p(beta.ptr), _stream_ptr(stream))


class BatchPlan:
    """Independent 3D wave shots of uneven shapes (stencil_batch_create)."""

    def __init__(self, shapes, radius: int, coeffs, halo: int | None = None, dtype: int = F32):
        self.shapes = [tuple(int(x) for x in s) for s in shapes]
        self.radius, self.dtype = radius, dtype
        self.halo = radius if halo is None else halo
        sh = np.ascontiguousarray(np.array(self.shapes, dtype=np.int64).reshape(-1, 3))
        c = (C.c_double * 5)(*([float(x) for x in coeffs] + [0.0] * (5 - len(coeffs))))
        h = C.c_void_p()
        call("stencil_batch_create", C.byref(h), len(self.shapes), sh.ctypes.data_as(C.c_void_p),
             radius, c, self.halo, dtype)
        self._h = h
        self._ws = _Workspace()
        self.layouts = []
        for i in range(len(self.shapes)):
            e, s, o, b = (C.c_int64 * 3)(), (C.c_int64 * 3)(), C.c_int64(), C.c_int64()
            call("stencil_batch_layout", self._h, i, e, s, C.byref(o), C.byref(b))
            self.layouts.append(Layout(tuple(e), tuple(s), o.value, b.value))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().stencil_destroy(h)
            except Exception:
                pass

    def field(self, shot: int, device="cuda") -> Field:
        return Field(self.layouts[shot], self.dtype, device)

    @property
    def variant(self) -> int:
        v = C.c_int()
        call("stencil_get_variant", self._h, C.byref(v))
        return v.value

    @variant.setter
    def variant(self, v: int):
        call("stencil_set_variant", self._h, int(v))

    def variant_count(self) -> int:
        n = C.c_int()
        call("stencil_variant_count", self._h, C.byref(n))
        return n.value

    def variant_name(self, v: int) -> str:
        buf = C.create_string_buffer(64)
        call("stencil_variant_name", self._h, int(v), buf, 64)
        return buf.value.decode()

    def tune(self, fields: list, reps: int = 2, stream=None) -> int:
        flat = [f.ptr for shot in fields for f in shot]
        ptrs = (C.c_void_p * len(flat))(*flat)
        call("stencil_tune", self._h, ptrs, int(reps), _stream_ptr(stream))
        return self.variant

    def run(self, fields: list, nsteps: int, srcs=None, src_amps=None, recs=None, rec_traces=None,
            stream=None):
        """fields: per shot [u_n, u_prev, beta]; permuted per shot in place."""
        ns = len(self.shapes)
        flat = [f.ptr for shot in fields for f in shot]
        ptrs = (C.c_void_p * len(flat))(*flat)
        keep = []
        S = R = None
        if srcs is not None:
            S = (Source * ns)()
            for i in range(ns):
                p = _Points(srcs[i], src_amps[i])
                keep.append(p)
                if p.n:
                    _check_f64_device(src_amps[i], (nsteps, p.n), "src_amp")
                    S[i] = p.source()
        if recs is not None:
            R = (Receivers * ns)()
            for i in range(ns):
                p = _Points(recs[i], rec_traces[i])
                keep.append(p)
                if p.n:
                    _check_f64_device(rec_traces[i], (nsteps, p.n), "rec_trace")
                    R[i] = p.receivers()
        self._ws.ensure(self._h, stream)
        call("stencil_batch_run", self._h, ptrs, int(nsteps), S, R, _stream_ptr(stream))
        for i in range(ns):
            if ptrs[3 * i] != fields[i][0].ptr:
                fields[i][0], fields[i][1] = fields[i][1], fields[i][0]
        return fields
