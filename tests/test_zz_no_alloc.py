"""The allocation-free run (stencil_run_noalloc) against stencil_run through
the C ABI: the same bits on two calls in a row, the second with a smaller
input (so the shared static scratch still holds the first call's tables),
for the plain and the temporally blocked wave sweeps, the point kernel with
coincident sources, sources with scales, receivers and the 2D heat; and a run
too large for the scratch is refused before any device work."""
import ctypes as C

import numpy as np
import pytest

import paper_2404_02218_amd as S
import workloads as W
from paper_2404_02218_amd import _abi
from _helpers import torch_f64, wave_inputs

pytestmark = pytest.mark.gpu


def _structs(src, amp, scale, rec, trace):
    keep = []
    s = r = None
    if src is not None:
        sp = np.ascontiguousarray(np.asarray(src, dtype=np.int64).reshape(len(src), -1))
        sp3 = np.zeros((len(sp), 3), dtype=np.int64)
        sp3[:, :sp.shape[1]] = sp
        keep.append(sp3)
        s = _abi.Source(len(sp3), sp3.ctypes.data_as(C.c_void_p), C.c_void_p(amp.data_ptr()),
                        C.c_void_p(scale.data_ptr()) if scale is not None else None)
    if rec is not None:
        rp = np.ascontiguousarray(np.asarray(rec, dtype=np.int64).reshape(len(rec), -1))
        rp3 = np.zeros((len(rp), 3), dtype=np.int64)
        rp3[:, :rp.shape[1]] = rp
        keep.append(rp3)
        r = _abi.Receivers(len(rp3), rp3.ctypes.data_as(C.c_void_p), C.c_void_p(trace.data_ptr()))
    return s, r, keep


def _run(plan, levels, nsteps, src=None, amp=None, scale=None, rec=None, noalloc=False):
    """One run through the C ABI from the given levels; returns the two
    newest levels (storage) and the traces."""
    import torch
    lib = _abi.lib()
    f = [plan.field() for _ in range(len(levels))]
    for fld, a in zip(f, levels):
        fld.load(W.embed(a, plan.halo))
    nrec = 0 if rec is None else len(rec)
    trace = torch.zeros((nsteps, max(nrec, 1)), dtype=torch.float64, device="cuda")
    plan._ws.ensure(plan.handle)
    s, r, keep = _structs(src, amp, scale, rec, trace)
    ptrs = (C.c_void_p * 3)(*[x.ptr for x in f] + [0] * (3 - len(f)))
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    fn = lib.stencil_run_noalloc if noalloc else lib.stencil_run
    st = fn(plan.handle, ptrs, int(nsteps), C.byref(s) if s else None, C.byref(r) if r else None, stream)
    assert st == 0, lib.stencil_last_error()
    torch.cuda.synchronize()
    del keep
    byptr = {x.ptr: x for x in f}
    return byptr[C.c_void_p(ptrs[0]).value].storage.clone(), byptr[C.c_void_p(ptrs[1]).value].storage.clone(), trace


def _same(plan, levels, nsteps, **kw):
    import torch
    a = _run(plan, levels, nsteps, **kw)
    b = _run(plan, levels, nsteps, noalloc=True, **kw)
    for x, y in zip(a, b):
        assert torch.equal(x, y), plan.variant_name(plan.variant)


def test_noalloc_equals_run_on_two_calls_in_a_row(device):
    import torch
    big, small = (40, 44, 72), (20, 18, 30)
    for variant_kind in ("zmarch", "tb2", "point"):
        # first call: the larger grid, more sources and steps
        for shape, nsteps, nsrc in ((big, 9, 5), (small, 5, 2)):
            u0, um1, beta = wave_inputs(shape, seed=401 + nsteps)
            plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4)
            names = [plan.variant_name(v) for v in range(plan.variant_count())]
            plan.variant = {"point": 0, "zmarch": 2,
                            "tb2": next(i for i, n in enumerate(names) if n.startswith("tb2_"))}[variant_kind]
            rng = np.random.default_rng(402 + nsrc)
            src = np.stack([rng.integers(0, n, nsrc) for n in shape], axis=1)
            src[-1] = src[0]   # two sources at one point
            amp = torch_f64(rng.standard_normal((nsteps, nsrc)), device)
            scale = torch_f64(rng.uniform(0.5, 2.0, nsrc), device)
            rec = np.stack([rng.integers(0, n, 3) for n in shape], axis=1)
            _same(plan, (u0, um1, beta), nsteps, src=src, amp=amp, rec=rec)
            _same(plan, (u0, um1, beta), nsteps, src=src, amp=amp, scale=scale, rec=rec)
    torch.cuda.synchronize()


def test_noalloc_2d_heat_and_1d_wave(device):
    rng = np.random.default_rng(411)
    for shape in ((60, 70), (20, 24)):
        plan = S.Plan(S.HEAT, shape, 1, S.heat_weights(2, 0.2), halo=1)
        u = W.round_to_storage(rng.random(shape), "f32")
        _same(plan, (u, np.zeros(shape)), 20)
    for n in (300, 90):
        plan = S.Plan(S.WAVE2, (n,), 4, S.second_derivative_weights(8), halo=4)
        u0, um1, beta = wave_inputs((n,), seed=412 + n)
        amp = torch_f64(rng.standard_normal((7, 2)), device)
        _same(plan, (u0, um1, beta), 7, src=[[n // 2], [n // 3]], amp=amp, rec=[[n // 4]])


def test_noalloc_refuses_a_run_beyond_its_scratch(device):
    import torch
    lib = _abi.lib()
    shape = (16, 16, 16)
    plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4)
    u0, um1, beta = wave_inputs(shape, seed=421)
    f = [plan.field() for _ in range(3)]
    for fld, a in zip(f, (u0, um1, beta)):
        fld.load(W.embed(a, 4))
    before = [x.storage.clone() for x in f]
    nsteps, nsrc = 600, 2000   # 600 x 2000 formed amounts: 9.6 MB > 8 MiB
    rng = np.random.default_rng(422)
    src = np.stack([rng.integers(0, 16, nsrc) for _ in range(3)], axis=1)
    amp = torch.zeros((nsteps, nsrc), dtype=torch.float64, device=device)
    scale = torch.ones(nsrc, dtype=torch.float64, device=device)
    s, r, keep = _structs(src, amp, scale, None, None)
    ptrs = (C.c_void_p * 3)(*[x.ptr for x in f])
    st = lib.stencil_run_noalloc(plan.handle, ptrs, nsteps, C.byref(s), None, None)
    assert st == -3
    assert b"static scratch" in lib.stencil_last_error()
    torch.cuda.synchronize()
    assert all(torch.equal(x.storage, y) for x, y in zip(f, before))
    # without scales the amounts are not formed, and the run fits
    s.scale = None
    assert lib.stencil_run_noalloc(plan.handle, ptrs, 4, C.byref(s), None, None) == 0
    torch.cuda.synchronize()
    del keep
