"""Host-side checks of the boundary added around the sweeps: every entry
point of include/stencil.h states the passage of the paper it implements (or
that it has none, or for the allocation-free run the callers it serves), the stability number of a plan's weights against its
closed form, and the argument checks of the workspace, point-scale,
gradient and check calls, which all fail before any device work."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import paper_2404_02218_amd as S
from paper_2404_02218_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stencil.h")


def _declarations():
    """(name, the comment block directly above the declaration or '')."""
    text = open(HEADER).read()
    out = []
    for m in re.finditer(r"^(?:stencil_status|const char\*|int)\s+(stencil_[a-z_]+)\s*\(", text, re.M):
        before = text[:m.start()].rstrip()
        comment = ""
        if before.endswith("*/"):
            comment = before[before.rindex("/*"):]
        out.append((m.group(1), comment))
    return out


def test_every_entry_point_cites_its_passage():
    decls = _declarations()
    assert len(decls) >= 35
    for name, comment in decls:
        assert comment, f"{name} has no comment of its own"
        # the allocation-free variant names its callers instead of a passage
        assert ("Section" in comment or "no passage" in comment or "cannot allocate" in comment), \
            f"{name}: {comment[:120]}"


def test_the_survey_boundary_calls_cite_a_section():
    """The calls of the method itself name the section that defines them."""
    decls = dict(_declarations())
    for name in ("stencil_create", "stencil_layout", "stencil_apply", "stencil_run", "stencil_adjoint",
                 "stencil_adjoint_workspace", "stencil_gradient", "stencil_forward_ckpt", "stencil_exchanges",
                 "stencil_halo_pack", "stencil_halo_unpack", "stencil_batch_create", "stencil_batch_run",
                 "stencil_wave_beta", "stencil_wave_point_scale"):
        assert re.search(r"Sections? \d", decls[name]), name


def _weights(so):
    return S.second_derivative_weights(so)


@pytest.mark.parametrize("so,ndim", [(2, 2), (4, 3), (8, 3), (8, 1), (6, 2)])
def test_stability_number_matches_the_symbol_at_pi(so, ndim):
    """For the centred second-difference weights the symbol
    -(c0 + 2 sum c_k cos k theta) peaks at theta = pi, where it is
    -(c0 + 2 sum (-1)^k c_k): 4 for order 2, 16/3 for order 4, 2048/315 for
    order 8."""
    r = so // 2
    shape = (9,) * ndim
    p = S.Plan(S.WAVE2, shape, r, _weights(so), halo=r)
    c = _weights(so)
    at_pi = -(c[0] + 2 * sum((-1) ** k * c[k] for k in range(1, r + 1)))
    assert p.stability() == pytest.approx(ndim * at_pi, rel=1e-12)
    known = {2: 4.0, 4: 16.0 / 3.0, 8: 2048.0 / 315.0}
    if so in known:
        assert p.stability() == pytest.approx(ndim * known[so], rel=1e-12)


def test_stability_number_of_heat_weights_includes_alpha():
    p = S.Plan(S.HEAT, (16, 16), 1, S.heat_weights(2, 0.2), halo=1)
    assert p.stability() == pytest.approx(2 * 4 * 0.2, rel=1e-12)   # 1.6 <= 2: stable
    q = S.Plan(S.HEAT, (8, 8, 8), 2, S.heat_weights(4, 0.2), halo=2)
    assert q.stability() / 2 > 1                                    # 3 * 16/3 * 0.2 = 3.2 > 2


def test_the_wave_workloads_timestep_is_half_the_stability_limit():
    """The timestep reading of the wave workloads (half the leapfrog limit):
    beta_max * D * S_max = 4 * 0.25 at the model's largest velocity."""
    import workloads as W
    P = W.wave3d_c3(shape=(24, 20, 28), nsteps=1)
    p = S.Plan(S.WAVE2, P.shape, 4, _weights(8), halo=4)
    bmax = float(P.beta.max())
    assert bmax * p.stability() / 4 == pytest.approx(0.25, rel=1e-9)


def _plan_handle(kind=S.WAVE2, shape=(8, 9, 10)):
    return S.Plan(kind, shape, 4 if kind == S.WAVE2 else 1,
                  _weights(8) if kind == S.WAVE2 else S.heat_weights(2, 0.1))


def test_workspace_calls_validate_arguments():
    lib = _abi.lib()
    b = C.c_size_t(123)
    assert lib.stencil_run_workspace(None, C.byref(b)) == -1
    p = _plan_handle()
    assert lib.stencil_run_workspace(p.handle, None) == -1
    # the default variant of a 3D wave plan needs no workspace
    assert lib.stencil_run_workspace(p.handle, C.byref(b)) == 0 and b.value == 0
    # a temporally blocked variant needs two fields
    names = [p.variant_name(v) for v in range(p.variant_count())]
    tb = names.index(next(n for n in names if n.startswith("tb2_")))
    p.variant = tb
    assert lib.stencil_run_workspace(p.handle, C.byref(b)) == 0
    fb = (p.layout.bytes + 255) // 256 * 256
    assert b.value == 2 * fb
    # ... and stencil_run refuses to run without one, before any device work
    ptrs = (C.c_void_p * 3)(0x10000, 0x20000, 0x30000)
    assert lib.stencil_run(p.handle, ptrs, 4, None, None, None) == -5
    assert b"workspace" in lib.stencil_last_error()
    # a bad size is refused
    assert lib.stencil_set_workspace(p.handle, C.c_void_p(0x40000), 7, None) == -1
    assert lib.stencil_set_workspace(None, None, 0, None) == -1
    assert lib.stencil_set_workspace(p.handle, None, 0, None) == 0   # detach


def test_point_scale_gradient_and_check_validate_arguments():
    lib = _abi.lib()
    p = _plan_handle()
    pos = np.array([[1, 2, 3], [8, 0, 0]], dtype=np.int64)   # z = 8 is outside 8 x 9 x 10
    out = C.c_void_p(0x50000)
    m = C.c_void_p(0x60000)
    assert lib.stencil_wave_point_scale(p.handle, m, 1e-3, 2, pos.ctypes.data_as(C.c_void_p), out, None) == -1
    assert lib.stencil_wave_point_scale(p.handle, m, -1.0, 1, pos.ctypes.data_as(C.c_void_p), out, None) == -1
    assert lib.stencil_wave_point_scale(p.handle, m, 1e-3, 0, None, None, None) == 0   # nothing to do
    heat = _plan_handle(S.HEAT, (8, 8))
    assert lib.stencil_wave_point_scale(heat.handle, m, 1e-3, 1, pos.ctypes.data_as(C.c_void_p), out, None) == -5
    # the single-call gradient: source scales are refused (they come from m)
    ptrs = (C.c_void_p * 3)(0x10000, 0x20000, 0x30000)
    sp = np.array([[1, 2, 3]], dtype=np.int64)
    src = _abi.Source(1, sp.ctypes.data_as(C.c_void_p), C.c_void_p(0x70000), C.c_void_p(0x80000))
    rec = _abi.Receivers(1, sp.ctypes.data_as(C.c_void_p), C.c_void_p(0x90000))
    ws = C.c_void_p(0xa0000)
    args = (p.handle, ptrs, m, 1e-3, 10.0, 4, 2)
    tail = (C.c_void_p(0xb0000), C.c_void_p(0xc0000), C.c_void_p(0xd0000), ws, 1 << 40, None)
    assert lib.stencil_gradient(*args, C.byref(src), C.byref(rec), *tail) == -1
    src.scale = None
    assert lib.stencil_gradient(*args, C.byref(src), None, *tail) == -1          # no receivers
    assert lib.stencil_gradient(p.handle, ptrs, m, 0.0, 10.0, 4, 2, C.byref(src), C.byref(rec), *tail) == -1
    small = (C.c_void_p(0xb0000), C.c_void_p(0xc0000), C.c_void_p(0xd0000), ws, 64, None)
    assert lib.stencil_gradient(*args, C.byref(src), C.byref(rec), *small) == -1  # workspace too small
    # the adjoint takes dt, not a free gradient scale
    assert lib.stencil_adjoint(p.handle, C.c_void_p(0x30000), 4, 2, None, None, None, None, -1.0,
                               C.c_void_p(0xd0000), ws, 1 << 40, None) == -1
    # stencil_check needs fields and a report
    rep = _abi.CheckReport()
    assert lib.stencil_check(p.handle, None, C.byref(rep), None) == -1
    assert lib.stencil_check(p.handle, ptrs, None, None) == -1
    zero = (C.c_void_p * 3)(0, 0, 0)
    assert lib.stencil_check(p.handle, zero, C.byref(rep), None) == -1
    d = C.c_double()
    assert lib.stencil_stability(None, C.byref(d)) == -1
    assert lib.stencil_stability(p.handle, None) == -1


def test_abi_version_is_2_and_source_struct_carries_scales():
    assert _abi.lib().stencil_abi_version() == 2
    assert [f[0] for f in _abi.Source._fields_] == ["n", "pos", "amp", "scale"]
    assert C.sizeof(_abi.CheckReport) == 56
    assert math.isclose(1.0, 1.0)
