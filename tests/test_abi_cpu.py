"""Host-side checks of the C ABI: the library loads and exports every entry
point declared in include/stencil.h, arguments are validated before any
device work, the field layout has the promised alignment, and the exchange
generator reproduces the paper's declarations.  No GPU needed: none of these
calls reaches the HIP runtime's device paths."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest

import oracle
import paper_2404_02218_amd as S
import workloads as W
from paper_2404_02218_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "stencil.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(stencil_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _abi.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_abi.EXPORTS) == names
    assert lib.stencil_abi_version() == 2


def _create(kind=S.WAVE2, shape=(8, 9, 10), radius=4, halo=4, dtype=S.F32, bc=S.BC_DIRICHLET0,
            coeffs=None):
    lib = _abi.lib()
    h = C.c_void_p()
    sh = (C.c_int64 * 3)(*shape)
    c = (C.c_double * 5)(*(coeffs or [1.0, 0.5, 0.25, 0.125, 0.0625]))
    st = lib.stencil_create(C.byref(h), kind, len(shape), sh, radius, c, halo, dtype, bc)
    return st, h



def test_library_loads_into_the_hip_runtime_torch_uses():
    """Loading the library from a fresh process, before anything imported
    torch, leaves exactly one HIP runtime in the process: torch's, which the
    device pointers and streams come from."""
    import subprocess
    import sys
    code = ("import json, paper_2404_02218_amd._abi as A; A.lib(); "
            "print(json.dumps(sorted({l.split()[-1] for l in open('/proc/self/maps') "
            "if 'libamdhip64' in l or 'libhsa-runtime64' in l})))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = json.loads(out.stdout.strip().splitlines()[-1])
    assert sum("libamdhip64" in x for x in libs) == 1, libs
    assert sum("libhsa-runtime64" in x for x in libs) == 1, libs
    import torch
    assert all(x.startswith(os.path.dirname(torch.__file__)) for x in libs), libs

@pytest.mark.parametrize("kw,status", [
    (dict(radius=5, halo=5), -2),
    (dict(radius=0), -2),
    (dict(halo=3), -1),
    (dict(kind=7), -1),
    (dict(dtype=9), -1),
    (dict(bc=4), -1),
    (dict(shape=(4, -1, 3)), -1),
    (dict(shape=(3, 3, 3), bc=S.BC_PERIODIC), -1),
    (dict(coeffs=[float("nan"), 1, 1, 1, 1]), -1),
])
def test_create_rejects_bad_arguments(kw, status):
    st, h = _create(**kw)
    assert st == status
    assert not h.value
    assert _abi.lib().stencil_last_error()


def test_create_rejects_ndim_4_and_null():
    lib = _abi.lib()
    h = C.c_void_p()
    sh = (C.c_int64 * 4)(4, 4, 4, 4)
    c = (C.c_double * 5)(1, 1, 1, 1, 1)
    assert lib.stencil_create(C.byref(h), 0, 4, sh, 1, c, 1, 0, 0) == -2
    assert lib.stencil_create(C.byref(h), 0, 3, None, 1, c, 1, 0, 0) == -1
    assert lib.stencil_create(None, 0, 3, sh, 1, c, 1, 0, 0) == -1


@pytest.mark.parametrize("dtype,esize", [(S.F32, 4), (S.BF16, 2), (S.F16, 2)])
@pytest.mark.parametrize("shape,halo", [((512, 512, 512), 4), ((37, 50, 71), 4), ((256, 256), 1),
                                        ((126,), 1), ((13, 7, 5), 2)])
def test_layout_alignment_and_bounds(shape, halo, dtype, esize):
    p = S.Plan(S.HEAT, shape, 1, [-2.0, 1.0], halo=halo, dtype=dtype)
    L = p.layout
    nd = len(shape)
    assert list(L.extents) == [n + 2 * halo for n in shape]
    assert L.strides[-1] == 1
    # first interior element of every row is 128-byte aligned
    first = L.offset + halo * sum(L.strides[:-1]) + halo
    assert (first * esize) % 128 == 0
    if nd >= 2:
        assert (L.strides[-2] * esize) % 128 == 0
        assert L.strides[-2] >= L.offset + L.extents[-1]
    last = L.offset + sum((e - 1) * s for e, s in zip(L.extents, L.strides))
    assert last < L.bytes // esize


def test_exchange_generator_matches_paper_example_through_abi():
    with open(os.path.join(ROOT, "tests", "golden", "dmp_exchange_example.json")) as f:
        g = json.load(f)
    p = S.Plan(S.WAVE2, g["interior"], g["radius"], [1, 1, 1, 1, 1], halo=g["halo"])
    ex = [e.as_dict(2) for e in p.exchanges(g["grid"], [0, 0], periodic=True)]
    assert [d for d in ex if d["to"][0] == 0] == g["printed_exchanges"]
    assert len(ex) == 4


@pytest.mark.parametrize("grid,coord,periodic", [([2, 2, 2], [0, 1, 1], False),
                                                 ([1, 3, 2], [0, 1, 0], False),
                                                 ([1, 1, 1], [0, 0, 0], True),
                                                 ([3, 1, 4], [2, 0, 3], True)])
def test_exchange_generator_matches_oracle(grid, coord, periodic):
    shape, halo, r = [12, 10, 14], 5, 3
    p = S.Plan(S.HEAT, shape, r, [1, 1, 1, 1], halo=halo)
    mine = [e.as_dict(3) for e in p.exchanges(grid, coord, periodic)]
    ref = [e.as_dict(3) for e in oracle.exchanges(shape, halo, r, grid, coord, periodic)]
    assert mine == ref


def test_exchange_generator_rejects_bad_coordinates():
    p = S.Plan(S.HEAT, [8, 8], 1, [1, 1])
    with pytest.raises(S.StencilError):
        p.exchanges([2, 2], [2, 0])


def test_product_weights_equal_oracle_derivation():
    for so in (2, 4, 6, 8):
        assert S.second_derivative_weights(so) == oracle.fd_weights_float(so)


def test_variants_are_listed():
    p = S.Plan(S.WAVE2, (64, 64, 64), 4, S.second_derivative_weights(8))
    n = p.variant_count()
    assert n == 24   # point, 20 z-marching (5 tile shapes x 4 z-chunks), 3 temporally blocked
    names = [p.variant_name(v) for v in range(n)]
    assert names[0] == "point" and len(set(names)) == n
    assert [x for x in names if x.startswith("tb2_")] == names[21:]
    assert "zmarch_128x16_t256_zc128_p8_nt" in names
    # temporal blocking covers the radius-4 wave with the zero halo only
    assert S.Plan(S.WAVE2, (64, 64, 64), 2, S.second_derivative_weights(4)).variant_count() == 21
    assert S.Plan(S.WAVE2, (64, 64, 64), 4, S.second_derivative_weights(8),
                  bc=S.BC_PERIODIC).variant_count() == 21
    # 2D heat (FP32, zero halo): the point kernel and four multi-step kernels
    p2 = S.Plan(S.HEAT, (64, 64), 1, S.heat_weights(2, 0.2))
    assert [p2.variant_name(v) for v in range(p2.variant_count())] == [
        "point", "tb2d_t4_16x16", "tb2d_t8_16x16", "tb2d_t8_32x32", "tb2d_t16_32x32"]
    assert p2.variant == 2
    assert S.Plan(S.HEAT, (64, 64), 1, S.heat_weights(2, 0.2), bc=S.BC_PERIODIC).variant_count() == 1
    assert S.Plan(S.HEAT, (64, 64), 1, S.heat_weights(2, 0.2), dtype=S.BF16).variant_count() == 1
    assert S.Plan(S.WAVE2, (64, 64), 1, [-2.0, 1.0]).variant_count() == 1
    with pytest.raises(S.StencilError):
        p.variant = n


def test_run_validates_before_any_device_work():
    p = S.Plan(S.WAVE2, (16, 16, 16), 4, S.second_derivative_weights(8))
    lib = _abi.lib()
    fake = (C.c_void_p * 3)(256, 512, 768)
    # NULL and misaligned pointers
    assert lib.stencil_run(p.handle, None, 1, None, None, None) == -1
    bad = (C.c_void_p * 3)(256, 513, 768)
    assert lib.stencil_run(p.handle, bad, 1, None, None, None) == -1
    same = (C.c_void_p * 3)(256, 256, 768)
    assert lib.stencil_run(p.handle, same, 1, None, None, None) == -1
    assert lib.stencil_run(p.handle, fake, -1, None, None, None) == -1
    # a source outside the interior
    pos = np.array([[0, 0, 16]], dtype=np.int64)
    src = _abi.Source(1, pos.ctypes.data_as(C.c_void_p), C.c_void_p(4096))
    assert lib.stencil_run(p.handle, fake, 1, C.byref(src), None, None) == -1
    assert b"outside" in lib.stencil_last_error()
    # the pointer array is untouched on error
    assert [fake[i] for i in range(3)] == [256, 512, 768]


def test_apply_rejects_boxes_outside_interior():
    p = S.Plan(S.HEAT, (10, 12), 1, S.heat_weights(2, 0.1))
    lib = _abi.lib()
    ins = (C.c_void_p * 3)(256, 0, 0)
    lo = (C.c_int64 * 3)(0, 0)
    hi = (C.c_int64 * 3)(11, 12)
    assert lib.stencil_apply(p.handle, C.c_void_p(512), ins, lo, hi, None) == -1
    hi2 = (C.c_int64 * 3)(10, 12)
    assert lib.stencil_apply(p.handle, C.c_void_p(256), ins, lo, hi2, None) == -1  # aliasing


def test_adjoint_workspace_and_state_errors():
    p = S.Plan(S.WAVE2, (20, 20, 20), 4, S.second_derivative_weights(8))
    b = p.adjoint_workspace_bytes(100, 25)
    assert b >= (2 * 4 + 25 + 5) * 1  # slots
    with pytest.raises(S.StencilError):
        p.adjoint_workspace_bytes(100, 0)
    h = S.Plan(S.HEAT, (20, 20, 20), 2, S.heat_weights(4, 0.05))
    with pytest.raises(S.StencilError) as e:
        h.adjoint_workspace_bytes(10, 5)
    assert e.value.status == -5
    p16 = S.Plan(S.WAVE2, (20, 20, 20), 4, S.second_derivative_weights(8), dtype=S.BF16)
    with pytest.raises(S.StencilError):
        p16.adjoint_workspace_bytes(10, 5)


def test_batch_plan_validation():
    with pytest.raises(S.StencilError):
        S.BatchPlan([(10, 10, 10)], 2, S.second_derivative_weights(4))
    bp = S.BatchPlan([(10, 12, 14), (20, 9, 33)], 4, S.second_derivative_weights(8))
    assert len(bp.layouts) == 2
    assert bp.variant_count() == 29
    assert bp.variant_name(21).startswith("tb2_")
    assert [bp.variant_name(v) for v in range(24, 28)] == [
        f"persistent_zmarch_64x16_t256_zc{zc}_nt" for zc in (256, 128, 64, 32)]
    assert bp.variant_name(28) == "shots_concurrent_4"
    # the concurrent variant runs the shots' own plans: no workspace until
    # one of them is tuned to the temporally blocked sweep
    bp.variant = 28
    assert bp.variant == 28
    assert list(bp.layouts[1].extents) == [28, 17, 41]
    with pytest.raises(S.StencilError):
        bp.variant = 0


def _program(shape=(8, 9, 10), halo=1, nin=2, nout=1, terms=None, dtype=S.F32):
    from paper_2404_02218_amd.program import Program
    terms = terms if terms is not None else [(0, 1.0, [(0, (0, 0, 1)), (1, (1, -1, 0))])]
    return Program(shape, halo, nin, nout, terms, dtype=dtype)


@pytest.mark.parametrize("kw,status", [
    (dict(terms=[(1, 1.0, [(0, (0, 0, 0))])]), -1),                    # output index
    (dict(terms=[(0, 1.0, [(2, (0, 0, 0))])]), -1),                    # input index
    (dict(terms=[(0, 1.0, [(0, (0, 0, 2))])]), -1),                    # beyond the halo
    (dict(halo=4, terms=[(0, 1.0, [(0, (0, 3, 0))])]), -2),            # beyond the kernel's reach
    (dict(terms=[(0, float("inf"), [(0, (0, 0, 0))])]), -1),
    (dict(terms=[]), -1),
    (dict(nin=5), -2),
    (dict(dtype=S.BF16), -2),
    (dict(shape=(8, 9), terms=[(0, 1.0, [(0, (1, 0))]), (0, 1.0, [(1, (0, -1))])]), 0),
])
def test_program_create_validates(kw, status):
    if status == 0:
        p = _program(**kw)
        assert p.layout.extents == (10, 11)
        return
    with pytest.raises(S.StencilError) as e:
        _program(**kw)
    assert e.value.status == status


def test_program_plans_refuse_sweeps_and_apply_validates():
    p = _program()
    lib = _abi.lib()
    fake = (C.c_void_p * 3)(256, 512, 768)
    assert lib.stencil_run(p.handle, fake, 1, None, None, None) == -5
    outs = (C.c_void_p * 1)(256)
    ins = (C.c_void_p * 2)(256, 512)
    assert lib.stencil_program_apply(p.handle, outs, ins, None) == -1       # output aliases input
    ins2 = (C.c_void_p * 2)(512, 769)
    assert lib.stencil_program_apply(p.handle, outs, ins2, None) == -1      # misaligned input
    sweep = S.Plan(S.HEAT, (8, 8, 8), 1, [1.0, 1.0])
    assert lib.stencil_program_apply(sweep.handle, outs, ins, None) == -5


@pytest.mark.parametrize("grid,coord,periodic", [([2, 2, 2], [0, 1, 1], False),
                                                 ([1, 3, 2], [0, 1, 0], False),
                                                 ([1, 1, 1], [0, 0, 0], True),
                                                 ([3, 1, 4], [2, 0, 3], True)])
def test_box_exchange_generator_matches_oracle(grid, coord, periodic):
    shape, halo = [12, 10, 14], 2
    p = _program(tuple(shape), halo=halo, terms=[(0, 1.0, [(0, (1, -2, 1))])])
    mine = [e.as_dict(3) for e in p.exchanges(grid, coord, periodic, box=True)]
    ref = [e.as_dict(3) for e in oracle.exchanges(shape, halo, 2, grid, coord, periodic, box=True)]
    assert mine == ref


def test_pw_advection_program_shape():
    from paper_2404_02218_amd.program import pw_advection_terms
    t = pw_advection_terms(1.0, 2.0, 3.0)
    assert len(t) == 60
    assert [sum(1 for o, _, _ in t if o == k) for k in range(3)] == [20, 20, 20]
    assert all(len(f) == 2 and max(abs(x) for _, off in f for x in off) == 1 or
               max(abs(x) for _, off in f for x in off) <= 1 for _, _, f in t)


def test_program_variants_and_compiled_kernel_limits():
    """Programs compile (hiprtc, gfx950) at creation: the largest one the
    limits allow (4 inputs and outputs, reach 2 on every axis, 64 terms: the
    most LDS) and 1D/2D ones.  The 64 x 32 compiled form is offered only where
    its LDS ring fits a compute unit (not for the 3D one here).  stencil_tune
    takes program plans; its argument checks come before any device call."""
    rng = np.random.default_rng(5)
    for ndim in (1, 2, 3):
        terms = [(int(rng.integers(0, 4)), float(rng.standard_normal()),
                  [(int(rng.integers(0, 4)), tuple(int(x) for x in rng.integers(-2, 3, size=ndim)))
                   for _ in range(int(rng.integers(1, 3)))]) for _ in range(64)]
        terms[0] = (0, 1.0, [(3, (2,) * ndim), (2, (-2,) * ndim)])
        p = _program(shape=(7, 9, 11)[3 - ndim:], halo=2, nin=4, nout=4, terms=terms)
        names = ["program_rtc_64x16_t256", "program_interp_64x16_t256", "program_rtc_tight_64x16_t256"]
        # LDS of the 64 x 32 form: 4 inputs x (2 rz + 2) planes x (32 + 2 ry) rows x 72 floats
        rz, ry = (2 if ndim == 3 else 0), (2 if ndim >= 2 else 0)
        if 4 * (2 * rz + 2) * (32 + 2 * ry) * 72 * 4 <= 160 * 1024:
            names.append("program_rtc_64x32_t512")
        assert ndim == 3 or len(names) == 4
        assert p.variant_count() == len(names)
        assert [p.variant_name(v) for v in range(len(names))] == names
        assert p.variant == 0
        p.variant = 1
        assert p.variant == 1
    lib = _abi.lib()
    fake = (C.c_void_p * 8)(*[256 * (k + 1) for k in range(8)])
    assert lib.stencil_tune(p.handle, fake, 0, None) == -1
    assert lib.stencil_tune(p.handle, None, 1, None) == -1


@pytest.mark.parametrize("shape", [(5, 6, 7), (4, 9), (11,), (1, 6, 5)])
def test_interp_weights_equal_the_oracle(shape):
    """stencil_interp_weights (host only) gives the oracle's corners and weights."""
    rng = np.random.default_rng(sum(shape))
    nd = len(shape)
    hi = np.array(shape, dtype=np.float64) - 1
    pos = rng.uniform(0, 1, size=(30, nd)) * hi
    pos[0], pos[1] = hi, 0
    plan = S.Plan(S.WAVE2, shape, 1, [-2.0, 1.0], halo=1)
    c, w = plan.interp_weights(pos)
    co, wo = oracle.interp(shape, pos)
    assert np.array_equal(c, co) and np.array_equal(w, wo)
    for bad in (-1e-9, hi[0] + 1e-9, float("nan")):
        p = pos[:1].copy()
        p[0, 0] = bad
        with pytest.raises(S.StencilError) as e:
            plan.interp_weights(p)
        assert e.value.status == -1


def test_damping_validation_and_profile_helper():
    plan = S.Plan(S.WAVE2, (6, 7, 8), 1, [-2.0, 1.0], halo=1)
    with pytest.raises(S.StencilError) as e:
        plan.set_damping([np.zeros(6), np.zeros(7), -np.ones(8)])
    assert e.value.status == -1
    with pytest.raises(ValueError):
        plan.set_damping([np.zeros(6), np.zeros(7)])
    with pytest.raises(S.StencilError) as e:
        S.Plan(S.HEAT, (6, 7, 8), 1, [1.0, 1.0]).set_damping([np.zeros(6), np.zeros(7), np.zeros(8)])
    assert e.value.status == -5
    with pytest.raises(S.StencilError) as e:
        S.Plan(S.WAVE2, (6, 7, 8), 1, [-2.0, 1.0], dtype=S.BF16).set_damping([np.zeros(n) for n in (6, 7, 8)])
    assert e.value.status == -2
    for n, width in ((20, 5), (7, 4), (1, 3)):
        assert np.array_equal(S.damping_profile(n, width, 0.3), W.damping_profiles((n,), width, 0.3)[0])
    p = S.damping_profile(20, 5, 0.3)
    assert p[0] == p[-1] == 0.3 and p[5] == 0 and p[4] == pytest.approx(0.3 / 25)
