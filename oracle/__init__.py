"""FP64 CPU oracle for the star-stencil sweep: heat/Jacobi, second-order
acoustic wave, its adjoint and misfit gradient, the halo exchange
declarations (faces, or faces, edges and corners) with pack/unpack, fused
stencil programs over several fields, and a flux-form C-grid advection.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
path: the arithmetic lives in `stencil_oracle.c` (plain C, FP64) and the
finite-difference weights are derived here from their moment conditions
(`fd_weights.py`).  Arrays are dense NumPy FP64 buffers whose bounds include
the halo.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .fd_weights import fd_weights, fd_weights_float, symbol  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class OracleError(RuntimeError):
    pass


class Exchange(C.Structure):
    """One exchange declaration: receive box [at, at+size), send box shifted by
    src_offset, partner at relative rank `to` (first ndim slots used)."""
    _fields_ = [("at", C.c_int64 * 3), ("size", C.c_int64 * 3),
                ("src_offset", C.c_int64 * 3), ("to", C.c_int32 * 3), ("pad_", C.c_int32)]

    def as_dict(self, ndim: int) -> dict:
        return {"at": list(self.at[:ndim]), "size": list(self.size[:ndim]),
                "src_offset": list(self.src_offset[:ndim]), "to": list(self.to[:ndim])}


def use_library(path: str) -> None:
    """Load the oracle from `path` (a build of the same source, e.g. one
    compiled for the host's own instruction set) instead of the in-tree
    library; must be called before the first oracle call."""
    global _lib, _LIB_PATH
    if _lib is not None:
        raise OracleError("the oracle library is already loaded")
    _LIB_PATH = path


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from .build import build
        build()
    lib = C.CDLL(_LIB_PATH)
    P = C.c_void_p
    I64 = C.c_int64
    lib.orc_star.argtypes = [C.c_int, P, C.c_int, C.c_int, P, P, P]
    lib.orc_heat_run.argtypes = [C.c_int, P, C.c_int, C.c_int, P, C.c_int, P, I64]
    lib.orc_wave_run.argtypes = [C.c_int, P, C.c_int, C.c_int, P, C.c_int, P, P, P, I64,
                                 I64, P, P, I64, P, P]
    lib.orc_wave_adjoint.argtypes = [C.c_int, P, C.c_int, C.c_int, P, P, I64, I64, P, P, P,
                                     I64, P, P]
    lib.orc_wave_gradient.argtypes = [C.c_int, P, C.c_int, C.c_int, P, P, I64, I64, P, P, I64,
                                      P, P, P, C.c_double, P, P, P]
    lib.orc_exchanges.argtypes = [C.c_int, P, C.c_int, C.c_int, P, P, C.c_int, P, P]
    lib.orc_exchanges_box.argtypes = [C.c_int, P, C.c_int, C.c_int, P, P, C.c_int, P, P]
    lib.orc_program.argtypes = [C.c_int, P, C.c_int, C.c_int, P, C.c_int, P, C.c_int, P]
    lib.orc_pw_advection.argtypes = [P, C.c_int, P, P, P, C.c_double, C.c_double, C.c_double, P, P, P]
    lib.orc_pack.argtypes = [C.c_int, P, C.c_int, P, P, C.c_int, P]
    lib.orc_unpack.argtypes = [C.c_int, P, C.c_int, P, P, C.c_int, P]
    lib.orc_interp.argtypes = [C.c_int, P, I64, P, P, P]
    lib.orc_wave_run_damped.argtypes = [C.c_int, P, C.c_int, C.c_int, P, P, P, P, P, I64, I64, P, P, I64, P, P]
    for f in ("orc_star", "orc_heat_run", "orc_wave_run", "orc_wave_adjoint",
              "orc_wave_gradient", "orc_exchanges", "orc_pack", "orc_unpack", "orc_interp",
              "orc_wave_run_damped"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _shape_of(buf, halo):
    return np.array([s - 2 * halo for s in buf.shape], dtype=np.int64)


def _coeffs(c):
    return np.ascontiguousarray([float(x) for x in c], dtype=np.float64)


def _pos(p, ndim):
    if p is None:
        return None, 0
    p = np.asarray(p, dtype=np.int64).reshape(-1, ndim)
    out = np.zeros((p.shape[0], 3), dtype=np.int64)
    out[:, :ndim] = p
    return np.ascontiguousarray(out), p.shape[0]


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def star(u, halo, radius, c):
    """(L u) on the interior; halo entries of the result are zero."""
    lib = _load()
    u = _f64(u)
    out = np.zeros_like(u)
    shape = _shape_of(u, halo)
    _check(lib.orc_star(u.ndim, _p(shape), halo, radius, _p(_coeffs(c)), _p(u), _p(out)), "star")
    return out


def heat_run(u, halo, radius, c, nsteps, periodic=False):
    """nsteps of u <- u + L u (weights already scaled by a dt / h^2)."""
    lib = _load()
    u = _f64(u).copy()
    shape = _shape_of(u, halo)
    _check(lib.orc_heat_run(u.ndim, _p(shape), halo, radius, _p(_coeffs(c)), int(periodic),
                            _p(u), int(nsteps)), "heat_run")
    return u


def wave_run(u_n, u_nm1, beta, halo, radius, c, nsteps, src=None, src_amp=None, rec=None,
             periodic=False, inplace=False):
    """nsteps leapfrog steps; returns (u^N, u^{N-1}, traces[N, nrec]).  With
    inplace=True the two levels must be C-contiguous FP64 arrays and are
    advanced where they are (no copies)."""
    lib = _load()
    if inplace:
        for x in (u_n, u_nm1):
            if x.dtype != np.float64 or not x.flags.c_contiguous:
                raise OracleError("in-place levels must be C-contiguous FP64 arrays")
        a, b = u_n, u_nm1
    else:
        a = _f64(u_n).copy()
        b = _f64(u_nm1).copy()
    beta = _f64(beta)
    ndim = a.ndim
    shape = _shape_of(a, halo)
    sp, ns = _pos(src, ndim)
    rp, nr = _pos(rec, ndim)
    amp = _f64(src_amp).reshape(-1) if ns else None
    if ns and amp.size < nsteps * ns:
        raise OracleError("src_amp must hold nsteps x nsrc values")
    traces = np.zeros((int(nsteps), nr), dtype=np.float64)
    _check(lib.orc_wave_run(ndim, _p(shape), halo, radius, _p(_coeffs(c)), int(periodic),
                            _p(beta), _p(a), _p(b), int(nsteps), ns, _p(sp), _p(amp), nr, _p(rp),
                            _p(traces)), "wave_run")
    return a, b, traces


def wave_run_damped(u_n, u_nm1, beta, gamma, halo, radius, c, nsteps, src=None, src_amp=None, rec=None):
    """The damped leapfrog (absorbing layer); gamma is a buffer like beta.
    Returns (u^N, u^{N-1}, traces[N, nrec])."""
    lib = _load()
    a = _f64(u_n).copy()
    b = _f64(u_nm1).copy()
    beta, gamma = _f64(beta), _f64(gamma)
    ndim = a.ndim
    shape = _shape_of(a, halo)
    sp, ns = _pos(src, ndim)
    rp, nr = _pos(rec, ndim)
    amp = _f64(src_amp).reshape(-1) if ns else None
    if ns and amp.size < nsteps * ns:
        raise OracleError("src_amp must hold nsteps x nsrc values")
    traces = np.zeros((int(nsteps), nr), dtype=np.float64)
    _check(lib.orc_wave_run_damped(ndim, _p(shape), halo, radius, _p(_coeffs(c)), _p(beta), _p(gamma), _p(a),
                                   _p(b), int(nsteps), ns, _p(sp), _p(amp), nr, _p(rp), _p(traces)),
           "wave_run_damped")
    return a, b, traces


def interp(shape, pos):
    """Corners [n, 2^ndim, ndim] (interior coordinates) and weights
    [n, 2^ndim] of real positions [n, ndim] (multilinear interpolation)."""
    lib = _load()
    ndim = len(shape)
    p = np.asarray(pos, dtype=np.float64).reshape(-1, ndim)
    n, nc = p.shape[0], 1 << ndim
    p3 = np.zeros((max(n, 1), 3))
    p3[:n, :ndim] = p
    corners = np.zeros((max(n, 1), nc, 3), dtype=np.int64)
    w = np.zeros((max(n, 1), nc))
    _check(lib.orc_interp(ndim, _p(np.asarray(shape, dtype=np.int64)), n, _p(p3), _p(corners), _p(w)), "interp")
    return corners[:n, :, :ndim], w[:n]


def wave_adjoint(beta, halo, radius, c, nsteps, rec, rec_w, resid, probe):
    """Adjoint sweep driven by residuals at receivers; returns lam^n at the
    probe points, shape [N, nprobe], row n = level n (0..N-1)."""
    lib = _load()
    beta = _f64(beta)
    ndim = beta.ndim
    shape = _shape_of(beta, halo)
    rp, nr = _pos(rec, ndim)
    pp, npb = _pos(probe, ndim)
    rec_w = _f64(rec_w).reshape(-1)
    resid = _f64(resid).reshape(-1)
    out = np.zeros((int(nsteps), npb), dtype=np.float64)
    _check(lib.orc_wave_adjoint(ndim, _p(shape), halo, radius, _p(_coeffs(c)), _p(beta),
                                int(nsteps), nr, _p(rp), _p(rec_w), _p(resid), npb, _p(pp),
                                _p(out)), "wave_adjoint")
    return out


def wave_gradient(beta, halo, radius, c, nsteps, src, src_amp, rec, dobs, rec_w, gscale):
    """Forward run, misfit and gradient; returns (traces[N, nrec], J, grad)."""
    lib = _load()
    beta = _f64(beta)
    ndim = beta.ndim
    shape = _shape_of(beta, halo)
    sp, ns = _pos(src, ndim)
    rp, nr = _pos(rec, ndim)
    amp = _f64(src_amp).reshape(-1)
    dobs = _f64(dobs).reshape(-1)
    rec_w = _f64(rec_w).reshape(-1)
    traces = np.zeros((int(nsteps), nr), dtype=np.float64)
    J = np.zeros(1, dtype=np.float64)
    grad = np.zeros(tuple(int(s) for s in shape), dtype=np.float64)
    _check(lib.orc_wave_gradient(ndim, _p(shape), halo, radius, _p(_coeffs(c)), _p(beta),
                                 int(nsteps), ns, _p(sp), _p(amp), nr, _p(rp), _p(dobs),
                                 _p(rec_w), float(gscale), _p(traces), _p(J), _p(grad)),
           "wave_gradient")
    return traces, float(J[0]), grad


def exchanges(shape, halo, radius, grid, coord, periodic=False, box=False):
    """Exchange declarations of one rank (list of Exchange): faces only, or
    with box=True faces, edges and corners (every neighbour direction)."""
    lib = _load()
    ndim = len(shape)
    shp = np.asarray(shape, dtype=np.int64)
    g = np.asarray(grid, dtype=np.int32)
    cc = np.asarray(coord, dtype=np.int32)
    arr = (Exchange * 26)()
    n = C.c_int(26)
    fn = lib.orc_exchanges_box if box else lib.orc_exchanges
    _check(fn(ndim, _p(shp), halo, radius, _p(g), _p(cc), int(periodic), C.cast(arr, C.c_void_p), C.byref(n)),
           "exchanges")
    return [arr[i] for i in range(n.value)]


class Term(C.Structure):
    """One program term: out += coeff * in[0](i + off[0]) (* in[1](i + off[1]))."""
    _fields_ = [("out", C.c_int32), ("nfac", C.c_int32), ("inp", C.c_int32 * 2),
                ("off", (C.c_int32 * 3) * 2), ("coeff", C.c_double)]


def program(ins, halo, nout, terms):
    """Evaluate a stencil program.  ins: equal-shape FP64 buffers (halo
    included); terms: (out, coeff, [(field, offset), ...]) with 1 or 2
    factors and offsets of len(shape) components.  Returns nout buffers with
    the interior computed and a zero halo."""
    lib = _load()
    ins = [_f64(a) for a in ins]
    ndim = ins[0].ndim
    shape = _shape_of(ins[0], halo)
    outs = [np.zeros_like(ins[0]) for _ in range(nout)]
    arr = (Term * max(1, len(terms)))()
    for t, (o, c, facs) in enumerate(terms):
        arr[t].out = o
        arr[t].coeff = c
        arr[t].nfac = len(facs)
        for k, (f, off) in enumerate(facs):
            arr[t].inp[k] = f
            off3 = [0] * (3 - ndim) + list(off)
            for a in range(3):
                arr[t].off[k][a] = int(off3[a])
    pin = (C.c_void_p * len(ins))(*[a.ctypes.data for a in ins])
    pout = (C.c_void_p * nout)(*[a.ctypes.data for a in outs])
    _check(lib.orc_program(ndim, _p(shape), halo, len(ins), C.cast(pin, C.c_void_p), nout,
                           C.cast(pout, C.c_void_p), len(terms), C.cast(arr, C.c_void_p)), "program")
    return outs


def pw_advection(u, v, w, halo, dx, dy, dz):
    """Advective tendencies (su, sv, sw) of a C-grid velocity (3D buffers with
    their halos already filled); interior computed, halo zero."""
    lib = _load()
    u, v, w = _f64(u), _f64(v), _f64(w)
    shape = _shape_of(u, halo)
    su, sv, sw = np.zeros_like(u), np.zeros_like(u), np.zeros_like(u)
    _check(lib.orc_pw_advection(_p(shape), halo, _p(u), _p(v), _p(w), float(dx), float(dy), float(dz),
                                _p(su), _p(sv), _p(sw)), "pw_advection")
    return su, sv, sw


def _ex_array(ex):
    arr = (Exchange * max(1, len(ex)))()
    for i, e in enumerate(ex):
        arr[i] = e
    return arr


def exchange_elems(ex, ndim):
    return int(np.prod([e for e in ex.size[:ndim]]))


def pack(field, halo, ex):
    lib = _load()
    field = _f64(field)
    ndim = field.ndim
    shape = _shape_of(field, halo)
    total = sum(exchange_elems(e, ndim) for e in ex)
    buf = np.zeros(max(total, 1), dtype=np.float64)
    _check(lib.orc_pack(ndim, _p(shape), halo, _p(field), C.cast(_ex_array(ex), C.c_void_p),
                        len(ex), _p(buf)), "pack")
    return buf[:total]


def unpack(field, halo, ex, buf):
    """Returns a copy of `field` with the receive boxes filled from `buf`."""
    lib = _load()
    field = _f64(field).copy()
    ndim = field.ndim
    shape = _shape_of(field, halo)
    buf = _f64(buf)
    _check(lib.orc_unpack(ndim, _p(shape), halo, _p(field), C.cast(_ex_array(ex), C.c_void_p),
                          len(ex), _p(buf)), "unpack")
    return field
