"""Stencil programs (stencil_program_create / stencil_program_apply): several
output fields, each a sum of linear or quadratic terms over several input
fields at arbitrary offsets, evaluated in one fused launch.

`pw_advection_terms` writes the flux-form, centred advection of a velocity
(u, v, w) on a staggered C grid as such a program (the Piacsek-Williams
scheme that Section 6.2 benchmarks as "PW advection"; the paper prints no
formulas, so the scheme is written here from its definition).
"""
from __future__ import annotations

import ctypes as C
from typing import NamedTuple

from . import F32, Plan, _i64
from ._abi import ACT_EXCHANGE, Action, Step, Term, call


def _term_array(terms, ndim):
    arr = (Term * max(1, len(terms)))()
    for t, (o, c, facs) in enumerate(terms):
        if not 1 <= len(facs) <= 2:
            raise ValueError("a term has 1 or 2 factors")
        arr[t].out = int(o)
        arr[t].coeff = float(c)
        arr[t].nfac = len(facs)
        for k, (f, off) in enumerate(facs):
            if len(off) != ndim:
                raise ValueError(f"offsets have {ndim} components")
            arr[t].inp[k] = int(f)
            off3 = [0] * (3 - ndim) + [int(x) for x in off]
            for a in range(3):
                arr[t].off[k][a] = off3[a]
    return arr


class Program(Plan):
    """A fused stencil program over `shape` (ndim 1..3) with halo `halo`.

    terms: sequence of (out, coeff, [(in_field, offset), ...]) with one or
    two factors; offsets have ndim components (C order) within min(halo, 2).
    Fields come from `field()` and share the plan's layout.  The sweep
    methods of Plan (run, apply, ...) are refused by the library for a
    program plan; exchanges, pack and unpack work as for any plan.
    """

    def __init__(self, shape, halo: int, nin: int, nout: int, terms, dtype: int = F32):
        self.kind, self.dtype, self.bc = -1, dtype, 0
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        self.halo = int(halo)
        self.nin, self.nout = int(nin), int(nout)
        self.terms = [(int(o), float(c), [(int(f), tuple(int(x) for x in off)) for f, off in facs])
                      for o, c, facs in terms]
        self.radius = max([1] + [abs(x) for _, _, facs in self.terms for _, off in facs for x in off])
        self.coeffs = []
        h = C.c_void_p()
        arr = _term_array(self.terms, self.ndim)
        call("stencil_program_create", C.byref(h), self.ndim, _i64(self.shape), self.halo, self.nin,
             self.nout, C.cast(arr, C.c_void_p), len(self.terms), dtype)
        self._h = h
        self.layout = self._layout()

    def apply_program(self, outs, ins, stream=None):
        """Evaluate once: outs (nout Fields) from ins (nin Fields)."""
        from . import _stream_ptr
        if len(outs) != self.nout or len(ins) != self.nin:
            raise ValueError(f"expected {self.nout} outputs and {self.nin} inputs")
        po = (C.c_void_p * self.nout)(*[f.ptr for f in outs])
        pi = (C.c_void_p * self.nin)(*[f.ptr for f in ins])
        call("stencil_program_apply", self._h, po, pi, _stream_ptr(stream))

    def halo_dirs(self, field: int) -> int:
        """Bit mask of the neighbour directions (C-order codes, as
        `dir_code`) in which the program reads input `field` outside the
        interior."""
        m = C.c_uint32()
        call("stencil_program_halo_dirs", self._h, int(field), C.byref(m))
        return m.value


def dir_code(to, ndim: int) -> int:
    """C-order code of a neighbour direction: sum_j (d_j + 1) 3^(ndim-1-j)."""
    c = 0
    for j in range(ndim):
        c = 3 * c + int(to[j]) + 1
    return c


def select(exchanges, dirs: int, ndim: int):
    """The entries of an exchange list whose direction is in the mask."""
    return [e for e in exchanges if dirs >> dir_code(e.to, ndim) & 1]


class Act(NamedTuple):
    kind: str      # "exchange" or "apply"
    step: int      # the step applied, or served first by the exchange (-1: prologue)
    field: int     # exchanged field id (-1 for an apply)
    dirs: int      # direction mask of an exchange


def schedule(steps, nfields: int, loop: bool = True):
    """Exchange schedule (stencil_schedule) of a sequence of applies.
    steps: [(program, input field ids, output field ids)].  Returns
    (prologue, body), lists of Act."""
    arr = (Step * max(1, len(steps)))()
    for k, (prog, ins, outs) in enumerate(steps):
        if len(ins) != prog.nin or len(outs) != prog.nout:
            raise ValueError(f"step {k}: expected {prog.nin} inputs and {prog.nout} outputs")
        arr[k].program = prog.handle
        for i, f in enumerate(ins):
            arr[k].inp[i] = int(f)
        for o, f in enumerate(outs):
            arr[k].out[o] = int(f)
    npro, nbod = C.c_int(0), C.c_int(0)
    call("stencil_schedule", C.cast(arr, C.c_void_p), len(steps), int(nfields), int(bool(loop)), None,
         C.byref(npro), None, C.byref(nbod))
    pro, bod = (Action * max(1, npro.value))(), (Action * max(1, nbod.value))()
    call("stencil_schedule", C.cast(arr, C.c_void_p), len(steps), int(nfields), int(bool(loop)),
         C.cast(pro, C.c_void_p), C.byref(npro), C.cast(bod, C.c_void_p), C.byref(nbod))

    def conv(a):
        return Act("exchange" if a.kind == ACT_EXCHANGE else "apply", a.step, a.field, a.dirs)
    return [conv(pro[i]) for i in range(npro.value)], [conv(bod[i]) for i in range(nbod.value)]


def _product(a, b, scale):
    """Terms of scale * (sum a) * (sum b); a, b: lists of (field, offset)."""
    return [(scale, [fa, fb]) for fa in a for fb in b]


def pw_advection_terms(dx: float, dy: float, dz: float):
    """Program terms (3 inputs u, v, w; 3 outputs su, sv, sw) of the
    flux-form centred advection on a C grid.  u[k][j][i] lives at the x face
    (i+1/2, j, k), v at (i, j+1/2, k), w at (i, j, k+1/2).  Each tendency is
    minus the divergence of its momentum flux, every flux a product of
    two-point averages at the flux position, e.g. for u:

        su = -[ ((u + u_{+x})/2)^2 - ((u_{-x} + u)/2)^2 ] / dx
             -[ (v + v_{+x})/2 (u + u_{+y})/2 - (v_{-y} + v_{-y+x})/2 (u_{-y} + u)/2 ] / dy
             -[ (w + w_{+x})/2 (u + u_{+z})/2 - (w_{-z} + w_{-z+x})/2 (u_{-z} + u)/2 ] / dz

    The squared x-averages are expanded with the u*u terms cancelled
    ((a+b)^2 - (c+a)^2 = b^2 + 2ab - c^2 - 2ca), so each output has 20 terms.
    Offsets are (dz, dy, dx)."""
    U, V, W = 0, 1, 2
    X, Y, Z, O = (0, 0, 1), (0, 1, 0), (1, 0, 0), (0, 0, 0)

    def add(*vs):
        return tuple(sum(c) for c in zip(*vs))

    def neg(v):
        return tuple(-c for c in v)

    def f(field, *offs):
        return (field, add(O, *offs))

    out = []

    def emit(o, pairs):
        for c, facs in pairs:
            out.append((o, c, facs))

    def own_axis(field, e, h):
        # -[((q + q_{+e})/2)^2 - ((q_{-e} + q)/2)^2] / h, expanded
        s = -1.0 / (4.0 * h)
        return [(s, [f(field, e), f(field, e)]), (2 * s, [f(field), f(field, e)]),
                (-s, [f(field, neg(e)), f(field, neg(e))]), (-2 * s, [f(field, neg(e)), f(field)])]

    def cross(q, qe, adv, ae, h):
        # -[ (adv + adv_{+ae})/2 (q + q_{+qe})/2
        #    - (adv_{-qe} + adv_{-qe+ae})/2 (q_{-qe} + q)/2 ] / h
        s = -1.0 / (4.0 * h)
        hi = _product([f(adv), f(adv, ae)], [f(q), f(q, qe)], s)
        lo = _product([f(adv, neg(qe)), f(adv, neg(qe), ae)], [f(q, neg(qe)), f(q)], -s)
        return hi + lo

    emit(0, own_axis(U, X, dx) + cross(U, Y, V, X, dy) + cross(U, Z, W, X, dz))
    emit(1, cross(V, X, U, Y, dx) + own_axis(V, Y, dy) + cross(V, Z, W, Y, dz))
    emit(2, cross(W, X, U, Z, dx) + cross(W, Y, V, Z, dy) + own_axis(W, Z, dz))
    return out
