"""ctypes declarations of libstencil.so (include/stencil.h), same names.

Argument marshalling only: every computation runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstencil.so")

STENCIL_OK = 0
STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_UNSUPPORTED", -3: "E_NOMEM", -4: "E_DEVICE",
                -5: "E_STATE"}

HEAT, WAVE2 = 0, 1
F32, BF16, F16 = 0, 1, 2
BC_DIRICHLET0, BC_PERIODIC = 0, 1


class StencilError(RuntimeError):
    def __init__(self, status: int, what: str, message: str):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}: {message}")


class Exchange(C.Structure):
    _fields_ = [("at", C.c_int64 * 3), ("size", C.c_int64 * 3),
                ("src_offset", C.c_int64 * 3), ("to", C.c_int32 * 3), ("reserved", C.c_int32)]

    def as_dict(self, ndim: int) -> dict:
        return {"at": list(self.at[:ndim]), "size": list(self.size[:ndim]),
                "src_offset": list(self.src_offset[:ndim]), "to": list(self.to[:ndim])}


class Term(C.Structure):
    """stencil_term: out += coeff * in[0](i + off[0]) (* in[1](i + off[1]))."""
    _fields_ = [("out", C.c_int32), ("nfac", C.c_int32), ("inp", C.c_int32 * 2),
                ("off", (C.c_int32 * 3) * 2), ("coeff", C.c_double)]


class Step(C.Structure):
    """stencil_step: a program plan and the field ids of its inputs and outputs."""
    _fields_ = [("program", C.c_void_p), ("inp", C.c_int32 * 4), ("out", C.c_int32 * 4)]


class Action(C.Structure):
    """stencil_action: an exchange of `field` in `dirs`, or an apply of `step`."""
    _fields_ = [("kind", C.c_int32), ("step", C.c_int32), ("field", C.c_int32), ("dirs", C.c_uint32)]


ACT_EXCHANGE, ACT_APPLY = 0, 1


class SourceInterp(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.c_void_p), ("amp", C.c_void_p)]


class ReceiversInterp(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.c_void_p), ("trace", C.c_void_p)]


class Source(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.c_void_p), ("amp", C.c_void_p), ("scale", C.c_void_p)]


class Receivers(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.c_void_p), ("trace", C.c_void_p)]


class CheckReport(C.Structure):
    """stencil_check_report."""
    _fields_ = [("nan_count", C.c_int64), ("inf_count", C.c_int64), ("max_abs", C.c_double),
                ("beta_max", C.c_double), ("stability", C.c_double), ("headroom", C.c_double),
                ("flags", C.c_int32), ("reserved", C.c_int32)]


CHECK_NONFINITE, CHECK_OVERFLOW, CHECK_UNSTABLE, CHECK_BAD_BETA = 1, 2, 4, 8


EXPORTS = [
    "stencil_create", "stencil_destroy", "stencil_layout", "stencil_apply", "stencil_run", "stencil_run_noalloc",
    "stencil_run_interp", "stencil_interp_weights", "stencil_wave_damping",
    "stencil_exchanges", "stencil_exchanges_box", "stencil_halo_pack", "stencil_halo_unpack",
    "stencil_program_create", "stencil_program_apply", "stencil_program_halo_dirs", "stencil_schedule",
    "stencil_batch_create",
    "stencil_batch_layout", "stencil_batch_run", "stencil_adjoint_workspace",
    "stencil_forward_ckpt", "stencil_adjoint", "stencil_gradient", "stencil_wave_beta",
    "stencil_wave_point_scale", "stencil_run_workspace", "stencil_set_workspace", "stencil_stability",
    "stencil_check", "stencil_variant_count",
    "stencil_variant_name", "stencil_get_variant", "stencil_set_variant", "stencil_tune",
    "stencil_last_error", "stencil_abi_version",
]

_lib = None


def lib():
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_2404_02218_amd/build.py`; there is no CPU fallback")
    # torch ships its own HIP runtime.  Loaded first, it is the one the
    # library's HIP dependency binds to, so device pointers and streams from
    # torch are valid here; loaded after the library, a second runtime would
    # come up beside the system one, and whichever initialises second finds
    # no device.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P, I, I64, D = C.c_void_p, C.c_int, C.c_int64, C.c_double
    st = C.c_int
    sig = {
        "stencil_create": [P, I, I, P, I, P, I, I, I],
        "stencil_destroy": [P],
        "stencil_layout": [P, P, P, P, P],
        "stencil_apply": [P, P, P, P, P, P],
        "stencil_run": [P, P, I64, P, P, P],
        "stencil_run_noalloc": [P, P, I64, P, P, P],
        "stencil_run_interp": [P, P, I64, P, P, P],
        "stencil_interp_weights": [P, I64, P, P, P],
        "stencil_wave_damping": [P, P],
        "stencil_exchanges": [P, P, P, I, P, P],
        "stencil_exchanges_box": [P, P, P, I, P, P],
        "stencil_program_create": [P, I, P, I, I, I, P, I, I],
        "stencil_program_apply": [P, P, P, P],
        "stencil_program_halo_dirs": [P, I, P],
        "stencil_schedule": [P, I, I, I, P, P, P, P],
        "stencil_halo_pack": [P, P, P, I, P, P],
        "stencil_halo_unpack": [P, P, P, I, P, P],
        "stencil_batch_create": [P, I, P, I, P, I, I],
        "stencil_batch_layout": [P, I, P, P, P, P],
        "stencil_batch_run": [P, P, I64, P, P, P],
        "stencil_adjoint_workspace": [P, I64, I64, P],
        "stencil_forward_ckpt": [P, P, I64, I64, P, P, P, C.c_size_t, P],
        "stencil_adjoint": [P, P, I64, I64, P, P, P, P, D, P, P, C.c_size_t, P],
        "stencil_gradient": [P, P, P, D, D, I64, I64, P, P, P, P, P, P, C.c_size_t, P],
        "stencil_wave_beta": [P, P, D, D, P, P],
        "stencil_wave_point_scale": [P, P, D, I64, P, P, P],
        "stencil_run_workspace": [P, P],
        "stencil_set_workspace": [P, P, C.c_size_t, P],
        "stencil_stability": [P, P],
        "stencil_check": [P, P, P, P],
        "stencil_variant_count": [P, P],
        "stencil_variant_name": [P, I, P, C.c_size_t],
        "stencil_get_variant": [P, P],
        "stencil_set_variant": [P, I],
        "stencil_tune": [P, P, I, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = st
    L.stencil_last_error.argtypes = []
    L.stencil_last_error.restype = C.c_char_p
    L.stencil_abi_version.argtypes = []
    L.stencil_abi_version.restype = C.c_int
    _lib = L
    return L


def check(status: int, what: str) -> None:
    if status != STENCIL_OK:
        msg = lib().stencil_last_error().decode(errors="replace")
        raise StencilError(status, what, msg)


def call(name: str, *args) -> None:
    check(getattr(lib(), name)(*args), name)
