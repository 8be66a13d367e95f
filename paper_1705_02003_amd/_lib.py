"""ctypes declarations of libens.so (include/ens.h).  Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libens.so")

ENS_OK = 0
ENS_EINVAL = -1
ENS_ENOMEM = -2
ENS_EHIP = -3
ENS_ENOTSUP = -4

CONVERGED, MAX_ITER, BREAKDOWN, ZERO_RHS = 0, 1, 2, 3
PRECOND_JACOBI, PRECOND_CHEBYSHEV, PRECOND_MULTIGRID = 0, 1, 2
FLAG_TIME_SPMV = 1
FLAG_FULL_STENCIL = 2
FLAG_MG_LEVELWISE = 4
NOALLOC_SCRATCH_BYTES = 64 << 20

i32 = C.c_int32
i32p = C.POINTER(C.c_int32)
f64 = C.c_double
f64p = C.POINTER(C.c_double)
vp = C.c_void_p
sz = C.c_size_t


class ens_problem(C.Structure):
    _fields_ = [("n", i32), ("d", i32), ("eps_model", i32), ("dim", i32), ("amp", f64)]


class ens_opts(C.Structure):
    _fields_ = [("precond", i32), ("cheb_degree", i32), ("cheb_ratio", f64), ("rtol", f64),
                ("max_iter", i32), ("poll_every", i32), ("tile_lines", i32),
                ("max_groups", i32), ("flags", i32), ("member_tile", i32)]


class ens_stats(C.Structure):
    _fields_ = [("ens_iters", i32), ("spmv_timed", i32), ("spmv_ms", f64),
                ("spmv_groups", i32), ("tile_lines", i32)]


class ens_batch_item(C.Structure):
    _fields_ = [("prob", ens_problem), ("S", i32), ("tile_lines", i32),
                ("V_dev", vp), ("b_dev", vp), ("x_dev", vp), ("ws_dev", vp), ("ws_bytes", sz),
                ("iters_host", i32p), ("status_host", i32p), ("relres_host", f64p),
                ("ens_iters", i32), ("member_tile", i32), ("seconds", f64)]


PP = C.POINTER(ens_problem)
OP = C.POINTER(ens_opts)
SP = C.POINTER(ens_stats)

# name -> (restype, argtypes); every symbol declared in include/ens.h
SIGNATURES = {
    "ens_assemble_ensemble": (C.c_int, [PP, i32, vp, vp, vp, vp]),
    "ens_matrix_slot_stride": (sz, [PP, i32]),
    "ens_pcg_workspace_bytes": (sz, [PP, OP, i32]),
    "ens_pcg_solve": (C.c_int, [PP, OP, i32, vp, vp, vp, i32p, i32p, f64p, i32p, SP, vp, sz, vp]),
    "ens_pcg_solve_noalloc": (C.c_int, [PP, OP, i32, vp, vp, vp, i32p, i32p, f64p, i32p, vp]),
    "ens_spmv": (C.c_int, [PP, i32, vp, vp, vp, vp]),
    "ens_cheb_apply": (C.c_int, [PP, OP, i32, vp, vp, vp, f64p, vp, sz, vp]),
    "ens_mg_apply": (C.c_int, [PP, OP, i32, vp, vp, vp, f64p, vp, sz, vp]),
    "ens_member_dot": (C.c_int, [i32, i32, vp, vp, i32, f64p, vp, sz, vp]),
    "ens_adjoint_grad": (C.c_int, [PP, OP, i32, vp, vp, vp, vp, vp, f64p, i32p, i32p, vp, sz, vp]),
    "ens_dqdy": (C.c_int, [PP, i32, vp, vp, vp, f64p, vp, sz, vp]),
    "ens_qoi_weights": (C.c_int, [PP, vp, vp]),
    "ens_group_samples": (C.c_int, [i32, i32, i32p, i32p, f64p, i32, f64p, i32, i32p, f64p]),
    "ens_sg_surpluses": (C.c_int, [i32, i32, i32p, i32p, f64p, f64p]),
    "ens_sg_expectation": (C.c_int, [i32, i32, i32p, i32p, f64p, f64p]),
    "ens_param_indicator": (C.c_int, [PP, i32, vp, f64p, vp, sz, vp]),
    "ens_group_variable": (C.c_int, [i32, f64p, i32, i32p, f64p, i32p, i32p, i32p, i32p, f64p]),
    "ens_sg_coords": (C.c_int, [i32, i32, i32p, i32p, f64p]),
    "ens_sg_refine": (C.c_int, [i32, i32, i32p, i32p, f64p, i32, f64, i32, i32, i32p, i32p, i32p]),
    "ens_batch_workspace_bytes": (sz, [i32]),
    "ens_batch_solve": (C.c_int, [OP, i32, C.POINTER(ens_batch_item), vp, sz, vp]),
    "ens_strerror": (C.c_char_p, [C.c_int]),
    "ens_last_hip_error": (C.c_int, []),
    "ens_version": (C.c_int, []),
    "ens_stream_triad": (C.c_int, [vp, vp, vp, f64, sz, vp]),
    "ens_stream_mix": (C.c_int, [vp, vp, sz, sz, i32, i32, vp]),
}

_lib = None


class EnsError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().ens_strerror(code).decode()
        if code == ENS_EHIP:
            msg += f" (hipError {lib().ens_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{code}]")
        self.code = code


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1705_02003_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int, where: str) -> None:
    if rc != ENS_OK:
        raise EnsError(rc, where)
