"""ctypes loader and struct mirrors of the C ABI in include/excmg.h.

The shared library is built in-tree (``paper_1507_05063_amd/libexcmg.so``).  There is no fallback: if the library is
missing, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libexcmg.so")

OK = 0
ERR_ARG, ERR_SHAPE, ERR_NONFINITE, ERR_NOCONV, ERR_BREAKDOWN, ERR_HIP, ERR_WORKSPACE = -1, -2, -3, -4, -5, -6, -7
ERR_SCRATCH = -8
NOALLOC_MAX_BYTES = 128 << 20
FP64, FP32_IR = 0, 1
WANT_HISTORY, WANT_TIMING, NO_GRAPHS, GUESS_QUADRATIC, GUESS_LINEAR, STOP_F_G = 1, 2, 4, 8, 16, 32
GUESS_KINDS = {"quartic": 0, "quadratic": 1, "linear": 2}
GUESS_FLAGS = {"quartic": 0, "quadratic": GUESS_QUADRATIC, "linear": GUESS_LINEAR}
STOP_F_G_BELOW_FINEST = 64
TWO_PASS_CG = 256
STOP_NORM_FLAGS = {"b": 0, "fg": STOP_F_G, "fg_coarse": STOP_F_G_BELOW_FINEST}
MAX_LEVELS, MAX_HISTORY = 16, 256

K_CLASSES = ["cg_a", "cg_b", "cg_a32", "cg_b32", "resid", "finalize", "rhs", "exp_finite", "exp_true", "dsolve",
             "gradient", "other", "cg_a0", "cg_b0"]


class Problem(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double * 3),
        ("n", ctypes.c_int32 * 3),
        ("n_coarse", ctypes.c_int32 * 3),
        ("tol", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("inner_tol", ctypes.c_double),
        ("max_iters", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("tol_order", ctypes.c_double),
        ("tol_coarse", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("n", (ctypes.c_int32 * 3) * MAX_LEVELS),
        ("iters", ctypes.c_int32 * MAX_LEVELS),
        ("ir_outer", ctypes.c_int32 * MAX_LEVELS),
        ("dsolve_iters", ctypes.c_int32 * 2),
        ("relres", ctypes.c_double * MAX_LEVELS),
        ("ms_level", ctypes.c_double * MAX_LEVELS),
        ("ms_total", ctypes.c_double),
        ("kernel_ms", ctypes.c_double * len(K_CLASSES)),
        ("kernel_calls", ctypes.c_int32 * len(K_CLASSES)),
        ("kernel_ms_finest", ctypes.c_double * len(K_CLASSES)),
        ("kernel_calls_finest", ctypes.c_int32 * len(K_CLASSES)),
        ("history_len", ctypes.c_int32),
        ("history", ctypes.c_double * MAX_HISTORY),
    ]

    def to_dict(self) -> dict:
        L = self.levels
        return {
            "levels": L,
            "n": [tuple(self.n[l]) for l in range(L)],
            "iters": [self.iters[l] for l in range(L)],
            "ir_outer": [self.ir_outer[l] for l in range(L)],
            "dsolve_iters": [self.dsolve_iters[0], self.dsolve_iters[1]],
            "relres": [self.relres[l] for l in range(L)],
            "ms_level": [self.ms_level[l] for l in range(L)],
            "ms_total": self.ms_total,
            "kernel_ms": {k: self.kernel_ms[i] for i, k in enumerate(K_CLASSES)},
            "kernel_calls": {k: self.kernel_calls[i] for i, k in enumerate(K_CLASSES)},
            "kernel_ms_finest": {k: self.kernel_ms_finest[i] for i, k in enumerate(K_CLASSES)},
            "kernel_calls_finest": {k: self.kernel_calls_finest[i] for i, k in enumerate(K_CLASSES)},
            "history": [self.history[q] for q in range(self.history_len)],
        }


class ExcmgError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().excmg_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_I32P = ctypes.POINTER(ctypes.c_int32)
_D3 = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"the HIP library {LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
                "(or paper_1507_05063_amd/build.py) first")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "excmg_workspace_bytes": ([ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t)], _I),
            "excmg_plan": ([ctypes.POINTER(Problem), _I32P, _I32P], _I),
            "excmg_setup": ([ctypes.POINTER(Problem), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)], _I),
            "excmg_solve": ([_P, _P, _P, _P, _P, ctypes.POINTER(Stats)], _I),
            "excmg_gradient": ([_P, _P, _P, _P, _P], _I),
            "excmg_adjoint": ([_P, _P, _P, _P, _P, ctypes.POINTER(Stats)], _I),
            "excmg_batch_workspace_bytes": ([ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)], _I),
            "excmg_solve_batched": ([ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                     ctypes.POINTER(_P), _P, ctypes.c_size_t, ctypes.POINTER(Stats),
                                     ctypes.POINTER(ctypes.c_double)], _I),
            "excmg_autotune_batched": ([ctypes.POINTER(_P), ctypes.c_int32, _P, ctypes.c_size_t, _I32P], _I),
            "excmg_batch_graph_counts": ([_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], _I),
            "excmg_destroy": ([_P], None),
            "excmg_set_timing": ([_P, ctypes.c_int32], _I),
            "excmg_get_sweep": ([_P, ctypes.c_int32, ctypes.c_int32, _I32P], _I),
            "excmg_set_sweep": ([_P, ctypes.c_int32, ctypes.c_int32, _I32P], _I),
            "excmg_get_batch_shape": ([_P, _I32P], _I),
            "excmg_set_batch_shape": ([_P, _I32P], _I),
            "excmg_solve_noalloc": ([ctypes.POINTER(Problem), _P, _P, _P, _P, _P, ctypes.POINTER(Stats)], _I),
            "excmg_autotune": ([_P, _I32P, _I32P], _I),
            "excmg_bandwidth_probe": ([_P, ctypes.c_size_t, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_double), _I32P],
                                      _I),
            "excmg_strerror": ([_I], ctypes.c_char_p),
            "excmg_op_apply": ([_I32P, _D3, _P, _P, _P], _I),
            "excmg_op_rhs": ([_I32P, _D3, _P, _P, _P, _P], _I),
            "excmg_op_exp_finite": ([_I32P, _P, _P, _P, _P, _P], _I),
            "excmg_op_exp_true": ([_I32P, _P, _P, _P, _P], _I),
            "excmg_op_initial_guess": ([ctypes.c_int32, _I32P, _P, _P, _P, _P, _P], _I),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(code: int, where: str, allow=()):
    if code != OK and code not in allow:
        raise ExcmgError(code, where)
    return code
