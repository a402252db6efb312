"""ctypes wrapper of the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg use this module.  The
GPU library and its Python binding never import it.

Arrays are numpy float64 node arrays of shape (nz+1, ny+1, nx+1) (x fastest), as in synth.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, ERR_ARG, ERR_SHAPE, ERR_NOCONV, ERR_BREAKDOWN, ERR_NOMEM = 0, -1, -2, -4, -5, -7


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP) into liboracle.so next to this file."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    src = os.path.join(_HERE, "oracle.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_POSIX_C_SOURCE=199309L", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-Wno-unknown-pragmas", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None

_D = ctypes.c_double
_I = ctypes.c_int
_P = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        g6 = [_I, _I, _I, _D, _D, _D]
        for name, args in [
            ("orc_apply_L", g6 + [_P, _P]),
            ("orc_apply_R", g6 + [_P, _P]),
            ("orc_apply_M", g6 + [_P, _P]),
            ("orc_rhs", g6 + [_P, _P, _P]),
            ("orc_cg", g6 + [_P, _P, _D, _I, _I, _P, _P, _P]),
            ("orc_direct_solve", g6 + [_P, _P]),
            ("orc_banded_M_apply", g6 + [_P, _P]),
            ("orc_exp_finite", [_I, _I, _I, _P, _P, _P, _P]),
            ("orc_exp_true", [_I, _I, _I, _P, _P, _P]),
            ("orc_gradient", g6 + [_P, _P, _P, _P]),
            ("orc_excmg", [_I, _I, _I, _D, _D, _D, _I, _I, _I, _P, _P, _D, _I, _P, _P, _P, _P, _P, _P, _P]),
            ("orc_adjoint", [_I, _I, _I, _D, _D, _D, _I, _I, _I, _P, _D, _I, _P, _P, _P, _P, _P, _P]),
            ("orc_apply_RT", [_I, _I, _I, _P, _P]),
            ("orc_apply_LIBT", g6 + [_P, _P]),
            ("orc_initial_guess", [_I, _I, _I, _I, _P, _P, _P, _P]),
            ("orc_excmg_variant", [_I, _I, _I, _I, _I, _D, _D, _D, _I, _I, _I, _P, _P, _D, _D, _I, _P, _P, _P, _P,
                                   _P, _P]),
        ]:
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = _I
        L.orc_lagrange4.argtypes = [_I, _D]
        L.orc_lagrange4.restype = _D
        L.orc_lagrange2.argtypes = [_I, _D]
        L.orc_lagrange2.restype = _D
        L.orc_set_threads.argtypes = [_I]
        L.orc_set_threads.restype = None
        L.orc_set_progress.argtypes = [_I]
        L.orc_set_progress.restype = None
        L.orc_get_threads.argtypes = []
        L.orc_get_threads.restype = _I
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where} failed with oracle status {code}")
        self.code = code


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data


def _dims(a):
    nz, ny, nx = (s - 1 for s in a.shape)
    return nx, ny, nz


def _check(code, where, allow=()):
    if code != OK and code not in allow:
        raise OracleError(code, where)
    return code


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int):
    lib().orc_set_threads(int(n))


def set_progress(on: bool):
    """Print a line on stderr after each grid of a cascade."""
    lib().orc_set_progress(int(bool(on)))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def _h(n, box):
    return tuple(float(box[d]) / float(n[d]) for d in range(3))


def apply_L(u, box=(1.0, 1.0, 1.0)):
    u = _c(u)
    n = _dims(u)
    out = np.empty_like(u)
    _check(lib().orc_apply_L(*n, *_h(n, box), _ptr(u), _ptr(out)), "apply_L")
    return out


def apply_R(f, box=(1.0, 1.0, 1.0)):
    f = _c(f)
    n = _dims(f)
    out = np.empty_like(f)
    _check(lib().orc_apply_R(*n, *_h(n, box), _ptr(f), _ptr(out)), "apply_R")
    return out


def apply_M(x, box=(1.0, 1.0, 1.0)):
    x = _c(x)
    n = _dims(x)
    out = np.empty_like(x)
    _check(lib().orc_apply_M(*n, *_h(n, box), _ptr(x), _ptr(out)), "apply_M")
    return out


def banded_M_apply(x, box=(1.0, 1.0, 1.0)):
    x = _c(x)
    n = _dims(x)
    out = np.empty_like(x)
    _check(lib().orc_banded_M_apply(*n, *_h(n, box), _ptr(x), _ptr(out)), "banded_M_apply")
    return out


def rhs(f, g, box=(1.0, 1.0, 1.0)):
    f, g = _c(f), _c(g)
    n = _dims(f)
    b = np.empty_like(f)
    _check(lib().orc_rhs(*n, *_h(n, box), _ptr(f), _ptr(g), _ptr(b)), "rhs")
    return b


def cg(b, u0, tol, box=(1.0, 1.0, 1.0), max_iters=100000, fixed_iters=-1, allow_noconv=False):
    """Returns (u, iters, true_relres, history)."""
    b = _c(b)
    u = _c(u0).copy()
    n = _dims(b)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    hist = np.zeros(max(max_iters, fixed_iters, 0) + 1, dtype=np.float64)
    code = lib().orc_cg(*n, *_h(n, box), _ptr(b), _ptr(u), float(tol), int(max_iters), int(fixed_iters),
                        ctypes.byref(it), ctypes.byref(rr), _ptr(hist))
    _check(code, "cg", allow=(ERR_NOCONV,) if allow_noconv else ())
    return u, it.value, rr.value, hist[: it.value + 1]


def direct_solve(b, g=None, box=(1.0, 1.0, 1.0)):
    b = _c(b)
    n = _dims(b)
    u = np.zeros_like(b) if g is None else _c(g).copy()
    _check(lib().orc_direct_solve(*n, *_h(n, box), _ptr(b), _ptr(u)), "direct_solve")
    return u


def lagrange4(a: int, t: float) -> float:
    return float(lib().orc_lagrange4(int(a), float(t)))


def exp_finite(u2h, u4h, g):
    u2h, u4h, g = _c(u2h), _c(u4h), _c(g)
    n = _dims(g)
    w = np.empty_like(g)
    _check(lib().orc_exp_finite(*n, _ptr(u2h), _ptr(u4h), _ptr(g), _ptr(w)), "exp_finite")
    return w


GUESS_QUARTIC, GUESS_QUADRATIC, GUESS_LINEAR = 0, 1, 2
GUESS_KINDS = {"quartic": GUESS_QUARTIC, "quadratic": GUESS_QUADRATIC, "linear": GUESS_LINEAR}


def lagrange2(a: int, t: float) -> float:
    return float(lib().orc_lagrange2(int(a), float(t)))


def initial_guess(kind, u2h, u4h, g):
    """The initial guess of the given kind ('quartic' = EXP_finite, 'quadratic', 'linear') on g's grid."""
    k = GUESS_KINDS[kind] if isinstance(kind, str) else int(kind)
    u2h, g = _c(u2h), _c(g)
    u4h = None if u4h is None else _c(u4h)
    n = _dims(g)
    w = np.empty_like(g)
    _check(lib().orc_initial_guess(k, *n, _ptr(u2h), _ptr(u4h), _ptr(g), _ptr(w)), "initial_guess")
    return w


STOP_NORMS = {"b": 0, "fg": 1, "fg_coarse": 2}


def excmg_guess(kind, f, g, box, n_coarse, tol, max_iters=100000, fixed_iters=None, stop_norm="b", want_ext=False,
                tol_order=0.0):
    """Algorithm 1 with the initial guess of the given kind on every level from 2 on, and the stopping test's norm
    read as stop_norm says ("b": the eliminated right-hand side; "fg": R f inside and g on the boundary; "fg_coarse":
    "fg" on every level below the finest and "b" on the finest); tol_order
    p > 0 relaxes level l of the finest Lt to tol * 2^(p (Lt - l)) (at most max(tol, 1e-2)).
    Returns dict(u, ut, w, iters, relres): w is the finest level's initial guess, ut EXP_true (want_ext)."""
    k = GUESS_KINDS[kind] if isinstance(kind, str) else int(kind)
    f, g = _c(f), _c(g)
    n = _dims(f)
    nl = levels_for(n, n_coarse)
    u, w = np.empty_like(f), np.empty_like(f)
    iters = np.zeros(nl, dtype=np.int32)
    relres = np.zeros(nl, dtype=np.float64)
    fx = None
    if fixed_iters is not None:
        fx = np.ascontiguousarray(fixed_iters, dtype=np.int32)
        assert fx.size == nl
    ut = np.empty_like(f) if want_ext else None
    code = lib().orc_excmg_variant(k, STOP_NORMS[stop_norm], *n, *(float(v) for v in box),
                                   *(int(v) for v in n_coarse), _ptr(f), _ptr(g), float(tol), float(tol_order),
                                   int(max_iters),
                                   None if fx is None else fx.ctypes.data, _ptr(u), _ptr(ut),
                                   _ptr(w) if nl >= 3 else None, iters.ctypes.data, relres.ctypes.data)
    _check(code, "excmg_guess")
    return dict(u=u, ut=ut, w=w if nl >= 3 else None, iters=iters, relres=relres)


def exp_true(uh, u2h):
    uh, u2h = _c(uh), _c(u2h)
    n = _dims(uh)
    ut = np.empty_like(uh)
    _check(lib().orc_exp_true(*n, _ptr(uh), _ptr(u2h), _ptr(ut)), "exp_true")
    return ut


def gradient(u, box=(1.0, 1.0, 1.0)):
    u = _c(u)
    n = _dims(u)
    ux, uy, uz = np.empty_like(u), np.empty_like(u), np.empty_like(u)
    _check(lib().orc_gradient(*n, *_h(n, box), _ptr(u), _ptr(ux), _ptr(uy), _ptr(uz)), "gradient")
    return ux, uy, uz


def levels_for(n, n_coarse):
    t = 0
    while t < 30:
        if all(int(n_coarse[d]) << t == int(n[d]) for d in range(3)):
            return t + 1
        t += 1
    raise ValueError("finest counts are not n_coarse * 2^L")


def excmg(f, g, box, n_coarse, tol, max_iters=100000, fixed_iters=None, want_ext=False, want_w=False,
          allow_noconv=False):
    """Run Algorithm 1.  Returns dict(u, ut, w, iters, relres, seconds)."""
    f, g = _c(f), _c(g)
    n = _dims(f)
    nl = levels_for(n, n_coarse)
    u = np.empty_like(f)
    ut = np.empty_like(f) if want_ext else None
    w = np.empty_like(f) if want_w else None
    iters = np.zeros(nl, dtype=np.int32)
    relres = np.zeros(nl, dtype=np.float64)
    secs = np.zeros(2, dtype=np.float64)
    fx = None
    if fixed_iters is not None:
        fx = np.ascontiguousarray(fixed_iters, dtype=np.int32)
        assert fx.size == nl
    code = lib().orc_excmg(*n, *(float(v) for v in box), *(int(v) for v in n_coarse), _ptr(f), _ptr(g),
                           float(tol), int(max_iters), None if fx is None else fx.ctypes.data, _ptr(u), _ptr(ut),
                           _ptr(w), iters.ctypes.data, relres.ctypes.data, secs.ctypes.data)
    _check(code, "excmg", allow=(ERR_NOCONV,) if allow_noconv else ())
    return dict(u=u, ut=ut, w=w, iters=iters, relres=relres, seconds=secs, status=code)


def adjoint(G, box, n_coarse, tol, max_iters=100000, fixed_iters=None):
    """Returns dict(dLdf, dLdg, lam, iters, relres)."""
    G = _c(G)
    n = _dims(G)
    nl = levels_for(n, n_coarse)
    dLdf, dLdg, lam = np.empty_like(G), np.empty_like(G), np.empty_like(G)
    iters = np.zeros(nl, dtype=np.int32)
    relres = np.zeros(nl, dtype=np.float64)
    fx = None
    if fixed_iters is not None:
        fx = np.ascontiguousarray(fixed_iters, dtype=np.int32)
    code = lib().orc_adjoint(*n, *(float(v) for v in box), *(int(v) for v in n_coarse), _ptr(G), float(tol),
                             int(max_iters), None if fx is None else fx.ctypes.data, _ptr(dLdf), _ptr(dLdg),
                             _ptr(lam), iters.ctypes.data, relres.ctypes.data)
    _check(code, "adjoint")
    return dict(dLdf=dLdf, dLdg=dLdg, lam=lam, iters=iters, relres=relres)


def apply_RT(lam):
    lam = _c(lam)
    n = _dims(lam)
    out = np.empty_like(lam)
    _check(lib().orc_apply_RT(*n, _ptr(lam), _ptr(out)), "apply_RT")
    return out


def apply_LIBT(lam, box=(1.0, 1.0, 1.0)):
    lam = _c(lam)
    n = _dims(lam)
    out = np.empty_like(lam)
    _check(lib().orc_apply_LIBT(*n, *_h(n, box), _ptr(lam), _ptr(out)), "apply_LIBT")
    return out


def norms(e, box):
    """Discrete L2 (sqrt(hx hy hz sum e^2) over all nodes) and max norm of a node array."""
    n = _dims(e)
    hx, hy, hz = _h(n, box)
    return float(np.sqrt(hx * hy * hz * np.sum(e * e))), float(np.max(np.abs(e)))
