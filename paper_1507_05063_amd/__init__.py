"""MI355X-native EXCMG solver for the 3D Dirichlet Poisson problem with the 19-point fourth-order compact scheme
(Pan, He & Hu, arXiv 1507.05063).

Thin Python binding over the C ABI (include/excmg.h): arguments are marshalled to device pointers of torch CUDA
tensors (float64 node arrays of shape (Nz+1, Ny+1, Nx+1), x fastest) and the current torch stream.  Every step of
the solver runs in the HIP library; nothing here computes.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

from . import _lib
from ._lib import ExcmgError, FP32_IR, FP64, K_CLASSES, LIB_PATH, NO_GRAPHS, WANT_HISTORY, WANT_TIMING

__all__ = ["Solver", "ExcmgError", "FP64", "FP32_IR", "plan", "workspace_bytes", "op_apply", "op_rhs",
           "op_exp_finite", "op_initial_guess", "op_exp_true", "solve_batched", "autotune_batched",
           "batch_workspace_bytes",
           "bandwidth_probe", "PROBE_KINDS", "K_CLASSES", "LIB_PATH"]


def _torch():
    import torch

    return torch


def _problem(n, box, tol, n_coarse=(0, 0, 0), precision=FP64, inner_tol=0.0, max_iters=0, flags=0,
             tol_order=0.0, tol_coarse=0.0):
    p = _lib.Problem()
    for d in range(3):
        p.box[d] = float(box[d])
        p.n[d] = int(n[d])
        p.n_coarse[d] = int(n_coarse[d])
    p.tol = float(tol)
    p.precision = int(precision)
    p.inner_tol = float(inner_tol)
    p.max_iters = int(max_iters)
    p.flags = int(flags)
    p.tol_order = float(tol_order)
    p.tol_coarse = float(tol_coarse)
    return p


def plan(n, n_coarse=(0, 0, 0), box=(1.0, 1.0, 1.0), tol=1e-10):
    """(levels, n_coarse) that the solver will use (host only)."""
    p = _problem(n, box, tol, n_coarse)
    L = ctypes.c_int32(0)
    nc = (ctypes.c_int32 * 3)()
    _lib.check(_lib.lib().excmg_plan(ctypes.byref(p), ctypes.byref(L), nc), "excmg_plan")
    return L.value, tuple(nc)


def workspace_bytes(n, n_coarse=(0, 0, 0), box=(1.0, 1.0, 1.0), tol=1e-10, precision=FP64) -> int:
    p = _problem(n, box, tol, n_coarse, precision)
    b = ctypes.c_size_t(0)
    _lib.check(_lib.lib().excmg_workspace_bytes(ctypes.byref(p), ctypes.byref(b)), "excmg_workspace_bytes")
    return int(b.value)


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_nodes(t, n, name):
    torch = _torch()
    shape = (int(n[2]) + 1, int(n[1]) + 1, int(n[0]) + 1)
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name}: expected a float64 CUDA tensor")
    if tuple(t.shape) != shape:
        raise ValueError(f"{name}: expected shape {shape}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")


class Solver:
    """A problem bound to its device workspace and a stream: ``solve``, ``gradient`` and ``adjoint``."""

    def __init__(self, n: Sequence[int], box=(1.0, 1.0, 1.0), tol: float = 1e-10, n_coarse=(0, 0, 0),
                 precision: int = FP64, inner_tol: float = 0.0, max_iters: int = 0, history: bool = False,
                 timing: bool = False, graphs: bool = True, guess: str = "quartic", stop_norm: str = "b",
                 tol_order: float = 0.0, tol_coarse: float = 0.0, two_pass_cg: bool = False, stream=None):
        """guess: the initial guess of every grid from the third on: "quartic" (EXP_finite, the paper's method),
        "quadratic" (the same extrapolation, tri-quadratic interpolation) or "linear" (CMG: trilinear u_2h).
        stop_norm: the ||f_h|| of the stopping test: "b" (the eliminated right-hand side), "fg" (R f inside, g on
        the boundary) or "fg_coarse" ("fg" on every grid below the finest, "b" on the finest).
        tol_order: p >= 0; grid l of L relaxes to tol * 2^(p (L-1-l)) (at most max(tol, 1e-2)): tol on the finest grid,
        looser on the coarser ones (0: tol everywhere, Algorithm 1).
        tol_coarse: 0, or in (0, 1) with tol_order 0: every grid below the finest relaxes to tol_coarse, the finest
        to tol.
        two_pass_cg: run the two-pass CG as written on every grid (default: the single-reduction form on the
        small grids below the finest, up to 2^18 unknowns, one launch per iteration)."""
        torch = _torch()
        self.n = tuple(int(v) for v in n)
        self.box = tuple(float(v) for v in box)
        self.tol = float(tol)
        self.precision = int(precision)
        if guess not in _lib.GUESS_FLAGS:
            raise ValueError(f"guess must be one of {sorted(_lib.GUESS_FLAGS)}, not {guess!r}")
        self.guess = guess
        if stop_norm not in _lib.STOP_NORM_FLAGS:
            raise ValueError(f"stop_norm must be one of {sorted(_lib.STOP_NORM_FLAGS)}, not {stop_norm!r}")
        self.stop_norm = stop_norm
        flags = (WANT_HISTORY if history else 0) | (WANT_TIMING if timing else 0) | (0 if graphs else NO_GRAPHS)
        flags |= _lib.GUESS_FLAGS[guess] | _lib.STOP_NORM_FLAGS[stop_norm] | (_lib.TWO_PASS_CG if two_pass_cg else 0)
        self.tol_order = float(tol_order)
        self.tol_coarse = float(tol_coarse)
        self._p = _problem(self.n, self.box, tol, n_coarse, precision, inner_tol, max_iters, flags, tol_order,
                           tol_coarse)
        nbytes = ctypes.c_size_t(0)
        _lib.check(_lib.lib().excmg_workspace_bytes(ctypes.byref(self._p), ctypes.byref(nbytes)),
                   "excmg_workspace_bytes")
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._h = ctypes.c_void_p(0)
        _lib.check(_lib.lib().excmg_setup(ctypes.byref(self._p), _ptr(self.workspace), nbytes, _stream_ptr(self.stream),
                                          ctypes.byref(self._h)), "excmg_setup")
        self.levels, self.n_coarse = plan(self.n, n_coarse, self.box, tol)

    @property
    def handle(self):
        return self._h

    def shape(self):
        return (self.n[2] + 1, self.n[1] + 1, self.n[0] + 1)

    def empty(self):
        return _torch().empty(self.shape(), dtype=_torch().float64, device="cuda")

    def solve(self, f, g, u=None, want_ext: bool = False, allow_noconv: bool = False):
        """Returns (u, u_ext or None, stats dict)."""
        _check_nodes(f, self.n, "f")
        _check_nodes(g, self.n, "g")
        u = self.empty() if u is None else u
        _check_nodes(u, self.n, "u")
        ue = self.empty() if want_ext else None
        st = _lib.Stats()
        code = _lib.lib().excmg_solve(self._h, _ptr(f), _ptr(g), _ptr(u), _ptr(ue), ctypes.byref(st))
        _lib.check(code, "excmg_solve", allow=(_lib.ERR_NOCONV,) if allow_noconv else ())
        d = st.to_dict()
        d["status"] = code
        return u, ue, d

    def gradient(self, u, out=None):
        _check_nodes(u, self.n, "u")
        ux, uy, uz = out if out is not None else (self.empty(), self.empty(), self.empty())
        _lib.check(_lib.lib().excmg_gradient(self._h, _ptr(u), _ptr(ux), _ptr(uy), _ptr(uz)), "excmg_gradient")
        return ux, uy, uz

    def adjoint(self, G, want_lambda: bool = False):
        """Returns (dLdf, dLdg, lambda or None, stats dict)."""
        _check_nodes(G, self.n, "G")
        dLdf, dLdg = self.empty(), self.empty()
        lam = self.empty() if want_lambda else None
        st = _lib.Stats()
        code = _lib.lib().excmg_adjoint(self._h, _ptr(G), _ptr(dLdf), _ptr(dLdg), _ptr(lam), ctypes.byref(st))
        _lib.check(code, "excmg_adjoint")
        return dLdf, dLdg, lam, st.to_dict()

    def autotune(self, with_depth: bool = False):
        """Time the CG sweep variants of every relaxed grid and keep the fastest.  Returns, per grid, the z chunk of
        (pass A, pass B) in FP64 and in FP32 (0 where unused); with_depth: also the prefetch depths, as a second
        list of the same form."""
        zc = (ctypes.c_int32 * (4 * self.levels))()
        dp = (ctypes.c_int32 * (4 * self.levels))()
        _lib.check(_lib.lib().excmg_autotune(self._h, zc, dp), "excmg_autotune")
        z = [tuple(zc[4 * l: 4 * l + 4]) for l in range(self.levels)]
        if with_depth:
            return z, [tuple(dp[4 * l: 4 * l + 4]) for l in range(self.levels)]
        return z

    def batch_graph_counts(self):
        """(replays, captures) of the batched-round graphs cached on this solver's handle (batches it leads)."""
        r, c = ctypes.c_int64(0), ctypes.c_int64(0)
        _lib.check(_lib.lib().excmg_batch_graph_counts(self._h, ctypes.byref(r), ctypes.byref(c)),
                   "excmg_batch_graph_counts")
        return r.value, c.value

    SWEEP_KINDS = {"a": 0, "b": 1, "a32": 2, "b32": 3, "a_first": 4, "b_first": 5}

    def get_sweep(self, level: int, kind: str):
        """(z chunk, prefetch depth, non-temporal policy, tile height) of a CG sweep of grid `level` (0 = coarsest);
        kind: "a", "b" (FP64 passes), "a32", "b32" (FP32 refinement), "a_first", "b_first" (a grid's first
        iteration)."""
        sh = (ctypes.c_int32 * 4)()
        _lib.check(_lib.lib().excmg_get_sweep(self._h, int(level), self.SWEEP_KINDS[kind], sh), "excmg_get_sweep")
        return tuple(sh)

    def set_sweep(self, level: int, kind: str, shape):
        """Use shape = (z chunk, prefetch depth, non-temporal policy, tile height) for that sweep from now on (for
        example one saved from get_sweep after autotune)."""
        sh = (ctypes.c_int32 * 4)(*[int(v) for v in shape])
        _lib.check(_lib.lib().excmg_set_sweep(self._h, int(level), self.SWEEP_KINDS[kind], sh), "excmg_set_sweep")

    def get_batch_shape(self):
        """(FP64 tile height, FP32 tile height, FP64 prefetch depth, FP32 prefetch depth) of the batched CG passes of
        the batches this solver leads."""
        sh = (ctypes.c_int32 * 4)()
        _lib.check(_lib.lib().excmg_get_batch_shape(self._h, sh), "excmg_get_batch_shape")
        return tuple(sh)

    def set_batch_shape(self, shape):
        """Set (FP64 tile height, FP32 tile height, FP64 depth, FP32 depth) of the batched CG passes of the batches this
        solver leads (heights 4, 8 or 16; depths 2, 3, 4 or 6)."""
        sh = (ctypes.c_int32 * 4)(*[int(v) for v in shape])
        _lib.check(_lib.lib().excmg_set_batch_shape(self._h, sh), "excmg_set_batch_shape")

    def set_timing(self, on: bool):
        """Kernel timing (stats kernel_ms, kernel_calls) on or off for later calls."""
        _lib.check(_lib.lib().excmg_set_timing(self._h, 1 if on else 0), "excmg_set_timing")

    def close(self):
        if self._h:
            _lib.lib().excmg_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_workspace_bytes(count: int) -> int:
    b = ctypes.c_size_t(0)
    _lib.check(_lib.lib().excmg_batch_workspace_bytes(int(count), ctypes.byref(b)), "excmg_batch_workspace_bytes")
    return int(b.value)


def autotune_batched(solvers, workspace=None):
    """Tune the z chunks of the batched CG sweeps for this batch of solvers (kept in the solvers' handles for later
    solve_batched calls).  Returns {grid t counted from the finest: (FP64 chunk, FP32 chunk)}, 0 where unused."""
    torch = _torch()
    count = len(solvers)
    if count == 0:
        raise ValueError("no solvers")
    nbytes = batch_workspace_bytes(count)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    H = (ctypes.c_void_p * count)(*[s.handle.value for s in solvers])
    zc = (ctypes.c_int32 * (2 * _lib.MAX_LEVELS))()
    _lib.check(_lib.lib().excmg_autotune_batched(H, count, _ptr(workspace), ctypes.c_size_t(workspace.numel()), zc),
               "excmg_autotune_batched")
    return {t: (zc[2 * t], zc[2 * t + 1]) for t in range(_lib.MAX_LEVELS) if zc[2 * t] or zc[2 * t + 1]}


def solve_batched(solvers, fs, gs, us=None, workspace=None, allow_noconv: bool = False):
    """Solve many problems (each bound to its own Solver) in one batched call on the stream of solvers[0].
    Returns (us, stats list, ms_per_problem list): ms_per_problem[b] is the device time from the start of the batch
    until problem b's finest grid converged."""
    torch = _torch()
    count = len(solvers)
    if count == 0 or len(fs) != count or len(gs) != count:
        raise ValueError("solvers, fs and gs must have the same nonzero length")
    for s, f, g in zip(solvers, fs, gs):
        _check_nodes(f, s.n, "f")
        _check_nodes(g, s.n, "g")
    us = [s.empty() for s in solvers] if us is None else us
    for s, u in zip(solvers, us):
        _check_nodes(u, s.n, "u")
    nbytes = batch_workspace_bytes(count)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    H = (ctypes.c_void_p * count)(*[s.handle.value for s in solvers])
    F = (ctypes.c_void_p * count)(*[f.data_ptr() for f in fs])
    G = (ctypes.c_void_p * count)(*[g.data_ptr() for g in gs])
    U = (ctypes.c_void_p * count)(*[u.data_ptr() for u in us])
    st = (_lib.Stats * count)()
    ms = (ctypes.c_double * count)()
    code = _lib.lib().excmg_solve_batched(H, count, F, G, U, _ptr(workspace), ctypes.c_size_t(workspace.numel()), st,
                                          ms)
    _lib.check(code, "excmg_solve_batched", allow=(_lib.ERR_NOCONV,) if allow_noconv else ())
    return us, [st[b].to_dict() for b in range(count)], [ms[b] for b in range(count)]


PROBE_KINDS = ("copy", "read", "copy_nt", "read_nt", "mix_nt", "mix", "write", "write_nt")


def bandwidth_probe(nbytes: int = 2 << 30, reps: int = 5, with_shapes: bool = False):
    """Achievable HBM bandwidth in this process: GB/s of streaming kernels over nbytes, by kind (copy, read, pass B's
    mix of three arrays read and two written, write; each with ordinary and with non-temporal accesses), the best
    over a sweep of launch shapes.  with_shapes: also, per kind, the fastest shape (workgroups per CU, 16-byte
    accesses in flight per lane, contiguous ranges per workgroup)."""
    torch = _torch()
    buf = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    rates = (ctypes.c_double * len(PROBE_KINDS))()
    shapes = (ctypes.c_int32 * (3 * len(PROBE_KINDS)))()
    _lib.check(_lib.lib().excmg_bandwidth_probe(_ptr(buf), int(nbytes), int(reps), _stream_ptr(), rates, shapes),
               "excmg_bandwidth_probe")
    del buf
    out = {k: rates[i] for i, k in enumerate(PROBE_KINDS)}
    if with_shapes:
        return out, {k: {"wg_per_cu": shapes[3 * i], "lanes_in_flight": shapes[3 * i + 1],
                         "contiguous": bool(shapes[3 * i + 2])} for i, k in enumerate(PROBE_KINDS)}
    return out


def _n3(n):
    return (ctypes.c_int32 * 3)(*[int(v) for v in n])


def _box3(box):
    return (ctypes.c_double * 3)(*[float(v) for v in box])


def op_apply(x, n, box=(1.0, 1.0, 1.0)):
    """y = M x, M = -A_h on the interior (boundary of x read as 0)."""
    _check_nodes(x, n, "x")
    y = _torch().empty_like(x)
    _lib.check(_lib.lib().excmg_op_apply(_n3(n), _box3(box), _ptr(x), _ptr(y), _stream_ptr()), "excmg_op_apply")
    return y


def op_rhs(f, g, n, box=(1.0, 1.0, 1.0)):
    _check_nodes(f, n, "f")
    b = _torch().empty_like(f)
    _lib.check(_lib.lib().excmg_op_rhs(_n3(n), _box3(box), _ptr(f), _ptr(g), _ptr(b), _stream_ptr()), "excmg_op_rhs")
    return b


def op_exp_finite(u2h, u4h, g, n):
    _check_nodes(g, n, "g")
    w = _torch().empty_like(g)
    _lib.check(_lib.lib().excmg_op_exp_finite(_n3(n), _ptr(u2h), _ptr(u4h), _ptr(g), _ptr(w), _stream_ptr()),
               "excmg_op_exp_finite")
    return w


def op_initial_guess(kind: str, u2h, u4h, g, n):
    """The initial guess of a kind ("quartic" = op_exp_finite, "quadratic", "linear"; u4h unused, may be None for
    "linear") on the grid n, with g on the boundary."""
    _check_nodes(g, n, "g")
    w = _torch().empty_like(g)
    _lib.check(_lib.lib().excmg_op_initial_guess(_lib.GUESS_KINDS[kind], _n3(n), _ptr(u2h),
                                                 None if u4h is None else _ptr(u4h), _ptr(g), _ptr(w), _stream_ptr()),
               "excmg_op_initial_guess")
    return w


def op_exp_true(uh, u2h, n):
    _check_nodes(uh, n, "uh")
    ut = _torch().empty_like(uh)
    _lib.check(_lib.lib().excmg_op_exp_true(_n3(n), _ptr(uh), _ptr(u2h), _ptr(ut), _stream_ptr()), "excmg_op_exp_true")
    return ut
