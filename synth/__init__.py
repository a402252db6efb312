"""Seeded synthetic inputs for the 3D Dirichlet Poisson problem u_xx + u_yy + u_zz = f, u = g on the boundary.

This module only evaluates closed-form functions on node grids and draws seeded parameters.  It holds none of the
solver's arithmetic (no difference operator, no extrapolation, no interpolation), so both the CPU oracle's tests and
the GPU path's tests and benchmark can take their inputs from here.

Grids follow the paper's Section 2: box [0,Lx]x[0,Ly]x[0,Lz], Nx, Ny, Nz uniform intervals, nodes
(i*hx, j*hy, k*hz), 0 <= i <= Nx, ...  A node array has numpy shape (Nz+1, Ny+1, Nx+1) (x fastest), float64.

Problems:
  * ``example(1..6)``: the six test problems of the paper's Section 5 (Examples 1-6, in printed order).
    Example 5's forcing term is not printed in the paper; it is derived here as Laplacian(x^3 y^3 z^3 / r^3).
  * ``smooth(seed, box)``: u = sum_{k=1..3} a_k sin(p_k pi x/Lx) sin(q_k pi y/Ly) sin(r_k pi z/Lz)
    + exp(x/Lx + y/Ly + z/Lz)/10 with a_k ~ U(0.5,1.5) and p,q,r in {1,2,3}, drawn from numpy's default_rng(seed)
    in the order: a (3 draws), then the 3x3 integer matrix of (p_k, q_k, r_k) rows.
  * ``r25()``: u = r^2.5 with r = |x - (0.5,0.5,0.5)| (lower regularity than any of the paper's examples).
  * ``batch(seed, count)``: per problem draws N (3 values from {32,64,96,128,192}), box edges ~U(0.5,2)
    (3 draws), then the smooth-field parameters as in ``smooth``.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Sequence

import numpy as np

Array = np.ndarray


@dataclasses.dataclass
class Problem:
    """Closed-form exact solution u, its Laplacian f and its gradient on a box."""

    name: str
    box: tuple
    u: Callable[[Array, Array, Array], Array]
    f: Callable[[Array, Array, Array], Array]
    grad: Callable[[Array, Array, Array], tuple]


def mesh(n: Sequence[int], box: Sequence[float]):
    """Broadcastable node coordinates (z, y, x order of axes) for n = (Nx, Ny, Nz) intervals."""
    nx, ny, nz = (int(v) for v in n)
    lx, ly, lz = (float(v) for v in box)
    x = (np.arange(nx + 1, dtype=np.float64) * (lx / nx))[None, None, :]
    y = (np.arange(ny + 1, dtype=np.float64) * (ly / ny))[None, :, None]
    z = (np.arange(nz + 1, dtype=np.float64) * (lz / nz))[:, None, None]
    return x, y, z


def boundary_mask(n: Sequence[int]) -> Array:
    """Boolean node array, True on the boundary of the box."""
    nx, ny, nz = (int(v) for v in n)
    m = np.zeros((nz + 1, ny + 1, nx + 1), dtype=bool)
    m[0, :, :] = m[-1, :, :] = True
    m[:, 0, :] = m[:, -1, :] = True
    m[:, :, 0] = m[:, :, -1] = True
    return m


def _full(v, shape):
    return np.broadcast_to(v, shape).astype(np.float64, copy=True)


def sample(p: Problem, n: Sequence[int]):
    """Return (f, g, u_exact) node arrays.

    f is sampled on every node (the compact right-hand side reads f on boundary nodes too).  g holds u on the
    boundary nodes and zero inside, so a solver that reads g inside the box is caught by the tests.
    """
    x, y, z = mesh(n, p.box)
    shape = (int(n[2]) + 1, int(n[1]) + 1, int(n[0]) + 1)
    f = _full(p.f(x, y, z), shape)
    u = _full(p.u(x, y, z), shape)
    g = np.where(boundary_mask(n), u, 0.0)
    return f, g, u


def exact_gradient(p: Problem, n: Sequence[int]):
    x, y, z = mesh(n, p.box)
    shape = (int(n[2]) + 1, int(n[1]) + 1, int(n[0]) + 1)
    gx, gy, gz = p.grad(x, y, z)
    return _full(gx, shape), _full(gy, shape), _full(gz, shape)


# ----------------------------------------------------------------------------------------------------------------
# Seeded smooth field (the workloads' synthetic stand-in for the paper's analytic examples)
# ----------------------------------------------------------------------------------------------------------------

def _smooth_from(a: Array, pqr: Array, box) -> Problem:
    lx, ly, lz = (float(v) for v in box)
    a = np.asarray(a, dtype=np.float64)
    pqr = np.asarray(pqr, dtype=np.int64)
    pi = np.pi

    def modes(x, y, z):
        out = []
        for k in range(3):
            p, q, r = (int(v) for v in pqr[k])
            kx, ky, kz = p * pi / lx, q * pi / ly, r * pi / lz
            out.append((a[k], kx, ky, kz))
        return out

    def u(x, y, z):
        s = np.exp(x / lx + y / ly + z / lz) / 10.0
        for ak, kx, ky, kz in modes(x, y, z):
            s = s + ak * np.sin(kx * x) * np.sin(ky * y) * np.sin(kz * z)
        return s

    def f(x, y, z):
        s = (1.0 / lx ** 2 + 1.0 / ly ** 2 + 1.0 / lz ** 2) * np.exp(x / lx + y / ly + z / lz) / 10.0
        for ak, kx, ky, kz in modes(x, y, z):
            s = s - ak * (kx * kx + ky * ky + kz * kz) * np.sin(kx * x) * np.sin(ky * y) * np.sin(kz * z)
        return s

    def grad(x, y, z):
        e = np.exp(x / lx + y / ly + z / lz) / 10.0
        gx, gy, gz = e / lx, e / ly, e / lz
        for ak, kx, ky, kz in modes(x, y, z):
            sx, sy, sz = np.sin(kx * x), np.sin(ky * y), np.sin(kz * z)
            cx, cy, cz = np.cos(kx * x), np.cos(ky * y), np.cos(kz * z)
            gx = gx + ak * kx * cx * sy * sz
            gy = gy + ak * ky * sx * cy * sz
            gz = gz + ak * kz * sx * sy * cz
        return gx, gy, gz

    return Problem("smooth", (lx, ly, lz), u, f, grad)


def smooth_params(seed: int):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 1.5, 3)
    pqr = rng.integers(1, 4, (3, 3))
    return a, pqr


def smooth(seed: int = 0, box=(1.0, 1.0, 1.0)) -> Problem:
    a, pqr = smooth_params(seed)
    p = _smooth_from(a, pqr, box)
    p.name = f"smooth(seed={seed})"
    return p


def batch(seed: int = 4, count: int = 96):
    """List of (n, Problem) for the batched workload: uneven cell counts and box edges per problem."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = tuple(int(v) for v in rng.choice([32, 64, 96, 128, 192], 3))
        box = tuple(float(v) for v in rng.uniform(0.5, 2.0, 3))
        a = rng.uniform(0.5, 1.5, 3)
        pqr = rng.integers(1, 4, (3, 3))
        p = _smooth_from(a, pqr, box)
        p.name = f"batch(seed={seed})"
        out.append((n, p))
    return out


def r25() -> Problem:
    c = 0.5

    def rr(x, y, z):
        return np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)

    def u(x, y, z):
        return rr(x, y, z) ** 2.5

    def f(x, y, z):
        # Laplacian of r^m in 3D is m(m+1) r^(m-2); m = 5/2.
        return 8.75 * np.sqrt(rr(x, y, z))

    def grad(x, y, z):
        s = 2.5 * np.sqrt(rr(x, y, z))
        return s * (x - c), s * (y - c), s * (z - c)

    return Problem("r^2.5", (1.0, 1.0, 1.0), u, f, grad)


def direction(seed: int, n: Sequence[int]):
    """Seeded unit direction (d_f on every node, d_g on boundary nodes), jointly normalised to 2-norm 1."""
    rng = np.random.default_rng(seed)
    shape = (int(n[2]) + 1, int(n[1]) + 1, int(n[0]) + 1)
    df = rng.standard_normal(shape)
    dg = np.where(boundary_mask(n), rng.standard_normal(shape), 0.0)
    s = np.sqrt(np.sum(df * df) + np.sum(dg * dg))
    return df / s, dg / s


# ----------------------------------------------------------------------------------------------------------------
# The paper's six examples (Section 5)
# ----------------------------------------------------------------------------------------------------------------

def _ex1():
    def u(x, y, z):
        return np.exp(z) * np.sin(x * y)

    def f(x, y, z):
        return np.exp(z) * np.sin(x * y) * (1.0 - x * x - y * y)

    def grad(x, y, z):
        e = np.exp(z)
        return e * y * np.cos(x * y), e * x * np.cos(x * y), e * np.sin(x * y)

    return Problem("ex1", (1.0, 1.0, 1.0), u, f, grad)


def _ex2():
    s2 = np.sqrt(2.0)

    def u(x, y, z):
        return np.exp(x + y) * np.sin(s2 * z)

    def f(x, y, z):
        return 0.0 * (x + y + z)

    def grad(x, y, z):
        e = np.exp(x + y)
        return e * np.sin(s2 * z), e * np.sin(s2 * z), s2 * e * np.cos(s2 * z)

    return Problem("ex2", (1.0, 1.0, 1.0), u, f, grad)


def _ex3():
    def s(x, y, z):
        return (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2

    def u(x, y, z):
        return np.exp(-3.0 * s(x, y, z))

    def f(x, y, z):
        return np.exp(-3.0 * s(x, y, z)) * (36.0 * s(x, y, z) - 18.0)

    def grad(x, y, z):
        v = np.exp(-3.0 * s(x, y, z))
        return -6.0 * (x - 0.5) * v, -6.0 * (y - 0.5) * v, -6.0 * (z - 0.5) * v

    return Problem("ex3", (1.0, 1.0, 1.0), u, f, grad)


def _ex4():
    pi = np.pi

    def u(x, y, z):
        return np.sin(2 * pi * x) * np.sin(pi * y) * np.sin(0.5 * pi * z)

    def f(x, y, z):
        return -5.25 * pi * pi * u(x, y, z)

    def grad(x, y, z):
        sx, sy, sz = np.sin(2 * pi * x), np.sin(pi * y), np.sin(0.5 * pi * z)
        cx, cy, cz = np.cos(2 * pi * x), np.cos(pi * y), np.cos(0.5 * pi * z)
        return 2 * pi * cx * sy * sz, pi * sx * cy * sz, 0.5 * pi * sx * sy * cz

    return Problem("ex4", (1.0, 1.0, 1.0), u, f, grad)


def _safe_r(x, y, z):
    r = np.sqrt(x * x + y * y + z * z)
    return np.where(r > 0.0, r, 1.0), r > 0.0


def _ex5():
    # u = P r^-3 with P = x^3 y^3 z^3.  Laplacian(P r^m) = r^m Lap(P) + 2m r^(m-2) (x . grad P) + m(m+1) r^(m-2) P,
    # Lap(P) = 6xyz(x^2y^2 + y^2z^2 + z^2x^2), x . grad P = 9P, m = -3:
    # f = 6xyz(x^2y^2 + y^2z^2 + z^2x^2)/r^3 - 48 P/r^5.  The value at the origin (never read) is set to 0.
    def u(x, y, z):
        r, ok = _safe_r(x, y, z)
        return np.where(ok, (x * y * z) ** 3 / r ** 3, 0.0)

    def f(x, y, z):
        r, ok = _safe_r(x, y, z)
        p = (x * y * z) ** 3
        s = x * x * y * y + y * y * z * z + z * z * x * x
        return np.where(ok, 6.0 * x * y * z * s / r ** 3 - 48.0 * p / r ** 5, 0.0)

    def grad(x, y, z):
        r, ok = _safe_r(x, y, z)
        p = (x * y * z) ** 3
        gx = 3 * x * x * (y * z) ** 3 / r ** 3 - 3 * p * x / r ** 5
        gy = 3 * y * y * (x * z) ** 3 / r ** 3 - 3 * p * y / r ** 5
        gz = 3 * z * z * (x * y) ** 3 / r ** 3 - 3 * p * z / r ** 5
        return np.where(ok, gx, 0.0), np.where(ok, gy, 0.0), np.where(ok, gz, 0.0)

    return Problem("ex5", (1.0, 1.0, 1.0), u, f, grad)


def _ex6():
    # u = xyz r, f = 8xyz/r (printed in the paper).
    def u(x, y, z):
        return x * y * z * np.sqrt(x * x + y * y + z * z)

    def f(x, y, z):
        r, ok = _safe_r(x, y, z)
        return np.where(ok, 8.0 * x * y * z / r, 0.0)

    def grad(x, y, z):
        r, ok = _safe_r(x, y, z)
        p = x * y * z
        gx = y * z * r + p * x / r
        gy = x * z * r + p * y / r
        gz = x * y * r + p * z / r
        return np.where(ok, gx, 0.0), np.where(ok, gy, 0.0), np.where(ok, gz, 0.0)

    return Problem("ex6", (1.0, 1.0, 1.0), u, f, grad)


_EXAMPLES = {1: _ex1, 2: _ex2, 3: _ex3, 4: _ex4, 5: _ex5, 6: _ex6}


def example(k: int) -> Problem:
    """Example k (1..6) in the paper's printed numbering."""
    return _EXAMPLES[int(k)]()


def polynomial(coeffs: dict, box=(1.0, 1.0, 1.0)) -> Problem:
    """u = sum c * x^a y^b z^c for {(a,b,c): c}; f and grad by exact differentiation of monomials."""
    items = [(tuple(int(e) for e in k), float(v)) for k, v in coeffs.items()]

    def mono(x, e):
        return x ** e if e > 0 else 1.0 + 0.0 * x

    def u(x, y, z):
        s = 0.0 * (x + y + z)
        for (a, b, c), v in items:
            s = s + v * mono(x, a) * mono(y, b) * mono(z, c)
        return s

    def d2(x, e):
        return e * (e - 1) * x ** (e - 2) if e >= 2 else 0.0 * x

    def d1(x, e):
        return e * x ** (e - 1) if e >= 1 else 0.0 * x

    def f(x, y, z):
        s = 0.0 * (x + y + z)
        for (a, b, c), v in items:
            s = s + v * (d2(x, a) * mono(y, b) * mono(z, c) + mono(x, a) * d2(y, b) * mono(z, c)
                         + mono(x, a) * mono(y, b) * d2(z, c))
        return s

    def grad(x, y, z):
        gx = gy = gz = 0.0 * (x + y + z)
        for (a, b, c), v in items:
            gx = gx + v * d1(x, a) * mono(y, b) * mono(z, c)
            gy = gy + v * mono(x, a) * d1(y, b) * mono(z, c)
            gz = gz + v * mono(x, a) * mono(y, b) * d1(z, c)
        return gx, gy, gz

    return Problem("poly", tuple(float(v) for v in box), u, f, grad)
