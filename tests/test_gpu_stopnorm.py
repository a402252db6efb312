"""The second reading of the stopping test's norm (Algorithm 1: ||A_h u_h - f_h|| <= eps ||f_h||, with f_h the vector
of the discrete equations before the Dirichlet values are eliminated: R f at the interior nodes, g at the boundary
nodes), EXCMG_STOP_F_G: parity of the HIP path with the oracle, the stopping test itself on the finest grid in both
precisions, and the adjoint, which keeps the default test.

Tolerances as in test_gpu_parity.py: whole solves relative L2 <= 1e-12 after matching the per-grid iteration counts
(free-running counts within one).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ex():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_05063_amd as m

    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().to("cpu").numpy()


def rel2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def fg_norm(orc, f, g, box):
    """||f_h|| of the second reading: R f over the interior nodes, g over the boundary nodes."""
    rf = orc.apply_R(f, box)[1:-1, 1:-1, 1:-1]
    bnd = np.ones(g.shape, dtype=bool)
    bnd[1:-1, 1:-1, 1:-1] = False
    return float(np.sqrt(np.sum(rf * rf) + np.sum(g[bnd] ** 2)))


def true_residual(ex, u, f, g, n, box):
    """||b - M u|| over the interior (M = -A_h on the interior, b the eliminated right-hand side)."""
    b = ex.op_rhs(f, g, n, box)
    ui = u.clone()
    ui[0, :, :] = 0
    ui[-1, :, :] = 0
    ui[:, 0, :] = 0
    ui[:, -1, :] = 0
    ui[:, :, 0] = 0
    ui[:, :, -1] = 0
    r = (b - ex.op_apply(ui, n, box))[1:-1, 1:-1, 1:-1]
    return float(torch.linalg.vector_norm(r))


@pytest.mark.parametrize("case", ["ex3-64", "ex2-128", "ex4-aniso", "ex6-ragged"])
def test_fg_below_finest_solve_parity(ex, orc, case):
    """The third reading (EXCMG_STOP_F_G_BELOW_FINEST: (R f, g) below the finest grid, b on it) against the oracle's
    stop_norm "fg_coarse" at matched iteration counts; the grids below the finest iterate as under the second
    reading, and the finest stops on the default test."""
    e, n, nc, tol = {
        "ex3-64": (3, (64, 64, 64), (4, 4, 4), 1e-11),
        "ex2-128": (2, (128, 128, 128), (4, 4, 4), 1e-14),
        "ex4-aniso": (4, (128, 64, 32), (8, 4, 2), 1e-9),
        "ex6-ragged": (6, (80, 48, 48), (10, 6, 6), 1e-13),
    }[case]
    p = synth.example(e)
    f, g, _ = synth.sample(p, n)
    s = ex.Solver(n, p.box, tol, n_coarse=nc, stop_norm="fg_coarse")
    ug, _, st = s.solve(dev(f), dev(g))
    ug = host(ug)
    free = orc.excmg_guess("quartic", f, g, p.box, s.n_coarse, tol, stop_norm="fg_coarse")
    gi = np.array(st["iters"], dtype=np.int32)
    assert np.all(np.abs(gi - free["iters"]) <= 1), (gi, free["iters"])
    ref = orc.excmg_guess("quartic", f, g, p.box, s.n_coarse, tol, fixed_iters=gi, stop_norm="fg_coarse")
    assert rel2(ug, ref["u"]) <= 1e-12
    fg = orc.excmg_guess("quartic", f, g, p.box, s.n_coarse, tol, stop_norm="fg")
    assert np.all(np.abs(gi[:-1] - fg["iters"][:-1]) <= 1), (gi, fg["iters"])
    assert st["relres"][-1] <= tol  # the default test on the finest grid


@pytest.mark.parametrize("case", ["ex1-32", "ex1-64", "ex4-aniso", "ex5-ragged"])
def test_fg_solve_parity(ex, orc, case):
    e, n, nc, tol = {
        "ex1-32": (1, (32, 32, 32), (4, 4, 4), 1e-14),
        "ex1-64": (1, (64, 64, 64), (4, 4, 4), 1e-14),
        "ex4-aniso": (4, (128, 64, 32), (8, 4, 2), 1e-9),
        "ex5-ragged": (5, (80, 48, 48), (10, 6, 6), 1e-12),
    }[case]
    p = synth.example(e)
    f, g, _ = synth.sample(p, n)
    s = ex.Solver(n, p.box, tol, n_coarse=nc, stop_norm="fg")
    ug, _, st = s.solve(dev(f), dev(g))
    ug = host(ug)
    free = orc.excmg_guess("quartic", f, g, p.box, s.n_coarse, tol, stop_norm="fg")
    gi = np.array(st["iters"], dtype=np.int32)
    assert np.all(np.abs(gi - free["iters"]) <= 1), (gi, free["iters"])
    ref = orc.excmg_guess("quartic", f, g, p.box, s.n_coarse, tol, fixed_iters=gi, stop_norm="fg")
    assert rel2(ug, ref["u"]) <= 1e-12
    # the second reading asks for more iterations than the first on the finest grid
    sb = ex.Solver(n, p.box, tol, n_coarse=nc)
    _, _, stb = sb.solve(dev(f), dev(g))
    assert st["iters"][-1] >= stb["iters"][-1], (st["iters"], stb["iters"])


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_fg_stopping_test_holds(ex, orc, precision):
    """Example 1 at 128^3 (2.1M interior unknowns: the mixed path refines in FP32 there), eps 1e-9: the finest grid's
    true residual meets eps ||f_h|| of the second reading.  (At much smaller eps the target falls below the rounding
    floor of the true residual b - M u, where |b| carries the h^-2 boundary couplings: the FP64 CG, which tests its
    recursive residual, still stops, the refinement, which tests the true one, cannot.)"""
    p = synth.example(1)
    n = (128, 128, 128)
    tol = 1e-9
    f, g, _ = synth.sample(p, n)
    prec = ex.FP64 if precision == "fp64" else ex.FP32_IR
    s = ex.Solver(n, p.box, tol, precision=prec, stop_norm="fg")
    fd, gd = dev(f), dev(g)
    u, _, st = s.solve(fd, gd)
    fgn = fg_norm(orc, f, g, p.box)
    rn = true_residual(ex, u, fd, gd, n, p.box)
    assert rn <= 1.5 * tol * fgn, (rn, tol * fgn)
    assert st["relres"][-1] <= tol
    if precision == "fp32_ir":
        assert st["ir_outer"][-1] >= 1


def test_fg_matches_fp64_in_mixed_precision(ex):
    p = synth.example(1)
    n = (128, 128, 128)
    f, g, _ = synth.sample(p, n)
    fd, gd = dev(f), dev(g)
    u64, _, _ = ex.Solver(n, p.box, 1e-9, stop_norm="fg").solve(fd, gd)
    u32, _, _ = ex.Solver(n, p.box, 1e-9, precision=ex.FP32_IR, stop_norm="fg").solve(fd, gd)
    d = float(torch.linalg.vector_norm(u32 - u64) / torch.linalg.vector_norm(u64))
    assert d <= 1e-8, d


def test_adjoint_keeps_the_default_test(ex):
    """The adjoint's data have zero Dirichlet values and no R: the flag leaves it alone, also right after a solve
    that set the boundary part of the norm."""
    p = synth.example(2)
    n = (48, 32, 64)
    nc = (6, 4, 8)
    f, g, _ = synth.sample(p, n)
    G = np.random.default_rng(5).standard_normal((n[2] + 1, n[1] + 1, n[0] + 1))
    sf = ex.Solver(n, p.box, 1e-12, n_coarse=nc, stop_norm="fg")
    sb = ex.Solver(n, p.box, 1e-12, n_coarse=nc)
    sf.solve(dev(f), dev(g))
    a = sf.adjoint(dev(G), want_lambda=True)
    b = sb.adjoint(dev(G), want_lambda=True)
    for x, y in zip(a[:3], b[:3]):
        assert torch.equal(x, y)
    assert a[3]["iters"] == b[3]["iters"]


def test_fg_repeat_is_bitwise(ex):
    p = synth.example(3)
    n = (64, 32, 48)
    f, g, _ = synth.sample(p, n)
    s = ex.Solver(n, p.box, 1e-11, n_coarse=(8, 4, 6), stop_norm="fg")
    u1, _, st1 = s.solve(dev(f), dev(g))
    u1 = u1.clone()
    u2, _, st2 = s.solve(dev(f), dev(g))
    assert torch.equal(u1, u2)
    assert st1["iters"] == st2["iters"]


def test_batched_solves_take_only_the_default_test(ex):
    p = synth.smooth(0)
    n = (32, 32, 32)
    f, g, _ = synth.sample(p, n)
    s = ex.Solver(n, p.box, 1e-10, stop_norm="fg")
    with pytest.raises(ex.ExcmgError):
        ex.solve_batched([s], [dev(f)], [dev(g)])


def test_bad_stop_norm_name(ex):
    with pytest.raises(ValueError):
        ex.Solver((16, 16, 16), stop_norm="f")


# ---------------------------------------------------------------------------------------------------------------
# level-dependent tolerance (tol_order): grid l of L relaxes to tol * 2^(p (L-1-l)), at most max(tol, 1e-2)
# ---------------------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["ex1-64-fg-p6", "ex4-aniso-b-p7.5", "ex5-ragged-fg-p3"])
def test_schedule_solve_parity(ex, orc, case):
    e, n, nc, tol, sn, po = {
        "ex1-64-fg-p6": (1, (64, 64, 64), (4, 4, 4), 1e-14, "fg", 6.0),
        "ex4-aniso-b-p7.5": (4, (128, 64, 32), (8, 4, 2), 1e-12, "b", 7.5),
        "ex5-ragged-fg-p3": (5, (80, 48, 48), (10, 6, 6), 1e-12, "fg", 3.0),
    }[case]
    p = synth.example(e)
    f, g, _ = synth.sample(p, n)
    s = ex.Solver(n, p.box, tol, n_coarse=nc, stop_norm=sn, tol_order=po)
    ug, _, st = s.solve(dev(f), dev(g))
    ug = host(ug)
    free = orc.excmg_guess("quartic", f, g, p.box, s.n_coarse, tol, stop_norm=sn, tol_order=po)
    gi = np.array(st["iters"], dtype=np.int32)
    assert np.all(np.abs(gi - free["iters"]) <= 1), (gi, free["iters"])
    ref = orc.excmg_guess("quartic", f, g, p.box, s.n_coarse, tol, fixed_iters=gi, stop_norm=sn, tol_order=po)
    assert rel2(ug, ref["u"]) <= 1e-12
    L = st["levels"]
    for l in range(2, L):
        if sn == "b":  # the reported relative residual is against the norm of the test
            assert st["relres"][l] <= min(tol * 2.0 ** (po * (L - 1 - l)), max(tol, 1e-2))


def test_schedule_in_mixed_precision(ex):
    """The refinement's outer test and its inner solves take the level's own tolerance."""
    p = synth.example(3)
    n = (128, 128, 128)
    f, g, _ = synth.sample(p, n)
    s = ex.Solver(n, p.box, 1e-9, precision=ex.FP32_IR, tol_order=4.0)
    _, _, st = s.solve(dev(f), dev(g))
    L = st["levels"]
    for l in range(2, L):
        assert st["relres"][l] <= min(1e-9 * 2.0 ** (4.0 * (L - 1 - l)), 1e-2)
    assert st["relres"][L - 2] > 1e-9  # the grid below the finest stopped at its looser tolerance


def _ext_l2(ex, p, n, tol, stop_norm="b", tol_order=0.0):
    f, g, u = synth.sample(p, n)
    s = ex.Solver(n, p.box, tol, stop_norm=stop_norm, tol_order=tol_order)
    _, ue, st = s.solve(dev(f), dev(g), want_ext=True)
    d = ue - dev(u)
    return float(torch.sqrt(torch.mean(d * d))), st["iters"]


def test_extrapolated_solution_keeps_sixth_order(ex):
    """Example 3 (the Gaussian, the paper's eps 1e-11): u~_h stops converging from 64^3 on with the uniform tolerance
    under the default norm (Section 5.1's remark); with eps 1e-15 under the (R f, g) norm it keeps sixth order to
    256^3, with the level schedule p = 6 as well (same finest-grid accuracy, fewer iterations on every coarser grid)."""
    p = synth.example(3)
    e = {}
    for key, tol, sn, po in (("paper", 1e-11, "b", 0.0), ("fg", 1e-15, "fg", 0.0), ("fg6", 1e-15, "fg", 6.0)):
        for N in (128, 256):
            e[key, N] = _ext_l2(ex, p, (N, N, N), tol, sn, po)
    order = lambda k: float(np.log2(e[k, 128][0] / e[k, 256][0]))
    assert order("paper") < 0.5, e
    assert order("fg") > 5.8, e
    assert order("fg6") > 5.8, e
    assert abs(e["fg6", 256][0] - e["fg", 256][0]) <= 0.02 * e["fg", 256][0]
    it_u, it_s = e["fg", 256][1], e["fg6", 256][1]
    assert all(a < b for a, b in zip(it_s[2:-1], it_u[2:-1])), (it_u, it_s)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_schedule_graphs_match_direct_launches(ex, precision):
    """The graphs of CG iteration batches (every grid below the finest) are captured with their grid's own tolerance:
    replaying them gives what direct launches give, bit for bit, over repeated solves."""
    p = synth.example(5)
    n = (128, 128, 128)
    f, g, _ = synth.sample(p, n)
    fd, gd = dev(f), dev(g)
    prec = ex.FP64 if precision == "fp64" else ex.FP32_IR
    kw = dict(n_coarse=(4, 4, 4), precision=prec, stop_norm="fg", tol_order=6.0)
    sg = ex.Solver(n, p.box, 1e-12, graphs=True, **kw)
    sd = ex.Solver(n, p.box, 1e-12, graphs=False, **kw)
    ud, _, std = sd.solve(fd, gd)
    ud = ud.clone()
    for _ in range(3):
        ug, _, stg = sg.solve(fd, gd)
        assert torch.equal(ug, ud)
        assert stg["iters"] == std["iters"]


@pytest.mark.parametrize("case", ["ex4-aniso", "ex2-ragged", "ex5-fp32"])
def test_coarse_tolerance_solve_parity(ex, orc, case):
    """tol_coarse: the grids below the finest stop at tol_coarse, the finest at tol (the reading that reproduces the
    anisotropic example's finest meshes).  Those grids are the grids of a run to the mesh n/2 at tol_coarse, so their
    counts are the oracle's for that run (within one); the finest count is within one of the oracle's free-running
    count from there (FP64), and u is the oracle's with the counts of the HIP path (FP32 refinement, whose finest
    count is of inner iterations: within 1% of the discretisation error, as in the mixed-precision parity tests)."""
    e, n, nc, tol, tc, prec = {
        "ex4-aniso": (4, (128, 64, 32), (8, 4, 2), 1e-9, 1e-11, ex.FP64),
        "ex2-ragged": (2, (80, 48, 112), (10, 6, 14), 1e-11, 1e-13, ex.FP64),
        # the finest grid in FP32 refinement to the discretisation error, the grids below at a looser tolerance
        "ex5-fp32": (5, (128, 128, 128), (4, 4, 4), 1e-14, 1e-12, ex.FP32_IR),
    }[case]
    p = synth.example(e)
    f, g, u = synth.sample(p, n)
    s = ex.Solver(n, p.box, tol, n_coarse=nc, tol_coarse=tc, precision=prec)
    ug, _, st = s.solve(dev(f), dev(g))
    ug = host(ug)
    gi = np.array(st["iters"], dtype=np.int32)
    L = st["levels"]
    half = orc.excmg(f[::2, ::2, ::2], g[::2, ::2, ::2], p.box, s.n_coarse, tc)
    assert np.all(np.abs(gi[:-1] - half["iters"]) <= 1), (gi, half["iters"])
    free = orc.excmg(f, g, p.box, s.n_coarse, tol, fixed_iters=np.r_[half["iters"], -1])
    if prec == ex.FP64:  # (the FP32 refinement counts inner iterations)
        assert abs(int(gi[-1]) - int(free["iters"][-1])) <= 1, (gi, free["iters"])
    for l in range(2, L):
        assert st["relres"][l] <= (tol if l == L - 1 else tc), (l, st["relres"])
    if prec == ex.FP64:
        ref = orc.excmg(f, g, p.box, s.n_coarse, tol, fixed_iters=gi)
        assert rel2(ug, ref["u"]) <= 1e-12
    else:
        rms = lambda a: float(np.sqrt(np.mean(np.square(a))))
        assert rms(ug - free["u"]) <= 0.01 * rms(free["u"] - u)
