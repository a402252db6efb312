"""Batched solves (many independent problems in shared launches) against the oracle and against one-at-a-time solves.

Bars: FP64 problems match the oracle run with the batch's per-grid iteration counts to a relative L2 of 1e-12 (the
parity bar of the single solve), with free-running counts within one of the oracle's.  Problems relaxed in FP32 inside
FP64 refinement take other iterates than any FP64 run, so they are held to what the refinement promises: at the
workload's tol 1e-10, the final FP64 residual meets the tolerance on every grid and the difference from the FP64
oracle solution (same tolerance) stays below half of that solution's error against the exact field (max norm); and at
tol 1e-13, where every problem's error is its discretisation error, the difference from the oracle is at most 1% of
that error.  (Two iterates that both meet a relative residual of 1e-10 can differ by a sizeable part of the
discretisation error on strongly anisotropic grids, where M is badly conditioned: on the 128 x 192 x 192 problem with
hx about 5 hy the difference is 15% of it.)
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


# Uneven shapes and boxes, different level counts (1 to 5 grids) and every relaxation kind: direct solves only, the
# single-workgroup CG (grids of <= 8000 unknowns), multi-workgroup FP64 CG.
MIXED = [
    ((32, 64, 96), (2, 4, 6), synth.smooth(0, (0.7, 1.3, 1.9))),
    ((64, 64, 64), (4, 4, 4), synth.smooth(1)),
    ((16, 16, 16), (4, 4, 4), synth.smooth(2, (1.0, 0.5, 0.8))),
    ((8, 8, 8), (4, 4, 4), synth.example(2)),
    ((6, 10, 14), (6, 10, 14), synth.example(3)),
    ((96, 32, 64), (6, 2, 4), synth.smooth(3, (1.5, 0.6, 1.1))),
    ((128, 64, 32), (8, 4, 2), synth.smooth(4)),
]


def _run(ex, cases, tol, precision):
    solvers, fs, gs, data = [], [], [], []
    for n, nc, p in cases:
        f, g, u = synth.sample(p, n)
        solvers.append(ex.Solver(n, p.box, tol, n_coarse=nc, precision=precision))
        fs.append(dev(f))
        gs.append(dev(g))
        data.append((f, g, u, p))
    us, stats, ms = ex.solve_batched(solvers, fs, gs)
    return solvers, fs, gs, data, us, stats, ms


def test_batched_fp64_matches_oracle(ex, orc):
    tol = 1e-10
    solvers, fs, gs, data, us, stats, ms = _run(ex, MIXED, tol, ex.FP64)
    for (n, nc, p), s, (f, g, u, _), ub, st, t in zip(MIXED, solvers, data, us, stats, ms):
        free = orc.excmg(f, g, p.box, s.n_coarse, tol)
        gi = np.array(st["iters"], dtype=np.int32)
        assert np.all(np.abs(gi - free["iters"]) <= 1), (n, gi, free["iters"])
        ref = orc.excmg(f, g, p.box, s.n_coarse, tol, fixed_iters=gi)
        ub = host(ub)
        assert rel2(ub, ref["u"]) <= 1e-12, n
        mask = synth.boundary_mask(n)
        assert np.array_equal(ub[mask], g[mask])
        for l in range(2, st["levels"]):
            assert st["relres"][l] <= tol
        assert t > 0.0


def test_batched_equals_single_solves(ex):
    tol = 1e-10
    solvers, fs, gs, data, us, stats, ms = _run(ex, MIXED, tol, ex.FP64)
    for s, f, g, ub, st in zip(solvers, fs, gs, us, stats):
        u1, _, st1 = s.solve(f, g)
        assert all(abs(a - b) <= 1 for a, b in zip(st["iters"], st1["iters"])), (st["iters"], st1["iters"])
        assert rel2(host(ub), host(u1)) <= 1e-11


def test_batched_repeatable(ex):
    solvers, fs, gs, data, us, stats, ms = _run(ex, MIXED[:3], 1e-10, ex.FP64)
    us2, stats2, _ = ex.solve_batched(solvers, fs, gs)
    for a, b in zip(us, us2):
        assert torch.equal(a, b)
    assert [s["iters"] for s in stats] == [s["iters"] for s in stats2]


def test_batched_autotune_keeps_results(ex, orc):
    """After the batched autotuner picks the z chunks of the batched sweeps, the batch still meets the parity bar
    against the oracle (FP64, the batch's per-grid iteration counts) and every chosen chunk is a candidate."""
    tol = 1e-10
    solvers, fs, gs, data, us, stats, ms = _run(ex, MIXED, tol, ex.FP64)
    zc = ex.autotune_batched(solvers)
    assert zc and all(a in (0, 2, 4, 8, 16, 32, 64, 128) and b == 0 for a, b in zc.values()), zc
    us, stats, ms = ex.solve_batched(solvers, fs, gs)
    for (n, nc, p), s, (f, g, u, _), ub, st in zip(MIXED, solvers, data, us, stats):
        ref = orc.excmg(f, g, p.box, s.n_coarse, tol, fixed_iters=np.array(st["iters"], dtype=np.int32))
        assert rel2(host(ub), ref["u"]) <= 1e-12, n


@pytest.mark.parametrize("ty,depth", [(4, 2), (8, 3), (16, 4), (4, 6), (16, 6)])
def test_batched_tile_heights_match_oracle(ex, orc, ty, depth):
    """The batched CG passes at each tile height and prefetch depth (set on the batch's first solver), FP64, against
    the oracle with the batch's per-grid iteration counts; bad shapes are refused."""
    tol = 1e-10
    solvers, fs, gs, data, us, stats, ms = _run(ex, MIXED, tol, ex.FP64)
    solvers[0].set_batch_shape((ty, ty, depth, depth))
    assert solvers[0].get_batch_shape() == (ty, ty, depth, depth)
    us, stats, ms = ex.solve_batched(solvers, fs, gs)
    for (n, nc, p), s, (f, g, u, _), ub, st in zip(MIXED, solvers, data, us, stats):
        ref = orc.excmg(f, g, p.box, s.n_coarse, tol, fixed_iters=np.array(st["iters"], dtype=np.int32))
        assert rel2(host(ub), ref["u"]) <= 1e-12, n
    for bad in [(12, 4, 2, 2), (4, 4, 5, 2)]:
        with pytest.raises(ex.ExcmgError):
            solvers[0].set_batch_shape(bad)


# two problems whose finest grids relax in FP32 (127 x 127 x 95 and 191 x 95 x 63 unknowns), and the oracle's solutions
BIG32 = [
    ((128, 128, 96), (8, 8, 6), synth.smooth(6, (1.0, 1.0, 0.75))),
    ((192, 96, 64), (12, 6, 4), synth.smooth(7, (1.5, 0.75, 0.5))),
]
_REF32 = {}


@pytest.mark.parametrize("ty,depth", [(4, 2), (8, 4), (16, 6)])
def test_batched_fp32_tile_heights_against_oracle(ex, orc, ty, depth):
    """The batched FP32 refinement passes at each tile height, against the FP64 oracle where both are limited by the
    discretisation error (tol 1e-13): the batch's solution within 1% of the oracle's own error against the exact field
    (root mean square over all nodes)."""
    tol = 1e-13
    solvers, fs, gs, data = [], [], [], []
    for n, nc, p in BIG32:
        f, g, u = synth.sample(p, n)
        solvers.append(ex.Solver(n, p.box, tol, n_coarse=nc, precision=ex.FP32_IR))
        fs.append(dev(f))
        gs.append(dev(g))
        data.append((f, g, u))
    solvers[0].set_batch_shape((4, ty, 2, depth))
    us, stats, ms = ex.solve_batched(solvers, fs, gs)
    rms = lambda a: float(np.sqrt(np.mean(np.square(a))))
    for q, ((n, nc, p), (f, g, u)) in enumerate(zip(BIG32, data)):
        assert stats[q]["ir_outer"][-1] >= 1, stats[q]["ir_outer"]  # the finest grid relaxed in FP32
        if q not in _REF32:
            _REF32[q] = orc.excmg(f, g, p.box, nc, tol)["u"]
        ref = _REF32[q]
        assert rms(host(us[q]) - ref) <= 0.01 * rms(ref - u), n


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_batched_graphs_match_direct_launches(ex, precision):
    """The CG iterations of each batched round run as graphs cached on the first handle; the same batch with every
    launch made directly (EXCMG_NO_GRAPHS on the first handle) must agree bit for bit, on every one of several calls
    (later calls replay cached graphs) with other device work in between."""
    prec = ex.FP64 if precision == "fp64" else ex.FP32_IR
    cases = MIXED if precision == "fp64" else [((128, 128, 128), (4, 4, 4), synth.smooth(2)), MIXED[1], MIXED[6]]
    fs, gs, graph, eager = [], [], [], []
    for n, nc, p in cases:
        f, g, _ = synth.sample(p, n)
        fs.append(dev(f))
        gs.append(dev(g))
        graph.append(ex.Solver(n, p.box, 1e-10, n_coarse=nc, precision=prec))
        eager.append(ex.Solver(n, p.box, 1e-10, n_coarse=nc, precision=prec, graphs=False))
    ref, st_ref, _ = ex.solve_batched(eager, fs, gs)
    assert eager[0].batch_graph_counts() == (0, 0)
    x = dev(np.random.default_rng(1).standard_normal((17, 17, 17)))
    for rep in range(3):
        us, st, _ = ex.solve_batched(graph, fs, gs)
        assert [a["iters"] for a in st] == [a["iters"] for a in st_ref], rep
        for a, b in zip(us, ref):
            assert torch.equal(a, b), rep
        ex.op_apply(x, (16, 16, 16))  # unrelated eager work between the calls
        torch.cuda.synchronize()
    replays, captures = graph[0].batch_graph_counts()
    assert captures >= 1 and replays >= 1, (replays, captures)


def test_batched_rejects_bad_workspace(ex):
    solvers, fs, gs, data, us, stats, ms = _run(ex, MIXED[3:4], 1e-10, ex.FP64)
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    import ctypes

    from paper_1507_05063_amd import _lib

    H = (ctypes.c_void_p * 1)(solvers[0].handle.value)
    P = (ctypes.c_void_p * 1)(fs[0].data_ptr())
    Q = (ctypes.c_void_p * 1)(gs[0].data_ptr())
    U = (ctypes.c_void_p * 1)(us[0].data_ptr())
    code = _lib.lib().excmg_solve_batched(H, 1, P, Q, U, ctypes.c_void_p(small.data_ptr()), 64, None, None)
    assert code == _lib.ERR_WORKSPACE


# ------------------------------------------------------------------------- the 96-problem workload, FP32 refinement

@pytest.fixture(scope="module")
def batch96(ex):
    """96 problems (master seed 4): cells per axis from {32, 64, 96, 128, 192}, box edges U(0.5, 2), coarsest grid
    N/16 per axis (5 grids), FP32-in-FP64 refinement, tolerance 1e-10."""
    cases = [(n, tuple(v // 16 for v in n), p) for n, p in synth.batch(4, 96)]
    solvers, fs, gs, data, us, stats, ms = _run(ex, cases, 1e-10, ex.FP32_IR)
    return cases, solvers, data, [host(u) for u in us], stats, ms


@pytest.fixture(scope="module")
def batch96_tight(ex):
    """The same 96 problems at tol 1e-13 (FP32-in-FP64 refinement), with the batched autotuner's chunks, where every
    problem's error is its discretisation error."""
    cases = [(n, tuple(v // 16 for v in n), p) for n, p in synth.batch(4, 96)]
    solvers, fs, gs, data = [], [], [], []
    for n, nc, p in cases:
        f, g, u = synth.sample(p, n)
        solvers.append(ex.Solver(n, p.box, 1e-13, n_coarse=nc, precision=ex.FP32_IR))
        fs.append(dev(f))
        gs.append(dev(g))
        data.append((f, g, u, p))
    ex.autotune_batched(solvers)
    us, stats, ms = ex.solve_batched(solvers, fs, gs)
    return cases, data, [host(u) for u in us], stats


@pytest.mark.timeout(600)
@pytest.mark.parametrize("b", range(0, 96, 16))
def test_batch96_fp32_ir_within_discretisation_error(ex, orc, batch96_tight, b):
    """Mixed precision against the FP64 oracle where both are discretisation-limited: the batch's FP32-refinement
    result differs from the oracle's FP64 cascade (same tolerance, 1e-13) by at most 1% of the oracle's own error
    against the exact field (max norm), on every problem."""
    cases, data, us, stats = batch96_tight
    for q in range(b, b + 16):
        n, nc, p = cases[q]
        f, g, u, _ = data[q]
        for l in range(2, 5):
            assert stats[q]["relres"][l] <= 1e-13, (q, n, stats[q]["relres"])
        ref = orc.excmg(f, g, p.box, nc, 1e-13)
        disc = np.max(np.abs(ref["u"] - u))
        diff = np.max(np.abs(us[q] - ref["u"]))
        assert diff <= 0.01 * disc, (q, n, diff, disc)


@pytest.mark.parametrize("b", range(0, 96, 8))
def test_batch96_fp32_ir_against_oracle(ex, orc, batch96, b):
    cases, solvers, data, us, stats, ms = batch96
    for q in range(b, b + 8):
        n, nc, p = cases[q]
        f, g, u, _ = data[q]
        st = stats[q]
        assert st["levels"] == 5
        for l in range(2, 5):
            assert st["relres"][l] <= 1e-10, (q, n, st["relres"])
        ref = orc.excmg(f, g, p.box, nc, 1e-10)
        disc = np.max(np.abs(ref["u"] - u))
        diff = np.max(np.abs(us[q] - ref["u"]))
        assert diff <= 0.5 * disc, (q, n, diff, disc)
        mask = synth.boundary_mask(n)
        assert np.array_equal(us[q][mask], g[mask])
        assert ms[q] > 0.0


def test_batched_single_and_mixed_precision(ex, orc):
    """A batch of one, and a batch mixing FP64 and FP32-refinement problems of different level counts."""
    n, nc, p = MIXED[1]
    solvers, fs, gs, data, us, stats, ms = _run(ex, [MIXED[1]], 1e-10, ex.FP64)
    f, g, _, _ = data[0]
    ref = orc.excmg(f, g, p.box, nc, 1e-10, fixed_iters=np.array(stats[0]["iters"], dtype=np.int32))
    assert rel2(host(us[0]), ref["u"]) <= 1e-12
    cases = [(n, nc, p), ((128, 128, 128), (4, 4, 4), synth.smooth(2)), MIXED[3]]
    precs = [ex.FP64, ex.FP32_IR, ex.FP32_IR]
    solvers, fs, gs, data = [], [], [], []
    for (n_, nc_, p_), pr in zip(cases, precs):
        f_, g_, u_ = synth.sample(p_, n_)
        solvers.append(ex.Solver(n_, p_.box, 1e-10, n_coarse=nc_, precision=pr))
        fs.append(dev(f_))
        gs.append(dev(g_))
        data.append((f_, g_, u_, p_))
    us, stats, ms = ex.solve_batched(solvers, fs, gs)
    # the 128^3 FP32-refinement problem refines in FP32 on its finest grid only (the coarser ones are < 2^20 unknowns)
    assert stats[1]["ir_outer"][-1] >= 1 and all(o == 0 for o in stats[1]["ir_outer"][:-1])
    for (n_, nc_, p_), s_, (f_, g_, u_, _), ub, st in zip(cases, solvers, data, us, stats):
        for l in range(2, st["levels"]):
            assert st["relres"][l] <= 1e-10
        ref = orc.excmg(f_, g_, p_.box, s_.n_coarse, 1e-10)
        disc = max(np.max(np.abs(ref["u"] - u_)), 1e-14)
        assert np.max(np.abs(host(ub) - ref["u"])) <= 0.5 * disc


def test_batched_errors(ex):
    """An iteration cap is reported as EXCMG_ERR_NOCONV with every output written; a NaN in one problem's data stops
    the batch with EXCMG_ERR_NONFINITE."""
    n, nc, p = MIXED[1]
    f, g, _ = synth.sample(p, n)
    s1 = ex.Solver(n, p.box, 1e-14, n_coarse=nc, max_iters=3)
    s2 = ex.Solver(n, p.box, 1e-10, n_coarse=nc)
    us, stats, ms = ex.solve_batched([s1, s2], [dev(f), dev(f)], [dev(g), dev(g)], allow_noconv=True)
    assert stats[0]["iters"][-1] == 3 and stats[1]["relres"][-1] <= 1e-10
    bad = f.copy()
    bad[3, 4, 5] = np.nan
    with pytest.raises(ex.ExcmgError) as e:
        ex.solve_batched([s2, s2.__class__(n, p.box, 1e-10, n_coarse=nc)], [dev(f), dev(bad)], [dev(g), dev(g)])
    assert e.value.code == -3
