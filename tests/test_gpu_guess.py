"""The initial guesses the paper compares (its EXP_finite, the tri-quadratic variant, CMG's trilinear prolongation):
parity of the HIP path with the oracle, step by step and for whole solves, and the ordering of the finest grid's
CG iterations that the remark after eq. (inter) in Section 4.3 predicts.

Tolerances as in test_gpu_parity.py: single steps max |gpu - oracle| <= 1e-13 max |oracle|; whole solves relative L2
<= 1e-12 after matching the per-grid iteration counts (free-running counts within one).
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


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def rel2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


RNG = np.random.default_rng(77)


def rnd(n):
    return RNG.standard_normal((n[2] + 1, n[1] + 1, n[0] + 1))


@pytest.mark.parametrize("kind,n", [("quartic", (16, 8, 24)), ("quadratic", (16, 8, 24)), ("quadratic", (72, 40, 8)),
                                    ("quadratic", (8, 8, 8)), ("linear", (10, 6, 14)), ("linear", (72, 40, 8)),
                                    ("linear", (2, 2, 2))])
def test_initial_guess_step(ex, orc, kind, n):
    u2 = rnd(tuple(v // 2 for v in n))
    u4 = rnd(tuple(v // 4 for v in n)) if kind != "linear" else None
    g = rnd(n)
    w = host(ex.op_initial_guess(kind, dev(u2), None if u4 is None else dev(u4), dev(g), n))
    ref = orc.initial_guess(kind, u2, u4, g)
    assert relmax(w, ref) <= 1e-13


@pytest.mark.parametrize("kind", ["quadratic", "linear"])
@pytest.mark.parametrize("case", ["cube64", "aniso"])
def test_guess_solve_parity(ex, orc, kind, case):
    p, n, nc, tol = {
        "cube64": (synth.smooth(0), (64, 64, 64), (4, 4, 4), 1e-10),
        "aniso": (synth.smooth(0), (128, 64, 32), (8, 4, 2), 1e-10),
    }[case]
    f, g, _ = synth.sample(p, n)
    s = ex.Solver(n, p.box, tol, n_coarse=nc, guess=kind)
    ug, _, st = s.solve(dev(f), dev(g))
    ug = host(ug)
    free = orc.excmg_guess(kind, f, g, p.box, s.n_coarse, tol)
    gi = np.array(st["iters"], dtype=np.int32)
    assert np.all(np.abs(gi - free["iters"]) <= 1), (gi, free["iters"])
    ref = orc.excmg_guess(kind, f, g, p.box, s.n_coarse, tol, fixed_iters=gi)
    assert rel2(ug, ref["u"]) <= 1e-12
    for l in range(2, st["levels"]):
        assert st["relres"][l] <= tol


def test_finest_iterations_follow_the_guess_order(ex):
    """On the seeded smooth field at 256^3 (from 4^3, tol 1e-10) the finest grid needs fewer CG iterations from the
    tri-quartic guess than from the tri-quadratic one, and fewer from that than from CMG's trilinear one; all three
    reach the same solution (to the tolerance)."""
    p = synth.smooth(0)
    n = (256, 256, 256)
    f, g, _ = synth.sample(p, n)
    f, g = dev(f), dev(g)
    its, sols = {}, {}
    for kind in ("quartic", "quadratic", "linear"):
        s = ex.Solver(n, p.box, 1e-10, guess=kind)
        u, _, st = s.solve(f, g)
        its[kind] = st["iters"][-1]
        sols[kind] = u
        del s
    assert its["quartic"] < its["quadratic"] < its["linear"], its
    for kind in ("quadratic", "linear"):
        d = float(torch.linalg.vector_norm(sols[kind] - sols["quartic"]) / torch.linalg.vector_norm(sols["quartic"]))
        assert d <= 1e-7, (kind, d)


def test_batched_solves_take_only_exp_finite(ex):
    p = synth.smooth(0)
    n = (32, 32, 32)
    f, g, _ = synth.sample(p, n)
    s = ex.Solver(n, p.box, 1e-10, guess="linear")
    with pytest.raises(ex.ExcmgError):
        ex.solve_batched([s], [dev(f)], [dev(g)])


def test_bad_guess_name(ex):
    with pytest.raises(ValueError):
        ex.Solver((16, 16, 16), guess="cubic")
