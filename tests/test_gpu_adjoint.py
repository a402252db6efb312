"""Differentiable solve: the GPU adjoint against the oracle's adjoint, and the autograd gradient against central
finite differences of the forward solve along seeded random directions.

The loss L = ||u(f, g) - u_t||^2 / 2 is quadratic in (f, g) for the exact discrete solution map, so the central
difference has no truncation error; what limits it is the forward solver: each forward solve stops at a residual of
tol * ||b||, so a perturbation is resolved only to about tol * ||b|| / ||perturbation of b||.  The step is therefore
relative to the data: (f, g) +- eps * ||(f, g)|| * d with d a unit direction and eps = 1e-6, and the forward solves of
the differences run at tol 1e-14 (the solve that is differentiated, and its adjoint, at 1e-13); the check threshold
is a relative 1e-5 of the directional derivative.  (At 256^3 with u = r^2.5, forward solves at 1e-13 measured up to
1.9e-5: the solver's stopping error, not the adjoint, set the difference.)
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


@pytest.mark.parametrize("n,nc,box", [((32, 32, 32), (4, 4, 4), (1.0, 1.0, 1.0)),
                                      ((32, 16, 16), (8, 4, 4), (1.0, 0.7, 1.2))])
def test_adjoint_matches_oracle(ex, orc, n, nc, box):
    p = synth.smooth(0, box)
    f, g, _ = synth.sample(p, n)
    _, _, ut = synth.sample(synth.smooth(5, box), n)
    s = ex.Solver(n, box, 1e-12, n_coarse=nc)
    u, _, _ = s.solve(dev(f), dev(g))
    G = host(u) - ut
    dLdf, dLdg, lam, st = s.adjoint(dev(G), want_lambda=True)
    ref = orc.adjoint(G, box, nc, 1e-12, fixed_iters=np.array(st["iters"], dtype=np.int32))
    for a, b in [(host(lam), ref["lam"]), (host(dLdf), ref["dLdf"]), (host(dLdg), ref["dLdg"])]:
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)
    assert np.all(host(dLdg)[~synth.boundary_mask(n)] == 0.0)


def _central_difference(s, f, g, df, dg, ut, eps):
    """(L(+eps d) - L(-eps d)) / (2 eps), summed as (u+ - u-).(u+ + u- - 2 u_t) / 2 so that the large loss values
    do not cancel."""
    up, _, _ = s.solve(f + eps * df, g + eps * dg)
    um, _, _ = s.solve(f - eps * df, g - eps * dg)
    return 0.5 * float(torch.sum((up - um) * (up + um - 2.0 * ut))) / (2.0 * eps)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("N", [64, 256])
@pytest.mark.parametrize("problem", ["smooth", "r25"])
def test_autograd_against_central_differences(ex, problem, N):
    """256^3 is the differentiation workload (7 grids from 4^3); 64^3 the same check on a small grid."""
    from paper_1507_05063_amd.autograd import solve as dsolve

    n = (N, N, N)
    p = synth.smooth(0) if problem == "smooth" else synth.r25()
    f_np, g_np, _ = synth.sample(p, n)
    _, _, ut_np = synth.sample(synth.smooth(5), n)
    s = ex.Solver(n, p.box, 1e-13)
    f = dev(f_np).requires_grad_(True)
    g = dev(g_np).requires_grad_(True)
    ut = dev(ut_np)
    u = dsolve(f, g, s)
    L = 0.5 * torch.sum((u - ut) ** 2)
    L.backward()
    gf, gg = f.grad.detach(), g.grad.detach()
    sfd = ex.Solver(n, p.box, 1e-14)  # the forward solves of the central differences
    for seed in range(6, 14):  # 8 seeded directions
        df, dg = synth.direction(seed, n)
        df, dg = dev(df), dev(dg)
        an = float(torch.sum(gf * df) + torch.sum(gg * dg))
        scale = float(torch.sqrt(torch.sum(f.detach() ** 2) + torch.sum(g.detach() ** 2)))
        with torch.no_grad():
            fd = _central_difference(sfd, f.detach(), g.detach(), df, dg, ut, 1e-6 * scale)
        print(f"{problem} {N}^3 direction seed {seed}: adjoint {an:.12e} central difference {fd:.12e} "
              f"rel {abs(fd - an) / abs(an):.2e}", flush=True)
        assert abs(fd - an) <= 1e-5 * abs(an), (seed, fd, an)
