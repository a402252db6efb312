"""excmg_solve_noalloc, the solve for callers that cannot allocate device memory, against excmg_solve through the C
ABI: the same kernels on the same inputs, so the outputs must agree bit for bit (both launch every CG iteration
directly or replay graphs of the same launches, which give the same bits), on two calls in a row, the second on a
smaller problem than the first (the fixed scratch array keeps the first call's contents).  A problem larger than
the array is rejected before any device work."""
import ctypes

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


def noalloc_solve(ex, n, box, tol, f, g, precision, want_ext=True):
    from paper_1507_05063_amd import _lib

    p = ex._problem(n, box, tol, (0, 0, 0), precision)
    shape = (n[2] + 1, n[1] + 1, n[0] + 1)
    u = torch.empty(shape, dtype=torch.float64, device="cuda")
    ue = torch.empty(shape, dtype=torch.float64, device="cuda") if want_ext else None
    st = _lib.Stats()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = _lib.lib().excmg_solve_noalloc(ctypes.byref(p), ctypes.c_void_p(f.data_ptr()),
                                          ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                          ctypes.c_void_p(ue.data_ptr()) if want_ext else None, stream,
                                          ctypes.byref(st))
    return code, u, ue, st.to_dict()


def test_noalloc_matches_solve_on_two_calls(ex):
    from paper_1507_05063_amd import _lib

    # first 128^3 in FP32 refinement (117 MiB of workspace), then a smaller 64^3 problem in FP64
    for n, prec, seed in (((128, 128, 128), ex.FP32_IR, 0), ((64, 64, 64), ex.FP64, 3)):
        p = synth.smooth(seed)
        assert ex.workspace_bytes(n, precision=prec) <= _lib.NOALLOC_MAX_BYTES
        f_np, g_np, _ = synth.sample(p, n)
        f, g = dev(f_np), dev(g_np)
        s = ex.Solver(n, p.box, 1e-10, precision=prec)
        ref_u, ref_ue, ref_st = s.solve(f, g, want_ext=True)
        code, u, ue, st = noalloc_solve(ex, n, p.box, 1e-10, f, g, prec)
        assert code == 0, code
        assert st["iters"] == ref_st["iters"] and st["ir_outer"] == ref_st["ir_outer"]
        assert torch.equal(u, ref_u) and torch.equal(ue, ref_ue)
        del s


def test_noalloc_rejects_problems_over_the_array(ex):
    from paper_1507_05063_amd import _lib

    n = (256, 256, 256)
    assert ex.workspace_bytes(n) > _lib.NOALLOC_MAX_BYTES
    z = torch.zeros((n[2] + 1, n[1] + 1, n[0] + 1), dtype=torch.float64, device="cuda")
    code, _, _, _ = noalloc_solve(ex, n, (1.0, 1.0, 1.0), 1e-10, z, z, ex.FP64, want_ext=False)
    assert code == _lib.ERR_SCRATCH
