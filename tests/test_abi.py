"""C-ABI checks that need no GPU: the library loads, exports every declared symbol, and its host-only entry points
(level plan, workspace size, argument validation, error strings) behave as documented in include/excmg.h."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "excmg.h")


@pytest.fixture(scope="module")
def abi():
    from paper_1507_05063_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_1507_05063_amd import build

        build.build()
    return _lib


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char \*)\s*\**\s*(excmg_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_path():
    names = declared_functions()
    for required in ["excmg_setup", "excmg_solve", "excmg_gradient", "excmg_adjoint", "excmg_solve_batched",
                     "excmg_workspace_bytes", "excmg_destroy", "excmg_strerror"]:
        assert required in names


def test_library_exports_every_declared_symbol(abi):
    L = ctypes.CDLL(abi.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def _plan(abi, n, nc=(0, 0, 0), tol=1e-10, box=(1, 1, 1), precision=0):
    import paper_1507_05063_amd as ex

    return ex.plan(n, nc, box, tol)


@pytest.mark.parametrize("n,levels,nc", [
    ((64, 64, 64), 5, (4, 4, 4)),            # uniform levels 4 -> 64
    ((512, 512, 512), 8, (4, 4, 4)),         # 4 -> 512, 8 grids
    ((1024, 512, 256), 8, (8, 4, 2)),        # unequal meshsizes, coarsest 8x4x2
    ((32, 96, 192), 5, (2, 6, 12)),          # uneven batch shape: N/16
    ((256, 256, 256), 7, (4, 4, 4)),
    ((6, 10, 14), 1, (6, 10, 14)),           # halves would be odd: one grid, solved directly
    ((20, 12, 36), 2, (10, 6, 18)),
    ((4, 4, 4), 1, (4, 4, 4)),
])
def test_automatic_level_plan(abi, n, levels, nc):
    assert _plan(abi, n) == (levels, nc)


def test_explicit_coarsest(abi):
    assert _plan(abi, (128, 64, 32), (8, 4, 2)) == (5, (8, 4, 2))
    assert _plan(abi, (8, 8, 8), (2, 2, 2)) == (3, (2, 2, 2))


@pytest.mark.parametrize("n,nc", [((12, 12, 12), (3, 3, 3)),   # odd coarsest under a three-grid cascade
                                  ((16, 16, 16), (3, 3, 3)),   # 3 * 2^L never 16
                                  ((16, 16, 16), (4, 4, 2)),   # axes disagree on L
                                  ((1, 4, 4), (0, 0, 0))])
def test_bad_shapes(abi, n, nc):
    import paper_1507_05063_amd as ex

    with pytest.raises(ex.ExcmgError) as e:
        ex.plan(n, nc)
    assert e.value.code == abi.ERR_SHAPE


def test_bad_arguments(abi):
    import paper_1507_05063_amd as ex

    for kw in [dict(tol=0.0), dict(tol=-1.0), dict(box=(1, 0, 1)), dict(tol=float("nan"))]:
        with pytest.raises(ex.ExcmgError) as e:
            ex.plan((16, 16, 16), (0, 0, 0), kw.get("box", (1, 1, 1)), kw.get("tol", 1e-10))
        assert e.value.code == abi.ERR_ARG
    L = abi.lib()
    assert L.excmg_plan(None, None, None) == abi.ERR_ARG
    assert L.excmg_set_timing(None, 1) == abi.ERR_ARG
    sh = (ctypes.c_int32 * 4)(16, 2, 0, 4)
    assert L.excmg_get_sweep(None, 0, 0, sh) == abi.ERR_ARG
    assert L.excmg_set_sweep(None, 0, 0, sh) == abi.ERR_ARG
    bs = (ctypes.c_int32 * 4)(4, 4, 2, 2)
    assert L.excmg_get_batch_shape(None, bs) == abi.ERR_ARG
    assert L.excmg_set_batch_shape(None, bs) == abi.ERR_ARG


@pytest.mark.parametrize("flags,tol_order,ok", [(0, 0.0, True), (0, 6.0, True), (0, 16.0, True), (0, -1.0, False),
                                                (0, 16.5, False), (0, float("nan"), False), (32, 6.0, True),
                                                (64, 0.0, True), (32 | 64, 0.0, False), (128, 0.0, False), (256, 0.0, True),
                                                (8 | 16, 0.0, False)])
def test_problem_validation(abi, flags, tol_order, ok):
    """Flags (EXCMG_STOP_F_G = 32 accepted, unknown bits and both compared guesses rejected) and the level-dependent
    tolerance's order (0 <= p <= 16)."""
    import paper_1507_05063_amd as ex

    p = ex._problem((16, 16, 16), (1.0, 1.0, 1.0), 1e-10, flags=flags, tol_order=tol_order)
    b = ctypes.c_size_t(0)
    code = abi.lib().excmg_workspace_bytes(ctypes.byref(p), ctypes.byref(b))
    assert (code == abi.OK) == ok, code
    if not ok:
        assert code == abi.ERR_ARG


@pytest.mark.parametrize("tol_coarse,tol_order,ok", [(1e-11, 0.0, True), (0.5, 0.0, True), (0.0, 6.0, True),
                                                     (1e-11, 6.0, False), (-1e-11, 0.0, False), (1.0, 0.0, False),
                                                     (float("nan"), 0.0, False), (float("inf"), 0.0, False)])
def test_coarse_tolerance_validation(abi, tol_coarse, tol_order, ok):
    """The tolerance of the grids below the finest: 0 (off) or in (0, 1), and not together with tol_order."""
    import paper_1507_05063_amd as ex

    p = ex._problem((16, 16, 16), (1.0, 1.0, 1.0), 1e-9, tol_order=tol_order, tol_coarse=tol_coarse)
    b = ctypes.c_size_t(0)
    code = abi.lib().excmg_workspace_bytes(ctypes.byref(p), ctypes.byref(b))
    assert code == (abi.OK if ok else abi.ERR_ARG), code


def test_workspace_bytes_scale(abi):
    import paper_1507_05063_amd as ex

    b64 = ex.workspace_bytes((512, 512, 512))
    b32 = ex.workspace_bytes((512, 512, 512), precision=ex.FP32_IR)
    node = 513 ** 3 * 8
    # three finest FP64 work vectors plus the cascade's solutions (about 8/7 of a finest array), pitched rows
    assert 4.0 * node < b64 < 4.6 * node
    assert b32 - b64 > 1.9 * node  # four FP32 vectors more
    assert ex.workspace_bytes((64, 64, 64)) < b64


def test_setup_rejects_bad_workspace(abi):
    p = abi.Problem()
    for d in range(3):
        p.box[d] = 1.0
        p.n[d] = 16
    p.tol = 1e-10
    h = ctypes.c_void_p(0)
    L = abi.lib()
    assert L.excmg_setup(ctypes.byref(p), None, 0, None, ctypes.byref(h)) == abi.ERR_WORKSPACE
    assert L.excmg_setup(ctypes.byref(p), ctypes.c_void_p(256), 10, None, ctypes.byref(h)) == abi.ERR_WORKSPACE
    assert L.excmg_setup(ctypes.byref(p), ctypes.c_void_p(4096 + 8), 1 << 40, None, ctypes.byref(h)) == \
        abi.ERR_WORKSPACE
    assert not h.value


def test_strerror(abi):
    L = abi.lib()
    for code in [0, -1, -2, -3, -4, -5, -6, -7, -8]:
        assert L.excmg_strerror(code)
    assert L.excmg_strerror(-99) == b"unknown error code"


def test_product_path_does_not_import_the_oracle():
    """The GPU binding and the oracle share nothing: no import of oracle/ anywhere in the package or the C sources."""
    pkg = os.path.join(ROOT, "paper_1507_05063_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "oracle.h" not in txt, fn


def test_noalloc_argument_errors(abi):
    """excmg_solve_noalloc checks its arguments and the problem's size against its fixed array before any device
    call: null pointers, a bad plan, and a workspace over EXCMG_NOALLOC_MAX_BYTES."""
    import paper_1507_05063_amd as ex

    L = abi.lib()
    dummy = ctypes.c_void_p(4096)  # never dereferenced: every case returns before device work
    p = ex._problem((32, 32, 32), (1, 1, 1), 1e-10)
    assert L.excmg_solve_noalloc(None, dummy, dummy, dummy, None, None, None) == abi.ERR_ARG
    assert L.excmg_solve_noalloc(ctypes.byref(p), None, dummy, dummy, None, None, None) == abi.ERR_ARG
    assert L.excmg_solve_noalloc(ctypes.byref(p), dummy, dummy, None, None, None, None) == abi.ERR_ARG
    bad = ex._problem((30, 32, 32), (1, 1, 1), 1e-10, n_coarse=(4, 4, 4))
    assert L.excmg_solve_noalloc(ctypes.byref(bad), dummy, dummy, dummy, None, None, None) == abi.ERR_SHAPE
    big = ex._problem((256, 256, 256), (1, 1, 1), 1e-10)
    assert ex.workspace_bytes((256, 256, 256)) > abi.NOALLOC_MAX_BYTES
    assert L.excmg_solve_noalloc(ctypes.byref(big), dummy, dummy, dummy, None, None, None) == abi.ERR_SCRATCH
    one = ex._problem((4, 4, 4), (1, 1, 1), 1e-10, n_coarse=(4, 4, 4))  # one grid: no extrapolated solution
    assert L.excmg_solve_noalloc(ctypes.byref(one), dummy, dummy, dummy, dummy, None, None) == abi.ERR_SHAPE


def test_batch_workspace_bytes(abi):
    import paper_1507_05063_amd as ex

    one = ex.batch_workspace_bytes(1)
    many = ex.batch_workspace_bytes(96)
    assert 0 < one < many < 96 * 32 * 1024
    with pytest.raises(ex.ExcmgError):
        ex.batch_workspace_bytes(0)


def test_batched_argument_errors(abi):
    """Argument checks that return before any device call."""
    import ctypes

    from paper_1507_05063_amd import _lib

    L = _lib.lib()
    assert L.excmg_solve_batched(None, 1, None, None, None, None, 0, None, None) == _lib.ERR_ARG
    H = (ctypes.c_void_p * 1)(None)
    P = (ctypes.c_void_p * 1)(None)
    assert L.excmg_solve_batched(H, 1, P, P, P, None, 0, None, None) == _lib.ERR_ARG
    assert L.excmg_solve_batched(H, 0, P, P, P, None, 0, None, None) == _lib.ERR_ARG


def test_bandwidth_probe_argument_errors(abi):
    """Argument checks of the probe return before any device call; the kinds match the header's enum."""
    import paper_1507_05063_amd as ex

    L = abi.lib()
    rates = (ctypes.c_double * len(ex.PROBE_KINDS))()
    assert L.excmg_bandwidth_probe(None, 1 << 20, 1, None, rates, None) == abi.ERR_ARG
    assert L.excmg_bandwidth_probe(ctypes.c_void_p(16), 1024, 1, None, rates, None) == abi.ERR_ARG  # too few bytes
    assert L.excmg_bandwidth_probe(ctypes.c_void_p(8), 1 << 20, 1, None, rates, None) == abi.ERR_ARG  # misaligned
    assert L.excmg_bandwidth_probe(ctypes.c_void_p(16), 1 << 20, 0, None, rates, None) == abi.ERR_ARG  # no reps
    assert L.excmg_bandwidth_probe(ctypes.c_void_p(16), 1 << 20, 1, None, None, None) == abi.ERR_ARG  # no output
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    assert int(re.search(r"EXCMG_PROBE_KINDS\s*=\s*(\d+)", src).group(1)) == len(ex.PROBE_KINDS)


def test_initial_guess_argument_errors(abi):
    """The guess operator and the guess flags are checked before any device call."""
    L = abi.lib()
    n = (ctypes.c_int32 * 3)(8, 8, 8)
    p = ctypes.c_void_p(256)
    assert L.excmg_op_initial_guess(3, n, p, p, p, p, None) == abi.ERR_ARG  # unknown kind
    assert L.excmg_op_initial_guess(1, n, p, None, p, p, None) == abi.ERR_ARG  # the quadratic guess needs u4h
    n6 = (ctypes.c_int32 * 3)(8, 6, 8)
    assert L.excmg_op_initial_guess(1, n6, p, p, p, p, None) == abi.ERR_SHAPE  # not multiples of 8
    prob = abi.Problem()
    prob.box[:] = (1.0, 1.0, 1.0)
    prob.n[:] = (32, 32, 32)
    prob.tol = 1e-10
    prob.flags = abi.GUESS_QUADRATIC | abi.GUESS_LINEAR  # at most one of the two
    nbytes = ctypes.c_size_t(0)
    assert L.excmg_workspace_bytes(ctypes.byref(prob), ctypes.byref(nbytes)) == abi.ERR_ARG
    prob.flags = abi.GUESS_LINEAR
    assert L.excmg_workspace_bytes(ctypes.byref(prob), ctypes.byref(nbytes)) == abi.OK


def _auto_rule(n):
    """The automatic coarsest grid, restated: halve while the halves are all even, at least 2, and the largest is at
    least 4."""
    c, L = tuple(n), 1
    while True:
        h = tuple(v // 2 for v in c)
        if any(v % 2 for v in c) or any(v % 2 or v < 2 for v in h) or max(h) < 4:
            return L, c
        c, L = h, L + 1


from hypothesis import given, settings, strategies as st  # noqa: E402


@settings(max_examples=300, deadline=None)
@given(st.tuples(st.integers(1, 12), st.integers(1, 12), st.integers(1, 12)), st.integers(0, 6))
def test_level_plan_properties(abi, c, s):
    """Random hierarchies n = c * 2^s: the explicit coarsest c is accepted exactly when the cascade is well formed
    (every grid that serves as u_4h has even counts, i.e. c even or at most two grids, and c >= 2 on every axis), and
    the automatic plan follows the halving rule."""
    import paper_1507_05063_amd as ex

    n = tuple(v << s for v in c)
    L = s + 1
    ok = min(c) >= 2 and (L <= 2 or all(v % 2 == 0 for v in c))
    if ok:
        assert ex.plan(n, c) == (L, c)
        b = ex.workspace_bytes(n, c)
        assert b > 8 * (n[0] + 1) * (n[1] + 1) * (n[2] + 1)
    else:
        with pytest.raises(ex.ExcmgError):
            ex.plan(n, c)
    if min(n) >= 2:
        assert ex.plan(n) == _auto_rule(n)


def test_host_logic_under_sanitizers(tmp_path):
    """The library's host logic (level plans, workspace sizes, argument checks, error strings) built with
    AddressSanitizer and UndefinedBehaviorSanitizer on its host code only, driven by tests/abi_sanitize_main.c with
    leak detection: no invalid access, undefined operation or leak.  Needs no GPU."""
    import shutil
    import subprocess

    hipcc = shutil.which("hipcc")
    clang = "/opt/rocm/llvm/bin/clang"
    if hipcc is None or not os.path.exists(clang):
        pytest.skip("hipcc or the ROCm clang not found")
    csrc = os.path.join(ROOT, "paper_1507_05063_amd", "csrc")
    srcs = [os.path.join(csrc, f) for f in ("excmg.hip", "kernels_cg.hip", "kernels_transfer.hip", "kernels_grad.hip",
                                            "kernels_probe.hip")]
    lib = str(tmp_path / "libexcmg_san.so")
    cmd = [hipcc, "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-o", lib, *srcs]
    built = subprocess.run(cmd, capture_output=True, text=True)
    if built.returncode != 0:
        pytest.skip("no host sanitizer build: " + built.stderr[-300:])
    exe = str(tmp_path / "abi_san")
    link = [clang, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
            "-fno-omit-frame-pointer", os.path.join(ROOT, "tests", "abi_sanitize_main.c"), f"-L{tmp_path}",
            "-lexcmg_san", f"-Wl,-rpath,{tmp_path}", "-o", exe]
    linked = subprocess.run(link, capture_output=True, text=True)
    assert linked.returncode == 0, linked.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    if run.returncode != 0 and "does not come first in initial library list" in run.stderr:
        pytest.skip("the sanitizer runtime cannot come first in this process environment")
    assert run.returncode == 0, run.stderr[-3000:]
    assert "all checks passed" in run.stdout
