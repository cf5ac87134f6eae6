"""The C ABI without a GPU: the library loads, exports every entry point the
header declares, and rejects invalid arguments before any HIP call."""
import ctypes
import os
import re

import pytest

tc = pytest.importorskip("paper_1402_6601_amd")
HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "tchol.h")


@pytest.fixture(scope="module")
def lib():
    try:
        return tc.load()
    except ImportError as e:
        pytest.skip(str(e))


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:TCHOL_API\s+)?(?:const\s+)?\w+\s*\*?\s*(tchol_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ["tchol_factor", "tchol_solve", "tchol_workspace_bytes", "tchol_strerror", "tchol_factor_ex",
                     "tchol_solve_ex", "tchol_plan_query", "tchol_version"]:
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_internal_symbols_are_not_exported(lib):
    for name in ["tchol_dev_launch", "tchol_dev_max_grid", "tchol_dev_compact_grid", "tchol_refine_convert", "tchol_refine_residual",
                 "tchol_refine_colmax", "tchol_refine_axpy"]:
        with pytest.raises(AttributeError):
            getattr(lib, name)


def test_workspace_bytes_validation(lib):
    assert lib.tchol_workspace_bytes(7, 10, 16, 0) == -1
    assert lib.tchol_workspace_bytes(0, -1, 16, 0) == -2
    for nb in (0, 8, 24, 100, 528, 1024):
        assert lib.tchol_workspace_bytes(0, 10, nb, 0) == -3
    assert lib.tchol_workspace_bytes(1, 10, 16, -1) == -4
    assert lib.tchol_workspace_bytes(0, 0, 16, 0) > 0
    a = lib.tchol_workspace_bytes(0, 1024, 128, 0)
    b = lib.tchol_workspace_bytes(0, 2048, 128, 0)
    assert 0 < a < b and a % 256 == 0


FAKE = ctypes.c_void_p(0x10000)       # never dereferenced: every call below fails validation first
FAKE_MISALIGNED = ctypes.c_void_p(0x10008)


def test_factor_validation_before_any_hip_call(lib):
    need = lib.tchol_workspace_bytes(0, 256, 64, 0)
    assert lib.tchol_factor(FAKE, -1, 64, FAKE, need, None) == -2
    assert lib.tchol_factor(FAKE, 256, 40, FAKE, need, None) == -3
    assert lib.tchol_factor(FAKE, 256, 8, FAKE, need, None) == -3
    assert lib.tchol_factor(None, 0, 64, None, 0, None) == 0          # nothing to do
    assert lib.tchol_factor(None, 256, 64, FAKE, need, None) == -1
    assert lib.tchol_factor(FAKE, 256, 64, None, need, None) == -4
    assert lib.tchol_factor(FAKE, 256, 64, FAKE, 0, None) == -5
    assert lib.tchol_factor(FAKE, 256, 64, FAKE, 1024, None) == -5        # too small
    # the query covers the inverse-applying TRSMs (opts.inv_trsm), which need all of it
    o = tc.Opts()
    o.inv_trsm = 1
    assert lib.tchol_factor_ex(FAKE, 256, 64, FAKE, need - 256, None, ctypes.byref(o)) == -5
    assert lib.tchol_factor(FAKE, 256, 64, FAKE_MISALIGNED, need, None) == -4


def test_solve_validation_before_any_hip_call(lib):
    need = lib.tchol_workspace_bytes(1, 256, 64, 4)
    assert lib.tchol_solve(FAKE, -1, 64, FAKE, 4, FAKE, need, None) == -2
    assert lib.tchol_solve(FAKE, 256, 12, FAKE, 4, FAKE, need, None) == -3
    assert lib.tchol_solve(FAKE, 256, 64, FAKE, -1, FAKE, need, None) == -5
    assert lib.tchol_solve(FAKE, 256, 64, FAKE, 0, FAKE, need, None) == 0
    assert lib.tchol_solve(None, 256, 64, FAKE, 4, FAKE, need, None) == -1
    assert lib.tchol_solve(FAKE, 256, 64, None, 4, FAKE, need, None) == -4
    assert lib.tchol_solve(FAKE, 256, 64, FAKE, 4, None, need, None) == -6
    assert lib.tchol_solve(FAKE, 256, 64, FAKE, 4, FAKE, 16, None) == -7
    assert lib.tchol_solve(FAKE, 256, 64, FAKE, 4, FAKE_MISALIGNED, need, None) == -6


def test_mixed_validation_before_any_hip_call(lib):
    n, nb, k = 256, 64, 4
    need = lib.tchol_mixed_workspace_bytes(n, nb, k)
    # the FP32 working copy (ld n + 3 rounded up to 4) and the FP64 diagonal tiles dominate
    assert need >= 4 * 260 * n + 8 * 4 * nb * nb + 2 * 8 * n * k
    assert lib.tchol_mixed_workspace_bytes(-1, nb, k) == -1
    assert lib.tchol_mixed_workspace_bytes(n, 24, k) == -2
    assert lib.tchol_mixed_workspace_bytes(n, nb, -1) == -3
    berr = (ctypes.c_double * k)()
    it = ctypes.c_int32(-7)

    def call(A=FAKE, n_=n, nb_=nb, B=FAKE, k_=k, lowp=1, tol=1e-12, maxit=10, ws=FAKE, wsb=need):
        return lib.tchol_solve_mixed(A, n_, nb_, B, k_, lowp, tol, maxit, berr, ctypes.byref(it), ws, wsb, None, None)

    assert call(n_=-1) == -2
    assert call(nb_=40) == -3
    assert call(k_=-1) == -5
    assert call(lowp=0) == -6 and call(lowp=3) == -6
    # BF16 updates need room for the panels' three BF16 terms as well
    need_bf16 = lib.tchol_mixed_workspace_bytes_ex(n, nb, k, 2)
    assert need_bf16 >= need + 2 * 3 * n * n
    assert lib.tchol_mixed_workspace_bytes_ex(n, nb, k, 1) == need
    assert lib.tchol_mixed_workspace_bytes_ex(n, nb, k, 3) == -4
    assert call(lowp=2) == -12
    assert call(lowp=2, wsb=need_bf16 - 256) == -12
    assert call(tol=0.0) == -7 and call(tol=float("nan")) == -7
    assert call(maxit=-1) == -8
    assert call(n_=0) == 0 and it.value == 0
    assert call(k_=0) == 0
    assert call(A=None) == -1
    assert call(B=None) == -4
    assert call(ws=None) == -11
    assert call(ws=FAKE_MISALIGNED) == -11
    assert call(wsb=0) == -12
    assert call(wsb=need - 256) == -12


def test_mixed_workspace_query_over_sizes(lib):
    # ragged last tiles of every shape (one row, odd, padded), one-tile and multi-tile plans
    prev = 0
    for n, nb in [(1, 16), (17, 16), (513, 512), (999, 160), (1000, 128), (1024, 256), (2048, 512), (4097, 512)]:
        b = lib.tchol_mixed_workspace_bytes(n, nb, 4)
        assert b > 0 and b % 256 == 0
        if nb == 512:
            assert b > prev
            prev = b


def test_backward_validation_before_any_hip_call(lib):
    need = lib.tchol_workspace_bytes(3, 256, 64, 0)
    assert need >= 2 * 8 * 256 * 256 + 8 * 6 * 64 * 64
    assert lib.tchol_backward(FAKE, -1, 64, FAKE, FAKE, need, None) == -2
    assert lib.tchol_backward(FAKE, 256, 40, FAKE, FAKE, need, None) == -3
    assert lib.tchol_backward(None, 0, 64, None, None, 0, None) == 0
    assert lib.tchol_backward(None, 256, 64, FAKE, FAKE, need, None) == -1
    assert lib.tchol_backward(FAKE, 256, 64, None, FAKE, need, None) == -4
    assert lib.tchol_backward(FAKE, 256, 64, FAKE, None, need, None) == -5
    assert lib.tchol_backward(FAKE, 256, 64, FAKE, FAKE_MISALIGNED, need, None) == -5
    assert lib.tchol_backward(FAKE, 256, 64, FAKE, FAKE, 0, None) == -6
    assert lib.tchol_backward(FAKE, 256, 64, FAKE, FAKE, need - 256, None) == -6
    assert lib.tchol_backward(FAKE, 16 * 161, 16, FAKE, FAKE, need, None) == tc.E_UNSUPPORTED


def test_strerror_and_version(lib):
    for code in (0, 5, -3, tc.E_HIP, tc.E_TIMEOUT, tc.E_UNSUPPORTED, tc.E_INTERNAL, tc.E_NOCONV, -999):
        assert isinstance(tc.strerror(code), str) and tc.strerror(code)
    assert "gfx950" in tc.version()


def test_plan_query_validation(lib):
    with pytest.raises(tc.TcholError):
        tc.plan_query(6, 100, 16)
    with pytest.raises(tc.TcholError):
        tc.plan_query(0, 100, 20)
    with pytest.raises(tc.TcholError):
        tc.plan_query(0, 100, 16, policy=9)


def test_unsupported_size(lib):
    assert lib.tchol_workspace_bytes(0, 16 * 2000, 16, 0) == tc.E_UNSUPPORTED


def test_zeroed_options_select_the_default_policy(lib):
    """A zero-initialised tchol_opts and NULL options select the same claim
    order: the header numbers the list schedule 0, the binding agrees, and the
    plan built for policy 0 is the list schedule, whose ticket order differs
    from the task-by-task rank order."""
    text = open(HEADER).read()
    m = re.search(r"#define\s+TCHOL_POLICY_LIST\s+(\d+)", text)
    assert m and int(m.group(1)) == 0 == tc.POLICY_LIST
    assert tc.Opts().policy == tc.POLICY_LIST
    values = {int(v) for v in re.findall(r"#define\s+TCHOL_POLICY_\w+\s+(\d+)", text)}
    assert values == {0, 1, 2, 3}
    a = tc.plan_query(0, 2048, 128, 0)
    b = tc.plan_query(0, 2048, 128, tc.POLICY_LIST)
    r = tc.plan_query(0, 2048, 128, tc.POLICY_RANK)
    assert (a["item_task"] == b["item_task"]).all()
    assert not (a["item_task"] == r["item_task"]).all()



def test_noalloc_validation_and_scratch_limit(lib):
    f = lib.tchol_factor_solve_noalloc
    assert f(FAKE, -1, 128, FAKE, 1, None) == -2
    assert f(FAKE, 100, 24, FAKE, 1, None) == -3
    assert f(FAKE, 100, 128, FAKE, -1, None) == -5
    assert f(None, 0, 128, None, 1, None) == 0
    assert f(None, 100, 128, FAKE, 1, None) == -1
    assert f(FAKE, 100, 128, None, 1, None) == -4
    # problems whose scheduler scratch exceeds the fixed array are refused
    # before any HIP call; the bench configuration (n = 32768, nb = 512) fits.
    # Its solve substitutes against the diagonal tiles, so it needs what the
    # batched launch of the one system needs (no inverses, no y vector)
    fs = lambda n, nb: tc.batched_workspace_bytes([n], [nb])
    assert fs(32768, 512) <= tc.NOALLOC_SCRATCH_BYTES
    assert fs(32768, 256) > tc.NOALLOC_SCRATCH_BYTES
    assert lib.tchol_factor_solve_workspace_bytes(32768, 512, 16) > fs(32768, 512)
    assert f(FAKE, 32768, 256, FAKE, 16, None) == tc.E_SCRATCH
    assert "scratch" in tc.strerror(tc.E_SCRATCH)


def test_trace_buffer_too_small_is_refused(lib):
    """A trace buffer shorter than 4 words per work item of the launch is an
    invalid options argument, refused before anything is launched (the
    buffer is never written)."""
    n, nb, nrhs = 1024, 128, 2
    items = tc.plan_query(tc.OP_FACTOR_SOLVE, n, nb)["nitem"]
    o = tc.Opts()
    o.trace = FAKE
    o.trace_words = 4 * items - 1
    big = 1 << 40
    assert lib.tchol_factor_solve(FAKE, n, nb, FAKE, nrhs, FAKE, big, None, ctypes.byref(o)) == -9
    o.trace_words = 4 * tc.plan_query(tc.OP_SOLVE, n, nb)["nitem"] - 4
    assert lib.tchol_solve_ex(FAKE, n, nb, FAKE, nrhs, FAKE, big, None, ctypes.byref(o)) == -9
    o.trace_words = 4 * tc.plan_query(tc.OP_FACTOR, n, nb)["nitem"] - 1
    assert lib.tchol_factor_ex(FAKE, n, nb, FAKE, big, None, ctypes.byref(o)) == -7
