"""Host-side checks of the C ABI: the library loads, exports every call that
include/lmrs.h declares, sizes workspaces consistently and rejects bad
arguments before enqueuing anything (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lmrs.h")


@pytest.fixture(scope="module")
def M():
    from paper_2504_12905_amd import lmrs
    return lmrs


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:lmrs_status|size_t|const char\*)\s+(lmrs_\w+)\s*\(", text, re.M)))


def test_header_declares_the_eight_hot_path_calls():
    names = declared_functions()
    for n in ("lmrs_project", "lmrs_bin_tiles", "lmrs_render", "lmrs_jvp", "lmrs_vjp", "lmrs_gn_product",
              "lmrs_pcg", "lmrs_lm_step"):
        assert n in names


def test_library_exports_every_declared_symbol(M):
    lib = C.CDLL(M.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(M.EXPORTS)


def frame(M, **kw):
    f = M._Frame()
    f.n, f.sh_degree, f.n_views, f.width, f.height, f.k, f.capacity = 1000, 3, 8, 800, 800, 26, 10 ** 6
    for k, v in kw.items():
        setattr(f, k, v)
    return f


def test_workspace_sizes(M):
    ws = lambda op, **kw: M._lib.lmrs_workspace_bytes(op, C.byref(frame(M, **kw)))
    assert ws(M.OP_GN) >= 8 * 1000 * (12 + 9) * 4
    assert ws(M.OP_PCG) > ws(M.OP_GN) > ws(M.OP_JVP)
    assert ws(M.OP_LM) > ws(M.OP_PCG)
    assert ws(M.OP_BIN, capacity=2 * 10 ** 6) > ws(M.OP_BIN)
    assert all(ws(op) % 256 == 0 for op in range(1, 8))
    assert M._lib.lmrs_workspace_bytes(M.OP_GN, None) == 0


def test_deterministic_workspace_holds_fixed_point_rows(M):
    """Deterministic accumulation keeps 32 64-bit words per screen-gradient
    row (9 components as two integers each, a poison word, padding to whole
    128-byte lines) instead of 16 floats, and 80 per Gram row instead of 32
    floats."""
    ws = lambda op, **kw: M._lib.lmrs_workspace_bytes(op, C.byref(frame(M, **kw)))
    VN = 8 * 1000
    grow_grad = VN * (32 * 8 - 16 * 4)
    grow_gram = VN * (80 * 8 - 32 * 4)
    for op, grow in ((M.OP_GN, grow_grad), (M.OP_DIAG, grow_gram), (M.OP_PCG, grow_grad + grow_gram),
                     (M.OP_LM, grow_grad + grow_gram), (M.OP_JVP, 0)):
        d = ws(op, deterministic=1) - ws(op)
        assert abs(d - grow) <= 2 * 256, (op, d, grow)   # up to the 256-byte alignment of each buffer
    f = frame(M, deterministic=2)
    f.beta = 1
    assert M._lib.lmrs_render(C.byref(f), C.byref(M.default_opts()), None) == M.LMRS_EINVAL


@pytest.mark.parametrize("bad", [dict(n=0), dict(sh_degree=-1), dict(width=100), dict(n_views=0),
                                 dict(k=0), dict(k=300)])
def test_invalid_frames_rejected_on_host(M, bad):
    f = frame(M, **bad)
    f.beta = 1  # never dereferenced: validation fails first
    opts = M.default_opts()
    st = M._lib.lmrs_render(C.byref(f), C.byref(opts), None)
    assert st == M.LMRS_EINVAL
    assert M._lib.lmrs_last_error()


@pytest.mark.parametrize("big", [dict(sh_degree=4), dict(width=2064, height=2048)])
def test_unsupported_frames_rejected_on_host(M, big):
    """Well-formed but beyond what the library builds: SH degree 4, a view of
    more than 16384 tiles."""
    f = frame(M, **big)
    f.beta = 1
    st = M._lib.lmrs_render(C.byref(f), C.byref(M.default_opts()), None)
    assert st == M.LMRS_EUNSUPPORTED
    assert M._lib.lmrs_status_str(st) == b"not supported by this library"


def test_report_status(M):
    """lmrs_report_status reads the failure bits of a host copy of a report."""
    rep = (C.c_float * M.REPORT_FLOATS)()
    assert M._lib.lmrs_report_status(rep) == M.LMRS_OK
    rep[M.REP["status"]] = float(M.FAIL_BREAKDOWN)
    assert M._lib.lmrs_report_status(rep) == M.LMRS_ENUMERIC
    assert b"breakdown" in M._lib.lmrs_last_error()
    rep[M.REP["status"]] = float(M.FAIL_NONFINITE)
    assert M._lib.lmrs_report_status(rep) == M.LMRS_ENUMERIC
    assert b"non-finite" in M._lib.lmrs_last_error()
    assert M._lib.lmrs_report_status(None) == M.LMRS_EINVAL


def test_missing_buffers_and_small_workspace_rejected(M):
    f = frame(M)
    f.beta = 1
    opts = M.default_opts()
    assert M._lib.lmrs_render(C.byref(f), C.byref(opts), None) == M.LMRS_EINVAL  # pix NULL with k=26
    f.k = 256
    assert M._lib.lmrs_render(C.byref(f), C.byref(opts), None) == M.LMRS_EINVAL  # rec NULL
    assert b"rec" in M._lib.lmrs_last_error()
    for name in ("rec", "rect", "tile_start", "ids", "cams", "trans", "last"):
        setattr(f, name, 256)
    st = M._lib.lmrs_gn_product(C.byref(f), C.byref(opts), 256, C.c_float(0.1), None, 512, 256, 16, None)
    assert st == M.LMRS_EINVAL and b"sched" in M._lib.lmrs_last_error()  # no tile schedule buffer
    f.sched = 256
    st = M._lib.lmrs_gn_product(C.byref(f), C.byref(opts), 256, C.c_float(0.1), None, 512, 256, 16, None)
    assert st == M.LMRS_EWORKSPACE
    assert M._lib.lmrs_status_str(st) == b"workspace too small"
