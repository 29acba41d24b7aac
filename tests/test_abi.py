"""C-ABI checks that need no GPU: the library loads, exports every function
include/los.h declares, and rejects bad arguments before touching HIP."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "los.h")
LIB = os.path.join(ROOT, "paper_2509_25110_amd", "liblos.so")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2509_25110_amd import build
        build.build(verbose=False)
    from paper_2509_25110_amd import los
    return los.load_library(LIB)


def test_header_lists_expected_entry_points():
    names = header_functions()
    for n in ("los_bessel_table", "los_project", "cl_integrate", "los_ctx_create",
              "los_ctx_destroy", "los_last_error", "los_version"):
        assert n in names, names


def test_every_declared_symbol_is_exported(lib):
    for name in header_functions():
        assert hasattr(lib, name), "liblos.so does not export %s" % name
    from paper_2509_25110_amd import los
    assert set(los.EXPORTS) == set(header_functions())


def test_version_and_empty_error(lib):
    assert b"gfx950" in lib.los_version()
    assert isinstance(lib.los_last_error(), bytes)


def _dummy_ctx():
    # validation runs before the context is used, so any non-NULL handle works here
    buf = ctypes.create_string_buffer(64)
    return ctypes.cast(buf, ctypes.c_void_p), buf


def test_null_context_rejected(lib):
    rc = lib.los_project(None, 2, 10, 4, 8, 1.0, None, None, None, None, 1, 0, None, None)
    assert rc == 1 and b"ctx" in lib.los_last_error()
    rc = lib.los_bessel_table(None, None, 1, 0, 3, None, None)
    assert rc == 1
    rc = lib.los_ctx_create(None, None)
    assert rc == 1


def test_project_argument_validation(lib):
    ctx, _keep = _dummy_ctx()
    p = ctypes.c_void_p(16)  # never dereferenced: every call below fails validation
    cases = [
        dict(lmin=1, lmax=10),          # lmin < 2
        dict(lmin=10, lmax=9),          # lmax < lmin
        dict(lmax=20000),               # lmax too large
        dict(nk=0),
        dict(ntau=0),
        dict(ntau=9000),                # beyond the supported tau grid
        dict(nsrc=0),
        dict(nsrc=5),
        dict(prec=7),                   # unknown precision
    ]
    for c in cases:
        a = dict(lmin=2, lmax=10, nk=4, ntau=8, nsrc=1, prec=0)
        a.update(c)
        rc = lib.los_project(ctx, a["lmin"], a["lmax"], a["nk"], a["ntau"], 1.0, p, p, p, p,
                             a["nsrc"], a["prec"], p, None)
        assert rc == 1, (c, rc, lib.los_last_error())
    rc = lib.los_project(ctx, 2, 10, 4, 8, 1.0, p, None, p, p, 1, 0, p, None)
    assert rc == 1 and b"NULL" in lib.los_last_error()


def test_project_kernels_validation(lib):
    ctx, _keep = _dummy_ctx()
    p = ctypes.c_void_p(16)
    # a kernel-mask bit for a source that does not exist
    assert lib.los_project_kernels(ctx, 2, 10, 4, 8, 1.0, p, p, p, p, 2, 0b100, 0, p, None) == 1
    assert b"mask" in lib.los_last_error()
    # the E-mode kernel is FP64 only
    assert lib.los_project_kernels(ctx, 2, 10, 4, 8, 1.0, p, p, p, p, 2, 0b10, 2, p, None) == 4


def test_project_tensor_validation(lib):
    ctx, _keep = _dummy_ctx()
    p = ctypes.c_void_p(16)
    assert lib.los_project_tensor(None, 2, 10, 4, 8, 1.0, p, p, p, p, p, None) == 1
    for lmin, lmax, nk, ntau in [(1, 10, 4, 8), (10, 9, 4, 8), (2, 20000, 4, 8), (2, 10, 0, 8),
                                 (2, 10, 4, 0), (2, 10, 4, 9000)]:
        rc = lib.los_project_tensor(ctx, lmin, lmax, nk, ntau, 1.0, p, p, p, p, p, None)
        assert rc == 1, (lmin, lmax, nk, ntau, lib.los_last_error())
    assert lib.los_project_tensor(ctx, 2, 10, 4, 8, 1.0, p, p, p, None, p, None) == 1
    assert b"NULL" in lib.los_last_error()
    assert lib.los_project_tensor(ctx, 2, 10, 4, 8, float("nan"), p, p, p, p, p, None) == 1


def test_cl_noalloc_validation(lib):
    ctx, _keep = _dummy_ctx()
    p = ctypes.c_void_p(16)
    pairs = (ctypes.c_int32 * 2)(0, 0)
    assert lib.cl_integrate_noalloc(None, p, 0, 1, 10, 4, p, p, pairs, 1, p, None) == 1
    assert b"ctx" in lib.los_last_error()
    assert lib.cl_integrate_noalloc(ctx, p, 0, 0, 10, 4, p, p, pairs, 1, p, None) == 1  # nsrc = 0
    assert lib.cl_integrate_noalloc(ctx, None, 0, 1, 10, 4, p, p, pairs, 1, p, None) == 1
    # 16 pairs at 16000 multipoles need more partial sums than the fixed scratch holds
    many = (ctypes.c_int32 * 32)(*([0, 0] * 16))
    assert lib.cl_integrate_noalloc(ctx, p, 0, 1, 16000, 20, p, p, many, 16, p, None) == 1
    assert b"scratch" in lib.los_last_error()


def test_cl_and_table_validation(lib):
    ctx, _keep = _dummy_ctx()
    p = ctypes.c_void_p(16)
    pairs = (ctypes.c_int32 * 2)(0, 3)
    assert lib.cl_integrate(ctx, p, 0, 2, 10, 4, p, p, pairs, 1, p, None) == 1  # index 3 >= nsrc
    pairs = (ctypes.c_int32 * 2)(0, 0)
    assert lib.cl_integrate(ctx, p, 0, 0, 10, 4, p, p, pairs, 1, p, None) == 1  # nsrc = 0
    assert lib.cl_integrate(ctx, p, 0, 1, 10, 4, p, p, pairs, 17, p, None) == 1  # npairs > 16
    assert lib.cl_integrate(ctx, p, 9, 1, 10, 4, p, p, pairs, 1, p, None) == 1  # bad delta prec
    assert lib.los_bessel_table(ctx, p, 5, 4, 3, p, None) == 1                   # lmax < lmin
    assert lib.los_bessel_table(ctx, p, -1, 0, 3, p, None) == 1                  # nx < 0
    assert lib.los_bessel_table(ctx, None, 0, 0, 3, None, None) == 0             # nx == 0: no-op


def test_spline_validation(lib):
    ctx, _keep = _dummy_ctx()
    p = ctypes.c_void_p(16)
    m = ctypes.c_void_p(32)
    sp, ip = lib.los_spline_sources, lib.los_interp_sources
    assert sp(ctx, 1, 1, 8, p, p, m, None) == 1           # nkc < 2
    assert sp(ctx, 1, 2 + 16 * 1024 + 1, 8, p, p, m, None) == 1  # nkc too large
    assert sp(ctx, 0, 10, 8, p, p, m, None) == 1          # nsrc = 0
    assert sp(ctx, 65, 10, 8, p, p, m, None) == 1         # nsrc > 64
    assert sp(ctx, 1, 10, 0, p, p, m, None) == 1          # ntau = 0
    assert sp(ctx, 1, 10, 8, p, p, p, None) == 1          # M aliases Sc
    assert b"alias" in lib.los_last_error()
    assert sp(ctx, 1, 10, 8, None, p, m, None) == 1       # NULL q
    s = ctypes.c_void_p(48)
    assert ip(ctx, 1, 10, 8, p, p, m, 4, p, 7, s, None) == 1   # bad out_prec
    assert ip(ctx, 1, 10, 8, p, p, m, -1, p, 0, s, None) == 1  # nk < 0
    assert ip(ctx, 1, 10, 8, p, p, m, 4, p, 0, m, None) == 1   # S aliases M
    assert ip(ctx, 1, 10, 8, p, p, m, 0, None, 0, None, None) == 0  # nk == 0: no-op
    assert sp(None, 1, 10, 8, p, p, m, None) == 1


def test_lsample_validation(lib):
    ctx, _keep = _dummy_ctx()
    p = ctypes.c_void_p(16)
    d = ctypes.c_void_p(64)
    ls = (ctypes.c_int32 * 3)(2, 5, 9)
    f = lib.los_project_lsample
    bad = (ctypes.c_int32 * 3)(2, 5, 5)
    assert f(ctx, 2, 9, bad, 3, 4, 8, 1.0, p, p, p, p, 1, 0, d, None) == 1       # not increasing
    out = (ctypes.c_int32 * 2)(2, 12)
    assert f(ctx, 2, 9, out, 2, 4, 8, 1.0, p, p, p, p, 1, 0, d, None) == 1       # beyond lmax
    assert f(ctx, 2, 9, ls, 0, 4, 8, 1.0, p, p, p, p, 1, 0, d, None) == 1        # nls = 0
    assert f(ctx, 2, 9, ls, 3, 4, 8, 1.0, p, p, p, p, 1, 0b10, d, None) == 1     # mask bit >= nsrc
    ci = lib.los_cl_interp
    assert ci(ctx, 2, ls, 3, p, 2, 10, d, None) == 1      # last sample != lmax
    assert ci(ctx, 2, ls, 3, p, 3, 9, d, None) == 1       # first sample != lmin
    assert ci(ctx, 2, ls, 3, p, 2, 9, p, None) == 1       # cl aliases cls
    assert ci(ctx, 0, ls, 3, p, 2, 9, d, None) == 1       # npairs = 0
    assert ci(None, 2, ls, 3, p, 2, 9, d, None) == 1


def test_emu_spectra_validation(lib):
    """The per-spectrum inference and merge reject bad arguments before any device work."""
    p = ctypes.c_void_p(16)
    assert lib.emu_infer_spectra(None, p, 4, p, p, p, 1e-3, None) == 1
    rows = (ctypes.c_int64 * 2)(0, 1)
    assert lib.emu_merge_spectrum(None, 0, rows, 2, p, p, 4, None, None, None) == 1
    emu, _keep = _dummy_ctx()   # validation runs before the handle is used
    assert lib.emu_merge_spectrum(emu, 4, rows, 2, p, p, 4, None, None, None) == 1  # no 5th spectrum
    assert lib.emu_merge_spectrum(emu, -1, rows, 2, p, p, 4, None, None, None) == 1
    assert lib.emu_merge_spectrum(emu, 0, rows, 3, p, p, 2, None, None, None) == 1  # nf > n
    bad = (ctypes.c_int64 * 2)(1, 1)
    assert lib.emu_merge_spectrum(emu, 0, bad, 2, p, p, 4, None, None, None) == 1
    assert b"twice" in lib.los_last_error()
    out = (ctypes.c_int64 * 2)(0, 7)
    assert lib.emu_merge_spectrum(emu, 0, out, 2, p, p, 4, None, None, None) == 1
    assert lib.emu_merge_spectrum(emu, 0, rows, 0, None, None, 4, None, None, None) == 0  # no-op
