"""The C-ABI library loads and exports what include/rnnls.h declares; host-side
argument checks (no device work: these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_0812_4547_amd import rnnls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rnnls.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rnnls_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rnnls.LIB_PATH):
        from paper_0812_4547_amd import build
        build.build()
    return rnnls.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("rnnls_srht_sketch", "rnnls_nnls_solve", "rnnls_rand_nnls",
                 "rnnls_workspace_bytes"):
        assert want in names
    assert set(names) == set(rnnls.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version(lib):
    assert lib.rnnls_version() == 10000


def _sketch(lib, n=4096, d=4, r=100, A=1, lda=4096, b=None, SA=1, ldsa=100, Sb=None, opts=None):
    o = opts if opts is not None else rnnls.Opts()
    return lib.rnnls_srht_sketch(n, d, r, 1, A, lda, b, SA, ldsa, Sb, None, None, None, None,
                                 ctypes.byref(o), None, 0, None)


def test_sketch_argument_checks(lib):
    assert _sketch(lib, n=1) == -1
    assert _sketch(lib, n=(1 << 30) + 1) == -1
    assert _sketch(lib, d=0) == -2
    assert _sketch(lib, d=rnnls.MAX_D_SOLVE + 1) == -2
    assert _sketch(lib, r=0) == -3
    assert _sketch(lib, n=3000, r=4096) == -3          # r must be < n' = 4096
    assert _sketch(lib, r=rnnls.MAX_R + 1, n=1 << 20, lda=1 << 20) == -3
    assert _sketch(lib, A=None) == -5
    assert _sketch(lib, lda=4095) == -6
    assert _sketch(lib, SA=None) == -8
    assert _sketch(lib, ldsa=99) == -9
    assert _sketch(lib, b=1, Sb=None) == -10
    assert _sketch(lib, opts=rnnls.Opts(7, 0, 0, 0, 0.0)) == -15
    assert _sketch(lib, opts=rnnls.Opts(0, 2, 0, 0, 0.0)) == -15       # unknown precision


def test_solve_argument_checks(lib):
    o = rnnls.Opts()

    def solve(m=10, d=3, M=1, ldm=10, f=1, x=1):
        return lib.rnnls_nnls_solve(m, d, M, ldm, f, None, x, None, None, None, None,
                                    ctypes.byref(o), None, 0, None)
    assert solve(m=0) == -1
    assert solve(d=0) == -2
    assert solve(d=rnnls.MAX_D_SOLVE + 1) == -2
    assert solve(M=None) == -3
    assert solve(ldm=9) == -4
    assert solve(f=None) == -5
    assert solve(x=None) == -7


def test_rand_nnls_argument_checks(lib):
    o = rnnls.Opts()

    def run(n=4096, d=4, r=100, A=1, lda=4096, b=1, x=1, SA=None, ldsa=0):
        return lib.rnnls_rand_nnls(n, d, r, 3, A, lda, b, x, None, None, None, SA, ldsa, None,
                                   None, None, ctypes.byref(o), None, 0, None)
    assert run(n=1) == -1
    assert run(d=rnnls.MAX_D_SOLVE + 1) == -2
    assert run(r=4096) == -3
    assert run(A=None) == -5
    assert run(lda=10) == -6
    assert run(b=None) == -7
    assert run(x=None) == -8
    assert run(SA=1, ldsa=50) == -13


def test_stream_read_argument_checks(lib):
    # rejected before any device work
    assert lib.rnnls_stream_read(None, -1, 16, None) == -1
    assert lib.rnnls_stream_read(None, 8, 16, None) == -1          # NULL x with n > 0
    assert lib.rnnls_stream_read(16, 8, None, None) == -1          # NULL partials
    assert lib.rnnls_stream_read(20, 8, 16, None) == -1            # x not 16-byte aligned


def test_rand_nnls_boost_argument_checks(lib):
    o = rnnls.Opts()

    def run(n=4096, d=4, r=100, k=3, A=1, lda=4096, b=1, x=1):
        return lib.rnnls_rand_nnls_boost(n, d, r, k, 3, A, lda, b, x, None, None, None,
                                         ctypes.byref(o), None, 0, None)
    assert run(n=1) == -1
    assert run(d=rnnls.MAX_D_SOLVE + 1) == -2
    assert run(r=4096) == -3
    assert run(k=0) == -4
    assert run(k=rnnls.MAX_BOOST + 1) == -4
    assert run(A=None) == -6
    assert run(lda=10) == -7
    assert run(b=None) == -8
    assert run(x=None) == -9


def test_rand_box_argument_checks(lib):
    o = rnnls.Opts()

    def run(n=4096, d=4, r=100, A=1, lda=4096, b=1, lo=1, hi=1, x=1):
        return lib.rnnls_rand_box(n, d, r, 3, A, lda, b, lo, hi, x, None, None, None,
                                  ctypes.byref(o), None, 0, None)
    assert run(n=1) == -1
    assert run(d=0) == -2
    assert run(d=rnnls.MAX_BOX_D + 1) == -2
    assert run(r=4096) == -3
    assert run(A=None) == -5
    assert run(lda=10) == -6
    assert run(b=None) == -7
    assert run(lo=None) == -8
    assert run(hi=None) == -9
    assert run(x=None) == -10


def test_tuning_cache_save_and_load(lib, tmp_path):
    """The autotuner's cache: a file of entries merges in, is written back
    identically, a malformed file merges nothing (no device work)."""
    rnnls.tuning_cache_clear()
    assert rnnls.tuning_cache_entries() == 0
    src = tmp_path / "tune.txt"
    src.write_text("00000000000000ab 14 2\n0123456789abcdef 13 4\n")
    rnnls.tuning_cache_load(str(src))
    assert rnnls.tuning_cache_entries() == 2
    out = tmp_path / "out.txt"
    rnnls.tuning_cache_save(str(out))
    assert out.read_text() == src.read_text()
    bad = tmp_path / "bad.txt"
    bad.write_text("00000000000000cd 14 2\nnot a line\n")
    with pytest.raises(rnnls.RnnlsError):
        rnnls.tuning_cache_load(str(bad))
    odd = tmp_path / "odd.txt"
    odd.write_text("00000000000000ce 11 3\n")  # not a tile shape the autotuner tries
    with pytest.raises(rnnls.RnnlsError):
        rnnls.tuning_cache_load(str(odd))
    assert rnnls.tuning_cache_entries() == 2
    with pytest.raises(rnnls.RnnlsError):
        rnnls.tuning_cache_load(str(tmp_path / "missing.txt"))
    assert lib.rnnls_tuning_cache_save(None) == -1
    rnnls.tuning_cache_clear()
    assert rnnls.tuning_cache_entries() == 0
