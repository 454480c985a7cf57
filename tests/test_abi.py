"""The C-ABI library loads and exports every function include/gmm.h
declares; host-side argument checks run without a GPU."""
import ctypes
import os
import re

import pytest

from paper_2307_00071_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gmm_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2307_00071_amd import build
        build.build()
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.EXPORTS, name


def test_status_strings(lib):
    for code in range(7):
        s = lib.gmm_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.gmm_status_string(99).decode() == "unknown status"


def test_host_side_argument_errors(lib):
    opts = _lib.FitOpts(5, 1e-3, 0, 0)
    # n <= 0, k <= 0, k > n, k above the limit: rejected before any HIP call
    for n, k, want in ((0, 1, 1), (10, 0, 1), (10, 11, 1), (5000, 2000, 6)):
        st = lib.gmm_fit(None, n, k, None, None, None, None, None,
                         ctypes.byref(opts), None, 0, None)
        assert st == want, (n, k, st)
        assert lib.gmm_last_error().decode()
    st = lib.gmm_loglik(None, -3, None, 2, None, None, None, None, None, None, 0, None)
    assert st == 1
    # profiling repeats outside [0, 64]; 0 (off) is accepted
    assert lib.gmm_profile_enable(-1) == 1
    assert lib.gmm_profile_enable(65) == 1
    assert lib.gmm_profile_enable(0) == 0
    with pytest.raises(_lib.GmmError):
        _lib.check(1)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


def test_kmeanspp_host_checks(lib):
    """Sizes and NULL pointers are rejected on the host, before any
    device work is enqueued."""
    assert lib.gmm_kmeanspp_workspace_size(0, 1) == 0
    assert lib.gmm_kmeanspp_workspace_size(10, 11) == 0
    assert lib.gmm_kmeanspp_workspace_size(10, 0) == 0
    assert lib.gmm_kmeanspp_workspace_size(1000, 10) > 8000
    st = lib.gmm_kmeanspp(None, 100, 4, None, None, None, None, 0, None)
    assert st == 1
    st = lib.gmm_kmeanspp(None, 3, 4, None, None, None, None, 0, None)
    assert st == 1
