"""The C-ABI libraries load and export every function declared in
include/dfa_spec.h (GPU library) and include/dfa_host.h (host multicore
matcher); no GPU compute call is made, so this runs without a GPU."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "dfa_spec.h")
HOST_HEADER = os.path.join(ROOT, "include", "dfa_host.h")


def declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(dfa_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def libdfa():
    import paper_1210_5093_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1210_5093_amd import build
        build.build()
    return pkg.lib()


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ("dfa_create", "dfa_match", "dfa_match_async", "dfa_match_batch", "dfa_info",
              "dfa_destroy", "dfa_strerror"):
        assert f in fns


def test_library_exports_every_declared_symbol(libdfa):
    missing = [f for f in declared_functions() if not hasattr(libdfa, f)]
    assert not missing, missing


def test_strerror_without_gpu(libdfa):
    libdfa.dfa_strerror.restype = ctypes.c_char_p
    assert libdfa.dfa_strerror(-4) == b"input byte outside the alphabet"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_1210_5093_amd as pkg
    monkeypatch.setattr(pkg, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pkg, "_lib", None)
    with pytest.raises(RuntimeError):
        pkg.lib()


def test_host_library_exports_every_declared_symbol():
    from paper_1210_5093_amd import host
    if not os.path.exists(host.HOST_LIB_PATH):
        from paper_1210_5093_amd import build
        build.build_host()
    L = host.lib()
    fns = declared_functions(HOST_HEADER)
    assert "dfa_host_match" in fns and "dfa_host_partition" in fns
    missing = [f for f in fns if not hasattr(L, f)]
    assert not missing, missing
