"""The C-ABI library loads and exports every entry point include/tk.h declares
(no compute: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1906_01211_amd", "libtk.so")


def declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(tk_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1906_01211_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "tk_nblist_build" in names and "tk_polarize_pcg" in names
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (tk_[a-z0-9_]+)$", out, flags=re.M))
    assert set(names) <= exported


def test_binding_covers_the_header():
    from paper_1906_01211_amd import tk
    assert set(declared()) == set(tk.exported_symbols())


def test_strerror_without_gpu(lib):
    lib.tk_strerror.restype = ctypes.c_char_p
    assert lib.tk_strerror(-2) == b"cutoff exceeds half the box edge"
    assert lib.tk_strerror(0) == b"ok"
