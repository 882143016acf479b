"""Host-side checks of the C ABI library (no GPU needed).

The library must load, export every function declared in include/ifsvgp.h,
and its host-only Gauss-Hermite rule must agree with the textbook rule
(numpy's hermgauss, Golub-Welsch).
"""
import os
import re
import subprocess

import numpy as np
import pytest
from numpy.polynomial.hermite import hermgauss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ifsvgp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ifsvgp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2604_00697_amd import lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2604_00697_amd import build
        build.build()
    return L


def test_header_declares_the_binding_surface(lib):
    assert declared_functions() == lib.EXPORTED


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ifsvgp_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    lib.load()  # every declared symbol resolves through ctypes


def test_version_and_strerror(lib):
    L = lib.load()
    assert L.ifsvgp_version() >= 100
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert len(lib.strerror(code)) > 0
    assert lib.strerror(-99) == "unknown status code"


@pytest.mark.parametrize("n", [1, 2, 3, 5, 10, 20, 21, 40, 64])
def test_gh_rule_matches_golub_welsch(lib, n):
    t, w = lib.gh_rule(n)
    tr, wr = hermgauss(n)
    assert np.allclose(t, tr, rtol=0, atol=1e-12)
    assert np.allclose(w, wr, rtol=1e-10, atol=1e-300)


def test_gh_rule_rejects_bad_sizes(lib):
    for n in (0, -1, 65):
        with pytest.raises(lib.IFSVGPError) as e:
            lib.gh_rule(n)
        assert e.value.code == lib.EINVAL


def test_create_rejects_bad_arguments_before_touching_the_device(lib):
    import ctypes
    L = lib.load()
    h = ctypes.c_void_p()
    for args in [(0, 10, 2, 0, 0, 20), (10, 0, 2, 0, 0, 20), (10, 10, 0, 0, 0, 20),
                 (10, 10, 65, 0, 0, 20), (10, 10, 2, 3, 0, 20), (10, 10, 2, 0, 2, 20),
                 (10, 10, 2, 0, 1, 0), (10, 10, 2, 0, 1, 65),
                 # the size limits: M, B_max and M * B_max
                 (32769, 10, 2, 0, 0, 20), (10, (1 << 24) + 1, 2, 0, 0, 20),
                 (32768, (1 << 16) + 1, 2, 0, 0, 20)]:
        assert L.ifsvgp_create(ctypes.byref(h), *args) == lib.EINVAL
    assert L.ifsvgp_natgrad(None, None, None, None, None, None, None, 1, None) == lib.EINVAL
    assert L.ifsvgp_status(None) == lib.EINVAL


def test_product_path_does_not_import_the_oracle():
    """The binding and autograd modules never reference the oracle package."""
    pkg = os.path.join(ROOT, "paper_2604_00697_amd")
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle|from\s+\.\.\s*import\s+oracle)"
                     r"|#include\s*[<\"].*oracle", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not pat.search(src), f
                assert "importlib" not in src, f
