"""The C-ABI library loads and exports every entry point declared in include/mpc3.h
(no compute call: these run without a GPU), and the product path never touches the oracle."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpc3.h")
PKG = os.path.join(ROOT, "paper_2411_09287_amd")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(mpc3_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def libpath():
    path = os.path.join(PKG, "libmpc3.so")
    if not os.path.exists(path):
        from paper_2411_09287_amd import build
        build.build()
    return path


def test_header_declares_the_boundary():
    names = declared()
    for must in ["mpc3_ctx_create", "mpc3_share", "mpc3_inner", "mpc3_mult", "mpc3_trunc_pair", "mpc3_trunc",
                 "mpc3_verify", "mpc3_reconstruct", "mpc3_comm_stats", "mpc3_inject", "mpc3_set_variant"]:
        assert must in names


def test_library_exports_every_declared_symbol(libpath):
    L = ctypes.CDLL(libpath)
    for name in declared():
        assert hasattr(L, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2411_09287_amd import mpc3
    assert set(declared()) == set(mpc3.SIGNATURES)


def test_strerror_without_gpu(libpath):
    L = ctypes.CDLL(libpath)
    L.mpc3_strerror.restype = ctypes.c_char_p
    assert L.mpc3_strerror(-4).startswith(b"aborted")


def test_argument_errors_without_gpu(libpath):
    L = ctypes.CDLL(libpath)
    assert L.mpc3_ctx_create(None, 64, 13, 0, None, None) == -1
    assert L.mpc3_set_variant(None, 0) == -1
    assert L.mpc3_inject(None, 1, 0, 0) == -1


def test_product_path_does_not_import_the_oracle():
    pat = re.compile(r"^\s*(from|import)\s+oracle\b", re.M)
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not pat.search(text), f
                assert "oracle." not in text or f.endswith(".md"), f
