"""The C-ABI library builds, loads, and exports every symbol its headers
declare (no compute call: these run without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1606_01273_amd", "libcaspt2.so")


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        for m in re.finditer(r"CASPT2_API\s+[\w\s\*]+?\b((?:caspt2|xms)_\w+)\s*\(", txt):
            names.add(m.group(1))
    return sorted(names)


def test_headers_declare_the_abi():
    names = declared_symbols()
    for n in ("caspt2_create", "caspt2_residual", "caspt2_solve_amplitudes", "caspt2_solve_lambda",
              "xms_rotate", "xms_heff"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libcaspt2.so not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_abi():
    from paper_1606_01273_amd import _lib
    assert set(declared_symbols()) <= set(_lib.SIGNATURES)
    lib = _lib.load()
    assert lib.caspt2_strerror(-6) == b"not implemented"
