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


def test_many_entry_points_reject_bad_arguments_before_any_device_call():
    """caspt2_create_many and caspt2_residual_all_many check their arguments
    on the host (no device needed): n < 1, nthreads < 1, NULL arrays and a
    repeated handle are E_ARG; the Python helpers accept empty lists."""
    import ctypes
    from paper_1606_01273_amd import _lib, Caspt2, residual_all_many
    lib = _lib.load()
    E_ARG = _lib.E_ARG
    ds = (_lib.Dims * 1)()
    ins = (_lib.Inputs * 1)()
    sp = (ctypes.c_void_p * 1)()
    hs = (ctypes.c_void_p * 1)()
    st = (ctypes.c_int32 * 1)()
    assert lib.caspt2_create_many(0, ds, ins, 0, sp, 1, hs, st) == E_ARG
    assert lib.caspt2_create_many(1, ds, ins, 0, sp, 0, hs, st) == E_ARG
    assert lib.caspt2_create_many(1, None, ins, 0, sp, 1, hs, st) == E_ARG
    assert lib.caspt2_create_many(1, ds, ins, 0, sp, 1, hs, None) == E_ARG
    fake = (ctypes.c_void_p * 2)(0x1000, 0x1000)   # never dereferenced: rejected as repeated
    xp = (ctypes.c_void_p * 2)()
    st2 = (ctypes.c_int32 * 2)()
    assert lib.caspt2_residual_all_many(0, fake, 1, xp, xp, 1, st2) == E_ARG
    assert lib.caspt2_residual_all_many(2, fake, 1, xp, xp, 1, st2) == E_ARG
    assert lib.caspt2_residual_all_many(2, fake, 1, xp, xp, 0, st2) == E_ARG
    nul = (ctypes.c_void_p * 1)()
    assert lib.caspt2_residual_all_many(1, nul, 1, xp, xp, 1, st2) == E_ARG
    assert Caspt2.create_many([]) == []
    assert residual_all_many([], [], []) is None
