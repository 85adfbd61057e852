"""The library's host engine (block definitions of Eq. 8 and the Wick
pairings of the external operators on the closed-shell core) against the
oracle's own enumeration: every pairing of <bra| E_xy |ket> and of the
overlap, for all pairs of blocks, operator types and orbital classes of x
and y, with its coefficient and active strings per spin assignment.

The engine is compiled for the CPU with g++ (it holds no device code); the
oracle side is plain Python.  They share no code."""
import itertools
import shutil
import subprocess
from pathlib import Path

import pytest

from oracle.ic import ACT, BLOCKS, CLO, VIR, E, Op, matrix_element_terms

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_1606_01273_amd" / "csrc"


def _engine_lines(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "engine_pairings"
    subprocess.run([gxx, "-std=c++17", "-O1", f"-I{CSRC}", str(CSRC / "engine.cpp"),
                    str(ROOT / "tests" / "host" / "engine_pairings.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return sorted(out.splitlines())


def _act(lst):
    return "".join(f"{o.kind}:{o.label}:{s};" for (o, s) in lst)


def _oracle_lines():
    lines = []
    suffix = lambda ops, s: [Op(o.kind, o.label + s, o.space, o.spin + s) for o in ops]
    comps = [("S", None)] + [(cx + cy, E("x_o", cx, "y_o", cy, "so"))
                             for cx, cy in itertools.product((CLO, ACT, VIR), repeat=2)]
    for bb in BLOCKS:
        for kb in BLOCKS:
            for tag, op in comps:
                for (tb, tmb), (tk, tmk) in itertools.product(enumerate(bb.types), enumerate(kb.types)):
                    terms = matrix_element_terms(suffix(tmb, "_b"), op or [], suffix(tmk, "_k"))
                    for classes, entries in terms.items():
                        pk = "".join(p + "," for p in sorted("=".join(sorted(c)) for c in classes))
                        for (coeff, ba, ma, ka) in entries:
                            lines.append(f"{bb.name} {kb.name} {tag} {tb} {tk}|{pk}|{coeff:.12g}|"
                                         f"{_act(ba)}|{_act(ma)}|{_act(ka)}")
    return sorted(lines)


def test_engine_pairings_match_oracle(tmp_path):
    eng = _engine_lines(tmp_path)
    ora = _oracle_lines()
    assert len(eng) > 500
    missing = sorted(set(ora) - set(eng))[:5]
    extra = sorted(set(eng) - set(ora))[:5]
    assert eng == ora, f"oracle-only: {missing}; engine-only: {extra}"


def test_within_block_term_forms(tmp_path):
    """Classification of the coupling terms of a block with itself (Fock
    elements inside the closed or the virtual space): which run as a GEMM
    along one slot, with which permutation of the ket slots, and which
    permutations leave the amplitude tensor unchanged."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "slot_forms"
    subprocess.run([gxx, "-std=c++17", "-O1", f"-I{CSRC}", str(CSRC / "engine.cpp"),
                    str(ROOT / "tests" / "host" / "slot_forms.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "ok"

