"""The closed forms of the ccvv and cavv residual rows (oracle/ccvv_closed.py,
oracle/cavv_closed.py: Eq. 10 with a diagonal Fock operator) against the
factorised oracle on every row of those blocks in small problems, and against
properties that fix them on their own:

* every ccvv and cavv row of O2's packed residual (with and without the
  source, every state L, MS-MR with XMS), element by element at 1e-12 of the
  largest, and the source alone (x = 0) at 1e-12 of its largest element;
* the row index of a representative (pair(i, j) * pairs_v + pair(a, b)) is
  O2's storage order;
* the XMS energies recomputed from occupation numbers are O2's E_L^(0);
* for a generic representative the metric eigenvalues are 4 ('+') and
  12 ('-'): without source, sigma / (gap * t) is 4 and 12.

CPU only."""
import numpy as np
import pytest

from synth.gen import make_problem
from oracle.ic import Caspt2Oracle
from oracle.aavv_closed import aavv_rows
from oracle.cavv_closed import cavv_rows, xms_states_diagonal_f
from oracle.ccav_closed import ccav_rows
from oracle.ccvv_closed import ccvv_pair_index, ccvv_rows, xms_energies_diagonal_f

CASES = [((3, 2, 5, 30, 2), 1), ((2, 3, 4, 30, 3), 2), ((4, 0, 6, 30, 1), 3), ((1, 2, 3, 20, 1), 4)]


def _reps(nc, nv, minus):
    out = []
    for i in range(nc):
        for j in range(i if minus else i + 1):
            for a in range(nv):
                for b in range(a if minus else a + 1):
                    out.append((i, j, a, b))
    return out


@pytest.mark.parametrize("dims,seed", CASES)
def test_closed_form_matches_factorised_oracle(dims, seed):
    p = make_problem(*dims, seed=seed, reading="A", shift=0.2)
    o = Caspt2Oracle(p, "MSMR")
    np.testing.assert_allclose(xms_energies_diagonal_f(p), o.e0, atol=1e-13)
    ents = {(e["block"].name, e["chi"]): e for e in o.layout}
    ep, em = ents[("ccvv", (1, 1))], ents[("ccvv", (-1, -1))]
    nst = p.nst
    reps_p, reps_m = _reps(p.nc, p.nv, False), _reps(p.nc, p.nv, True)
    assert [tuple(r) for r in ep["reps"]] == reps_p
    assert [tuple(r) for r in em["reps"]] == reps_m
    npv_p, npv_m = p.nv * (p.nv + 1) // 2, p.nv * (p.nv - 1) // 2
    for r, (i, j, a, b) in enumerate(reps_p):
        assert ccvv_pair_index(i, j, False) * npv_p + ccvv_pair_index(a, b, False) == r
    for r, (i, j, a, b) in enumerate(reps_m):
        assert ccvv_pair_index(i, j, True) * npv_m + ccvv_pair_index(a, b, True) == r
    x = np.random.default_rng(seed + 10).standard_normal(o.length)
    xp = x[ep["offset"]: ep["offset"] + ep["nrow"] * nst].reshape(-1, nst)
    xm = x[em["offset"]: em["offset"] + em["nrow"] * nst].reshape(-1, nst)
    t_minus = []
    for (i, j, a, b) in reps_p:
        if i > j and a > b:
            t_minus.append(xm[ccvv_pair_index(i, j, True) * npv_m + ccvv_pair_index(a, b, True)])
        else:
            t_minus.append(None)
    zero = np.zeros_like(x)
    for xv, src in ((x, True), (x, False), (zero, True)):
        for L in range(nst):
            sig = o.residual(L, xv, with_source=src)
            ref_p = sig[ep["offset"]: ep["offset"] + ep["nrow"] * nst].reshape(-1, nst)
            ref_m = sig[em["offset"]: em["offset"] + em["nrow"] * nst].reshape(-1, nst)
            if xv is zero:
                got_p, got_m = ccvv_rows(p, L, reps_p, np.zeros_like(xp),
                                         [None if t is None else 0.0 * t for t in t_minus], with_source=True)
            else:
                got_p, got_m = ccvv_rows(p, L, reps_p, xp, t_minus, with_source=src)
            scale = max(np.abs(ref_p).max(), np.abs(ref_m).max() if ref_m.size else 0.0)
            assert np.abs(got_p - ref_p).max() <= 1e-12 * scale
            sel = [k for k, (i, j, a, b) in enumerate(reps_p) if i > j and a > b]
            assert len(sel) == len(reps_m)
            if sel:
                assert np.abs(got_m[sel] - ref_m).max() <= 1e-12 * scale
                assert np.all(np.isnan(np.delete(got_m, sel, axis=0)))


def test_generic_metric_eigenvalues():
    p = make_problem(3, 2, 5, 30, 2, seed=5, reading="A", shift=0.3)
    E = xms_energies_diagonal_f(p)
    i, j, a, b = 2, 0, 4, 1
    t = np.array([[1.0, -0.5]])
    sp, sm = ccvv_rows(p, 1, [(i, j, a, b)], t, [2.0 * t[0]], with_source=False)
    v0 = p.nc + p.na
    gap = p.eps[v0 + a] + p.eps[v0 + b] - p.eps[i] - p.eps[j] + p.shift - E[1] + E
    np.testing.assert_allclose(sp[0], 4.0 * gap * t[0], rtol=1e-14)
    np.testing.assert_allclose(sm[0], 12.0 * gap * 2.0 * t[0], rtol=1e-14)


CAVV_CASES = [((3, 2, 5, 30, 2), 1), ((2, 3, 4, 30, 3), 2), ((1, 4, 3, 20, 2), 4), ((2, 1, 4, 20, 1), 5)]


@pytest.mark.parametrize("dims,seed", CAVV_CASES)
def test_cavv_closed_form_matches_factorised_oracle(dims, seed):
    p = make_problem(*dims, seed=seed, reading="A", shift=0.2)
    o = Caspt2Oracle(p, "MSMR")
    ci, E, _ = xms_states_diagonal_f(p)
    np.testing.assert_allclose(E, o.e0, atol=1e-13)
    np.testing.assert_allclose(ci, o.ci, atol=1e-13)
    ents = {(e["block"].name, e["chi"]): e for e in o.layout}
    ep, em = ents[("cavv", (1,))], ents[("cavv", (-1,))]
    n = ep["nalpha"]
    assert n == p.nst * p.na
    reps_p = [(i, a, b) for i in range(p.nc) for a in range(p.nv) for b in range(a + 1)]
    reps_m = [(i, a, b) for i in range(p.nc) for a in range(p.nv) for b in range(a)]
    assert [tuple(r) for r in ep["reps"]] == reps_p
    assert [tuple(r) for r in em["reps"]] == reps_m
    npv_p, npv_m = p.nv * (p.nv + 1) // 2, p.nv * (p.nv - 1) // 2
    for r, (i, a, b) in enumerate(reps_p):
        assert i * npv_p + ccvv_pair_index(a, b, False) == r
    for r, (i, a, b) in enumerate(reps_m):
        assert i * npv_m + ccvv_pair_index(a, b, True) == r
    x = np.random.default_rng(seed + 20).standard_normal(o.length)
    xp = x[ep["offset"]: ep["offset"] + ep["nrow"] * n].reshape(-1, n)
    xm = x[em["offset"]: em["offset"] + em["nrow"] * n].reshape(-1, n)
    tm = [xm[i * npv_m + ccvv_pair_index(a, b, True)] if a > b else None for (i, a, b) in reps_p]
    sel = [k for k, (i, a, b) in enumerate(reps_p) if a > b]
    zero = np.zeros_like(x)
    dens = None
    for xv, src in ((x, True), (x, False), (zero, True)):
        for L in range(p.nst):
            sig = o.residual(L, xv, with_source=src)
            ref_p = sig[ep["offset"]: ep["offset"] + ep["nrow"] * n].reshape(-1, n)
            ref_m = sig[em["offset"]: em["offset"] + em["nrow"] * n].reshape(-1, n)
            if xv is zero:
                got_p, got_m, dens = cavv_rows(p, L, reps_p, np.zeros_like(xp),
                                               [None if t is None else 0.0 * t for t in tm],
                                               with_source=True, dens=dens)
            else:
                got_p, got_m, dens = cavv_rows(p, L, reps_p, xp, tm, with_source=src, dens=dens)
            scale = max(np.abs(ref_p).max(), np.abs(ref_m).max() if ref_m.size else 0.0)
            assert scale > 0.0
            assert np.abs(got_p - ref_p).max() <= 1e-12 * scale
            if sel:
                assert np.abs(got_m[sel] - ref_m).max() <= 1e-12 * scale
            assert np.all(np.isnan(np.delete(got_m, sel, axis=0)))


AAVV_CASES = [((2, 2, 5, 30, 2), 1), ((1, 3, 4, 30, 3), 2), ((2, 4, 3, 20, 2), 4), ((1, 2, 4, 20, 1), 6)]


@pytest.mark.parametrize("dims,seed", AAVV_CASES)
def test_aavv_closed_form_matches_factorised_oracle(dims, seed):
    p = make_problem(*dims, seed=seed, reading="A", shift=0.2)
    o = Caspt2Oracle(p, "MSMR")
    ents = {(e["block"].name, e["chi"]): e for e in o.layout}
    ep, em = ents[("aavv", (1,))], ents[("aavv", (-1,))]
    n = ep["nalpha"]
    assert n == p.nst * p.na * p.na
    reps_p = [(a, b) for a in range(p.nv) for b in range(a + 1)]
    reps_m = [(a, b) for a in range(p.nv) for b in range(a)]
    assert [tuple(r) for r in ep["reps"]] == reps_p
    assert [tuple(r) for r in em["reps"]] == reps_m
    for r, (a, b) in enumerate(reps_p):
        assert ccvv_pair_index(a, b, False) == r
    for r, (a, b) in enumerate(reps_m):
        assert ccvv_pair_index(a, b, True) == r
    x = np.random.default_rng(seed + 30).standard_normal(o.length)
    sel = [k for k, (a, b) in enumerate(reps_p) if a > b]
    prods = None
    for xv, src in ((x, True), (x, False), (np.zeros_like(x), True)):
        xp = xv[ep["offset"]: ep["offset"] + ep["nrow"] * n].reshape(-1, n)
        xm = xv[em["offset"]: em["offset"] + em["nrow"] * n].reshape(-1, n)
        tm = [xm[ccvv_pair_index(a, b, True)] if a > b else None for (a, b) in reps_p]
        for L in range(p.nst):
            sig = o.residual(L, xv, with_source=src)
            ref_p = sig[ep["offset"]: ep["offset"] + ep["nrow"] * n].reshape(-1, n)
            ref_m = sig[em["offset"]: em["offset"] + em["nrow"] * n].reshape(-1, n)
            got_p, got_m, prods = aavv_rows(p, L, reps_p, xp, tm, with_source=src, prods=prods)
            scale = max(np.abs(ref_p).max(), np.abs(ref_m).max() if ref_m.size else 0.0)
            assert scale > 0.0
            assert np.abs(got_p - ref_p).max() <= 1e-12 * scale
            if sel:
                assert np.abs(got_m[sel] - ref_m).max() <= 1e-12 * scale
            assert np.all(np.isnan(np.delete(got_m, sel, axis=0)))


CCAV_CASES = [((3, 2, 5, 30, 2), 1), ((3, 3, 4, 30, 3), 2), ((2, 4, 3, 20, 2), 4), ((2, 1, 3, 20, 1), 7)]


@pytest.mark.parametrize("dims,seed", CCAV_CASES)
def test_ccav_closed_form_matches_factorised_oracle(dims, seed):
    p = make_problem(*dims, seed=seed, reading="A", shift=0.2)
    o = Caspt2Oracle(p, "MSMR")
    ents = {(e["block"].name, e["chi"]): e for e in o.layout}
    ep, em = ents[("ccav", (1,))], ents[("ccav", (-1,))]
    n = ep["nalpha"]
    assert n == p.nst * p.na
    reps_p = [(i, j, a) for i in range(p.nc) for j in range(i + 1) for a in range(p.nv)]
    reps_m = [(i, j, a) for i in range(p.nc) for j in range(i) for a in range(p.nv)]
    assert [tuple(r) for r in ep["reps"]] == reps_p
    assert [tuple(r) for r in em["reps"]] == reps_m
    for r, (i, j, a) in enumerate(reps_p):
        assert ccvv_pair_index(i, j, False) * p.nv + a == r
    for r, (i, j, a) in enumerate(reps_m):
        assert ccvv_pair_index(i, j, True) * p.nv + a == r
    x = np.random.default_rng(seed + 40).standard_normal(o.length)
    sel = [k for k, (i, j, a) in enumerate(reps_p) if i > j]
    dens = None
    for xv, src in ((x, True), (x, False), (np.zeros_like(x), True)):
        xp = xv[ep["offset"]: ep["offset"] + ep["nrow"] * n].reshape(-1, n)
        xm = xv[em["offset"]: em["offset"] + em["nrow"] * n].reshape(-1, n)
        tm = [xm[ccvv_pair_index(i, j, True) * p.nv + a] if i > j else None for (i, j, a) in reps_p]
        for L in range(p.nst):
            sig = o.residual(L, xv, with_source=src)
            ref_p = sig[ep["offset"]: ep["offset"] + ep["nrow"] * n].reshape(-1, n)
            ref_m = sig[em["offset"]: em["offset"] + em["nrow"] * n].reshape(-1, n)
            got_p, got_m, dens = ccav_rows(p, L, reps_p, xp, tm, with_source=src, dens=dens)
            scale = max(np.abs(ref_p).max(), np.abs(ref_m).max() if ref_m.size else 0.0)
            assert scale > 0.0
            assert np.abs(got_p - ref_p).max() <= 1e-12 * scale
            if sel:
                assert np.abs(got_m[sel] - ref_m).max() <= 1e-12 * scale
            assert np.all(np.isnan(np.delete(got_m, sel, axis=0)))
