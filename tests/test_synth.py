"""The seeded input generator against the recipe it states (synth/gen.py):
orbital energies in their class intervals, sorted; symmetric DF factors with
Frobenius norms exp(-0.05 Q); the Fock operator of each reading (A: the
orbital energies alone; B: the same diagonal with closed-active,
active-virtual and closed-virtual blocks and nothing else off the diagonal;
C: Reading B rotated inside the closed and inside the virtual space, with
h^c and the DF factors rotated by the same matrices and the reference states
unchanged); orthonormal reference states that are the lowest roots of the
active Hamiltonian (Sec. II.A, Eqs. 1-2) in the full Ms = 0 determinant
space; coupling blocks small next to the orbital-energy gaps at every size;
and the same seed drawing the same problem.  CPU only; none of the
perturbation method is involved."""
import math

import numpy as np
import pytest

from synth.gen import make_problem, strings

DIMS = [(3, 4, 9, 40, 2), (5, 2, 13, 50, 1), (2, 6, 7, 45, 3)]


def _slices(p):
    return slice(0, p.nc), slice(p.nc, p.nc + p.na), slice(p.nc + p.na, p.nc + p.na + p.nv)


@pytest.mark.parametrize("dims", DIMS)
def test_orbital_energies_and_df_factors(dims):
    p = make_problem(*dims, seed=3, reading="A")
    clo, act, vir = _slices(p)
    for sl, lo, hi in ((clo, -2.0, -0.5), (act, -0.3, 0.3), (vir, 0.5, 4.0)):
        e = p.eps[sl]
        assert np.all(np.diff(e) >= 0.0)
        assert np.all((e >= lo) & (e <= hi))
    assert np.array_equal(p.B, np.transpose(p.B, (0, 2, 1)))
    norms = np.linalg.norm(p.B.reshape(p.naux, -1), axis=1)
    np.testing.assert_allclose(norms, np.exp(-0.05 * np.arange(p.naux)), rtol=1e-13)
    np.testing.assert_array_equal(p.fock, np.diag(p.eps))


@pytest.mark.parametrize("dims", DIMS)
def test_reading_b_fock_structure(dims):
    p = make_problem(*dims, seed=5, reading="B")
    clo, act, vir = _slices(p)
    f = p.fock
    assert np.array_equal(f, f.T)
    np.testing.assert_array_equal(np.diag(f), p.eps)
    for sl in (clo, act, vir):
        blk = f[sl, sl]
        assert np.array_equal(blk, np.diag(np.diag(blk)))
    for b1, b2 in ((clo, act), (act, vir), (clo, vir)):
        if f[b1, b2].size:
            assert np.any(f[b1, b2] != 0.0)


@pytest.mark.parametrize("dims", DIMS)
def test_reading_c_is_reading_b_rotated(dims):
    pb = make_problem(*dims, seed=7, reading="B")
    pc = make_problem(*dims, seed=7, reading="C")
    clo, act, vir = _slices(pb)
    U = np.eye(pb.nc + pb.na + pb.nv)
    U[clo, clo] = pc.rot_c
    U[vir, vir] = pc.rot_v
    for R in (pc.rot_c, pc.rot_v):
        np.testing.assert_allclose(R.T @ R, np.eye(R.shape[0]), atol=1e-14)
    np.testing.assert_allclose(pc.fock, U.T @ pb.fock @ U, atol=1e-13)
    np.testing.assert_allclose(pc.hcore, U.T @ pb.hcore @ U, atol=1e-13)
    np.testing.assert_allclose(pc.B, np.einsum("xp,Qxy,yq->Qpq", U, pb.B, U), atol=1e-14)
    np.testing.assert_array_equal(pc.ci, pb.ci)
    np.testing.assert_array_equal(pc.eref, pb.eref)
    # the rotation keeps the spectra of the closed and virtual Fock blocks
    np.testing.assert_allclose(np.linalg.eigvalsh(pc.fock[clo, clo]), pb.eps[clo], atol=1e-13)
    np.testing.assert_allclose(np.linalg.eigvalsh(pc.fock[vir, vir]), pb.eps[vir], atol=1e-13)


def _cas_energy_matrix(p):
    """<I|H_act|J> by Slater-Condon rules over the alpha x beta string
    determinants (the determinant order and phase convention of the
    generator's header), written out here independently of the generator's
    own Hamiltonian builder."""
    na, nc = p.na, p.nc
    act = slice(nc, nc + na)
    h = p.hcore[act, act]
    Ba = p.B[:, act, act]
    g = np.einsum("Qpq,Qrs->pqrs", Ba, Ba)
    sa, sb = strings(na, p.nalpha), strings(na, p.nbeta)
    dets = [(a, b) for a in sa for b in sb]
    # spin orbitals: alpha p -> p, beta p -> na + p; creation order alpha
    # ascending, then beta ascending
    def occ(d):
        a, b = d
        return [q for q in range(na) if a >> q & 1] + [na + q for q in range(na) if b >> q & 1]

    def h1(P, Q):
        return h[P % na, Q % na] if (P < na) == (Q < na) else 0.0

    def g2(P, Q, R, S):   # <PQ|RS> in physicists' order
        if (P < na) != (R < na) or (Q < na) != (S < na):
            return 0.0
        return g[P % na, R % na, Q % na, S % na]

    n = len(dets)
    H = np.zeros((n, n))
    occs = [occ(d) for d in dets]
    for I in range(n):
        oi = occs[I]
        for J in range(n):
            oj = occs[J]
            si, sj = set(oi), set(oj)
            diff_i = [q for q in oi if q not in sj]
            diff_j = [q for q in oj if q not in si]
            if len(diff_i) > 2:
                continue
            if len(diff_i) == 0:
                e = sum(h1(P, P) for P in oi)
                e += 0.5 * sum(g2(P, Q, P, Q) - g2(P, Q, Q, P) for P in oi for Q in oi)
                H[I, J] = e
                continue
            # bring the differing orbitals of each determinant to the front;
            # the phase is the parity of the moves
            def front(o, d):
                o = list(o)
                sgn = 1
                for k, q in enumerate(d):
                    pos = o.index(q)
                    sgn *= (-1) ** (pos - k)
                    o.insert(k, o.pop(pos))
                return o, sgn
            _, s1 = front(oi, diff_i)
            rest, s2 = front(oj, diff_j)
            sgn = s1 * s2
            common = rest[len(diff_j):]
            if len(diff_i) == 1:
                P, Q = diff_i[0], diff_j[0]
                e = h1(P, Q) + sum(g2(P, R, Q, R) - g2(P, R, R, Q) for R in common)
            else:
                P, Q = diff_i
                R, S = diff_j
                e = g2(P, Q, R, S) - g2(P, Q, S, R)
            H[I, J] = sgn * e
    return H


@pytest.mark.parametrize("dims", DIMS)
def test_reference_states_are_lowest_cas_roots(dims):
    p = make_problem(*dims, seed=11, reading="B")
    ndet = math.comb(p.na, p.nalpha) * math.comb(p.na, p.nbeta)
    assert p.ci.shape == (p.nst, ndet)
    np.testing.assert_allclose(p.ci @ p.ci.T, np.eye(p.nst), atol=1e-13)
    assert np.all(np.diff(p.eref) >= 0.0)
    H = _cas_energy_matrix(p)
    np.testing.assert_allclose(H, H.T, atol=1e-14)
    w = np.linalg.eigvalsh(H)
    np.testing.assert_allclose(p.eref, w[:p.nst], atol=1e-12)
    for N in range(p.nst):
        np.testing.assert_allclose(H @ p.ci[N], p.eref[N] * p.ci[N], atol=1e-11)


@pytest.mark.parametrize("nc,nv", [(4, 20), (10, 120), (30, 400)])
def test_coupling_blocks_stay_small(nc, nv):
    """Spectral norms of the closed-active, active-virtual and closed-virtual
    blocks of f stay well below the smallest orbital-energy gap between
    classes (0.2) at every size, the property the 1/sqrt(n) scaling is for."""
    p = make_problem(nc, 2, nv, 60, 1, seed=2, reading="B")
    clo, act, vir = _slices(p)
    for b1, b2 in ((clo, act), (act, vir), (clo, vir)):
        assert np.linalg.norm(p.fock[b1, b2], 2) < 0.15


def test_same_seed_same_problem():
    a = make_problem(3, 4, 9, 40, 2, seed=4, reading="C", shift=0.2)
    b = make_problem(3, 4, 9, 40, 2, seed=4, reading="C", shift=0.2)
    for name in ("eps", "fock", "hcore", "B", "ci", "eref"):
        assert np.array_equal(getattr(a, name), getattr(b, name)), name
    c = make_problem(3, 4, 9, 40, 2, seed=5, reading="C", shift=0.2)
    assert not np.array_equal(a.B, c.B)
