"""Pins of the CPU oracle against things other than itself.

* O1 (explicit determinants) against Slater-Condon sums (single determinant
  reference) and the closed-form DF-MP2 energy (no active orbitals);
* O2 (factorised engine) against O1 element by element (operator, sources,
  metric) and on energies, amplitudes and lambda;
* invariances and identities the paper states: MS-MR invariance under a
  rotation of the reference states (Sec. II.B), MS = XMS at U = 1 (end of
  Sec. II.A), the lambda equation as the stationarity condition of the
  Lagrangian (Eqs. 18-20), Hylleraas stationarity, orbital-rotation
  invariance inside the closed and virtual spaces.
"""
import numpy as np
import pytest

from synth.gen import make_problem
from oracle.brute import BruteSystem, solve_brute
from oracle.ic import BLOCKS, Caspt2Oracle
from tests._slater import mp2_like_energy

# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------

# O1 operator type -> (block, ext slots from (p, q, r, s), type in block, act slots)
_MAP = {
    0: ("ccvv", (1, 3, 0, 2), 0, ()),
    1: ("cavv", (3, 0, 2), 0, (1,)),
    2: ("aavv", (0, 2), 0, (1, 3)),
    3: ("ccav", (1, 3, 0), 0, (2,)),
    4: ("ccaa", (1, 3), 0, (0, 2)),
    5: ("aaav", (0,), 0, (1, 2, 3)),
    6: ("caaa", (1,), 0, (0, 2, 3)),
    7: ("caav", (1, 0), 0, (2, 3)),
    8: ("caav", (3, 0), 1, (1, 2)),
}


def _perm(o2, keys, L):
    """Embedding of O1 function indices into the flattened all-orderings
    space of O2 (block by block, in BLOCKS order)."""
    p = o2.p
    nc, na = p.nc, p.na
    offs, shapes, off = {}, {}, 0
    for b in BLOCKS:
        shape = tuple(o2.dimsp[sp] for (_, sp) in b.ext) + (o2.nalpha[b.name],)
        offs[b.name], shapes[b.name] = off, shape
        off += int(np.prod(shape))
    pos = np.zeros(len(keys), dtype=np.int64)
    for k, (t, pqrs, N) in enumerate(keys):
        name, ext_sl, ty, act_sl = _MAP[t]
        b = next(bb for bb in BLOCKS if bb.name == name)
        ext = []
        for (lab, sp), sidx in zip(b.ext, ext_sl):
            v = pqrs[sidx]
            ext.append(v if sp == "c" else v - nc - na)
        act = [pqrs[s] - nc for s in act_sl]
        ntup = na ** len(b.act)
        tup = 0
        for a in act:
            tup = tup * na + a
        st = N if o2.scheme == "MSMR" else 0
        alpha = (st * len(b.types) + ty) * ntup + tup
        pos[k] = offs[name] + np.ravel_multi_index(tuple(ext) + (alpha,), shapes[name])
    return pos, offs, shapes, off


def _flat(o2, xall):
    return np.concatenate([xall[b.name].ravel() for b in BLOCKS])


def _unflat(o2, v, offs, shapes):
    return {b.name: v[offs[b.name]: offs[b.name] + int(np.prod(shapes[b.name]))].reshape(shapes[b.name])
            for b in BLOCKS}


# --------------------------------------------------------------------------
# O1 pins
# --------------------------------------------------------------------------

def test_o1_reproduces_cas_hamiltonian():
    """The CI vectors are eigenvectors of the explicit H in the CAS space
    with eigenvalues eref + one core constant (Eq. 2)."""
    from oracle.brute import dot
    p = make_problem(2, 3, 2, 14, 3, seed=11, reading="B")
    s = BruteSystem(p)
    refs = s.reference_states()
    H = np.array([[dot(a, s.apply_ham(b)) for b in refs] for a in refs])
    const = H[0, 0] - p.eref[0]
    assert np.allclose(H - np.diag(p.eref + const), 0.0, atol=1e-12)


def _single_det_problem(nc, nv, naux, seed, shift):
    p = make_problem(nc, 2, nv, naux, 1, seed=seed, reading="A", shift=shift, nelec=2)
    ci = np.zeros_like(p.ci)
    ci[0, 0] = 1.0          # alpha and beta both in the first active orbital
    return p.replace(ci=ci)


@pytest.mark.parametrize("shift", [0.0, 0.3])
def test_single_determinant_matches_slater_condon(shift):
    """P2: a closed-shell single-determinant reference; the IC space spans
    the H-projection of every single and double excitation leaving the CAS,
    so E2 equals the Slater-Condon sum (all eight blocks contribute)."""
    p = _single_det_problem(2, 3, 16, 3, shift)
    s = BruteSystem(p)
    cas = list(range(p.nc, p.nc + p.na))
    occ = list(range(p.nc)) + [p.nc]
    ref = mp2_like_energy(s.h, s.eri, p.eps, occ, cas, shift)
    o1 = solve_brute(p, "MSMR", xms=False, want_lambda=False)
    e1 = o1["heff"][0, 0] - o1["href"][0, 0]
    o2 = Caspt2Oracle(p, "MSMR", xms=False).run()
    e2 = o2.H_eff[0, 0] - o2.href[0, 0]
    assert abs(e1 - ref) < 1e-12
    assert abs(e2 - ref) < 1e-12


def test_single_determinant_larger_o2():
    p = _single_det_problem(4, 9, 40, 7, 0.2)
    s = BruteSystem(p)
    cas = list(range(p.nc, p.nc + p.na))
    occ = list(range(p.nc)) + [p.nc]
    ref = mp2_like_energy(s.h, s.eri, p.eps, occ, cas, 0.2)
    o2 = Caspt2Oracle(p, "MSMR", xms=False).run()
    assert abs((o2.H_eff[0, 0] - o2.href[0, 0]) - ref) < 1e-12


@pytest.mark.parametrize("shift", [0.0, 0.25])
def test_no_active_orbitals_is_df_mp2(shift):
    """P3: na = 0 leaves only ccvv; E2 is the closed-form DF-MP2 energy with
    the shift correction of Eq. 15."""
    p = make_problem(5, 0, 11, 40, 1, seed=4, reading="A", shift=shift)
    nc = p.nc
    B = p.B
    ovov = np.einsum("Qia,Qjb->iajb", B[:, :nc, nc:], B[:, :nc, nc:])
    ec, ev = p.eps[:nc], p.eps[nc:]
    d = ev[None, :, None, None] + ev[None, None, None, :] - ec[:, None, None, None] - ec[None, None, :, None]
    g = -1.0 / (d + shift) - shift / (d + shift) ** 2
    ref = np.sum(ovov * (2 * ovov - ovov.transpose(0, 3, 2, 1)) * g)
    o2 = Caspt2Oracle(p).run()
    assert abs((o2.H_eff[0, 0] - o2.href[0, 0]) - ref) < 1e-12
    o1 = solve_brute(make_problem(2, 0, 3, 10, 1, seed=4, reading="A", shift=shift), "MSMR")
    p1 = make_problem(2, 0, 3, 10, 1, seed=4, reading="A", shift=shift)
    B, nc = p1.B, p1.nc
    ovov = np.einsum("Qia,Qjb->iajb", B[:, :nc, nc:], B[:, :nc, nc:])
    ec, ev = p1.eps[:nc], p1.eps[nc:]
    d = ev[None, :, None, None] + ev[None, None, None, :] - ec[:, None, None, None] - ec[None, None, :, None]
    g = -1.0 / (d + shift) - shift / (d + shift) ** 2
    ref1 = np.sum(ovov * (2 * ovov - ovov.transpose(0, 3, 2, 1)) * g)
    assert abs((o1["heff"][0, 0] - o1["href"][0, 0]) - ref1) < 1e-12


# --------------------------------------------------------------------------
# O2 against O1, element by element
# --------------------------------------------------------------------------

CASES = [
    ("B", "MSMR", (2, 3, 3, 16, 3), True),
    ("B", "SSSR", (2, 3, 3, 16, 3), True),
    ("C", "MSMR", (2, 2, 3, 14, 2), True),
    ("A", "MSMR", (2, 3, 2, 14, 2), False),
]


@pytest.mark.parametrize("reading,scheme,dims,xms", CASES)
def test_o2_matches_o1_elementwise(reading, scheme, dims, xms):
    p = make_problem(*dims, seed=5, reading=reading, shift=0.15)
    o1 = solve_brute(p, scheme, xms=xms)
    o2 = Caspt2Oracle(p, scheme, xms=xms).run()
    rng = np.random.default_rng(0)
    assert np.allclose(o1["U"], o2.U, atol=1e-12)
    assert np.allclose(o1["e0"], o2.e0, atol=1e-13)
    for L in range(p.nst):
        d = o1["L"][L]
        pos, offs, shapes, n = _perm(o2, d["keys"], L)
        assert len(np.unique(pos)) == n == len(pos)
        y = rng.standard_normal(len(pos))
        x = np.zeros(n)
        x[pos] = y
        sig = _flat(o2, o2.apply_A(L, _unflat(o2, x, offs, shapes)))
        ref = np.zeros(n)
        ref[pos] = d["A"] @ y
        assert np.abs(sig - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
        for N in range(p.nst):
            v = _flat(o2, o2.source_all(L, N))
            vref = np.zeros(n)
            vref[pos] = d["V"][:, N]
            assert np.abs(v - vref).max() < 1e-13
        # amplitudes and lambda in the packed layout are unique
        T1 = np.zeros(n)
        T1[pos] = d["T"]
        T1p = o2.pack(_unflat(o2, T1, offs, shapes))
        assert np.linalg.norm(T1p - o2.T[L]) <= 1e-8 * np.linalg.norm(o2.T[L])
        l1 = np.zeros(n)
        l1[pos] = d["lam"]
        l1p = o2.pack(_unflat(o2, l1, offs, shapes))
        lam_scale = max(np.linalg.norm(v) for v in o2.lam)
        assert np.linalg.norm(l1p - o2.lam[L]) <= 1e-8 * lam_scale
    c1 = o1["heff"] - o1["href"]
    c2 = o2.H_eff - o2.href
    assert np.abs(c1 - c2).max() < 1e-11


# --------------------------------------------------------------------------
# identities and invariances (at sizes the brute force cannot reach)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def mid():
    p = make_problem(3, 4, 7, 30, 3, seed=21, reading="B", shift=0.2)
    return p, Caspt2Oracle(p, "MSMR").run()


def test_xms_diagonalises_fock_in_reference_space(mid):
    p, o = mid
    Fr = o.U.T @ o.fref @ o.U
    assert np.abs(Fr - np.diag(np.diag(Fr))).max() < 1e-13
    assert np.allclose(np.diag(Fr), o.e0, atol=1e-13)
    assert np.all(np.diff(o.e0) >= 0)


def test_msmr_invariant_to_reference_rotation(mid):
    """MS-MR XMS-CASPT2 is invariant to rotations among reference states."""
    p, o = mid
    rng = np.random.default_rng(3)
    W, _ = np.linalg.qr(rng.standard_normal((p.nst, p.nst)))
    o2 = Caspt2Oracle(p, "MSMR", rotate_states=W).run()
    assert np.abs(o2.e_ms - o.e_ms).max() < 1e-10


def test_operator_symmetric_and_hylleraas(mid):
    p, o = mid
    rng = np.random.default_rng(1)
    L = 1
    x = rng.standard_normal(o.length)
    y = rng.standard_normal(o.length)
    Ax = o.residual(L, x, with_source=False)
    Ay = o.residual(L, y, with_source=False)
    assert abs(x @ Ay - y @ Ax) < 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(y)
    V = o.source(L, L)
    T = o.T[L]
    J = lambda t: 2 * t @ V + t @ o.residual(L, t, with_source=False)
    assert abs(J(T) - T @ V) < 1e-12
    d = o._from_orth(L, [np.random.default_rng(2).standard_normal(a.shape) for a in o._to_orth(L, T)])
    h = 1e-4
    assert abs((J(T + h * d) - J(T - h * d)) / (2 * h)) < 1e-9


def test_lambda_from_lagrangian_fd_shift():
    """dE^MS_P/dE_s = sum_L lambda_L S T_L - sum_L R_LP^2 T_L S T_L
    (the explicit shift dependence of the Lagrangian Eq. 18)."""
    base = make_problem(3, 4, 7, 30, 3, seed=21, reading="B", shift=0.2)
    P = 0
    o = Caspt2Oracle(base, "MSMR").run(P)
    ana = sum(o.lam[L] @ o.apply_S(L, o.T[L]) - o.R[L, P] ** 2 * o.T[L] @ o.apply_S(L, o.T[L])
              for L in range(base.nst))
    h = 1e-4
    ep = Caspt2Oracle(base.replace(shift=0.2 + h), "MSMR").run(P).e_ms[P]
    em = Caspt2Oracle(base.replace(shift=0.2 - h), "MSMR").run(P).e_ms[P]
    fd = (ep - em) / (2 * h)
    assert abs(fd - ana) < 1e-8 * max(1.0, abs(ana))


def test_lambda_from_lagrangian_fd_virtual_energy():
    """dE^MS_P/d eps_a = sum_L <lambda_L| E_aa |T_L> (Eq. 18, f enters only
    through the operator)."""
    base = make_problem(2, 3, 5, 24, 2, seed=8, reading="B", shift=0.2)
    P = 1
    o = Caspt2Oracle(base, "MSMR").run(P)
    a = 2
    na_ = base.nc + base.na + a
    ana = 0.0
    for L in range(base.nst):
        lam, T = o.unpack(o.lam[L]), o.unpack(o.T[L])
        # <lambda| E_aa |T> through the operator with unit f at (a, a)
        f1 = np.zeros_like(base.fock)
        f1[na_, na_] = 1.0
        o1 = Caspt2Oracle(base.replace(fock=f1, shift=0.0), "MSMR")
        o1.ci, o1.U = o.ci, o.U
        o1.e0 = np.zeros(base.nst)
        AT = o1.apply_A(L, T)
        ana += sum(np.sum(lam[k] * AT[k]) for k in lam)
    h = 1e-4
    def e(dv):
        f = base.fock.copy()
        f[na_, na_] += dv
        eps = base.eps.copy()
        eps[na_] += dv
        return Caspt2Oracle(base.replace(fock=f, eps=eps), "MSMR").run(P).e_ms[P]
    fd = (e(h) - e(-h)) / (2 * h)
    assert abs(fd - ana) < 1e-8 * max(1.0, abs(ana))


def test_nst1_lambda_equals_t_without_shift():
    p = make_problem(3, 4, 8, 30, 1, seed=2, reading="B", shift=0.0)
    o = Caspt2Oracle(p).run()
    assert np.linalg.norm(o.lam[0] - o.T[0]) < 1e-10 * np.linalg.norm(o.T[0])


def test_sssr_equals_msmr_at_one_state():
    p = make_problem(3, 4, 8, 30, 1, seed=2, reading="B", shift=0.2)
    a = Caspt2Oracle(p, "MSMR").run()
    b = Caspt2Oracle(p, "SSSR").run()
    assert abs(a.e_ms[0] - b.e_ms[0]) < 1e-12
    assert np.linalg.norm(a.T[0] - b.T[0]) < 1e-10 * np.linalg.norm(a.T[0])


def test_ms_is_xms_with_unit_rotation_and_differs_otherwise(mid):
    p, o = mid
    ms = Caspt2Oracle(p, "MSMR", xms=False).run()
    assert np.allclose(ms.U, np.eye(p.nst))
    assert np.allclose(ms.e0, np.diag(ms.fref))
    assert np.abs(ms.e_ms - o.e_ms).max() > 1e-8


def test_reading_a_converges_in_one_step_and_decouples_states():
    p = make_problem(3, 4, 8, 30, 3, seed=21, reading="A", shift=0.2)
    o = Caspt2Oracle(p, "MSMR").run()
    assert all(i["iters"] <= 1 for i in o.T_info)
    # ccvv amplitudes on N != L vanish (no couplings between blocks)
    for L in range(p.nst):
        cc = o.unpack(o.T[L])["ccvv"]
        for N in range(p.nst):
            if N != L:
                assert np.abs(cc[..., N]).max() < 1e-14


def test_closed_virtual_rotation_invariance():
    pb = make_problem(3, 3, 7, 26, 2, seed=9, reading="B", shift=0.2)
    pc = make_problem(3, 3, 7, 26, 2, seed=9, reading="C", shift=0.2)
    eb = Caspt2Oracle(pb).run().e_ms
    ec = Caspt2Oracle(pc).run().e_ms
    assert np.abs(eb - ec).max() < 1e-10


def test_active_rotation_invariance():
    """E^MS does not depend on the basis of the active orbitals when f, h^c,
    the DF factors and the reference states are transformed together: the
    functions of Eq. 8 span the same space, the truncation of Sec. II.B acts
    on metric eigenvalues that an orthogonal change of the active index
    leaves alone, and the XMS Fock matrix of Eq. 3 is a scalar over the
    reference space.  Catches an active index contracted in the wrong slot
    of a Gamma tensor or of the active Fock block."""
    from synth.gen import rotate_active
    for reading in ("A", "B"):
        p = make_problem(2, 3, 4, 20, 2, seed=5, reading=reading, shift=0.15)
        pr = rotate_active(p, seed=11)
        assert np.abs(pr.eref - p.eref).max() < 1e-12
        e = Caspt2Oracle(p).run().e_ms
        er = Caspt2Oracle(pr).run().e_ms
        assert np.abs(e - er).max() < 1e-10, (reading, e, er)


@pytest.mark.parametrize("reading", ["A", "B", "C"])
def test_operator_vanishes_on_metric_null_space(reading):
    """A coefficient vector in the null space of a block's metric S describes
    the zero function (Eq. 8 functions are linearly dependent), so the
    operator of Eq. 10 maps it to zero in every block, couplings included.
    The metric and the Fock metric are evaluated separately (the Fock one
    through the Fock-contracted fourth-order density), so this catches a
    dropped or misplaced pairing in one of them."""
    p = make_problem(2, 3, 4, 20, 2, seed=5, reading=reading, shift=0.15)
    o = Caspt2Oracle(p)
    ort = o.ortho(0)
    rng = np.random.default_rng(3)
    checked = 0
    for k, ent in enumerate(o.layout):
        S = ort[k]["S"]
        if ent["nrow"] == 0 or S.size == 0:
            continue
        w, V = np.linalg.eigh(S)
        null = V[:, np.abs(w) < 1e-10 * np.abs(w).max()]
        if null.shape[1] == 0:
            continue
        na_, off = ent["nalpha"], ent["offset"]
        for r in rng.choice(ent["nrow"], size=min(2, ent["nrow"]), replace=False):
            sl = slice(off + r * na_, off + (r + 1) * na_)
            x = np.zeros(o.length)
            v = null @ rng.standard_normal(null.shape[1])
            x[sl] = v / np.linalg.norm(v)
            y = np.zeros(o.length)
            y[sl] = V[:, -1]          # a unit vector of the same row off the null space
            for L in range(p.nst):
                ref = np.linalg.norm(o.residual(L, y, with_source=False))
                got = np.linalg.norm(o.residual(L, x, with_source=False))
                assert got < 1e-10 * ref, (reading, k, int(r), L, got, ref)
                checked += 1
    assert checked >= 8


def test_amplitudes_transform_covariantly():
    """With the closed and virtual orbitals rotated (Reading C), T and lambda
    are the Reading B ones with every closed and virtual slot transformed by
    the same rotation: the functions of Eq. 8 transform as their external
    orbitals, and the solution of Eq. 10 in the kept space of Sec. II.B (and
    of Eq. 20) is unique.  Element by element, relative to each block's
    largest amplitude."""
    from oracle.ic import CLO, VIR
    pb = make_problem(3, 3, 7, 26, 2, seed=9, reading="B", shift=0.2)
    pc = make_problem(3, 3, 7, 26, 2, seed=9, reading="C", shift=0.2)
    ob = Caspt2Oracle(pb).run()
    oc = Caspt2Oracle(pc).run()
    U = {CLO: pc.rot_c, VIR: pc.rot_v}
    for L in range(pb.nst):
        for vb, vc in ((ob.T[L], oc.T[L]), (ob.lam[L], oc.lam[L])):
            tb, tc = ob.unpack(vb), oc.unpack(vc)
            for b in BLOCKS:
                t = tb[b.name]
                if t.size == 0:
                    continue
                for ax, (_, sp) in enumerate(b.ext):
                    t = np.moveaxis(np.tensordot(U[sp], t, axes=([0], [ax])), 0, ax)
                scale = max(np.abs(tc[b.name]).max(), 1e-300)
                assert np.abs(t - tc[b.name]).max() < 1e-9 * scale, (L, b.name)


def test_threshold_insensitivity(mid):
    p, o = mid
    for th in (1e-12, 1e-7):
        e = Caspt2Oracle(p, "MSMR", thresh=th).run().e_ms
        assert np.abs(e - o.e_ms).max() < 1e-10


def test_degenerate_xms_rotation_invariance():
    """With every CAS state a reference, F^ref has a degenerate eigenvalue
    here; any rotation inside that eigenspace is a valid XMS rotation
    (Eqs. 3-5).  Without shift E^MS is the same for every such choice; with
    a real shift it is not (the shift term of Eq. 15 is diagonal in the
    rotated basis), which the library documents as a reading."""
    import numpy as np
    from oracle.ic import Caspt2Oracle
    for shift, same in ((0.0, True), (0.3, False)):
        p = make_problem(2, 2, 3, 12, 4, seed=5, reading="B", shift=shift)
        o = Caspt2Oracle(p, "MSMR").run(P=0)
        i = int(np.argmin(np.diff(o.e0)))
        assert np.diff(o.e0)[i] < 1e-12
        G = np.eye(4)
        c, s_ = np.cos(0.5), np.sin(0.5)
        G[i, i], G[i, i + 1], G[i + 1, i], G[i + 1, i + 1] = c, -s_, s_, c
        o2 = Caspt2Oracle(p, "MSMR", xms=False, rotate_states=o.U @ G).run(P=0)
        d = np.abs(np.sort(o2.e_ms) - np.sort(o.e_ms)).max()
        assert (d < 1e-12) if same else (d > 1e-6), (shift, d)


# --------------------------------------------------------------------------
# correlated densities (Sec. II.D): O1's written-out definitions against
# finite differences of E^MS_P, which is stationary in T, lambda and R
# (Eqs. 18-20), so its derivative with respect to a parameter of H or f at
# fixed reference states is the parameter's explicit derivative of the
# Lagrangian, i.e. a contraction with the densities
# --------------------------------------------------------------------------

def _richardson(fun, h=1e-4):
    """Central difference with one Richardson step (error O(h^4))."""
    d1 = (fun(h) - fun(-h)) / (2 * h)
    d2 = (fun(h / 2) - fun(-h / 2)) / h
    return (4 * d2 - d1) / 3


@pytest.fixture(scope="module", params=["MSMR", "SSSR"])
def dens_case(request):
    from oracle.brute import densities_brute
    scheme = request.param
    p = make_problem(2, 2, 2, 12, 2, seed=5, reading="B", shift=0.15)
    P = 1
    o = solve_brute(p, scheme, xms=True, target=P)
    return p, scheme, P, o, densities_brute(p, o)


def test_density_d1_is_the_hcore_derivative(dens_case):
    """dE^MS_P/dh^c along a symmetric direction = sum (gamma_P + d1) Dh:
    <P|E_xy|P> from H^ref and d^(1) from the sources of Eqs. 10 and 15."""
    p, scheme, P, o, d = dens_case
    rng = np.random.default_rng(3)
    Dh = rng.standard_normal((p.nmo, p.nmo))
    Dh = Dh + Dh.T
    fd = _richardson(lambda e: solve_brute(p.replace(hcore=p.hcore + e * Dh), scheme, xms=True, target=P,
                                           want_lambda=False)["e_ms"][P])
    ana = float(np.sum(Dh * (d["gamma_P"] + d["d1"])))
    assert abs(fd - ana) < 1e-9 * max(1.0, abs(ana))


def test_density_D1_is_the_eri_derivative(dens_case):
    """dE^MS_P/d(xy|zw) along a random direction with the symmetry of real
    integrals = 1/2 sum (Gamma_P + D1) D (bare h held fixed)."""
    p, scheme, P, o, d = dens_case
    rng = np.random.default_rng(4)
    n = p.nmo
    De = rng.standard_normal((n, n, n, n))
    De = De + De.transpose(1, 0, 2, 3)
    De = De + De.transpose(0, 1, 3, 2)
    De = De + De.transpose(2, 3, 0, 1)

    def e(eps):
        s = BruteSystem(p)
        s.eri = s.eri + eps * De
        return solve_brute(p, scheme, xms=True, target=P, want_lambda=False, sysm=s)["e_ms"][P]
    fd = _richardson(e)
    ana = float(0.5 * np.sum(De * (d["Gamma_P"] + d["D1"])))
    assert abs(fd - ana) < 1e-9 * max(1.0, abs(ana))


def test_density_d2_is_the_fock_derivative(dens_case):
    """dE^MS_P/df at fixed XMS rotation = sum d2 Df - 2 tr(Df_cc) sum_L N_L:
    d-bar^(2) from the operator of Eq. 10, -N_L <L|E|L> from E_L^(0) (Eq. 14),
    and the closed constant of the normal ordering (Eq. 12)."""
    p, scheme, P, o, d = dens_case
    rng = np.random.default_rng(5)
    Df = rng.standard_normal((p.nmo, p.nmo))
    Df = Df + Df.T
    fd = _richardson(lambda e: solve_brute(p.replace(fock=p.fock + e * Df), scheme, xms=True, target=P,
                                           want_lambda=False, fixed_U=o["U"])["e_ms"][P])
    ana = float(np.sum(Df * d["d2"]) - 2.0 * np.trace(Df[:p.nc, :p.nc]) * d["NL"].sum())
    assert abs(fd - ana) < 1e-9 * max(1.0, abs(ana))


def test_density_norms_are_metric_products(dens_case):
    """N_L = lambda_L . S . T_L in the function basis of state L."""
    p, scheme, P, o, d = dens_case
    for L in range(p.nst):
        dL = o["L"][L]
        assert abs(d["NL"][L] - dL["lam"] @ dL["S"] @ dL["T"]) < 1e-12 * max(1.0, abs(d["NL"][L]))


@pytest.mark.parametrize("reading,scheme,dims,xms", [
    ("B", "MSMR", (2, 2, 2, 12, 2), True), ("B", "SSSR", (2, 2, 2, 12, 2), True),
    ("C", "MSMR", (2, 2, 3, 14, 2), True), ("A", "MSMR", (2, 3, 2, 14, 2), False)])
def test_o2_densities_match_o1(reading, scheme, dims, xms):
    """The factorised densities (Wick terms and active Gram tensors contracted
    with T, lambda, R) equal O1's written-out ones element by element: d^(1),
    D^(1) on the classes of the two-body part of H acting on the references,
    d-bar^(2), N_L, d^(2)."""
    from oracle.brute import densities_brute
    p = make_problem(*dims, seed=5, reading=reading, shift=0.15)
    P = 1
    d = densities_brute(p, solve_brute(p, scheme, xms=xms, target=P))
    e = Caspt2Oracle(p, scheme, xms=xms).run(P).densities()
    sl = {"c": slice(0, p.nc), "a": slice(p.nc, p.nc + p.na), "v": slice(p.nc + p.na, p.nmo)}
    tol = 1e-12
    assert np.abs(d["d1"] - e["d1"]).max() < tol
    assert len(e["D1"]) == 15
    for k, v in e["D1"].items():
        assert np.abs(d["D1"][sl[k[0]], sl[k[1]], sl[k[2]], sl[k[3]]] - v).max() < tol, k
    assert np.abs(d["dbar2"] - e["dbar2"]).max() < tol
    assert np.abs(d["d2"] - e["d2"]).max() < tol
    assert np.abs(d["NL"] - e["NL"]).max() < tol
