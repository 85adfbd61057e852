"""Seeded synthetic inputs for the (X)MS-CASPT2 amplitude / lambda hot path.

This module only *draws* problem inputs: orbital energies, density-fitting
factors, the core one-electron Hamiltonian h^c, the reference CAS-CI states
and the Fock matrix handed to the perturbation step.  It contains none of the
perturbation method itself (no internally contracted functions, no metrics,
no residuals, no XMS rotation).  Both the CPU oracle and the HIP library read
its output; neither imports the other.

The reference states are eigenvectors of the active-space Hamiltonian
(paper Sec. II.A, Eqs. 1-2); the Fock operator follows Eq. 11 with the
state-averaged density of Eq. 13 (weights 1/N_st, Sec. II.A).

Conventions fixed here and relied on by every consumer
------------------------------------------------------
* Orbital order: closed 0..nc-1 | active nc..nc+na-1 | virtual.
* Active determinants: alpha string times beta string.  A string is a bit
  mask over the na active orbitals; strings of a given electron count are
  enumerated in increasing integer value.  Determinant index
  I = ia * n_beta_strings + ib, and |I> = prod_{p in alpha, ascending}
  a+_{p alpha} prod_{p in beta, ascending} a+_{p beta} |vac>.
* ci[N, I] are the CAS-CI coefficients of state N (unrotated), each column
  normalised, sign fixed so that its largest-magnitude entry is positive.
* B[Q, p, q] = B[Q, q, p]; (pq|rs) = sum_Q B[Q,p,q] B[Q,r,s].
* eref[N] are active-space CAS-CI energies (no core constant).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

__all__ = ["Problem", "make_problem", "workload_problem", "batch_sizes", "strings"]


def strings(norb: int, nel: int) -> np.ndarray:
    """All bit strings over norb orbitals with nel bits set, ascending."""
    out = [s for s in range(1 << norb) if bin(s).count("1") == nel]
    return np.array(out, dtype=np.int64)


@dataclasses.dataclass
class Problem:
    nc: int
    na: int
    nv: int
    naux: int
    nst: int
    nelec: int
    nalpha: int
    nbeta: int
    seed: int
    reading: str
    shift: float
    eps: np.ndarray        # [nmo] orbital energies (diagonal of f)
    fock: np.ndarray       # [nmo, nmo] symmetric Fock matrix f
    hcore: np.ndarray      # [nmo, nmo] symmetric h^c (core-dressed one-electron part)
    B: np.ndarray          # [naux, nmo, nmo] DF factors
    ci: np.ndarray         # [nst, ndet] CAS-CI vectors (unrotated)
    eref: np.ndarray       # [nst] CAS-CI energies (active part only)
    natocc: np.ndarray     # [na] natural occupations of the SA density (diagnostic)
    rot_c: np.ndarray | None = None   # Reading C closed rotation (diagnostic)
    rot_v: np.ndarray | None = None   # Reading C virtual rotation (diagnostic)

    @property
    def nmo(self) -> int:
        return self.nc + self.na + self.nv

    @property
    def ndet(self) -> int:
        return self.ci.shape[1]

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# active-space determinant algebra used only to build the reference states
# --------------------------------------------------------------------------

def _string_excitations(strs: np.ndarray, norb: int):
    """For each (p, q): rows (target index), cols (source index), signs of
    a+_p a_q acting on the strings of one spin."""
    index = {int(s): k for k, s in enumerate(strs)}
    table = {}
    for p in range(norb):
        for q in range(norb):
            rows, cols, sgn = [], [], []
            for k, s in enumerate(strs):
                s = int(s)
                if not (s >> q) & 1:
                    continue
                t = s & ~(1 << q)
                if (t >> p) & 1:
                    continue
                lo, hi = min(p, q), max(p, q)
                between = bin(s & (((1 << hi) - 1) ^ ((1 << (lo + 1)) - 1))).count("1") if hi > lo else 0
                t |= 1 << p
                rows.append(index[t])
                cols.append(k)
                sgn.append(-1.0 if between % 2 else 1.0)
            table[(p, q)] = (np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64),
                             np.array(sgn))
    return table


def _epq_matrices(norb: int, na_el: int, nb_el: int):
    """Sparse matrices of the spin-summed E_pq on the (na_el, nb_el) space."""
    sa, sb = strings(norb, na_el), strings(norb, nb_el)
    ta, tb = _string_excitations(sa, norb), _string_excitations(sb, norb)
    nA, nB = len(sa), len(sb)
    n = nA * nB
    E = {}
    ib = np.arange(nB)
    ia = np.arange(nA)
    for p in range(norb):
        for q in range(norb):
            r_a, c_a, s_a = ta[(p, q)]
            rows = (r_a[:, None] * nB + ib[None, :]).ravel()
            cols = (c_a[:, None] * nB + ib[None, :]).ravel()
            vals = np.repeat(s_a, nB)
            r_b, c_b, s_b = tb[(p, q)]
            rows = np.concatenate([rows, (ia[:, None] * nB + r_b[None, :]).ravel()])
            cols = np.concatenate([cols, (ia[:, None] * nB + c_b[None, :]).ravel()])
            vals = np.concatenate([vals, np.tile(s_b, nA)])
            E[(p, q)] = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    return E


def _cas_hamiltonian(h: np.ndarray, g: np.ndarray, na_el: int, nb_el: int) -> tuple[np.ndarray, dict]:
    norb = h.shape[0]
    E = _epq_matrices(norb, na_el, nb_el)
    k = h - 0.5 * np.einsum("prrq->pq", g)
    n = E[(0, 0)].shape[0]
    H = sp.csr_matrix((n, n))
    for p in range(norb):
        for q in range(norb):
            H = H + k[p, q] * E[(p, q)]
    for r in range(norb):
        for s in range(norb):
            M = sp.csr_matrix((n, n))
            for p in range(norb):
                for q in range(norb):
                    if g[p, q, r, s] != 0.0:
                        M = M + g[p, q, r, s] * E[(p, q)]
            H = H + 0.5 * (M @ E[(r, s)])
    return H.toarray(), E


# --------------------------------------------------------------------------
# the generator
# --------------------------------------------------------------------------

def _sym(m: np.ndarray) -> np.ndarray:
    return 0.5 * (m + m.T)


def make_problem(nc: int, na: int, nv: int, naux: int, nst: int, seed: int,
                 reading: str = "B", shift: float = 0.0, nelec: int | None = None,
                 coupling_sigma: float = 0.02, f_ai_zero: bool = False) -> Problem:
    """Draw one problem.

    reading 'A': f = diag(eps) (orbital energies only).
    reading 'B': f = diag(eps) plus closed-active, active-virtual and
                 closed-virtual blocks of h^c + g(d_sa) (Eq. 11, Eq. 13).
    reading 'C': reading B rotated inside the closed and inside the virtual
                 space by seeded orthogonal matrices (f, h^c and B together).
    """
    reading = reading.upper()
    if reading not in ("A", "B", "C"):
        raise ValueError("reading must be A, B or C")
    nelec = na if nelec is None else nelec
    if na == 0:
        nelec = 0
    nalpha = (nelec + 1) // 2
    nbeta = nelec // 2
    nmo = nc + na + nv
    rng = np.random.Generator(np.random.PCG64(seed))
    e_c = np.sort(rng.uniform(-2.0, -0.5, nc))
    e_a = np.sort(rng.uniform(-0.3, 0.3, na))
    e_v = np.sort(rng.uniform(0.5, 4.0, nv))
    eps = np.concatenate([e_c, e_a, e_v])

    B = np.empty((naux, nmo, nmo))
    for Q in range(naux):
        G = rng.standard_normal((nmo, nmo))
        S = _sym(G)
        B[Q] = S * (math.exp(-0.05 * Q) / np.linalg.norm(S))

    act = slice(nc, nc + na)
    Ba = np.ascontiguousarray(B[:, act, act]).reshape(naux, na * na)
    g_act = (Ba.T @ Ba).reshape(na, na, na, na)
    sigma_h = float(np.sqrt(np.mean(g_act ** 2))) if na else 0.0
    G_act = rng.standard_normal((na, na))
    hcore = np.zeros((nmo, nmo))
    hcore[act, act] = sigma_h * _sym(G_act)
    clo, vir = slice(0, nc), slice(nc + na, nmo)
    for (b1, b2) in ((clo, act), (act, vir), (clo, vir)):
        n1, n2 = b1.stop - b1.start, b2.stop - b2.start
        # entries scaled by 1/sqrt(max(n1, n2)): the spectral norm of each
        # off-diagonal block stays about 2 coupling_sigma at any orbital-space
        # size, so the couplings remain small next to the orbital-energy gaps
        blk = coupling_sigma / math.sqrt(max(n1, n2, 1)) * rng.standard_normal((n1, n2))
        hcore[b1, b2] = blk
        hcore[b2, b1] = blk.T

    # reference states: lowest nst roots of the active-space Hamiltonian
    if na > 0:
        H, E = _cas_hamiltonian(hcore[act, act], g_act, nalpha, nbeta)
        w, v = np.linalg.eigh(H)
        if nst > H.shape[0]:
            raise ValueError("more states than determinants")
        ci = v[:, :nst].T.copy()
        eref = w[:nst].copy()
        # sign: the first determinant whose weight is within 1e-6 of the largest
        # is positive (entries of equal magnitude by spin symmetry differ only
        # by rounding, which varies between BLAS builds; a plain argmax would
        # let that rounding pick the sign)
        for N in range(nst):
            a = np.abs(ci[N])
            k = int(np.flatnonzero(a >= (1.0 - 1e-6) * a.max())[0])
            if ci[N, k] < 0:
                ci[N] = -ci[N]
        d_sa = np.zeros((na, na))
        for N in range(nst):
            for p in range(na):
                for q in range(na):
                    d_sa[p, q] += ci[N] @ (E[(p, q)] @ ci[N]) / nst
    else:
        if nst != 1:
            raise ValueError("na = 0 needs nst = 1")
        ci = np.ones((1, 1))
        eref = np.zeros(1)
        d_sa = np.zeros((0, 0))
    natocc = np.linalg.eigvalsh(_sym(d_sa))[::-1] if na else np.zeros(0)

    fock = np.diag(eps).copy()
    if reading in ("B", "C") and nmo:
        # g(d)_xy = sum_zw d_zw [ (xy|zw) - 1/2 (xw|zy) ], z,w active
        Bx = B  # [Q, x, y]
        J = np.einsum("Qxy,Qzw,zw->xy", Bx, B[:, act, act], d_sa) if na else np.zeros((nmo, nmo))
        K = np.einsum("Qxw,Qzy,zw->xy", B[:, :, act], B[:, act, :], d_sa) if na else np.zeros((nmo, nmo))
        gd = J - 0.5 * K
        full = hcore + gd
        for (b1, b2) in ((clo, act), (act, vir), (clo, vir)):
            if not (f_ai_zero and b1 == clo and b2 == vir):
                fock[b1, b2] = full[b1, b2]
                fock[b2, b1] = full[b2, b1]
        fock = _sym(fock)

    rot_c = rot_v = None
    if reading == "C":
        def haar(n):
            A = rng.standard_normal((n, n))
            q, r = np.linalg.qr(A)
            return q * np.sign(np.diag(r))[None, :]
        rot_c, rot_v = haar(nc), haar(nv)
        U = np.eye(nmo)
        U[clo, clo] = rot_c
        U[vir, vir] = rot_v
        fock = U.T @ fock @ U
        hcore = U.T @ hcore @ U
        B = np.einsum("xp,Qxy,yq->Qpq", U, B, U, optimize=True)
        fock = _sym(fock)
        hcore = _sym(hcore)

    return Problem(nc=nc, na=na, nv=nv, naux=naux, nst=nst, nelec=nelec, nalpha=nalpha,
                   nbeta=nbeta, seed=seed, reading=reading, shift=float(shift), eps=eps,
                   fock=fock, hcore=hcore, B=B, ci=ci, eref=eref, natocc=natocc,
                   rot_c=rot_c, rot_v=rot_v)


def rotate_active(prob: Problem, seed: int) -> Problem:
    """The same problem in active orbitals rotated by a seeded orthogonal
    matrix: f, h^c and the DF factors transformed together, the reference
    states recomputed as the lowest roots of the rotated active Hamiltonian
    (same energies; sign fixed as in make_problem)."""
    na, nc = prob.na, prob.nc
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.standard_normal((na, na))
    q, r = np.linalg.qr(A)
    Ua = q * np.sign(np.diag(r))[None, :]
    U = np.eye(prob.nmo)
    act = slice(nc, nc + na)
    U[act, act] = Ua
    fock = _sym(U.T @ prob.fock @ U)
    hcore = _sym(U.T @ prob.hcore @ U)
    B = np.einsum("xp,Qxy,yq->Qpq", U, prob.B, U, optimize=True)
    Ba = np.ascontiguousarray(B[:, act, act]).reshape(prob.naux, na * na)
    g_act = (Ba.T @ Ba).reshape(na, na, na, na)
    H, _ = _cas_hamiltonian(hcore[act, act], g_act, prob.nalpha, prob.nbeta)
    w, v = np.linalg.eigh(H)
    ci = v[:, :prob.nst].T.copy()
    for N in range(prob.nst):
        a = np.abs(ci[N])
        k = int(np.flatnonzero(a >= (1.0 - 1e-6) * a.max())[0])
        if ci[N, k] < 0:
            ci[N] = -ci[N]
    return prob.replace(fock=fock, hcore=hcore, B=B, ci=ci, eref=w[:prob.nst].copy(),
                        eps=np.diag(fock).copy())


# sizes of the named workloads: (nc, na, nv, naux, nst, seed, shift); the
# seed of the large one is the first whose denominators are all positive at
# shift 0.2 for every state (no intruder state)
WORKLOAD_SIZES = {
    "small": (4, 4, 20, 60, 1, 0, 0.0),
    "mid": (10, 6, 120, 400, 3, 1, 0.2),
    "full": (30, 8, 400, 1500, 4, 8, 0.2),
}


def workload_problem(name: str, reading: str = "B") -> Problem:
    nc, na, nv, naux, nst, seed, shift = WORKLOAD_SIZES[name]
    return make_problem(nc, na, nv, naux, nst, seed, reading=reading, shift=shift)


def batch_sizes(n: int = 64, seed: int = 4):
    """Sizes of the uneven batch: closed 4-16, active 4-6, virtual 20-150,
    states 1-4 (uniform, inclusive), naux = 3 (nc + na + nv); one child seed
    per instance from SeedSequence(seed).spawn(n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kids = np.random.SeedSequence(seed).spawn(n)
    out = []
    for k in range(n):
        nc = int(rng.integers(4, 17))
        na = int(rng.integers(4, 7))
        nv = int(rng.integers(20, 151))
        nst = int(rng.integers(1, 5))
        child = int(kids[k].generate_state(1)[0])
        out.append((nc, na, nv, 3 * (nc + na + nv), nst, child))
    return out


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded standard-normal vector (trial amplitudes for residual checks)."""
    return np.random.default_rng(seed).standard_normal(n)


def sample_positions(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct sorted positions in [0, n), seeded."""
    return np.sort(np.random.default_rng(seed).choice(n, k, replace=False))
