"""O1: brute-force oracle in the determinant basis.  TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
anything under oracle/; the product path never does.

Everything here is the plain definition of what the perturbation step
computes, written out on explicit Slater determinants (tiny sizes only):

* reference states |N> = core (all closed orbitals doubly occupied) times the
  active CI vector; virtual orbitals empty (Sec. II.A, Eqs. 1-2);
* XMS rotation: diagonalise <L|f|M> in the reference space (Eqs. 3-5), or
  U = 1 for MS-CASPT2 (end of Sec. II.A);
* internally contracted functions E_Omega |N~>, with the nine operator types
  of Eq. 8 in product form E_pq E_rs, generated from every reference state
  (MS-MR, Eq. 7) or from |L~> only (SS-SR, Eq. 9);
* the amplitude equation Eq. 10 projected on every function, with the
  overlap eigenvalues below the threshold removed (Sec. II.B);
* the effective Hamiltonian Eq. 15, its eigenpairs Eq. 16, and the lambda
  equation Eq. 20.

Operators: f^ = sum_xy f_xy E_xy - 2 sum_i f_ii (normal ordering with respect
to the closed vacuum, read as {E_ij}_C = E_ij - 2 delta_ij), and the full
Hamiltonian H = sum h_xy E_xy + 1/2 sum (xy|zw) (E_xy E_zw - delta_yz E_xw)
with the bare h = h^c - sum_i [2 (xy|ii) - (xi|iy)]; the core constant is
dropped (it cancels in every projected equation and in every energy
difference that is compared).

Spin orbitals: index so = sigma * nmo + p (all alpha before all beta);
a determinant is an int bit mask; |D> = prod over set bits in ascending
order of a+_so acting on the vacuum.
"""
from __future__ import annotations

import itertools

import numpy as np

# ---------------------------------------------------------------------------
# second quantisation on explicit determinants
# ---------------------------------------------------------------------------


def _popcount_below(det: int, so: int) -> int:
    return bin(det & ((1 << so) - 1)).count("1")


def ann(det: int, so: int):
    """a_so |det> -> (sign, det') or None."""
    if not (det >> so) & 1:
        return None
    return (-1.0 if _popcount_below(det, so) % 2 else 1.0), det & ~(1 << so)


def cre(det: int, so: int):
    """a+_so |det> -> (sign, det') or None."""
    if (det >> so) & 1:
        return None
    return (-1.0 if _popcount_below(det, so) % 2 else 1.0), det | (1 << so)


def apply_string(vec: dict, ops) -> dict:
    """Apply a product of spin-orbital operators (rightmost acts first).
    ops: list of ('c'|'a', so)."""
    out = vec
    for kind, so in reversed(ops):
        new = {}
        f = cre if kind == "c" else ann
        for det, c in out.items():
            r = f(det, so)
            if r is None:
                continue
            s, d2 = r
            new[d2] = new.get(d2, 0.0) + s * c
        out = new
    return out


def axpy(acc: dict, a: float, vec: dict) -> None:
    for d, c in vec.items():
        acc[d] = acc.get(d, 0.0) + a * c


def apply_E(vec: dict, p: int, q: int, nmo: int) -> dict:
    """Spin-summed E_pq = sum_sigma a+_{p sigma} a_{q sigma}."""
    out: dict = {}
    for s in (0, 1):
        axpy(out, 1.0, apply_string(vec, [("c", s * nmo + p), ("a", s * nmo + q)]))
    return out


def dot(u: dict, v: dict) -> float:
    if len(u) > len(v):
        u, v = v, u
    return sum(c * v.get(d, 0.0) for d, c in u.items())


class BruteSystem:
    """Operators of one problem on explicit determinants."""

    def __init__(self, prob):
        self.p = prob
        self.nmo = prob.nmo
        nc, na = prob.nc, prob.na
        self.clo = list(range(nc))
        self.act = list(range(nc, nc + na))
        self.vir = list(range(nc + na, prob.nmo))
        B = prob.B
        self.eri = np.einsum("Qpq,Qrs->pqrs", B, B)
        # bare one-electron h from h^c: h = h^c - sum_i [2 (xy|ii) - (xi|iy)]
        h = prob.hcore.copy()
        for i in self.clo:
            h -= 2.0 * self.eri[:, :, i, i] - self.eri[:, i, i, :]
        self.h = h
        self.f = prob.fock

    # -- reference states ------------------------------------------------
    def reference_states(self):
        p = self.p
        na, nc, nmo = p.na, p.nc, self.nmo
        from itertools import combinations
        def strs(n):
            return sorted(sum(1 << k for k in c) for c in combinations(range(na), n))
        sa, sb = strs(p.nalpha), strs(p.nbeta)
        core = 0
        for i in self.clo:
            core |= 1 << i
            core |= 1 << (nmo + i)
        states = []
        for N in range(p.nst):
            vec = {}
            for ia, a in enumerate(sa):
                for ib, b in enumerate(sb):
                    c = p.ci[N, ia * len(sb) + ib]
                    if c == 0.0:
                        continue
                    # build |core> with active alpha then active beta creators
                    # in the alpha-string-then-beta-string order of the CI
                    # convention: a+_{a1 al} .. a+_{b1 be} .. |core>
                    ops = [("c", nc + k) for k in range(na) if (a >> k) & 1]
                    ops += [("c", nmo + nc + k) for k in range(na) if (b >> k) & 1]
                    r = apply_string({core: 1.0}, ops)
                    axpy(vec, c, r)
            states.append(vec)
        return states

    # -- operators -------------------------------------------------------
    def apply_fock(self, vec: dict) -> dict:
        out: dict = {}
        f = self.f
        n = self.nmo
        for x in range(n):
            for y in range(n):
                if f[x, y] != 0.0:
                    axpy(out, f[x, y], apply_E(vec, x, y, n))
        const = -2.0 * sum(f[i, i] for i in self.clo)
        axpy(out, const, vec)
        return out

    def apply_ham(self, vec: dict) -> dict:
        n = self.nmo
        out: dict = {}
        Ev = {}
        for x in range(n):
            for y in range(n):
                e = apply_E(vec, x, y, n)
                if e:
                    Ev[(x, y)] = e
        for (x, y), e in Ev.items():
            if self.h[x, y] != 0.0:
                axpy(out, self.h[x, y], e)
        # 1/2 sum (xy|zw) E_xy E_zw
        for (z, w), e in Ev.items():
            for x in range(n):
                for y in range(n):
                    g = self.eri[x, y, z, w]
                    if g != 0.0:
                        axpy(out, 0.5 * g, apply_E(e, x, y, n))
        # -1/2 sum (xy|yw) E_xw  (over every y, also where E_yw |vec> = 0)
        kk = np.einsum("xyyw->xw", self.eri)
        for (x, w), e in Ev.items():
            axpy(out, -0.5 * kk[x, w], e)
        return out


# ---------------------------------------------------------------------------
# internally contracted functions, Eq. 8
# ---------------------------------------------------------------------------

# The nine operator types in the order of Eq. 8: each is E_pq E_rs with the
# orbital classes of (p, q, r, s) ('c' closed, 'a' active, 'v' virtual).
OPERATOR_TYPES = [
    ("ai,bj", "vcvc"), ("ar,bi", "vavc"), ("ar,bs", "vava"), ("ai,rj", "vcac"),
    ("ri,sj", "acac"), ("ar,st", "vaaa"), ("ri,st", "acaa"), ("ai,rs", "vcaa"),
    ("ar,si", "vaac"),
]


def ic_labels(sysm: BruteSystem):
    """Every (type, (p, q, r, s)) of Eq. 8, all index values, all orderings."""
    spaces = {"c": sysm.clo, "a": sysm.act, "v": sysm.vir}
    out = []
    for t, (name, cls) in enumerate(OPERATOR_TYPES):
        for p, q, r, s in itertools.product(*(spaces[c] for c in cls)):
            out.append((t, (p, q, r, s)))
    return out


def solve_brute(prob, scheme: str = "MSMR", xms: bool = True, thresh: float = 1e-9,
                target: int = 0, want_lambda: bool = True, sysm: BruteSystem | None = None,
                fixed_U: np.ndarray | None = None):
    """Galerkin solution of Eq. 10 in the explicit IC space; Eq. 15-17; Eq. 20.

    Returns a dict with U, e0 (E_L^(0)), heff, e_ms, R, and per state L the
    overlap S, operator A_L, source b_L (non-orthogonal, over the IC labels x
    states in the function basis of that L), T_L and lambda_L.
    sysm: operators to use instead of BruteSystem(prob) (e.g. with changed
    integrals); fixed_U: XMS rotation to use instead of diagonalising F^ref
    (derivatives at fixed reference states).
    """
    if sysm is None:
        sysm = BruteSystem(prob)
    n = sysm.nmo
    nst = prob.nst
    refs = sysm.reference_states()
    # XMS rotation, Eq. 3-5
    fref = np.array([[dot(refs[L], sysm.apply_fock(refs[M])) for M in range(nst)]
                     for L in range(nst)])
    if fixed_U is not None:
        U = np.array(fixed_U, dtype=float)
    elif xms:
        w, U = np.linalg.eigh(0.5 * (fref + fref.T))
        for k in range(nst):
            if U[np.argmax(np.abs(U[:, k])), k] < 0:
                U[:, k] = -U[:, k]
    else:
        U = np.eye(nst)
    rot = []
    for M in range(nst):
        v: dict = {}
        for N in range(nst):
            axpy(v, U[N, M], refs[N])
        rot.append(v)
    # Eq. 14: E_L^(0) = <L~| f^ |L~> (only the active part survives)
    fvecs = [sysm.apply_fock(v) for v in rot]
    e0 = np.array([dot(rot[L], fvecs[L]) for L in range(nst)])
    # H^ref_MN = <M~|H|N~>
    hvecs = [sysm.apply_ham(v) for v in rot]
    href = np.array([[dot(rot[M], hvecs[N]) for N in range(nst)] for M in range(nst)])

    labels = ic_labels(sysm)

    def functions(states):
        cols, keys = [], []
        for (t, (p, q, r, s)) in labels:
            for N in states:
                v = apply_E(apply_E(rot[N], r, s, n), p, q, n)
                cols.append(v)
                keys.append((t, (p, q, r, s), N))
        return cols, keys

    out = {"U": U, "e0": e0, "href": href, "fref": fref, "L": {}, "rot": rot, "sysm": sysm,
           "scheme": scheme}
    Ts, Vs, Ss, keys_all, As = [], [], [], [], []
    for L in range(nst):
        states = list(range(nst)) if scheme == "MSMR" else [L]
        if scheme == "MSMR" and L > 0:
            cols, keys, S, Fm = cache
        else:
            cols, keys = functions(states)
            dets = sorted({d for c in cols for d in c})
            index = {d: k for k, d in enumerate(dets)}
            Vm = np.zeros((len(dets), len(cols)))
            for j, c in enumerate(cols):
                for d, val in c.items():
                    Vm[index[d], j] = val
            FV = np.zeros_like(Vm)
            for j, c in enumerate(cols):
                for d, val in sysm.apply_fock(c).items():
                    k = index.get(d)
                    if k is not None:
                        FV[k, j] += val
            S = Vm.T @ Vm
            Fm = Vm.T @ FV
            cache = (cols, keys, S, Fm)
            out.setdefault("Vm", {})[L] = (Vm, dets)
        Vm, dets = out["Vm"][0] if scheme == "MSMR" else out["Vm"][L]
        index = {d: k for k, d in enumerate(dets)}
        A = Fm + (prob.shift - e0[L]) * S
        # sources <M~| E_Omega^+ H |N~> for every N (columns of the ket)
        Vsrc = np.zeros((len(cols), nst))
        for Nk in range(nst):
            hv = np.zeros(len(dets))
            for d, val in hvecs[Nk].items():
                k = index.get(d)
                if k is not None:
                    hv[k] = val
            Vsrc[:, Nk] = Vm.T @ hv
        w, Q = np.linalg.eigh(S)
        keep = w >= thresh
        X = Q[:, keep] / np.sqrt(w[keep])[None, :]
        At = X.T @ A @ X
        b = Vsrc[:, L]
        t = np.linalg.solve(At, -(X.T @ b))
        T = X @ t
        out["L"][L] = dict(S=S, F=Fm, A=A, V=Vsrc, T=T, keys=keys, X=X,
                            eig=w, nkeep=int(keep.sum()))
    # Eq. 15: effective Hamiltonian
    heff = href.copy()
    for L in range(nst):
        for Lp in range(nst):
            dL = out["L"][L]
            dLp = out["L"][Lp]
            heff[L, Lp] += 0.5 * (dL["T"] @ dL["V"][:, Lp] + dLp["T"] @ dLp["V"][:, L])
        dL = out["L"][L]
        heff[L, L] -= prob.shift * dL["T"] @ dL["S"] @ dL["T"]
    w, R = np.linalg.eigh(0.5 * (heff + heff.T))
    for k in range(nst):
        if R[np.argmax(np.abs(R[:, k])), k] < 0:
            R[:, k] = -R[:, k]
    out.update(heff=heff, e_ms=w, R=R)
    if want_lambda:
        P = target
        for L in range(nst):
            dL = out["L"][L]
            src = R[L, P] * (dL["V"] @ R[:, P]) - 2.0 * prob.shift * R[L, P] ** 2 * (dL["S"] @ dL["T"])
            X = dL["X"]
            At = X.T @ dL["A"] @ X
            lt = np.linalg.solve(At, -(X.T @ src))
            dL["lam"] = X @ lt
        out["target"] = P
    return out


# ---------------------------------------------------------------------------
# correlated density matrices, Sec. II.D
# ---------------------------------------------------------------------------

def _first_order_vector(out, L, coef) -> dict:
    """sum_k coef[k] E_Omega(k)|N~> over the function set of state L, as an
    explicit determinant expansion."""
    Vm, dets = out["Vm"][0] if out["scheme"] == "MSMR" else out["Vm"][L]
    v = Vm @ coef
    return {d: c for d, c in zip(dets, v) if c != 0.0}


def _apply_E2(vec: dict, x: int, y: int, z: int, w: int, n: int) -> dict:
    """E_xy,zw = E_xy E_zw - delta_yz E_xw (the two-particle excitation)."""
    r = apply_E(apply_E(vec, z, w, n), x, y, n)
    if y == z:
        axpy(r, -1.0, apply_E(vec, x, w, n))
    return r


def densities_brute(prob, out) -> dict:
    """The correlated densities of Sec. II.D written out on explicit
    determinants, from a solve_brute result with lambda (target P):

      |P> = sum_M |M~> R_MP,   T_PN = sum_M T_MN R_MP (mixed states),
      d1_xy   = sum_M <M~|T_PM^+ E_xy|P> + sum_MN <M~|lambda_NM^+ E_xy|N~>,
      D1_xyzw = the same with E_xy,zw = E_xy E_zw - delta_yz E_xw,
      dbar2_xy = sum_LMN <M~|lambda_LM^+ E_xy T_LN|N~>,
      N_L = sum_MN <M~|lambda_LM^+ T_LN|N~>  (the dagger the printed N_L lacks),
      d2_xy = dbar2_xy - sum_L N_L <L~|E_xy|L~> for active x, y; dbar2_xy otherwise.

    Orbital indices are absolute (closed | active | virtual).  Also returned:
    gamma_P = <P|E_xy|P> and Gamma_P = <P|E_xy,zw|P> (the reference part,
    needed by the finite-difference checks)."""
    sysm, rot = out["sysm"], out["rot"]
    n = sysm.nmo
    nst = prob.nst
    P = out["target"]
    R = out["R"]
    Pv: dict = {}
    for M in range(nst):
        axpy(Pv, R[M, P], rot[M])
    psi = [_first_order_vector(out, L, out["L"][L]["T"]) for L in range(nst)]
    lam = [_first_order_vector(out, L, out["L"][L]["lam"]) for L in range(nst)]
    # T_P = sum_L R_LP Psi1_L  (the bra of the first term of d1 and D1)
    tp: dict = {}
    for L in range(nst):
        axpy(tp, R[L, P], psi[L])
    d1 = np.zeros((n, n))
    D1 = np.zeros((n, n, n, n))
    gam = np.zeros((n, n))
    Gam = np.zeros((n, n, n, n))
    for x in range(n):
        for y in range(n):
            eP = apply_E(Pv, x, y, n)
            gam[x, y] = dot(Pv, eP)
            d1[x, y] = dot(tp, eP) + sum(dot(lam[N], apply_E(rot[N], x, y, n)) for N in range(nst))
            for z in range(n):
                for w in range(n):
                    e2 = _apply_E2(Pv, x, y, z, w, n)
                    Gam[x, y, z, w] = dot(Pv, e2)
                    D1[x, y, z, w] = dot(tp, e2) + sum(dot(lam[N], _apply_E2(rot[N], x, y, z, w, n))
                                                       for N in range(nst))
    dbar2 = np.zeros((n, n))
    for x in range(n):
        for y in range(n):
            dbar2[x, y] = sum(dot(lam[L], apply_E(psi[L], x, y, n)) for L in range(nst))
    NL = np.array([dot(lam[L], psi[L]) for L in range(nst)])
    d2 = dbar2.copy()
    act = range(prob.nc, prob.nc + prob.na)
    for L in range(nst):
        for r in act:
            for t in act:
                d2[r, t] -= NL[L] * dot(rot[L], apply_E(rot[L], r, t, n))
    return dict(d1=d1, D1=D1, dbar2=dbar2, NL=NL, d2=d2, gamma_P=gam, Gamma_P=Gam)
