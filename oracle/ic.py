"""O2: the scalable CPU oracle for the (X)MS-CASPT2 amplitude and lambda
equations.  TEST INFRASTRUCTURE ONLY: only tests/, __graft_entry__.smoke()
and bench.py's cpu_baseline leg may use anything under oracle/.

What is computed (paper Sec. II.A-II.C):
  * XMS rotation of the reference states (Eqs. 3-5; U = 1 gives MS-CASPT2),
  * E_L^(0) (Eq. 14), H^ref (Eq. 6),
  * the amplitude equation Eq. 10 for every state L, in the internally
    contracted space spanned by E_Omega |N~> (Eq. 7 MS-MR, Eq. 9 SS-SR) with
    the nine operator types of Eq. 8 in product form, after removing overlap
    eigenvalues below the threshold (Sec. II.B),
  * the effective Hamiltonian Eq. 15, its eigenpairs (Eqs. 16-17),
  * the lambda equation Eq. 20 for a target state P.

How matrix elements are evaluated.  The reference |N> is the closed core
(doubly occupied) times an active CI vector; virtual orbitals are empty.
Every product of spin-orbital operators that appears in a matrix element
<core,M| Y |core,N> is split, by a stable reordering that moves all closed
and virtual operators to the left (with the sign of that permutation), into
an external string and an active string; then

    <core,M| Y |core,N> = sign * <core| Y_ext |core> * <M| Y_act |N>.

<core|Y_ext|core> is a sum over pairings (Wick contractions) of external
operators; each pairing identifies two orbital labels.  The value of one
pairing is obtained by placing every identified pair on its own concrete
orbital and applying the string to an explicit determinant.  <M|Y_act|N> is
an inner product of operator-applied CI vectors (the active-space reduced
density matrices of the paper's Eq. 38, up to Gamma_3 and the Fock-contracted
Gamma_4, formed here as products of vectors instead of being stored).

Amplitudes are held in the packed layout of the C ABI (one row per external
orbit and character, one column per compound active index); internally the
oracle works on all orderings of the external indices and packs at the end.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from functools import lru_cache

import numpy as np

CLO, ACT, VIR = "c", "a", "v"

# ---------------------------------------------------------------------------
# active space: sector strings and spin-orbital operators on CI vectors
# ---------------------------------------------------------------------------


class ActiveSpace:
    """Determinant sectors (n_alpha, n_beta) over na active orbitals.

    Vectors are arrays [..., n_alpha_strings, n_beta_strings]; a determinant
    is alpha creators (ascending orbital) to the left of beta creators
    (ascending orbital) acting on the vacuum."""

    def __init__(self, na: int):
        self.na = na
        self._strs = {}
        self._maps = {}

    def strings(self, n: int) -> np.ndarray:
        if n not in self._strs:
            if n < 0 or n > self.na:
                self._strs[n] = np.zeros(0, dtype=np.int64)
            else:
                self._strs[n] = np.array(sorted(sum(1 << k for k in c)
                                                for c in itertools.combinations(range(self.na), n)),
                                         dtype=np.int64)
        return self._strs[n]

    def dim(self, sector) -> tuple[int, int]:
        return len(self.strings(sector[0])), len(self.strings(sector[1]))

    def _map(self, kind: str, r: int, n: int):
        """Map strings with n electrons under a_r (kind 'a') or a+_r ('c'):
        (source positions, target positions, parity of electrons below r)."""
        key = (kind, r, n)
        if key not in self._maps:
            src = self.strings(n)
            n2 = n - 1 if kind == "a" else n + 1
            tgt = {int(s): k for k, s in enumerate(self.strings(n2))}
            si, ti, par = [], [], []
            for k, s in enumerate(src):
                s = int(s)
                occ = (s >> r) & 1
                if (kind == "a" and not occ) or (kind == "c" and occ):
                    continue
                t = s ^ (1 << r)
                si.append(k)
                ti.append(tgt[t])
                par.append(bin(s & ((1 << r) - 1)).count("1") % 2)
            self._maps[key] = (np.array(si, dtype=np.int64), np.array(ti, dtype=np.int64),
                               np.array(par, dtype=np.int64))
        return self._maps[key]

    def apply(self, kind: str, r: int, spin: int, vec: np.ndarray, sector):
        """Apply a_{r spin} ('a') or a+_{r spin} ('c') to vec in sector."""
        na_, nb_ = sector
        d = -1 if kind == "a" else 1
        if spin == 0:
            new = (na_ + d, nb_)
            si, ti, par = self._map(kind, r, na_)
            out = np.zeros(vec.shape[:-2] + self.dim(new))
            sgn = np.where(par == 1, -1.0, 1.0)
            if len(si):
                out[..., ti, :] = vec[..., si, :] * sgn[:, None]
        else:
            new = (na_, nb_ + d)
            si, ti, par = self._map(kind, r, nb_)
            out = np.zeros(vec.shape[:-2] + self.dim(new))
            sgn = np.where(par == 1, -1.0, 1.0) * (-1.0 if na_ % 2 else 1.0)
            if len(si):
                out[..., :, ti] = vec[..., :, si] * sgn[None, :]
        return out, new


# ---------------------------------------------------------------------------
# operator strings with labels
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Op:
    kind: str      # 'c' creator, 'a' annihilator
    label: str     # orbital label
    space: str     # 'c', 'a', 'v'
    spin: str      # spin variable name


def E(p: str, sp: str, q: str, sq: str, spin: str):
    """One spin-summed excitation E_pq as the pair a+_{p s} a_{q s}."""
    return [Op("c", p, sp, spin), Op("a", q, sq, spin)]


def dagger(ops):
    return [Op("a" if o.kind == "c" else "c", o.label, o.space, o.spin) for o in reversed(ops)]


# ---------------------------------------------------------------------------
# the eight blocks (Eq. 8; E_ai,rs and E_ar,si share one block)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Block:
    name: str
    ext: list          # [(label, space)] external slots in storage order
    act: list          # active labels in storage order
    types: list        # operator strings (one per operator type)
    swaps: list        # list of (slot k, slot l) pairs that may be exchanged


def _blocks():
    s, t = "s1", "s2"
    return [
        Block("ccvv", [("i", CLO), ("j", CLO), ("a", VIR), ("b", VIR)], [],
              [E("a", VIR, "i", CLO, s) + E("b", VIR, "j", CLO, t)], [(0, 1), (2, 3)]),
        Block("cavv", [("i", CLO), ("a", VIR), ("b", VIR)], ["r"],
              [E("a", VIR, "r", ACT, s) + E("b", VIR, "i", CLO, t)], [(1, 2)]),
        Block("aavv", [("a", VIR), ("b", VIR)], ["r", "s"],
              [E("a", VIR, "r", ACT, s) + E("b", VIR, "s", ACT, t)], [(0, 1)]),
        Block("ccav", [("i", CLO), ("j", CLO), ("a", VIR)], ["r"],
              [E("a", VIR, "i", CLO, s) + E("r", ACT, "j", CLO, t)], [(0, 1)]),
        Block("ccaa", [("i", CLO), ("j", CLO)], ["r", "s"],
              [E("r", ACT, "i", CLO, s) + E("s", ACT, "j", CLO, t)], [(0, 1)]),
        Block("aaav", [("a", VIR)], ["r", "s", "t"],
              [E("a", VIR, "r", ACT, s) + E("s", ACT, "t", ACT, t)], []),
        Block("caaa", [("i", CLO)], ["r", "s", "t"],
              [E("r", ACT, "i", CLO, s) + E("s", ACT, "t", ACT, t)], []),
        Block("caav", [("i", CLO), ("a", VIR)], ["r", "s"],
              [E("a", VIR, "i", CLO, s) + E("r", ACT, "s", ACT, t),
               E("a", VIR, "r", ACT, s) + E("s", ACT, "i", CLO, t)], []),
    ]


BLOCKS = _blocks()
BLOCK_NAMES = [b.name for b in BLOCKS]


# ---------------------------------------------------------------------------
# external strings on concrete orbitals (closed: occupied, virtual: empty)
# ---------------------------------------------------------------------------

def _ext_value(ops, orb_of_label, spins, nclo):
    """<core| ops |core> with concrete orbitals; spin orbital = 2*orb + spin.
    Closed concrete orbitals are 0..nclo-1 (doubly occupied)."""
    det = 0
    for k in range(nclo):
        det |= 0b11 << (2 * k)
    coeff = 1.0
    for o in reversed(ops):
        so = 2 * orb_of_label[o.label] + spins[o.spin]
        occ = (det >> so) & 1
        below = bin(det & ((1 << so) - 1)).count("1")
        if o.kind == "a":
            if not occ:
                return 0.0
            det &= ~(1 << so)
        else:
            if occ:
                return 0.0
            det |= 1 << so
        if below % 2:
            coeff = -coeff
    ref = 0
    for k in range(nclo):
        ref |= 0b11 << (2 * k)
    return coeff if det == ref else 0.0


def _pairings(ext_ops):
    """All ways of pairing external operators that can contract on the core
    vacuum: a virtual annihilator with a virtual creator, a closed creator
    with a closed annihilator.  Yields lists of (label, label)."""
    va = [o.label for o in ext_ops if o.space == VIR and o.kind == "a"]
    vc = [o.label for o in ext_ops if o.space == VIR and o.kind == "c"]
    cc = [o.label for o in ext_ops if o.space == CLO and o.kind == "c"]
    ca = [o.label for o in ext_ops if o.space == CLO and o.kind == "a"]
    if len(va) != len(vc) or len(cc) != len(ca):
        return
    for pv in itertools.permutations(vc):
        for pc in itertools.permutations(ca):
            yield list(zip(va, pv)) + list(zip(cc, pc))


# ---------------------------------------------------------------------------
# generic matrix element engine
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Term:
    """One Wick pairing of <bra| op |ket>: label classes and, per spin
    assignment, the coefficient and the active string."""
    classes: list          # list of frozensets of labels identified together
    active: list           # list of (coeff, bra_act_ops, mid_act_ops, ket_act_ops) per spin set


def _spin_vars(ops):
    out = []
    for o in ops:
        if o.spin not in out:
            out.append(o.spin)
    return out


def matrix_element_terms(bra_ops, op_ops, ket_ops):
    """Decompose sum_spins <core,M| bra^+ op ket |core,N> into pairings.

    bra_ops / ket_ops: operator strings of the bra / ket functions (labels of
    the two must be distinct); op_ops: the operator between them.
    Returns {frozenset(classes): [(coeff, bra_act, mid_act, ket_act, spins)]}.
    """
    Y = dagger(bra_ops) + list(op_ops) + list(ket_ops)
    nb = len(bra_ops)
    nm = len(op_ops)
    region = ["b"] * nb + ["m"] * nm + ["k"] * len(ket_ops)
    ext_idx = [k for k, o in enumerate(Y) if o.space != ACT]
    act_idx = [k for k, o in enumerate(Y) if o.space == ACT]
    # sign of the stable partition (ext first): count inversions
    inv = 0
    for k in act_idx:
        inv += sum(1 for e in ext_idx if e > k)
    psign = -1.0 if inv % 2 else 1.0
    ext_ops = [Y[k] for k in ext_idx]
    svars = _spin_vars(Y)
    out = {}
    for pairing in _pairings(ext_ops):
        # concrete orbitals: one per pair; closed pairs 0.., virtual after
        orb = {}
        nclo = sum(1 for (x, y) in pairing if _space_of(ext_ops, x) == CLO)
        kc, kv = 0, nclo
        for (x, y) in pairing:
            if _space_of(ext_ops, x) == CLO:
                orb[x] = orb[y] = kc
                kc += 1
            else:
                orb[x] = orb[y] = kv
                kv += 1
        classes = frozenset(frozenset(p) for p in pairing)
        entries = []
        for svals in itertools.product((0, 1), repeat=len(svars)):
            spins = dict(zip(svars, svals))
            v = _ext_value(ext_ops, orb, spins, nclo)
            if v == 0.0:
                continue
            bra_act = [(o, spins[o.spin]) for o in bra_ops if o.space == ACT]
            mid_act = [(o, spins[o.spin]) for o in op_ops if o.space == ACT]
            ket_act = [(o, spins[o.spin]) for o in ket_ops if o.space == ACT]
            entries.append((psign * v, bra_act, mid_act, ket_act))
        if entries:
            out[classes] = entries
    return out


def _space_of(ops, label):
    for o in ops:
        if o.label == label:
            return o.space
    raise KeyError(label)


def _relabel(ops, suffix):
    return [Op(o.kind, o.label + suffix, o.space, o.spin + suffix) for o in ops]


# ---------------------------------------------------------------------------
# active factors: operator-applied CI vectors and their inner products
# ---------------------------------------------------------------------------

def _apply_string(space: ActiveSpace, ops_spins, base: np.ndarray, sector):
    """Apply an active string (rightmost first) to base [nst, A, B].

    Every label becomes a leading axis (in order of first application from
    the right); returns (array [labels..., nst, A', B'], label list, sector)."""
    arr, labels, sec = base, [], sector
    if ops_spins and space.na == 0:
        return None, None, None
    for (o, s) in reversed(ops_spins):
        outs = []
        new_sec = None
        for r in range(space.na):
            v, new_sec = space.apply(o.kind, r, s, arr, sec)
            outs.append(v)
        if new_sec[0] < 0 or new_sec[1] < 0 or new_sec[0] > space.na or new_sec[1] > space.na:
            return None, None, None
        arr = np.stack(outs, axis=0)
        labels = [o.label] + labels
        sec = new_sec
    return arr, labels, sec


def _apply_onebody(space: ActiveSpace, C: np.ndarray, spin: int, vec: np.ndarray, sector):
    """sum_xy C[x, y] a+_{x spin} a_{y spin} applied to vec (same sector)."""
    Z, sec1 = [], None
    for y in range(space.na):
        v, sec1 = space.apply("a", y, spin, vec, sector)
        Z.append(v)
    if sec1 is None or min(sec1) < 0:
        return np.zeros_like(vec)
    Zc = np.tensordot(C, np.stack(Z, axis=0), axes=([1], [0]))
    out = np.zeros_like(vec)
    for x in range(space.na):
        w, _ = space.apply("c", x, spin, Zc[x], sec1)
        out += w
    return out


def active_gram(space, ci, sector, bra_act, mid_act, ket_act, ket_base=None, mid_coef=None):
    """G[mid labels..., bra labels..., M, ket labels..., N] =
    <M| (bra string)^+ (mid string) (ket string) |N>.  Labels are returned
    with the axis order.  ket_base replaces ci on the ket side (sources).
    With mid_coef, the mid string must be a+_x a_y of one spin and is summed
    with the coefficients mid_coef[x, y] before the inner product (no mid
    axes in G)."""
    kb = ci if ket_base is None else ket_base
    U, ul, us = _apply_string(space, bra_act, ci, sector)
    if mid_coef is not None:
        W, wl, ws = _apply_string(space, list(ket_act), kb, sector)
        if W is not None:
            (ox, sx), (oy, sy) = mid_act
            assert ox.kind == "c" and oy.kind == "a" and sx == sy
            W = _apply_onebody(space, mid_coef, sx, W, ws)
        nm = 0
    else:
        W, wl, ws = _apply_string(space, list(mid_act) + list(ket_act), kb, sector)
        nm = len(mid_act)
    if U is None or W is None or us != ws:
        return None, None
    nu = len(ul)
    nw = len(wl)
    # mid labels come first in wl (they were applied last), ket labels after
    G = np.tensordot(U, W, axes=([nu + 1, nu + 2], [nw + 1, nw + 2]))
    # G axes: [ul..., M, wl..., N]; reorder to [mid..., ul..., M, ket..., N]
    ax_ul = list(range(nu))
    ax_M = [nu]
    ax_mid = list(range(nu + 1, nu + 1 + nm))
    ax_ket = list(range(nu + 1 + nm, nu + 1 + nw))
    ax_N = [nu + 1 + nw]
    G = np.transpose(G, ax_mid + ax_ul + ax_M + ax_ket + ax_N)
    return G, (wl[:nm], ul, wl[nm:])


# ---------------------------------------------------------------------------
# the oracle proper
# ---------------------------------------------------------------------------

_LETTERS = "abcdefghijklmnopqrstuvwxyz"


class Caspt2Oracle:
    """Plain FP64 evaluation of Eq. 10 / Eq. 15-17 / Eq. 20 for one problem."""

    def __init__(self, prob, scheme: str = "MSMR", xms: bool = True, thresh: float = 1e-9,
                 rotate_states: np.ndarray | None = None):
        assert scheme in ("MSMR", "SSSR")
        self.p = prob
        self.scheme = scheme
        self.thresh = thresh
        nc, na, nv = prob.nc, prob.na, prob.nv
        self.nc, self.na, self.nv, self.nst = nc, na, nv, prob.nst
        self.sl = {CLO: slice(0, nc), ACT: slice(nc, nc + na), VIR: slice(nc + na, nc + na + nv)}
        self.dimsp = {CLO: nc, ACT: na, VIR: nv}
        self.space = ActiveSpace(na)
        self.sector = (prob.nalpha, prob.nbeta)
        A, Bn = self.space.dim(self.sector)
        ci = prob.ci.reshape(prob.nst, A, Bn).copy()
        if rotate_states is not None:       # arbitrary orthogonal pre-rotation of inputs
            ci = np.einsum("NM,NAB->MAB", rotate_states, ci)
        self.ci_raw = ci
        self.f = prob.fock
        # --- XMS, Eqs. 3-5 -------------------------------------------------
        fa = self.f[self.sl[ACT], self.sl[ACT]]
        self.fref = self._one_body(fa, ci)
        if xms:
            w, U = np.linalg.eigh(0.5 * (self.fref + self.fref.T))
            for k in range(self.nst):
                if U[np.argmax(np.abs(U[:, k])), k] < 0:
                    U[:, k] = -U[:, k]
        else:
            U = np.eye(self.nst)
        self.U = U
        self.ci = np.einsum("NAB,NM->MAB", ci, U)
        # Eq. 14
        fr = self._one_body(fa, self.ci)
        self.e0 = np.diag(fr).copy()
        # H^ref (Eq. 6): CI vectors are eigenvectors of H_act
        eref = prob.eref if rotate_states is None else None
        if eref is None:
            # energies are invariant; the input rotation mixes states of H
            hr = rotate_states.T @ np.diag(prob.eref) @ rotate_states
        else:
            hr = np.diag(eref)
        self.href = U.T @ hr @ U
        # --- integrals ---------------------------------------------------
        self.B = prob.B
        self._eri_cache = {}
        # --- layout ------------------------------------------------------
        self.ntup = {b.name: na ** len(b.act) for b in BLOCKS}
        self.nstα = self.nst if scheme == "MSMR" else 1
        self.nalpha = {b.name: self.nstα * len(b.types) * self.ntup[b.name] for b in BLOCKS}
        self._gram_cache = {}
        self._plans = {}
        self.layout = self._make_layout()

    # -- helpers ----------------------------------------------------------
    def _one_body(self, fa, ci):
        """<M| sum_rs fa_rs E_rs |N>."""
        nst = ci.shape[0]
        out = np.zeros((nst, nst))
        for r in range(self.na):
            for s in range(self.na):
                if fa[r, s] == 0.0:
                    continue
                for sp in (0, 1):
                    v, sec = self.space.apply("a", s, sp, ci, self.sector)
                    v, sec = self.space.apply("c", r, sp, v, sec)
                    out += fa[r, s] * np.einsum("MAB,NAB->MN", ci, v)
        return out

    def eri(self, spaces):
        if spaces not in self._eri_cache:
            p, q, r, s = (self.sl[x] for x in spaces)
            B1 = self.B[:, p, q]
            B2 = self.B[:, r, s]
            self._eri_cache[spaces] = np.einsum("Qpq,Qrs->pqrs", B1, B2, optimize=True)
        return self._eri_cache[spaces]

    def states_of(self, L):
        return list(range(self.nst)) if self.scheme == "MSMR" else [L]

    # -- layout (packed, the C ABI order) ----------------------------------
    def _characters(self, b: Block):
        if b.name == "ccvv":
            return [(1, 1), (-1, -1)]
        if b.swaps:
            return [(1,), (-1,)]
        return [()]

    def _orbits(self, b: Block, chi):
        """Canonical orbit representatives in storage order."""
        dims = [self.dimsp[sp] for (_, sp) in b.ext]
        reps = []
        # iterate slots in storage order; a swap (k, l) requires e[k] >= e[l]
        # (strictly for a -1 character)
        for e in itertools.product(*(range(d) for d in dims)):
            ok = True
            for (k, l), c in zip(b.swaps, chi):
                if e[k] < e[l] or (c == -1 and e[k] == e[l]):
                    ok = False
            if ok:
                reps.append(e)
        # storage order: pair indices row-major; itertools order is lexicographic
        # in the slots, which for (k,l) adjacent pairs with e[k] >= e[l] equals
        # ascending pair index k(k+1)/2 + l (or k(k-1)/2 + l).
        return reps

    def _make_layout(self):
        lay = []
        off = 0
        for b in BLOCKS:
            for chi in self._characters(b):
                reps = self._orbits(b, chi)
                n = len(reps) * self.nalpha[b.name]
                lay.append(dict(block=b, chi=chi, reps=reps, offset=off, nrow=len(reps),
                                nalpha=self.nalpha[b.name]))
                off += n
        self.length = off
        return lay

    def _orbit_images(self, b, e0):
        """Distinct images of e0 under the swap group with the swap subset."""
        imgs = {}
        for bits in itertools.product((0, 1), repeat=len(b.swaps)):
            e = list(e0)
            for (k, l), f in zip(b.swaps, bits):
                if f:
                    e[k], e[l] = e[l], e[k]
            imgs.setdefault(tuple(e), bits)
        return imgs

    def _pack_maps(self, ent):
        """Per layout entry: flat indices of the images of every orbit
        representative and their weights chi(pi_e) / sqrt(|orbit|)."""
        if "maps" in ent:
            return ent["maps"]
        b, chi = ent["block"], ent["chi"]
        dims = tuple(self.dimsp[sp] for (_, sp) in b.ext)
        nimg = 1 << len(b.swaps)
        idx = np.zeros((nimg, ent["nrow"]), dtype=np.int64)
        coef = np.zeros((nimg, ent["nrow"]))
        for r, e0 in enumerate(ent["reps"]):
            imgs = self._orbit_images(b, e0)
            w = 1.0 / math.sqrt(len(imgs))
            for k, (e, bits) in enumerate(imgs.items()):
                sgn = 1.0
                for c, f in zip(chi, bits):
                    if f:
                        sgn *= c
                idx[k, r] = np.ravel_multi_index(e, dims) if dims else 0
                coef[k, r] = w * sgn
        ent["maps"] = (idx, coef)
        return ent["maps"]

    def pack(self, xall: dict) -> np.ndarray:
        """All orderings -> packed rows x_chi[orbit] = sum_e w chi(pi_e) x[e]."""
        out = np.zeros(self.length)
        for ent in self.layout:
            b = ent["block"]
            if ent["nrow"] == 0 or ent["nalpha"] == 0:
                continue
            idx, coef = self._pack_maps(ent)
            arr = xall[b.name].reshape(-1, ent["nalpha"])
            rows = np.einsum("kr,krA->rA", coef, arr[idx])
            out[ent["offset"]: ent["offset"] + ent["nrow"] * ent["nalpha"]] = rows.ravel()
        return out

    def unpack(self, x: np.ndarray) -> dict:
        """Packed rows -> all orderings (the transpose of pack)."""
        xall = {}
        for b in BLOCKS:
            shape = tuple(self.dimsp[sp] for (_, sp) in b.ext) + (self.nalpha[b.name],)
            xall[b.name] = np.zeros(shape)
        for ent in self.layout:
            b = ent["block"]
            if ent["nrow"] == 0 or ent["nalpha"] == 0:
                continue
            idx, coef = self._pack_maps(ent)
            blk = x[ent["offset"]: ent["offset"] + ent["nrow"] * ent["nalpha"]].reshape(ent["nrow"], ent["nalpha"])
            flat = xall[b.name].reshape(-1, ent["nalpha"])
            for k in range(idx.shape[0]):
                np.add.at(flat, idx[k], coef[k][:, None] * blk)
        return xall

    # -- operator terms ------------------------------------------------------
    def _gram(self, key, bra_act, mid_act, ket_act, ket_base=None, mid_coef=None):
        G, labels = active_gram(self.space, self.ci, self.sector, bra_act, mid_act, ket_act,
                                ket_base=ket_base, mid_coef=mid_coef)
        return G, labels

    def _block_pair_terms(self, bb: Block, op_ops, kb: Block | None, mid_coef=None):
        """Collect, per pairing, the summed active tensor for <bra| op |ket>.

        Returns list of (classes, op_labels, G[opact..., alpha_bra, alpha_ket]).
        alpha = (state, type, tuple); for kb None the ket is |L> and
        alpha_ket runs over the ket state only."""
        out = {}
        nst = self.nst
        for tb, tmpl_b in enumerate(bb.types):
            bra = [Op(o.kind, o.label + "_b", o.space, o.spin + "_b") for o in tmpl_b]
            ket_types = [None] if kb is None else list(enumerate(kb.types))
            for tk_entry in ket_types:
                if kb is None:
                    tk, ket = 0, []
                else:
                    tk, tmpl_k = tk_entry
                    ket = [Op(o.kind, o.label + "_k", o.space, o.spin + "_k") for o in tmpl_k]
                terms = matrix_element_terms(bra, op_ops, ket)
                for classes, entries in terms.items():
                    acc = out.get(classes)
                    for (coef, bra_act, mid_act, ket_act) in entries:
                        G, labels = self._gram(None, bra_act, mid_act, ket_act, mid_coef=mid_coef)
                        if G is None:
                            continue
                        mid_l, bra_l, ket_l = labels
                        # reorder label axes to block storage order
                        bra_order = [lbl + "_b" for lbl in bb.act]
                        ket_order = [] if kb is None else [lbl + "_k" for lbl in kb.act]
                        mid_order = [] if mid_coef is not None else [o.label for o in op_ops if o.space == ACT]
                        nm, nb_, nk = len(mid_l), len(bra_l), len(ket_l)
                        perm = ([mid_l.index(x) for x in mid_order]
                                + [nm + bra_l.index(x) for x in bra_order]
                                + [nm + nb_]
                                + [nm + nb_ + 1 + ket_l.index(x) for x in ket_order]
                                + [nm + nb_ + 1 + nk])
                        G = np.transpose(G, perm)
                        # flatten to [mid..., alpha_b, alpha_k] with alpha = (state, type, tuple)
                        nt_b = self.ntup[bb.name]
                        nt_k = 1 if kb is None else self.ntup[kb.name]
                        G = G.reshape(G.shape[:nm] + (nt_b, nst, nt_k, nst))
                        if acc is None:
                            nty_b = len(bb.types)
                            nty_k = 1 if kb is None else len(kb.types)
                            acc = np.zeros(G.shape[:nm] + (nst, nty_b, nt_b, nst, nty_k, nt_k))
                        # acc[..., M, tb, tupb, N, tk, tupk]
                        Gt = np.moveaxis(G, nm + 1, nm)          # [..., M, tupb, tupk, N]
                        Gt = np.moveaxis(Gt, nm + 3, nm + 2)     # [..., M, tupb, N, tupk]
                        acc[..., :, tb, :, :, tk, :] += coef * Gt
                    if acc is not None:
                        out[classes] = acc
        res = []
        for classes, acc in out.items():
            nm = acc.ndim - 6
            sh = acc.shape
            res.append((classes, acc.reshape(sh[:nm] + (sh[nm] * sh[nm + 1] * sh[nm + 2],
                                                         sh[nm + 3] * sh[nm + 4] * sh[nm + 5]))))
        return res

    # -- operator components ----------------------------------------------
    def fock_components(self):
        """f^ = sum_xy f_xy E_xy - 2 sum_i f_ii (Eq. 11-12), split by orbital
        classes of (x, y); every piece is an (ops, coefficient, C labels)."""
        comps = []
        f = self.f
        for sx in (CLO, ACT, VIR):
            for sy in (CLO, ACT, VIR):
                blk = f[self.sl[sx], self.sl[sy]]
                if blk.size == 0 or not np.any(blk):
                    continue
                ops = E("x_o", sx, "y_o", sy, "so")
                comps.append((ops, blk, ["x_o", "y_o"]))
        return comps

    def ham_components(self):
        """The part of H that acts on |core, L> with something left (closed
        creators and virtual annihilators removed), one-body part h^c:
        sum_{p in av, q in ac} h^c_pq E_pq
        + 1/2 sum_{p,r in av; q,s in ac} (pq|rs) a+_p a+_r a_s a_q."""
        comps = []
        hc = self.p.hcore
        for sp in (ACT, VIR):
            for sq in (ACT, CLO):
                if sp == ACT and sq == ACT:
                    continue
                blk = hc[self.sl[sp], self.sl[sq]]
                if blk.size == 0:
                    continue
                comps.append((E("p_o", sp, "q_o", sq, "so"), blk, ["p_o", "q_o"]))
        for sp, sq, sr, ss in itertools.product((ACT, VIR), (ACT, CLO), (ACT, VIR), (ACT, CLO)):
            if sp == sq == sr == ss == ACT:
                continue
            if 0 in (self.dimsp[sp], self.dimsp[sq], self.dimsp[sr], self.dimsp[ss]):
                continue
            ops = [Op("c", "p_o", sp, "so"), Op("c", "r_o", sr, "to"),
                   Op("a", "s_o", ss, "to"), Op("a", "q_o", sq, "so")]
            comps.append((ops, 0.5 * self.eri((sp, sq, sr, ss)), ["p_o", "q_o", "r_o", "s_o"]))
        return comps

    def _spec(self, bb, kb, op_ops, clabels, classes):
        letters = iter(_LETTERS)
        cl = {}
        for c in classes:
            l = next(letters)
            for lab in c:
                cl[lab] = l
        for o in op_ops:
            if o.space == ACT and o.label not in cl:
                cl[o.label] = next(letters)
        out = "".join(cl[lab + "_b"] for (lab, _) in bb.ext) + "Y"
        c_str = "".join(cl[lab] for lab in clabels)
        mid = [o.label for o in op_ops if o.space == ACT]
        g_str = "".join(cl[lab] for lab in mid) + "YZ"
        if kb is None:
            return f"{c_str},{g_str}->{out}Z"
        x_str = "".join(cl[lab + "_k"] for (lab, _) in kb.ext) + "Z"
        return f"{c_str},{g_str},{x_str}->{out}"

    def _plan(self, key, bb, kb, op_ops, coef, clabels, precontract=False):
        """Einsum plans of <bra| op |ket> per pairing.  With precontract the
        op is a one-body operator on active orbitals whose coefficients are
        summed into the ket vectors first; the plan then takes C = 1."""
        if key not in self._plans:
            if precontract:
                terms = self._block_pair_terms(bb, op_ops, kb, mid_coef=coef)
                self._plans[key] = [(self._spec(bb, kb, [], [], classes), G, classes)
                                    for classes, G in terms]
            else:
                terms = self._block_pair_terms(bb, op_ops, kb)
                self._plans[key] = [(self._spec(bb, kb, op_ops, clabels, classes), G, classes)
                                    for classes, G in terms]
        return [(s, coef, G, c) for (s, G, c) in self._plans[key]]

    def _alpha_slice(self, b: Block, L: int):
        """Columns of the all-states alpha that belong to state L (SS-SR)."""
        n = len(b.types) * self.ntup[b.name]
        return slice(L * n, (L + 1) * n)

    def _restrict(self, G, bb, kb, L):
        if self.scheme == "MSMR":
            return G
        sb = self._alpha_slice(bb, L)
        if kb is None:
            return G[..., sb, :]
        return G[..., sb, self._alpha_slice(kb, L)]

    # -- residual, Eq. 10 ----------------------------------------------------
    def apply_A(self, L: int, xall: dict) -> dict:
        """(f^ - E_L^(0) + E_s) restricted to the IC space, on all orderings."""
        out = {b.name: np.zeros_like(xall[b.name]) for b in BLOCKS}
        shiftL = self.p.shift - self.e0[L] - 2.0 * np.trace(self.f[self.sl[CLO], self.sl[CLO]])
        for bb in BLOCKS:
            for kb in BLOCKS:
                x = xall[kb.name]
                # scalar part: (E_s - E_L - 2 tr f_cc) times the overlap
                if bb is kb:
                    for spec, _, G, _ in self._plan(("S", bb.name), bb, kb, [], 1.0, []):
                        Gr = self._restrict(G, bb, kb, L)
                        s2 = spec.split(",", 1)[1]
                        out[bb.name] += shiftL * np.einsum(s2, Gr, x, optimize=True)
                for ci_, (ops, C, clabels) in enumerate(self.fock_components()):
                    key = ("F", ci_, bb.name, kb.name)
                    pre = all(o.space == ACT for o in ops)
                    for spec, _, G, _ in self._plan(key, bb, kb, ops, C, clabels, precontract=pre):
                        Gr = self._restrict(G, bb, kb, L)
                        Cx = np.float64(1.0) if pre else C
                        out[bb.name] += np.einsum(spec, Cx, Gr, x, optimize=True)
        return out

    def sources(self) -> dict:
        """V^(N)[e, alpha] = <f_{e,alpha}| H |N~> for every ket N (last axis)."""
        if hasattr(self, "_src"):
            return self._src
        out = {}
        for bb in BLOCKS:
            shape = tuple(self.dimsp[sp] for (_, sp) in bb.ext) + (self.nst * len(bb.types) * self.ntup[bb.name], self.nst)
            acc = np.zeros(shape)
            for hi, (ops, C, clabels) in enumerate(self.ham_components()):
                for spec, _, G, _ in self._plan(("H", hi, bb.name), bb, None, ops, C, clabels):
                    acc += np.einsum(spec, C, G, optimize=True)
            out[bb.name] = acc
        self._src = out
        return out

    def source_all(self, L: int, N: int) -> dict:
        """Source <f(L-space)| H |N~> on all orderings, alpha restricted to
        the function set of state L."""
        src = self.sources()
        out = {}
        for b in BLOCKS:
            v = src[b.name][..., N]
            if self.scheme == "SSSR":
                v = v[..., self._alpha_slice(b, L)]
            out[b.name] = v
        return out

    def residual(self, L: int, x: np.ndarray, with_source: bool = True) -> np.ndarray:
        """sigma_L = A_L x (+ V^(L)) in the packed layout (Eq. 10)."""
        xall = self.unpack(x)
        s = self.apply_A(L, xall)
        if with_source:
            v = self.source_all(L, L)
            for k in s:
                s[k] = s[k] + v[k]
        return self.pack(s)

    def source(self, L: int, N: int) -> np.ndarray:
        return self.pack(self.source_all(L, N))

    # -- metric and Fock metric per character; orthogonal basis -------------
    def _perm_sign(self, b: Block, classes, chi):
        sgn = 1.0
        for (k, l), c in zip(b.swaps, chi):
            lk = b.ext[k][0]
            ll = b.ext[l][0]
            if frozenset((lk + "_b", ll + "_k")) in classes:
                sgn *= c
        return sgn

    def metric_chi(self, b: Block, chi, L: int = 0):
        n = self.nalpha[b.name]
        S = np.zeros((n, n))
        for spec, _, G, classes in self._plan(("S", b.name), b, b, [], 1.0, []):
            S += self._perm_sign(b, classes, chi) * self._restrict(G, b, b, L)
        return S

    def fock_metric_chi(self, b: Block, chi, L: int = 0):
        """<f| f_act |f'> (active block of f only) per character."""
        n = self.nalpha[b.name]
        F = np.zeros((n, n))
        fa = self.f[self.sl[ACT], self.sl[ACT]]
        ops = E("x_o", ACT, "y_o", ACT, "so")
        for spec, _, G, classes in self._plan(("FA", b.name), b, b, ops, fa, ["x_o", "y_o"],
                                              precontract=True):
            F += self._perm_sign(b, classes, chi) * self._restrict(G, b, b, L)
        return F

    def ortho(self, L: int = 0):
        """Per (block, character): X (kept overlap eigenvectors scaled by
        lambda^-1/2, rotated to diagonalise X^T F X) and mu (Sec. II.B)."""
        key = L if self.scheme == "SSSR" else 0
        if not hasattr(self, "_ortho"):
            self._ortho = {}
        if key in self._ortho:
            return self._ortho[key]
        res = []
        for ent in self.layout:
            b, chi = ent["block"], ent["chi"]
            S = self.metric_chi(b, chi, L)
            F = self.fock_metric_chi(b, chi, L)
            w, Q = np.linalg.eigh(S)
            keep = w >= self.thresh
            X0 = Q[:, keep] / np.sqrt(w[keep])[None, :]
            Fo = X0.T @ F @ X0
            mu, Z = np.linalg.eigh(0.5 * (Fo + Fo.T))
            X = X0 @ Z
            dropped = w[~keep]
            res.append(dict(X=X, mu=mu, S=S, F=F, emin_kept=float(w[keep].min()) if keep.any() else np.inf,
                            emax_dropped=float(dropped.max()) if dropped.size else -np.inf))
        self._ortho[key] = res
        return res

    def ext_energy(self, ent):
        """Sum of virtual minus closed diagonal Fock elements per orbit row."""
        b = ent["block"]
        eps = np.diag(self.f)
        reps = np.array(ent["reps"], dtype=np.int64).reshape(ent["nrow"], len(b.ext))
        out = np.zeros(ent["nrow"])
        for k, (lab, sp) in enumerate(b.ext):
            e = eps[self.sl[sp]][reps[:, k]]
            out += e if sp == VIR else -e
        return out

    def _to_orth(self, L, x):
        """Packed amplitudes -> orthogonal coordinates (X^T x per row)."""
        parts = []
        for ent, o in zip(self.layout, self.ortho(L)):
            blk = x[ent["offset"]: ent["offset"] + ent["nrow"] * ent["nalpha"]].reshape(ent["nrow"], ent["nalpha"])
            parts.append(blk @ o["X"])
        return parts

    def _from_orth(self, L, parts):
        x = np.zeros(self.length)
        for ent, o, t in zip(self.layout, self.ortho(L), parts):
            x[ent["offset"]: ent["offset"] + ent["nrow"] * ent["nalpha"]] = (t @ o["X"].T).ravel()
        return x

    def denominators(self, L):
        out = []
        for ent, o in zip(self.layout, self.ortho(L)):
            d = self.ext_energy(ent)[:, None] + o["mu"][None, :] + self.p.shift - self.e0[L]
            out.append(d)
        return out

    def solve(self, L: int, source: np.ndarray, tol: float = 1e-12, maxiter: int = 500, x0=None):
        """PCG on X^T A_L X t = -X^T source (orthogonal basis, Sec. II.B)."""
        D = self.denominators(L)
        dmin = min(float(d.min()) for d in D if d.size)
        if dmin <= 0.0:
            raise ArithmeticError(f"non-positive denominator {dmin}")
        bt = self._to_orth(L, source)
        def Aop(parts):
            x = self._from_orth(L, parts)
            return self._to_orth(L, self.residual(L, x, with_source=False))
        flat = lambda parts: np.concatenate([p.ravel() for p in parts]) if parts else np.zeros(0)
        shapes = [p.shape for p in bt]
        def unflat(v):
            out, k = [], 0
            for sh in shapes:
                n = int(np.prod(sh))
                out.append(v[k:k + n].reshape(sh))
                k += n
            return out
        b = -flat(bt)
        d = flat(D)
        t = np.zeros_like(b) if x0 is None else flat(self._to_orth(L, x0))
        r = b - flat(Aop(unflat(t)))
        z = r / d
        pvec = z.copy()
        rz = r @ z
        hist = [float(np.linalg.norm(r))]
        it = 0
        while hist[-1] > tol and it < maxiter:
            Ap = flat(Aop(unflat(pvec)))
            pAp = pvec @ Ap
            if pAp <= 0:
                raise ArithmeticError("operator not positive definite")
            alpha = rz / pAp
            t = t + alpha * pvec
            r = r - alpha * Ap
            z = r / d
            rz_new = r @ z
            pvec = z + (rz_new / rz) * pvec
            rz = rz_new
            it += 1
            hist.append(float(np.linalg.norm(r)))
        return self._from_orth(L, unflat(t)), dict(iters=it, resnorm=hist[-1], hist=hist)

    def apply_S(self, L: int, x: np.ndarray) -> np.ndarray:
        out = np.zeros_like(x)
        for ent, o in zip(self.layout, self.ortho(L)):
            sl = slice(ent["offset"], ent["offset"] + ent["nrow"] * ent["nalpha"])
            out[sl] = (x[sl].reshape(ent["nrow"], ent["nalpha"]) @ o["S"]).ravel()
        return out

    # -- energies, Eq. 15-17 -------------------------------------------------
    def solve_amplitudes(self, tol=1e-12, maxiter=500):
        self.T = []
        self.T_info = []
        for L in range(self.nst):
            T, info = self.solve(L, self.source(L, L), tol=tol, maxiter=maxiter)
            self.T.append(T)
            self.T_info.append(info)
        return self.T

    def heff(self):
        nst = self.nst
        H = self.href.copy()
        for L in range(nst):
            for Lp in range(nst):
                H[L, Lp] += 0.5 * (self.T[L] @ self.source(L, Lp) + self.T[Lp] @ self.source(Lp, L))
            H[L, L] -= self.p.shift * self.T[L] @ self.apply_S(L, self.T[L])
        w, R = np.linalg.eigh(0.5 * (H + H.T))
        for k in range(nst):
            if R[np.argmax(np.abs(R[:, k])), k] < 0:
                R[:, k] = -R[:, k]
        self.H_eff, self.e_ms, self.R = H, w, R
        return H, w, R

    def lambda_source(self, L, P):
        """R_LP sum_N R_NP V^(N) - 2 E_s R_LP^2 S T_L (Eq. 20)."""
        R = self.R
        src = np.zeros(self.length)
        for N in range(self.nst):
            src += R[L, P] * R[N, P] * self.source(L, N)
        src -= 2.0 * self.p.shift * R[L, P] ** 2 * self.apply_S(L, self.T[L])
        return src

    def solve_lambda(self, P: int = 0, tol=1e-12, maxiter=500):
        self.lam = []
        self.lam_info = []
        for L in range(self.nst):
            lam, info = self.solve(L, self.lambda_source(L, P), tol=tol, maxiter=maxiter)
            self.lam.append(lam)
            self.lam_info.append(info)
        return self.lam

    def run(self, P: int = 0, tol=1e-12):
        self.solve_amplitudes(tol=tol)
        self.heff()
        self.solve_lambda(P, tol=tol)
        self.target = P
        return self

    # -- correlated densities, Sec. II.D ------------------------------------
    @staticmethod
    def _einsum_to(spec_in: str, out: str, shape, *ops):
        """einsum into the output subscripts `out` (array of the given shape).
        `out` may repeat a letter (a pairing that sets two operator indices
        equal: the result goes on that diagonal) and may hold letters absent
        from the inputs (an operator index contracted with the other one of
        the same operator: the result does not depend on it)."""
        uniq = "".join(dict.fromkeys(out))
        ins = set(spec_in.replace(",", ""))
        present = "".join(c for c in uniq if c in ins)
        r = np.einsum(f"{spec_in}->{present}", *ops, optimize=True)
        if present == out:
            return r
        dims = [shape[out.index(c)] for c in uniq]
        idx = np.indices(dims)
        val = r[tuple(idx[uniq.index(c)] for c in present)] if present else np.full(dims, float(r))
        full = np.zeros(shape)
        np.add.at(full, tuple(idx[uniq.index(c)] for c in out), val)
        return full

    def _space_of_label(self, ops, lab):
        return next(o.space for o in ops if o.label == lab)

    def densities(self):
        """d^(1), D^(1), d-bar^(2), N_L and d^(2) of Sec. II.D for the target
        state P of run(P), in factorised form: every density element is the
        derivative of a matrix element already used by the amplitude
        equation with respect to its operator coefficient, i.e. the same Wick
        terms and active Gram tensors contracted with T, lambda and R instead
        of with the integrals or f.

        Returns d1 [nmo][nmo], D1 {spaces (p, q, r, s): [p][q][r][s]} over the
        classes of the two-body part of H that act on the references
        (creators p, r active or virtual; annihilators q, s active or closed;
        not all active), dbar2 and d2 [nmo][nmo], NL [nst]."""
        P = self.target
        nst, R = self.nst, self.R
        nmo = self.nc + self.na + self.nv
        T_all = [self.unpack(v) for v in self.T]
        l_all = [self.unpack(v) for v in self.lam]
        # weights W[e..., alpha over every state's functions, ket N]
        W = {}
        for b in BLOCKS:
            shape = tuple(self.dimsp[sp] for (_, sp) in b.ext) + (self.nst * len(b.types) * self.ntup[b.name], nst)
            W[b.name] = np.zeros(shape)
        for L in range(nst):
            for b in BLOCKS:
                sl = slice(None) if self.scheme == "MSMR" else self._alpha_slice(b, L)
                for N in range(nst):
                    W[b.name][..., sl, N] += R[L, P] * R[N, P] * T_all[L][b.name]
                W[b.name][..., sl, L] += l_all[L][b.name]
        d1 = np.zeros((nmo, nmo))
        D1 = {}
        for hi, (ops, C, clabels) in enumerate(self.ham_components()):
            spaces = tuple(self._space_of_label(ops, lab) for lab in clabels)
            acc = np.zeros(C.shape)
            for bb in BLOCKS:
                for spec, _, G, _ in self._plan(("H", hi, bb.name), bb, None, ops, C, clabels):
                    cstr, rest = spec.split(",", 1)
                    gstr, outz = rest.split("->")
                    acc += self._einsum_to(f"{outz},{gstr}", cstr, acc.shape, W[bb.name], G)
            if len(clabels) == 2:
                d1[self.sl[spaces[0]], self.sl[spaces[1]]] += acc
            else:
                D1[spaces] = acc
        # d-bar^(2): every block of f, whatever its values
        dbar2 = np.zeros((nmo, nmo))
        for sx in (CLO, ACT, VIR):
            for sy in (CLO, ACT, VIR):
                if self.dimsp[sx] == 0 or self.dimsp[sy] == 0:
                    continue
                ops = E("x_o", sx, "y_o", sy, "so")
                dummy = np.zeros((self.dimsp[sx], self.dimsp[sy]))
                acc = np.zeros_like(dummy)
                for bb in BLOCKS:
                    for kb in BLOCKS:
                        plans = self._plan(("D2", sx, sy, bb.name, kb.name), bb, kb, ops, dummy,
                                           ["x_o", "y_o"])
                        for spec, _, G, _ in plans:
                            cstr, gstr, rest = spec.split(",")
                            xstr, outs = rest.split("->")
                            for L in range(nst):
                                Gr = self._restrict(G, bb, kb, L)
                                acc += self._einsum_to(f"{outs},{gstr},{xstr}", cstr, acc.shape,
                                                       l_all[L][bb.name], Gr, T_all[L][kb.name])
                dbar2[self.sl[sx], self.sl[sy]] += acc
        NL = np.array([self.lam[L] @ self.apply_S(L, self.T[L]) for L in range(nst)])
        d2 = dbar2.copy()
        sa = self.sl[ACT]
        for r in range(self.na):
            for t in range(self.na):
                unit = np.zeros((self.na, self.na))
                unit[r, t] = 1.0
                g = self._one_body(unit, self.ci)
                d2[sa.start + r, sa.start + t] -= sum(NL[L] * g[L, L] for L in range(nst))
        return dict(d1=d1, D1=D1, dbar2=dbar2, NL=NL, d2=d2)
