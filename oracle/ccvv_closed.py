"""Closed form of the ccvv rows of the amplitude residual for a diagonal Fock
operator.  TEST INFRASTRUCTURE ONLY: only tests/, __graft_entry__.smoke()
and bench.py's cpu_baseline leg may use anything under oracle/.

What is computed (paper Sec. II.B, Eq. 10, with the Fock operator of
Eqs. 11-12 restricted to its diagonal, f_pq = eps_p delta_pq, and the XMS
reference states of Eqs. 3-5 and 14), for the functions E_ai E_bj |M~> of
the MS-MR space (Eq. 7), row by row, so that single rows can be evaluated
at any problem size:

  * Both operators of E_ai E_bj act on closed and virtual orbitals only, so
    for a ket function E_ck E_dl |N~> the overlap factorises into the
    closed-shell value <core| E_jb E_ia E_ck E_dl |core> times <M~|N~>:
        4 d_ac d_ik d_bd d_jl + 4 d_ad d_il d_bc d_jk
      - 2 d_ac d_bd d_il d_jk - 2 d_ad d_bc d_ik d_jl.
  * With a diagonal f the commutator [f, E_ai E_bj] is
    (eps_a + eps_b - eps_i - eps_j) E_ai E_bj, and f acting on |core, N~>
    leaves the active part sum_t eps_t E_tt, whose matrix between rotated
    reference states is diag(E~) (the XMS rotation diagonalises it).  So
    the operator of Eq. 10 becomes, on these functions,
        S_ext * (eps_a + eps_b - eps_i - eps_j + E_s - E~_L + E~_M).
  * The source <M~| E_jb E_ia H |L~> is delta_ML (4 (ai|bj) - 2 (aj|bi)):
    only the two-electron part with all four indices external survives.

Rows are those of the packed layout: one row per canonical representative
(i >= j, a >= b; strictly for the '-' character) and character (+,+) or
(-,-) over the two index swaps; the packed value of a row is
sum_e chi(e) sigma[e] / sqrt(|orbit|) over the distinct images e of the
representative, and an individual function's coefficient is
x[e] = sum_chi chi(e) t_chi / sqrt(|orbit|).

The XMS rotation is recomputed here from the CI vectors (occupation numbers
of the determinants: f is diagonal), independently of the other oracle
modules.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["xms_energies_diagonal_f", "ccvv_pair_index", "ccvv_rows"]


def _strings(norb: int, nel: int) -> np.ndarray:
    return np.array([s for s in range(1 << norb) if bin(s).count("1") == nel], dtype=np.int64)


def xms_energies_diagonal_f(prob) -> np.ndarray:
    """E~ (ascending) of the XMS rotation (Eqs. 3-5): the eigenvalues of
    F_MN = <M| sum_t eps_t E_tt |N> over the reference states, for a Fock
    operator that is diagonal in the active orbitals."""
    nc, na = prob.nc, prob.na
    if na == 0:
        return np.zeros(prob.nst)
    f_act = np.asarray(prob.fock)[nc:nc + na, nc:nc + na]
    if np.any(f_act != np.diag(np.diag(f_act))):
        raise ValueError("the active Fock block is not diagonal")
    eps = np.diag(f_act)
    sa, sb = _strings(na, prob.nalpha), _strings(na, prob.nbeta)
    occ = np.array([[((a >> t) & 1) + ((b >> t) & 1) for t in range(na)] for a in sa for b in sb], dtype=float)
    w = occ @ eps                                  # diagonal of sum_t eps_t n_t per determinant
    ci = np.asarray(prob.ci)
    F = (ci * w[None, :]) @ ci.T
    return np.linalg.eigvalsh(0.5 * (F + F.T))


def ccvv_pair_index(k: int, l: int, minus: bool) -> int:
    """Index of the pair (k, l), k >= l ('+') or k > l ('-'), in ascending
    lexicographic order."""
    return k * (k - 1) // 2 + l if minus else k * (k + 1) // 2 + l


def _images(e):
    """Distinct images of (i, j, a, b) under the swaps (i j) and (a b), with
    the swap bits that first reach them."""
    i, j, a, b = e
    out = {}
    for sij in (0, 1):
        for sab in (0, 1):
            img = ((j, i) if sij else (i, j)) + ((b, a) if sab else (a, b))
            out.setdefault(img, (sij, sab))
    return out


def ccvv_rows(prob, L: int, reps, t_plus, t_minus, with_source: bool = True):
    """Packed residual rows of state L at the given representatives.

    reps: list of (i, j, a, b) with i >= j, a >= b (closed indices i, j in
    0..nc-1, virtual indices a, b in 0..nv-1).  t_plus[k], t_minus[k]: the
    packed rows (length nst, one column per state M) of representative k for
    the two characters; t_minus[k] is ignored (and may be None) where the
    '-' row does not exist (i == j or a == b).  Returns (sig_plus, sig_minus)
    as arrays [len(reps), nst]; sig_minus rows without a '-' row are NaN."""
    nc, na, nv, nst = prob.nc, prob.na, prob.nv, prob.nst
    eps = np.asarray(prob.eps)
    fock = np.asarray(prob.fock)
    if np.any(fock != np.diag(np.diag(fock))):
        raise ValueError("the closed form needs a diagonal Fock operator")
    E = xms_energies_diagonal_f(prob)
    B = np.asarray(prob.B)
    v0 = nc + na
    shift = float(prob.shift)
    sig_p = np.full((len(reps), nst), np.nan)
    sig_m = np.full((len(reps), nst), np.nan)
    for r, (i, j, a, b) in enumerate(reps):
        if not (nc > i >= j >= 0 and nv > a >= b >= 0):
            raise ValueError("not a canonical representative")
        imgs = _images((i, j, a, b))
        w = 1.0 / math.sqrt(len(imgs))
        has_minus = i > j and a > b
        tp = np.asarray(t_plus[r], dtype=float)
        tm = np.asarray(t_minus[r], dtype=float) if has_minus else np.zeros(nst)
        # coefficients of the individual functions (all orderings)
        x = {e: w * (tp + (-1) ** (bits[0] + bits[1]) * tm) for e, bits in imgs.items()}
        # the operator on every image: overlap pattern times the diagonal factor
        gap = eps[v0 + a] + eps[v0 + b] - eps[i] - eps[j] + shift - E[L] + E
        sig = {}
        for (p, q, c, d) in imgs:
            s = (4.0 * x[(p, q, c, d)] + 4.0 * x[(q, p, d, c)]
                 - 2.0 * x[(q, p, c, d)] - 2.0 * x[(p, q, d, c)])
            s = gap * s
            if with_source:
                # 4 (c p|d q) - 2 (c q|d p), all orbital indices absolute
                vpq = float(B[:, v0 + c, p] @ B[:, v0 + d, q])
                vqp = float(B[:, v0 + c, q] @ B[:, v0 + d, p])
                s = s.copy()
                s[L] += 4.0 * vpq - 2.0 * vqp
            sig[(p, q, c, d)] = s
        sig_p[r] = sum(w * sig[e] for e in imgs)
        if has_minus:
            sig_m[r] = sum(w * (-1) ** (bits[0] + bits[1]) * sig[e] for e, bits in imgs.items())
    return sig_p, sig_m
