"""Closed form of the cavv rows of the amplitude residual for a diagonal Fock
operator.  TEST INFRASTRUCTURE ONLY: only tests/, __graft_entry__.smoke()
and bench.py's cpu_baseline leg may use anything under oracle/.

What is computed (paper Sec. II.B, Eq. 10, with the Fock operator of
Eqs. 11-12 restricted to its diagonal, f_pq = eps_p delta_pq, and the XMS
reference states of Eqs. 3-5 and 14), for the functions E_ar E_bi |M~> of
the MS-MR space (Eq. 7, i closed, r active, a and b virtual), row by row:

  * Contracting the closed and virtual operators of <M~| E_ib E_ra E_a'r'
    E_b'i' |N~> (virtual orbitals empty, closed orbitals full) leaves
        d_ii' (2 d_aa' d_bb' - d_ab' d_ba') <M~| E_rr' |N~>,
    the direct pairing of both virtual indices (two spin sums, one of them
    through the closed hole) and the crossed one (a single spin sum).
  * With a diagonal f, [f, E_ar E_bi] = (eps_a - eps_r + eps_b - eps_i)
    E_ar E_bi, and f on |core, N~> leaves f_act = sum_t eps_t E_tt, so the
    operator of Eq. 10 on these functions is the same external pattern times
        <M~| E_rr' f_act |N~> + (eps_a' + eps_b' - eps_i' - eps_r' + E_s - E~_L)
        <M~| E_rr' |N~>.
  * The source <M~| E_ib E_ra H |L~>: only the two-electron terms
    (a't|b'i') E_a't E_b'i' reach these functions, so it is
        sum_t <M~| E_rt |L~> (2 (at|bi) - (bt|ai)).

Rows are those of the packed layout: one per representative (i, a, b) with
a >= b (strictly for the '-' character of the (a b) swap), columns
(state M, active r) with the state slowest; packing and unpacking follow the
orbit rule of the layout (1/sqrt(|orbit|), the character's sign on the
swapped image).

The XMS rotation and the transition one-particle densities are recomputed
here from the CI vectors (determinant strings with alpha creators left of
beta creators), independently of the other oracle modules.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["xms_states_diagonal_f", "cavv_rows"]


def _strings(norb: int, nel: int) -> np.ndarray:
    return np.array([s for s in range(1 << norb) if bin(s).count("1") == nel], dtype=np.int64)


def _hop(strs: np.ndarray, r: int, q: int):
    """a+_r a_q on every string of one spin: (source index, target index,
    sign) of the strings it does not annihilate."""
    pos = {int(s): k for k, s in enumerate(strs)}
    src, tgt, sgn = [], [], []
    for k, s in enumerate(strs):
        s = int(s)
        if not (s >> q) & 1:
            continue
        s1 = s & ~(1 << q)
        n1 = bin(s1 & ((1 << q) - 1)).count("1")          # electrons passed by a_q
        if (s1 >> r) & 1:
            continue
        n2 = bin(s1 & ((1 << r) - 1)).count("1")          # electrons passed by a+_r
        src.append(k)
        tgt.append(pos[s1 | (1 << r)])
        sgn.append(-1.0 if (n1 + n2) % 2 else 1.0)
    return np.array(src, dtype=np.int64), np.array(tgt, dtype=np.int64), np.array(sgn)


def _apply_E(ci: np.ndarray, r: int, q: int, sa, sb, hops) -> np.ndarray:
    """E_rq (both spins) on CI arrays [..., n_alpha_strings, n_beta_strings].
    A beta pair a+ a passes every alpha creator twice, so only its own
    string's parity counts."""
    out = np.zeros_like(ci)
    s, t, g = hops[("a", r, q)]
    out[..., t, :] += g[:, None] * ci[..., s, :]
    s, t, g = hops[("b", r, q)]
    out[..., :, t] += g[None, :] * ci[..., :, s]
    return out


def xms_states_diagonal_f(prob):
    """(rotated CI [nst, nA, nB], E~ ascending, occupation-weighted
    energies w[nA, nB]) of the XMS rotation (Eqs. 3-5) for an active Fock
    block that is diagonal; each rotation column's largest-magnitude entry
    is made positive."""
    nc, na, nst = prob.nc, prob.na, prob.nst
    f_act = np.asarray(prob.fock)[nc:nc + na, nc:nc + na]
    if np.any(f_act != np.diag(np.diag(f_act))):
        raise ValueError("the active Fock block is not diagonal")
    eps = np.diag(f_act)
    sa, sb = _strings(na, prob.nalpha), _strings(na, prob.nbeta)
    occ_a = np.array([[(s >> t) & 1 for t in range(na)] for s in sa], dtype=float)
    occ_b = np.array([[(s >> t) & 1 for t in range(na)] for s in sb], dtype=float)
    w = (occ_a @ eps)[:, None] + (occ_b @ eps)[None, :]
    ci = np.asarray(prob.ci).reshape(nst, len(sa), len(sb))
    F = np.einsum("MAB,AB,NAB->MN", ci, w, ci)
    e, U = np.linalg.eigh(0.5 * (F + F.T))
    for k in range(nst):
        if U[np.argmax(np.abs(U[:, k])), k] < 0:
            U[:, k] = -U[:, k]
    return np.einsum("NAB,NM->MAB", ci, U), e, w


def _densities(prob):
    """Gamma[M, N, r, q] = <M~|E_rq|N~> and G[M, N, r, q] = <M~|E_rq f_act|N~>."""
    na, nst = prob.na, prob.nst
    sa, sb = _strings(na, prob.nalpha), _strings(na, prob.nbeta)
    hops = {}
    for r in range(na):
        for q in range(na):
            hops[("a", r, q)] = _hop(sa, r, q)
            hops[("b", r, q)] = _hop(sb, r, q)
    ci, E, w = xms_states_diagonal_f(prob)
    fci = ci * w[None]
    gam = np.zeros((nst, nst, na, na))
    g = np.zeros((nst, nst, na, na))
    for r in range(na):
        for q in range(na):
            gam[:, :, r, q] = np.einsum("MAB,NAB->MN", ci, _apply_E(ci, r, q, sa, sb, hops))
            g[:, :, r, q] = np.einsum("MAB,NAB->MN", ci, _apply_E(fci, r, q, sa, sb, hops))
    return gam, g, E


def cavv_rows(prob, L: int, reps, t_plus, t_minus, with_source: bool = True, dens=None):
    """Packed residual rows of state L at the given representatives.

    reps: list of (i, a, b) with a >= b (i closed 0..nc-1, a and b virtual
    0..nv-1).  t_plus[k], t_minus[k]: the packed rows (length nst * na,
    columns (M, r)) of representative k for the two characters; t_minus[k]
    is ignored (and may be None) where a == b.  dens: the result of an
    earlier call's densities (optional, to reuse).  Returns
    (sig_plus, sig_minus, dens) with arrays [len(reps), nst * na];
    sig_minus rows without a '-' row are NaN."""
    nc, na, nv, nst = prob.nc, prob.na, prob.nv, prob.nst
    if na == 0:
        raise ValueError("cavv needs active orbitals")
    fock = np.asarray(prob.fock)
    if np.any(fock != np.diag(np.diag(fock))):
        raise ValueError("the closed form needs a diagonal Fock operator")
    eps = np.asarray(prob.eps)
    if dens is None:
        dens = _densities(prob)
    gam, g, E = dens
    B = np.asarray(prob.B)
    a0, v0 = nc, nc + na
    shift = float(prob.shift)
    eps_act = eps[a0:a0 + na]
    n = nst * na
    # K[(M r), (N q)] without the external energies: G + (E_s - E~_L - eps_q) Gamma
    K0 = (g + (shift - E[L] - eps_act[None, None, None, :]) * gam).transpose(0, 2, 1, 3).reshape(n, n)
    Gm = gam.transpose(0, 2, 1, 3).reshape(n, n)
    sig_p = np.full((len(reps), n), np.nan)
    sig_m = np.full((len(reps), n), np.nan)
    for k, (i, a, b) in enumerate(reps):
        if not (nc > i >= 0 and nv > a >= b >= 0):
            raise ValueError("not a canonical representative")
        imgs = [(i, a, b)] if a == b else [(i, a, b), (i, b, a)]
        wgt = 1.0 / math.sqrt(len(imgs))
        tp = np.asarray(t_plus[k], dtype=float)
        tm = np.asarray(t_minus[k], dtype=float) if a > b else np.zeros(n)
        x = {imgs[0]: wgt * (tp + tm)}
        if a > b:
            x[imgs[1]] = wgt * (tp - tm)
        gap = eps[v0 + a] + eps[v0 + b] - eps[i]
        Kx = {e: K0 @ x[e] + gap * (Gm @ x[e]) for e in imgs}
        sig = {}
        for (p, c, d) in imgs:
            s = 2.0 * Kx[(p, c, d)] - Kx[(p, d, c)]
            if with_source:
                # sum_t <M~|E_rt|L~> (2 (c t|d p) - (d t|c p))
                ct = B[:, v0 + c, a0:a0 + na]          # [Q, t]
                dt = B[:, v0 + d, a0:a0 + na]
                v = 2.0 * (ct.T @ B[:, v0 + d, p]) - dt.T @ B[:, v0 + c, p]    # [t]
                s = s + (gam[:, L, :, :] @ v).reshape(n)
            sig[(p, c, d)] = s
        sig_p[k] = wgt * sum(sig[e] for e in imgs)
        if a > b:
            sig_m[k] = wgt * (sig[imgs[0]] - sig[imgs[1]])
    return sig_p, sig_m, dens
