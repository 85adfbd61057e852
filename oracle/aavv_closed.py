"""Closed form of the aavv rows of the amplitude residual for a diagonal Fock
operator.  TEST INFRASTRUCTURE ONLY: only tests/, __graft_entry__.smoke()
and bench.py's cpu_baseline leg may use anything under oracle/.

What is computed (paper Sec. II.B, Eq. 10, with the Fock operator of
Eqs. 11-12 restricted to its diagonal and the XMS reference states of
Eqs. 3-5 and 14), for the functions E_ar E_bs |M~> of the MS-MR space
(Eq. 7; a, b virtual, r, s active), row by row:

  * Contracting the virtual operators of <M~| E_sb E_ra E_a'r' E_b's' |N~>
    (virtual orbitals empty) leaves an active operator: for the direct
    pairing (a = a', b = b') E_rr' E_ss' - d_r's E_rs', for the crossed one
    (a = b', b = a') E_sr' E_rs' - d_rr' E_ss' (commuting the virtual
    operators through the active ones).
  * With a diagonal f, [f, E_a'r' E_b's'] = (eps_a' + eps_b' - eps_r' -
    eps_s') E_a'r' E_b's', and f on |core, N~> leaves f_act; the operator of
    Eq. 10 is the same pattern with the active operator followed by
    f_act + eps_a' + eps_b' - eps_r' - eps_s' + E_s - E~_L.
  * The source <M~| E_sb E_ra H |L~>: only 1/2 sum (a't|b'u) E_a't E_b'u
    reaches these functions (both virtual indices run over every pair, so
    (a', b') = (a, b) and (b, a) each pair once), so it is
    1/2 sum_tu [(at|bu) <M~|E_rt E_su - d_ts E_ru|L~>
              + (bt|au) <M~|E_st E_ru - d_rt E_su|L~>].

Rows are those of the packed layout: one per representative a >= b
(strictly for the '-' character), columns (state M, r, s) with the state
slowest; the orbit rule of the layout packs and unpacks them.  The XMS
states are recomputed from the CI vectors (oracle/cavv_closed.py).
"""
from __future__ import annotations

import math

import numpy as np

from oracle.cavv_closed import _apply_E, _hop, _strings, xms_states_diagonal_f

__all__ = ["aavv_rows"]


def _products(prob):
    """D[M,N,p,q,r,s] = <M~|E_pq E_rs|N~>, DF = <M~|E_pq E_rs f_act|N~>,
    Gamma[M,N,p,q] = <M~|E_pq|N~>, G = <M~|E_pq f_act|N~>, and E~."""
    na, nst = prob.na, prob.nst
    sa, sb = _strings(na, prob.nalpha), _strings(na, prob.nbeta)
    hops = {}
    for r in range(na):
        for q in range(na):
            hops[("a", r, q)] = _hop(sa, r, q)
            hops[("b", r, q)] = _hop(sb, r, q)
    ci, E, w = xms_states_diagonal_f(prob)
    kets = np.stack([ci, ci * w[None]])                      # [2, N, A, B]: |N~>, f_act |N~>
    one = np.zeros((2, nst, nst, na, na))
    two = np.zeros((2, nst, nst, na, na, na, na))
    for r in range(na):
        for s in range(na):
            v = _apply_E(kets, r, s, sa, sb, hops)             # E_rs |.>
            one[:, :, :, r, s] = np.einsum("MAB,kNAB->kMN", ci, v)
            for p in range(na):
                for q in range(na):
                    u = _apply_E(v, p, q, sa, sb, hops)       # E_pq E_rs |.>
                    two[:, :, :, p, q, r, s] = np.einsum("MAB,kNAB->kMN", ci, u)
    return two[0], two[1], one[0], one[1], E


def aavv_rows(prob, L: int, reps, t_plus, t_minus, with_source: bool = True, prods=None):
    """Packed residual rows of state L at the given representatives.

    reps: list of (a, b) with a >= b (virtual indices 0..nv-1).  t_plus[k],
    t_minus[k]: the packed rows (length nst * na * na, columns (M, r, s)) of
    representative k; t_minus[k] is ignored (and may be None) where a == b.
    prods: an earlier call's active products (optional, to reuse).  Returns
    (sig_plus, sig_minus, prods) with arrays [len(reps), nst * na * na];
    sig_minus rows without a '-' row are NaN."""
    nc, na, nv, nst = prob.nc, prob.na, prob.nv, prob.nst
    if na == 0:
        raise ValueError("aavv needs active orbitals")
    fock = np.asarray(prob.fock)
    if np.any(fock != np.diag(np.diag(fock))):
        raise ValueError("the closed form needs a diagonal Fock operator")
    eps = np.asarray(prob.eps)
    if prods is None:
        prods = _products(prob)
    D, DF, Gam, G, E = prods
    a0, v0 = nc, nc + na
    eye = np.eye(na)
    # direct and crossed active operators as [M, r, s, N, r', s'] matrices
    # direct: E_rr' E_ss' - d_r's E_rs'
    Kd1 = D.transpose(0, 2, 4, 1, 3, 5) - np.einsum("ps,MNrq->MrsNpq", eye, Gam)
    Kdf = DF.transpose(0, 2, 4, 1, 3, 5) - np.einsum("ps,MNrq->MrsNpq", eye, G)
    # crossed: E_sr' E_rs' - d_rr' E_ss'
    Kx1 = D.transpose(0, 4, 2, 1, 3, 5) - np.einsum("rp,MNsq->MrsNpq", eye, Gam)
    Kxf = DF.transpose(0, 4, 2, 1, 3, 5) - np.einsum("rp,MNsq->MrsNpq", eye, G)
    n = nst * na * na
    Kd1, Kdf, Kx1, Kxf = (m.reshape(n, n) for m in (Kd1, Kdf, Kx1, Kxf))
    e_act = eps[a0:a0 + na]
    col = np.tile((e_act[:, None] + e_act[None, :]).ravel(), nst)     # eps_r' + eps_s' per column
    shift = float(prob.shift)
    sig_p = np.full((len(reps), n), np.nan)
    sig_m = np.full((len(reps), n), np.nan)
    for k, (a, b) in enumerate(reps):
        if not (nv > a >= b >= 0):
            raise ValueError("not a canonical representative")
        imgs = [(a, b)] if a == b else [(a, b), (b, a)]
        wgt = 1.0 / math.sqrt(len(imgs))
        tp = np.asarray(t_plus[k], dtype=float)
        tm = np.asarray(t_minus[k], dtype=float) if a > b else np.zeros(n)
        x = {imgs[0]: wgt * (tp + tm)}
        if a > b:
            x[imgs[1]] = wgt * (tp - tm)
        c0 = eps[v0 + a] + eps[v0 + b] + shift - E[L]

        def apply(Kf, K1, v):
            y = v * (c0 - col)
            return Kf @ v + K1 @ y

        sig = {}
        for (c, d) in imgs:
            s = apply(Kdf, Kd1, x[(c, d)]) + apply(Kxf, Kx1, x[(d, c)])
            if with_source:
                ct = B_vt(prob, v0 + c, a0, na)            # (c t|d u) = sum_Q B[Q,c,t] B[Q,d,u]
                dt = B_vt(prob, v0 + d, a0, na)
                g_cd = ct.T @ dt                           # [t, u] = (c t|d u)
                g_dc = dt.T @ ct                           # [t, u] = (d t|c u)
                # 1/2 sum_tu (ct|du) <M|E_rt E_su - d_ts E_ru|L> + (dt|cu) <M|E_st E_ru - d_rt E_su|L>
                DL, GL = D[:, L], Gam[:, L]                # [M, p, q, r, s], [M, p, q]
                v1 = np.einsum("tu,Mrtsu->Mrs", g_cd, DL) - np.einsum("su,Mru->Mrs", g_cd, GL)
                v2 = np.einsum("tu,Mstru->Mrs", g_dc, DL) - np.einsum("ru,Msu->Mrs", g_dc, GL)
                s = s + 0.5 * (v1 + v2).reshape(n)
            sig[(c, d)] = s
        sig_p[k] = wgt * sum(sig[e] for e in imgs)
        if a > b:
            sig_m[k] = wgt * (sig[imgs[0]] - sig[imgs[1]])
    return sig_p, sig_m, prods


def B_vt(prob, v: int, a0: int, na: int) -> np.ndarray:
    """B[Q, v, t] over the active t: [naux, na]."""
    return np.asarray(prob.B)[:, v, a0:a0 + na]
