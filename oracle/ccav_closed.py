"""Closed form of the ccav rows of the amplitude residual for a diagonal Fock
operator.  TEST INFRASTRUCTURE ONLY: only tests/, __graft_entry__.smoke()
and bench.py's cpu_baseline leg may use anything under oracle/.

What is computed (paper Sec. II.B, Eq. 10, with the Fock operator of
Eqs. 11-12 restricted to its diagonal and the XMS reference states of
Eqs. 3-5 and 14), for the functions E_ai E_rj |M~> of the MS-MR space
(Eq. 7; i, j closed, a virtual, r active), row by row:

  * Contracting the virtual a (empty) and then commuting the closed
    operators through (closed orbitals full) turns
    <M~| E_jr E_ia E_a'i' E_r'j' |N~> into
        d_aa' (2 d_ii' d_jj' - d_ij' d_ji') <M~| 2 d_rr' - E_r'r |N~>,
    the hole-type density of the active index.
  * With a diagonal f, [f, E_a'i' E_r'j'] = (eps_a' - eps_i' + eps_r' -
    eps_j') E_a'i' E_r'j', and f on |core, N~> leaves f_act, whose matrix
    between XMS states is diag(E~); the operator of Eq. 10 is the same
    pattern with <M~| (2 d_rr' - E_r'r) (f_act + eps_a' - eps_i' - eps_j'
    + eps_r' + E_s - E~_L) |N~>.
  * The source <M~| E_jr E_ia H |L~>: the two-electron terms
    (a'i'|tj') E_a'i' E_tj' (from both orderings of the index classes) give
        sum_t (2 (ai|tj) - (aj|ti)) <M~| 2 d_rt - E_tr |L~>.

Rows are those of the packed layout: one per representative (i, j, a) with
i >= j (strictly for the '-' character of the (i j) swap), columns
(state M, active r) with the state slowest.  The XMS states and the
transition densities come from oracle/cavv_closed.py's CI helpers.
"""
from __future__ import annotations

import math

import numpy as np

from oracle.cavv_closed import _densities

__all__ = ["ccav_rows"]


def ccav_rows(prob, L: int, reps, t_plus, t_minus, with_source: bool = True, dens=None):
    """Packed residual rows of state L at the given representatives.

    reps: list of (i, j, a) with i >= j (closed 0..nc-1, virtual a in
    0..nv-1).  t_plus[k], t_minus[k]: the packed rows (length nst * na,
    columns (M, r)) of representative k; t_minus[k] is ignored (and may be
    None) where i == j.  dens: an earlier call's densities (optional).
    Returns (sig_plus, sig_minus, dens) with arrays [len(reps), nst * na];
    sig_minus rows without a '-' row are NaN."""
    nc, na, nv, nst = prob.nc, prob.na, prob.nv, prob.nst
    if na == 0:
        raise ValueError("ccav needs active orbitals")
    fock = np.asarray(prob.fock)
    if np.any(fock != np.diag(np.diag(fock))):
        raise ValueError("the closed form needs a diagonal Fock operator")
    eps = np.asarray(prob.eps)
    if dens is None:
        dens = _densities(prob)
    gam, g, E = dens                                   # gam[M, N, p, q] = <M~|E_pq|N~>
    B = np.asarray(prob.B)
    a0, v0 = nc, nc + na
    shift = float(prob.shift)
    n = nst * na
    two = 2.0 * np.einsum("MN,rq->MrNq", np.eye(nst), np.eye(na))
    # [M, r, N, r'] = <M~| 2 d_rr' - E_r'r |N~> and the same followed by f_act
    H1 = (two - gam.transpose(0, 3, 1, 2)).reshape(n, n)
    HF = (two * E[None, None, :, None] - g.transpose(0, 3, 1, 2)).reshape(n, n)
    eps_col = np.tile(eps[a0:a0 + na], nst)            # eps_r' per column (N, r')
    sig_p = np.full((len(reps), n), np.nan)
    sig_m = np.full((len(reps), n), np.nan)
    for k, (i, j, a) in enumerate(reps):
        if not (nc > i >= j >= 0 and nv > a >= 0):
            raise ValueError("not a canonical representative")
        imgs = [(i, j, a)] if i == j else [(i, j, a), (j, i, a)]
        wgt = 1.0 / math.sqrt(len(imgs))
        tp = np.asarray(t_plus[k], dtype=float)
        tm = np.asarray(t_minus[k], dtype=float) if i > j else np.zeros(n)
        x = {imgs[0]: wgt * (tp + tm)}
        if i > j:
            x[imgs[1]] = wgt * (tp - tm)
        c0 = eps[v0 + a] - eps[i] - eps[j] + shift - E[L]
        Kx = {e: HF @ x[e] + H1 @ (x[e] * (c0 + eps_col)) for e in imgs}
        sig = {}
        for (p, q, c) in imgs:
            s = 2.0 * Kx[(p, q, c)] - Kx[(q, p, c)]
            if with_source:
                # w_t = 2 (c p|t q) - (c q|t p)
                wt = (2.0 * (B[:, a0:a0 + na, q].T @ B[:, v0 + c, p])
                      - B[:, a0:a0 + na, p].T @ B[:, v0 + c, q])
                v = -np.einsum("Mtr,t->Mr", gam[:, L], wt)
                v[L] += 2.0 * wt
                s = s + v.reshape(n)
            sig[(p, q, c)] = s
        sig_p[k] = wgt * sum(sig[e] for e in imgs)
        if i > j:
            sig_m[k] = wgt * (sig[imgs[0]] - sig[imgs[1]])
    return sig_p, sig_m, dens
