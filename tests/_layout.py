"""The packed amplitude layout of the C ABI, written from its description in
include/caspt2.h, for comparing the library with the brute-force oracle
(O1, explicit determinants) without going through the factorised oracle.

O1 works in the basis of the individual functions E_Omega|N~> of Eq. 8: one
coefficient per operator type of Eq. 8, per value of its four orbital
indices and per ket state N (MS-MR) or N = L (SS-SR).  The library stores
per block and exchange character a row per canonical orbit representative
of the external indices; a function with external indices e relates to the
packed rows by x[e] = sum_chi chi(pi_e) t_chi[rep] / sqrt(|orbit|).  This
module builds that map as a dense matrix U (functions x packed), so that
packed quantities are U^T applied to O1's (residuals, sources, T, lambda) and
O1's trial vectors are U t.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

# Blocks in the packed order; per block: the external slots with their orbital
# space, the swaps of external slots, the number of active indices, and for
# every operator type of Eq. 8 in the block (O1 type index, where each slot
# comes from in (p, q, r, s) of E_pq E_rs, where each active index comes from).
_BLOCKS = [
    # ccvv  E_ai E_bj  slots (i, j, a, b)
    ("ccvv", "ccvv", [(0, 1), (2, 3)], 0, [(0, (1, 3, 0, 2), ())]),
    # cavv  E_ar E_bi  slots (i, a, b)
    ("cavv", "cvv", [(1, 2)], 1, [(1, (3, 0, 2), (1,))]),
    # aavv  E_ar E_bs  slots (a, b)
    ("aavv", "vv", [(0, 1)], 2, [(2, (0, 2), (1, 3))]),
    # ccav  E_ai E_rj  slots (i, j, a)
    ("ccav", "ccv", [(0, 1)], 1, [(3, (1, 3, 0), (2,))]),
    # ccaa  E_ri E_sj  slots (i, j)
    ("ccaa", "cc", [(0, 1)], 2, [(4, (1, 3), (0, 2))]),
    # aaav  E_ar E_st  slot (a)
    ("aaav", "v", [], 3, [(5, (0,), (1, 2, 3))]),
    # caaa  E_ri E_st  slot (i)
    ("caaa", "c", [], 3, [(6, (1,), (0, 2, 3))]),
    # caav  E_ai E_rs (type 0), E_ar E_si (type 1)  slots (i, a)
    ("caav", "cv", [], 2, [(7, (1, 0), (2, 3)), (8, (3, 0), (1, 2))]),
]


def _characters(name, swaps):
    if name == "ccvv":
        return [(1, 1), (-1, -1)]
    if swaps:
        return [(1,), (-1,)]
    return [()]


class PackedLayout:
    """Packed layout of one function set (all states in MS-MR, or one in
    SS-SR) for orbital spaces nc, na, nv and nst reference states."""

    def __init__(self, nc, na, nv, nst, scheme="MSMR"):
        self.nc, self.na, self.nv, self.nst = nc, na, nv, nst
        self.nsta = nst if scheme == "MSMR" else 1
        dim = {"c": nc, "v": nv}
        self.entries = []        # (block, chi, reps, offset, nalpha)
        self.row_of = {}         # (block, chi) -> {rep: row}
        off = 0
        for name, spaces, swaps, nact, types in _BLOCKS:
            nalpha = self.nsta * len(types) * na ** nact
            ranges = [range(dim[sp]) for sp in spaces]
            for chi in _characters(name, swaps):
                reps = []
                for e in itertools.product(*ranges):
                    if all(e[k] > e[l] or (e[k] == e[l] and c == 1) for (k, l), c in zip(swaps, chi)):
                        reps.append(e)
                self.entries.append((name, chi, reps, off, nalpha))
                self.row_of[(name, chi)] = {e: r for r, e in enumerate(reps)}
                off += len(reps) * nalpha
        self.length = off

    def _images(self, swaps, e0):
        """Distinct images of e0 under subsets of the swaps, with the swap
        subset that first produced each."""
        out = {}
        for bits in itertools.product((0, 1), repeat=len(swaps)):
            e = list(e0)
            for (k, l), f in zip(swaps, bits):
                if f:
                    e[k], e[l] = e[l], e[k]
            out.setdefault(tuple(e), bits)
        return out

    def unpack_matrix(self, keys):
        """U [len(keys)][length]: coefficient of each O1 function (keys from
        oracle.brute: (type, (p, q, r, s), N)) in terms of the packed rows."""
        nc, na = self.nc, self.na
        U = np.zeros((len(keys), self.length))
        info = {name: (spaces, swaps, nact, types) for name, spaces, swaps, nact, types in _BLOCKS}
        ent = {(name, chi): (reps, off, nalpha) for name, chi, reps, off, nalpha in self.entries}
        for kidx, (t, pqrs, N) in enumerate(keys):
            for name, (spaces, swaps, nact, types) in info.items():
                hit = [(ti, src, asrc) for ti, (tt, src, asrc) in enumerate(types) if tt == t]
                if hit:
                    break
            ti, src, asrc = hit[0]
            e = []
            for sp, k in zip(spaces, src):
                v = pqrs[k]
                e.append(v if sp == "c" else v - nc - na)
            e = tuple(e)
            tup = 0
            for k in asrc:
                tup = tup * na + (pqrs[k] - nc)
            st = N if self.nsta > 1 else 0
            alpha = (st * len(types) + ti) * na ** nact + tup
            # the canonical representative of e's orbit and the swaps that map it to e
            for chi in _characters(name, swaps):
                reps, off, nalpha = ent[(name, chi)]
                rows = self.row_of[(name, chi)]
                # find rep: sort each swapped pair into (larger, smaller)
                r = list(e)
                for (k, l) in swaps:
                    if r[k] < r[l]:
                        r[k], r[l] = r[l], r[k]
                r = tuple(r)
                if r not in rows:
                    continue          # e.g. a '-' character of a pair with equal indices
                imgs = self._images(swaps, r)
                bits = imgs[e]
                sgn = 1.0
                for c, f in zip(chi, bits):
                    if f:
                        sgn *= c
                U[kidx, off + rows[r] * nalpha + alpha] += sgn / math.sqrt(len(imgs))
        return U
