"""Independent Slater-Condon evaluation for a single closed-shell
determinant reference (test helper; shares no code with oracle/)."""
import itertools

import numpy as np


def _sign_apply(det, ops):
    """Apply spin-orbital ops (list of ('c'|'a', so), rightmost first) to a
    determinant bit mask; return (sign, det) or None."""
    sgn = 1
    for kind, so in reversed(ops):
        occ = (det >> so) & 1
        below = bin(det & ((1 << so) - 1)).count("1")
        if kind == "a":
            if not occ:
                return None
            det &= ~(1 << so)
        else:
            if occ:
                return None
            det |= 1 << so
        if below % 2:
            sgn = -sgn
    return sgn, det


def mp2_like_energy(h, eri, eps, occ_spatial, cas_spatial, shift):
    """Second-order energy of a single determinant with doubly occupied
    spatial orbitals occ_spatial, over every single and double excitation
    that leaves the CAS (i.e. touches a non-CAS orbital), with diagonal
    zeroth-order energies sum of occupied orbital energies, and the shift
    correction: E2 = sum_D h_D^2 [-1/(d+s) - s/(d+s)^2]."""
    nmo = h.shape[0]
    nso = 2 * nmo
    sp = lambda so: so % nmo
    spin = lambda so: so // nmo
    def g(p, q, r, s):   # <pq|rs> in spin orbitals
        if spin(p) != spin(r) or spin(q) != spin(s):
            return 0.0
        return eri[sp(p), sp(r), sp(q), sp(s)]
    def ga(p, q, r, s):
        return g(p, q, r, s) - g(p, q, s, r)
    def H1(p, q):
        return h[sp(p), sp(q)] if spin(p) == spin(q) else 0.0
    occ = [s * nmo + i for s in (0, 1) for i in occ_spatial]
    vir = [so for so in range(nso) if so not in occ]
    phi = sum(1 << so for so in occ)
    e_of = lambda det: sum(eps[sp(so)] for so in range(nso) if (det >> so) & 1)
    e0 = e_of(phi)
    inside = lambda so: sp(so) in cas_spatial
    total = 0.0
    # singles a+_a a_i
    for i in occ:
        for a in vir:
            if inside(i) and inside(a):
                continue
            hd = H1(a, i) + sum(ga(a, j, i, j) for j in occ)
            if hd == 0.0:
                continue
            d = e_of(_sign_apply(phi, [("c", a), ("a", i)])[1]) - e0
            total += hd * hd * (-1.0 / (d + shift) - shift / (d + shift) ** 2)
    for i, j in itertools.combinations(occ, 2):
        for a, b in itertools.combinations(vir, 2):
            if all(inside(x) for x in (i, j, a, b)):
                continue
            hd = ga(a, b, i, j)
            if hd == 0.0:
                continue
            r = _sign_apply(phi, [("c", a), ("c", b), ("a", j), ("a", i)])
            d = e_of(r[1]) - e0
            total += hd * hd * (-1.0 / (d + shift) - shift / (d + shift) ** 2)
    return total
