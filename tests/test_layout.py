"""CPU checks of the packed-layout helper used by the brute-force GPU test:
the map from packed rows to individual functions is an isometry, and with it
the brute-force oracle's operator, T and lambda reproduce the factorised
oracle's packed ones (two oracles, two routes to the packed layout)."""
import numpy as np

from oracle.brute import solve_brute
from oracle.ic import Caspt2Oracle
from synth.gen import make_problem
from tests._layout import PackedLayout


def test_layout_isometry_and_o1_packed_parity():
    p = make_problem(2, 3, 2, 14, 2, seed=5, reading="B", shift=0.15)
    o1 = solve_brute(p, "MSMR", xms=True)
    o2 = Caspt2Oracle(p, "MSMR", xms=True).run()
    lay = PackedLayout(p.nc, p.na, p.nv, p.nst, "MSMR")
    assert lay.length == o2.length
    rng = np.random.default_rng(0)
    for L in range(p.nst):
        d = o1["L"][L]
        U = lay.unpack_matrix(d["keys"])
        assert np.abs(U.T @ U - np.eye(lay.length)).max() < 1e-14
        x = rng.standard_normal(lay.length)
        ref = o2.residual(L, x, with_source=True)
        got = U.T @ (d["A"] @ (U @ x) + d["V"][:, L])
        assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
        assert np.linalg.norm(U.T @ d["T"] - o2.T[L]) <= 1e-8 * np.linalg.norm(o2.T[L])
