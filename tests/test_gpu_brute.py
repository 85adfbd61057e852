"""Parity of the HIP library with the brute-force oracle (O1) directly.

O1 builds every internally contracted function E_Omega|N~> of Eq. 8 on
explicit Slater determinants and takes S = V^T V, A_L = V^T (f - E_L + E_s) V
and the sources V^T H|N~> from the full operators (Eqs. 10, 15-17, 20); it
shares nothing with the library's factorised set-up.  The packed layout of
the C ABI is mapped onto O1's function basis by tests/_layout.py, written
from the header's description of that layout.  Compared: the XMS rotation
and E^(0) (1e-12), the sources of every ket state and the operator on random
vectors (1e-12 relative), T and lambda in the packed layout (1e-8 relative),
H^eff and E^MS (1e-10 Eh).  Cases: Readings A, B and C of the Fock matrix,
MS-MR and SS-SR, XMS and MS, on tiny inputs.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth.gen import make_problem  # noqa: E402
from tests._layout import PackedLayout  # noqa: E402

CASES = [
    # (reading, scheme, dims (nc, na, nv, naux, nst), xms)
    ("B", "MSMR", (2, 3, 3, 16, 3), True),
    ("B", "SSSR", (2, 3, 3, 16, 3), True),
    ("C", "MSMR", (2, 2, 3, 14, 2), True),
    ("A", "MSMR", (2, 3, 2, 14, 2), False),
    ("B", "MSMR", (2, 2, 3, 14, 2), False),
]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1606_01273_amd import lib
    lib()
    return torch.device("cuda")


def _ok(err, tol, what):
    err = float(err)
    if not err < tol:
        pytest.fail(f"{what}: error {err:.3e} >= {tol:.1e}")


def _rel(a, b):
    return float(np.abs(a - b).max() / max(1.0, np.abs(b).max()))


@pytest.mark.parametrize("reading,scheme,dims,xms", CASES)
def test_library_matches_brute_force(dev, reading, scheme, dims, xms):
    from oracle.brute import solve_brute
    from paper_1606_01273_amd import MSMR, SSSR, Caspt2, lib
    print("case", reading, scheme, dims, xms, flush=True)
    p = make_problem(*dims, seed=5, reading=reading, shift=0.15)
    o1 = solve_brute(p, scheme, xms=xms)
    lay = PackedLayout(p.nc, p.na, p.nv, p.nst, scheme)
    g = Caspt2.from_problem(p, scheme=MSMR if scheme == "MSMR" else SSSR, xms=xms)
    assert g.length == lay.length
    for k, (name, off, rows, nalpha) in enumerate(g.layout()):
        _, _, reps, off_r, nalpha_r = lay.entries[k]
        assert (off, rows, nalpha) == (off_r, len(reps), nalpha_r), f"layout entry {name}"
    U, e0 = g.xms_rotate()
    _ok(np.abs(U - o1["U"]).max(), 1e-12, "XMS U")
    _ok(np.abs(e0 - o1["e0"]).max(), 1e-12, "E0")
    rng = np.random.default_rng(17)
    Umap = {}
    for L in range(p.nst):
        d = o1["L"][L]
        Um = lay.unpack_matrix(d["keys"])
        Umap[L] = Um
        st = L if scheme == "SSSR" else 0
        # sources <M~|E_Omega^+ H|N~> of every ket state N
        if scheme == "SSSR" or L == 0:
            for N in range(p.nst):
                t = torch.empty(g.length, dtype=torch.float64, device=dev)
                assert lib().caspt2_debug_source(g._h, st, N, t.data_ptr()) == 0
                _ok(_rel(t.cpu().numpy(), Um.T @ d["V"][:, N]), 1e-12, f"source set {st} N {N}")
        # the operator of Eq. 10 with its source, on a random packed vector
        x = rng.standard_normal(g.length)
        ref = Um.T @ (d["A"] @ (Um @ x) + d["V"][:, L])
        tx = torch.tensor(x, device=dev)
        ts = torch.empty_like(tx)
        g.residual(L, tx, ts, with_source=True)
        _ok(_rel(ts.cpu().numpy(), ref), 1e-12, f"residual L {L}")
    rc, _ = g.solve_amplitudes(tol=1e-11, maxiter=300)
    assert rc == 0, f"amplitude solve status {rc}"
    H, w, R = g.heff()
    # O1's H^ref is <M~|H|N~> of the explicit Hamiltonian, which carries the
    # core energy constant on its diagonal; the library drops that constant
    # (H^ref = U^T diag(E^ref) U, Eq. 6): compare with it removed
    href_lib = o1["U"].T @ np.diag(p.eref) @ o1["U"]
    core = o1["href"] - href_lib
    const = float(np.mean(np.diag(core)))
    _ok(np.abs(core - const * np.eye(p.nst)).max(), 1e-10, "H^ref up to the core constant")
    _ok(np.abs(H + const * np.eye(p.nst) - o1["heff"]).max(), 1e-10, "H_eff")
    _ok(np.abs(w + const - o1["e_ms"]).max(), 1e-10, "E_MS")
    for L in range(p.nst):
        ref = Umap[L].T @ o1["L"][L]["T"]
        T = g.amplitudes(L).cpu().numpy()
        _ok(np.linalg.norm(T - ref) / max(np.linalg.norm(ref), 1e-300), 1e-8, f"T L {L}")
    rc, _ = g.solve_lambda(0, tol=1e-11, maxiter=300)
    assert rc == 0, f"lambda solve status {rc}"
    refs = [Umap[L].T @ o1["L"][L]["lam"] for L in range(p.nst)]
    scale = max(np.linalg.norm(v) for v in refs)
    for L in range(p.nst):
        lam = g.lam(L).cpu().numpy()
        _ok(np.linalg.norm(lam - refs[L]) / scale, 1e-8, f"lambda L {L}")
    g.close()
