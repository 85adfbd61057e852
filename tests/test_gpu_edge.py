"""Degenerate and edge cases of the method against the CPU oracle: no active
orbitals (the CASPT2 equations reduce to MP2), no closed or no virtual
orbitals (empty excitation blocks), a fully occupied and an empty active
space, an odd electron count, every CAS state a reference state, and the
smallest non-trivial problem.  FP64 bars: 1e-10 Eh on E^MS, 1e-8 relative
on T and lambda, 1e-12 relative on the residual of a random vector.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth.gen import make_problem, random_vector  # noqa: E402

CASES = [
    # (dims, extra generator arguments, shift)
    ((3, 0, 6, 20, 1), {}, 0.3),              # no active orbitals
    ((0, 3, 6, 20, 2), {}, 0.3),              # no closed orbitals
    ((3, 3, 0, 20, 2), {}, 0.3),              # no virtual orbitals
    ((2, 3, 4, 20, 1), {"nelec": 6}, 0.3),    # active space full (one determinant)
    ((2, 3, 4, 20, 1), {"nelec": 0}, 0.3),    # active space empty
    ((2, 3, 4, 20, 3), {"nelec": 1}, 0.3),    # odd electron count
    ((2, 2, 3, 12, 4), {}, 0.0),              # every CAS state a reference (degenerate F^ref)
    ((1, 2, 1, 8, 2), {}, 0.3),               # one closed, one virtual orbital
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


@pytest.mark.parametrize("reading", ["A", "B"])
@pytest.mark.parametrize("dims,kw,shift", CASES)
def test_edge_case_matches_oracle(dev, dims, kw, shift, reading):
    from oracle.ic import Caspt2Oracle
    from paper_1606_01273_amd import Caspt2
    print("case", dims, kw, shift, reading, flush=True)
    p = make_problem(*dims, seed=5, reading=reading, shift=shift, **kw)
    o = Caspt2Oracle(p, "MSMR").run(P=0)
    g = Caspt2.from_problem(p)
    assert g.length == o.length
    U, e0 = g.xms_rotate()
    _ok(np.abs(e0 - o.e0).max(), 1e-12, "E0")
    gaps = np.diff(np.sort(o.e0))
    if gaps.size and gaps.min() < 1e-8:     # degenerate F^ref: rotation not unique
        assert shift == 0.0, "E^MS is unique for a degenerate F^ref only without shift"
        _ok(np.abs(U.T @ U - np.eye(p.nst)).max(), 1e-12, "U orthogonal")
        D = U.T @ o.fref @ U
        _ok(np.abs(D - np.diag(np.diag(D))).max(), 1e-10, "U^T F^ref U diagonal")
        _ok(np.abs(np.diag(D) - o.e0).max(), 1e-10, "its diagonal = E0")
        rc, info = g.solve_amplitudes(tol=1e-11, maxiter=300)
        assert rc == 0
        H, w, R = g.heff()
        _ok(np.abs(w - o.e_ms).max(), 1e-10, "E_MS (degenerate F^ref)")
        g.close()
        return
    x = random_vector(g.length, 3)
    for L in range(p.nst):
        ts = torch.empty(g.length, dtype=torch.float64, device=dev)
        g.residual(L, torch.tensor(x, device=dev), ts, with_source=True)
        ref = o.residual(L, x, with_source=True)
        _ok(np.abs(ts.cpu().numpy() - ref).max() / max(np.abs(ref).max(), 1.0), 1e-12, f"residual L {L}")
    rc, info = g.solve_amplitudes(tol=1e-11, maxiter=300)
    assert rc == 0
    H, w, R = g.heff()
    _ok(np.abs(w - o.e_ms).max(), 1e-10, "E_MS")
    for L in range(p.nst):
        T = g.amplitudes(L).cpu().numpy()
        _ok(np.linalg.norm(T - o.T[L]) / max(np.linalg.norm(o.T[L]), 1e-12), 1e-8, f"T L {L}")
    rc, info = g.solve_lambda(0, tol=1e-11, maxiter=300)
    assert rc == 0
    scale = max(max(np.linalg.norm(v) for v in o.lam), 1e-12)
    for L in range(p.nst):
        _ok(np.linalg.norm(g.lam(L).cpu().numpy() - o.lam[L]) / scale, 1e-8, f"lambda L {L}")
    g.close()
