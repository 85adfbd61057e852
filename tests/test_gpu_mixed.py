"""Mixed-precision mode (FP64 refinement around an FP32 inner PCG) against
the CPU oracle and against the FP64 mode of the library.

Bar: energies (H_eff, E^MS) within 1e-8 Eh of the FP64 oracle; amplitudes
and lambda within 1e-8 relative.  The refinement loop converges the FP64
residual to the same tolerance as the FP64 solver, so the observed errors
are printed next to the bars.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth.gen import make_problem  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1606_01273_amd import lib
    lib()
    return torch.device("cuda")


def _ok(err, tol, what):
    err = float(err)
    print(f"  {what}: {err:.3e} (bar {tol:.0e})", flush=True)
    if not err < tol:
        pytest.fail(f"{what}: error {err:.3e} >= {tol:.1e}")


def test_debug_gemm_f32_matches_numpy(dev):
    from paper_1606_01273_amd import lib
    rng = np.random.default_rng(0)
    for (M, N, K, nk) in [(1, 1, 1, 1), (17, 33, 5, 1), (64, 64, 16, 0), (130, 70, 37, 0),
                          (200, 129, 300, 1), (1000, 8, 8, 0)]:
        A = rng.standard_normal((M, K)).astype(np.float32)
        B = (rng.standard_normal((N, K)) if nk else rng.standard_normal((K, N))).astype(np.float32)
        ta = torch.tensor(A, device=dev)
        tb = torch.tensor(B, device=dev)
        tc = torch.empty((M, N), dtype=torch.float32, device=dev)
        assert lib().caspt2_debug_gemm_f32(nk, M, N, K, ta.data_ptr(), tb.data_ptr(), tc.data_ptr()) == 0
        ref = A.astype(np.float64) @ (B.T if nk else B).astype(np.float64)
        # FP32 dot products of length K: error below K * 2^-24 * sum |a_k b_k|
        bound = K * 2.0 ** -24 * (np.abs(A).astype(np.float64) @ np.abs(B.T if nk else B).astype(np.float64))
        excess = np.abs(tc.cpu().numpy().astype(np.float64) - ref) - bound
        assert excess.max() <= 0.0, f"gemm_f32 {(M, N, K, nk)} exceeds the rounding bound"


@pytest.mark.parametrize("reading", ["A", "B"])
def test_residual_f32_matches_oracle(dev, reading):
    """The FP32 residual of the inner solver against the FP64 oracle, without
    the source term.  Six active orbitals and two states: the entries with 72,
    144 and 432 internal functions take the dense FP32 MFMA path, with 1 to
    2485 rows (several tiles and ragged tails in both dimensions).

    Bar: the FP32 path chains three products (basis transform, dense block,
    back transform) of length at most 2 * 432; each adds at most n * 2^-24
    relative to the magnitudes it sums, so ||sigma32 - sigma|| / ||sigma||
    stays below 3 * 864 * 2^-24 = 1.6e-4 for the well-conditioned random x
    used here; a wrong operand or output layout gives O(1)."""
    from oracle.ic import Caspt2Oracle
    from paper_1606_01273_amd import MIXED, Caspt2, lib
    p = make_problem(2, 6, 70, 100, 2, seed=7, reading=reading, shift=0.1)
    o = Caspt2Oracle(p, "MSMR", xms=True)
    g = Caspt2.from_problem(p, precision=MIXED)
    assert g.length == o.length
    g.xms_rotate()
    rng = np.random.default_rng(5)
    for L in range(p.nst):
        x = rng.standard_normal(g.length)
        tx = torch.tensor(x, dtype=torch.float32, device=dev)
        ts = torch.empty_like(tx)
        assert lib().caspt2_debug_residual_f32(g._h, L, tx.data_ptr(), ts.data_ptr()) == 0
        ref = o.residual(L, x, with_source=False)
        got = ts.cpu().numpy().astype(np.float64)
        _ok(np.linalg.norm(got - ref) / np.linalg.norm(ref), 1.6e-4, f"FP32 residual L {L}")
    g.close()


CASES = [
    ((2, 3, 3, 16, 3), 7, "A", "MSMR", True, 0.15),
    ((5, 4, 30, 70, 2), 8, "A", "MSMR", True, 0.2),
    ((3, 4, 10, 40, 2), 7, "B", "SSSR", True, 0.2),
    ((5, 4, 30, 70, 2), 8, "B", "MSMR", True, 0.2),
    ((3, 3, 9, 30, 3), 7, "B", "MSMR", False, 0.1),
    ((3, 3, 7, 26, 2), 9, "C", "MSMR", True, 0.2),
]


@pytest.mark.parametrize("dims,seed,reading,scheme,xms,shift", CASES)
def test_mixed_matches_oracle(dev, dims, seed, reading, scheme, xms, shift):
    from oracle.ic import Caspt2Oracle
    from paper_1606_01273_amd import MIXED, MSMR, SSSR, Caspt2
    print("case", dims, seed, reading, scheme, xms, shift, flush=True)
    p = make_problem(*dims, seed=seed, reading=reading, shift=shift)
    o = Caspt2Oracle(p, scheme, xms=xms).run(P=0)
    g = Caspt2.from_problem(p, scheme=MSMR if scheme == "MSMR" else SSSR, xms=xms, precision=MIXED)
    rc, info = g.solve_amplitudes(tol=1e-11, maxiter=400)
    assert rc == 0, f"amplitude solve status {rc}"
    assert all(i["refinements"] >= 1 for i in info)
    print("  amplitude solve: FP32 iterations", [i["iters"] for i in info],
          "refinements", [i["refinements"] for i in info], flush=True)
    H, w, R = g.heff()
    _ok(np.abs(H - o.H_eff).max(), 1e-8, "H_eff vs oracle (Eh)")
    _ok(np.abs(w - o.e_ms).max(), 1e-8, "E_MS vs oracle (Eh)")
    for L in range(p.nst):
        T = g.amplitudes(L).cpu().numpy()
        _ok(np.linalg.norm(T - o.T[L]) / max(np.linalg.norm(o.T[L]), 1e-300), 1e-8, f"T L {L}")
    rc, info = g.solve_lambda(0, tol=1e-11, maxiter=400)
    assert rc == 0, f"lambda solve status {rc}"
    scale = max(np.linalg.norm(v) for v in o.lam)
    for L in range(p.nst):
        lam = g.lam(L).cpu().numpy()
        _ok(np.linalg.norm(lam - o.lam[L]) / scale, 1e-8, f"lambda L {L}")
        _ok(abs(np.linalg.norm(lam) - np.linalg.norm(o.lam[L])) / scale, 1e-8, f"|lambda| L {L}")
    g.close()


def test_mixed_matches_fp64_mid_size(dev):
    """Three-state XMS problem with 10 closed, 6 active, 120 virtual orbitals
    (the aavv entries take the dense FP32 GEMM path): the mixed mode against
    the FP64 mode of the library, couplings on."""
    from paper_1606_01273_amd import FP64, MIXED, Caspt2
    p = make_problem(10, 6, 120, 400, 3, seed=1, reading="B", shift=0.2)
    res = {}
    for prec in (FP64, MIXED):
        g = Caspt2.from_problem(p, precision=prec)
        rc, info = g.solve_amplitudes(tol=1e-10, maxiter=400)
        assert rc == 0
        H, w, R = g.heff()
        rc, linfo = g.solve_lambda(0, tol=1e-10, maxiter=400)
        assert rc == 0
        res[prec] = (w, [g.lam(L).cpu().numpy() for L in range(p.nst)],
                     [i["iters"] for i in info], [i["refinements"] for i in info])
        g.close()
    print("  FP64 iterations", res[FP64][2], "mixed FP32 iterations", res[MIXED][2],
          "refinements", res[MIXED][3], flush=True)
    _ok(np.abs(res[FP64][0] - res[MIXED][0]).max(), 1e-8, "E_MS mixed vs FP64 (Eh)")
    scale = max(np.linalg.norm(v) for v in res[FP64][1])
    for L in range(p.nst):
        _ok(np.linalg.norm(res[FP64][1][L] - res[MIXED][1][L]) / scale, 1e-8, f"lambda L {L}")
