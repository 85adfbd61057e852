"""Correlated density matrices (Sec. II.D: d^(1), D^(1), d-bar^(2), N_L,
d^(2)) of the HIP library against the oracle: the brute-force one (explicit
determinants, every density written out as its matrix elements) at tiny
sizes, the factorised one at sizes spanning several tiles and ragged rows.
Both oracles are pinned on the CPU by finite differences of E^MS_P with
respect to h^c, the integrals and f.  Bar: 1e-10 of each quantity's largest
element (FP64)."""
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


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(1e-300, np.abs(b).max()))


def _library(p, scheme, xms, P):
    from paper_1606_01273_amd import MSMR, SSSR, Caspt2
    g = Caspt2.from_problem(p, scheme=MSMR if scheme == "MSMR" else SSSR, xms=xms)
    rc, _ = g.solve_amplitudes(tol=1e-12, maxiter=400)
    assert rc == 0
    g.heff()
    rc, _ = g.solve_lambda(P, tol=1e-12, maxiter=400)
    assert rc == 0
    d = g.densities()
    g.close()
    return d


@pytest.mark.parametrize("reading,scheme,dims,xms", [
    ("B", "MSMR", (2, 2, 2, 12, 2), True), ("B", "SSSR", (2, 2, 2, 12, 2), True),
    ("C", "MSMR", (2, 2, 3, 14, 2), True), ("A", "MSMR", (2, 3, 2, 14, 2), False)])
def test_densities_match_brute_force(dev, reading, scheme, dims, xms):
    from oracle.brute import densities_brute, solve_brute
    print("case", reading, scheme, dims, xms, flush=True)
    p = make_problem(*dims, seed=5, reading=reading, shift=0.15)
    P = 1
    ref = densities_brute(p, solve_brute(p, scheme, xms=xms, target=P))
    d = _library(p, scheme, xms, P)
    sl = {"c": slice(0, p.nc), "a": slice(p.nc, p.nc + p.na), "v": slice(p.nc + p.na, p.nmo)}
    _ok(_rel(d["d1"], ref["d1"]), 1e-10, "d1")
    scale = max(np.abs(ref["D1"]).max(), 1e-300)
    for k, v in d["D1"].items():
        r = ref["D1"][sl[k[0]], sl[k[1]], sl[k[2]], sl[k[3]]]
        _ok(np.abs(v.cpu().numpy() - r).max() / scale, 1e-10, f"D1 {''.join(k)}")
    _ok(_rel(d["dbar2"], ref["dbar2"]), 1e-10, "dbar2")
    _ok(_rel(d["d2"], ref["d2"]), 1e-10, "d2")
    _ok(_rel(d["NL"], ref["NL"]), 1e-10, "N_L")


@pytest.mark.parametrize("reading,scheme,dims,seed,xms", [
    ("B", "MSMR", (3, 4, 10, 40, 2), 7, True), ("B", "SSSR", (3, 4, 10, 40, 2), 7, True),
    ("B", "MSMR", (5, 4, 30, 70, 2), 8, True), ("C", "MSMR", (3, 3, 7, 26, 2), 9, True),
    ("A", "MSMR", (3, 3, 9, 30, 3), 7, False)])
def test_densities_match_oracle(dev, reading, scheme, dims, seed, xms):
    from oracle.ic import Caspt2Oracle
    print("case", reading, scheme, dims, seed, xms, flush=True)
    p = make_problem(*dims, seed=seed, reading=reading, shift=0.2)
    P = p.nst - 1
    ref = Caspt2Oracle(p, scheme, xms=xms).run(P).densities()
    d = _library(p, scheme, xms, P)
    _ok(_rel(d["d1"], ref["d1"]), 1e-10, "d1")
    scale = max(np.abs(v).max() for v in ref["D1"].values())
    for k, v in d["D1"].items():
        _ok(np.abs(v.cpu().numpy() - ref["D1"][k]).max() / scale, 1e-10, f"D1 {''.join(k)}")
    _ok(_rel(d["dbar2"], ref["dbar2"]), 1e-10, "dbar2")
    _ok(_rel(d["d2"], ref["d2"]), 1e-10, "d2")
    _ok(_rel(d["NL"], ref["NL"]), 1e-10, "N_L")


def test_densities_need_lambda(dev):
    from paper_1606_01273_amd import Caspt2, Caspt2Error, E_STATE
    p = make_problem(2, 2, 3, 12, 1, seed=1, reading="B", shift=0.1)
    g = Caspt2.from_problem(p)
    with pytest.raises(Caspt2Error) as ex:
        g.densities()
    assert ex.value.code == E_STATE
    g.close()
