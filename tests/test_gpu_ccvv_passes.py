"""Coupling terms (Eq. 10 with the Fock operator of Eq. 11) applied in
packed-row passes -- the up terms into ccvv (from cavv through f(active,
closed), from ccav through f(virtual, active), from caav through f(virtual,
closed)), the down terms out of ccvv into cavv, caav and ccav, and the terms
between cavv and aavv/aaav -- against the same terms applied one at a time
through the all-orderings tensors and their packing (the form every other
coupling takes, itself checked against both oracles in the parity tests).

Bars: FP64 residuals of every state within 1e-12 of the largest element (the
two forms only sum the same products in another order); FP32 residuals of
the inner solver within 1e-5 relative of each other (both round every
product to FP32; the passes keep their partial sums in FP64).  Cases: several
closed pairs and a single one (no '-' rows), virtual counts off the 16-wide
tile (ragged tiles), 1-4 states (1-4 columns -- four takes the vector row
accesses --, and the 1-column function sets of SS-SR), rotated orbitals (Reading C: within-block terms into ccvv keep
the all-orderings sigma beside the passes), forty closed orbitals (the
in-pass active contraction in more than one round of matrix-core tiles), and
a Fock operator with only the closed-virtual block between orbital spaces
(one pass alone)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth.gen import make_problem, random_vector  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1606_01273_amd import lib
    lib()
    return torch.device("cuda")


def _rel(a, b):
    return float(torch.max(torch.abs(a - b))) / max(float(torch.max(torch.abs(b))), 1e-300)


def _pair(p, scheme, precision=None):
    """(term-by-term handle, packed-row-pass handle) of one problem"""
    from paper_1606_01273_amd import MIXED, MSMR, SSSR, Caspt2, lib
    L = lib()
    kw = {"scheme": MSMR if scheme == "MSMR" else SSSR}
    if precision is not None:
        kw["precision"] = MIXED
    prev = L.caspt2_debug_ccvv_passes(0)
    try:
        g0 = Caspt2.from_problem(p, **kw)
    finally:
        L.caspt2_debug_ccvv_passes(1)
    g1 = Caspt2.from_problem(p, **kw)
    L.caspt2_debug_ccvv_passes(prev)
    return g0, g1


CASES = [
    ((10, 6, 120, 400, 3), 1, "B", "MSMR"),
    ((3, 4, 10, 40, 2), 7, "B", "SSSR"),
    ((1, 3, 5, 20, 2), 3, "B", "MSMR"),
    ((4, 4, 17, 50, 1), 4, "B", "MSMR"),
    ((5, 4, 30, 70, 2), 9, "C", "MSMR"),
    ((40, 6, 5, 120, 3), 2, "B", "MSMR"),
    ((4, 4, 18, 50, 4), 6, "B", "MSMR"),
]


@pytest.mark.parametrize("dims,seed,reading,scheme", CASES)
def test_passes_match_term_path(dev, dims, seed, reading, scheme):
    from paper_1606_01273_amd import lib
    L = lib()
    print("case", dims, seed, reading, scheme, flush=True)
    p = make_problem(*dims, seed=seed, reading=reading, shift=0.2)
    g0, g1 = _pair(p, scheme)
    nsets = p.nst if scheme == "SSSR" else 1
    for s in range(nsets):
        assert L.caspt2_debug_ccvv_passes_used(g0._h, s) == 0
        assert L.caspt2_debug_ccvv_passes_used(g1._h, s) == 7   # ccvv up, ccvv down, cavv
    x = torch.tensor(random_vector(g0.length, seed + 100), device=dev)
    for st in range(p.nst):
        ref = torch.empty_like(x)
        got = torch.empty_like(x)
        g0.residual(st, x, ref, with_source=True)
        g1.residual(st, x, got, with_source=True)
        r = _rel(got, ref)
        print(f"  state {st}: {r:.3e}", flush=True)
        assert r < 1e-12
    g0.close()
    g1.close()


def test_passes_match_term_path_full_workload(dev):
    """The benchmark's workload (30 closed, 8 active, 400 virtual orbitals,
    1500 auxiliary functions, 4 states, Reading B): the residual of one state
    with the packed-row passes (four columns: whole-row vector accesses)
    against the term-by-term path, 1e-12 of the largest element."""
    from synth.gen import workload_problem
    from paper_1606_01273_amd import lib
    L = lib()
    p = workload_problem("full", "B")
    g0, g1 = _pair(p, "MSMR")
    assert L.caspt2_debug_ccvv_passes_used(g1._h, 0) == 7
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    x = torch.randn(g0.length, dtype=torch.float64, device=dev, generator=gen)
    ref = torch.empty_like(x)
    got = torch.empty_like(x)
    g0.residual(1, x, ref, with_source=True)
    g0.close()
    g1.residual(1, x, got, with_source=True)
    g1.close()
    r = _rel(got, ref)
    print(f"  full workload, state 1: {r:.3e}", flush=True)
    assert r < 1e-12


def test_passes_closed_virtual_block_only(dev):
    """Only f(closed, virtual) couples orbital spaces: the caav terms alone
    (the virtual-pair passes without the cavv contractions)."""
    import copy
    p = make_problem(4, 4, 20, 60, 2, seed=11, reading="B", shift=0.2)
    q = copy.deepcopy(p)
    f = np.array(q.fock, copy=True)
    nc, na = q.nc, q.na
    act = slice(nc, nc + na)
    f[act, :nc] = f[:nc, act] = 0.0
    f[act, nc + na:] = f[nc + na:, act] = 0.0
    q.fock = f
    g0, g1 = _pair(q, "MSMR")
    x = torch.tensor(random_vector(g0.length, 12), device=dev)
    for st in range(q.nst):
        ref = torch.empty_like(x)
        got = torch.empty_like(x)
        g0.residual(st, x, ref, with_source=False)
        g1.residual(st, x, got, with_source=False)
        r = _rel(got, ref)
        print(f"  state {st}: {r:.3e}", flush=True)
        assert r < 1e-12
    g0.close()
    g1.close()


@pytest.mark.parametrize("dims,seed", [((10, 6, 120, 400, 3), 1), ((3, 4, 17, 40, 2), 5), ((3, 4, 17, 40, 4), 5)])
def test_passes_fp32(dev, dims, seed):
    from paper_1606_01273_amd import lib
    L = lib()
    p = make_problem(*dims, seed=seed, reading="B", shift=0.2)
    g0, g1 = _pair(p, "MSMR", precision="mixed")
    rng = np.random.default_rng(seed)
    for st in range(p.nst):
        x = torch.tensor(rng.standard_normal(g0.length), dtype=torch.float32, device=dev)
        s0 = torch.empty_like(x)
        s1 = torch.empty_like(x)
        assert L.caspt2_debug_residual_f32(g0._h, st, x.data_ptr(), s0.data_ptr()) == 0
        assert L.caspt2_debug_residual_f32(g1._h, st, x.data_ptr(), s1.data_ptr()) == 0
        r = float(torch.linalg.norm((s1 - s0).double()) / torch.linalg.norm(s0.double()))
        print(f"  FP32 state {st}: {r:.3e}", flush=True)
        assert r < 1e-5
    g0.close()
    g1.close()
