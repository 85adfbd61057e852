"""caspt2_residual_all (the benchmark's step): every state's residual
(Eq. 10, with the source) of one problem in one call.  The states alternate
between two streams, the second in reverse entry order and, with couplings,
on the handle's second work set; the results must equal the one-state calls
bit for bit (the same launches on the same data).  Checked at the mid size
with and without couplings and autotuned launches, and at the full size in
the benchmark's launch configuration.  The one-state residual itself is
checked against the oracle in the parity and stored-value tests.
"""
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


def _check(g, nst, seed):
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    x = torch.randn((nst, g.length), dtype=torch.float64, device="cuda", generator=gen)
    s_all = torch.empty_like(x)
    g.residual_all(x, s_all)
    one = torch.empty(g.length, dtype=torch.float64, device="cuda")
    for L in range(nst):
        g.residual(L, x[L], one, with_source=True)
        diff = float(torch.max(torch.abs(one - s_all[L])))
        print(f"  state {L}: max |all - one| = {diff:.3e}", flush=True)
        assert torch.equal(one, s_all[L]), f"state {L}"


@pytest.mark.parametrize("reading", ["A", "B"])
def test_residual_all_equals_single_states_mid(dev, reading):
    from paper_1606_01273_amd import Caspt2
    p = make_problem(10, 6, 120, 400, 3, seed=1, reading=reading, shift=0.2)
    g = Caspt2.from_problem(p)
    _check(g, p.nst, 3)
    g.autotune()
    _check(g, p.nst, 4)
    g.close()


def test_residual_all_equals_single_states_full(dev):
    from paper_1606_01273_amd import Caspt2
    p = make_problem(30, 8, 400, 1500, 4, seed=8, reading="A", shift=0.2)
    g = Caspt2.from_problem(p)
    g.autotune()
    _check(g, p.nst, 0)
    g.close()
