"""Batched solves (caspt2_batch_solve): many uneven problems in one grouped
PCG with amplitude and lambda systems interleaved.

Each problem of a small uneven batch is checked against the CPU oracle at
the FP64 bars (1e-10 Eh on energies, 1e-8 relative on amplitudes and
lambda); a larger batch drawn like the 64-instance workload is checked
against the per-problem solves of the library.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth.gen import batch_sizes, make_problem  # noqa: E402


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


# (dims, seed, reading, shift, target): uneven orbital spaces and state counts
SMALL = [
    ((2, 3, 3, 16, 3), 7, "B", 0.15, 2),
    ((4, 4, 20, 60, 1), 7, "A", 0.0, 0),
    ((5, 4, 30, 70, 2), 8, "B", 0.2, 1),
    ((3, 3, 9, 30, 3), 7, "A", 0.1, 0),
    ((3, 4, 10, 40, 2), 7, "B", 0.2, 0),
    ((1, 2, 5, 16, 2), 3, "B", 0.2, 1),
]


def test_batch_matches_oracle(dev):
    from oracle.ic import Caspt2Oracle
    from paper_1606_01273_amd import Caspt2, batch_solve
    probs = [make_problem(*d, seed=s, reading=r, shift=sh) for d, s, r, sh, _ in SMALL]
    targets = [c[4] for c in SMALL]
    gs = [Caspt2.from_problem(p) for p in probs]
    rc, ainfo, linfo = batch_solve(gs, targets, tol=1e-11, maxiter=300)
    assert rc == 0, f"batch status {rc}"
    for i, (p, g, P) in enumerate(zip(probs, gs, targets)):
        print("problem", i, SMALL[i][:3], "amp iters", [a["iters"] for a in ainfo[i]],
              "lambda iters", [a["iters"] for a in linfo[i]], flush=True)
        o = Caspt2Oracle(p, "MSMR").run(P=P)
        assert all(a["flags"] & 1 for a in ainfo[i]) and all(a["flags"] & 1 for a in linfo[i])
        for L in range(p.nst):
            T = g.amplitudes(L).cpu().numpy()
            _ok(np.linalg.norm(T - o.T[L]) / max(np.linalg.norm(o.T[L]), 1e-300), 1e-8, f"T {i} L {L}")
        H, w, R = g.heff()
        _ok(np.abs(H - o.H_eff).max(), 1e-10, f"H_eff {i}")
        _ok(np.abs(w - o.e_ms).max(), 1e-10, f"E_MS {i}")
        scale = max(np.linalg.norm(v) for v in o.lam)
        for L in range(p.nst):
            lam = g.lam(L).cpu().numpy()
            _ok(np.linalg.norm(lam - o.lam[L]) / scale, 1e-8, f"lambda {i} L {L}")
    for g in gs:
        g.close()


def test_batch_mixed_matches_oracle(dev):
    """The same uneven batch in the mixed mode (FP32 grouped inner PCG, FP64
    refinement per system): energies within 1e-8 Eh of the oracle, T and
    lambda within 1e-6 relative, every system with a non-zero right-hand side
    refined at least once."""
    from oracle.ic import Caspt2Oracle
    from paper_1606_01273_amd import MIXED, Caspt2, batch_solve
    probs = [make_problem(*d, seed=s, reading=r, shift=sh) for d, s, r, sh, _ in SMALL]
    targets = [c[4] for c in SMALL]
    gs = [Caspt2.from_problem(p, precision=MIXED) for p in probs]
    rc, ainfo, linfo = batch_solve(gs, targets, tol=1e-10, maxiter=400)
    assert rc == 0, f"batch status {rc}"
    for i, (p, g, P) in enumerate(zip(probs, gs, targets)):
        print("problem", i, SMALL[i][:3], "amp iters/refinements",
              [(a["iters"], a["refinements"]) for a in ainfo[i]],
              "lambda", [(a["iters"], a["refinements"]) for a in linfo[i]], flush=True)
        assert all(a["flags"] & 1 and a["resnorm"] <= 1e-10 for a in ainfo[i] + linfo[i])
        # a system whose right-hand side vanishes (a lambda state with R_LP = 0)
        # is solved at the start, without refinement
        assert all(a["refinements"] >= 1 or a["iters"] == 0 for a in ainfo[i] + linfo[i])
        o = Caspt2Oracle(p, "MSMR").run(P=P)
        for L in range(p.nst):
            T = g.amplitudes(L).cpu().numpy()
            _ok(np.linalg.norm(T - o.T[L]) / max(np.linalg.norm(o.T[L]), 1e-300), 1e-6, f"T {i} L {L}")
        H, w, R = g.heff()
        _ok(np.abs(w - o.e_ms).max(), 1e-8, f"E_MS {i}")
        scale = max(np.linalg.norm(v) for v in o.lam)
        for L in range(p.nst):
            lam = g.lam(L).cpu().numpy()
            _ok(np.linalg.norm(lam - o.lam[L]) / scale, 1e-6, f"lambda {i} L {L}")
    for g in gs:
        g.close()


def test_batch_matches_single_solves(dev):
    """First 12 problems of the 64-instance uneven workload (closed 4-16,
    active 4-6, virtual 20-150, 1-4 states, shift 0.2, Fock couplings on):
    batched results equal the per-problem solves of the library.  Problems
    whose operator is not positive definite at this shift (intruder states:
    a non-positive denominator, or couplings between blocks that bring an
    eigenvalue below zero) must fail with E_INDEFINITE in both forms without
    stopping the others."""
    from paper_1606_01273_amd import E_INDEFINITE, Caspt2, Caspt2Error, batch_solve
    sizes = batch_sizes(64, seed=4)[:12]
    probs = [make_problem(nc, na, nv, nx, ns, seed=sd, reading="B", shift=0.2)
             for nc, na, nv, nx, ns, sd in sizes]
    single = []
    for p in probs:
        g = Caspt2.from_problem(p)
        try:
            rc, _ = g.solve_amplitudes(tol=1e-10, maxiter=300)
        except Caspt2Error as ex:
            assert ex.code == E_INDEFINITE
            print("single solve:", ex, flush=True)
            single.append(None)
            g.close()
            continue
        assert rc == 0
        H, w, R = g.heff()
        rc, _ = g.solve_lambda(0, tol=1e-10, maxiter=300)
        assert rc == 0
        single.append((w, [g.lam(L).cpu().numpy() for L in range(p.nst)]))
        g.close()
    gs = [Caspt2.from_problem(p) for p in probs]
    rc, ainfo, linfo = batch_solve(gs, [0] * len(gs), tol=1e-10, maxiter=300)
    n_bad = sum(s is None for s in single)
    print("intruder problems", [i for i, s in enumerate(single) if s is None], flush=True)
    assert rc == (E_INDEFINITE if n_bad else 0), f"batch status {rc}"
    for i, g in enumerate(gs):
        if single[i] is None:
            assert not all(a["flags"] & 1 for a in ainfo[i])
            assert not any(a["flags"] & 1 for a in linfo[i])
            g.close()
            continue
        H, w, R = g.heff()
        _ok(np.abs(w - single[i][0]).max(), 1e-10, f"E_MS {i}")
        scale = max(max(np.linalg.norm(v) for v in single[i][1]), 1e-300)
        for L in range(probs[i].nst):
            _ok(np.linalg.norm(g.lam(L).cpu().numpy() - single[i][1][L]) / scale, 1e-8, f"lambda {i} L {L}")
        g.close()


def test_batch_argument_errors(dev):
    from paper_1606_01273_amd import E_ARG, MIXED, Caspt2, Caspt2Error, batch_solve
    p = make_problem(2, 2, 3, 12, 2, seed=1, reading="A", shift=0.1)
    g = Caspt2.from_problem(p)
    with pytest.raises(Caspt2Error) as ex:
        batch_solve([g, g])
    assert ex.value.code == E_ARG
    with pytest.raises(Caspt2Error) as ex:
        batch_solve([g], [2])
    assert ex.value.code == E_ARG
    gm = Caspt2.from_problem(p, precision=MIXED)
    with pytest.raises(Caspt2Error) as ex:
        batch_solve([g, gm])             # precisions differ
    assert ex.value.code == E_ARG
    rc, a, l = batch_solve([g], [1])      # a batch of one
    assert rc == 0 and len(a) == 1 and len(a[0]) == 2
    g.close()
    gm.close()


def test_batch_workload_matches_stored_oracle(dev):
    """The 64-instance uneven workload solved in one batch against the CPU
    oracle's results stored in tests/golden/batch_B.jsonl (written by
    tests/golden/make_batch_golden.py, which calls the oracle only): E^MS of
    every problem the oracle solved (1e-10 Eh), and every problem the oracle
    finds not positive definite at this shift (a non-positive preconditioner
    denominator, or p.Ap <= 0) fails in the batch too, without stopping the
    others."""
    import json
    import os
    from paper_1606_01273_amd import E_INDEFINITE, Caspt2, batch_solve
    path = os.path.join(os.path.dirname(__file__), "golden", "batch_B.jsonl")
    with open(path) as fh:
        recs = [json.loads(line) for line in fh if line.strip()]
    sizes = batch_sizes(64, seed=4)
    assert sorted(r["index"] for r in recs) == list(range(64))
    for r in recs:
        assert tuple(r["dims"]) == sizes[r["index"]][:5] and r["seed"] == sizes[r["index"]][5]
    probs = [make_problem(nc, na, nv, nx, ns, seed=sd, reading="B", shift=0.2)
             for nc, na, nv, nx, ns, sd in sizes]
    gs = [Caspt2.from_problem(p) for p in probs]
    rc, ainfo, linfo = batch_solve(gs, [0] * len(gs), tol=1e-10, maxiter=300)
    bad_oracle = [r["index"] for r in recs if r["indefinite"]]
    print(f"{len(recs)} stored problems, {len(bad_oracle)} indefinite: {bad_oracle}", flush=True)
    assert rc in (0, E_INDEFINITE)
    for r in recs:
        i = r["index"]
        solved = all(a["flags"] & 1 for a in ainfo[i])
        if r["indefinite"]:
            assert not solved, f"problem {i}: the oracle finds it indefinite, the batch solved it"
            continue
        assert solved, f"problem {i}: the oracle solves it, the batch did not"
        H, w, R = gs[i].heff()
        _ok(np.abs(w - np.asarray(r["e_ms"])).max(), 1e-10, f"E_MS problem {i}")
    for g in gs:
        g.close()
