"""Parity beyond the oracle's interactive sizes.

* Mid size (10 closed, 6 active, 120 virtual, 400 auxiliary, 3 states,
  Fock couplings on): stored oracle values in tests/golden/mid_B.json, written
  by tests/golden/make_golden.py (which calls the oracle only): the residual
  of Eq. 10 of every state at 256 sampled positions (and of state 0 at 64
  more), E^MS, and T and lambda at 256 sampled positions of every state.
  Bars: 1e-12 of the largest sampled residual; E^MS 1e-10 Eh (FP64) and
  1e-8 Eh (mixed); T and lambda elements 1e-8 of each vector's largest
  element, in both modes (the mixed mode refines to the same FP64 residual
  tolerance).
* Full size (30 closed, 8 active, 400 virtual, 1500 auxiliary, 4 states),
  in the launch configuration the benchmark times: properties that hold at
  any size -- the residual without source is linear in x and its operator is
  symmetric (Eq. 10 with a symmetric f and metric), with the Fock couplings
  between blocks on; and, with the canonical Fock operator, the ccvv, cavv,
  aavv and ccav rows (98.6 % of the vector, the dominant kernel and the
  dense matrix-core block among them) at sampled representatives against
  their closed forms (oracle/*_closed.py, each checked against the
  factorised oracle on every row of its block in small problems): every
  state, both characters, with the source on one stream and without it on
  two, at 1e-12 of the largest sampled value; then the FP32 operator of the
  mixed mode on the same rows (FP32-rounded x) at 1e-5.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth.gen import make_problem, random_vector  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


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


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_mid_matches_stored_oracle(dev, mode):
    from paper_1606_01273_amd import FP64, MIXED, Caspt2
    with open(os.path.join(HERE, "golden", "mid_B.json")) as fh:
        rec = json.load(fh)
    p = make_problem(*rec["dims"], seed=rec["seed"], reading=rec["reading"], shift=rec["shift"])
    g = Caspt2.from_problem(p, precision=FP64 if mode == "fp64" else MIXED)
    assert g.length == rec["length"]
    e_tol, v_tol = (1e-10, 1e-8) if mode == "fp64" else (1e-8, 1e-8)
    idx = np.asarray(rec["sample_index"])
    if mode == "fp64":
        x = torch.tensor(random_vector(g.length, rec["residual_x_seed"]), device=dev)
        s = torch.empty_like(x)
        g.residual(0, x, s, with_source=True)
        got = s.cpu().numpy()[np.asarray(rec["residual_index"])]
        ref = np.asarray(rec["residual_value"])
        _ok(np.abs(got - ref).max() / np.abs(ref).max(), 1e-12, "residual at sampled positions")
        for L in range(p.nst):
            g.residual(L, x, s, with_source=True)
            ref = np.asarray(rec["residual_sample"][L])
            _ok(np.abs(s.cpu().numpy()[idx] - ref).max() / np.abs(ref).max(), 1e-12, f"residual L {L} (256 samples)")
    rc, info = g.solve_amplitudes(tol=1e-11, maxiter=400)
    assert rc == 0
    H, w, R = g.heff()
    _ok(np.abs(w - np.asarray(rec["e_ms"])).max(), e_tol, f"E_MS ({mode}, Eh)")
    for L in range(p.nst):
        T = g.amplitudes(L)
        tn = float(torch.linalg.vector_norm(T))
        _ok(abs(tn - rec["t_norm"][L]) / rec["t_norm"][L], v_tol, f"|T| L {L}")
        got = T.cpu().numpy()[idx]
        _ok(np.abs(got - np.asarray(rec["t_sample"][L])).max() / rec["t_absmax"][L], 1e-8,
            f"T L {L} sampled elements")
    rc, info = g.solve_lambda(rec["target"], tol=1e-11, maxiter=400)
    assert rc == 0
    scale = max(rec["lambda_norm"])
    lscale = max(rec["lambda_absmax"])
    for L in range(p.nst):
        lam = g.lam(L)
        ln = float(torch.linalg.vector_norm(lam))
        _ok(abs(ln - rec["lambda_norm"][L]) / scale, v_tol, f"|lambda| L {L}")
        got = lam.cpu().numpy()[idx]
        _ok(np.abs(got - np.asarray(rec["lambda_sample"][L])).max() / lscale, 1e-8,
            f"lambda L {L} sampled elements")
    g.close()


def test_full_size_operator_linear_and_symmetric(dev):
    from paper_1606_01273_amd import Caspt2
    p = make_problem(30, 8, 400, 1500, 4, seed=8, reading="B", shift=0.2)
    g = Caspt2.from_problem(p)
    n = g.length
    print("full size vector length", n, flush=True)
    x = torch.tensor(random_vector(n, 21), device=dev)
    y = torch.tensor(random_vector(n, 22), device=dev)
    ax = torch.empty_like(x)
    ay = torch.empty_like(x)
    L = p.nst - 1
    g.residual(L, x, ax, with_source=False)
    g.residual(L, y, ay, with_source=False)
    xay = float(torch.dot(x, ay))
    yax = float(torch.dot(y, ax))
    _ok(abs(xay - yax) / max(abs(xay), 1e-300), 1e-11, "x.(A y) - y.(A x), relative")
    x.add_(y)                      # x + y
    axy = torch.empty_like(x)
    g.residual(L, x, axy, with_source=False)
    axy.sub_(ax).sub_(ay)
    _ok(float(torch.linalg.vector_norm(axy)) / float(torch.linalg.vector_norm(ax)), 1e-12,
        "A(x + y) - A x - A y, relative")
    g.close()


def test_full_A_rows_closed_form(dev):
    from oracle.aavv_closed import aavv_rows
    from oracle.cavv_closed import cavv_rows
    from oracle.ccav_closed import ccav_rows
    from oracle.ccvv_closed import ccvv_pair_index, ccvv_rows
    from paper_1606_01273_amd import Caspt2
    p = make_problem(30, 8, 400, 1500, 4, seed=8, reading="A", shift=0.2)
    g = Caspt2.from_problem(p)
    g.autotune()
    nc, na, nv, nst = p.nc, p.na, p.nv, p.nst
    npc_p, npv_p = nc * (nc + 1) // 2, nv * (nv + 1) // 2
    npc_m, npv_m = nc * (nc - 1) // 2, nv * (nv - 1) // 2
    lay = {name: (off, rows, n) for name, off, rows, n in g.layout()}
    assert lay["ccvv+"] == (0, npc_p * npv_p, nst)
    assert lay["ccvv-"] == (npc_p * npv_p * nst, npc_m * npv_m, nst)
    off_cp = (npc_p * npv_p + npc_m * npv_m) * nst
    assert lay["cavv+"] == (off_cp, nc * npv_p, nst * na)
    off_cm = off_cp + nc * npv_p * nst * na
    assert lay["cavv-"] == (off_cm, nc * npv_m, nst * na)
    off_ap = off_cm + nc * npv_m * nst * na
    assert lay["aavv+"] == (off_ap, npv_p, nst * na * na)
    off_am = off_ap + npv_p * nst * na * na
    assert lay["aavv-"] == (off_am, npv_m, nst * na * na)
    off_vp = off_am + npv_m * nst * na * na
    assert lay["ccav+"] == (off_vp, npc_p * nv, nst * na)
    off_vm = off_vp + npc_p * nv * nst * na
    assert lay["ccav-"] == (off_vm, npc_m * nv, nst * na)
    rng = np.random.default_rng(42)
    reps = [(0, 0, 0, 0), (nc - 1, nc - 1, nv - 1, nv - 1), (nc - 1, 0, nv - 1, 0), (5, 5, 300, 17),
            (17, 3, 250, 250)]
    while len(reps) < 256:
        i, j = sorted(int(v) for v in rng.integers(0, nc, 2))[::-1]
        a, b = sorted(int(v) for v in rng.integers(0, nv, 2))[::-1]
        reps.append((i, j, a, b))
    creps = [(0, 0, 0), (nc - 1, nv - 1, nv - 1), (nc - 1, nv - 1, 0), (7, 123, 123)]
    while len(creps) < 256:
        a, b = sorted(int(v) for v in rng.integers(0, nv, 2))[::-1]
        creps.append((int(rng.integers(0, nc)), a, b))
    areps = [(0, 0), (nv - 1, nv - 1), (nv - 1, 0), (211, 211)]
    while len(areps) < 128:
        areps.append(tuple(sorted(int(v) for v in rng.integers(0, nv, 2))[::-1]))
    vreps = [(0, 0, 0), (nc - 1, nc - 1, nv - 1), (nc - 1, 0, nv - 1), (9, 9, 77)]
    while len(vreps) < 128:
        i, j = sorted(int(v) for v in rng.integers(0, nc, 2))[::-1]
        vreps.append((i, j, int(rng.integers(0, nv))))
    xh = random_vector(g.length, 41)

    def gather(rows_p, rows_m, width, off_p, off_m):
        """positions and packed rows of the sampled representatives"""
        pos, tp, tm, sel = [], [], [], []
        for k, (rp, rm) in enumerate(zip(rows_p, rows_m)):
            tp.append(xh[off_p + rp * width: off_p + (rp + 1) * width])
            pos.append(off_p + rp * width)
            if rm is None:
                tm.append(None)
            else:
                tm.append(xh[off_m + rm * width: off_m + (rm + 1) * width])
                sel.append(k)
        pos += [off_m + rm * width for rm in rows_m if rm is not None]
        cols = np.arange(width)
        return (np.asarray(pos)[:, None] + cols).ravel(), tp, tm, sel

    ccvv_p = [ccvv_pair_index(i, j, False) * npv_p + ccvv_pair_index(a, b, False) for i, j, a, b in reps]
    ccvv_m = [ccvv_pair_index(i, j, True) * npv_m + ccvv_pair_index(a, b, True) if i > j and a > b else None
              for i, j, a, b in reps]
    cavv_p = [i * npv_p + ccvv_pair_index(a, b, False) for i, a, b in creps]
    cavv_m = [i * npv_m + ccvv_pair_index(a, b, True) if a > b else None for i, a, b in creps]
    pos1, t1p, t1m, sel1 = gather(ccvv_p, ccvv_m, nst, 0, lay["ccvv-"][0])
    pos2, t2p, t2m, sel2 = gather(cavv_p, cavv_m, nst * na, off_cp, off_cm)
    aavv_p = [ccvv_pair_index(a, b, False) for a, b in areps]
    aavv_m = [ccvv_pair_index(a, b, True) if a > b else None for a, b in areps]
    pos3, t3p, t3m, sel3 = gather(aavv_p, aavv_m, nst * na * na, off_ap, off_am)
    ccav_p = [ccvv_pair_index(i, j, False) * nv + a for i, j, a in vreps]
    ccav_m = [ccvv_pair_index(i, j, True) * nv + a if i > j else None for i, j, a in vreps]
    pos4, t4p, t4m, sel4 = gather(ccav_p, ccav_m, nst * na, off_vp, off_vm)
    idx4 = torch.tensor(pos4, device=dev)
    idx1 = torch.tensor(pos1, device=dev)
    idx2 = torch.tensor(pos2, device=dev)
    idx3 = torch.tensor(pos3, device=dev)
    x = torch.from_numpy(xh).to(dev).unsqueeze(0).expand(nst, -1).contiguous()
    sig = torch.empty_like(x)
    dens = prods = None
    for streams, src in ((1, True), (2, False)):
        print(f"full A ccvv, cavv, aavv and ccav rows: {streams} stream(s), source {src}", flush=True)
        g.set_streams(streams)
        sig.fill_(float("nan"))
        g.residual_all(x, sig, with_source=src)
        torch.cuda.synchronize()
        for L in range(nst):
            got = sig[L].index_select(0, idx1).cpu().numpy()
            rp, rm = ccvv_rows(p, L, reps, t1p, t1m, with_source=src)
            ref = np.concatenate([rp.ravel(), rm[sel1].ravel()])
            _ok(np.abs(got - ref).max() / np.abs(ref).max(), 1e-12,
                f"ccvv rows, state {L} ({len(reps)} '+', {len(sel1)} '-' rows)")
            got = sig[L].index_select(0, idx2).cpu().numpy()
            rp, rm, dens = cavv_rows(p, L, creps, t2p, t2m, with_source=src, dens=dens)
            ref = np.concatenate([rp.ravel(), rm[sel2].ravel()])
            _ok(np.abs(got - ref).max() / np.abs(ref).max(), 1e-12,
                f"cavv rows, state {L} ({len(creps)} '+', {len(sel2)} '-' rows)")
            got = sig[L].index_select(0, idx3).cpu().numpy()
            rp, rm, prods = aavv_rows(p, L, areps, t3p, t3m, with_source=src, prods=prods)
            ref = np.concatenate([rp.ravel(), rm[sel3].ravel()])
            _ok(np.abs(got - ref).max() / np.abs(ref).max(), 1e-12,
                f"aavv rows, state {L} ({len(areps)} '+', {len(sel3)} '-' rows)")
            got = sig[L].index_select(0, idx4).cpu().numpy()
            rp, rm, dens = ccav_rows(p, L, vreps, t4p, t4m, with_source=src, dens=dens)
            ref = np.concatenate([rp.ravel(), rm[sel4].ravel()])
            _ok(np.abs(got - ref).max() / np.abs(ref).max(), 1e-12,
                f"ccav rows, state {L} ({len(vreps)} '+', {len(sel4)} '-' rows)")
    # the FP32 operator of the mixed mode (Eq. 10 without the source) on the
    # FP32-rounded x, same rows: 1e-5 of the largest sampled value
    from paper_1606_01273_amd import MIXED, lib
    g.set_precision(MIXED)
    x32 = x[0].float()
    del x, sig
    s32 = torch.empty_like(x32)

    def r32(rows):
        return [None if t is None else np.asarray(t, dtype=np.float32).astype(np.float64) for t in rows]

    checks = [("ccvv", idx1, lambda L: ccvv_rows(p, L, reps, r32(t1p), r32(t1m), with_source=False), sel1),
              ("cavv", idx2, lambda L: cavv_rows(p, L, creps, r32(t2p), r32(t2m), with_source=False,
                                                 dens=dens)[:2], sel2),
              ("aavv", idx3, lambda L: aavv_rows(p, L, areps, r32(t3p), r32(t3m), with_source=False,
                                                 prods=prods)[:2], sel3),
              ("ccav", idx4, lambda L: ccav_rows(p, L, vreps, r32(t4p), r32(t4m), with_source=False,
                                                 dens=dens)[:2], sel4)]
    for L in range(nst):
        print(f"full A, FP32 operator, state {L}", flush=True)
        s32.fill_(float("nan"))
        assert lib().caspt2_debug_residual_f32(g._h, L, x32.data_ptr(), s32.data_ptr()) == 0
        torch.cuda.synchronize()
        for name, idx, fn, sel in checks:
            got = s32.index_select(0, idx).double().cpu().numpy()
            rp, rm = fn(L)
            ref = np.concatenate([rp.ravel(), rm[sel].ravel()])
            _ok(np.abs(got - ref).max() / np.abs(ref).max(), 1e-5, f"FP32 {name} rows, state {L}")
    g.close()
