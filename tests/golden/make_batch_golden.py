"""Writes the stored oracle results of the 64-problem batch workload by
running the CPU oracle (oracle/ic.py) only.

  python tests/golden/make_batch_golden.py [--jobs J] [--first K]

Problems: sizes and seeds from synth.gen.batch_sizes(64, seed=4) (closed
4-16, active 4-6, virtual 20-150, 1-4 states, naux = 3 nmo), Fock couplings
between orbital classes, shift 0.2, MS-MR XMS.  Per problem: E^MS (Eqs.
15-17) when the amplitude equation is positive definite, else the reason it
is not (a non-positive preconditioner denominator, or p.Ap <= 0 in the
conjugate gradients: an intruder state at this shift).  One JSON object per
line in tests/golden/batch_B.jsonl, in problem order.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def one(args):
    k, (nc, na, nv, naux, nst, child) = args
    import numpy as np
    from synth.gen import make_problem
    from oracle.ic import Caspt2Oracle
    t0 = time.time()
    p = make_problem(nc, na, nv, naux, nst, child, reading="B", shift=0.2)
    rec = {"index": k, "dims": [nc, na, nv, naux, nst], "seed": int(child)}
    o = Caspt2Oracle(p, "MSMR")
    try:
        o.run(P=0, tol=1e-12)
        rec["e_ms"] = [float(v) for v in o.e_ms]
        rec["indefinite"] = False
    except ArithmeticError as ex:
        dmin = min(float(d.min()) for L in range(p.nst) for d in o.denominators(L) if d.size)
        rec["indefinite"] = True
        rec["reason"] = str(ex)
        rec["min_denominator"] = dmin
    rec["seconds"] = round(time.time() - t0, 1)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=3)
    ap.add_argument("--first", type=int, default=64)
    a = ap.parse_args()
    from synth.gen import batch_sizes
    sizes = batch_sizes(64, seed=4)[:a.first]
    out = os.path.join(HERE, "batch_B.jsonl")
    os.environ.setdefault("OMP_NUM_THREADS", "2")
    with mp.get_context("spawn").Pool(a.jobs) as pool:
        recs = []
        for rec in pool.imap(one, list(enumerate(sizes))):
            recs.append(rec)
            print(json.dumps(rec), flush=True)
    with open(out, "w") as fh:
        for rec in recs:
            fh.write(json.dumps(rec) + "\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
