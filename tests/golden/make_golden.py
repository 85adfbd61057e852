"""Writes the stored expected values of the golden GPU tests by running the
CPU oracle (oracle/ic.py) only.

  python tests/golden/make_golden.py            # writes tests/golden/mid_B.json

Problem: the three-state XMS workload with 10 closed, 6 active (6e), 120
virtual orbitals and 400 auxiliary functions (seed 1, Fock couplings between
orbital classes, shift 0.2).  Stored: E^MS (Eqs. 15-17), the norms of T_L and
of lambda_L for target state 0 (Eq. 20), their values at 256 sampled
positions of every state (with the largest magnitude of each vector, the
scale of the element-wise bar), and the residual (Eq. 10, with the source)
at 64 sampled positions of state 0 and 256 of every state for a seeded
random x.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from synth.gen import make_problem, random_vector, sample_positions  # noqa: E402
from oracle.ic import Caspt2Oracle  # noqa: E402

DIMS = (10, 6, 120, 400, 3)
SEED, READING, SHIFT = 1, "B", 0.2


def main():
    p = make_problem(*DIMS, seed=SEED, reading=READING, shift=SHIFT)
    o = Caspt2Oracle(p, "MSMR")
    x = random_vector(o.length, 11)
    sigma = o.residual(0, x, with_source=True)
    idx = sample_positions(o.length, 64, 12)
    o.run(P=0, tol=1e-12)
    sidx = sample_positions(o.length, 256, 13)
    sig_all = [o.residual(L, x, with_source=True) for L in range(p.nst)]
    rec = {"dims": DIMS, "seed": SEED, "reading": READING, "shift": SHIFT, "target": 0,
           "length": int(o.length), "e_ms": [float(v) for v in o.e_ms],
           "t_norm": [float(np.linalg.norm(v)) for v in o.T],
           "lambda_norm": [float(np.linalg.norm(v)) for v in o.lam],
           "residual_x_seed": 11, "residual_index_seed": 12, "residual_index": [int(i) for i in idx],
           "residual_value": [float(sigma[i]) for i in idx],
           "sample_index_seed": 13, "sample_index": [int(i) for i in sidx],
           "t_absmax": [float(np.abs(v).max()) for v in o.T],
           "t_sample": [[float(v[i]) for i in sidx] for v in o.T],
           "lambda_absmax": [float(np.abs(v).max()) for v in o.lam],
           "lambda_sample": [[float(v[i]) for i in sidx] for v in o.lam],
           "residual_sample": [[float(v[i]) for i in sidx] for v in sig_all]}
    with open(os.path.join(HERE, "mid_B.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print("wrote mid_B.json")


if __name__ == "__main__":
    main()
