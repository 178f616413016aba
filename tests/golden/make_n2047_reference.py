"""Write n2047_oracle_rows.npz: the oracle's direct solve u = H^{-1} f of the
n = 2047 layered workload (32 x 8 decomposition, 48-node PML, 64 sources on
depth row 164) for two of its sources, stored on selected depth rows.

The values come from the oracle only (oracle.direct.DirectSolver: sparse LU
of the nested-dissection-ordered operator of App. A, refined with the
assembled operator's residual); the inputs from the seeded generators of
paper_1510_01831_amd.media.  The whole field of one source is 67 MB, so the
file keeps the rows on which the method's errors show: the source row, the
first physical row of every layer (a trace row of each interface) and the
middle row of every layer (a reconstructed row), across all 2047 columns.

Run:  python tests/golden/make_n2047_reference.py   (about 60 GB of host
memory at peak and tens of minutes on 8 cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.direct import DirectSolver  # noqa: E402
from oracle.discretization import Problem, partition  # noqa: E402
from paper_1510_01831_amd import media  # noqa: E402

SOURCES = (0, 40)


def stored_rows(w):
    parts = partition(w.n, w.layers)
    rows = {w.src_z}
    for a, b in parts:
        rows.add(a)
        rows.add((a + b) // 2)
    return np.array(sorted(rows), dtype=np.int64)


def main():
    w = media.workload("C4")
    c = media.velocity("C4")
    t0 = time.time()
    prob = Problem(c, w.omega, w.n_pml)
    solver = DirectSolver(prob)
    print(f"factor {time.time() - t0:.0f} s", flush=True)
    f = media.point_sources(w.n, tuple(w.src_x[k] for k in SOURCES), w.src_z)
    F = np.stack([prob.extend(x).ravel() for x in f], axis=1)
    t0 = time.time()
    U, res = solver.solve(F)
    print(f"solve {time.time() - t0:.0f} s, relative residuals {res}", flush=True)
    rows = stored_rows(w)
    u = prob.restrict(U.T.reshape(len(SOURCES), prob.W, prob.W))[:, rows - 1, :]
    np.savez_compressed(os.path.join(HERE, "n2047_oracle_rows.npz"),
                        sources=np.array(SOURCES, dtype=np.int64), rows=rows,
                        u=np.ascontiguousarray(u), rel_residual=res,
                        u_norm=np.linalg.norm(prob.restrict(U.T.reshape(len(SOURCES), prob.W,
                                                                        prob.W)), axis=(1, 2)))
    print(f"wrote {len(rows)} rows x {w.n} columns for sources {SOURCES}", flush=True)


if __name__ == "__main__":
    main()
