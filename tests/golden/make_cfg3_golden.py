"""Write tests/golden/cfg3_cell3_oracle.npz from the FP64 oracle (no GPU code).

Workload: cell 3 of the uneven batch (a 2x2x2 diamond supercell, 64 atoms,
N = 832, with a random symmetric strain of up to 3 % and +-0.05 Angstrom
displacements; grids 48^3 / 96^3; its ratio drawn from U[5, 8]).
Stored: E_x, per-domain pivot lists and counts, the whole K, and the whole
diagonal block of W of every window domain.  Runs for several minutes on
8 cores.

usage: python tests/golden/make_cfg3_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pipeline  # noqa: E402
from workloads import batched_cells  # noqa: E402


def main():
    t0 = time.time()
    (s,) = batched_cells(32, cells=[3])
    r = pipeline.run(s)
    counts = np.array([len(p) for p in r.pivots], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    wblk = np.concatenate([r.W[offs[d]:offs[d + 1], offs[d]:offs[d + 1]].ravel() for d in range(1, len(counts))])
    np.savez_compressed(
        os.path.join(HERE, "cfg3_cell3_oracle.npz"),
        E_x=np.array(r.E_x),
        counts=counts,
        pivots=np.concatenate(r.pivots).astype(np.int64),
        K_full=r.K,
        W_offsets=offs,
        W_window_blocks=wblk,
        times=np.array([r.times[k] for k in ("plan", "basis", "diag", "select", "fit", "coulomb", "exchange")]),
    )
    print("E_x", r.E_x, "per atom", r.E_x / s.n_atoms, "wall", time.time() - t0, r.times)


if __name__ == "__main__":
    main()
