"""Write tests/golden/cfg2_oracle.npz from the FP64 oracle (no GPU code).

Workload: 2x2x2 diamond supercell (64 atoms, N = 832), grids 32^3 / 64^3 /
128^3, 8 points per owned function (N_mu = 6656), 128 occupied orbitals.
Stored: E_x, per-domain pivot lists and counts, the whole K (and 64 seeded
rows of it under the older key), a seeded 96 x 96 sample of W, the whole
diagonal block of W of every window domain, and the diagonal and 32 seeded
rows of the universal domain's block.  Runs for about 12 minutes on 8 cores.

usage: python tests/golden/make_cfg2_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pipeline  # noqa: E402
from workloads import config  # noqa: E402


def main():
    t0 = time.time()
    s = config(2)
    r = pipeline.run(s)
    rng = np.random.default_rng(2024)
    rows = np.sort(rng.choice(s.n_basis, 64, replace=False))
    wr = np.sort(rng.choice(r.W.shape[0], 96, replace=False))
    wc = np.sort(rng.choice(r.W.shape[0], 96, replace=False))
    counts = np.array([len(p) for p in r.pivots], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    # whole diagonal blocks of the window domains (domain 0 is the universal grid)
    wblk = np.concatenate([r.W[offs[d]:offs[d + 1], offs[d]:offs[d + 1]].ravel() for d in range(1, len(counts))])
    urows = np.sort(rng.choice(int(counts[0]), 32, replace=False))
    np.savez_compressed(
        os.path.join(HERE, "cfg2_oracle.npz"),
        E_x=np.array(r.E_x),
        counts=counts,
        pivots=np.concatenate(r.pivots).astype(np.int64),
        K_rows=rows,
        K=r.K[rows],
        W_rows=wr,
        W_cols=wc,
        W=r.W[np.ix_(wr, wc)],
        K_full=r.K,
        W_offsets=offs,
        W_window_blocks=wblk,
        W_univ_diag=np.diag(r.W)[: counts[0]].copy(),
        W_univ_rows=urows,
        W_univ=r.W[urows, : counts[0]],
        times=np.array([r.times[k] for k in ("plan", "basis", "diag", "select", "fit", "coulomb", "exchange")]),
    )
    print("E_x", r.E_x, "per atom", r.E_x / s.n_atoms, "wall", time.time() - t0, r.times)


if __name__ == "__main__":
    main()
