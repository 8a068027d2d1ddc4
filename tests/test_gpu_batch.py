"""Batched fits of independent cells (isdf_fit_batch) on the GPU.

Cells come from the uneven batch workload (strained, displaced 1x1x1, 2x1x1
and 2x2x1 diamond cells, ratio U[5, 8]).  The batch must give exactly the
fits of the plans run one by one (same kernels, each plan on its own
stream), and the smallest cell is checked against the oracle.
"""
import time

import numpy as np
import pytest

from paper_2404_09373_amd import binding
from workloads import batched_cells

pytestmark = pytest.mark.gpu

CELLS = [0, 1, 2, 4, 5, 6]  # two of each of the three smaller shapes


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def cells():
    return batched_cells(32, cells=CELLS)


def _exchange(torch, fit, s):
    D = torch.tensor(s.D, dtype=torch.float64, device="cuda")
    K, e = fit.exchange(D)
    return K.cpu().numpy(), e


def test_batch_equals_sequential(torch, cells):
    plans = [binding.Plan(s) for s in cells]
    for p in plans:  # warm: tables uploaded, device blocks cached
        p.fit().close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [p.fit() for p in plans]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    t0 = time.perf_counter()
    fits = binding.fit_batch(plans, max_concurrent=4)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    print(f"[batch] {len(cells)} cells: batch {t_batch:.3f} s, one by one {t_seq:.3f} s")
    for i, (s, fb, fs) in enumerate(zip(cells, fits, seq)):
        assert fb is not None
        for d in range(plans[i].n_domains):
            assert np.array_equal(fb.get("points", d), fs.get("points", d))
        assert np.array_equal(fb.get("W"), fs.get("W"))
        Kb, eb = _exchange(torch, fb, s)
        Ks, es = _exchange(torch, fs, s)
        assert np.array_equal(Kb, Ks) and eb == es
        print(f"[batch] cell {CELLS[i]} ({s.n_atoms} atoms, N_mu {fb.n_mu}): E_x {eb:.10f}")
    for f in fits + seq:
        f.close()
    for p in plans:
        p.close()


def test_batch_smallest_cell_matches_oracle(torch, cells):
    from oracle import pipeline

    s = cells[0]
    ref = pipeline.run(s)
    plans = [binding.Plan(c) for c in cells[:3]]
    fits = binding.fit_batch(plans, max_concurrent=3)
    f = fits[0]
    for d in range(plans[0].n_domains):
        assert np.array_equal(f.get("points", d), ref.pivots[d])
    K, e = _exchange(torch, f, s)
    dK = float(np.max(np.abs(K - ref.K)))
    dE = abs(e - ref.E_x) / s.n_atoms
    print(f"[batch vs oracle] cell {CELLS[0]}: max|dK| {dK:.2e} |dE|/atom {dE:.2e}")
    assert dK <= 1e-7 and dE <= 1e-6
    for x in fits:
        x.close()
    for p in plans:
        p.close()


def test_batch_strained_64_atom_cell_matches_oracle(torch):
    """Cell 3 of the batch (2x2x2, strained and displaced, grids 48^3 / 96^3)
    fitted in a batch beside two smaller cells, against the stored oracle
    values of tests/golden/make_cfg3_golden.py: pivots identical, the whole
    diagonal W block of every window within 1e-9 relative, the whole K within
    1e-7 Ha, |dE_x| <= 1e-6 Ha/atom."""
    import os

    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg3_cell3_oracle.npz"))
    three, small0, small1 = batched_cells(32, cells=[3, 0, 1])
    plans = [binding.Plan(c) for c in (three, small0, small1)]
    fits = binding.fit_batch(plans, max_concurrent=3)
    f = fits[0]
    assert np.array_equal(f.counts(), g["counts"])
    piv = np.concatenate([f.get("points", d) for d in range(plans[0].n_domains)])
    assert np.array_equal(piv, g["pivots"])
    W = f.get("W")
    offs = g["W_offsets"]
    blocks = np.concatenate([W[offs[d]:offs[d + 1], offs[d]:offs[d + 1]].ravel() for d in range(1, len(offs) - 1)])
    dW = float(np.max(np.abs(blocks - g["W_window_blocks"])) / np.max(np.abs(g["W_window_blocks"])))
    K, e = _exchange(torch, f, three)
    dK = float(np.max(np.abs(K - g["K_full"])))
    dE = abs(e - float(g["E_x"])) / three.n_atoms
    print(f"[batch vs oracle] cell 3 (64 atoms, strained): W blocks rel {dW:.2e} max|dK| {dK:.2e} |dE|/atom {dE:.2e}")
    assert dW <= 1e-9 and dK <= 1e-7 and dE <= 1e-6
    for x in fits:
        x.close()
    for p in plans:
        p.close()


def test_batch_rejects_repeated_plan(cells):
    p = binding.Plan(cells[0])
    with pytest.raises(binding.IsdfError):
        binding.fit_batch([p, p])
    p.close()
