"""Poisson solves on the line lengths of the 384-atom cell's grids
(18, 36, 72, 144 along z; 24, 48, 96, 192 along x and y) and on odd-eighth
x lengths (36, 72, generic passes), against the oracle's numpy FFTs: the
whole fit and exchange of a one-atom cell on each ladder, pivots identical,
W within 1e-9 relative, max|dK| <= 1e-7 Ha, |dE_x| <= 1e-6 Ha/atom."""
import numpy as np
import pytest

from oracle import pipeline
from paper_2404_09373_amd import binding
from workloads import tiny_system

pytestmark = pytest.mark.gpu

LADDERS = [
    ((24, 24, 18), (48, 48, 36)),
    ((48, 48, 36), (96, 96, 72)),
    ((96, 96, 72), (192, 192, 144)),
    ((36, 36, 36), (72, 72, 72)),
]


@pytest.mark.parametrize("grids", LADDERS, ids=lambda g: "x".join(map(str, g[1])))
def test_fit_and_exchange_on_grid_ladder(grids):
    import torch

    assert torch.cuda.is_available()
    s = tiny_system("one_atom", grids=grids, n_occ=2)
    ref = pipeline.run(s)
    plan = binding.Plan(s)
    fit = plan.fit()
    for d in range(plan.n_domains):
        assert np.array_equal(fit.get("points", d), np.asarray(ref.pivots[d])), d
    W = fit.get("W")
    dW = float(np.max(np.abs(W - ref.W)) / np.max(np.abs(ref.W)))
    D = torch.tensor(s.D, dtype=torch.float64, device="cuda")
    K, e = fit.exchange(D)
    dK = float(np.max(np.abs(K.cpu().numpy() - ref.K)))
    dE = abs(e - ref.E_x) / s.n_atoms
    print(f"[grids {grids}] W rel {dW:.2e} max|dK| {dK:.2e} |dE|/atom {dE:.2e}")
    assert dW <= 1e-9 and dK <= 1e-7 and dE <= 1e-6
    fit.close()
    plan.close()
