"""The benchmark's headline configuration at full size (2x2x2 diamond,
N = 832, grids 32^3 / 64^3 / 128^3, N_mu = 6656) against the stored
FP64-oracle values (tests/golden/make_cfg2_golden.py): BF16-split x6
contractions, the learned candidate selector trained as the benchmark trains
it, the tuned tile table, and the factored-density exchange replayed from its
captured graph.

The selector is exact, so the pivots equal the oracle's; the energy must agree
to 1e-6 Ha/atom (the mixed-precision bar of the benchmark; measured ~1e-10),
max|dK| stays within 2e-6 Ha (measured 8.1e-7), and every replay gives the
same K."""
import os

import numpy as np
import pytest

from paper_2404_09373_amd import binding
from workloads import config

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden", "cfg2_oracle.npz")
TUNE = os.path.join(ROOT, "paper_2404_09373_amd", "tune", "gfx950.json")


def test_headline_configuration_matches_oracle():
    import torch

    import bench

    assert torch.cuda.is_available()
    g = np.load(GOLD)
    weights, _ = bench.train_selector(torch, lambda msg: None)
    s = config(2)
    plan = binding.Plan(s, precision=binding.MIXED_X6, selector=binding.SEL_MLP, mlp_weights=weights,
                        mlp_keep=2.0, mlp_cutoff=0.05, tune_file=TUNE)
    fit = plan.fit()
    piv = np.concatenate([fit.get("points", d) for d in range(plan.n_domains)])
    assert np.array_equal(piv, g["pivots"])
    C = torch.tensor(s.C_occ, dtype=torch.float64, device="cuda")
    K = torch.empty((plan.n_basis, plan.n_basis), dtype=torch.float64, device="cuda")
    energies, first = [], None
    for r in range(3):  # the first call captures the graph, the others replay it
        _, e = fit.exchange_occ(C, K)
        torch.cuda.synchronize()
        energies.append(e)
        if first is None:
            first = K.clone()
        else:
            assert torch.equal(K, first)
    Kh = K.cpu().numpy()
    dE = abs(energies[-1] - float(g["E_x"])) / s.n_atoms
    dK = float(np.max(np.abs(Kh[g["K_rows"]] - g["K"])))
    info = fit.selection()
    print(f"[headline] candidates {int(np.sum(info['n_candidates']))}, fallbacks {int(np.sum(info['fallback']))}; "
          f"E_x {energies[-1]:.12f} oracle {float(g['E_x']):.12f} |dE|/atom {dE:.2e} max|dK| {dK:.2e}")
    assert len(set(energies)) == 1
    # the gate is |dE| <= 1e-6 Ha/atom; max|dK| is held at about twice its
    # measured value (8.1e-7: x6 operands carry 24 bits, an FP32-class
    # relative error per split product on K entries of order 1 Ha)
    assert dE <= 1e-6 and dK <= 2e-6
    fit.close()
    plan.close()
