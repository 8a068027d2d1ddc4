"""Full-size parity on the 64-atom benchmark workload (2x2x2 diamond,
N = 832, grids 32^3 / 64^3 / 128^3, N_mu = 6656) in the launch configuration
bench.py times, against values stored by tests/golden/make_cfg2_golden.py
(FP64 oracle only), plus properties that hold at any size.

Tolerances as in test_gpu_parity.py: pivots identical, W samples 1e-9
relative, max |dK| <= 1e-7 Ha on the stored rows, |dE_x| <= 1e-6 Ha/atom.
"""
import os

import numpy as np
import pytest

from oracle import basis, isdf
from oracle import plan as oplan
from paper_2404_09373_amd import binding
from workloads import config

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg2_oracle.npz")


@pytest.fixture(scope="module")
def run():
    import torch

    assert torch.cuda.is_available()
    g = np.load(GOLD)
    s = config(2)
    plan = binding.Plan(s, stream=torch.cuda.current_stream().cuda_stream)
    fit = plan.fit()
    D = torch.tensor(s.D, dtype=torch.float64, device="cuda")
    K, ex = fit.exchange(D)
    yield s, g, plan, fit, K.cpu().numpy(), ex
    fit.close()
    plan.close()


def test_cfg2_pivots_identical(run):
    s, g, plan, fit, K, ex = run
    counts = fit.counts()
    assert np.array_equal(counts, g["counts"])
    piv = np.concatenate([fit.get("points", d) for d in range(plan.n_domains)])
    assert np.array_equal(piv, g["pivots"])


def test_cfg2_exchange_matches_oracle(run):
    s, g, plan, fit, K, ex = run
    dE = abs(ex - float(g["E_x"])) / s.n_atoms
    dK = float(np.max(np.abs(K[g["K_rows"]] - g["K"])))
    print(f"[cfg2] E_x gpu {ex:.12f} oracle {float(g['E_x']):.12f} |dE|/atom {dE:.2e} max|dK| {dK:.2e}")
    assert dE <= 1e-6 and dK <= 1e-7


def test_cfg2_metric_samples(run):
    s, g, plan, fit, K, ex = run
    W = fit.get("W")
    sub = W[np.ix_(g["W_rows"], g["W_cols"])]
    e = float(np.max(np.abs(sub - g["W"])) / np.max(np.abs(g["W"])))
    print(f"[cfg2] W sample rel {e:.2e}")
    assert e <= 1e-9
    assert np.array_equal(W, W.T)


def test_cfg2_whole_k_and_diagonal_w_blocks(run):
    """The whole K and the whole diagonal W block of every window against the
    stored oracle values; the universal block on its diagonal and 32 rows."""
    s, g, plan, fit, K, ex = run
    dK = float(np.max(np.abs(K - g["K_full"])))
    W = fit.get("W")
    offs = g["W_offsets"]
    blocks = np.concatenate([W[offs[d]:offs[d + 1], offs[d]:offs[d + 1]].ravel() for d in range(1, len(offs) - 1)])
    dWb = float(np.max(np.abs(blocks - g["W_window_blocks"])) / np.max(np.abs(g["W_window_blocks"])))
    n0 = int(offs[1])
    U = W[:n0, :n0]
    dWu = max(float(np.max(np.abs(np.diag(U) - g["W_univ_diag"]))),
              float(np.max(np.abs(U[g["W_univ_rows"]] - g["W_univ"])))) / float(np.max(np.abs(g["W_univ"])))
    print(f"[cfg2] whole K max|dK| {dK:.2e}; window diagonal W blocks rel {dWb:.2e}; universal block rel {dWu:.2e}")
    assert dK <= 1e-7
    assert dWb <= 1e-9 and dWu <= 1e-9


def test_cfg2_exchange_properties(run):
    s, g, plan, fit, K, ex = run
    assert np.max(np.abs(K - K.T)) <= 1e-12 * np.max(np.abs(K))
    assert ex < 0
    ev = np.linalg.eigvalsh(-0.5 * (K + K.T))
    assert ev[0] >= -1e-10 * ev[-1]


def test_cfg2_sampled_windows_stagewise(run):
    """Basis values, Gram diagonal, pivots and fitting functions of a few
    sampled windows recomputed one by one by the oracle."""
    s, g, plan, fit, K, ex = run
    op = oplan.build_plan(s)
    for d in (1, 40, 64, 65, 100, 128):
        dom = op.domains[d]
        Phi = basis.domain_values(op, dom)
        gp = fit.get("phi", d)
        assert np.max(np.abs(gp - Phi)) <= 1e-12 * np.max(np.abs(Phi))
        piv, _, _, _ = isdf.pivoted_cholesky(Phi, dom.L.size, dom.n_mu, s.eps_isdf, s.tie_tol)
        assert np.array_equal(fit.get("points", d), piv)
        F, _, _ = isdf.fit_functions(Phi, dom.L.size, piv)
        assert np.max(np.abs(fit.get("F", d) - F)) <= 1e-7 * np.max(np.abs(F))


def test_cfg2_mixed_occ_ri_chunked_against_oracle(run):
    """x6 occ-RI K C on the 64-atom workload, Q held in row blocks of 2048
    (the last one ragged) and the Z products' 2 N_mu = 13312 columns in two K
    chunks (8192 and 5120, the second accumulating): against the oracle's
    whole K times C_occ.  Bound as for the smaller cells' x6 occ-RI: the
    split-BF16 products carry about 2^-24 relative error per product."""
    import torch

    s, g, plan, fit, K, ex = run
    xplan = binding.Plan(s, precision=binding.MIXED_X6, ri_rows=2048,
                         stream=torch.cuda.current_stream().cuda_stream)
    xfit = xplan.fit()
    assert np.array_equal(xfit.counts(), g["counts"])
    C = torch.tensor(s.C_occ, dtype=torch.float64, device="cuda")
    KC = torch.empty_like(C)
    _, e = xfit.exchange_occ_ri(C, KC)
    ref = g["K_full"] @ s.C_occ
    dKC = float(np.max(np.abs(KC.cpu().numpy() - ref)))
    dE = abs(e - float(g["E_x"])) / s.n_atoms
    print(f"[cfg2 x6 occ-RI chunked] max|dKC| {dKC:.2e} |dE|/atom {dE:.2e}")
    xfit.close()
    xplan.close()
    assert dKC <= 1e-5 and dE <= 1e-6
