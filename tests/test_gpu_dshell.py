"""d shells and the full-cell domain mode on the GPU against the FP64
oracle, stage by stage (same tolerances as test_gpu_parity: basis values and
X rows 1e-12 relative, pivots identical, Theta 1e-11, F 1e-7, W 1e-9,
max|dK| <= 1e-7 Ha and |dE_x| <= 1e-6 Ha/atom)."""
import numpy as np
import pytest

from oracle import pipeline
from paper_2404_09373_amd import binding
from test_gpu_parity import _check_all
from workloads import tiny_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.mark.parametrize("kind", ["d_atom", "d_two"])
def test_d_shell_cells_stage_parity(torch, kind):
    """Cells whose shells include d functions on the universal grid (d 0.5)
    and on the atom windows (d 2.5)."""
    s = tiny_system(kind, n_occ=3)
    ref = pipeline.run(s)
    plan = binding.Plan(s)
    print(f"[{kind}] N {plan.n_basis} N_mu {plan.n_mu} domains {plan.n_domains}", flush=True)
    fit = plan.fit()
    K, ex = _check_all(s, ref, plan, fit, torch, kind)
    assert np.max(np.abs(K - K.T)) <= 1e-12 * np.max(np.abs(K)) and ex < 0


def test_d_shell_strained_cell_stage_parity(torch):
    s = tiny_system("d_two", n_occ=3)
    s.lattice = s.lattice @ (np.eye(3) + np.array([[0.03, -0.01, 0.0], [-0.01, 0.0, 0.02],
                                                   [0.0, 0.02, -0.02]]))
    from workloads import periodic_overlap, random_density
    S = periodic_overlap(s.lattice, s.xyz, s.shell_atom, s.shell_l, s.shell_alpha)
    s.C_occ, s.D = random_density(S, 3, 11)
    ref = pipeline.run(s)
    plan = binding.Plan(s)
    fit = plan.fit()
    _check_all(s, ref, plan, fit, torch, "d_two_strained")


def test_full_cell_domain_mode_stage_parity(torch):
    """domain_mode = 1: one full-grid domain per level (the finer level's
    domain carries every coarser function as N)."""
    s = tiny_system("d_two", grids=((10, 10, 10), (20, 20, 20)), n_occ=3)
    s.domain_mode = 1
    ref = pipeline.run(s)
    plan = binding.Plan(s)
    assert plan.n_domains == 2
    fit = plan.fit()
    _check_all(s, ref, plan, fit, torch, "full_cell")


def test_d_shell_mixed_precision_within_gate(torch):
    """BF16 x6 exchange and W rows on a d-shell cell against the oracle:
    |dE_x| <= 1e-6 Ha/atom (the accuracy gate of the mixed path)."""
    s = tiny_system("d_two", n_occ=3)
    ref = pipeline.run(s)
    plan = binding.Plan(s, precision=binding.MIXED_X6)
    fit = plan.fit()
    D = torch.tensor(s.D, dtype=torch.float64, device="cuda")
    K, ex = fit.exchange(D)
    dK = float(np.max(np.abs(K.cpu().numpy() - ref.K)))
    dE = abs(ex - ref.E_x) / s.n_atoms
    print(f"[d_two x6] max|dK| {dK:.2e} |dE|/atom {dE:.2e}")
    assert dE <= 1e-6 and dK <= 1e-6


@pytest.mark.parametrize("ratio", [9.0, 13.0, 16.0])
def test_window_rows_45_to_80_against_oracle(torch, ratio):
    """Windows of 45, 65 and 80 fitting functions: their rows of W run on the
    48- and 80-row tiles of the grouped metric products, and their Theta on
    the 48- and 80-column tiles (the 384-atom
    workload's windows have 45 and 65).  Pivots identical, the windows'
    Theta to 1e-11 and F to 1e-7 against the oracle; W to 1e-9 relative
    against the oracle's metric of the same fitting functions.  (At these ratios the universal domain takes
    more points than its pair products have rank, so its F, and the oracle's
    W built on the oracle's F, carry that conditioning.)"""
    s = tiny_system("d_two", n_occ=3, n_mu_ratio=ratio)
    ref = pipeline.run(s)
    plan = binding.Plan(s)
    fit = plan.fit()
    counts = fit.counts()
    assert list(counts[1:]) == [int(round(5 * ratio))] * 2
    for d in range(plan.n_domains):
        assert np.array_equal(fit.get("points", d), ref.pivots[d])
    from oracle import basis, isdf

    for d in range(1, plan.n_domains):
        dom = ref.plan.domains[d]
        F_ref, Theta_ref, _ = isdf.fit_functions(basis.domain_values(ref.plan, dom), dom.L.size, ref.pivots[d])
        th = fit.get("theta", d)  # 45 / 65-80 columns: the 48- / 80-column Theta tiles
        e_th = float(np.max(np.abs(th - Theta_ref)) / np.max(np.abs(Theta_ref)))
        assert e_th <= 1e-11, f"Theta d={d} {e_th:.2e}"
        F = fit.get("F", d)
        e = float(np.max(np.abs(F - F_ref)) / np.max(np.abs(F_ref)))
        assert e <= 1e-7, f"F d={d} {e:.2e}"
    # the metric stage alone: the oracle's W from the fitting functions the
    # GPU formed (the same input on both sides), whole and window block
    from oracle import coulomb

    Wr = coulomb.coulomb_metric(ref.plan, [fit.get("F", d) for d in range(plan.n_domains)])
    W = fit.get("W")
    n0 = int(counts[0])
    e_w = float(np.max(np.abs(W - Wr)) / np.max(np.abs(Wr)))
    e_b = float(np.max(np.abs(W[n0:, n0:] - Wr[n0:, n0:])) / np.max(np.abs(Wr[n0:, n0:])))
    print(f"[rows {int(5 * ratio)}] W from the GPU's F rel {e_w:.2e}, window block {e_b:.2e}")
    assert e_w <= 1e-9 and e_b <= 1e-9
