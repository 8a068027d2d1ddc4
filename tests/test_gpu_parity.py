"""GPU path (through the C ABI) against the FP64 oracle, stage by stage.

Tolerances:
  basis values, Gram diagonal, X rows  1e-12 relative to the largest value
      (same closed form; only exp rounding and summation order differ)
  pivots                               identical
  Theta                                1e-11 relative (one more contraction)
  F                                    1e-7 relative: F = Theta M^-1 with
      cond(M) up to ~1e8 (residual diagonals fall to ~1e-5 of the first)
  W                                    1e-9 relative
  K                                    max |dK| <= 1e-7 Ha and |dE_x| <= 1e-6 Ha/atom
"""
import numpy as np
import pytest

from oracle import basis, isdf, pipeline
from paper_2404_09373_amd import binding
from workloads import tiny_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _rel(a, b):
    scale = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / scale) if a.size else 0.0


def _check_all(s, ref, plan, fit, torch, tag, points_pinned=False):
    op = ref.plan
    for d, dom in enumerate(op.domains):
        Phi = basis.domain_values(op, dom)
        g_phi = fit.get("phi", d)
        assert _rel(g_phi, Phi) <= 1e-12, f"{tag} phi d={d} {_rel(g_phi, Phi):.2e}"
        assert _rel(fit.get("diag", d), ref.diag[d]) <= 1e-12, f"{tag} diag d={d}"
        piv = fit.get("points", d)
        assert np.array_equal(piv, ref.pivots[d]), f"{tag} pivots d={d}"
        F_ref, Theta_ref, _ = isdf.fit_functions(Phi, dom.L.size, ref.pivots[d])
        e_th = _rel(fit.get("theta", d), Theta_ref)
        e_f = _rel(fit.get("F", d), F_ref)
        assert e_th <= 1e-11, f"{tag} theta d={d} {e_th:.2e}"
        assert e_f <= 1e-7, f"{tag} F d={d} {e_f:.2e}"
    assert _rel(fit.get("XL"), ref.XL) <= 1e-12
    assert _rel(fit.get("XN"), ref.XN) <= 1e-12 if ref.XN.any() else np.all(fit.get("XN") == 0)
    W = fit.get("W")
    e_w = _rel(W, ref.W)
    assert e_w <= 1e-9, f"{tag} W {e_w:.2e}"
    D = torch.tensor(s.D, dtype=torch.float64, device="cuda")
    K, ex = fit.exchange(D)
    K = K.cpu().numpy()
    dK = float(np.max(np.abs(K - ref.K)))
    dE = abs(ex - ref.E_x) / s.n_atoms
    print(f"[{tag}] W {e_w:.2e} max|dK| {dK:.2e} |dE|/atom {dE:.2e} E_x {ex:.10f}")
    assert dK <= 1e-7 and dE <= 1e-6
    return K, ex


@pytest.mark.parametrize("kind", ["one_atom", "two_atom"])
def test_tiny_cells_stage_parity(torch, kind):
    s = tiny_system(kind, n_occ=2 if kind == "one_atom" else 3)
    ref = pipeline.run(s)
    plan = binding.Plan(s)
    fit = plan.fit()
    _check_all(s, ref, plan, fit, torch, kind)


def test_single_level_textbook(torch):
    s = tiny_system("one_atom", grids=((15, 15, 15),), alpha_bound=(), n_mu_ratio=4.0)
    ref = pipeline.run(s)
    plan = binding.Plan(s)
    fit = plan.fit()
    _check_all(s, ref, plan, fit, torch, "single_level")


def test_cfg1_stage_parity(torch, cfg1_oracle):
    s, ref = cfg1_oracle
    plan = binding.Plan(s)
    fit = plan.fit()
    K, ex = _check_all(s, ref, plan, fit, torch, "cfg1")
    assert np.max(np.abs(K - K.T)) <= 1e-12 * np.max(np.abs(K))
    assert ex < 0


def test_cfg1_pinned_points(torch, cfg1_oracle):
    """Numeric parity independent of the selection: the oracle's points are
    handed to isdf_fit_with_points."""
    s, ref = cfg1_oracle
    plan = binding.Plan(s)
    fit = plan.fit(points=ref.pivots)
    _check_all(s, ref, plan, fit, torch, "cfg1-pinned")


def test_rank_short_domain_reports_and_matches(torch):
    """More points requested than the pair space has rank: the domain stops by
    eps_isdf, the call returns ISDF_E_RANK and the fit still matches."""
    s = tiny_system("one_atom", grids=((10, 10, 10),), alpha_bound=(), n_mu_ratio=40.0)
    ref = pipeline.run(s)
    plan = binding.Plan(s)
    fit = plan.fit(allow_rank=True)
    assert fit.status == -5
    assert fit.counts()[0] == len(ref.pivots[0]) < plan.domain(0)["n_mu"]
    _check_all(s, ref, plan, fit, torch, "rank-short")


def test_duplicate_pinned_points_not_spd(torch):
    s = tiny_system("one_atom")
    plan = binding.Plan(s)
    pts = [np.arange(plan.domain(d)["n_mu"]) for d in range(plan.n_domains)]
    pts[0][1] = pts[0][0]
    with pytest.raises(binding.IsdfError) as e:
        plan.fit(points=pts)
    assert e.value.status == -4


def test_nan_density_rejected(torch):
    s = tiny_system("one_atom")
    plan = binding.Plan(s)
    fit = plan.fit()
    D = torch.tensor(s.D, dtype=torch.float64, device="cuda")
    D[0, 0] = float("nan")
    with pytest.raises(binding.IsdfError) as e:
        fit.exchange(D)
    assert e.value.status == -1
