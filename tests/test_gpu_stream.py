"""Domain-group streaming of the basis values (phi_budget_mb) and domains
that take every one of their points (F = I).

Streaming changes only where the basis values live: each domain's
selection, Theta, solve and Coulomb rows run the same kernels on the same
values, so the streamed fit must equal the one-pass fit bit for bit
(pivots, X, F, W, K).  An all-point domain is checked against the oracle,
which takes the same reading (pivots 0..pts-1, F = I), at the parity
tolerances (max|dK| <= 1e-7 Ha, |dE_x| <= 1e-6 Ha/atom)."""
import numpy as np
import pytest

from oracle import pipeline
from paper_2404_09373_amd import binding
from workloads import config, initial_weights, tiny_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _fit_arrays(plan, fit):
    piv = [fit.get("points", d) for d in range(plan.n_domains)]
    return dict(counts=fit.counts(), piv=np.concatenate(piv), XL=fit.get("XL"), XN=fit.get("XN"),
                W=fit.get("W"), F=[fit.get("F", d) for d in range(plan.n_domains)])


@pytest.mark.parametrize("selector", ["full", "learned"])
def test_streamed_fit_is_the_one_pass_fit(torch, selector):
    s = config(2)
    kw = {}
    if selector == "learned":
        kw = dict(selector=binding.SEL_MLP, mlp_weights=initial_weights(3).astype(np.float32), mlp_keep=3.0,
                  mlp_cutoff=0.5)
    one = binding.Plan(s, **kw)
    grp = binding.Plan(s, phi_budget_mb=1500, **kw)
    f1 = one.fit()
    f2 = grp.fit()
    a, b = _fit_arrays(one, f1), _fit_arrays(grp, f2)
    print(f"[stream {selector}] N_mu {int(a['counts'].sum())} stages one-pass {np.round(one.stage_times()[:6], 1)} "
          f"streamed {np.round(grp.stage_times()[:6], 1)}")
    for k in ("counts", "piv", "XL", "XN", "W"):
        assert np.array_equal(a[k], b[k]), k
    for d in range(one.n_domains):
        assert np.array_equal(a["F"][d], b["F"][d]), d
    with pytest.raises(binding.IsdfError):
        f2.get("phi", 1)
    D = torch.tensor(s.D, dtype=torch.float64, device="cuda")
    K1, e1 = f1.exchange(D)
    K2, e2 = f2.exchange(D)
    assert torch.equal(K1, K2) and e1 == e2


def test_all_point_domain_matches_oracle(torch):
    s = tiny_system("d_atom", grids=((6, 6, 6), (24, 24, 24)), n_occ=3)
    s.n_mu_ratio = 30.0  # universal domain capped at its 216 points, window 150 of 3701
    ref = pipeline.run(s)
    for budget in (0, 1):  # one pass, then one domain per group
        plan = binding.Plan(s, phi_budget_mb=budget)
        fit = plan.fit()
        assert np.array_equal(fit.get("points", 0), np.arange(216))
        assert np.array_equal(fit.get("F", 0), np.eye(216))
        assert np.array_equal(fit.get("points", 1), np.asarray(ref.pivots[1]))
        D = torch.tensor(s.D, dtype=torch.float64, device="cuda")
        K, e = fit.exchange(D)
        dK = float(np.max(np.abs(K.cpu().numpy() - ref.K)))
        dE = abs(e - ref.E_x) / s.n_atoms
        print(f"[all-points budget {budget}] max|dK| {dK:.2e} |dE|/atom {dE:.2e}")
        assert dK <= 1e-7 and dE <= 1e-6
        fit.close()
        plan.close()


@pytest.mark.parametrize("precision", ["fp64", "x6"])
def test_occ_ri_row_blocks(torch, precision, cfg1_oracle):
    """K C with Q held in row blocks (ri_rows; 624 rows in blocks of 200,
    the last one ragged) equals the one-block result and the oracle."""
    s, ref = cfg1_oracle
    prec = binding.FP64 if precision == "fp64" else binding.MIXED_X6
    C = torch.tensor(s.C_occ, dtype=torch.float64, device="cuda")
    out = {}
    for rows in (0, 200):
        plan = binding.Plan(s, precision=prec, ri_rows=rows)
        fit = plan.fit()
        KC = torch.empty_like(C)
        _, e = fit.exchange_occ_ri(C, KC)
        _, e2 = fit.exchange_occ_ri(C, KC)  # the replayed graph
        assert e2 == e
        out[rows] = (KC.cpu().numpy(), e)
        fit.close()
        plan.close()
    (a, ea), (b, eb) = out[0], out[200]
    scale = float(np.max(np.abs(a)))
    d_blk = float(np.max(np.abs(a - b))) / scale
    ref_kc = ref.K @ s.C_occ
    dK = float(np.max(np.abs(b - ref_kc)))
    dE = abs(eb - ref.E_x) / s.n_atoms
    print(f"[occ-RI rows {precision}] blocks vs one block rel {d_blk:.2e}; vs oracle max|dKC| {dK:.2e} "
          f"|dE|/atom {dE:.2e}")
    assert d_blk <= 1e-12
    assert dE <= 1e-6
    assert dK <= (1e-7 if precision == "fp64" else 1e-5)


def test_repeated_fits_take_no_new_blocks(torch):
    """A plan's second fit and exchange (streamed basis values, learned
    selector, occ-RI rows in blocks) are served from the blocks the first
    ones released: no new device allocation."""
    s = config(2)
    plan = binding.Plan(s, precision=binding.MIXED_X6, selector=binding.SEL_MLP,
                        mlp_weights=initial_weights(3).astype(np.float32), mlp_keep=3.0, mlp_cutoff=0.5,
                        phi_budget_mb=1500, ri_rows=2048)
    C = torch.tensor(s.C_occ, dtype=torch.float64, device="cuda")
    KC = torch.empty_like(C)
    for rep in range(3):
        fit = plan.fit()
        fit.exchange_occ_ri(C, KC)
        fit.close()
        st = plan.alloc_stats()
        print(f"[alloc] after fit {rep}: {st}")
        if rep == 1:
            first = st
    assert st["calls"] == first["calls"] and st["bytes"] == first["bytes"]
    plan.close()
