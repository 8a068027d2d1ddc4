"""Universal grid with every point as a fitting function on the GPU
(isdf_exchange_universal): the diffuse-diffuse exchange from occupied pair
densities by FFT Poisson solves, (R_U|R_U') never stored.

* one-level system: the universal domain owns every pair, so the result is
  the exact exchange (oracle brute force, both routes pinned);
* 8-atom cell: every entry against the oracle's occ-RI route;
* 64-atom cell at its full size: sampled occupied columns against the
  oracle, and C^T K_UU C symmetric and negative semidefinite;
* argument errors and a plan without a universal domain.
"""
import numpy as np
import pytest

from paper_2404_09373_amd import binding
from workloads import config, tiny_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available()
    return t


def _run(torch, s):
    plan = binding.Plan(s)
    fit = plan.fit()
    C = torch.tensor(s.C_occ, dtype=torch.float64, device="cuda")
    KC, e = fit.exchange_universal(C)
    out = KC.cpu().numpy()
    fit.close()
    plan.close()
    return out, e


def test_universal_single_level_is_exact(torch):
    from oracle import brute
    from oracle import plan as oplan

    s = tiny_system("one_atom", grids=((15, 15, 15),), alpha_bound=(), n_occ=2)
    KC, e = _run(torch, s)
    Kt, _ = brute.exchange_tensor_route(oplan.build_plan(s), s.D)
    ref = Kt @ s.C_occ
    d = float(np.max(np.abs(KC - ref))) / float(np.max(np.abs(ref)))
    print(f"[universal] one level 15^3: rel max|dKC| vs exact {d:.2e}, E {e:.12f} / {np.sum(s.D * Kt):.12f}")
    assert d <= 1e-11 and abs(e - np.sum(s.D * Kt)) <= 1e-11 * abs(e)


def test_universal_cfg1_matches_oracle(torch):
    from oracle import universal
    from oracle import plan as oplan

    s = config(1)
    KC, e = _run(torch, s)
    ref = universal.universal_exchange_occ_ri(oplan.build_plan(s), s.C_occ)
    d = float(np.max(np.abs(KC - ref))) / float(np.max(np.abs(ref)))
    e_ref = float(np.sum(s.C_occ * ref))
    print(f"[universal] cfg1: rel max|dKC| {d:.2e}, E_UU {e:.12f} / {e_ref:.12f}")
    assert d <= 1e-11 and abs(e - e_ref) <= 1e-11 * abs(e_ref)


def test_universal_cfg2_sampled_columns(torch):
    from oracle import universal
    from oracle import plan as oplan

    s = config(2)
    KC, e = _run(torch, s)
    cols = [0, 77, s.n_occ - 1]
    ref = universal.universal_exchange_occ_ri(oplan.build_plan(s), s.C_occ, cols=cols)
    d = float(np.max(np.abs(KC[:, cols] - ref))) / float(np.max(np.abs(ref)))
    G = s.C_occ.T @ KC  # C^T K_UU C
    asym = float(np.max(np.abs(G - G.T))) / float(np.max(np.abs(G)))
    ev = np.linalg.eigvalsh(0.5 * (G + G.T))
    print(f"[universal] cfg2 sampled columns {cols}: rel max|dKC| {d:.2e}; C'KC asym {asym:.1e}, "
          f"eig max {ev[-1]:.2e} min {ev[0]:.2e}, E_UU {e:.10f} tr {np.trace(G):.10f}")
    assert d <= 1e-11
    assert asym <= 1e-12 and ev[-1] <= 1e-12 * abs(ev[0])
    assert abs(e - np.trace(G)) <= 1e-12 * abs(e)


def test_universal_rejects_bad_arguments(torch):
    s = config(1)
    plan = binding.Plan(s)
    fit = plan.fit()
    n = plan.n_basis
    with pytest.raises(ValueError):
        fit.exchange_universal(torch.zeros((n + 1, 4), dtype=torch.float64, device="cuda"))
    C0 = torch.zeros((n, 4), dtype=torch.float64, device="cuda")
    KC = torch.empty_like(C0)
    lib = binding.load()
    for bad in (0, n + 1):
        assert lib.isdf_exchange_universal(plan.handle, fit.handle, binding.C.c_void_p(C0.data_ptr()), bad,
                                           binding.C.c_void_p(KC.data_ptr()), None) == -1
    fit.close()
    plan.close()
    # every shell above the bound: the plan holds atom windows only
    t = tiny_system("one_atom", grids=((12, 12, 12), (24, 24, 24)), alpha_bound=(0.1,), n_occ=2)
    p2 = binding.Plan(t)
    f2 = p2.fit()
    C2 = torch.tensor(t.C_occ, dtype=torch.float64, device="cuda")
    with pytest.raises(binding.IsdfError) as err:
        f2.exchange_universal(C2)
    assert err.value.status == -7
    f2.close()
    p2.close()


# ------------------------------- the method with every universal point a fitting function
def _all_points_cell():
    s = config(1)
    s.grids = np.array([[12, 12, 12], [36, 36, 36]])
    return s


@pytest.mark.parametrize("precision", [binding.FP64, binding.MIXED_X6])
def test_all_points_method_matches_oracle(torch, precision):
    """universal_all_points: no selection on the universal grid, windows as
    usual, cross terms through W_Uw and the universal block by FFT; K C
    against the oracle's dense form of the same method."""
    from oracle import universal

    s = _all_points_cell()
    ref, piv = universal.paper_exchange_occ_ri(s, s.C_occ)
    plan = binding.Plan(s, precision=precision, universal_all_points=True)
    fit = plan.fit()
    assert fit.get("points", 0).size == 0
    for d in range(1, plan.n_domains):
        assert np.array_equal(fit.get("points", d), piv[d]), f"domain {d}"
    C = torch.tensor(s.C_occ, dtype=torch.float64, device="cuda")
    KC, e = fit.exchange_occ_ri(C)
    KC2, e2 = fit.exchange_occ_ri(C)  # a second call on the same fit
    KC, KC2 = KC.cpu().numpy(), KC2.cpu().numpy()
    d = float(np.max(np.abs(KC - ref))) / float(np.max(np.abs(ref)))
    e_ref = float(np.sum(s.C_occ * ref))
    dE = abs(e - e_ref) / s.n_atoms
    # the same cell with a fitted universal grid, for scale
    pf = binding.Plan(s, precision=precision)
    ff = pf.fit()
    _, e_fit = ff.exchange_occ_ri(C)
    print(f"[all points] precision {precision}: rel max|dKC| {d:.2e}, |dE|/atom {dE:.2e}, "
          f"E_x {e:.10f} (fitted universal grid {e_fit:.10f})")
    tol = 1e-11 if precision == binding.FP64 else 1e-5
    assert d <= tol and dE <= (1e-11 if precision == binding.FP64 else 1e-7)
    assert np.array_equal(KC, KC2) and e == e2
    with pytest.raises(binding.IsdfError) as err:
        fit.exchange_occ(C)
    assert err.value.status == -7
    for f in (fit, ff):
        f.close()
    for p in (plan, pf):
        p.close()


def test_all_points_needs_windows():
    s = tiny_system("one_atom", grids=((15, 15, 15),), alpha_bound=(), n_occ=2)
    with pytest.raises(binding.IsdfError) as err:
        binding.Plan(s, universal_all_points=True)
    assert err.value.status == -7


@pytest.mark.parametrize("n_occ", [1, 3])
def test_universal_few_orbitals(torch, n_occ):
    """An odd number of pair densities (one complex array half empty) and a
    single orbital, against the oracle."""
    from oracle import universal
    from oracle import plan as oplan

    s = config(1)
    C_sub = np.ascontiguousarray(s.C_occ[:, :n_occ])
    plan = binding.Plan(s)
    fit = plan.fit()
    KC, e = fit.exchange_universal(torch.tensor(C_sub, dtype=torch.float64, device="cuda"))
    ref = universal.universal_exchange_occ_ri(oplan.build_plan(s), C_sub)
    d = float(np.max(np.abs(KC.cpu().numpy() - ref))) / float(np.max(np.abs(ref)))
    print(f"[universal] cfg1 n_occ {n_occ}: rel max|dKC| {d:.2e}")
    assert d <= 1e-11 and abs(e - float(np.sum(C_sub * ref))) <= 1e-11 * abs(e)
    fit.close()
    plan.close()


def test_all_points_single_orbital(torch):
    from oracle import universal

    s = _all_points_cell()
    C_sub = np.ascontiguousarray(s.C_occ[:, :1])
    ref, _ = universal.paper_exchange_occ_ri(s, C_sub)
    plan = binding.Plan(s, universal_all_points=True)
    fit = plan.fit()
    KC, e = fit.exchange_occ_ri(torch.tensor(C_sub, dtype=torch.float64, device="cuda"))
    d = float(np.max(np.abs(KC.cpu().numpy() - ref))) / float(np.max(np.abs(ref)))
    print(f"[all points] n_occ 1: rel max|dKC| {d:.2e}")
    assert d <= 1e-11
    fit.close()
    plan.close()


def test_all_points_with_learned_selector(torch):
    """The learned candidate selector on the windows of an all-points plan
    (the universal domain requests no points and is left out): the same
    pivots and the same K C as full selection, whatever the weights (here
    an untrained network; failed candidate lists fall back to full
    selection)."""
    from oracle import mlp as omlp

    s = _all_points_cell()
    C = torch.tensor(s.C_occ, dtype=torch.float64, device="cuda")
    pf = binding.Plan(s, universal_all_points=True)
    pm = binding.Plan(s, universal_all_points=True, selector=binding.SEL_MLP,
                      mlp_weights=omlp.init_params(0).astype(np.float32), mlp_keep=2.0, mlp_cutoff=0.05)
    ff, fm = pf.fit(), pm.fit()
    for d in range(pf.n_domains):
        assert np.array_equal(ff.get("points", d), fm.get("points", d)), f"domain {d}"
    KCf, ef = ff.exchange_occ_ri(C)
    KCm, em = fm.exchange_occ_ri(C)
    info = fm.selection()
    print(f"[all points] learned selector: candidates {int(np.sum(info['n_candidates']))}, "
          f"fallbacks {int(np.sum(info['fallback']))}, E_x {em:.12f} / {ef:.12f}")
    assert torch.equal(KCf, KCm) and ef == em
    for f in (ff, fm):
        f.close()
    for p in (pf, pm):
        p.close()


def test_universal_tiles_of_pair_rows(torch):
    """A budget of 1 MB holds a few pair rows at a time (the 8-atom cell's
    24^3 grid: 110 kB a potential): many tiles give the same K_UU C as one
    tile (sums in another order), also inside the all-points exchange."""
    s = config(1)
    C = torch.tensor(s.C_occ, dtype=torch.float64, device="cuda")
    out = {}
    for mb in (0, 1):
        plan = binding.Plan(s, universal_tile_mb=mb)
        fit = plan.fit()
        KC, e = fit.exchange_universal(C)
        out[mb] = (KC.cpu().numpy(), e)
        fit.close()
        plan.close()
    d = float(np.max(np.abs(out[0][0] - out[1][0]))) / float(np.max(np.abs(out[0][0])))
    print(f"[universal] 1 MB tiles vs one tile: rel max|dKC| {d:.2e}")
    assert d <= 1e-13 and abs(out[0][1] - out[1][1]) <= 1e-13 * abs(out[0][1])
    s2 = _all_points_cell()
    C2 = torch.tensor(s2.C_occ, dtype=torch.float64, device="cuda")
    res = []
    for mb in (0, 1):
        plan = binding.Plan(s2, universal_all_points=True, universal_tile_mb=mb)
        fit = plan.fit()
        KC, e = fit.exchange_occ_ri(C2)
        res.append(KC.cpu().numpy())
        fit.close()
        plan.close()
    d2 = float(np.max(np.abs(res[0] - res[1]))) / float(np.max(np.abs(res[0])))
    print(f"[all points] 1 MB tiles vs one tile: rel max|dKC| {d2:.2e}")
    assert d2 <= 1e-13
    with pytest.raises(binding.IsdfError) as err:
        binding.Plan(s, universal_tile_mb=-1)
    assert err.value.status == -1
