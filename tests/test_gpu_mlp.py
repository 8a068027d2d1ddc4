"""Learned candidate selector on the GPU: features, forward and gradients
against the FP64 oracle, the candidate-restricted selection, training, and
what the trained network gains over full selection.

Tolerances: features 1e-5 (FP32 output of FP64 arithmetic), logits 1e-5
relative, gradients 1e-4 of the largest component (FP32 sums over 4096 rows),
restricted pivots identical to the full ones whenever the exactness check
passes, exchange energies then equal to 1e-10 Ha/atom.
"""
import time

import numpy as np
import pytest

from oracle import basis, isdf, mlp, pipeline
from oracle import plan as oplan
from paper_2404_09373_amd import binding
from workloads import config, diamond_system, tiny_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available()
    return t


def test_features_match_oracle(torch):
    for s in (tiny_system("two_atom"), config(1, with_density=False)):
        plan = binding.Plan(s)
        fit = plan.fit()
        X, _ = fit.features(with_labels=False)
        X = X.cpu().numpy()
        op = oplan.build_plan(s)
        off = 0
        for d, dom in enumerate(op.domains):
            n = dom.points.size
            if d in (0, 1, len(op.domains) - 1):
                F, _ = mlp.domain_features(op, dom, s)
                err = np.abs(X[off:off + n] - F) / np.maximum(1.0, np.abs(F))
                assert err.max() <= 1e-5, (s.name, d, err.max(axis=0))
            off += n


def test_forward_and_gradient_match_oracle(torch):
    rng = np.random.default_rng(3)
    th = mlp.init_params(7)
    th[mlp.OFF_B1:mlp.OFF_W2] = 0.1 * rng.standard_normal(mlp.NH)
    X = rng.standard_normal((4096, mlp.NF)).astype(np.float32)
    y = (rng.random(4096) < 0.1).astype(np.float32)
    Xd = torch.tensor(X, device="cuda")
    yd = torch.tensor(y, device="cuda")
    z = binding.mlp_forward(th.astype(np.float32), Xd).cpu().numpy()
    th32 = th.astype(np.float32).astype(np.float64)
    z_ref, _ = mlp.forward(th32, X.astype(np.float64))
    assert np.max(np.abs(z - z_ref)) <= 1e-5 * max(1.0, np.max(np.abs(z_ref)))
    loss, g = binding.mlp_loss_grad(th.astype(np.float32), Xd, yd, 9.0)
    loss_ref, g_ref = mlp.loss_grad(th32, X.astype(np.float64), y.astype(np.float64), 9.0)
    assert abs(loss - loss_ref) <= 1e-5 * abs(loss_ref)
    assert np.max(np.abs(g - g_ref)) <= 1e-4 * np.max(np.abs(g_ref))


def test_candidate_selection_exact_and_detected(torch, cfg1_oracle):
    """Candidates = the oracle's needed set plus random extras: the GPU's
    restricted selection returns the full pivots and passes the check; a set
    missing one needed point is flagged."""
    s, ref = cfg1_oracle
    op = ref.plan
    rng = np.random.default_rng(1)
    good, bad = [], []
    for d, dom in enumerate(op.domains):
        Phi = basis.domain_values(op, dom)
        piv, L, _, d0 = isdf.pivoted_cholesky(Phi, dom.L.size, dom.n_mu, s.eps_isdf, s.tie_tol)
        dlast = L[piv[-1], len(piv) - 1] ** 2
        need = isdf.needed_points(d0, dlast, s.tie_tol)
        extra = rng.choice(dom.points.size, min(300, dom.points.size), replace=False)
        cand = np.union1d(need, extra)
        good.append(cand)
        worst = need[np.argmin(d0[need])]
        bad.append(np.setdiff1d(cand, [worst]) if d > 0 else cand)
    plan = binding.Plan(s)
    fit = plan.fit(candidates=good)
    rep = fit.selection()
    assert not rep["fallback"].any()
    for d in range(plan.n_domains):
        assert np.array_equal(fit.get("points", d), ref.pivots[d])
    D = torch.tensor(s.D, dtype=torch.float64, device="cuda")
    _, ex = fit.exchange(D)
    assert abs(ex - ref.E_x) / s.n_atoms <= 1e-10
    fit2 = plan.fit(candidates=bad)
    assert fit2.selection()["fallback"][1:].all()


def _train_on(fits, torch, epochs=12):
    Xs, Ys = [], []
    for f in fits:
        X, Y = f.features()
        Xs.append(X)
        Ys.append(Y)
    X = torch.cat(Xs)
    Y = torch.cat(Ys)
    w0 = mlp.init_params(0).astype(np.float32)
    w, hist = binding.mlp_train(X, Y, w0, epochs=epochs, batch=16384, lr=2e-3, seed=1)
    return w, hist, X, Y


def test_training_reduces_loss_and_recalls_needed_points(torch):
    s = config(1, with_density=False)
    plan = binding.Plan(s)
    fit = plan.fit()
    w, hist, X, Y = _train_on([fit], torch, epochs=15)
    assert hist[-1] < 0.5 * hist[0], hist
    z = binding.mlp_forward(w, X).cpu().numpy()
    y = Y.cpu().numpy()
    p = 1 / (1 + np.exp(-z))
    recall = (p[y > 0.5] >= 0.05).mean()
    assert recall > 0.98, recall


def test_learned_selector_gain_on_64_atoms(torch):
    """Trained on selections of the 8-atom cell and of a differently
    displaced 64-atom cell, the network prunes the windows of the benchmark
    64-atom cell; every domain either passes the exactness check or falls
    back, so E_x equals full selection, and the selection stage is faster."""
    train_sys = [config(1, with_density=False),
                 diamond_system((2, 2, 2), ((32, 32, 32), (64, 64, 64), (128, 128, 128)), 8.0, 128,
                                0.05, 0.0, 777, 778, with_density=False)]
    fits = []
    for ts in train_sys:
        pl = binding.Plan(ts)
        fits.append(pl.fit())
    w, hist, _, _ = _train_on(fits, torch, epochs=10)
    for f in fits:
        f.close()
    s = config(2)
    D = torch.tensor(s.D, dtype=torch.float64, device="cuda")
    full = binding.Plan(s)
    learned = binding.Plan(s, selector=binding.SEL_MLP, mlp_weights=w, mlp_keep=2.0, mlp_cutoff=0.05)
    f0 = full.fit()  # warm both paths once
    f0.close()
    f1 = learned.fit()
    f1.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ff = full.fit()
    t_full = time.perf_counter() - t0
    sel_full = full.stage_times()[1]
    t0 = time.perf_counter()
    fl = learned.fit()
    t_mlp = time.perf_counter() - t0
    sel_mlp = learned.stage_times()[1]
    rep = fl.selection()
    _, e_full = ff.exchange(D)
    _, e_mlp = fl.exchange(D)
    win = np.arange(1, full.n_domains)
    pts = np.array([full.domain(d)["points"].size for d in win])
    prune = pts.sum() / rep["n_candidates"][win].sum()
    print(f"[mlp gain] fit full {t_full:.3f}s mlp {t_mlp:.3f}s; selection full {sel_full:.1f}ms "
          f"mlp {sel_mlp:.1f}ms; window points pruned {prune:.1f}x; fallbacks "
          f"{int(rep['fallback'].sum())}/{full.n_domains}; dE/atom {abs(e_mlp - e_full) / s.n_atoms:.2e}")
    assert abs(e_mlp - e_full) / s.n_atoms <= 1e-10
    for d in range(full.n_domains):
        assert np.array_equal(fl.get("points", d), ff.get("points", d))
    assert rep["fallback"].sum() < 0.25 * full.n_domains
    assert prune > 2.0
    assert sel_mlp < sel_full
