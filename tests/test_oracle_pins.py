"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(no GPU).  Each test names the slip it is meant to catch."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import basis, brute, coulomb, exchange, isdf, pipeline
from oracle import plan as oplan
from workloads import config, periodic_overlap, tiny_system
from workloads.diamond import System


# ---------------------------------------------------------------- basis (T1)
def test_basis_overlap_closed_form_cfg1_universal():
    """Grid quadrature of level-0 functions on the 24^3 grid equals the
    analytic periodic overlap (catches normalisation, p components, image
    lists).  Aliasing exp(-pi^2/(p h^2)) ~ 1e-20 here; the remaining gap is
    the pointwise image cutoff (terms below tau = 1e-10 are dropped)."""
    s = config(1, with_density=False)
    p = oplan.build_plan(s)
    dom = p.domains[0]
    Phi = basis.evaluate(p, 0, dom.points, dom.L)
    dV = p.level_spacing_volume(0)
    S_grid = dV * Phi.T @ Phi
    S_ref = periodic_overlap(s.lattice, s.xyz, s.shell_atom, s.shell_l, s.shell_alpha)
    S_ref = S_ref[np.ix_(dom.L, dom.L)]
    assert np.max(np.abs(S_grid - S_ref)) <= 3e-9 * np.max(np.abs(S_ref))
    assert np.allclose(np.diag(S_grid), np.diag(S_ref), rtol=3e-9)


def test_basis_overlap_closed_form_triclinic_fine_grid():
    """All functions of a strained two-atom cell on its fine grid (catches
    lattice-vector and fractional-coordinate slips in triclinic cells)."""
    s = tiny_system("two_atom", grids=((16, 16, 16), (32, 32, 32)))
    s.lattice = s.lattice @ (np.eye(3) + np.array([[0.02, 0.01, 0.0], [0.01, -0.015, 0.02], [0.0, 0.02, 0.01]]))
    p = oplan.build_plan(s)
    pts = np.arange(32 ** 3)
    Phi = basis.evaluate(p, 1, pts, np.arange(p.n_basis))
    S_grid = p.level_spacing_volume(1) * Phi.T @ Phi
    S_ref = periodic_overlap(s.lattice, s.xyz, s.shell_atom, s.shell_l, s.shell_alpha)
    # aliasing of the sharpest product (p = 8.1, h ~ 0.19) is ~1e-11
    assert np.max(np.abs(S_grid - S_ref)) <= 1e-8 * np.max(np.abs(S_ref))


def test_image_sum_matches_large_box():
    """The image list + pointwise cutoff reproduce an unscreened sum over a
    large box of translations to the cutoff level."""
    s = tiny_system("one_atom")
    p = oplan.build_plan(s)
    pts = np.array([0, 17, 999, 1727])
    Phi = basis.evaluate(p, 0, pts, np.arange(p.n_basis))
    pos = oplan.grid_positions(p.lattice, p.grids[0], pts)
    ref = np.zeros_like(Phi)
    n = np.arange(-6, 7)
    T = np.array(np.meshgrid(n, n, n, indexing="ij")).reshape(3, -1).T @ p.lattice
    for f in range(p.n_basis):
        a = p.f_alpha[f]
        A = p.xyz[p.f_atom[f]]
        nrm = basis.shell_norm(int(p.f_l[f]), a)
        d = pos[:, None, :] - (A + T)[None]
        g = nrm * np.exp(-a * np.sum(d * d, axis=2))
        ref[:, f] = g.sum(1) if p.f_comp[f] < 0 else (g * d[:, :, p.f_comp[f]]).sum(1)
    assert np.max(np.abs(Phi - ref)) < 1e-8


# ------------------------------------------------------------ plan / domains
def test_plan_counts_cfg1_cfg2():
    s1 = config(1, with_density=False)
    p1 = oplan.build_plan(s1)
    assert p1.n_basis == 104 and len(p1.domains) == 9 and p1.n_mu == 624
    assert p1.domains[0].L.size == 88 and p1.domains[0].points.size == 24 ** 3
    assert all(d.L.size == 2 and d.n_mu == 12 for d in p1.domains[1:])
    s2 = config(2, with_density=False)
    assert s2.n_basis == 832
    assert np.allclose(s2.alpha_bound, [8.0 / 9.0, 32.0 / 9.0], rtol=1e-12)


def test_window_points_bruteforce():
    """Window membership equals an explicit minimum-image distance test over
    every grid point of a strained cell."""
    lat = np.diag([7.0, 6.5, 6.8]) @ (np.eye(3) + np.array([[0.0, 0.03, 0.0], [0.03, 0.0, -0.02], [0.0, -0.02, 0.0]]))
    grid = (20, 18, 22)
    centre = np.array([0.3, 6.2, 1.1])
    r = 2.3
    got = oplan.window_points(lat, grid, centre, r)
    allp = np.arange(np.prod(grid))
    pos = oplan.grid_positions(lat, grid, allp)
    n = np.arange(-2, 3)
    T = np.array(np.meshgrid(n, n, n, indexing="ij")).reshape(3, -1).T @ lat
    dmin = np.min(np.linalg.norm(pos[:, None, :] - centre - T[None], axis=2), axis=1)
    want = allp[dmin <= r]
    assert np.array_equal(got, want)


def _owner_counts(p):
    N = p.n_basis
    cnt = np.zeros((N, N), dtype=int)
    for dom in p.domains:
        cnt += brute._pair_mask(dom, N)
    return cnt


@pytest.mark.parametrize("which", ["cfg1", "two_atom"])
def test_pair_coverage(which):
    """Every ordered pair with a non-negligible overlap is owned by exactly one
    domain mask L G + N L, and no pair is owned twice (catches the double
    count of same-level pairs on two windows)."""
    s = config(1, with_density=False) if which == "cfg1" else tiny_system("two_atom")
    p = oplan.build_plan(s)
    cnt = _owner_counts(p)
    assert cnt.max() <= 1
    assert np.array_equal(cnt, cnt.T)
    S = periodic_overlap(s.lattice, s.xyz, s.shell_atom, s.shell_l, s.shell_alpha)
    sig = np.abs(S) > 1e-7
    assert np.all(cnt[sig] == 1)


# ------------------------------------------------------------- Gram / pivots
def _random_domain(seed, npts=60, nL=2, nN=4):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((npts, nL + nN)), nL


def _explicit_Z(Phi, nL):
    """Rows: ordered pairs of the L G + N L mask; columns: points."""
    G = Phi.shape[1]
    rows = []
    for a in range(G):
        for b in range(G):
            if a < nL or b < nL:
                rows.append(Phi[:, a] * Phi[:, b])
    return np.array(rows)


def test_gram_equals_explicit_pair_sum():
    """M(R,R') = A_L (A_L + 2 A_N) equals sum over the ordered masked pairs of
    Eq. M(R,R) (catches a dropped factor 2 or a wrong mask)."""
    Phi, nL = _random_domain(1)
    Z = _explicit_Z(Phi, nL)
    M = Z.T @ Z
    cols = np.arange(Phi.shape[0])
    assert np.allclose(isdf.gram_columns(Phi, nL, cols), M, rtol=1e-12, atol=1e-12)
    assert np.allclose(isdf.gram_diag(Phi, nL), np.diag(M), rtol=1e-12)


def test_pivots_match_lapack_dpstrf():
    """Greedy pivots equal LAPACK's pivoted Cholesky on the explicit Gram."""
    Phi, nL = _random_domain(2, npts=50)
    M = isdf.gram_columns(Phi, nL, np.arange(50))
    c, piv, rank, info = sla.lapack.dpstrf(M, lower=1, tol=1e-13)
    k = min(int(rank), 12)
    got, _, _, _ = isdf.pivoted_cholesky(Phi, nL, k, 1e-14, 1e-12)
    assert np.array_equal(got, piv[:k] - 1)


def test_pivots_match_pivoted_qr():
    """Pivoted Cholesky on M gives the pivots of column-pivoted QR on the
    pair matrix (the equivalence stated in the Interpolative decomposition
    section)."""
    Phi, nL = _random_domain(3, npts=40)
    Z = _explicit_Z(Phi, nL)
    _, _, P = sla.qr(Z, pivoting=True, mode="economic")
    got, _, _, _ = isdf.pivoted_cholesky(Phi, nL, 10, 1e-14, 1e-12)
    assert np.array_equal(got, P[:10])


def test_tie_rule_smallest_index():
    """Exactly equal residuals: the smallest point index wins."""
    rng = np.random.default_rng(4)
    base = rng.standard_normal((5, 4))
    Phi = np.concatenate([base, base[[2]], base[[0]]], axis=0)  # rows 5, 6 duplicate 2, 0
    Phi[0] *= 3.0
    Phi[6] *= 3.0
    piv, _, _, _ = isdf.pivoted_cholesky(Phi, 2, 1, 1e-14, 1e-10)
    assert piv[0] == 0  # rows 0 and 6 tie for the maximum


def test_fit_lstsq_interpolation_and_cholesky_route():
    """F solves the least squares of Eq. lsqr, interpolates at the pivots,
    and equals L L_xi^{-1} from the pivoted-Cholesky factor."""
    Phi, nL = _random_domain(5, npts=70, nL=2, nN=3)
    piv, Lf, _, _ = isdf.pivoted_cholesky(Phi, nL, 8, 1e-14, 1e-12)
    F, Theta, Mxi = isdf.fit_functions(Phi, nL, piv)
    Z = _explicit_Z(Phi, nL)
    Ft, *_ = np.linalg.lstsq(Z[:, piv], Z, rcond=None)
    assert np.allclose(F, Ft.T, atol=1e-9)
    assert np.allclose(F[piv], np.eye(len(piv)), atol=1e-10)
    F2 = Lf @ np.linalg.inv(Lf[piv])
    assert np.allclose(F, F2, atol=1e-8)


# ------------------------------------------------------------ Coulomb (T2, T6)
def _gauss_density(lattice, grid, P, p):
    pts = np.arange(int(np.prod(grid)))
    pos = oplan.grid_positions(lattice, grid, pts)
    n = np.arange(-3, 4)
    T = np.array(np.meshgrid(n, n, n, indexing="ij")).reshape(3, -1).T @ lattice
    d = pos[:, None, :] - (P + T)[None]
    return ((p / np.pi) ** 1.5 * np.exp(-p * np.sum(d * d, axis=2))).sum(1)


def _gauss_coulomb_closed(lattice, P1, p1, P2, p2, mmax=40):
    """(rho1|rho2) = 4 pi / Omega sum_{G != 0} e^{-G^2/4p1 - G^2/4p2}
    cos(G.(P1-P2)) / G^2 for normalised periodic Gaussian charges."""
    B = 2 * np.pi * np.linalg.inv(lattice).T
    m = np.arange(-mmax, mmax + 1)
    M = np.array(np.meshgrid(m, m, m, indexing="ij")).reshape(3, -1).T
    M = M[np.any(M != 0, axis=1)]
    G = M @ B
    g2 = np.sum(G * G, axis=1)
    vol = abs(np.linalg.det(lattice))
    return 4 * np.pi / vol * np.sum(np.exp(-g2 / (4 * p1) - g2 / (4 * p2)) * np.cos(G @ (P1 - P2)) / g2)


def test_coulomb_gaussian_closed_form_same_and_cross_level():
    """FFT Poisson solve reproduces the analytic periodic Coulomb integral of
    Gaussian charges, on one grid and across grids through the coarse band
    (catches 4 pi/G^2 scaling, Omega/N_g normalisation, G = 0, Nyquist and
    the fine-to-coarse index map)."""
    lat = np.diag([6.3, 6.9, 6.6]) @ (np.eye(3) + np.array([[0, 0.02, 0.01], [0.02, 0, 0], [0.01, 0, 0]]))
    gc, gf = (24, 26, 24), (48, 52, 48)
    P1, p1 = np.array([1.1, 2.3, 0.7]), 0.9
    P2, p2 = np.array([4.0, 0.4, 3.9]), 1.4
    r1c = _gauss_density(lat, gc, P1, p1)
    r2f = _gauss_density(lat, gf, P2, p2)
    r1f = _gauss_density(lat, gf, P1, p1)
    vol = abs(np.linalg.det(lat))
    vc = coulomb.coulomb_kernel(lat, gc)
    vf = coulomb.coulomb_kernel(lat, gf)
    # same level, fine grid
    spec2 = coulomb.spectrum(r2f[:, None], gf)
    Vf = coulomb.potential_on(spec2, gf, gf, vf)[:, 0]
    e_ff = vol / np.prod(gf) * np.dot(r1f, Vf)
    ref = _gauss_coulomb_closed(lat, P1, p1, P2, p2)
    assert abs(e_ff - ref) <= 1e-10 * abs(ref)
    # cross level: coarse function against the fine one restricted to J_coarse
    Vc = coulomb.potential_on(spec2, gf, gc, vc)[:, 0]
    e_cf = vol / np.prod(gc) * np.dot(r1c, Vc)
    assert abs(e_cf - ref) <= 1e-10 * abs(ref)
    # self energy
    spec1 = coulomb.spectrum(r1c[:, None], gc)
    e_11 = vol / np.prod(gc) * np.dot(r1c, coulomb.potential_on(spec1, gc, gc, vc)[:, 0])
    assert abs(e_11 - _gauss_coulomb_closed(lat, P1, p1, P1, p1)) <= 1e-10 * e_11


def test_metric_all_points_is_circulant():
    """A single universal level with every point as a fitting function (F = I)
    gives W = Omega/N_g^2 c(R - R'), c(d) = sum_{m in J\\0} v(m) cos(G.d)
    (the circulant (R_U|R_U') of the paper), here for an odd and an even
    axis of a triclinic cell."""
    lat = np.array([[5.0, 0.3, 0.0], [0.2, 4.6, 0.4], [0.0, 0.5, 5.4]])
    grid = (5, 6, 4)
    s = System(lattice=lat, xyz=np.zeros((1, 3)), shell_atom=np.zeros(1, np.int32),
               shell_l=np.zeros(1, np.int32), shell_alpha=np.array([0.5]),
               grids=np.array([grid]), alpha_bound=np.zeros(0))
    p = oplan.build_plan(s)
    ng = int(np.prod(grid))
    W = coulomb.coulomb_metric(p, [np.eye(ng)])
    pos = oplan.grid_positions(lat, grid, np.arange(ng))
    B = 2 * np.pi * np.linalg.inv(lat).T
    ms = []
    for m1 in range(-3, 4):
        for m2 in range(-3, 4):
            for m3 in range(-3, 4):
                m = (m1, m2, m3)
                if all(2 * abs(mi) < n for mi, n in zip(m, grid)) and any(m):
                    ms.append(m)
    G = np.array(ms) @ B
    v = 4 * np.pi / np.sum(G * G, axis=1)
    d = pos[:, None, :] - pos[None, :, :]
    c = np.einsum("m,ijm->ij", v, np.cos(np.einsum("mk,ijk->ijm", G, d)))
    vol = abs(np.linalg.det(lat))
    assert np.allclose(W, vol / ng ** 2 * c, rtol=1e-12, atol=1e-12 * np.abs(W).max())


def test_metric_symmetric_psd_cfg1(cfg1_oracle):
    s, r = cfg1_oracle
    W = r.W
    ev = np.linalg.eigvalsh(W)
    assert ev[0] >= -1e-12 * ev[-1]


# ---------------------------------------------------------- exchange (T7-T9)
@pytest.fixture(scope="module")
def tiny_brute():
    s = tiny_system("one_atom", n_occ=2)
    p = oplan.build_plan(s)
    Kt, _ = brute.exchange_tensor_route(p, s.D)
    Ko = brute.exchange_orbital_route(p, s.C_occ)
    return s, p, Kt, Ko


def test_brute_force_two_routes_agree(tiny_brute):
    """Pair-tensor and occupied-orbital exact exchange agree (catches index
    slips in the D contraction)."""
    s, p, Kt, Ko = tiny_brute
    assert np.max(np.abs(Kt - Ko)) <= 1e-11 * np.max(np.abs(Kt))
    assert np.max(np.abs(Kt - Kt.T)) <= 1e-12 * np.max(np.abs(Kt))


def test_isdf_reaches_exact_exchange(tiny_brute):
    """With enough points to reach the rank of every domain's pair space the
    four-term ISDF exchange equals the exact one; with fewer points the
    error is larger (error -> 0 as the point count grows)."""
    s, p, Kt, _ = tiny_brute
    errs = []
    for ratio in (1.0, 2.0, 40.0):
        s.n_mu_ratio = ratio
        r = pipeline.run(s)
        errs.append(abs(r.E_x - float(np.sum(s.D * Kt))))
        if ratio == 40.0:
            assert np.max(np.abs(r.K - Kt)) <= 1e-8 * np.max(np.abs(Kt))
    assert errs[-1] <= 1e-9
    assert errs[0] > errs[-1]
    s.n_mu_ratio = 6.0


def test_isdf_two_atom_exact_limit():
    """Same limit with two atoms: cross-atom windows and the same-level
    ownership rule are exercised."""
    s = tiny_system("two_atom", n_occ=3)
    p = oplan.build_plan(s)
    Kt, _ = brute.exchange_tensor_route(p, s.D)
    s.n_mu_ratio = 40.0
    r = pipeline.run(s)
    assert np.max(np.abs(r.K - Kt)) <= 1e-8 * np.max(np.abs(Kt))


def test_exchange_invariants_cfg1(cfg1_oracle):
    """K symmetric, E_x = tr(DK) < 0 and -K positive semidefinite (the exchange
    matrix is negative definite)."""
    s, r = cfg1_oracle
    K = r.K
    assert np.max(np.abs(K - K.T)) <= 1e-12 * np.max(np.abs(K))
    assert r.E_x < 0
    ev = np.linalg.eigvalsh(-0.5 * (K + K.T))
    assert ev[0] >= -1e-10 * ev[-1]


def test_occ_ri_output_matches_full_exchange(cfg1_oracle):
    """occ-RI output (K C for D = C C^T): the oracle's contraction over
    n_occ-wide products equals the full four-term K built from D = C C^T and
    then applied to C, and sum(C o KC) is the same E_x (catches a swapped
    L/N block or a transposed pair product in the occupied-orbital form)."""
    s, r = cfg1_oracle
    C = s.C_occ
    KC = exchange.exchange_occ_ri(r.XL, r.XN, r.W, C)
    D = C @ C.T
    K_full = exchange.exchange_matrix(r.XL, r.XN, r.W, D)
    ref = K_full @ C
    assert np.max(np.abs(KC - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert abs(np.sum(C * KC) - exchange.exchange_energy(D, K_full)) <= 1e-12 * abs(r.E_x)
    # and the pipeline's own K (from the density of the workload) agrees
    assert np.max(np.abs(KC - r.K @ C)) <= 1e-10 * np.max(np.abs(ref))


def test_single_level_textbook_thc():
    """One level, one universal domain: the four-term formula reduces to the
    textbook K = -X^T [(X D X^T) o W] X."""
    s = tiny_system("one_atom", grids=((15, 15, 15),), alpha_bound=())
    r = pipeline.run(s)
    assert np.all(r.XN == 0)
    X = r.XL
    K2 = -X.T @ ((X @ s.D @ X.T) * r.W) @ X
    assert np.allclose(r.K, K2, rtol=1e-13, atol=1e-13 * np.abs(K2).max())


# ------------------------------------------------------------- MLP (T13)
def test_mlp_backward_matches_finite_differences():
    """The oracle's analytic backward of the scoring network equals central
    finite differences of its loss (catches a wrong ReLU mask, a transposed
    weight or a dropped pos-weight)."""
    from oracle import mlp

    rng = np.random.default_rng(11)
    X = rng.standard_normal((40, mlp.NF))
    y = (rng.random(40) < 0.2).astype(float)
    th = mlp.init_params(3)
    th[mlp.OFF_B1:mlp.OFF_W2] = 0.05 * rng.standard_normal(mlp.NH)
    th[mlp.OFF_B2:mlp.OFF_W3] = 0.05 * rng.standard_normal(mlp.NH)
    loss, g = mlp.loss_grad(th, X, y, 4.0)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 60, replace=False), [mlp.OFF_B3, mlp.OFF_W3]])
    eps = 1e-6
    for i in idx:
        tp = th.copy(); tp[i] += eps
        tm = th.copy(); tm[i] -= eps
        fd = (mlp.loss_grad(tp, X, y, 4.0)[0] - mlp.loss_grad(tm, X, y, 4.0)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_mlp_loss_is_weighted_bce():
    """Loss of a network with zero weights and bias b3 = z0 is the closed
    form pw y softplus(-z0) + (1-y) softplus(z0) averaged."""
    from oracle import mlp

    th = np.zeros(mlp.NPARAM)
    th[mlp.OFF_B3] = 0.7
    X = np.ones((5, mlp.NF))
    y = np.array([1, 0, 0, 1, 0], float)
    loss, _ = mlp.loss_grad(th, X, y, 3.0)
    sp = lambda v: np.log1p(np.exp(v))  # noqa: E731
    want = np.mean(3.0 * y * sp(-0.7) + (1 - y) * sp(0.7))
    assert abs(loss - want) < 1e-14


def test_mlp_features_simple_cases():
    """Feature definitions on a one-atom cell: the diagonal feature equals the
    Gram diagonal, distances are zero at the atom's grid point."""
    from oracle import isdf, mlp
    from oracle import plan as oplan

    s = tiny_system("one_atom")
    s.xyz = np.array([[0.0, 0.0, 0.0]])
    p = oplan.build_plan(s)
    dom = p.domains[1]
    F, Phi = mlp.domain_features(p, dom, s)
    g = isdf.gram_diag(Phi, dom.L.size)
    assert np.allclose(10 ** (10 * F[:, 2]), g, rtol=1e-12)
    assert np.isclose(F[:, 3].max(), 1.0)
    at = np.nonzero(dom.points == 0)[0][0]
    assert F[at, 8] == 0.0 and F[at, 9] == 0.0
    assert np.allclose(F[:, 1], 0.0) and np.allclose(F[:, 0], 1.0)


def test_restricted_selection_equals_full_on_needed_set():
    """Greedy selection restricted to the points whose initial diagonal is at
    least (1 - tau) times the last pivot residual (plus arbitrary extras)
    returns the full selection's pivots; dropping one needed point is caught
    by the exactness check."""
    s = config(1, with_density=False)
    p = oplan.build_plan(s)
    rng = np.random.default_rng(5)
    for d in (1, 4):
        dom = p.domains[d]
        Phi = basis.domain_values(p, dom)
        piv, L, _, d0 = isdf.pivoted_cholesky(Phi, dom.L.size, dom.n_mu, s.eps_isdf, s.tie_tol)
        dlast = L[piv[-1], len(piv) - 1] ** 2
        need = isdf.needed_points(d0, dlast, s.tie_tol)
        assert need.size < 0.2 * dom.points.size
        extra = rng.choice(dom.points.size, 200, replace=False)
        cand = np.union1d(need, extra)
        piv_r, Lr, _, _ = isdf.pivoted_cholesky(Phi, dom.L.size, dom.n_mu, s.eps_isdf, s.tie_tol, candidates=cand)
        assert np.array_equal(piv_r, piv)
        assert isdf.restriction_is_exact(d0, cand, Lr[piv_r[-1], len(piv_r) - 1] ** 2, s.tie_tol)
        worst = need[np.argmin(d0[need])]
        assert not isdf.restriction_is_exact(d0, np.setdiff1d(cand, [worst]), dlast, s.tie_tol)


# ------------------------------------------- thresholds (Eq. Ggrid, rank cap)
def _gaussian_spectrum(lattice, alpha, nref=48):
    """|DFT| / DFT[0] of the periodic Gaussian sum_T exp(-alpha |r - T|^2)
    sampled on an nref^3 grid; nref is chosen so that the Gaussian's
    spectrum is below 1e-16 at the reference grid's Nyquist plane, so the
    values are its Fourier coefficients (no aliasing at the levels tested)."""
    f = np.arange(nref) / nref
    F = np.stack(np.meshgrid(f, f, f, indexing="ij"), axis=-1).reshape(-1, 3)
    R = F @ lattice
    vol = abs(np.linalg.det(lattice))
    width = min(vol / np.linalg.norm(np.cross(lattice[(i + 1) % 3], lattice[(i + 2) % 3])) for i in range(3))
    k = int(np.ceil(np.sqrt(np.log(1e18) / alpha) / width)) + 1
    vals = np.zeros(R.shape[0])
    for n1 in range(-k, k + 1):
        for n2 in range(-k, k + 1):
            for n3 in range(-k, k + 1):
                d = R - np.array([n1, n2, n3], dtype=np.float64) @ lattice
                vals += np.exp(-alpha * np.sum(d * d, axis=1))
    c = np.abs(np.fft.fftn(vals.reshape(nref, nref, nref)))
    m = np.rint(np.fft.fftfreq(nref) * nref).astype(int)
    M = np.stack(np.meshgrid(m, m, m, indexing="ij"), axis=-1)
    return c / c[0, 0, 0], M


def _smaller_even_smooth(n):
    for c in range(n - 2, 1, -2):
        if all(p in (2, 3, 5) for p in _prime_factors(c)):
            return c
    return None


def _prime_factors(n):
    out, p = [], 2
    while n > 1:
        while n % p == 0:
            out.append(p)
            n //= p
        p += 1
    return out


_SKEWED = np.array([[6.0, 0.0, 0.0], [1.5, 5.5, 0.0], [0.8, 1.1, 5.2]])
_OBLIQUE = np.array([[7.0, 0.0, 0.0], [3.5, 3.0, 0.0], [1.0, 1.0, 4.0]])


@pytest.mark.parametrize("lattice,alpha,eps", [
    (np.eye(3) * 6.74, 0.45, 1e-2), (np.eye(3) * 6.74, 1.35, 1e-2), (np.eye(3) * 6.74, 1.35, 1e-3),
    (np.eye(3) * 6.74, 1.35, 1e-5), (np.eye(3) * 6.74, 0.45, 1e-8), (np.eye(3) * 6.74, 0.3, 0.3),
    (_SKEWED, 0.8, 1e-2), (_SKEWED, 0.8, 1e-4), (_SKEWED, 1.2, 1e-6),
    (_OBLIQUE, 0.8, 1e-2), (_OBLIQUE, 0.8, 1e-4), (_OBLIQUE, 0.3, 1e-3),
])
def test_threshold_grid_resolves_the_gaussian(lattice, alpha, eps):
    """The eps_K grid (Eq. Ggrid) keeps every Fourier coefficient of the
    level's sharpest Gaussian that is at least eps_K of the mean, measured by
    FFT of its samples: every coefficient outside the kept band |m_i| <=
    n_i/2 - 1 is below eps_K, and on the next smaller even smooth length of
    any axis some dropped coefficient is not (minimality).  Catches a wrong
    factor in G_max (2 alpha, ln without the 4), a kept Nyquist plane and a
    transposed reciprocal basis (skewed cell)."""
    n = oplan.grids_for_threshold(lattice, [0.1, alpha], [], eps)[0]
    rel, M = _gaussian_spectrum(lattice, alpha)
    outside = np.any(np.abs(M) >= n // 2, axis=-1)
    assert rel[outside].max() < eps
    for i in range(3):
        n_small = _smaller_even_smooth(int(n[i]))
        if n_small is None:
            continue
        dropped = np.abs(M[..., i]) >= n_small // 2
        assert rel[dropped].max() >= eps, f"axis {i}: {n_small} would do"


def test_threshold_ladder_levels():
    """Two levels: the coarse grid follows the largest exponent below the
    bound, the fine grid the largest overall, and the fine grid is never
    coarser than the coarse one (catches the level rule applied with <=,
    or the wrong exponent per level)."""
    lat = np.eye(3) * 6.74
    g = oplan.grids_for_threshold(lat, [0.15, 1.35, 2.0, 12.15], [2.0], 1e-2)
    coarse = oplan.grids_for_threshold(lat, [0.15, 1.35], [], 1e-2)[0]
    fine = oplan.grids_for_threshold(lat, [2.0, 12.15], [], 1e-2)[0]
    assert np.array_equal(g[0], coarse) and np.array_equal(g[1], fine)
    # a sharp exponent sits exactly at the bound: it belongs to the fine level
    g2 = oplan.grids_for_threshold(lat, [0.15, 2.0], [2.0], 1e-2)
    assert np.array_equal(g2[0], oplan.grids_for_threshold(lat, [0.15], [], 1e-2)[0])
    # a fine level below the coarse one is raised to it
    g3 = oplan.grids_for_threshold(lat, [0.16, 1.9, 2.0], [1.95], 1e-2)
    assert np.all(g3[1] >= g3[0])
    with pytest.raises(ValueError):
        oplan.grids_for_threshold(lat, [0.15, 0.3], [2.0], 1e-2)  # fine level empty


def test_threshold_only_cap_bounds_the_pair_rank():
    """With r <= 0 the plan caps N_mu,d at |L|(|L|+1)/2 + |L||N|.  The
    numerical rank of every domain's pair Gram (Eq. M(R,R)) is at most that
    bound, and the eps-only selection stops by the threshold at or below
    it, so the cap never cuts a selection short (catches a cap that counts
    only L L pairs or forgets the L N pairs)."""
    s = tiny_system("two_atom", grids=((10, 10, 10), (16, 16, 16)), n_mu_ratio=0.0)
    p = oplan.build_plan(s)
    for dom in p.domains:
        Phi = basis.domain_values(p, dom)
        nL, nN = dom.L.size, dom.N.size
        M = isdf.gram_columns(Phi, nL, np.arange(Phi.shape[0]))
        rank = np.linalg.matrix_rank(M, tol=1e-12 * np.max(np.abs(M)))
        assert rank <= nL * (nL + 1) // 2 + nL * nN
        assert dom.n_mu == min(dom.points.size, nL * (nL + 1) // 2 + nL * nN)
        piv, _, d, d0 = isdf.pivoted_cholesky(Phi, nL, dom.n_mu, 1e-10, s.tie_tol)
        assert piv.size < dom.n_mu or np.max(d) <= 1e-10 * np.max(d0)
        assert abs(piv.size - rank) <= max(2, rank // 10)


# ------------------------------------- universal grid, all points (occ-RI)
def test_universal_all_points_equals_exact_single_level():
    """One level: the universal domain owns every pair, so with every grid
    point as a fitting function its occ-RI exchange is the exact exchange
    (pair-tensor and occupied-orbital routes).  Catches a missing dV, a
    wrong pair product (E_i E_i) or a transposed Phi."""
    from oracle import universal

    s = tiny_system("one_atom", grids=((15, 15, 15),), alpha_bound=(), n_occ=2)
    p = oplan.build_plan(s)
    Kt, _ = brute.exchange_tensor_route(p, s.D)
    Ko = brute.exchange_orbital_route(p, s.C_occ)
    KC = universal.universal_exchange_occ_ri(p, s.C_occ)
    scale = np.max(np.abs(Kt @ s.C_occ))
    assert np.max(np.abs(KC - Kt @ s.C_occ)) <= 1e-12 * scale
    assert np.max(np.abs(KC - Ko @ s.C_occ)) <= 1e-12 * scale
    sub = universal.universal_exchange_occ_ri(p, s.C_occ, cols=[1])
    assert np.array_equal(sub[:, 0], KC[:, 1])


def test_universal_all_points_two_levels_is_the_diffuse_block():
    """Two levels: only diffuse-diffuse pairs belong to the universal grid.
    The result equals the exact exchange of a system that keeps only the
    diffuse shells on the universal grid, and rows of sharp functions are
    zero (catches pairs of sharp functions leaking into the universal
    block)."""
    import dataclasses

    from oracle import universal

    s = tiny_system("two_atom", grids=((12, 12, 12), (24, 24, 24)), alpha_bound=(2.0,), n_occ=3)
    p = oplan.build_plan(s)
    KC = universal.universal_exchange_occ_ri(p, s.C_occ)
    keep = s.shell_alpha < 2.0
    red = dataclasses.replace(s, shell_atom=s.shell_atom[keep], shell_l=s.shell_l[keep],
                              shell_alpha=s.shell_alpha[keep], grids=s.grids[:1],
                              alpha_bound=np.zeros(0))
    pr = oplan.build_plan(red)
    L0 = p.domains[0].G
    assert pr.n_basis == L0.size
    Kr, _ = brute.exchange_tensor_route(pr, s.D[np.ix_(L0, L0)])
    ref = Kr @ s.C_occ[L0]
    assert np.max(np.abs(KC[L0] - ref)) <= 1e-12 * np.max(np.abs(ref))
    others = np.setdiff1d(np.arange(p.n_basis), L0)
    assert others.size > 0 and np.all(KC[others] == 0.0)


def test_paper_exchange_reaches_exact_two_levels():
    """Every universal point a fitting function and windows at the exact
    limit (enough points for their pair rank): K C equals the exact
    exchange of the two-level plan (catches a cross block between the
    universal points and the windows taken with the wrong scale or
    orientation)."""
    from oracle import universal

    s = tiny_system("two_atom", grids=((12, 12, 12), (24, 24, 24)), alpha_bound=(2.0,), n_occ=3,
                    n_mu_ratio=40.0)
    p = oplan.build_plan(s)
    Kt, _ = brute.exchange_tensor_route(p, s.D)
    KC, piv = universal.paper_exchange_occ_ri(s, s.C_occ, plan=p)
    ref = Kt @ s.C_occ
    assert piv[0].size == 0 and all(x.size > 0 for x in piv[1:])
    assert np.max(np.abs(KC - ref)) <= 1e-8 * np.max(np.abs(ref))
    s.n_mu_ratio = 2.0  # fewer window points: a fitting error appears
    KC2, _ = universal.paper_exchange_occ_ri(s, s.C_occ)
    assert np.max(np.abs(KC2 - ref)) > 1e-6 * np.max(np.abs(ref))
