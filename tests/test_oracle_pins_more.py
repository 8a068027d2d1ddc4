"""More pins of the FP64 oracle (no GPU): d shells, the optimiser of the
point-scoring network, every selector feature, the window image screen, the
multi-level assembly of the Coulomb metric and the full-cell domain mode.
Each test names the slip it is meant to catch."""
import dataclasses

import numpy as np
import pytest

from oracle import basis, brute, coulomb, exchange, isdf, mlp, pipeline
from oracle import plan as oplan
from workloads import config, periodic_overlap, primitive_norm, tiny_system


# ------------------------------------------------------------- d shells (T1)
def _hermite_nodes(n=6):
    x, w = np.polynomial.hermite.hermgauss(n)
    return x, w


def test_d_harmonics_are_an_orthonormal_harmonic_basis():
    """The oracle's five d angular factors are quadratic forms r^T A_m r with
    tr A_m = 0 (harmonic: the Laplacian of r^T A r is 2 tr A), homogeneous of
    degree 2, mutually orthogonal with equal norm on the sphere
    (int (r^T A r)(r^T B r) dOmega = 8 pi/15 tr(AB) for traceless A, B; norm
    4 pi/5 <=> tr(A^2) = 3/2) and satisfy the addition theorem
    sum_m Y_m(r)^2 = r^4.  Catches a wrong coefficient (sqrt3 vs 3, 1/2 vs
    1), a non-traceless m = 0 term or a duplicated component."""
    E = np.eye(3)
    A = np.zeros((5, 3, 3))
    for m in range(5):
        for i in range(3):
            A[m, i, i] = basis.solid_harmonic(2, m, E[i][None])[0]
        for i in range(3):
            for j in range(i + 1, 3):
                v = basis.solid_harmonic(2, m, (E[i] + E[j])[None])[0]
                A[m, i, j] = A[m, j, i] = 0.5 * (v - A[m, i, i] - A[m, j, j])
    rng = np.random.default_rng(3)
    r = rng.standard_normal((50, 3))
    for m in range(5):
        assert abs(np.trace(A[m])) < 1e-15
        got = basis.solid_harmonic(2, m, r)
        assert np.allclose(got, np.einsum("pi,ij,pj->p", r, A[m], r), rtol=1e-14, atol=1e-14)
        assert np.allclose(basis.solid_harmonic(2, m, 2.0 * r), 4.0 * got, rtol=1e-14)
    G = np.einsum("mij,nji->mn", A, A)
    assert np.allclose(G, 1.5 * np.eye(5), atol=1e-14)
    tot = sum(basis.solid_harmonic(2, m, r) ** 2 for m in range(5))
    assert np.allclose(tot, np.sum(r * r, axis=1) ** 2, rtol=1e-13)


@pytest.mark.parametrize("l", [0, 1, 2])
def test_single_centre_unit_norm_gauss_hermite(l):
    """int (N_l Y_lm(r) exp(-a r^2))^2 d^3r = 1 for every component, by
    tensor Gauss-Hermite quadrature (exact for a polynomial of degree <= 11
    times exp(-2 a r^2)); the components are orthogonal.  Catches a wrong
    normalisation constant (N_d = N_s 4a/sqrt3) independently of the closed
    form overlap."""
    a = 0.7
    x, w = _hermite_nodes(8)
    s = 1.0 / np.sqrt(2.0 * a)  # exp(-2 a r^2) = exp(-(r/s)^2)
    X, Y, Z = np.meshgrid(x * s, x * s, x * s, indexing="ij")
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]) * s ** 3
    d = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
    W = W.ravel()
    nrm = basis.shell_norm(l, a)
    assert np.isclose(nrm, primitive_norm(l, a), rtol=1e-15)
    nc = 2 * l + 1
    Yv = np.array([basis.solid_harmonic(l, c if l else -1, d) for c in range(nc)])
    G = nrm * nrm * (Yv * W) @ Yv.T
    assert np.allclose(G, np.eye(nc), atol=1e-13)


def test_basis_overlap_closed_form_d_shells():
    """Grid quadrature of every function (s, p, d on both levels) of a
    strained two-atom cell equals the Obara-Saika periodic overlap (catches
    the d normalisation, the component order and the image sum)."""
    s = tiny_system("d_two", grids=((16, 16, 16), (40, 40, 40)))
    s.lattice = s.lattice @ (np.eye(3) + np.array([[0.02, 0.01, 0.0], [0.01, -0.015, 0.02],
                                                   [0.0, 0.02, 0.01]]))
    p = oplan.build_plan(s)
    pts = np.arange(40 ** 3)
    Phi = basis.evaluate(p, 1, pts, np.arange(p.n_basis))
    S_grid = p.level_spacing_volume(1) * Phi.T @ Phi
    S_ref = periodic_overlap(s.lattice, s.xyz, s.shell_atom, s.shell_l, s.shell_alpha)
    # aliasing of the sharpest product (p = 5, h ~ 0.15) is ~1e-20; the gap
    # (4e-9) is the pointwise image cutoff (tau = 1e-10) of the diffuse shells
    assert np.max(np.abs(S_grid - S_ref)) <= 1e-8 * np.max(np.abs(S_ref))


def test_overlap_large_cell_single_centre():
    """In a cell much larger than the functions, the periodic overlap of one
    atom's shells is the single-centre identity (unit norm, orthogonal
    components within a shell) and s-d / p-p cross terms take their closed
    values (catches an Obara-Saika recursion slip)."""
    lat = np.eye(3) * 30.0
    xyz = np.array([[3.0, 4.0, 5.0]])
    sl = np.array([0, 1, 2, 2])
    sa = np.array([0.8, 0.9, 1.1, 2.0])
    S = periodic_overlap(lat, xyz, np.zeros(4, np.int64), sl, sa)
    assert np.allclose(np.diag(S), 1.0, atol=1e-14)
    assert np.allclose(S[1:4, 1:4], np.eye(3), atol=1e-14)
    assert np.allclose(S[4:9, 4:9], np.eye(5), atol=1e-14)
    # s with d on the same centre: only m = 0 survives by symmetry and it
    # vanishes too (traceless); d(a) with d(b) on one centre: diagonal
    # (2 sqrt(ab) / (a + b))^(7/2)
    assert np.allclose(S[0, 4:14], 0.0, atol=1e-14)
    want = (2.0 * np.sqrt(1.1 * 2.0) / 3.1) ** 3.5
    assert np.allclose(S[4:9, 9:14], want * np.eye(5), atol=1e-14)


@pytest.mark.parametrize("kind", ["d_atom", "d_two"])
def test_isdf_reaches_exact_exchange_with_d_shells(kind):
    """With d shells on both levels the four-term ISDF exchange reaches the
    brute-force exact exchange at the rank limit, and is further from it
    with fewer points."""
    s = tiny_system(kind, grids=((12, 12, 12), (24, 24, 24)), n_occ=3)
    p = oplan.build_plan(s)
    Kt, _ = brute.exchange_tensor_route(p, s.D)
    s.n_mu_ratio = 60.0
    r = pipeline.run(s)
    assert np.max(np.abs(r.K - Kt)) <= 1e-8 * np.max(np.abs(Kt))
    s.n_mu_ratio = 2.0
    r2 = pipeline.run(s)
    assert np.max(np.abs(r2.K - Kt)) > 1e-6 * np.max(np.abs(Kt))


def test_pair_coverage_d_shells():
    """Every ordered pair with a non-negligible overlap is owned by exactly
    one domain mask, with d functions on both levels."""
    s = tiny_system("d_two")
    p = oplan.build_plan(s)
    cnt = np.zeros((p.n_basis, p.n_basis), dtype=int)
    for dom in p.domains:
        cnt += brute._pair_mask(dom, p.n_basis)
    S = periodic_overlap(s.lattice, s.xyz, s.shell_atom, s.shell_l, s.shell_alpha)
    assert cnt.max() <= 1 and np.all(cnt[np.abs(S) > 1e-7] == 1)


def test_large_configuration_counts():
    """The 384-atom configuration: 44 functions per atom (8 s, 7 p, 3 d),
    four levels with bounds 0.125 / 0.5 / 2, and per-level function counts
    9 / 9 / 13 / 13 per atom."""
    s = config(5, with_density=False)
    assert s.n_basis == 384 * 44
    assert np.allclose(s.alpha_bound, [0.125, 0.5, 2.0], rtol=1e-9)
    lev = np.searchsorted(s.alpha_bound, s.shell_alpha[:18], side="right")
    per = [int(np.sum((2 * s.shell_l[:18] + 1)[lev == k])) for k in range(4)]
    assert per == [9, 9, 13, 13]


# ------------------------------------------------------------ Adam (network)
def test_adam_first_two_steps_closed_form():
    """Two Adam steps with gradients g1, g2 from zero moments: the bias
    corrected moments are g1, g1^2 after step 1 and (b1 g1 + g2)/(1 + b1),
    (b2 g1^2 + g2^2)/(1 + b2) after step 2.  Catches a missing bias
    correction, b1/b2 swapped, or eps inside the square root."""
    rng = np.random.default_rng(8)
    th0 = rng.standard_normal(50)
    g1, g2 = rng.standard_normal(50), rng.standard_normal(50)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    m = v = np.zeros(50)
    th1, m, v = mlp.adam_step(th0, g1, m, v, 1, lr, b1, b2, eps)
    assert np.allclose(th1, th0 - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    th2, m, v = mlp.adam_step(th1, g2, m, v, 2, lr, b1, b2, eps)
    mh = (b1 * g1 + g2) / (1 + b1)
    vh = (b2 * g1 ** 2 + g2 ** 2) / (1 + b2)
    assert np.allclose(th2, th1 - lr * mh / (np.sqrt(vh) + eps), rtol=0, atol=1e-15)
    # constant gradient: every step moves by lr g / (|g| + eps)
    thc, mc, vc = th0, np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        prev = thc
        thc, mc, vc = mlp.adam_step(thc, g1, mc, vc, t, lr, b1, b2, eps)
        assert np.allclose(prev - thc, lr * g1 / (np.abs(g1) + eps), rtol=1e-12)


# -------------------------------------------------------- selector features
def _one_atom_plan():
    s = tiny_system("one_atom", grids=((12, 12, 12), (24, 24, 24)))
    s.xyz = np.array([[0.0, 0.0, 0.0]])
    return s, oplan.build_plan(s)


def test_features_all_sixteen_on_constructed_values():
    """Every feature on hand-built basis values and points whose answers
    follow from the definitions: two L columns and one N column at four
    points of the window of an atom at the origin (points: the atom's own
    grid point, one step along x, two steps along y, one step along z)."""
    s, p = _one_atom_plan()
    dom = dataclasses.replace(p.domains[1])
    n1 = 24
    dom.points = np.array([0, 1, 2 * n1, n1 * n1])
    nL = dom.L.size
    assert nL == 1  # one s shell (4.05) on the fine level of this cell
    # rebuild the domain with two L columns and one N column
    dom.L = np.array([0, 1])
    dom.N = np.array([2])
    dom.n_mu = 3
    Phi = np.array([[1.0, 0.0, 0.0],      # aL 1, aN 0, g 1,   mL 1, sL 1
                    [1.0, 1.0, 1.0],      # aL 2, aN 1, g 8,   mL 1, sL 2
                    [2.0, 0.0, 3.0],      # aL 4, aN 9, g 88,  mL 4, sL 2
                    [0.5, -0.5, 0.0]])    # aL .5, aN 0, g .25, mL .25, sL 0
    F = mlp.features(p, dom, Phi, s.eps_r, s.alpha_bound)
    g = np.array([1.0, 8.0, 88.0, 0.25])
    aL = np.array([1.0, 2.0, 4.0, 0.5])
    aN = np.array([0.0, 1.0, 9.0, 0.0])
    h = 6.0 / 24
    rs = np.sqrt(-np.log(s.eps_r) / s.alpha_bound[0])
    lg = lambda x: np.log10(np.maximum(x, 1e-300)) / 10  # noqa: E731
    assert np.allclose(F[:, 0], 1.0)                      # level 1 of levels 0..1
    assert np.allclose(F[:, 1], 0.0)                      # a window
    assert np.allclose(F[:, 2], lg(g))
    assert np.allclose(F[:, 3], g / 88.0)
    assert np.allclose(F[:, 4], lg(aL))
    assert np.allclose(F[:, 5], [-30.0, 0.0, lg(9.0), -30.0])
    assert np.allclose(F[:, 6], lg(aL + aN))
    assert np.allclose(F[:, 7], [1.0, 0.5, 1.0, 0.5])
    assert np.allclose(F[:, 8], np.array([0.0, h, 2 * h, h]) / rs)
    assert np.allclose(F[:, 9], F[:, 8])                  # the only atom is the nearest
    assert np.allclose(F[:, 10], F[:, 8])                 # one atom: second nearest = nearest
    assert np.allclose(F[:, 11], np.sqrt(g / 88.0))
    assert np.allclose(F[:, 12], 10.0 * 3 / 4)
    assert np.allclose(F[:, 13], h / rs)
    assert np.allclose(F[:, 14], [0.5, 1.0, 0.5, 0.0])    # sL^2 / (|L| aL)
    assert np.allclose(F[:, 15], lg(g / g.mean()))


def test_features_universal_domain_and_second_atom():
    """Universal-domain flags and scale radius (the next level's window
    radius), and the nearest / second-nearest distances with two atoms."""
    s = tiny_system("two_atom", grids=((12, 12, 12), (24, 24, 24)))
    s.xyz = np.array([[0.0, 0.0, 0.0], [3.0, 0.0, 0.0]])
    p = oplan.build_plan(s)
    dom = p.domains[0]
    Phi = basis.domain_values(p, dom)
    F = mlp.features(p, dom, Phi, s.eps_r, s.alpha_bound)
    rs = np.sqrt(-np.log(s.eps_r) / s.alpha_bound[0])
    h0 = 6.0 / 12
    assert np.allclose(F[:, 0], 0.0) and np.allclose(F[:, 1], 1.0) and np.allclose(F[:, 8], 0.0)
    assert np.allclose(F[:, 13], h0 / rs)
    # grid point 2 sits at x = 1.0: nearest atom 1.0 away, second 2.0 away
    assert np.isclose(F[2, 9], 1.0 / rs) and np.isclose(F[2, 10], 2.0 / rs)
    # grid point 6 sits at x = 3.0 on the second atom
    assert np.isclose(F[6, 9], 0.0) and np.isclose(F[6, 10], 3.0 / rs)


# -------------------------------------------------------- window image screen
@pytest.mark.parametrize("which", ["cfg1", "d_two_strained"])
def test_window_screen_equals_unscreened(which):
    """Skipping image centres farther than r_img + r_max from the window
    centre leaves every basis value on the window points unchanged (catches
    a screen radius that drops a contributing image)."""
    if which == "cfg1":
        s = config(1, with_density=False)
        doms = (1, 5)
    else:
        s = tiny_system("d_two", grids=((12, 12, 12), (24, 24, 24)))
        s.lattice = s.lattice @ (np.eye(3) + np.array([[0.03, -0.01, 0.0], [-0.01, 0.0, 0.02],
                                                       [0.0, 0.02, -0.02]]))
        doms = (1, 2)
    p = oplan.build_plan(s)
    for d in doms:
        dom = p.domains[d]
        scr = basis.evaluate(p, dom.level, dom.points, dom.G, window_centre=p.xyz[dom.atom],
                             window_radius=dom.r_max)
        full = basis.evaluate(p, dom.level, dom.points, dom.G)
        assert np.array_equal(scr, full)


# ------------------------------------------------ Coulomb metric assembly
def _gauss_density(lattice, grid, P, p):
    pts = np.arange(int(np.prod(grid)))
    pos = oplan.grid_positions(lattice, grid, pts)
    n = np.arange(-3, 4)
    T = np.array(np.meshgrid(n, n, n, indexing="ij")).reshape(3, -1).T @ lattice
    d = pos[:, None, :] - (P + T)[None]
    return ((p / np.pi) ** 1.5 * np.exp(-p * np.sum(d * d, axis=2))).sum(1)


def _gauss_coulomb_closed(lattice, P1, p1, P2, p2, mmax=40):
    B = 2 * np.pi * np.linalg.inv(lattice).T
    m = np.arange(-mmax, mmax + 1)
    M = np.array(np.meshgrid(m, m, m, indexing="ij")).reshape(3, -1).T
    M = M[np.any(M != 0, axis=1)]
    G = M @ B
    g2 = np.sum(G * G, axis=1)
    vol = abs(np.linalg.det(lattice))
    return 4 * np.pi / vol * np.sum(np.exp(-g2 / (4 * p1) - g2 / (4 * p2)) * np.cos(G @ (P1 - P2)) / g2)


def test_coulomb_metric_assembly_across_levels():
    """Two Gaussian charges placed as fitting functions on a coarse full-grid
    domain and again on a fine windowed domain: every block of the assembled
    W (same level, coarse x fine, fine x coarse after mirroring, and the
    averaged same-level block) equals the closed-form periodic Coulomb
    integral of the two charges.  Catches a block placed at the wrong
    offsets, a mirror without transpose, or a missing average."""
    lat = np.diag([10.0, 10.6, 9.8]) @ (np.eye(3) + np.array([[0, 0.02, 0.01], [0.02, 0, 0], [0.01, 0, 0]]))
    gc, gf = (32, 36, 32), (64, 72, 64)
    P = [np.array([2.1, 3.3, 1.7]), np.array([5.0, 2.4, 4.9])]
    pe = [0.9, 1.4]
    ref = np.array([[_gauss_coulomb_closed(lat, P[i], pe[i], P[j], pe[j]) for j in range(2)]
                    for i in range(2)])

    class _Dom:
        def __init__(self, level, points):
            self.level, self.points = level, points

    class _Plan:
        pass

    pl = _Plan()
    pl.lattice = lat
    pl.grids = np.array([gc, gf])
    vol = abs(np.linalg.det(lat))
    pl.level_spacing_volume = lambda lev: vol / float(np.prod(pl.grids[lev]))
    coarse = np.stack([_gauss_density(lat, gc, P[i], pe[i]) for i in range(2)], axis=1)
    fine_all = np.stack([_gauss_density(lat, gf, P[i], pe[i]) for i in range(2)], axis=1)
    # fine domain: the points where either charge is above 1e-15 of its peak
    keep = np.nonzero(np.max(fine_all / fine_all.max(axis=0), axis=1) > 1e-15)[0]
    assert keep.size < fine_all.shape[0]
    pl.domains = [_Dom(0, np.arange(coarse.shape[0])), _Dom(1, keep)]
    W = coulomb.coulomb_metric(pl, [coarse, fine_all[keep]])
    want = np.block([[ref, ref], [ref, ref]])
    assert np.allclose(W, want, rtol=1e-9, atol=1e-10 * np.abs(ref).max())
    assert np.array_equal(W, W.T)


# -------------------------------------------------- full-cell domain mode
def test_domain_mode_full_cell_plan_and_exact_limit():
    """domain_mode = 1: one domain per level over the whole grid, L = the
    level's functions, N = all coarser ones; every ordered pair is owned
    exactly once, and at the rank limit the ISDF exchange equals the exact
    exchange of that plan."""
    s = tiny_system("d_two", grids=((10, 10, 10), (20, 20, 20)), n_occ=3)
    s.domain_mode = 1
    p = oplan.build_plan(s)
    assert len(p.domains) == 2
    assert all(d.atom == -1 and d.points.size == np.prod(s.grids[d.level]) for d in p.domains)
    assert np.array_equal(np.sort(np.concatenate([d.L for d in p.domains])), np.arange(p.n_basis))
    assert np.array_equal(p.domains[1].N, p.domains[0].L)
    cnt = np.zeros((p.n_basis, p.n_basis), dtype=int)
    for dom in p.domains:
        cnt += brute._pair_mask(dom, p.n_basis)
    assert np.all(cnt == 1)
    Kt, _ = brute.exchange_tensor_route(p, s.D)
    s.n_mu_ratio = 80.0
    r = pipeline.run(s)
    assert np.max(np.abs(r.K - Kt)) <= 1e-8 * np.max(np.abs(Kt))


# ------------------------------------------- every domain point requested
def test_all_points_domain_is_identity_fit():
    """A domain asked for at least as many points as it has takes all of
    them in ascending order with F = I (the paper's all-points universal
    grid).  The fitted pair densities are then exact on the grid, so with
    enough window points the ISDF exchange equals the brute-force one."""
    s = tiny_system("d_atom", grids=((6, 6, 6), (24, 24, 24)), n_occ=3)
    s.n_mu_ratio = 400.0
    p = oplan.build_plan(s)
    assert p.domains[0].n_mu == p.domains[0].points.size == 216
    r = pipeline.run(s)
    assert np.array_equal(r.pivots[0], np.arange(216))
    assert np.array_equal(r.F[0], np.eye(216))
    Kt, _ = brute.exchange_tensor_route(p, s.D)
    assert np.max(np.abs(r.K - Kt)) <= 1e-8 * np.max(np.abs(Kt))


def test_threshold_mode_cap_still_selects():
    """In the threshold-only mode (ratio <= 0) the cap n_mu_d = points is an
    upper limit, not a request for every point: the capped universal domain
    of this cell is still selected greedily, its first pivot the tie-rule
    argmax of the Gram diagonal, not the first grid point."""
    s = tiny_system("d_two", grids=((4, 4, 4), (24, 24, 24)), n_occ=3)
    s.n_mu_ratio = 0.0
    s.eps_isdf = 1e-6
    p = oplan.build_plan(s)
    dom = p.domains[0]
    assert dom.n_mu == dom.points.size == 64 and dom.N.size == 0
    r = pipeline.run(s)
    Phi = basis.domain_values(p, dom)
    dg = np.sum(Phi ** 2, axis=1) ** 2  # a_L (a_L + 2 a_N) with N empty
    first = int(np.min(np.nonzero(dg >= (1.0 - s.tie_tol) * dg.max())[0]))
    assert r.pivots[0][0] == first != 0
    assert not np.array_equal(r.pivots[0], np.arange(r.pivots[0].size))


# ------------------------------------------- density screening (occ-RI)
@pytest.fixture(scope="module")
def cfg1_bonds():
    from workloads import bond_orbitals

    s = config(1)
    C, D, bonds = bond_orbitals(s)
    s.C_occ, s.D = C, D
    return s, pipeline.run(s)


def test_bond_orbitals_are_orthonormal_and_local():
    """One bond orbital per bond (two per carbon), S-orthonormal, and most of
    its weight on the two bonded atoms."""
    from workloads import bond_orbitals

    s = config(1, with_density=False)
    C, D, bonds = bond_orbitals(s)
    assert len(bonds) == 2 * s.n_atoms == C.shape[1]
    S = periodic_overlap(s.lattice, s.xyz, s.shell_atom, s.shell_l, s.shell_alpha)
    assert np.max(np.abs(C.T @ S @ C - np.eye(C.shape[1]))) <= 1e-12
    fatom = np.repeat(s.shell_atom, 2 * s.shell_l + 1)
    for k, (a, b) in enumerate(bonds):
        w = C[:, k] * (S @ C[:, k])  # Mulliken weights, sum 1
        assert abs(w.sum() - 1.0) <= 1e-12
        assert w[(fatom == a) | (fatom == b)].sum() >= 0.6


def test_screened_occ_ri_without_screening_is_occ_ri(cfg1_bonds):
    s, r = cfg1_bonds
    KC, bound, kept = exchange.exchange_occ_ri_screened(r.XL, r.XN, r.W, s.C_occ, 64, 0.0)
    assert kept == 1.0 and np.max(bound) == 0.0
    ref = exchange.exchange_occ_ri(r.XL, r.XN, r.W, s.C_occ)
    assert np.max(np.abs(KC - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_screened_occ_ri_within_its_bound(cfg1_bonds):
    """Tile bounds cover every |Q| entry; leaving out the tiles below tau
    moves K C by no more than the stated elementwise bound; and the screened
    K C is K_s C for the dense four-term K_s built from the same masked Q
    blocks, which is symmetric only when Q_LG leaves out exactly the
    transposed tiles of Q_GL."""
    s, r = cfg1_bonds
    C, XL, XN, W = s.C_occ, r.XL, r.XN, r.W
    block = 64
    BGG, BGL, BLL = exchange.occ_ri_tile_bounds(XL, XN, W, C, block)
    EG, EL = (XL + XN) @ C, XL @ C
    m = W.shape[0]
    tiles = np.arange(m) // block
    for B, Q in ((BGG, (EG @ EG.T) * W), (BGL, (EG @ EL.T) * W), (BLL, (EL @ EL.T) * W)):
        assert np.all(np.abs(Q) <= B[np.ix_(tiles, tiles)] * (1 + 1e-12))
    tau = float(np.quantile(np.concatenate([BGG.ravel(), BGL.ravel(), BLL.ravel()]), 0.4))
    KC, bound, kept = exchange.exchange_occ_ri_screened(XL, XN, W, C, block, tau)
    assert 0.3 < kept < 0.9
    full = exchange.exchange_occ_ri(XL, XN, W, C)
    dKC = np.abs(KC - full)
    assert np.max(dKC) > 0.0
    assert np.all(dKC <= bound + 1e-12 * np.max(np.abs(full)))
    # the dense form of the same screened blocks
    keep = lambda B: np.repeat(np.repeat(B >= tau, block, 0), block, 1)[:m, :m]
    EN = XN @ C
    QGG = (EG @ EG.T) * W * keep(BGG)
    QGL = (EG @ EL.T) * W * keep(BGL)
    QLG = (EL @ EG.T) * W * keep(BGL).T
    QLL = (EL @ EL.T) * W * keep(BLL)
    Ks = -(XL.T @ QGG @ XL + XL.T @ QGL @ XN + XN.T @ QLG @ XL + XN.T @ QLL @ XN)
    assert np.max(np.abs(Ks - Ks.T)) <= 1e-12 * np.max(np.abs(Ks))
    assert np.max(np.abs(Ks @ C - KC)) <= 1e-12 * np.max(np.abs(KC))
