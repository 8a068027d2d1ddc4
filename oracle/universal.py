"""Universal grid with every point as a fitting function.

Sections "Building the exchange matrix" and the discussion of the two kinds
of fitting functions in the Results section: on the sparse universal grid
the fitting functions are the uniformly placed sinc functions, one per grid
point, so no interpolation points are chosen there (F = I), the Coulomb
operator between grid points, (R_U|R_U'), is circulant and is applied by
FFT instead of being stored, and the exchange of the pairs the universal
grid holds is formed from occupied pair densities each SCF iteration
(occ-RI).

With E = Phi_U C (Phi_U the values of the universal domain's functions on
all its points), the pairs owned by the universal domain give

    (K_UU C)(mu, i) = - dV sum_R phi_mu(R) sum_j E(R, j) V[E_j E_i](R),

where V[rho] is the potential of a grid density in the convention of
``coulomb.potential_on`` (band J_0 without G = 0) and dV the volume per
point.  Rows of functions outside the universal domain are zero.
TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from . import basis
from .coulomb import coulomb_kernel, potential_on, spectrum


def universal_domain(plan):
    dom = plan.domains[0]
    if dom.atom >= 0 or dom.level != 0:
        raise ValueError("the plan has no universal domain")
    return dom


def universal_exchange_occ_ri(plan, C_occ: np.ndarray, cols=None, workers: int = -1) -> np.ndarray:
    """K_UU C for the occupied columns `cols` (all if None): [N, len(cols)]."""
    dom = universal_domain(plan)
    grid = plan.grids[0]
    ng = int(np.prod(grid))
    Phi = basis.domain_values(plan, dom)  # [ng, |G_U|]
    E = Phi @ C_occ[dom.G]  # [ng, n_occ]
    v = coulomb_kernel(plan.lattice, grid)
    dV = plan.level_spacing_volume(0)
    cols = list(range(C_occ.shape[1])) if cols is None else list(cols)
    KC = np.zeros((plan.n_basis, len(cols)))
    for c, i in enumerate(cols):
        rho = E * E[:, [i]]  # rho_ij(R) = E(R, j) E(R, i), one column per j
        V = potential_on(spectrum(rho, grid, workers), grid, grid, v, workers)
        Z = np.sum(E * V, axis=1)  # sum over j
        KC[dom.G, c] = -dV * (Phi.T @ Z)
    assert ng == Phi.shape[0]
    return KC


def paper_exchange_occ_ri(sysm, C_occ: np.ndarray, plan=None, workers: int = -1):
    """K C of the method with the universal grid taken at every point: the
    universal domain's fitting functions are its grid points (F = I, X rows
    = Phi_U), the atom windows are fitted as usual (greedy pivoted Cholesky,
    Eq. lsqr), W = (xi|xi') over all of them (Eq. (xi|xi'), here formed
    densely, which is only affordable on small grids), and K C follows the
    occ-RI form of the four-term exchange (``exchange.exchange_occ_ri``).

    Returns (KC, window pivots per domain, with an empty entry for the
    universal domain)."""
    from . import isdf
    from .coulomb import coulomb_metric
    from .exchange import build_X, exchange_occ_ri
    from .plan import build_plan

    plan = plan if plan is not None else build_plan(sysm)
    universal_domain(plan)
    piv_list, F_list, rows_list, pivots = [], [], [], []
    for d, dom in enumerate(plan.domains):
        Phi = basis.domain_values(plan, dom)
        if d == 0:
            piv = np.arange(Phi.shape[0], dtype=np.int64)
            F = np.eye(Phi.shape[0])
            pivots.append(np.zeros(0, dtype=np.int64))
        else:
            piv, _, _, _ = isdf.pivoted_cholesky(Phi, dom.L.size, dom.n_mu, sysm.eps_isdf, sysm.tie_tol)
            F, _, _ = isdf.fit_functions(Phi, dom.L.size, piv)
            pivots.append(piv)
        piv_list.append(piv)
        F_list.append(F)
        rows_list.append(Phi[piv, :])
    XL, XN = build_X(plan, piv_list, rows_list)
    W = coulomb_metric(plan, F_list, workers)
    return exchange_occ_ri(XL, XN, W, C_occ), pivots
