"""Exact exchange without ISDF, for small cells.

Every ordered pair (mu, nu) is owned by exactly one domain (its L G + N L
mask); its density mu(R) nu(R) is kept on that domain's points and zero
elsewhere, and pair densities are coupled with the same Coulomb form as the
fitting functions.  This is the quantity the ISDF factorisation
approximates, so the ISDF exchange must approach it as the number of
interpolation points reaches the number of domain points.

Two independent routes:
* tensor:   K_mu,sig = - sum_{nu lam} D_nu,lam (mu nu | lam sig) from the
            full pair-density Coulomb matrix;
* orbitals: with D = C C^T, K_mu,sig = - sum_i (rho^i_mu | rho^i_sig) where
            rho^i_mu = sum_nu mu nu C_nu,i over the pairs each domain owns
            (n_occ N Poisson solves, the occupied-orbital route of the
            Interpolative decomposition section).
"""
from __future__ import annotations

import numpy as np

from . import basis
from .coulomb import pair_coulomb


def _pair_mask(dom, N):
    """Boolean [N, N] mask of ordered pairs owned by the domain."""
    inL = np.zeros(N, dtype=bool)
    inN = np.zeros(N, dtype=bool)
    inL[dom.L] = True
    inN[dom.N] = True
    inG = inL | inN
    return (inL[:, None] & inG[None, :]) | (inN[:, None] & inL[None, :])


def exchange_tensor_route(plan, D: np.ndarray):
    N = plan.n_basis
    dens = []
    owners = []  # (domain, mu, nu)
    for d, dom in enumerate(plan.domains):
        Phi = basis.domain_values(plan, dom)
        G = dom.G
        mask = _pair_mask(dom, N)
        cols = []
        for a, mu in enumerate(G):
            for b, nu in enumerate(G):
                if mask[mu, nu]:
                    cols.append(Phi[:, a] * Phi[:, b])
                    owners.append((mu, nu))
        if cols:
            dens.append((dom.level, dom.points, np.stack(cols, axis=1)))
    C = pair_coulomb(plan, dens, None)
    owners = np.array(owners)
    # (mu nu | lam sig) = C[p, q]; K_mu,sig = - sum D_nu,lam C[(mu,nu),(lam,sig)]
    K = np.zeros((N, N))
    mu, nu = owners[:, 0], owners[:, 1]
    # Dq[p, q] = D[nu_p, lam_q]
    Dw = D[nu[:, None], mu[None, :]]  # lam_q = first index of pair q
    contrib = C * Dw  # [p, q]
    # accumulate into K[mu_p, sig_q]
    np.add.at(K, (mu[:, None].repeat(len(nu), 1), nu[None, :].repeat(len(mu), 0)), -contrib)
    # coverage check: every pair with a non-negligible product is owned once
    return K, owners


def exchange_orbital_route(plan, C_occ: np.ndarray):
    N = plan.n_basis
    nocc = C_occ.shape[1]
    dens = []
    for d, dom in enumerate(plan.domains):
        Phi = basis.domain_values(plan, dom)
        G = dom.G
        mask = _pair_mask(dom, N)
        # rho^i_mu(R) = sum_nu [mask mu,nu] mu(R) nu(R) C_nu,i  for mu in G
        sub = mask[np.ix_(G, G)].astype(float)  # [a, b]
        Csub = C_occ[G, :]  # [b, i]
        # psi[R, a, i] = sum_b sub[a,b] Phi[R,b] C[b,i]
        t = np.einsum("ab,Rb,bi->Rai", sub, Phi, Csub)
        vals = Phi[:, :, None] * t  # [R, a, i]
        # columns ordered (i, mu)
        full = np.zeros((Phi.shape[0], nocc, N))
        full[:, :, G] = vals.transpose(0, 2, 1)
        dens.append((dom.level, dom.points, full.reshape(Phi.shape[0], nocc * N)))
    Cm = pair_coulomb(plan, dens, None)
    nd = len(dens)
    K = np.zeros((N, N))
    blk = nocc * N
    for d in range(nd):
        for e in range(nd):
            B = Cm[d * blk:(d + 1) * blk, e * blk:(e + 1) * blk].reshape(nocc, N, nocc, N)
            K -= np.einsum("iaib->ab", B)
    return K
