"""Four-term multigrid THC exchange (Eq. ints, section "Building the exchange
matrix").

(mu nu|xi) = X^L_xi,mu X^G_xi,nu + X^N_xi,mu X^L_xi,nu with
X^S_xi,mu = mu(r_xi) [mu in S_d(xi)], and (mu nu|lam sig) = sum (mu nu|xi)
W_xi,xi' (lam sig|xi').  Contracting with the density,
K_mu,sig = - sum_{nu lam} D_nu,lam (mu nu|lam sig), gives

  K = -[ X^L' ((X^G D X^G') o W) X^L + X^L' ((X^G D X^L') o W) X^N
       + X^N' ((X^L D X^G') o W) X^L + X^N' ((X^L D X^L') o W) X^N ].

Readings: the two printed lines of Eq. ints are joined by "=" but the four
terms must be added (they are the expansion of the L G + N L pair mask on
both pair indices); the sign makes K negative definite as the paper states
for the exchange matrix, and E_x = tr(D K) with D per spin.
"""
from __future__ import annotations

import numpy as np


def build_X(plan, piv_list, Phi_rows_list):
    """X^L, X^N (N_mu x N) from the basis values at the pivots of each domain.

    Phi_rows_list[d] is Phi_d[piv_d, :] with columns ordered [L | N]."""
    nmu = sum(len(p) for p in piv_list)
    N = plan.n_basis
    XL = np.zeros((nmu, N))
    XN = np.zeros((nmu, N))
    r = 0
    for dom, piv, rows in zip(plan.domains, piv_list, Phi_rows_list):
        k = len(piv)
        nL = dom.L.size
        XL[r:r + k][:, dom.L] = rows[:, :nL]
        XN[r:r + k][:, dom.N] = rows[:, nL:]
        r += k
    return XL, XN


def exchange_matrix(XL: np.ndarray, XN: np.ndarray, W: np.ndarray, D: np.ndarray) -> np.ndarray:
    XG = XL + XN
    P_GG = XG @ D @ XG.T
    P_GL = XG @ D @ XL.T
    P_LG = XL @ D @ XG.T
    P_LL = XL @ D @ XL.T
    K = -(
        XL.T @ (P_GG * W) @ XL
        + XL.T @ (P_GL * W) @ XN
        + XN.T @ (P_LG * W) @ XL
        + XN.T @ (P_LL * W) @ XN
    )
    return K


def exchange_energy(D: np.ndarray, K: np.ndarray) -> float:
    return float(np.sum(D * K))


def exchange_occ_ri(XL: np.ndarray, XN: np.ndarray, W: np.ndarray, C: np.ndarray) -> np.ndarray:
    """K C for a factored density D = C C^T (occ-RI output, the occupied
    orbitals of the exchange section): the pair products X^S D X^T' become
    (X^S C)(X^T C)', and K is applied to C without forming it, so every
    product has an n_occ-wide side:

      K C = -[ X^L' (P_GG o W) E_L + X^L' (P_GL o W) E_N
             + X^N' (P_LG o W) E_L + X^N' (P_LL o W) E_N ],

    E_S = X^S C, P_ST = E_S E_T'.  E_x = tr(D K) = sum(C o (K C))."""
    XG = XL + XN
    EG, EL, EN = XG @ C, XL @ C, XN @ C
    P_GG = EG @ EG.T
    P_GL = EG @ EL.T
    P_LG = EL @ EG.T
    P_LL = EL @ EL.T
    return -(
        XL.T @ ((P_GG * W) @ EL)
        + XL.T @ ((P_GL * W) @ EN)
        + XN.T @ ((P_LG * W) @ EL)
        + XN.T @ ((P_LL * W) @ EN)
    )
