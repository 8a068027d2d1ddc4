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


def occ_ri_tile_bounds(XL: np.ndarray, XN: np.ndarray, W: np.ndarray, C: np.ndarray, block: int):
    """Bounds on the tiles of the occ-RI Q products for density screening
    (the near-sightedness of the density matrix, Conclusions).

    Fitting indices are cut into tiles of `block` consecutive indices.  For
    tile b of rows and c of columns and S, T in {G, L}:

      |Q_ST(mu, nu)| = |W(mu, nu)| |sum_i E_S(mu, i) E_T(nu, i)|
                    <= max_{b x c} |W| sum_i NS(b, i) NT(c, i) = B_ST(b, c),

    NS(b, i) = max_{mu in b} |E_S(mu, i)|, E_S = X_S C.  With localised
    orbitals i, E_S(mu, i) is small unless the point mu is near orbital i,
    so B_ST is small for tiles of points far apart.  Returns
    (B_GG, B_GL, B_LL) of shape (n_tiles, n_tiles)."""
    m = W.shape[0]
    nt = (m + block - 1) // block
    EG, EL = (XL + XN) @ C, XL @ C

    def tile_max(A):
        out = np.zeros((nt, A.shape[1]))
        for b in range(nt):
            out[b] = np.max(np.abs(A[b * block:(b + 1) * block]), axis=0)
        return out

    Wt = np.zeros((nt, nt))
    for b in range(nt):
        for c in range(nt):
            Wt[b, c] = np.max(np.abs(W[b * block:(b + 1) * block, c * block:(c + 1) * block]))
    NG, NL = tile_max(EG), tile_max(EL)
    return Wt * (NG @ NG.T), Wt * (NG @ NL.T), Wt * (NL @ NL.T)


def exchange_occ_ri_screened(XL: np.ndarray, XN: np.ndarray, W: np.ndarray, C: np.ndarray, block: int,
                             tau: float):
    """K C of exchange_occ_ri with every Q tile whose bound (occ_ri_tile_bounds)
    is below tau left out (set to zero), and an elementwise bound on the
    change of K C.  Q_LG = Q_GL^T leaves out the transposed tiles of Q_GL.

    With dZ1 = the left-out part of Q_GG E_L + Q_GL E_N and dZ2 that of
    Q_LG E_L + Q_LL E_N, and P_c the indices of tile c,

      |dZ1(mu, i)| <= sum_{c out} B_GG(b, c) sum_{nu in P_c} |E_L(nu, i)|
                    + sum_{c out} B_GL(b, c) sum_{nu in P_c} |E_N(nu, i)|

    (b the tile of mu; likewise dZ2 with B_GL^T and B_LL), and
    |d(K C)(a, i)| <= sum_mu |X_L(mu, a)| |dZ1(mu, i)| + |X_N(mu, a)| |dZ2(mu, i)|.
    Returns (K C, bound, kept fraction of the tiles of the three products)."""
    m = W.shape[0]
    nt = (m + block - 1) // block
    BGG, BGL, BLL = occ_ri_tile_bounds(XL, XN, W, C, block)
    keep = {"GG": BGG >= tau, "GL": BGL >= tau, "LL": BLL >= tau}
    keep["LG"] = keep["GL"].T

    def expand(mask):  # tile mask -> element mask (m x m)
        e = np.repeat(np.repeat(mask, block, axis=0), block, axis=1)
        return e[:m, :m]

    XG = XL + XN
    EG, EL, EN = XG @ C, XL @ C, XN @ C
    Q = {"GG": (EG @ EG.T) * W, "GL": (EG @ EL.T) * W, "LG": (EL @ EG.T) * W, "LL": (EL @ EL.T) * W}
    for k in Q:
        Q[k] = Q[k] * expand(keep[k])
    Z1 = Q["GG"] @ EL + Q["GL"] @ EN
    Z2 = Q["LG"] @ EL + Q["LL"] @ EN
    KC = -(XL.T @ Z1 + XN.T @ Z2)

    def colsum(A):  # per tile c, sum over its rows of |A|
        out = np.zeros((nt, A.shape[1]))
        for c in range(nt):
            out[c] = np.sum(np.abs(A[c * block:(c + 1) * block]), axis=0)
        return out

    SL, SN = colsum(EL), colsum(EN)
    out = {k: np.where(keep[k], 0.0, v) for k, v in (("GG", BGG), ("GL", BGL), ("LG", BGL.T), ("LL", BLL))}
    dZ1t = out["GG"] @ SL + out["GL"] @ SN  # per row tile b
    dZ2t = out["LG"] @ SL + out["LL"] @ SN
    rows = np.minimum(np.arange(m) // block, nt - 1)
    dZ1, dZ2 = dZ1t[rows], dZ2t[rows]
    bound = np.abs(XL).T @ dZ1 + np.abs(XN).T @ dZ2
    kept = float(np.mean(np.concatenate([keep["GG"].ravel(), keep["GL"].ravel(), keep["LL"].ravel()])))
    return KC, bound, kept
