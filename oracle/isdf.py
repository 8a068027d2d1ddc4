"""Local ISDF on one domain: pair Gram, pivoted-Cholesky points, fitting
functions.

Pair densities (mu nu | R) = mu(R) nu(R) are fitted on the domain whose
masks own the pair: ordered pairs L x G plus N x L (Eq. "mg product
density" and the four-term Eq. ints).  With A_X(R, R') = sum_{mu in X}
mu(R) mu(R'), the Gram of Eq. M(R,R) over exactly those ordered pairs is

    M(R, R') = A_L (A_L + 2 A_N)        (elementwise),

because L x G = L x L + L x N and the N x L half doubles the cross term.

Points are chosen by greedy pivoted Cholesky on M without randomisation
(Interpolative decomposition section; the paper notes it gives the pivots of
pivoted QR on (mu nu | R)).  Fitting functions solve the least-squares
problem of Eq. lsqr through its normal equations: F = Theta M_xi^{-1} with
Theta = M(P_d, xi) and M_xi = M(xi, xi).

Readings:
* tie rule: the pivot is the smallest point index among candidates whose
  residual diagonal is within a relative window tie_tol of the maximum;
* stop when the chosen residual is <= eps_isdf times the largest initial
  diagonal, or when n_mu points are chosen;
* residual diagonals are clamped at zero and chosen points never re-enter.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def gram_diag(Phi: np.ndarray, nL: int) -> np.ndarray:
    aL = np.sum(Phi[:, :nL] ** 2, axis=1)
    aN = np.sum(Phi[:, nL:] ** 2, axis=1)
    return aL * (aL + 2.0 * aN)


def gram_columns(Phi: np.ndarray, nL: int, cols) -> np.ndarray:
    """M(:, cols) = A_L (A_L + 2 A_N) for the given point rows `cols`."""
    AL = Phi[:, :nL] @ Phi[cols, :nL].T
    AN = Phi[:, nL:] @ Phi[cols, nL:].T
    return AL * (AL + 2.0 * AN)


def pick_pivot(d: np.ndarray, active: np.ndarray, tie_tol: float) -> int:
    """Smallest index among active points with d >= (1 - tie_tol) max d."""
    vals = np.where(active, d, -np.inf)
    mx = np.max(vals)
    return int(np.nonzero(vals >= (1.0 - tie_tol) * mx)[0][0])


def pivoted_cholesky(Phi: np.ndarray, nL: int, n_max: int, eps: float, tie_tol: float,
                     candidates=None):
    """Greedy pivoted Cholesky of M = A_L (A_L + 2 A_N).

    Returns (pivots as row indices of Phi, Lfac [n_rows x k], residual
    diagonal after the last step, initial diagonal).
    Only rows in `candidates` (all rows if None) may become pivots; the
    factor columns are still formed over all rows.
    """
    n = Phi.shape[0]
    d = gram_diag(Phi, nL)
    d0 = d.copy()
    active = np.zeros(n, dtype=bool)
    if candidates is None:
        active[:] = True
    else:
        active[np.asarray(candidates)] = True
    dmax0 = float(np.max(np.where(active, d0, 0.0))) if n else 0.0
    n_max = min(n_max, int(active.sum()))
    Lfac = np.zeros((n, n_max))
    piv = []
    for k in range(n_max):
        p = pick_pivot(d, active, tie_tol)
        if d[p] <= eps * dmax0:
            break
        col = gram_columns(Phi, nL, [p])[:, 0] - Lfac[:, :k] @ Lfac[p, :k]
        Lfac[:, k] = col / np.sqrt(d[p])
        d = np.maximum(d - Lfac[:, k] ** 2, 0.0)
        active[p] = False
        piv.append(p)
    k = len(piv)
    return np.array(piv, dtype=np.int64), Lfac[:, :k], d, d0


def fit_functions(Phi: np.ndarray, nL: int, piv: np.ndarray):
    """Theta = M(:, piv), M_xi = M(piv, piv), F = Theta M_xi^{-1} (Eq. lsqr)."""
    Theta = gram_columns(Phi, nL, piv)
    Mxi = Theta[piv, :]
    cf = sla.cho_factor(Mxi, lower=True)
    F = sla.cho_solve(cf, Theta.T).T
    return F, Theta, Mxi


def needed_points(d0: np.ndarray, d_last: float, tie_tol: float) -> np.ndarray:
    """Points a candidate set must contain for the restricted greedy selection
    to reproduce the full one: residual diagonals never grow, so a point whose
    initial diagonal is below (1 - tie_tol) d_last can never reach the tie
    window of any step whose pivot residual is at least d_last."""
    return np.nonzero(d0 >= (1.0 - tie_tol) * d_last)[0]


def restriction_is_exact(d0: np.ndarray, candidates, d_last: float, tie_tol: float) -> bool:
    mask = np.ones(d0.size, dtype=bool)
    mask[np.asarray(candidates)] = False
    excl = d0[mask]
    return bool(excl.size == 0 or excl.max() < (1.0 - tie_tol) * d_last)
