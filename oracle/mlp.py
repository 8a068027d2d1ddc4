"""FP64 reference of the point-scoring network that prunes candidates before
pivoted Cholesky (not part of the paper's method; it only decides which
grid points may become pivots, and the greedy selection of the
Interpolative decomposition section then runs over those candidates).

Features (16 per grid point R of domain d, all local and size-independent):
  aL = sum_{mu in L} mu(R)^2, aN = sum_{mu in N} mu(R)^2,
  g = aL (aL + 2 aN) (the Gram diagonal), mL = max_{mu in L} mu(R)^2,
  sL = sum_{mu in L} mu(R), gmax / gmean = max / mean of g over the domain,
  r_s = the domain's window radius (universal domain: the radius a window
  of the next level would have, else 10 h_0), h = the level's spacing.
   0 level / max(n_levels - 1, 1)        8 |r - A_d| / r_s (0 for the universal domain)
   1 1 for the universal domain          9 nearest-atom distance / r_s
   2 log10(g) / 10                      10 second-nearest-atom distance / r_s
   3 g / gmax                           11 sqrt(g / gmax)
   4 log10(aL) / 10                     12 10 n_mu,d / pts_d
   5 log10(aN) / 10                     13 h / r_s
   6 log10(aL + aN) / 10                14 sL^2 / (|L| aL)
   7 mL / aL                            15 log10(g / gmean) / 10
  (log10 of x uses max(x, 1e-300)).

Network: 16 -> 64 -> 64 -> 1, ReLU, ReLU, sigmoid; parameters packed as
W1[64][16], b1[64], W2[64][64], b2[64], w3[64], b3 (5313 values).
Loss: mean weighted binary cross-entropy,
  l = -(pw y log p + (1 - y) log(1 - p)), p = sigmoid(z),
so dl/dz = pw y (p - 1) + (1 - y) p.
Optimiser: Adam (Kingma and Ba) with bias-corrected moments,
  m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
  theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

from . import basis as obasis
from .plan import grid_positions

NF, NH = 16, 64
OFF_W1, OFF_B1 = 0, NH * NF
OFF_W2 = OFF_B1 + NH
OFF_B2 = OFF_W2 + NH * NH
OFF_W3 = OFF_B2 + NH
OFF_B3 = OFF_W3 + NH
NPARAM = OFF_B3 + 1


def unpack(theta):
    W1 = theta[OFF_W1:OFF_B1].reshape(NH, NF)
    b1 = theta[OFF_B1:OFF_W2]
    W2 = theta[OFF_W2:OFF_B2].reshape(NH, NH)
    b2 = theta[OFF_B2:OFF_W3]
    w3 = theta[OFF_W3:OFF_B3]
    b3 = theta[OFF_B3]
    return W1, b1, W2, b2, w3, b3


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases: the seeded initial weights of the
    shared input generators (``workloads.selector_init``)."""
    from workloads.selector_init import initial_weights

    th = initial_weights(seed)
    assert th.size == NPARAM
    return th


def forward(theta, X):
    W1, b1, W2, b2, w3, b3 = unpack(np.asarray(theta, dtype=np.float64))
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    return z, (a1, h1, a2, h2)


def loss_grad(theta, X, y, pw):
    """Mean weighted BCE and its gradient (analytic backward)."""
    theta = np.asarray(theta, dtype=np.float64)
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    n = X.shape[0]
    z, (a1, h1, a2, h2) = forward(theta, X)
    # log p = -softplus(-z), log(1-p) = -softplus(z)
    sp_neg = np.logaddexp(0.0, -z)
    sp_pos = np.logaddexp(0.0, z)
    loss = float(np.mean(pw * y * sp_neg + (1.0 - y) * sp_pos))
    p = 1.0 / (1.0 + np.exp(-z))
    dz = (pw * y * (p - 1.0) + (1.0 - y) * p) / n
    g = np.zeros(NPARAM)
    g[OFF_W3:OFF_B3] = h2.T @ dz
    g[OFF_B3] = dz.sum()
    dh2 = np.outer(dz, w3) * (a2 > 0)
    g[OFF_W2:OFF_B2] = (dh2.T @ h1).ravel()
    g[OFF_B2:OFF_W3] = dh2.sum(0)
    dh1 = (dh2 @ W2) * (a1 > 0)
    g[OFF_W1:OFF_B1] = (dh1.T @ X).ravel()
    g[OFF_B1:OFF_W2] = dh1.sum(0)
    return loss, g


def _min_image(lattice, pos, centre):
    """|pos - centre| under the minimum image over the 27 neighbour cells."""
    inv = np.linalg.inv(lattice)
    f = (pos - centre) @ inv
    f -= np.round(f)
    best = np.full(pos.shape[0], np.inf)
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                c = (f + np.array([i, j, k])) @ lattice
                best = np.minimum(best, np.sqrt(np.sum(c * c, axis=1)))
    return best


def scale_radius(plan, dom, eps_r: float, alpha_bound) -> float:
    if dom.atom >= 0:
        return float(dom.r_max)
    if len(alpha_bound) > 0:
        return float(np.sqrt(-np.log(eps_r) / alpha_bound[0]))
    h0 = max(np.linalg.norm(plan.lattice[i]) / plan.grids[0][i] for i in range(3))
    return 10.0 * h0


def features(plan, dom, Phi, eps_r: float, alpha_bound) -> np.ndarray:
    nL = dom.L.size
    aL = np.sum(Phi[:, :nL] ** 2, axis=1)
    aN = np.sum(Phi[:, nL:] ** 2, axis=1)
    mL = np.max(Phi[:, :nL] ** 2, axis=1)
    sL = np.sum(Phi[:, :nL], axis=1)
    g = aL * (aL + 2.0 * aN)
    gmax = g.max()
    gmean = g.mean()
    lev = dom.level
    nlev = plan.grids.shape[0]
    h = max(np.linalg.norm(plan.lattice[i]) / plan.grids[lev][i] for i in range(3))
    rs = scale_radius(plan, dom, eps_r, alpha_bound)
    pos = grid_positions(plan.lattice, plan.grids[lev], dom.points)
    dists = np.stack([_min_image(plan.lattice, pos, plan.xyz[a]) for a in range(plan.xyz.shape[0])], axis=1)
    dists.sort(axis=1)
    d1 = dists[:, 0]
    d2 = dists[:, 1] if dists.shape[1] > 1 else dists[:, 0]
    own = _min_image(plan.lattice, pos, plan.xyz[dom.atom]) if dom.atom >= 0 else np.zeros(pos.shape[0])
    lg = lambda x: np.log10(np.maximum(x, 1e-300)) / 10.0  # noqa: E731
    F = np.zeros((Phi.shape[0], NF))
    F[:, 0] = lev / max(nlev - 1, 1)
    F[:, 1] = 1.0 if dom.atom < 0 else 0.0
    F[:, 2] = lg(g)
    F[:, 3] = g / gmax
    F[:, 4] = lg(aL)
    F[:, 5] = lg(aN)
    F[:, 6] = lg(aL + aN)
    F[:, 7] = mL / np.maximum(aL, 1e-300)
    F[:, 8] = own / rs
    F[:, 9] = d1 / rs
    F[:, 10] = d2 / rs
    F[:, 11] = np.sqrt(g / gmax)
    F[:, 12] = 10.0 * dom.n_mu / dom.points.size
    F[:, 13] = h / rs
    F[:, 14] = sL ** 2 / np.maximum(nL * aL, 1e-300)
    F[:, 15] = lg(g / gmean)
    return F


def domain_features(plan, dom, sysm):
    Phi = obasis.domain_values(plan, dom)
    return features(plan, dom, Phi, sysm.eps_r, sysm.alpha_bound), Phi


def top_candidates(scores: np.ndarray, k: int) -> np.ndarray:
    """The k highest scores (ties: smaller index first), ascending indices."""
    k = min(k, scores.size)
    order = np.lexsort((np.arange(scores.size), -scores))
    return np.sort(order[:k])


def adam_step(theta, g, m, v, t: int, lr: float, b1: float, b2: float, eps: float):
    """One Adam update at step t (1-based); returns (theta, m, v), all new
    arrays (FP64)."""
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return np.asarray(theta, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v
