"""Periodic Gaussian basis values on level grids.

mu(r) = sum_T N_l(a) Y_l(r - A - T) exp(-a |r - A - T|^2) with
N_s = (2a/pi)^(3/4), N_p = N_s 2 sqrt(a), N_d = N_s 4a/sqrt(3), Y_p =
(x, y, z) and Y_d the five real solid harmonics in the order m = -2..2:
sqrt3 xy, sqrt3 yz, z^2 - (x^2 + y^2)/2, sqrt3 xz, sqrt3/2 (x^2 - y^2)
(each with integral of Y^2 over the unit sphere 4 pi/5, so one N_d
normalises all five).  The paper evaluates atomic orbitals directly on the
real-space grids (Results, first paragraph); its basis sets are
uncontracted Gaussians with d functions (same paragraph).  Image terms with
a |r - A - T|^2 > ln(1/tau) are dropped.
"""
from __future__ import annotations

import numpy as np

from .plan import Plan, grid_positions


def shell_norm(l: int, a: float) -> float:
    n = (2.0 * a / np.pi) ** 0.75
    if l == 1:
        return n * 2.0 * np.sqrt(a)
    if l == 2:
        return n * 4.0 * a / np.sqrt(3.0)
    return n


def solid_harmonic(l: int, comp: int, d: np.ndarray) -> np.ndarray:
    """Angular factor Y_l,comp(d) of displacements d[..., 3]; comp is the
    Cartesian axis for p and the index of m = -2..2 for d."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    if l == 0:
        return np.ones_like(x)
    if l == 1:
        return d[..., comp]
    r3 = np.sqrt(3.0)
    return (r3 * x * y, r3 * y * z, z * z - 0.5 * (x * x + y * y), r3 * x * z,
            0.5 * r3 * (x * x - y * y))[comp]


def min_image_dist_many(lattice: np.ndarray, X: np.ndarray, y: np.ndarray) -> np.ndarray:
    """min over the 27 neighbour translations of the reduced difference
    |X_i - y - T| (exact for cells whose Voronoi cell is spanned by the 26
    neighbour vectors, which holds for the near-orthogonal cells used)."""
    inv = np.linalg.inv(lattice)
    f = (X - y) @ inv
    f -= np.round(f)
    shifts = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)], float)
    cart = (f[:, None, :] + shifts[None]) @ lattice
    return np.min(np.linalg.norm(cart, axis=2), axis=1)


def evaluate(plan: Plan, level: int, points: np.ndarray, funcs: np.ndarray,
             window_centre=None, window_radius=None, chunk: int = 8192) -> np.ndarray:
    """Phi[R, c] = funcs[c](r_R) for flat points on grid `level`.

    Returns an array of shape (len(points), len(funcs)).  When the points form
    a window (centre, radius), image centres farther than r_img + radius from
    every image of the window centre are skipped: they cannot pass the
    pointwise cutoff anywhere on the window, so values are unchanged.
    """
    pos_all = grid_positions(plan.lattice, plan.grids[level], points)
    out = np.zeros((points.shape[0], len(funcs)))
    lnt = plan.ln_inv_tau
    col_of = {}
    for c, f in enumerate(funcs):
        col_of.setdefault(int(plan.f_shell[f]), []).append((c, int(plan.f_comp[f])))
    for s, cols in col_of.items():
        f0 = int(np.nonzero(plan.f_shell == s)[0][0])
        a = float(plan.f_alpha[f0])
        l = int(plan.f_l[f0])
        nrm = shell_norm(l, a)
        imgs = plan.shell_images[s]
        if window_centre is not None and imgs.shape[0]:
            r_img = np.sqrt(lnt / a)
            dmin = min_image_dist_many(plan.lattice, imgs, window_centre)
            imgs = imgs[dmin <= r_img + window_radius + 1e-9]
        if imgs.shape[0] == 0:
            continue
        for p0 in range(0, points.shape[0], chunk):
            pos = pos_all[p0:p0 + chunk]
            diff = pos[:, None, :] - imgs[None, :, :]  # [P, I, 3]
            r2 = np.einsum("pic,pic->pi", diff, diff)
            m = a * r2 <= lnt
            g = np.where(m, nrm * np.exp(-a * np.where(m, r2, 0.0)), 0.0)
            for (c, comp) in cols:
                if l == 0:
                    out[p0:p0 + chunk, c] = g.sum(axis=1)
                else:
                    out[p0:p0 + chunk, c] = np.einsum("pi,pi->p", g, solid_harmonic(l, comp, diff))
    return out


def domain_values(plan: Plan, dom) -> np.ndarray:
    """Phi_d with columns ordered [L | N]."""
    if dom.atom < 0:
        return evaluate(plan, dom.level, dom.points, dom.G)
    return evaluate(plan, dom.level, dom.points, dom.G,
                    window_centre=plan.xyz[dom.atom], window_radius=dom.r_max)
