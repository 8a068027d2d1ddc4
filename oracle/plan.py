"""Multigrid plan: basis functions, levels, periodic images and domains.

Follows the "Computational details" section of the paper:

* Basis functions are uncontracted Gaussians, split by exponent into grids
  of increasing resolution (sharp/diffuse split, generalised to L levels).
* The coarsest level is a universal grid spanning the cell; every finer
  level consists of atom-centred spherical windows of radius
  r_max = sqrt(-ln(eps_r) / alpha_min) (Eq. rcut), where alpha_min is the
  exponent bound separating that level from the coarser one.
* On the window of atom A the local set L holds the level functions centred
  on A, the global set G every function with a non-negligible value on the
  window, and N = G \\ L (Eq. "mg product density" and the text after it).

Readings (the paper is silent or ambiguous):

* Image rule: the image list of a shell (atom A, exponent a) is every lattice
  translation T with |A + T - c| <= r_img(a) + R_c, where r_img =
  sqrt(ln(1/tau)/a), c is the cell centre and R_c the cell circumradius; a
  term is dropped pointwise when a |r - A - T|^2 > ln(1/tau).
* A shell lives on the coarsest level l with alpha < alpha_bound[l].
* Window points: grid points within r_max of any image of A, in ascending
  flat index i1 + n1 (i2 + n2 i3); the whole grid when 2 r_max reaches the
  smallest perpendicular width of the cell.
* G of a window: its own level functions, every function of a coarser
  level, and the same-level functions of atoms with a larger index; a
  function is kept only if its atom lies within r_img(alpha) + r_max of the
  window centre (minimum image).  Giving a same-level pair of two different
  atoms only to the window of the lower atom index removes the double count
  that the literal L/G/N sets would give.
* domain_mode = 1 (the alternative kept in the C ABI): one domain per level
  over the whole level grid, L = the level's functions, N = every function
  of a coarser level; an ordered pair is then fitted on the level of its
  sharper function.
* Points per domain: N_mu,d = floor(r |L_d| + 1/2), capped at the domain's
  point count.  r <= 0 (threshold only, stop by eps_isdf): N_mu,d is the
  smaller of the point count and |L|(|L| + 1)/2 + |L||N|, the number of
  distinct pair products the domain fits, which bounds the rank of its pair
  Gram (Eq. M(R,R)), so the cap never ends a selection that the threshold
  would continue.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np


@dataclasses.dataclass
class Domain:
    level: int
    atom: int  # -1 for the universal domain
    points: np.ndarray  # int64 flat indices on the level grid, ascending
    L: np.ndarray  # global function indices of the local set
    N: np.ndarray  # global function indices of the non-local set
    n_mu: int  # requested interpolation points
    r_max: float  # window radius (inf for the universal domain)

    @property
    def G(self) -> np.ndarray:
        return np.concatenate([self.L, self.N])


@dataclasses.dataclass
class Plan:
    lattice: np.ndarray
    xyz: np.ndarray
    grids: np.ndarray
    # per function
    f_shell: np.ndarray
    f_atom: np.ndarray
    f_l: np.ndarray
    f_comp: np.ndarray  # -1 for s, 0/1/2 for p_x/p_y/p_z, 0..4 for d (m = -2..2)
    f_alpha: np.ndarray
    f_level: np.ndarray
    # per shell
    shell_level: np.ndarray
    shell_images: List[np.ndarray]  # (n_img, 3) image centres A + T
    domains: List[Domain]
    ln_inv_tau: float
    volume: float

    @property
    def n_basis(self) -> int:
        return int(self.f_atom.shape[0])

    @property
    def n_mu(self) -> int:
        return int(sum(d.n_mu for d in self.domains))

    def level_spacing_volume(self, lev: int) -> float:
        return self.volume / float(np.prod(self.grids[lev]))


def cell_centre_radius(lattice: np.ndarray):
    """Cell centre c = (a1 + a2 + a3)/2 and circumradius R_c (largest corner
    distance from c)."""
    c = 0.5 * lattice.sum(axis=0)
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], float) @ lattice
    return c, float(np.max(np.linalg.norm(corners - c, axis=1)))


def perpendicular_widths(lattice: np.ndarray) -> np.ndarray:
    vol = abs(np.linalg.det(lattice))
    w = []
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        w.append(vol / np.linalg.norm(np.cross(lattice[j], lattice[k])))
    return np.array(w)


def translations_within(lattice: np.ndarray, x: np.ndarray, centre: np.ndarray, radius: float) -> np.ndarray:
    """All lattice vectors T with |x + T - centre| <= radius."""
    inv = np.linalg.inv(lattice)
    f = (centre - x) @ inv  # fractional position of centre relative to x
    rng = []
    for i in range(3):
        e = radius * np.linalg.norm(inv[:, i])
        rng.append(np.arange(int(np.floor(f[i] - e)) - 1, int(np.ceil(f[i] + e)) + 2))
    n = np.array(np.meshgrid(*rng, indexing="ij")).reshape(3, -1).T
    T = n @ lattice
    d = np.linalg.norm(x + T - centre, axis=1)
    return T[d <= radius]


def min_image_distance(lattice: np.ndarray, x: np.ndarray, y: np.ndarray) -> float:
    """min_T |x - y - T|."""
    _, rc = cell_centre_radius(lattice)
    T = translations_within(lattice, y, x, rc + 1e-9)
    if T.shape[0] == 0:
        T = translations_within(lattice, y, x, 2 * rc)
    return float(np.min(np.linalg.norm(x - y - T, axis=1)))


def grid_positions(lattice: np.ndarray, grid, flat: np.ndarray) -> np.ndarray:
    """Cartesian position of flat grid indices i1 + n1 (i2 + n2 i3)."""
    n1, n2, n3 = (int(g) for g in grid)
    i1 = flat % n1
    i2 = (flat // n1) % n2
    i3 = flat // (n1 * n2)
    frac = np.stack([i1 / n1, i2 / n2, i3 / n3], axis=1)
    return frac @ lattice


def window_points(lattice: np.ndarray, grid, centre: np.ndarray, radius: float) -> np.ndarray:
    """Flat indices (ascending) of grid points within `radius` of any image of
    `centre`."""
    grid = np.asarray(grid, dtype=np.int64)
    inv = np.linalg.inv(lattice)
    c, rc = cell_centre_radius(lattice)
    images = translations_within(lattice, centre, c, radius + rc)
    marks = []
    for T in images:
        ctr = centre + T
        f = ctr @ inv
        ranges = []
        for i in range(3):
            e = radius * np.linalg.norm(inv[:, i])
            lo = max(int(np.ceil((f[i] - e) * grid[i])) - 1, 0)
            hi = min(int(np.floor((f[i] + e) * grid[i])) + 1, int(grid[i]) - 1)
            ranges.append(np.arange(lo, hi + 1))
        if any(r.size == 0 for r in ranges):
            continue
        I1, I2, I3 = np.meshgrid(*ranges, indexing="ij")
        flat = (I1 + grid[0] * (I2 + grid[1] * I3)).ravel()
        pos = grid_positions(lattice, grid, flat)
        d2 = np.sum((pos - ctr) ** 2, axis=1)
        marks.append(flat[d2 <= radius * radius])
    if not marks:
        return np.zeros(0, dtype=np.int64)
    return np.unique(np.concatenate(marks)).astype(np.int64)


def build_plan(sysm) -> Plan:
    lattice = np.asarray(sysm.lattice, dtype=np.float64)
    xyz = np.asarray(sysm.xyz, dtype=np.float64)
    grids = np.asarray(sysm.grids, dtype=np.int64)
    nlev = grids.shape[0]
    bounds = np.asarray(sysm.alpha_bound, dtype=np.float64)
    ln_inv_tau = -np.log(sysm.image_tol)
    c, rc = cell_centre_radius(lattice)

    # shell levels: coarsest level whose bound exceeds the exponent
    shell_level = np.full(len(sysm.shell_alpha), nlev - 1, dtype=np.int64)
    for s, a in enumerate(sysm.shell_alpha):
        for lev in range(nlev - 1):
            if a < bounds[lev]:
                shell_level[s] = lev
                break

    # functions: shell order, p components x, y, z, d components m = -2..2
    f_shell, f_atom, f_l, f_comp, f_alpha, f_level = [], [], [], [], [], []
    for s in range(len(sysm.shell_alpha)):
        l = int(sysm.shell_l[s])
        if l not in (0, 1, 2):
            raise ValueError("shells with l = 0, 1 or 2 only")
        comps = [-1] if l == 0 else list(range(2 * l + 1))
        for cpt in comps:
            f_shell.append(s)
            f_atom.append(int(sysm.shell_atom[s]))
            f_l.append(l)
            f_comp.append(cpt)
            f_alpha.append(float(sysm.shell_alpha[s]))
            f_level.append(int(shell_level[s]))
    f_shell = np.array(f_shell)
    f_atom = np.array(f_atom)
    f_level = np.array(f_level)
    f_alpha = np.array(f_alpha)

    # periodic images per shell
    shell_images = []
    for s in range(len(sysm.shell_alpha)):
        A = xyz[sysm.shell_atom[s]]
        r_img = np.sqrt(ln_inv_tau / sysm.shell_alpha[s])
        T = translations_within(lattice, A, c, r_img + rc)
        shell_images.append(A + T)

    widths = perpendicular_widths(lattice)
    ratio = float(sysm.n_mu_ratio)

    def n_mu_for(nL: int, nN: int, npts: int) -> int:
        if ratio <= 0:
            return int(min(npts, nL * (nL + 1) // 2 + nL * nN))
        return int(min(np.floor(ratio * nL + 0.5), npts))

    domains: List[Domain] = []
    if int(getattr(sysm, "domain_mode", 0)) == 1:
        for lev in range(nlev):
            L = np.nonzero(f_level == lev)[0]
            if L.size == 0:
                continue
            N = np.nonzero(f_level < lev)[0]
            npts = int(np.prod(grids[lev]))
            domains.append(Domain(lev, -1, np.arange(npts, dtype=np.int64), L, N,
                                  n_mu_for(L.size, N.size, npts), np.inf))
        return Plan(lattice=lattice, xyz=xyz, grids=grids, f_shell=f_shell, f_atom=f_atom,
                    f_l=np.array(f_l), f_comp=np.array(f_comp), f_alpha=f_alpha, f_level=f_level,
                    shell_level=shell_level, shell_images=shell_images, domains=domains,
                    ln_inv_tau=float(ln_inv_tau), volume=float(abs(np.linalg.det(lattice))))
    # universal domain (level 0)
    L0 = np.nonzero(f_level == 0)[0]
    if L0.size:
        npts = int(np.prod(grids[0]))
        domains.append(
            Domain(0, -1, np.arange(npts, dtype=np.int64), L0, np.zeros(0, dtype=np.int64),
                   n_mu_for(L0.size, 0, npts), np.inf)
        )
    # atom windows on finer levels
    for lev in range(1, nlev):
        r_max = float(np.sqrt(-np.log(sysm.eps_r) / bounds[lev - 1]))
        for A in range(xyz.shape[0]):
            L = np.nonzero((f_level == lev) & (f_atom == A))[0]
            if L.size == 0:
                continue
            if 2.0 * r_max >= widths.min():
                pts = np.arange(int(np.prod(grids[lev])), dtype=np.int64)
            else:
                pts = window_points(lattice, grids[lev], xyz[A], r_max)
            cand = np.nonzero((f_level < lev) | ((f_level == lev) & (f_atom > A)))[0]
            keep = []
            dist_cache = {}
            for f in cand:
                B = int(f_atom[f])
                if B not in dist_cache:
                    dist_cache[B] = min_image_distance(lattice, xyz[B], xyz[A])
                if dist_cache[B] <= np.sqrt(ln_inv_tau / f_alpha[f]) + r_max:
                    keep.append(f)
            N = np.array(keep, dtype=np.int64)
            domains.append(Domain(lev, A, pts, L, N, n_mu_for(L.size, N.size, pts.size), r_max))

    return Plan(
        lattice=lattice,
        xyz=xyz,
        grids=grids,
        f_shell=f_shell,
        f_atom=f_atom,
        f_l=np.array(f_l),
        f_comp=np.array(f_comp),
        f_alpha=f_alpha,
        f_level=f_level,
        shell_level=shell_level,
        shell_images=shell_images,
        domains=domains,
        ln_inv_tau=float(ln_inv_tau),
        volume=float(abs(np.linalg.det(lattice))),
    )


def _smooth235(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def grids_for_threshold(lattice, shell_alpha, alpha_bound, eps_K: float) -> np.ndarray:
    """Grid ladder [n_levels, 3] from the Fourier threshold eps_K (Eq. Ggrid
    and the threshold table of the "Computational details" section).

    Readings: the exponent of Eq. Ggrid for a level is the largest exponent
    living on it (the shell level rule above), G_max = sqrt(-4 a ln eps_K);
    every reciprocal vector G = 2 pi m . B (B rows: b_j with a_i . b_j =
    delta_ij) with |G| <= G_max must lie in the kept band, which for an even
    axis of n points is |m_i| <= n/2 - 1 (the Nyquist plane is not kept);
    axes are even and 2,3,5-smooth; a level is never coarser than the one
    below it.
    """
    lattice = np.asarray(lattice, dtype=np.float64).reshape(3, 3)
    alphas = np.asarray(shell_alpha, dtype=np.float64)
    bounds = np.asarray(alpha_bound, dtype=np.float64).reshape(-1)
    if not (0.0 < eps_K < 1.0) or np.any(~(alphas > 0)):
        raise ValueError("eps_K must lie in (0, 1) and exponents must be positive")
    nlev = bounds.size + 1
    level = np.full(alphas.size, nlev - 1)
    for s, a in enumerate(alphas):
        for lev in range(nlev - 1):
            if a < bounds[lev]:
                level[s] = lev
                break
    recip = np.linalg.inv(lattice).T  # rows b_j
    out = np.zeros((nlev, 3), dtype=np.int64)
    for lev in range(nlev):
        on = alphas[level == lev]
        if on.size == 0:
            raise ValueError(f"level {lev} holds no shell")
        gmax = np.sqrt(-4.0 * on.max() * np.log(eps_K))
        lim = np.floor(gmax * np.linalg.norm(lattice, axis=1) / (2.0 * np.pi)).astype(np.int64)
        need = np.zeros(3, dtype=np.int64)
        m2, m3 = np.meshgrid(np.arange(-lim[1], lim[1] + 1), np.arange(-lim[2], lim[2] + 1), indexing="ij")
        m2, m3 = m2.ravel(), m3.ravel()
        for m1 in range(-lim[0], lim[0] + 1):
            M = np.stack([np.full(m2.size, m1), m2, m3], axis=1)
            G = 2.0 * np.pi * (M @ recip)
            inside = np.sum(G * G, axis=1) <= gmax * gmax
            if inside.any():
                need = np.maximum(need, np.abs(M[inside]).max(axis=0))
        for i in range(3):
            n = 2 * (int(need[i]) + 1)
            while not _smooth235(n):
                n += 2
            if lev > 0:
                n = max(n, int(out[lev - 1, i]))
            out[lev, i] = n
    return out
