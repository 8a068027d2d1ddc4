"""Synthetic diamond workloads (Bohr / Hartree throughout).

The paper benchmarks diamond supercells built from the 8-atom conventional
cell with uncontracted Gaussian bases (Results section).  The real GTH-cc
basis sets are not used here; instead every carbon carries the same explicit
primitive set, chosen so that the basis-function counts per configuration
are 13 per atom:

    s shells at 0.15 * 3**k (k = 0..4) and sp shells (one s and one p that
    share an exponent) at 0.3 and 1.2 Bohr^-2.

Grid ladders follow the two-grid scheme of the paper (a coarse universal
grid plus atom-centred dense windows) extended to L levels.  The exponent
bound of level l scales with the inverse square grid spacing (the
Fourier-cutoff argument of the universal-grid equation), calibrated so that
a 24-point axis over the 3.567 Angstrom cell admits exponents below 2.

The density matrix is D = C C^T for n_occ random orbitals that are made
orthonormal in the overlap metric of the periodic basis (closed-shell, per
spin, no factor 2).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

BOHR_PER_ANGSTROM = 1.0 / 0.529177210903
DIAMOND_A_ANGSTROM = 3.567
DIAMOND_A_BOHR = DIAMOND_A_ANGSTROM * BOHR_PER_ANGSTROM

# fractional coordinates of the 8 atoms of the conventional diamond cell
_DIAMOND_FRAC = np.array(
    [
        [0.0, 0.0, 0.0],
        [0.0, 0.5, 0.5],
        [0.5, 0.0, 0.5],
        [0.5, 0.5, 0.0],
        [0.25, 0.25, 0.25],
        [0.25, 0.75, 0.75],
        [0.75, 0.25, 0.75],
        [0.75, 0.75, 0.25],
    ]
)

# per-atom primitive shells (l, alpha), ascending exponent, s before p
CARBON_SHELLS: Tuple[Tuple[int, float], ...] = (
    (0, 0.15),
    (0, 0.3),
    (1, 0.3),
    (0, 0.45),
    (0, 1.2),
    (1, 1.2),
    (0, 1.35),
    (0, 4.05),
    (0, 12.15),
)


@dataclasses.dataclass
class System:
    """A periodic cell with uncontracted shells, grid ladder and thresholds.

    lattice     (3,3) rows a1, a2, a3 in Bohr
    xyz         (n_atoms, 3) Cartesian atom positions in Bohr
    shell_atom  (n_shells,) int atom index of each shell (atom-major order)
    shell_l     (n_shells,) int angular momentum (0 or 1)
    shell_alpha (n_shells,) float exponent in Bohr^-2
    grids       (n_levels, 3) int grid points per axis, coarse -> fine
    alpha_bound (n_levels-1,) shells with alpha < alpha_bound[l] live on
                level l (the coarsest such level), the rest on the finest
    image_tol   periodic-image cutoff tau
    eps_r       window accuracy of the atom-centred radius equation
    n_mu_ratio  interpolation points per owned function (<= 0: threshold only)
    eps_isdf    relative stop of the pivoted Cholesky
    tie_tol     relative tie window of the pivot argmax
    n_occ       occupied orbitals
    C_occ       (N, n_occ) S-orthonormal occupied orbitals
    D           (N, N) density matrix C_occ C_occ^T
    name        label
    """

    lattice: np.ndarray
    xyz: np.ndarray
    shell_atom: np.ndarray
    shell_l: np.ndarray
    shell_alpha: np.ndarray
    grids: np.ndarray
    alpha_bound: np.ndarray
    image_tol: float = 1e-10
    eps_r: float = 1e-5
    n_mu_ratio: float = 6.0
    eps_isdf: float = 1e-14
    tie_tol: float = 1e-8
    n_occ: int = 0
    C_occ: Optional[np.ndarray] = None
    D: Optional[np.ndarray] = None
    name: str = ""

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_basis(self) -> int:
        return int(np.sum(2 * self.shell_l + 1))

    @property
    def n_levels(self) -> int:
        return int(self.grids.shape[0])


def level_bounds(lattice: np.ndarray, grids: np.ndarray) -> np.ndarray:
    """alpha_bound[l] = 2 * (h0 / h_l)^2 with h0 = a_diamond / 24 and h_l the
    largest axis spacing of level l (l < n_levels - 1)."""
    h0 = DIAMOND_A_BOHR / 24.0
    out = []
    for lev in range(len(grids) - 1):
        h = max(np.linalg.norm(lattice[i]) / grids[lev][i] for i in range(3))
        out.append(2.0 * (h0 / h) ** 2)
    return np.array(out, dtype=np.float64)


def _shells_for_atoms(n_atoms: int, shells=CARBON_SHELLS):
    atom, l, alpha = [], [], []
    for a in range(n_atoms):
        for (ll, al) in shells:
            atom.append(a)
            l.append(ll)
            alpha.append(al)
    return (
        np.array(atom, dtype=np.int32),
        np.array(l, dtype=np.int32),
        np.array(alpha, dtype=np.float64),
    )


def diamond_geometry(
    reps: Sequence[int] = (1, 1, 1),
    displacement_angstrom: float = 0.0,
    strain: float = 0.0,
    seed: Optional[int] = None,
) -> Tuple[np.ndarray, np.ndarray]:
    """Diamond supercell: lattice rows and Cartesian positions (Bohr).

    strain: symmetric strain components drawn from U[-strain, strain];
    displacement: per Cartesian component U[-d, d] Angstrom.
    """
    rng = np.random.default_rng(seed)
    a = DIAMOND_A_BOHR
    lattice = np.diag([a * reps[0], a * reps[1], a * reps[2]]).astype(np.float64)
    frac = []
    for i in range(reps[0]):
        for j in range(reps[1]):
            for k in range(reps[2]):
                for f in _DIAMOND_FRAC:
                    frac.append(
                        [(f[0] + i) / reps[0], (f[1] + j) / reps[1], (f[2] + k) / reps[2]]
                    )
    frac = np.array(frac)
    if strain > 0.0:
        e = rng.uniform(-strain, strain, size=(3, 3))
        e = 0.5 * (e + e.T)
        lattice = lattice @ (np.eye(3) + e)
    xyz = frac @ lattice
    if displacement_angstrom > 0.0:
        xyz = xyz + rng.uniform(
            -displacement_angstrom, displacement_angstrom, size=xyz.shape
        ) * BOHR_PER_ANGSTROM
    return lattice, xyz


def periodic_overlap(lattice, xyz, shell_atom, shell_l, shell_alpha) -> np.ndarray:
    """Closed-form overlap S_uv = sum_T <u_0 | v_0(. - T)> of normalised
    periodic s/p Gaussians (Gaussian product theorem).

    Normalisation: N_s = (2a/pi)^(3/4), N_p = N_s * 2 sqrt(a), p = (x, y, z).
    Used to build an S-orthonormal density and as an analytic reference for
    grid quadratures.
    """
    lattice = np.asarray(lattice, dtype=np.float64)
    nsh = len(shell_alpha)
    offs = np.concatenate([[0], np.cumsum(2 * np.asarray(shell_l) + 1)])
    N = int(offs[-1])
    S = np.zeros((N, N))
    amin = float(np.min(shell_alpha))
    # translations within the decay range of the most diffuse product
    rmax = np.sqrt(60.0 / (amin / 2.0)) + 2.0 * np.max(np.linalg.norm(lattice, axis=1))
    inv = np.linalg.inv(lattice)
    nmax = [int(np.ceil(rmax * np.linalg.norm(inv[:, i]))) + 1 for i in range(3)]
    rng = [np.arange(-n, n + 1) for n in nmax]
    T = np.array(np.meshgrid(*rng, indexing="ij")).reshape(3, -1).T @ lattice
    for i in range(nsh):
        a = shell_alpha[i]
        A = xyz[shell_atom[i]]
        Na = (2 * a / np.pi) ** 0.75 * (2 * np.sqrt(a) if shell_l[i] == 1 else 1.0)
        for j in range(nsh):
            b = shell_alpha[j]
            B = xyz[shell_atom[j]] + T  # (nT, 3)
            Nb = (2 * b / np.pi) ** 0.75 * (2 * np.sqrt(b) if shell_l[j] == 1 else 1.0)
            p = a + b
            mu = a * b / p
            AB = A - B
            r2 = np.sum(AB * AB, axis=1)
            keep = mu * r2 < 80.0
            Bk = B[keep]
            E0 = np.exp(-mu * r2[keep]) * (np.pi / p) ** 1.5
            P = (a * A + b * Bk) / p
            PA = P - A
            PB = P - Bk
            li, lj = shell_l[i], shell_l[j]
            oi, oj = offs[i], offs[j]
            if li == 0 and lj == 0:
                S[oi, oj] = Na * Nb * np.sum(E0)
            elif li == 1 and lj == 0:
                S[oi : oi + 3, oj] = Na * Nb * (PA * E0[:, None]).sum(0)
            elif li == 0 and lj == 1:
                S[oi, oj : oj + 3] = Na * Nb * (PB * E0[:, None]).sum(0)
            else:
                blk = np.einsum("ti,tj,t->ij", PA, PB, E0) + np.eye(3) * np.sum(E0) / (2 * p)
                S[oi : oi + 3, oj : oj + 3] = Na * Nb * blk
    return 0.5 * (S + S.T)


def random_density(S: np.ndarray, n_occ: int, seed: int):
    """C = C0 (C0^T S C0)^(-1/2) with C0 ~ N(0,1); returns (C, D = C C^T)."""
    rng = np.random.default_rng(seed)
    C0 = rng.standard_normal((S.shape[0], n_occ))
    G = C0.T @ S @ C0
    w, U = np.linalg.eigh(G)
    C = C0 @ (U @ np.diag(w ** -0.5) @ U.T)
    return C, C @ C.T


def diamond_system(
    reps=(1, 1, 1),
    grids=((24, 24, 24), (48, 48, 48)),
    n_mu_ratio=6.0,
    n_occ=None,
    displacement_angstrom=0.0,
    strain=0.0,
    geom_seed=None,
    dens_seed=1,
    alpha_bound=None,
    name="",
    with_density=True,
    tie_tol=1e-8,
) -> System:
    lattice, xyz = diamond_geometry(reps, displacement_angstrom, strain, geom_seed)
    sa, sl, sal = _shells_for_atoms(xyz.shape[0])
    grids = np.array(grids, dtype=np.int64)
    if alpha_bound is None:
        alpha_bound = level_bounds(lattice, grids)
    sysm = System(
        lattice=lattice,
        xyz=xyz,
        shell_atom=sa,
        shell_l=sl,
        shell_alpha=sal,
        grids=grids,
        alpha_bound=np.asarray(alpha_bound, dtype=np.float64),
        n_mu_ratio=float(n_mu_ratio),
        n_occ=int(n_occ if n_occ is not None else 2 * xyz.shape[0]),
        name=name,
        tie_tol=tie_tol,
    )
    if with_density:
        S = periodic_overlap(lattice, xyz, sa, sl, sal)
        sysm.C_occ, sysm.D = random_density(S, sysm.n_occ, dens_seed)
    return sysm


def config(k: int, with_density: bool = True) -> System:
    """The benchmark configurations.

    1: 8-atom cubic diamond cell, perfect lattice, grids 24^3 / 48^3,
       alpha bound 2, 6 points per owned function, 16 occupied orbitals.
    2: 2x2x2 supercell (64 atoms) with +-0.05 Angstrom displacements,
       grids 32^3 / 64^3 / 128^3, 8 points per owned function, 128 occupied.
    4: 3x3x3 supercell (216 atoms), grids 40^3 / 80^3 / 160^3, ratio 8,
       432 occupied (the learned-selector inference workload).
    """
    if k == 1:
        return diamond_system(
            (1, 1, 1), ((24, 24, 24), (48, 48, 48)), 6.0, 16, 0.0, 0.0, 100, 101,
            alpha_bound=[2.0], name="cfg1", with_density=with_density,
        )
    if k == 2:
        return diamond_system(
            (2, 2, 2), ((32, 32, 32), (64, 64, 64), (128, 128, 128)), 8.0, 128,
            0.05, 0.0, 200, 201, name="cfg2", with_density=with_density,
        )
    if k == 4:
        return diamond_system(
            (3, 3, 3), ((40, 40, 40), (80, 80, 80), (160, 160, 160)), 8.0, 432,
            0.05, 0.0, 400, 401, name="cfg4", with_density=with_density,
        )
    raise ValueError(f"unknown config {k}")


def batched_cells(n_cells: int = 32, seed0: int = 300, cells=None,
                  with_density: bool = True) -> List[System]:
    """Uneven batch: cells of 1x1x1, 2x1x1, 2x2x1 and 2x2x2 diamond, each with
    a random symmetric strain (+-3 %) and +-0.05 Angstrom displacements,
    two levels with 24 and 48 points per conventional-cell repeat, ratio
    drawn from U[5, 8].  `cells` picks a subset by index (cell c depends on
    c alone)."""
    shapes = [(1, 1, 1), (2, 1, 1), (2, 2, 1), (2, 2, 2)]
    out = []
    for c in (range(n_cells) if cells is None else cells):
        reps = shapes[c % 4]
        rng = np.random.default_rng(seed0 + 2 * c)
        ratio = float(rng.uniform(5.0, 8.0))
        grids = ((24 * reps[0], 24 * reps[1], 24 * reps[2]), (48 * reps[0], 48 * reps[1], 48 * reps[2]))
        out.append(
            diamond_system(
                reps, grids, ratio, 16 * reps[0] * reps[1] * reps[2], 0.05, 0.03,
                seed0 + 2 * c, seed0 + 2 * c + 1, alpha_bound=[2.0], name=f"cfg3_{c}",
                with_density=with_density,
            )
        )
    return out


def tiny_system(
    kind: str = "one_atom",
    grids=((12, 12, 12), (24, 24, 24)),
    n_mu_ratio: float = 6.0,
    dens_seed: int = 7,
    n_occ: int = 2,
    alpha_bound=(2.0,),
    cell_bohr: float = 6.0,
    tie_tol: float = 1e-8,
) -> System:
    """Small cells for brute-force checks.

    one_atom: a single carbon-like atom with shells s0.3, p0.3 (sp), s1.2, s4.05
    two_atom: two such atoms in a cubic cell, one of them off-centre.
    """
    shells = ((0, 0.3), (1, 0.3), (0, 1.2), (0, 4.05))
    lattice = np.eye(3) * cell_bohr
    if kind == "one_atom":
        xyz = np.array([[0.37, 0.21, 0.11]]) * cell_bohr
    elif kind == "two_atom":
        xyz = np.array([[0.12, 0.2, 0.31], [0.61, 0.55, 0.47]]) * cell_bohr
    else:
        raise ValueError(kind)
    sa, sl, sal = _shells_for_atoms(xyz.shape[0], shells)
    sysm = System(
        lattice=lattice,
        xyz=xyz,
        shell_atom=sa,
        shell_l=sl,
        shell_alpha=sal,
        grids=np.array(grids, dtype=np.int64),
        alpha_bound=np.array(alpha_bound, dtype=np.float64),
        n_mu_ratio=n_mu_ratio,
        n_occ=n_occ,
        name=f"tiny_{kind}",
        tie_tol=tie_tol,
    )
    S = periodic_overlap(lattice, xyz, sa, sl, sal)
    sysm.C_occ, sysm.D = random_density(S, n_occ, dens_seed)
    return sysm
