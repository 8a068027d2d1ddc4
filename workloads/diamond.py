"""Synthetic diamond workloads (Bohr / Hartree throughout).

The paper benchmarks diamond supercells built from the 8-atom conventional
cell with uncontracted Gaussian bases (Results section).  The real GTH-cc
basis sets are not used here; instead every carbon carries the same explicit
primitive set, chosen so that the basis-function counts per configuration
are 13 per atom:

    s shells at 0.15 * 3**k (k = 0..4) and sp shells (one s and one p that
    share an exponent) at 0.3 and 1.2 Bohr^-2.

The large 384-atom configuration carries 44 functions per atom with d
shells (LARGE_SHELLS): s, p and d primitives at 0.1 * 2.5**k, the d shells
as the five real solid harmonics.

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


# the large configuration's per-atom set: exponents 0.1 * 2.5**k with s at
# k = 0..7, p at k = 0..6 and d (real solid harmonics) at k = 0..2, i.e.
# 8 s + 7 p + 3 d shells = 44 functions, ascending exponent, s, p, d
LARGE_SHELLS: Tuple[Tuple[int, float], ...] = tuple(
    sorted(
        [(0, 0.1 * 2.5 ** k) for k in range(8)]
        + [(1, 0.1 * 2.5 ** k) for k in range(7)]
        + [(2, 0.1 * 2.5 ** k) for k in range(3)],
        key=lambda t: (t[1], t[0]),
    )
)


@dataclasses.dataclass
class System:
    """A periodic cell with uncontracted shells, grid ladder and thresholds.

    lattice     (3,3) rows a1, a2, a3 in Bohr
    xyz         (n_atoms, 3) Cartesian atom positions in Bohr
    shell_atom  (n_shells,) int atom index of each shell (atom-major order)
    shell_l     (n_shells,) int angular momentum (0, 1 or 2; d as real solid
                harmonics, 5 functions)
    shell_alpha (n_shells,) float exponent in Bohr^-2
    grids       (n_levels, 3) int grid points per axis, coarse -> fine
    alpha_bound (n_levels-1,) shells with alpha < alpha_bound[l] live on
                level l (the coarsest such level), the rest on the finest
    image_tol   periodic-image cutoff tau
    eps_r       window accuracy of the atom-centred radius equation
    n_mu_ratio  interpolation points per owned function (<= 0: threshold only)
    eps_isdf    relative stop of the pivoted Cholesky
    tie_tol     relative tie window of the pivot argmax
    domain_mode 0: universal grid + atom windows, 1: one full-cell domain per
                level
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
    domain_mode: int = 0
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


# Cartesian monomials (x^i y^j z^k) of each angular momentum, and the real
# solid harmonics (Racah normalisation, sum_m S_lm^2 = r^(2l)) as rows of
# coefficients over those monomials, in the order m = -l .. l:
#   d: sqrt3 xy, sqrt3 yz, z^2 - (x^2 + y^2)/2, sqrt3 xz, sqrt3/2 (x^2 - y^2)
_CART = {
    0: ((0, 0, 0),),
    1: ((1, 0, 0), (0, 1, 0), (0, 0, 1)),
    2: ((2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 1, 0), (1, 0, 1), (0, 1, 1)),
}
_R3 = np.sqrt(3.0)
_SPH = {
    0: np.eye(1),
    1: np.eye(3),
    2: np.array(
        [
            [0.0, 0.0, 0.0, _R3, 0.0, 0.0],
            [0.0, 0.0, 0.0, 0.0, 0.0, _R3],
            [-0.5, -0.5, 1.0, 0.0, 0.0, 0.0],
            [0.0, 0.0, 0.0, 0.0, _R3, 0.0],
            [0.5 * _R3, -0.5 * _R3, 0.0, 0.0, 0.0, 0.0],
        ]
    ),
}


def primitive_norm(l: int, a: float) -> float:
    """N with int (N S_lm(r) exp(-a r^2))^2 d^3r = 1 for every m:
    N_s = (2a/pi)^(3/4), N_p = N_s 2 sqrt(a), N_d = N_s 4a/sqrt(3)."""
    n = (2.0 * a / np.pi) ** 0.75
    return n * (1.0, 2.0 * np.sqrt(a), 4.0 * a / _R3)[int(l)]


def _os_1d(la: int, lb: int, PA: np.ndarray, PB: np.ndarray, p: float):
    """One-dimensional Obara-Saika overlap ratios s[i][j] = S_ij / S_00 for
    i <= la, j <= lb (vectorised over the last axis):
    s[i+1][j] = PA s[i][j] + (i s[i-1][j] + j s[i][j-1]) / 2p, and the same
    with PB for j + 1."""
    h = 0.5 / p
    s = [[None] * (lb + 1) for _ in range(la + 1)]
    s[0][0] = np.ones_like(PA)
    for i in range(la + 1):
        for j in range(lb + 1):
            if i == 0 and j == 0:
                continue
            if i > 0:
                v = PA * s[i - 1][j]
                if i > 1:
                    v = v + (i - 1) * h * s[i - 2][j]
                if j > 0:
                    v = v + j * h * s[i - 1][j - 1]
            else:
                v = PB * s[i][j - 1]
                if j > 1:
                    v = v + (j - 1) * h * s[i][j - 2]
            s[i][j] = v
    return s


def periodic_overlap(lattice, xyz, shell_atom, shell_l, shell_alpha) -> np.ndarray:
    """Closed-form overlap S_uv = sum_T <u_0 | v_0(. - T)> of normalised
    periodic Gaussians with l <= 2 (Gaussian product theorem and the
    Obara-Saika recursion for the Cartesian factors, then the Cartesian ->
    real-solid-harmonic map of each shell).

    Functions: N_l(a) S_lm(r - A) exp(-a |r - A|^2) with primitive_norm N_l;
    p = (x, y, z), d in the order m = -2..2 of _SPH.  Used to build an
    S-orthonormal density and as an analytic reference for grid quadratures.
    Shells are grouped by (l, exponent) and every group pair is evaluated
    for all atom pairs and translations at once.
    """
    lattice = np.asarray(lattice, dtype=np.float64)
    xyz = np.asarray(xyz, dtype=np.float64)
    shell_atom = np.asarray(shell_atom, dtype=np.int64)
    shell_l = np.asarray(shell_l, dtype=np.int64)
    shell_alpha = np.asarray(shell_alpha, dtype=np.float64)
    if shell_l.max() > 2:
        raise ValueError("shells up to l = 2")
    nsh = shell_alpha.size
    nat = xyz.shape[0]
    offs = np.concatenate([[0], np.cumsum(2 * shell_l + 1)]).astype(np.int64)
    N = int(offs[-1])
    S = np.zeros((N, N))
    cut = 80.0  # mu |A - B - T|^2 beyond this contributes < e^-80
    amin = float(np.min(shell_alpha))
    rmax = np.sqrt(cut / (amin / 2.0))
    # ordered atom pairs and translations with |A - B - T| <= rmax: reduce
    # A - B to the cell around the origin, then scan the translations that
    # can bring it within rmax
    inv = np.linalg.inv(lattice)
    ia, ib = np.meshgrid(np.arange(nat), np.arange(nat), indexing="ij")
    ia, ib = ia.ravel(), ib.ravel()
    f = (xyz[ia] - xyz[ib]) @ inv
    dred = (f - np.round(f)) @ lattice
    reach = rmax + float(np.max(np.linalg.norm(dred, axis=1)))
    nmax = [int(np.ceil(reach * np.linalg.norm(inv[:, i]))) + 1 for i in range(3)]
    rng = [np.arange(-n, n + 1) for n in nmax]
    Tall = np.array(np.meshgrid(*rng, indexing="ij")).reshape(3, -1).T @ lattice
    Tall = Tall[np.linalg.norm(Tall, axis=1) <= reach]
    pa_l, pb_l, d_l = [], [], []
    for T in Tall:
        dAB = dred - T  # A - (B + T') for some lattice vector T'
        r2 = np.einsum("ij,ij->i", dAB, dAB)
        k = r2 <= rmax * rmax
        if k.any():
            pa_l.append(ia[k])
            pb_l.append(ib[k])
            d_l.append(dAB[k])
    pa = np.concatenate(pa_l)
    pb = np.concatenate(pb_l)
    dAB = np.concatenate(d_l)
    r2 = np.einsum("ij,ij->i", dAB, dAB)
    order = np.argsort(r2, kind="stable")  # nearest first: a cutoff is a prefix
    pa, pb, dAB, r2 = pa[order], pb[order], dAB[order], r2[order]
    ap = pa * nat + pb
    # shell groups: (l, alpha) -> shell index per atom (-1 if absent)
    keys = sorted({(int(l), float(a)) for l, a in zip(shell_l, shell_alpha)})
    of_atom = {}
    for key in keys:
        m = np.full(nat, -1, dtype=np.int64)
        for s in range(nsh):
            if (int(shell_l[s]), float(shell_alpha[s])) == key:
                if m[shell_atom[s]] >= 0:
                    raise ValueError("two shells of one atom share (l, alpha)")
                m[shell_atom[s]] = s
        of_atom[key] = m
    for (la, a) in keys:
        ra = of_atom[(la, a)]
        for (lb, b) in keys:
            rb = of_atom[(lb, b)]
            p = a + b
            mu = a * b / p
            n = int(np.searchsorted(r2, cut / mu, side="right"))
            if n == 0:
                continue
            d = dAB[:n]
            E0 = np.exp(-mu * r2[:n]) * (np.pi / p) ** 1.5
            PA = -(b / p) * d  # P - A with P = (a A + b (B + T)) / p
            PB = (a / p) * d   # P - (B + T)
            s1 = [_os_1d(la, lb, PA[:, x], PB[:, x], p) for x in range(3)]
            ca, cb = _CART[la], _CART[lb]
            cart = np.empty((len(ca), len(cb), n))
            for u, (i1, i2, i3) in enumerate(ca):
                for v, (j1, j2, j3) in enumerate(cb):
                    cart[u, v] = E0 * s1[0][i1][j1] * s1[1][i2][j2] * s1[2][i3][j3]
            sph = cart * (primitive_norm(la, a) * primitive_norm(lb, b))
            if la == 2:
                sph = np.tensordot(_SPH[2], sph, axes=(1, 0))
            if lb == 2:
                sph = np.tensordot(_SPH[2], sph, axes=(1, 1)).transpose(1, 0, 2)
            # sum over translations per atom pair, then place the shell pairs
            A_, B_ = np.nonzero((ra[:, None] >= 0) & (rb[None, :] >= 0))
            oi, oj = offs[ra[A_]], offs[rb[B_]]
            for m_ in range(sph.shape[0]):
                for n_ in range(sph.shape[1]):
                    acc = np.bincount(ap[:n], weights=sph[m_, n_], minlength=nat * nat)
                    S[oi + m_, oj + n_] = acc.reshape(nat, nat)[A_, B_]
    return 0.5 * (S + S.T)


def random_density(S: np.ndarray, n_occ: int, seed: int):
    """C = C0 (C0^T S C0)^(-1/2) with C0 ~ N(0,1); returns (C, D = C C^T)."""
    rng = np.random.default_rng(seed)
    C0 = rng.standard_normal((S.shape[0], n_occ))
    G = C0.T @ S @ C0
    w, U = np.linalg.eigh(G)
    C = C0 @ (U @ np.diag(w ** -0.5) @ U.T)
    return C, C @ C.T


def bond_orbitals(sysm: "System", hybrid_alpha: float = 0.3, mix: float = 0.3, seed: int = 0):
    """Localised occupied orbitals of a diamond-like cell: one per bond.

    Bonds are the atom pairs closer than 1.2 times the shortest minimum-image
    distance (each carbon has four, so there are 2 n_atoms of them, the
    closed-shell count).  Orbital b of bond (A, B) starts as the sum of two
    sp3 hybrids, s + sqrt3 (u . p) on A and on B, built from the s and p
    shells whose exponent is closest to `hybrid_alpha`, u the unit vector
    from the atom to its partner, plus `mix` times seeded N(0, 1)
    coefficients on every function of A and B (so that every shell of the
    two atoms, sharp ones included, takes part); the set is then made
    S-orthonormal by C = C0 (C0^T S C0)^(-1/2), the orthonormal set closest
    to C0 (Loewdin), which keeps it localised.  Returns (C, D = C C^T, bond
    atom pairs)."""
    lat = np.asarray(sysm.lattice, dtype=np.float64)
    xyz = np.asarray(sysm.xyz, dtype=np.float64)
    n = xyz.shape[0]
    inv = np.linalg.inv(lat)
    shifts = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)], dtype=np.float64)

    def min_image(d):
        f = d @ inv
        f -= np.round(f)
        cand = (f[None, :] + shifts) @ lat
        return cand[np.argmin(np.sum(cand * cand, axis=1))]

    vec = {}
    dmin = np.inf
    for a in range(n):
        for b in range(a + 1, n):
            v = min_image(xyz[b] - xyz[a])
            vec[(a, b)] = v
            dmin = min(dmin, float(np.linalg.norm(v)))
    bonds = [(a, b) for (a, b), v in vec.items() if np.linalg.norm(v) < 1.2 * dmin]
    # function index of each shell's first component (atom-major order)
    first, off = [], 0
    for l in sysm.shell_l:
        first.append(off)
        off += 2 * int(l) + 1
    nb = off

    def hybrid(atom, u):
        h = np.zeros(nb)
        sh = [i for i in range(len(sysm.shell_atom)) if sysm.shell_atom[i] == atom]
        s_sh = min((i for i in sh if sysm.shell_l[i] == 0), key=lambda i: abs(sysm.shell_alpha[i] - hybrid_alpha))
        p_sh = min((i for i in sh if sysm.shell_l[i] == 1), key=lambda i: abs(sysm.shell_alpha[i] - hybrid_alpha))
        h[first[s_sh]] = 1.0
        h[first[p_sh]:first[p_sh] + 3] = np.sqrt(3.0) * u
        return h

    fatom = np.repeat(np.asarray(sysm.shell_atom), 2 * np.asarray(sysm.shell_l) + 1)
    rng = np.random.default_rng(seed)
    C0 = np.zeros((nb, len(bonds)))
    for k, (a, b) in enumerate(bonds):
        u = vec[(a, b)] / np.linalg.norm(vec[(a, b)])
        C0[:, k] = hybrid(a, u) + hybrid(b, -u)
        on = np.nonzero((fatom == a) | (fatom == b))[0]
        C0[on, k] += mix * rng.standard_normal(on.size)
    S = periodic_overlap(lat, xyz, sysm.shell_atom, sysm.shell_l, sysm.shell_alpha)
    G = C0.T @ S @ C0
    w, U = np.linalg.eigh(G)
    C = C0 @ (U @ np.diag(w ** -0.5) @ U.T)
    return C, C @ C.T, bonds


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
    shells=CARBON_SHELLS,
) -> System:
    lattice, xyz = diamond_geometry(reps, displacement_angstrom, strain, geom_seed)
    sa, sl, sal = _shells_for_atoms(xyz.shape[0], shells)
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
    5: 4x4x3 supercell (384 atoms) with +-0.05 Angstrom displacements, the
       44-function set LARGE_SHELLS (N = 16896), four isotropic levels
       24x24x18 / 48x48x36 / 96x96x72 / 192x192x144 (exponent bounds
       0.125 / 0.5 / 2 from level_bounds), 5 points per owned function,
       768 occupied.
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
    if k == 5:
        return diamond_system(
            (4, 4, 3), ((24, 24, 18), (48, 48, 36), (96, 96, 72), (192, 192, 144)), 5.0, 768,
            0.05, 0.0, 500, 501, name="cfg5", with_density=with_density, shells=LARGE_SHELLS,
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
    d_atom:   one atom with d shells on both levels: s0.3, p0.3, d0.5,
              s1.2, d2.5
    d_two:    two d_atom atoms (cross-atom d-d pairs on the fine windows)
    """
    shells = ((0, 0.3), (1, 0.3), (0, 1.2), (0, 4.05))
    lattice = np.eye(3) * cell_bohr
    if kind in ("d_atom", "d_two"):
        shells = ((0, 0.3), (1, 0.3), (2, 0.5), (0, 1.2), (2, 2.5))
    if kind in ("one_atom", "d_atom"):
        xyz = np.array([[0.37, 0.21, 0.11]]) * cell_bohr
    elif kind in ("two_atom", "d_two"):
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
