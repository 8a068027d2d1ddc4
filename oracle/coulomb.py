"""Coulomb metric (xi|xi') by FFT Poisson solves (Eq. (xi|xi')).

A fitting function is known by its values on its level grid.  Its Fourier
coefficients are  F^(m) = N_g^-1 sum_R F(R) exp(-i G_m . r_R)  with
G_m = sum_i m_i b_i (b_i the reciprocal vectors, a_i . b_j = 2 pi delta_ij),
and the periodic Coulomb integral of two such functions is

    (xi|xi') = Omega sum_{m in J \\ {0}} conj(F^_xi(m)) 4 pi/|G_m|^2 F^_xi'(m).

Readings (the paper does not spell these out):
* J_l = {m : |m_i| < n_l,i / 2}: the Nyquist planes of even grids are
  dropped; the G = 0 term is dropped (no Madelung correction);
* functions on different levels are coupled through the band of the coarser
  level, J_min(l, l');
* real-space form used here:  V_{xi'->l} = C2R_l(restrict_{J_l}(v F^_xi')),
  (xi|xi') = dV_l sum_{R in P_xi} F_xi(R) V_{xi'->l}(R), l = level(xi) <=
  level(xi').
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft


def signed_index(n: int) -> np.ndarray:
    j = np.arange(n)
    return np.where(j <= (n - 1) // 2, j, j - n)


def band_mask(grid) -> np.ndarray:
    """Boolean array on grid index space: m in J and m != 0."""
    m = [signed_index(int(n)) for n in grid]
    ok = [np.abs(mi) * 2 < int(n) for mi, n in zip(m, grid)]
    mask = ok[0][:, None, None] & ok[1][None, :, None] & ok[2][None, None, :]
    mask[0, 0, 0] = False
    return mask


def coulomb_kernel(lattice: np.ndarray, grid) -> np.ndarray:
    """v(m) = 4 pi / |G_m|^2 on J \\ {0}, zero elsewhere; array indexed
    [j1, j2, j3] in FFT order."""
    B = 2.0 * np.pi * np.linalg.inv(lattice).T  # rows b_i
    m = [signed_index(int(n)) for n in grid]
    M1, M2, M3 = np.meshgrid(*m, indexing="ij")
    G = M1[..., None] * B[0] + M2[..., None] * B[1] + M3[..., None] * B[2]
    g2 = np.sum(G * G, axis=-1)
    mask = band_mask(grid)
    v = np.zeros(g2.shape)
    v[mask] = 4.0 * np.pi / g2[mask]
    return v


def to_grid3(values_flat: np.ndarray, grid) -> np.ndarray:
    """Flat index i1 + n1 (i2 + n2 i3) -> array [i1, i2, i3] (Fortran order)."""
    n1, n2, n3 = (int(g) for g in grid)
    return values_flat.reshape((n3, n2, n1) + values_flat.shape[1:]).transpose(
        (2, 1, 0) + tuple(range(3, values_flat.ndim + 2))
    )


def from_grid3(arr: np.ndarray) -> np.ndarray:
    n1, n2, n3 = arr.shape[:3]
    rest = arr.shape[3:]
    return arr.transpose((2, 1, 0) + tuple(range(3, arr.ndim))).reshape((n1 * n2 * n3,) + rest)


def spectrum(F_flat: np.ndarray, grid, workers: int = -1) -> np.ndarray:
    """F^(m) = N_g^-1 sum_R F(R) e^{-i G.r_R}; F_flat (N_g, k) -> (n1,n2,n3,k)."""
    a = to_grid3(F_flat, grid)
    return sfft.fftn(a, axes=(0, 1, 2), workers=workers) / float(np.prod(grid))


def potential_on(spec_fine: np.ndarray, fine_grid, coarse_grid, v_coarse: np.ndarray,
                 workers: int = -1) -> np.ndarray:
    """V(R) = sum_{m in J_coarse \\ 0} v(m) F^(m) e^{i G.r_R} on the coarse grid
    (flat, real) from the fine-grid spectrum (n1,n2,n3,k)."""
    idx = []
    for nf, nc in zip(fine_grid, coarse_grid):
        m = signed_index(int(nc))
        idx.append(np.mod(m, int(nf)))
    sub = spec_fine[np.ix_(idx[0], idx[1], idx[2])]
    sub = sub * v_coarse[..., None]
    ng = float(np.prod(coarse_grid))
    V = sfft.ifftn(sub, axes=(0, 1, 2), workers=workers) * ng
    return from_grid3(V.real)


def coulomb_metric(plan, F_list, workers: int = -1, batch: int = 64) -> np.ndarray:
    """W[xi, xi'] over all domains; F_list[d] is (pts_d, n_d) on the domain
    points.  Rows of domain d against columns of domain d' are formed when
    level(d) <= level(d'); same-level blocks are averaged with their mirror
    and the rest mirrored."""
    doms = plan.domains
    offs = np.concatenate([[0], np.cumsum([F.shape[1] for F in F_list])]).astype(int)
    nmu = int(offs[-1])
    W = np.zeros((nmu, nmu))
    done = np.zeros((len(doms), len(doms)), dtype=bool)
    nlev = plan.grids.shape[0]
    vker = [coulomb_kernel(plan.lattice, plan.grids[l]) for l in range(nlev)]
    for dp, domp in enumerate(doms):
        lp = domp.level
        gp = plan.grids[lp]
        ngp = int(np.prod(gp))
        Fp = F_list[dp]
        for b0 in range(0, Fp.shape[1], batch):
            b1 = min(b0 + batch, Fp.shape[1])
            full = np.zeros((ngp, b1 - b0))
            full[domp.points] = Fp[:, b0:b1]
            spec = spectrum(full, gp, workers)
            for l in range(lp + 1):
                V = potential_on(spec, gp, plan.grids[l], vker[l], workers)
                dV = plan.level_spacing_volume(l)
                for d, dom in enumerate(doms):
                    if dom.level != l:
                        continue
                    W[offs[d]:offs[d + 1], offs[dp] + b0:offs[dp] + b1] = dV * (
                        F_list[d].T @ V[dom.points]
                    )
        for d, dom in enumerate(doms):
            if dom.level <= lp:
                done[d, dp] = True
    # symmetrise: average where both orders were formed, mirror otherwise
    for d in range(len(doms)):
        for dp in range(len(doms)):
            if d > dp and done[d, dp] and done[dp, d]:
                a = W[offs[d]:offs[d + 1], offs[dp]:offs[dp + 1]]
                b = W[offs[dp]:offs[dp + 1], offs[d]:offs[d + 1]].T
                m = 0.5 * (a + b)
                W[offs[d]:offs[d + 1], offs[dp]:offs[dp + 1]] = m
                W[offs[dp]:offs[dp + 1], offs[d]:offs[d + 1]] = m.T
            elif done[d, dp] and not done[dp, d]:
                W[offs[dp]:offs[dp + 1], offs[d]:offs[d + 1]] = W[offs[d]:offs[d + 1], offs[dp]:offs[dp + 1]].T
    for d in range(len(doms)):
        blk = W[offs[d]:offs[d + 1], offs[d]:offs[d + 1]]
        W[offs[d]:offs[d + 1], offs[d]:offs[d + 1]] = 0.5 * (blk + blk.T)
    return W


def pair_coulomb(plan, dens_list, levels, workers: int = -1) -> np.ndarray:
    """Coulomb Gram of arbitrary grid densities: dens_list[i] = (level,
    points, values[pts, k_i]); returns the full (sum k_i)^2 matrix using the
    same convention as coulomb_metric (used by the brute-force exchange)."""
    class _D:
        pass
    doms = []
    F_list = []
    for (lev, pts, vals) in dens_list:
        d = _D()
        d.level = lev
        d.points = pts
        doms.append(d)
        F_list.append(vals)

    class _P:
        pass
    p = _P()
    p.domains = doms
    p.grids = plan.grids
    p.lattice = plan.lattice
    p.level_spacing_volume = plan.level_spacing_volume
    return coulomb_metric(p, F_list, workers)
