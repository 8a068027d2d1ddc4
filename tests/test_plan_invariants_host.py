"""The C ABI's plan checked against facts that hold by definition, computed
here by brute force with no use of the oracle's plan code (no GPU):

* window membership: a point is in the window of atom A on level l exactly
  when its minimum-image distance to A is at most r_max = sqrt(-ln eps_r /
  alpha_bound[l-1]) (Eq. rcut; the whole grid once 2 r_max reaches the
  smallest perpendicular width);
* L = the level's functions on A; N = the coarser functions and the
  same-level functions of higher-index atoms whose atom lies within
  r_img(alpha) + r_max of A (minimum image), r_img = sqrt(ln(1/tau)/alpha);
* pair coverage: every ordered pair of functions with a non-negligible
  closed-form overlap is owned by exactly one domain mask L G + N L;
* the point counts n_mu,d = floor(r |L| + 1/2), capped at the point count.
"""
import numpy as np
import pytest

from paper_2404_09373_amd import binding
from workloads import batched_cells, config, periodic_overlap, tiny_system


def _translations(lat, k=1):
    n = np.arange(-k, k + 1)
    return np.array(np.meshgrid(n, n, n, indexing="ij")).reshape(3, -1).T @ lat


def _min_image(lat, X, y, T):
    """min over lattice vectors of |X - y - T|: the difference is first
    reduced to fractional coordinates in [-1/2, 1/2), then every neighbour
    translation in T (the 27 of k = 1; enough for the near-orthogonal cells
    tested, whose reduced differences lie within one cell of the nearest
    image) is tried."""
    inv = np.linalg.inv(lat)
    f = (X - y) @ inv
    r = (f - np.round(f)) @ lat
    best = np.full(X.shape[0], np.inf)
    for t in T:
        best = np.minimum(best, np.linalg.norm(r - t, axis=1))
    return best


def _functions(s):
    """(atom, level, alpha) of every function, shells in order, 2l+1 each."""
    lev = np.searchsorted(np.asarray(s.alpha_bound), s.shell_alpha, side="right")
    out = []
    for a, l, al, lv in zip(s.shell_atom, s.shell_l, s.shell_alpha, lev):
        out += [(int(a), int(lv), float(al))] * (2 * int(l) + 1)
    return np.array(out, dtype=[("atom", int), ("level", int), ("alpha", float)])


def _check(s):
    plan = binding.Plan(s)
    lat = np.asarray(s.lattice, dtype=float)
    xyz = np.asarray(s.xyz, dtype=float)
    T = _translations(lat)
    fn = _functions(s)
    N = fn.size
    vol = abs(np.linalg.det(lat))
    widths = [vol / np.linalg.norm(np.cross(lat[(i + 1) % 3], lat[(i + 2) % 3])) for i in range(3)]
    ln_inv_tau = -np.log(s.image_tol)
    owned = np.zeros((N, N), dtype=int)
    for d in range(plan.n_domains):
        g = plan.domain(d)
        lev, A = g["level"], g["atom"]
        funcs = g["funcs"]
        L, Nn = funcs[:g["nL"]], funcs[g["nL"]:]
        grid = np.asarray(s.grids[lev])
        ng = int(np.prod(grid))
        if A < 0:  # the universal grid: every point, every level-0 function
            assert lev == 0 and np.array_equal(g["points"], np.arange(ng))
            assert np.array_equal(L, np.nonzero(fn["level"] == 0)[0]) and Nn.size == 0
        else:
            r_max = np.sqrt(-np.log(s.eps_r) / s.alpha_bound[lev - 1])
            flat = np.arange(ng)
            i1, i2, i3 = flat % grid[0], (flat // grid[0]) % grid[1], flat // (grid[0] * grid[1])
            pos = np.stack([i1 / grid[0], i2 / grid[1], i3 / grid[2]], axis=1) @ lat
            if 2 * r_max >= min(widths):
                want = flat
            else:
                want = flat[_min_image(lat, pos, xyz[A], T) <= r_max]
            assert np.array_equal(g["points"], want), f"domain {d} window"
            assert np.array_equal(L, np.nonzero((fn["level"] == lev) & (fn["atom"] == A))[0])
            dist = _min_image(lat, xyz, xyz[A], T)
            cand = (fn["level"] < lev) | ((fn["level"] == lev) & (fn["atom"] > A))
            keep = cand & (dist[fn["atom"]] <= np.sqrt(ln_inv_tau / fn["alpha"]) + r_max)
            assert np.array_equal(np.sort(Nn), np.nonzero(keep)[0]), f"domain {d} N set"
        want_mu = min(int(np.floor(s.n_mu_ratio * L.size + 0.5)), g["points"].size)
        assert g["n_mu"] == want_mu
        inL = np.zeros(N, bool)
        inG = np.zeros(N, bool)
        inL[L] = True
        inG[funcs] = True
        inN = inG & ~inL
        owned += (inL[:, None] & inG[None, :]) | (inN[:, None] & inL[None, :])
    S = periodic_overlap(lat, xyz, s.shell_atom, s.shell_l, s.shell_alpha)
    assert owned.max() <= 1, "a pair is owned by two domains"
    assert np.all(owned[np.abs(S) > 1e-7] == 1), "a non-negligible pair is not owned"
    plan.close()


@pytest.mark.parametrize("which", ["cfg1", "two_atom", "d_two_strained", "cfg3_cell3"])
def test_plan_invariants_by_brute_force(which):
    if which == "cfg1":
        s = config(1, with_density=False)
    elif which == "two_atom":
        s = tiny_system("two_atom")
    elif which == "d_two_strained":
        s = tiny_system("d_two", grids=((12, 12, 12), (24, 24, 24)))
        s.lattice = s.lattice @ (np.eye(3) + np.array([[0.03, -0.01, 0.0], [-0.01, 0.0, 0.02],
                                                       [0.0, 0.02, -0.02]]))
    else:
        s = batched_cells(4, with_density=False)[3]
        s.grids = np.array([[24, 48, 40], [48, 96, 80]])
    _check(s)
