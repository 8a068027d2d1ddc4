// Host-side multigrid plan: levels, periodic images, atom-centred windows and
// the L / G / N function sets of each domain.
//
// Section "Computational details" of the paper: shells are split by exponent
// over grids of increasing resolution; the coarsest grid is a universal grid
// over the whole cell; each finer level is a set of spherical windows of
// radius r_max = sqrt(-ln eps_r / alpha_min) around the atoms (Eq. rcut).
// On the window of atom A, L holds A's functions of that level, G every
// function with a non-negligible value there, N = G \ L (text around Eq.
// "mg product density").  Readings where the paper is silent:
//   * images of a shell: translations T with |A+T-c| <= r_img + R_c,
//     r_img = sqrt(ln(1/tau)/alpha), c the cell centre, R_c its circumradius;
//   * window = grid points within r_max of an image of A (whole grid when
//     2 r_max reaches the smallest perpendicular width);
//   * G of a window = own level functions, all coarser functions, and the
//     same-level functions of atoms with a larger index, screened by
//     min-image distance <= r_img(alpha) + r_max; a same-level pair of two
//     atoms is thus fitted once, on the lower atom's window;
//   * domain_mode 1 (the alternative of the C ABI): one full-grid domain per
//     level, L = the level's functions, N = all coarser functions;
//   * n_mu,d = floor(ratio |L_d| + 1/2) capped at the point count; with
//     ratio <= 0 (stop by eps_isdf only) the cap is the smaller of the point
//     count and the domain's distinct pair products |L|(|L|+1)/2 + |L||N|,
//     which bound the rank of its pair Gram.
#include <algorithm>
#include <cmath>
#include <set>

#include "common.h"

namespace isdf {
namespace {

struct V3 {
  double x, y, z;
};
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double norm(V3 a) { return std::sqrt(a.x * a.x + a.y * a.y + a.z * a.z); }

bool smooth235(int n) {
  if (n <= 0) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

void invert3(const double* a, double* inv, double* det_out) {
  double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
               a[2] * (a[3] * a[7] - a[4] * a[6]);
  double id = 1.0 / det;
  inv[0] = (a[4] * a[8] - a[5] * a[7]) * id;
  inv[1] = (a[2] * a[7] - a[1] * a[8]) * id;
  inv[2] = (a[1] * a[5] - a[2] * a[4]) * id;
  inv[3] = (a[5] * a[6] - a[3] * a[8]) * id;
  inv[4] = (a[0] * a[8] - a[2] * a[6]) * id;
  inv[5] = (a[2] * a[3] - a[0] * a[5]) * id;
  inv[6] = (a[3] * a[7] - a[4] * a[6]) * id;
  inv[7] = (a[1] * a[6] - a[0] * a[7]) * id;
  inv[8] = (a[0] * a[4] - a[1] * a[3]) * id;
  *det_out = det;
}

// x @ M for a row vector x and row-major 3x3 M
inline V3 rowmul(V3 x, const double* M) {
  return {x.x * M[0] + x.y * M[3] + x.z * M[6], x.x * M[1] + x.y * M[4] + x.z * M[7],
          x.x * M[2] + x.y * M[5] + x.z * M[8]};
}
inline V3 latvec(const double* L, double n1, double n2, double n3) {
  return rowmul({n1, n2, n3}, L);
}
// column norm of the inverse lattice: |frac_i| <= |v| * colnorm_i
inline double inv_colnorm(const double* inv, int i) {
  return std::sqrt(inv[0 * 3 + i] * inv[0 * 3 + i] + inv[1 * 3 + i] * inv[1 * 3 + i] +
                   inv[2 * 3 + i] * inv[2 * 3 + i]);
}

// All lattice vectors T with |x + T - centre| <= radius.
std::vector<V3> translations_within(const HostPlan& hp, V3 x, V3 centre, double radius) {
  V3 f = rowmul(sub(centre, x), hp.inv);
  double fv[3] = {f.x, f.y, f.z};
  int lo[3], hi[3];
  for (int i = 0; i < 3; ++i) {
    double e = radius * inv_colnorm(hp.inv, i);
    lo[i] = (int)std::floor(fv[i] - e) - 1;
    hi[i] = (int)std::ceil(fv[i] + e) + 1;
  }
  std::vector<V3> out;
  for (int a = lo[0]; a <= hi[0]; ++a)
    for (int b = lo[1]; b <= hi[1]; ++b)
      for (int c = lo[2]; c <= hi[2]; ++c) {
        V3 T = latvec(hp.lattice, a, b, c);
        if (norm(sub(add(x, T), centre)) <= radius) out.push_back(T);
      }
  return out;
}

void centre_radius(const HostPlan& hp, V3& c, double& rc) {
  c = {0.5 * (hp.lattice[0] + hp.lattice[3] + hp.lattice[6]),
       0.5 * (hp.lattice[1] + hp.lattice[4] + hp.lattice[7]),
       0.5 * (hp.lattice[2] + hp.lattice[5] + hp.lattice[8])};
  rc = 0.0;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k) rc = std::max(rc, norm(sub(latvec(hp.lattice, i, j, k), c)));
}

double min_image_distance(const HostPlan& hp, V3 x, V3 y) {
  V3 c;
  double rc;
  centre_radius(hp, c, rc);
  auto T = translations_within(hp, y, x, rc + 1e-9);
  if (T.empty()) T = translations_within(hp, y, x, 2 * rc);
  double best = 1e300;
  for (auto& t : T) best = std::min(best, norm(sub(sub(x, y), t)));
  return best;
}

std::vector<int32_t> window_points(const HostPlan& hp, const int* grid, V3 centre, double radius) {
  V3 c;
  double rc;
  centre_radius(hp, c, rc);
  auto images = translations_within(hp, centre, c, radius + rc);
  std::vector<int32_t> pts;
  for (auto& T : images) {
    V3 ctr = add(centre, T);
    V3 f = rowmul(ctr, hp.inv);
    double fv[3] = {f.x, f.y, f.z};
    int lo[3], hi[3];
    bool empty = false;
    for (int i = 0; i < 3; ++i) {
      double e = radius * inv_colnorm(hp.inv, i);
      lo[i] = std::max((int)std::ceil((fv[i] - e) * grid[i]) - 1, 0);
      hi[i] = std::min((int)std::floor((fv[i] + e) * grid[i]) + 1, grid[i] - 1);
      if (hi[i] < lo[i]) empty = true;
    }
    if (empty) continue;
    const double r2 = radius * radius;
    for (int i3 = lo[2]; i3 <= hi[2]; ++i3)
      for (int i2 = lo[1]; i2 <= hi[1]; ++i2)
        for (int i1 = lo[0]; i1 <= hi[0]; ++i1) {
          V3 pos = latvec(hp.lattice, (double)i1 / grid[0], (double)i2 / grid[1],
                          (double)i3 / grid[2]);
          V3 d = sub(pos, ctr);
          if (d.x * d.x + d.y * d.y + d.z * d.z <= r2)
            pts.push_back(i1 + grid[0] * (i2 + grid[1] * i3));
        }
  }
  std::sort(pts.begin(), pts.end());
  pts.erase(std::unique(pts.begin(), pts.end()), pts.end());
  return pts;
}

}  // namespace

isdf_status build_host_plan(const isdf_system* sys, HostPlan& hp) {
  if (!sys) {
    set_error("isdf_plan: null system");
    return ISDF_E_ARG;
  }
  if (sys->n_atoms <= 0 || !sys->xyz || sys->n_shells <= 0 || !sys->shell_atom || !sys->shell_l ||
      !sys->shell_alpha || sys->n_levels <= 0 || !sys->grid ||
      (sys->n_levels > 1 && !sys->alpha_bound)) {
    set_error("isdf_plan: missing arrays or non-positive counts");
    return ISDF_E_ARG;
  }
  if (sys->n_levels > 8) {
    set_error("isdf_plan: at most 8 levels");
    return ISDF_E_UNSUPPORTED;
  }
  if (!(sys->image_tol > 0 && sys->image_tol < 1) || !(sys->eps_r > 0 && sys->eps_r < 1) ||
      !(sys->tie_tol >= 0 && sys->tie_tol < 1) || !(sys->eps_isdf >= 0) ||
      std::isnan(sys->n_mu_ratio)) {
    set_error("isdf_plan: thresholds out of range");
    return ISDF_E_ARG;
  }
  for (int i = 0; i < 9; ++i) hp.lattice[i] = sys->lattice[i];
  invert3(hp.lattice, hp.inv, &hp.volume);
  hp.volume = std::fabs(hp.volume);
  if (!(hp.volume > 0) || std::isnan(hp.volume)) {
    set_error("isdf_plan: singular lattice");
    return ISDF_E_ARG;
  }
  hp.ln_inv_tau = -std::log(sys->image_tol);
  hp.n_atoms = sys->n_atoms;
  hp.xyz.assign(sys->xyz, sys->xyz + 3 * sys->n_atoms);
  for (double v : hp.xyz)
    if (!std::isfinite(v)) {
      set_error("isdf_plan: non-finite atom position");
      return ISDF_E_ARG;
    }
  hp.n_levels = sys->n_levels;
  for (int l = 0; l < hp.n_levels; ++l)
    for (int i = 0; i < 3; ++i) {
      int g = sys->grid[3 * l + i];
      if (g <= 0) {
        set_error("isdf_plan: non-positive grid size");
        return ISDF_E_ARG;
      }
      if (!smooth235(g) || g > 256) {
        set_error("isdf_plan: grid axes must be 2,3,5-smooth and at most 256");
        return ISDF_E_UNSUPPORTED;
      }
      hp.grid[l][i] = g;
    }
  for (int l = 1; l < hp.n_levels; ++l)
    for (int i = 0; i < 3; ++i)
      if (hp.grid[l][i] < hp.grid[l - 1][i]) {
        set_error("isdf_plan: levels must not get coarser");
        return ISDF_E_UNSUPPORTED;
      }
  hp.alpha_bound.assign(sys->alpha_bound, sys->alpha_bound + (hp.n_levels - 1));
  hp.eps_r = sys->eps_r;
  hp.n_mu_ratio = sys->n_mu_ratio;
  hp.eps_isdf = sys->eps_isdf;
  hp.tie_tol = sys->tie_tol;

  // shells -> levels, functions
  hp.n_shells = sys->n_shells;
  hp.shell_atom.assign(sys->shell_atom, sys->shell_atom + hp.n_shells);
  hp.shell_l.assign(sys->shell_l, sys->shell_l + hp.n_shells);
  hp.shell_alpha.assign(sys->shell_alpha, sys->shell_alpha + hp.n_shells);
  hp.shell_level.assign(hp.n_shells, hp.n_levels - 1);
  for (int s = 0; s < hp.n_shells; ++s) {
    if (hp.shell_atom[s] < 0 || hp.shell_atom[s] >= hp.n_atoms) {
      set_error("isdf_plan: shell atom out of range");
      return ISDF_E_ARG;
    }
    if (!(hp.shell_alpha[s] > 0) || !std::isfinite(hp.shell_alpha[s])) {
      set_error("isdf_plan: exponents must be positive and finite");
      return ISDF_E_ARG;
    }
    if (hp.shell_l[s] < 0 || hp.shell_l[s] > 2) {
      set_error("isdf_plan: only s, p and d shells are supported");
      return ISDF_E_UNSUPPORTED;
    }
    for (int l = 0; l < hp.n_levels - 1; ++l)
      if (hp.shell_alpha[s] < hp.alpha_bound[l]) {
        hp.shell_level[s] = l;
        break;
      }
    if (s > 0 && hp.shell_atom[s] < hp.shell_atom[s - 1]) {
      set_error("isdf_plan: shells must be given atom-major");
      return ISDF_E_ARG;
    }
  }
  // functions: 1 (s), 3 (p: x, y, z) or 5 (d: real solid harmonics,
  // m = -2..2) per shell
  hp.f_shell.clear();
  for (int s = 0; s < hp.n_shells; ++s) {
    const int nc = 2 * hp.shell_l[s] + 1;
    for (int c = 0; c < nc; ++c) {
      hp.f_shell.push_back(s);
      hp.f_atom.push_back(hp.shell_atom[s]);
      hp.f_comp.push_back(hp.shell_l[s] > 0 ? c : -1);
      hp.f_level.push_back(hp.shell_level[s]);
    }
  }
  hp.n_basis = (int)hp.f_shell.size();

  // periodic images per shell
  V3 c;
  double rc;
  centre_radius(hp, c, rc);
  hp.img_off.resize(hp.n_shells);
  hp.img_cnt.resize(hp.n_shells);
  hp.img_xyz.clear();
  for (int s = 0; s < hp.n_shells; ++s) {
    V3 A = {hp.xyz[3 * hp.shell_atom[s]], hp.xyz[3 * hp.shell_atom[s] + 1],
            hp.xyz[3 * hp.shell_atom[s] + 2]};
    double r_img = std::sqrt(hp.ln_inv_tau / hp.shell_alpha[s]);
    auto T = translations_within(hp, A, c, r_img + rc);
    hp.img_off[s] = (int)(hp.img_xyz.size() / 3);
    hp.img_cnt[s] = (int)T.size();
    for (auto& t : T) {
      V3 p = add(A, t);
      hp.img_xyz.push_back(p.x);
      hp.img_xyz.push_back(p.y);
      hp.img_xyz.push_back(p.z);
    }
  }

  // perpendicular widths
  double wmin = 1e300;
  for (int i = 0; i < 3; ++i) {
    int j = (i + 1) % 3, k = (i + 2) % 3;
    const double* a = hp.lattice;
    V3 aj = {a[3 * j], a[3 * j + 1], a[3 * j + 2]}, ak = {a[3 * k], a[3 * k + 1], a[3 * k + 2]};
    V3 cr = {aj.y * ak.z - aj.z * ak.y, aj.z * ak.x - aj.x * ak.z, aj.x * ak.y - aj.y * ak.x};
    wmin = std::min(wmin, hp.volume / norm(cr));
  }
  // threshold only: at most the number of distinct pair products of the
  // domain (L L pairs once, L N pairs), which bounds the rank of its Gram
  auto n_mu_for = [&](int nL, int nN, int npts) -> int {
    if (hp.n_mu_ratio <= 0)
      return (int)std::min<int64_t>(npts, (int64_t)nL * (nL + 1) / 2 + (int64_t)nL * nN);
    double v = std::floor(hp.n_mu_ratio * nL + 0.5);
    return (int)std::min<double>(v, npts);
  };

  hp.domains.clear();
  hp.domain_mode = sys->domain_mode;
  if (hp.domain_mode != 0 && hp.domain_mode != 1) {
    set_error("isdf_plan: domain_mode must be 0 or 1");
    return ISDF_E_ARG;
  }
  if (hp.domain_mode == 1) {
    // one domain per level over the whole level grid: L = the level's
    // functions, N = every coarser function (a pair is fitted on the level
    // of its sharper function)
    for (int lev = 0; lev < hp.n_levels; ++lev) {
      HostDomain d;
      d.level = lev;
      d.atom = -1;
      d.r_max = INFINITY;
      for (int f = 0; f < hp.n_basis; ++f)
        if (hp.f_level[f] == lev) d.funcs.push_back(f);
      d.nL = (int)d.funcs.size();
      if (d.nL == 0) continue;
      for (int f = 0; f < hp.n_basis; ++f)
        if (hp.f_level[f] < lev) d.funcs.push_back(f);
      d.nN = (int)d.funcs.size() - d.nL;
      const int64_t np = (int64_t)hp.grid[lev][0] * hp.grid[lev][1] * hp.grid[lev][2];
      d.points.resize(np);
      for (int64_t i = 0; i < np; ++i) d.points[i] = (int32_t)i;
      d.n_mu = n_mu_for(d.nL, d.nN, (int)np);
      hp.domains.push_back(std::move(d));
    }
  } else {
  {
    HostDomain d;
    d.level = 0;
    d.atom = -1;
    for (int f = 0; f < hp.n_basis; ++f)
      if (hp.f_level[f] == 0) d.funcs.push_back(f);
    d.nL = (int)d.funcs.size();
    d.nN = 0;
    if (d.nL > 0) {
      int64_t np = (int64_t)hp.grid[0][0] * hp.grid[0][1] * hp.grid[0][2];
      d.points.resize(np);
      for (int64_t i = 0; i < np; ++i) d.points[i] = (int32_t)i;
      d.n_mu = n_mu_for(d.nL, 0, (int)np);
      d.r_max = INFINITY;
      hp.domains.push_back(std::move(d));
    }
  }
  for (int lev = 1; lev < hp.n_levels; ++lev) {
    double r_max = std::sqrt(-std::log(hp.eps_r) / hp.alpha_bound[lev - 1]);
    for (int A = 0; A < hp.n_atoms; ++A) {
      HostDomain d;
      d.level = lev;
      d.atom = A;
      d.r_max = r_max;
      for (int f = 0; f < hp.n_basis; ++f)
        if (hp.f_level[f] == lev && hp.f_atom[f] == A) d.funcs.push_back(f);
      d.nL = (int)d.funcs.size();
      if (d.nL == 0) continue;
      V3 cA = {hp.xyz[3 * A], hp.xyz[3 * A + 1], hp.xyz[3 * A + 2]};
      if (2.0 * r_max >= wmin) {
        int64_t np = (int64_t)hp.grid[lev][0] * hp.grid[lev][1] * hp.grid[lev][2];
        d.points.resize(np);
        for (int64_t i = 0; i < np; ++i) d.points[i] = (int32_t)i;
      } else {
        d.points = window_points(hp, hp.grid[lev], cA, r_max);
      }
      std::vector<double> dist(hp.n_atoms, -1.0);
      for (int f = 0; f < hp.n_basis; ++f) {
        bool cand = hp.f_level[f] < lev || (hp.f_level[f] == lev && hp.f_atom[f] > A);
        if (!cand) continue;
        int B = hp.f_atom[f];
        if (dist[B] < 0) {
          V3 cB = {hp.xyz[3 * B], hp.xyz[3 * B + 1], hp.xyz[3 * B + 2]};
          dist[B] = min_image_distance(hp, cB, cA);
        }
        double alpha = hp.shell_alpha[hp.f_shell[f]];
        if (dist[B] <= std::sqrt(hp.ln_inv_tau / alpha) + r_max) d.funcs.push_back(f);
      }
      d.nN = (int)d.funcs.size() - d.nL;
      d.n_mu = n_mu_for(d.nL, d.nN, (int)d.points.size());
      hp.domains.push_back(std::move(d));
    }
  }
  }
  hp.n_mu_total = 0;
  for (auto& d : hp.domains) hp.n_mu_total += d.n_mu;
  if (hp.domains.empty()) {
    set_error("isdf_plan: no domain has local functions");
    return ISDF_E_ARG;
  }
  return ISDF_OK;
}

// Grid ladder for a Fourier threshold (Eq. Ggrid).  A level's grid must
// keep every reciprocal vector G = 2 pi (m1 b1 + m2 b2 + m3 b3) with
// |G| <= G_max = sqrt(-4 a ln eps_K), a the largest exponent living on the
// level.  Axis i keeps |m_i| <= n_i/2 - 1 (the Nyquist plane is dropped), so
// n_i is the smallest even 2,3,5-smooth length with n_i/2 - 1 >= the largest
// |m_i| over that ball; levels never get coarser than the one below.
isdf_status threshold_grids(const double* lattice, int n_shells, const double* shell_alpha,
                            int n_levels, const double* alpha_bound, double eps_K, int32_t* out) {
  if (!lattice || !shell_alpha || !out || n_shells <= 0 || n_levels <= 0 || n_levels > 8 ||
      (n_levels > 1 && !alpha_bound) || !(eps_K > 0 && eps_K < 1)) {
    set_error("isdf_grids_for_threshold: null pointers, bad counts or eps_K outside (0, 1)");
    return ISDF_E_ARG;
  }
  double inv[9], det;
  invert3(lattice, inv, &det);
  if (!(std::fabs(det) > 0) || !std::isfinite(det)) {
    set_error("isdf_grids_for_threshold: singular lattice");
    return ISDF_E_ARG;
  }
  std::vector<double> amax(n_levels, 0.0);
  for (int s = 0; s < n_shells; ++s) {
    const double a = shell_alpha[s];
    if (!(a > 0) || !std::isfinite(a)) {
      set_error("isdf_grids_for_threshold: non-positive exponent");
      return ISDF_E_ARG;
    }
    int lev = n_levels - 1;
    for (int l = 0; l < n_levels - 1; ++l)
      if (a < alpha_bound[l]) {
        lev = l;
        break;
      }
    amax[lev] = std::max(amax[lev], a);
  }
  // reciprocal basis b_j (rows): b_j . a_i = delta_ij, i.e. column j of inv
  double b[3][3];
  for (int j = 0; j < 3; ++j)
    for (int c = 0; c < 3; ++c) b[j][c] = inv[3 * c + j];
  double alen[3];
  for (int i = 0; i < 3; ++i)
    alen[i] = std::sqrt(lattice[3 * i] * lattice[3 * i] + lattice[3 * i + 1] * lattice[3 * i + 1] +
                        lattice[3 * i + 2] * lattice[3 * i + 2]);
  const double two_pi = 2.0 * M_PI;
  std::vector<int32_t> grid(3 * n_levels);
  for (int l = 0; l < n_levels; ++l) {
    if (!(amax[l] > 0)) {
      set_error("isdf_grids_for_threshold: a level holds no shell");
      return ISDF_E_ARG;
    }
    const double gmax = std::sqrt(-4.0 * amax[l] * std::log(eps_K));
    int box[3], need[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i) {
      const double bi = std::floor(gmax * alen[i] / two_pi);
      if (bi > 200) {
        set_error("isdf_grids_for_threshold: an axis would exceed 256 points");
        return ISDF_E_UNSUPPORTED;
      }
      box[i] = (int)bi;  // |m_i| <= G_max |a_i| / (2 pi) for every G in the ball
    }
    const double g2max = gmax * gmax;
    for (int m1 = -box[0]; m1 <= box[0]; ++m1)
      for (int m2 = -box[1]; m2 <= box[1]; ++m2)
        for (int m3 = -box[2]; m3 <= box[2]; ++m3) {
          double g[3];
          for (int c = 0; c < 3; ++c) g[c] = two_pi * (m1 * b[0][c] + m2 * b[1][c] + m3 * b[2][c]);
          if (g[0] * g[0] + g[1] * g[1] + g[2] * g[2] > g2max) continue;
          need[0] = std::max(need[0], std::abs(m1));
          need[1] = std::max(need[1], std::abs(m2));
          need[2] = std::max(need[2], std::abs(m3));
        }
    for (int i = 0; i < 3; ++i) {
      int n = 2 * (need[i] + 1);
      while (!smooth235(n)) n += 2;
      if (l > 0) n = std::max(n, (int)grid[3 * (l - 1) + i]);
      if (n > 256) {
        set_error("isdf_grids_for_threshold: an axis would exceed 256 points");
        return ISDF_E_UNSUPPORTED;
      }
      grid[3 * l + i] = n;
    }
  }
  std::copy(grid.begin(), grid.end(), out);
  return ISDF_OK;
}

}  // namespace isdf
