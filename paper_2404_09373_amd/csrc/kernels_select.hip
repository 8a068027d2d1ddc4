// Basis values on the level grids, the pair-Gram diagonal, greedy pivoted
// Cholesky point selection, and the gather of the interpolation rows.
//
// Basis (Results section: atomic orbitals evaluated directly on the grids):
//   mu(r) = sum_T N Y_l(r - A - T) exp(-alpha |r - A - T|^2), terms with
//   alpha |r - A - T|^2 > ln(1/tau) dropped; Y_l is 1 (s), x, y, z (p) or
//   the five real solid harmonics (d, m = -2..2).  One thread per grid point,
//   columns written point-fastest (coalesced), Gram diagonal
//   d(R) = a_L (a_L + 2 a_N), a_X = sum_{mu in X} mu(R)^2, fused in.
//
// Selection (Interpolative decomposition section, pivoted Cholesky on
// Eq. M(R,R); done per local grid as in "Computational details"):
//   per step k of every active domain
//     select : pivot p = smallest index with d >= (1 - tau) max d over the
//              remaining candidates; stop when d(p) <= eps * max d0 or k = n_mu
//     column : l_k(R) = [M(R,p) - sum_{j<k} l_j(R) l_j(p)] / sqrt(d(p)),
//              M(R,p) = a_L(R,p) (a_L(R,p) + 2 a_N(R,p)),
//              a_X(R,p) = sum_{mu in X} mu(R) mu(p);  d <- max(d - l_k^2, 0)
//   The column kernel reads the domain's basis columns and its factor once
//   per step (HBM-bound, left-looking) and leaves per-tile maxima so that
//   the select kernel can apply the tie rule exactly.
#include <climits>

#include "common.h"

namespace isdf {

// ---------------------------------------------------------------- basis
__global__ void __launch_bounds__(256)
basis_eval_kernel(LatticeArg lat, const ShellDev* __restrict__ shells,
                  const double* __restrict__ img, const ColShell* __restrict__ colshells,
                  const DomainDev* __restrict__ doms, const int32_t* __restrict__ points,
                  const BasisTile* __restrict__ tiles, double* __restrict__ phi,
                  double* __restrict__ diag, double* __restrict__ aux) {
  const BasisTile t = tiles[blockIdx.x];
  const DomainDev d = doms[t.domain];
  const int i = t.start + (int)threadIdx.x;
  if (i >= d.pts) return;
  const int flat = points[d.pts_off + i];
  const int n1 = lat.grid[d.level][0], n2 = lat.grid[d.level][1], n3 = lat.grid[d.level][2];
  const int i1 = flat % n1;
  const int rem = flat / n1;
  const int i2 = rem % n2;
  const int i3 = rem / n2;
  const double f1 = (double)i1 / (double)n1, f2 = (double)i2 / (double)n2,
               f3 = (double)i3 / (double)n3;
  const double x = f1 * lat.a[0] + f2 * lat.a[3] + f3 * lat.a[6];
  const double y = f1 * lat.a[1] + f2 * lat.a[4] + f3 * lat.a[7];
  const double z = f1 * lat.a[2] + f2 * lat.a[5] + f3 * lat.a[8];
  double aL = 0.0, aN = 0.0, mL = 0.0, sL = 0.0;
  double* out = phi + d.phi_off + i;
  const int64_t P = d.pts;
  for (int e = 0; e < d.colshell_cnt; ++e) {
    const ColShell cs = colshells[d.colshell_off + e];
    const ShellDev sh = shells[cs.shell];
    // s: v[0]; p: v[0..2] = x, y, z; d: v[0..4] = the real solid harmonics
    // sqrt3 xy, sqrt3 yz, z^2 - (x^2 + y^2)/2, sqrt3 xz, sqrt3/2 (x^2 - y^2)
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const double* c = img + 3 * (int64_t)sh.img_off;
    // the images that can reach the domain, in ascending order (the others
    // fail the cutoff test below at every point of the domain); bits at or
    // above the shell's image count are never set
    uint64_t todo = sh.img_cnt >= 64 ? cs.imask : cs.imask & ((1ull << sh.img_cnt) - 1);
    for (int m = 0; sh.img_cnt > 64 ? m < sh.img_cnt : todo != 0; ++m) {
      if (sh.img_cnt <= 64) {
        m = __builtin_ctzll(todo);
        todo &= todo - 1;
      }
      const double dx = x - c[3 * m], dy = y - c[3 * m + 1], dz = z - c[3 * m + 2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (sh.alpha * r2 <= lat.ln_inv_tau) {
        const double g = sh.norm * exp(-sh.alpha * r2);
        if (sh.l == 0) {
          v[0] += g;
        } else if (sh.l == 1) {
          v[0] += g * dx;
          v[1] += g * dy;
          v[2] += g * dz;
        } else {
          constexpr double R3 = 1.7320508075688772;
          v[0] += g * (R3 * dx * dy);
          v[1] += g * (R3 * dy * dz);
          v[2] += g * (dz * dz - 0.5 * (dx * dx + dy * dy));
          v[3] += g * (R3 * dx * dz);
          v[4] += g * (0.5 * R3 * (dx * dx - dy * dy));
        }
      }
    }
    const int nc = 2 * sh.l + 1;
    double s2 = 0.0, mx = 0.0, sm = 0.0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      if (q < nc) {
        out[(cs.col + q) * P] = v[q];
        s2 += v[q] * v[q];
        mx = fmax(mx, v[q] * v[q]);
        sm += v[q];
      }
    }
    if (cs.col < d.nL) {
      aL += s2;
      mL = fmax(mL, mx);
      sL += sm;
    } else {
      aN += s2;
    }
  }
  diag[d.diag_off + i] = aL * (aL + 2.0 * aN);
  if (aux) {
    double* a = aux + 4 * (d.diag_off + i);
    a[0] = aL;
    a[1] = aN;
    a[2] = mL;
    a[3] = sL;
  }
}

isdf_status launch_basis_eval(hipStream_t s, const LatticeArg& lat, const ShellDev* shells,
                              const double* img, const ColShell* colshells,
                              const DomainDev* doms, const int32_t* points,
                              const BasisTile* tiles, int ntiles, double* phi, double* diag,
                              double* aux) {
  if (ntiles <= 0) return ISDF_OK;
  hipLaunchKernelGGL(basis_eval_kernel, dim3(ntiles), dim3(256), 0, s, lat, shells, img,
                     colshells, doms, points, tiles, phi, diag, aux);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// ------------------------------------------------------------ wave helpers
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline int wave_min_int(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

// Tile partials: tmax = max residual over active points of the tile (-1 if
// none), tidx = smallest active index with d >= (1 - tau) tmax, and, when
// tval is given, the residual at that index (-1 if none).  The tile's
// points are consecutive indices starting at a multiple of 64, so the lane
// holding index mi is mi mod 64.
__device__ inline void tile_partial(double dv, bool active, int i, double tau, double* tmax,
                                    int32_t* tidx, int tile, double* tval = nullptr) {
  const double v = active ? dv : -1.0;
  const double m = wave_max(v);
  const double thr = (1.0 - tau) * m;
  const int cand = (active && m >= 0.0 && dv >= thr) ? i : INT_MAX;
  const int mi = wave_min_int(cand);
  const double vm = __shfl(dv, mi == INT_MAX ? 0 : (mi & 63), 64);
  if ((threadIdx.x & 63) == 0) {
    tmax[tile] = m;
    tidx[tile] = mi;
    if (tval) tval[tile] = mi == INT_MAX ? -1.0 : vm;
  }
}

__global__ void __launch_bounds__(64)
sel_init_kernel(const SelDomain* __restrict__ doms, const int32_t* __restrict__ tile_dom,
                int tile_base, const double* __restrict__ diag, double* __restrict__ tmax,
                int32_t* __restrict__ tidx, double tau, double* __restrict__ tval) {
  const int tile = tile_base + (int)blockIdx.x;
  const SelDomain D = doms[tile_dom[tile]];
  const int i = (tile - D.tile_off) * SEL_TILE + (int)threadIdx.x;
  const bool valid = i < D.pts;
  const double dv = valid ? diag[D.diag_off + i] : -1.0;
  tile_partial(dv, valid && dv >= 0.0, i, tau, tmax, tidx, tile, tval);
}

isdf_status launch_sel_init(hipStream_t s, const SelDomain* doms, const int32_t* tile_dom,
                            int tile_base, int ntiles, const double* diag, double* tmax,
                            int32_t* tidx, double tau, double* tval) {
  if (ntiles <= 0) return ISDF_OK;
  hipLaunchKernelGGL(sel_init_kernel, dim3(ntiles), dim3(64), 0, s, doms, tile_dom, tile_base,
                     diag, tmax, tidx, tau, tval);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// One workgroup per domain: pick the pivot of step k, or stop.
__global__ void __launch_bounds__(256)
sel_select_kernel(const SelDomain* __restrict__ doms, int dom_base, int k, SelState* __restrict__ st,
                  const double* __restrict__ phi, const double* __restrict__ lfac,
                  double* __restrict__ diag, const double* __restrict__ tmax,
                  const int32_t* __restrict__ tidx, double* __restrict__ prow,
                  int32_t* __restrict__ piv, double tau, double eps) {
  const int dom = dom_base + (int)blockIdx.x;
  const SelDomain D = doms[dom];
  __shared__ double s_red[256];
  __shared__ int s_redi[256];
  __shared__ int s_p;
  __shared__ int s_stop;
  if (st[dom].done) return;
  const int tid = threadIdx.x;
  if (k >= D.n_mu) {
    if (tid == 0) {
      st[dom].done = 1;
      st[dom].count = k;
      st[dom].reason = SEL_END_COUNT;
    }
    return;
  }
  // global max over the domain's tiles
  double m = -1.0;
  for (int t = tid; t < D.ntiles; t += 256) m = fmax(m, tmax[D.tile_off + t]);
  s_red[tid] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) s_red[tid] = fmax(s_red[tid], s_red[tid + o]);
    __syncthreads();
  }
  const double Mstar = s_red[0];
  if (k == 0 && tid == 0) st[dom].d0max = Mstar;
  __syncthreads();
  const double d0max = st[dom].d0max;
  if (Mstar < 0.0) {  // no candidates left
    if (tid == 0) {
      st[dom].done = 1;
      st[dom].count = k;
      st[dom].reason = SEL_END_EPS;
    }
    return;
  }
  const double thr = (1.0 - tau) * Mstar;
  // first tile holding a value >= thr
  int ft = INT_MAX;
  for (int t = tid; t < D.ntiles; t += 256)
    if (tmax[D.tile_off + t] >= thr) ft = min(ft, t);
  s_redi[tid] = ft;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) s_redi[tid] = min(s_redi[tid], s_redi[tid + o]);
    __syncthreads();
  }
  const int t0 = s_redi[0];
  __syncthreads();
  if (t0 == INT_MAX) {  // no finite candidate (non-finite input): stop the domain
    if (tid == 0) {
      st[dom].done = 1;
      st[dom].count = k;
      st[dom].reason = SEL_END_EPS;
    }
    return;
  }
  if (tid < 64) {
    const int i = t0 * SEL_TILE + tid;
    int cand = INT_MAX;
    const int quick = tidx[D.tile_off + t0];
    if (quick != INT_MAX && diag[D.diag_off + quick] >= thr) {
      cand = quick;
    } else if (i < D.pts) {
      const double dv = diag[D.diag_off + i];
      if (dv >= 0.0 && dv >= thr) cand = i;
    }
    cand = wave_min_int(cand);
    if (tid == 0) {
      s_p = cand;
      const double dp = cand == INT_MAX ? 0.0 : diag[D.diag_off + cand];
      s_stop = cand == INT_MAX || !(dp > eps * d0max);
      if (s_stop) {
        st[dom].done = 1;
        st[dom].count = k;
        st[dom].reason = SEL_END_EPS;
      } else {
        st[dom].dpiv = dp;
        st[dom].cur = cand;
        piv[D.piv_off + k] = cand;
      }
    }
  }
  __syncthreads();
  if (s_stop) return;
  const int p = s_p;
  double* pr = prow + D.prow_off;
  const int64_t P = D.pts;
  for (int c = tid; c < D.nG; c += 256) pr[c] = phi[D.phi_off + c * P + p];
  for (int j = tid; j < k; j += 256) pr[D.nG + j] = lfac[D.lfac_off + j * P + p];
  __syncthreads();
  if (tid == 0) diag[D.diag_off + p] = -1.0;  // chosen points leave the candidate set
}

isdf_status launch_sel_select(hipStream_t s, const SelDomain* doms, int dom_base, int ndom,
                              int k, SelState* st, const double* phi, const double* lfac,
                              double* diag, const double* tmax, const int32_t* tidx, double* prow,
                              int32_t* piv, double tau, double eps) {
  if (ndom <= 0) return ISDF_OK;
  hipLaunchKernelGGL(sel_select_kernel, dim3(ndom), dim3(256), 0, s, doms, dom_base, k, st, phi,
                     lfac, diag, tmax, tidx, prow, piv, tau, eps);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// 64 points per workgroup; the four waves split the basis columns and the
// factor columns, then wave 0 finishes the points.
__global__ void __launch_bounds__(256)
sel_column_kernel(const SelDomain* __restrict__ doms, const int32_t* __restrict__ tile_dom,
                  int tile_base, int k, const SelState* __restrict__ st,
                  const double* __restrict__ phi, double* __restrict__ lfac, double* __restrict__ diag,
                  const double* __restrict__ prow, double* __restrict__ tmax,
                  int32_t* __restrict__ tidx, double tau) {
  const int tile = tile_base + (int)blockIdx.x;
  const int dom = tile_dom[tile];
  if (st[dom].done) return;
  const SelDomain D = doms[dom];
  const int lane = threadIdx.x & 63;
  // the wave index is uniform within a wave; said so, the pivot-row values
  // pr[c] below are wave-uniform loads through the scalar cache instead of
  // one vector load per lane
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int i = (tile - D.tile_off) * SEL_TILE + lane;
  const bool valid = i < D.pts;
  const int ii = valid ? i : 0;
  const int64_t P = D.pts;
  const double* pr = prow + D.prow_off;
  const double* ph = phi + D.phi_off + ii;
  double sL = 0.0, sN = 0.0, sc = 0.0;
  {
    int c = w;
    // two iterations per trip: eight loads in flight per wave, the same sums
#pragma unroll 2
    for (; c + 12 < D.nL; c += 16) {
      const double a0 = ph[c * P], a1 = ph[(c + 4) * P], a2 = ph[(c + 8) * P], a3 = ph[(c + 12) * P];
      sL += a0 * pr[c] + a1 * pr[c + 4] + a2 * pr[c + 8] + a3 * pr[c + 12];
    }
    for (; c < D.nL; c += 4) sL += ph[c * P] * pr[c];
#pragma unroll 2
    for (; c + 12 < D.nG; c += 16) {
      const double a0 = ph[c * P], a1 = ph[(c + 4) * P], a2 = ph[(c + 8) * P], a3 = ph[(c + 12) * P];
      sN += a0 * pr[c] + a1 * pr[c + 4] + a2 * pr[c + 8] + a3 * pr[c + 12];
    }
    for (; c < D.nG; c += 4) sN += ph[c * P] * pr[c];
  }
  const double* lf = lfac + D.lfac_off + ii;
  int j = w;
#pragma unroll 2
  for (; j + 12 < k; j += 16) {
    const double b0 = lf[j * P], b1 = lf[(j + 4) * P], b2 = lf[(j + 8) * P], b3 = lf[(j + 12) * P];
    sc += b0 * pr[D.nG + j] + b1 * pr[D.nG + j + 4] + b2 * pr[D.nG + j + 8] + b3 * pr[D.nG + j + 12];
  }
  for (; j < k; j += 4) sc += lf[j * P] * pr[D.nG + j];
  __shared__ double red[3][4][64];
  red[0][w][lane] = sL;
  red[1][w][lane] = sN;
  red[2][w][lane] = sc;
  __syncthreads();
  if (w != 0) return;
  sL = (red[0][0][lane] + red[0][1][lane]) + (red[0][2][lane] + red[0][3][lane]);
  sN = (red[1][0][lane] + red[1][1][lane]) + (red[1][2][lane] + red[1][3][lane]);
  sc = (red[2][0][lane] + red[2][1][lane]) + (red[2][2][lane] + red[2][3][lane]);
  const double col = sL * (sL + 2.0 * sN) - sc;
  const double ell = col / sqrt(st[dom].dpiv);
  double dv = -1.0;
  if (valid) {
    lfac[D.lfac_off + k * P + i] = ell;
    dv = diag[D.diag_off + i];
    if (dv >= 0.0) {
      dv = fmax(dv - ell * ell, 0.0);
      diag[D.diag_off + i] = dv;
    }
  }
  tile_partial(dv, valid && dv >= 0.0, i, tau, tmax, tidx, tile);
}

isdf_status launch_sel_column(hipStream_t s, const SelDomain* doms, const int32_t* tile_dom,
                              int tile_base, int ntiles, int k, const SelState* st,
                              const double* phi, double* lfac, double* diag,
                              const double* prow, double* tmax, int32_t* tidx, double tau) {
  if (ntiles <= 0) return ISDF_OK;
  hipLaunchKernelGGL(sel_column_kernel, dim3(ntiles), dim3(256), 0, s, doms, tile_dom, tile_base,
                     k, st, phi, lfac, diag, prow, tmax, tidx, tau);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// --------------------------------------------------------------- gather X
// Xrows_d (column-major nG x count): Xrows[c + k nG] = Phi_d(piv_k, c);
// X^L / X^N (column-major N_mu x N) receive the same values in the columns
// of the domain's L and N functions.
__global__ void __launch_bounds__(256)
gather_x_kernel(const GatherDom* __restrict__ doms, const double* __restrict__ phi,
                const int32_t* __restrict__ piv, const int32_t* __restrict__ funcs,
                double* __restrict__ xrows, double* __restrict__ XL, double* __restrict__ XN,
                int64_t nmu) {
  const GatherDom D = doms[blockIdx.y];
  const int k = blockIdx.x;
  if (k >= D.count) return;
  const int p = piv[D.piv_off + k];
  const int64_t P = D.pts;
  for (int c = threadIdx.x; c < D.nG; c += blockDim.x) {
    const double v = phi[D.phi_off + c * P + p];
    xrows[D.xrow_off + (int64_t)k * D.nG + c] = v;
    const int64_t f = funcs[D.func_off + c];
    if (c < D.nL)
      XL[f * nmu + D.xoff + k] = v;
    else
      XN[f * nmu + D.xoff + k] = v;
  }
}

isdf_status launch_gather_x(hipStream_t s, const GatherDom* doms, int ndom, int max_rows,
                            const double* phi, const int32_t* piv, const int32_t* funcs,
                            double* xrows, double* XL, double* XN, int64_t nmu) {
  if (ndom <= 0 || max_rows <= 0) return ISDF_OK;
  hipLaunchKernelGGL(gather_x_kernel, dim3(max_rows, ndom), dim3(256), 0, s, doms, phi, piv,
                     funcs, xrows, XL, XN, nmu);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

}  // namespace isdf
