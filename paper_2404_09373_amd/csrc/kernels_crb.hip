// Candidate-restricted blocked pivoted Cholesky for a domain that is alone on
// its level (the universal grid): the greedy selection of the Interpolative
// decomposition section (Eq. M(R,R)) over many points with many pivots.
//
// A block starts from the exact residual diagonal d.  Its candidates C are
// the T points of largest d (ties at the cut included); theta is the largest
// d outside C.  Residual diagonals never grow, so as long as every pivot of
// the block has d > theta / (1 - tie_tol), no point outside C can be the
// maximum or enter a tie window: the greedy steps restricted to C are the
// greedy steps over all points.  The block runs on the small residual
// R_CC = M(C, C) - L(C, :) L(C, :)^T until that test (or the eps/count stop)
// ends it; then the block's factor columns of every point follow in bulk,
//   L(:, blk) = (M(:, P) - L(:, :kb) L(P, :kb)^T) U^{-T},  U = L(P, blk),
// and d loses their squares.  The next block starts over from the new d.
#include <climits>

#include "common.h"

namespace isdf {

namespace {
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline int wave_min_int(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline uint64_t dkey(double v) {  // order-preserving key of v >= 0
  return (uint64_t)__double_as_longlong(v);
}

template <typename T, typename Op>
__device__ inline T block_reduce(T v, T* red, Op op) {
  for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  T r = red[0];
  for (int i = 1; i < nw; ++i) r = op(r, red[i]);
  return r;
}
}  // namespace

// One workgroup of 1024 threads.  Active points: d >= 0 (chosen points hold
// -1).  Candidates: the T largest active d, ties at the cut included, listed
// in ascending point order (the tie rule's order) with their d.  The cut is
// the largest key with at least T active keys at or above it, found most
// significant bit first; each thread keeps the keys of its first CAND_KPT
// points in registers across the passes.  Once exactly T keys lie at or
// above the cut, lower bits can change neither the set nor theta, and the
// search stops.
constexpr int CAND_KPT = 32;
__global__ void __launch_bounds__(1024)
crb_candidates_kernel(const double* __restrict__ d, int n, int T, int32_t* __restrict__ cidx,
                      double* __restrict__ dC, CrbInfo* __restrict__ info) {
  __shared__ uint64_t red_u[16];
  __shared__ double red_d[16];
  __shared__ int32_t scan[1024];
  const int tid = threadIdx.x;
  auto add = [](uint64_t a, uint64_t b) { return a + b; };
  auto dmaxf = [](double a, double b) { return fmax(a, b); };
  // keys (0 for chosen points: never counted, since every trial key is >= 1),
  // active count and largest d
  uint64_t kr[CAND_KPT];
  uint32_t act = 0;  // bit j: register key j belongs to an active point
  uint64_t na = 0;
  double dm = -1.0;
#pragma unroll
  for (int j = 0; j < CAND_KPT; ++j) {
    const int i = tid + j * 1024;
    uint64_t key = 0;
    if (i < n) {
      const double v = d[i];
      if (v >= 0.0) {
        key = dkey(v);
        act |= 1u << j;
        ++na;
        dm = fmax(dm, v);
      }
    }
    kr[j] = key;
  }
  for (int i = tid + CAND_KPT * 1024; i < n; i += 1024) {
    const double v = d[i];
    if (v >= 0.0) {
      ++na;
      dm = fmax(dm, v);
    }
  }
  na = block_reduce<uint64_t>(na, red_u, add);
  dm = block_reduce<double>(dm, red_d, dmaxf);
  uint64_t cut = 0;
  if (na > (uint64_t)T) {
    for (int b = 63; b >= 0; --b) {
      const uint64_t trial = cut | (1ull << b);
      uint64_t c = 0;
#pragma unroll
      for (int j = 0; j < CAND_KPT; ++j) c += kr[j] >= trial ? 1 : 0;
      for (int i = tid + CAND_KPT * 1024; i < n; i += 1024) {
        const double v = d[i];
        c += (v >= 0.0 && dkey(v) >= trial) ? 1 : 0;
      }
      c = block_reduce<uint64_t>(c, red_u, add);
      if (c >= (uint64_t)T) {
        cut = trial;
        if (c == (uint64_t)T) break;
      }
    }
  }
  // largest d below the cut (outside the candidates)
  double th = -1.0;
  if (na > (uint64_t)T) {
#pragma unroll
    for (int j = 0; j < CAND_KPT; ++j)
      if (((act >> j) & 1u) && kr[j] < cut) th = fmax(th, __longlong_as_double((long long)kr[j]));
    for (int i = tid + CAND_KPT * 1024; i < n; i += 1024) {
      const double v = d[i];
      if (v >= 0.0 && dkey(v) < cut) th = fmax(th, v);
    }
  }
  th = block_reduce<double>(th, red_d, dmaxf);
  // compaction in point order: thread t owns a contiguous chunk
  const int chunk = (n + 1023) / 1024;
  const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
  int cnt = 0;
  for (int i = lo; i < hi; ++i) {
    const double v = d[i];
    cnt += (v >= 0.0 && dkey(v) >= cut) ? 1 : 0;
  }
  scan[tid] = cnt;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan
    const int add_v = tid >= o ? scan[tid - o] : 0;
    __syncthreads();
    scan[tid] += add_v;
    __syncthreads();
  }
  int pos = scan[tid] - cnt;
  for (int i = lo; i < hi; ++i) {
    const double v = d[i];
    if (v >= 0.0 && dkey(v) >= cut) {
      cidx[pos] = i;
      dC[pos] = v;
      ++pos;
    }
  }
  if (tid == 1023) {
    info->nc = scan[1023];
    info->nactive = (int32_t)na;
    info->theta = th;
    info->dmax = dm;
  }
}

isdf_status launch_crb_candidates(hipStream_t s, const double* d, int n, int T, int32_t* cidx,
                                  double* dC, CrbInfo* info) {
  if (n <= 0 || T <= 0) {
    set_error("crb: empty domain or candidate budget");
    return ISDF_E_ARG;
  }
  hipLaunchKernelGGL(crb_candidates_kernel, dim3(1), dim3(1024), 0, s, d, n, T, cidx, dC, info);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// One greedy step of a block on the candidates, pick and column in one
// launch.  Every workgroup redoes the pick of step k from the tile maxima of
// step k - 1 (all get the same pivot), then forms the column on its own
// 64-candidate tile; the diagonal, the tile maxima, the tiles' tie
// candidates and their residuals alternate between two copies, so no
// workgroup reads what another one writes in this launch.  Stops as the
// separate pick does (count, eps, block threshold); workgroup 0 records the
// state.  The pick is a chain of dependent reads; it is kept short: the
// done flag and the tile maxima are read together, the maxima stay in
// registers for the first-tile search, and the pivot's residual comes with
// its tile's candidate instead of from a read of the diagonal (the tile is
// scanned only when its own candidate lies below the global tie window).
__global__ void __launch_bounds__(256)
crb_step_kernel(int k, CrbBlock blk) {
  __shared__ double s_red[4];
  __shared__ int s_redi[4];
  __shared__ int s_cand;
  __shared__ double s_dp;
  __shared__ double red[4][64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  SelState* __restrict__ st = blk.st;
  const int nb = blk.nb, nc = blk.nc, c = k & 1;
  const double* __restrict__ R = blk.R;
  double* __restrict__ Lb = blk.Lb;
  const double* __restrict__ dcur = blk.d[c];
  double* __restrict__ dnext = blk.d[c ^ 1];
  const double* __restrict__ tcur = blk.t[c];
  const int32_t* __restrict__ icur = blk.i[c];
  const double* __restrict__ vcur = blk.v[c];
  double* __restrict__ tnext = blk.t[c ^ 1];
  int32_t* __restrict__ inext = blk.i[c ^ 1];
  double* __restrict__ vnext = blk.v[c ^ 1];
  int32_t* __restrict__ pivC = blk.pivC;
  const double tau = blk.tau, eps = blk.eps, dstop = blk.dstop, d0max = blk.d0max;
  const int ntiles = (nc + SEL_TILE - 1) / SEL_TILE;
  const int done = st->done;
  const double t_own = tid < ntiles ? tcur[tid] : -1.0;
  if (done) return;
  // ---- pick
  int reason = 0, p = INT_MAX;
  double dp = 0.0;
  if (k >= nb) {
    reason = SEL_END_COUNT;
  } else {
    double m = t_own;
    for (int t = tid + 256; t < ntiles; t += 256) m = fmax(m, tcur[t]);
    m = wave_max(m);
    if (lane == 0) s_red[w] = m;
    __syncthreads();
    const double Mstar = fmax(fmax(s_red[0], s_red[1]), fmax(s_red[2], s_red[3]));
    if (Mstar < 0.0) {
      reason = SEL_END_EPS;
    } else {
      const double thr = (1.0 - tau) * Mstar;
      int ft = (tid < ntiles && t_own >= thr) ? tid : INT_MAX;
      for (int t = tid + 256; t < ntiles; t += 256)
        if (tcur[t] >= thr) ft = min(ft, t);
      ft = wave_min_int(ft);
      if (lane == 0) s_redi[w] = ft;
      __syncthreads();
      const int t0 = min(min(s_redi[0], s_redi[1]), min(s_redi[2], s_redi[3]));
      if (t0 == INT_MAX) {
        reason = SEL_END_EPS;
      } else {
        if (w == 0) {
          const int quick = icur[t0];
          const double qv = vcur[t0];
          int cand;
          double cv;
          if (quick != INT_MAX && qv >= thr) {
            cand = quick;
            cv = qv;
          } else {
            const int i = t0 * SEL_TILE + lane;
            const double dv = i < nc ? dcur[i] : -1.0;
            cand = wave_min_int((i < nc && dv >= 0.0 && dv >= thr) ? i : INT_MAX);
            cv = __shfl(dv, cand == INT_MAX ? 0 : (cand & 63), 64);
          }
          if (lane == 0) {
            s_cand = cand;
            s_dp = cand == INT_MAX ? 0.0 : cv;
          }
        }
        __syncthreads();
        p = s_cand;
        dp = s_dp;
        if (p == INT_MAX || !(dp > eps * d0max)) reason = SEL_END_EPS;
        else if (!(dp > dstop)) reason = SEL_END_BLOCK;
      }
    }
  }
  if (reason) {
    if (blockIdx.x == 0 && tid == 0) {
      st->done = 1;
      st->count = k;
      st->reason = reason;
    }
    return;
  }
  if (blockIdx.x == 0 && tid == 0) {
    st->d0max = d0max;
    st->dpiv = dp;
    st->cur = p;
    pivC[k] = p;
  }
  // ---- column on this workgroup's tile: 4 waves split the block's columns
  const int i = blockIdx.x * SEL_TILE + lane;
  const bool valid = i < nc;
  const int ii = valid ? i : 0;
  const int64_t P = nc;
  // the pivot row of the residual and the old diagonal do not depend on the
  // column sum: their reads go out first
  double rv = 0.0, old = -1.0;
  if (w == 0) {
    rv = (ii >= p) ? R[ii + (int64_t)p * P] : R[p + (int64_t)ii * P];
    old = dcur[ii];
  }
  double sc = 0.0;
  const double* lf = Lb + ii;
  const double* lp = Lb + p;
  int j = w;
  for (; j + 12 < k; j += 16) {
    sc += lf[j * P] * lp[j * P] + lf[(j + 4) * P] * lp[(j + 4) * P] + lf[(j + 8) * P] * lp[(j + 8) * P] +
          lf[(j + 12) * P] * lp[(j + 12) * P];
  }
  for (; j < k; j += 4) sc += lf[j * P] * lp[j * P];
  red[w][lane] = sc;
  __syncthreads();
  if (w != 0) return;
  sc = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
  const double ell = (rv - sc) / sqrt(dp);
  double dv = -1.0;
  if (valid) {
    Lb[(int64_t)k * P + i] = ell;
    dv = (i == p) ? -1.0 : (old >= 0.0 ? fmax(old - ell * ell, 0.0) : old);
    dnext[i] = dv;
  }
  // tile maximum, the smallest index in its tie window and its residual
  const bool act = valid && dv >= 0.0;
  const double tm = wave_max(act ? dv : -1.0);
  const int cnd = (act && tm >= 0.0 && dv >= (1.0 - tau) * tm) ? i : INT_MAX;
  const int mi = wave_min_int(cnd);
  const double vm = __shfl(dv, mi == INT_MAX ? 0 : (mi & 63), 64);
  if (lane == 0) {
    tnext[blockIdx.x] = tm;
    inext[blockIdx.x] = mi;
    vnext[blockIdx.x] = mi == INT_MAX ? -1.0 : vm;
  }
}

isdf_status launch_crb_step(hipStream_t s, int k, const CrbBlock& b) {
  const int ntiles = (b.nc + SEL_TILE - 1) / SEL_TILE;
  hipLaunchKernelGGL(crb_step_kernel, dim3(ntiles), dim3(256), 0, s, k, b);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// dst[r + c ldd] = src[idx[r] + c lds], r < nr, c < nc
__global__ void __launch_bounds__(256)
crb_gather_kernel(const double* __restrict__ src, int64_t lds, const int32_t* __restrict__ idx, int nr,
                  int nc, double* __restrict__ dst, int64_t ldd) {
  const int c = blockIdx.y;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < nr; r += gridDim.x * 256)
    dst[r + c * ldd] = src[(int64_t)idx[r] + c * lds];
}

isdf_status launch_crb_gather(hipStream_t s, const double* src, int64_t lds, const int32_t* idx, int nr,
                              int nc, double* dst, int64_t ldd) {
  if (nr <= 0 || nc <= 0) return ISDF_OK;
  const int bx = std::min(64, (nr + 255) / 256);
  hipLaunchKernelGGL(crb_gather_kernel, dim3(bx, nc), dim3(256), 0, s, src, lds, idx, nr, nc, dst, ldd);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// X[:, jb : jb + nb] <- X[:, jb : jb + nb] U_bb^{-T} for the lower-triangular
// diagonal block U_bb = U[jb : jb + nb, jb : jb + nb] (nb <= 64), one row of X
// per thread (forward substitution).
__global__ void __launch_bounds__(256)
crb_trsm_block_kernel(double* __restrict__ X, int64_t ldx, int n, const double* __restrict__ U,
                      int64_t ldu, int jb, int nb) {
  __shared__ double Ub[64][65];
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int q = e % 64, c = e / 64;
    Ub[q][c] = (q < nb && c < nb) ? U[(jb + q) + (int64_t)(jb + c) * ldu] : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double x[64];
  double* xr = X + i + (int64_t)jb * ldx;
#pragma unroll
  for (int q = 0; q < 64; ++q) {
    if (q < nb) {
      double g = xr[(int64_t)q * ldx];
#pragma unroll
      for (int c = 0; c < q; ++c) g -= x[c] * Ub[q][c];
      x[q] = g / Ub[q][q];
      xr[(int64_t)q * ldx] = x[q];
    }
  }
}

isdf_status launch_crb_trsm_block(hipStream_t s, double* X, int64_t ldx, int n, const double* U,
                                  int64_t ldu, int jb, int nb) {
  if (n <= 0 || nb <= 0) return ISDF_OK;
  if (nb > 64) {
    set_error("crb: diagonal block wider than 64");
    return ISDF_E_ARG;
  }
  hipLaunchKernelGGL(crb_trsm_block_kernel, dim3((n + 255) / 256), dim3(256), 0, s, X, ldx, n, U, ldu,
                     jb, nb);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// d(i) <- max(d(i) - sum_q L(i, q)^2, 0) over the block's columns for active
// points; then the block's pivots leave (d = -1).
__global__ void __launch_bounds__(256)
crb_diag_kernel(double* __restrict__ d, int n, const double* __restrict__ L, int64_t ldl, int nb) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double v = d[i];
  if (!(v >= 0.0)) return;
  double a = 0.0;
  for (int q = 0; q < nb; ++q) {
    const double l = L[i + (int64_t)q * ldl];
    a += l * l;
  }
  d[i] = fmax(v - a, 0.0);
}
__global__ void crb_mark_kernel(double* __restrict__ d, const int32_t* __restrict__ piv, int nb) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < nb) d[piv[j]] = -1.0;
}

isdf_status launch_crb_diag(hipStream_t s, double* d, int n, const double* L, int64_t ldl, int nb,
                            const int32_t* piv) {
  if (n <= 0 || nb <= 0) return ISDF_OK;
  hipLaunchKernelGGL(crb_diag_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d, n, L, ldl, nb);
  ISDF_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(crb_mark_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, d, piv, nb);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

}  // namespace isdf
