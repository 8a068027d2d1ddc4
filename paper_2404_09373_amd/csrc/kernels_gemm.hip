// FP64 GEMM on the CDNA4 matrix cores (v_mfma_f64_16x16x4f64).
//
// One kernel serves every dense contraction of the path: the Hadamard Gram
// Theta = A_L o (A_L + 2 A_N) (Eq. M(R,R) restricted to the pivots), the
// triangular-solve updates of the least-squares fit (Eq. lsqr), the
// Coulomb-metric products W = dV F^T V (Eq. (xi|xi')) and the exchange
// products of Eq. ints.  Problems are column-major; a launch may carry a
// group of independent problems of different sizes (one per domain).
//
// Tiling: 64 x 64 output tile per 256-thread workgroup, 4 waves in 2 x 2,
// each wave 32 x 32 = 2 x 2 MFMA blocks of 16 x 16, K staged through LDS in
// chunks of 16.  The MFMA is fed B^T as its first operand and A^T as its
// second, so a lane's accumulators hold 16 consecutive rows of one C column:
// stores are contiguous along the column-major leading dimension.
//
// Lane layouts of v_mfma_f64_16x16x4f64 (wave64):
//   operand 1: lane l holds X[i = l % 16][k = l / 16]
//   operand 2: lane l holds Y[k = l / 16][j = l % 16]
//   result   : lane l, register v holds D[i = l / 16 + 4 v][j = l % 16]
#include "common.h"

namespace isdf {

typedef double d4v __attribute__((ext_vector_type(4)));

namespace {
constexpr int BM = 64, BN = 64, BK = 16, PAD = 2;

__device__ inline const GemmProblem* find_problem(const GemmProblem* probs, int nprob, int tile) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile_start <= tile) lo = mid; else hi = mid - 1;
  }
  return probs + lo;
}
}  // namespace

// TAG only separates the instantiations per role (selection Gram, Coulomb
// metric, fit solves, exchange) so that profiles attribute time per role.
template <int EPI, int TAG>
__global__ void __launch_bounds__(256)
gemm_f64_kernel(GemmProblem single, const GemmProblem* __restrict__ probs, int nprob) {
  const GemmProblem* pp = probs ? find_problem(probs, nprob, blockIdx.x) : &single;
  const GemmProblem p = *pp;
  const int tilesM = (p.M + BM - 1) / BM;
  const int local = (int)blockIdx.x - p.tile_start;
  const int tm = local % tilesM;
  const int tn = local / tilesM;
  const int m0 = tm * BM, n0 = tn * BN;
  if (n0 >= p.N) return;
  if (p.lower && m0 + BM <= n0) return;  // tile strictly above the diagonal

  __shared__ double As[BK][BM + PAD];
  __shared__ double Bs[BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  d4v acc[2][2], accN[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
      accN[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
    }

  double ra[4], rb[4];
  for (int k0 = 0; k0 < p.K; k0 += BK) {
    // ---- global -> registers
    if (!p.transA) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = tid & 63, k = (tid >> 6) + 4 * r;
        const int gm = m0 + m, gk = k0 + k;
        ra[r] = (gm < p.M && gk < p.K) ? p.A[(int64_t)gm + (int64_t)gk * p.lda] : 0.0;
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = tid & 15, m = (tid >> 4) + 16 * r;
        const int gm = m0 + m, gk = k0 + k;
        ra[r] = (gm < p.M && gk < p.K) ? p.A[(int64_t)gk + (int64_t)gm * p.lda] : 0.0;
      }
    }
    if (!p.transB) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = tid & 15, n = (tid >> 4) + 16 * r;
        const int gn = n0 + n, gk = k0 + k;
        double v = 0.0;
        if (gn < p.N && gk < p.K) {
          const int64_t kr = p.bidx ? (int64_t)p.bidx[gk] : (int64_t)gk;
          v = p.B[kr + (int64_t)gn * p.ldb];
        }
        rb[r] = v;
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = tid & 63, k = (tid >> 6) + 4 * r;
        const int gn = n0 + n, gk = k0 + k;
        rb[r] = (gn < p.N && gk < p.K) ? p.B[(int64_t)gn + (int64_t)gk * p.ldb] : 0.0;
      }
    }
    __syncthreads();
    // ---- registers -> LDS
    if (!p.transA) {
#pragma unroll
      for (int r = 0; r < 4; ++r) As[(tid >> 6) + 4 * r][tid & 63] = ra[r];
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) As[tid & 15][(tid >> 4) + 16 * r] = ra[r];
    }
    if (!p.transB) {
#pragma unroll
      for (int r = 0; r < 4; ++r) Bs[tid & 15][(tid >> 4) + 16 * r] = rb[r];
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) Bs[(tid >> 6) + 4 * r][tid & 63] = rb[r];
    }
    __syncthreads();
    // ---- MFMA
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      double xb[2], ya[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) xb[b] = Bs[kr][wn * 32 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a) ya[a] = As[kr][wm * 32 + a * 16 + (lane & 15)];
      if (EPI == EPI_THETA) {
        const int kb = k0 + kk * 4;
        if (kb + 4 <= p.kL) {
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[b], ya[a], acc[a][b], 0, 0, 0);
        } else if (kb >= p.kL) {
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
              accN[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[b], ya[a], accN[a][b], 0, 0, 0);
        } else {
          const bool inL = (kb + (lane >> 4)) < p.kL;
          double xL[2], xN[2];
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            xL[b] = inL ? xb[b] : 0.0;
            xN[b] = inL ? 0.0 : xb[b];
          }
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xL[b], ya[a], acc[a][b], 0, 0, 0);
              accN[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xN[b], ya[a], accN[a][b], 0, 0, 0);
            }
        }
      } else {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[b], ya[a], acc[a][b], 0, 0, 0);
      }
    }
  }
  // ---- epilogue: lane holds C(m0 + wm*32 + a*16 + lane%16, n0 + wn*32 + b*16 + lane/16 + 4v)
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int gm = m0 + wm * 32 + a * 16 + (lane & 15);
    if (gm >= p.M) continue;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gn = n0 + wn * 32 + b * 16 + (lane >> 4) + 4 * v;
        if (gn >= p.N) continue;
        double* cp = p.C + (int64_t)gm + (int64_t)gn * p.ldc;
        const double x = acc[a][b][v];
        if (EPI == EPI_THETA) {
          *cp = x * (x + 2.0 * accN[a][b][v]);
        } else if (EPI == EPI_HADAMARD) {
          double y = p.alpha * x * p.E[(int64_t)gm + (int64_t)gn * p.lde];
          if (p.beta != 0.0) y += p.beta * *cp;
          *cp = y;
        } else {
          double y = p.alpha * x;
          if (p.beta != 0.0) y += p.beta * *cp;
          *cp = y;
        }
      }
    }
  }
}

int gemm_tiles(int M, int N) { return ((M + BM - 1) / BM) * ((N + BN - 1) / BN); }

template <int TAG>
static void launch_tag(hipStream_t s, int epi, const GemmProblem& single, const GemmProblem* probs,
                       int nprob, int tiles) {
  if (epi == EPI_THETA)
    hipLaunchKernelGGL((gemm_f64_kernel<EPI_THETA, TAG>), dim3(tiles), dim3(256), 0, s, single, probs,
                       nprob);
  else if (epi == EPI_HADAMARD)
    hipLaunchKernelGGL((gemm_f64_kernel<EPI_HADAMARD, TAG>), dim3(tiles), dim3(256), 0, s, single,
                       probs, nprob);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<EPI_AXPBY, TAG>), dim3(tiles), dim3(256), 0, s, single, probs,
                       nprob);
}

static isdf_status launch(hipStream_t s, int epi, int tag, const GemmProblem& single,
                          const GemmProblem* probs, int nprob, int tiles) {
  if (tiles <= 0) return ISDF_OK;
  if (epi != EPI_AXPBY && epi != EPI_THETA && epi != EPI_HADAMARD) {
    set_error("gemm: bad epilogue");
    return ISDF_E_ARG;
  }
  switch (tag) {
    case 1: launch_tag<1>(s, epi, single, probs, nprob, tiles); break;
    case 2: launch_tag<2>(s, epi, single, probs, nprob, tiles); break;
    case 3: launch_tag<3>(s, epi, single, probs, nprob, tiles); break;
    case 4: launch_tag<4>(s, epi, single, probs, nprob, tiles); break;
    default: launch_tag<0>(s, epi, single, probs, nprob, tiles); break;
  }
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

isdf_status gemm_f64(hipStream_t s, int epi, const GemmProblem& p, int tag) {
  if (p.M <= 0 || p.N <= 0) return ISDF_OK;
  GemmProblem q = p;
  q.tile_start = 0;
  if (p.K <= 0) {
    // empty contraction: C = beta C (or zero); run with K = 0 to apply it
  }
  return launch(s, epi, tag, q, nullptr, 1, gemm_tiles(p.M, p.N));
}

isdf_status gemm_f64_grouped(hipStream_t s, int epi, const GemmProblem* d_probs, int nprob,
                             int total_tiles, int tag) {
  if (nprob <= 0) return ISDF_OK;
  GemmProblem dummy{};
  return launch(s, epi, tag, dummy, d_probs, nprob, total_tiles);
}

}  // namespace isdf
