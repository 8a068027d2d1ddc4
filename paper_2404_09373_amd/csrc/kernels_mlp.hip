// Learned candidate pruning for the pivoted-Cholesky selection.
//
// A 16 -> 64 -> 64 -> 1 network (ReLU, ReLU, sigmoid; FP32) scores every grid
// point of a domain from 16 local features; the best-scoring points form the
// candidate set over which the greedy pivoted Cholesky of the Interpolative
// decomposition section runs.  Feature definitions, parameter packing and
// the weighted cross-entropy loss match oracle/mlp.py.
//
// Kernels: features (from the basis-kernel side outputs and the geometry),
// inference, one training step (forward + backward of 32 points per
// workgroup, gradient partials reduced in a fixed order), Adam, per-domain
// score threshold for the top-k, and candidate compaction.
#include <climits>

#include "common.h"

namespace isdf {

// ------------------------------------------------------------- features
__device__ inline double lg10(double x) { return log10(fmax(x, 1e-300)) / 10.0; }

__device__ inline double min_image_dist(const MlpGeom& g, double x, double y, double z, double cx,
                                        double cy, double cz) {
  const double dx = x - cx, dy = y - cy, dz = z - cz;
  double f[3];
  for (int j = 0; j < 3; ++j) {
    f[j] = dx * g.inv[0 * 3 + j] + dy * g.inv[1 * 3 + j] + dz * g.inv[2 * 3 + j];
    f[j] -= rint(f[j]);
  }
  double best = 1e300;
  for (int i = -1; i <= 1; ++i)
    for (int j = -1; j <= 1; ++j)
      for (int k = -1; k <= 1; ++k) {
        const double a = f[0] + i, b = f[1] + j, c = f[2] + k;
        const double vx = a * g.lat[0] + b * g.lat[3] + c * g.lat[6];
        const double vy = a * g.lat[1] + b * g.lat[4] + c * g.lat[7];
        const double vz = a * g.lat[2] + b * g.lat[5] + c * g.lat[8];
        best = fmin(best, sqrt(vx * vx + vy * vy + vz * vz));
      }
  return best;
}

__global__ void __launch_bounds__(256)
features_kernel(MlpGeom g, const MlpDomain* __restrict__ doms, const int32_t* __restrict__ points,
                const BasisTile* __restrict__ tiles, const double* __restrict__ aux,
                const double* __restrict__ diag, const double* __restrict__ atoms,
                float* __restrict__ feats) {
  const BasisTile t = tiles[blockIdx.x];
  const MlpDomain D = doms[t.domain];
  const int i = t.start + (int)threadIdx.x;
  if (i >= D.pts) return;
  const int64_t gi = D.pts_off + i;
  const int flat = points[gi];
  const int n1 = D.grid[0], n2 = D.grid[1], n3 = D.grid[2];
  const int i1 = flat % n1, rem = flat / n1, i2 = rem % n2, i3 = rem / n2;
  const double f1 = (double)i1 / n1, f2 = (double)i2 / n2, f3 = (double)i3 / n3;
  const double x = f1 * g.lat[0] + f2 * g.lat[3] + f3 * g.lat[6];
  const double y = f1 * g.lat[1] + f2 * g.lat[4] + f3 * g.lat[7];
  const double z = f1 * g.lat[2] + f2 * g.lat[5] + f3 * g.lat[8];
  const double aL = aux[4 * gi], aN = aux[4 * gi + 1], mL = aux[4 * gi + 2], sL = aux[4 * gi + 3];
  const double gd = diag[gi];
  double d1 = 1e300, d2 = 1e300;
  for (int a = 0; a < g.n_atoms; ++a) {
    const double dd = min_image_dist(g, x, y, z, atoms[3 * a], atoms[3 * a + 1], atoms[3 * a + 2]);
    if (dd < d1) {
      d2 = d1;
      d1 = dd;
    } else if (dd < d2) {
      d2 = dd;
    }
  }
  if (g.n_atoms == 1) d2 = d1;
  const double own = D.atom >= 0 ? min_image_dist(g, x, y, z, atoms[3 * D.atom], atoms[3 * D.atom + 1],
                                                  atoms[3 * D.atom + 2])
                                 : 0.0;
  float* o = feats + gi * 16;
  o[0] = (float)((double)D.level / (double)(g.n_levels > 1 ? g.n_levels - 1 : 1));
  o[1] = D.atom < 0 ? 1.f : 0.f;
  o[2] = (float)lg10(gd);
  o[3] = (float)(gd / D.gmax);
  o[4] = (float)lg10(aL);
  o[5] = (float)lg10(aN);
  o[6] = (float)lg10(aL + aN);
  o[7] = (float)(mL / fmax(aL, 1e-300));
  o[8] = (float)(own / D.rs);
  o[9] = (float)(d1 / D.rs);
  o[10] = (float)(d2 / D.rs);
  o[11] = (float)sqrt(gd / D.gmax);
  o[12] = (float)(10.0 * D.n_mu / (double)D.pts);
  o[13] = (float)(D.h / D.rs);
  o[14] = (float)(sL * sL / fmax((double)D.nL * aL, 1e-300));
  o[15] = (float)lg10(gd / D.gmean);
}

isdf_status launch_features(hipStream_t s, const MlpGeom& g, const MlpDomain* doms,
                            const int32_t* points, const BasisTile* tiles, int ntiles,
                            const double* aux, const double* diag, const double* atoms,
                            float* feats) {
  if (ntiles <= 0) return ISDF_OK;
  hipLaunchKernelGGL(features_kernel, dim3(ntiles), dim3(256), 0, s, g, doms, points, tiles, aux,
                     diag, atoms, feats);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// per-domain max and mean of the Gram diagonal
__global__ void __launch_bounds__(256)
diag_stats_kernel(MlpDomain* __restrict__ doms, const double* __restrict__ diag) {
  MlpDomain* D = doms + blockIdx.x;
  __shared__ double smax[256], ssum[256];
  double m = 0.0, su = 0.0;
  for (int i = threadIdx.x; i < D->pts; i += 256) {
    const double v = diag[D->pts_off + i];
    m = fmax(m, v);
    su += v;
  }
  smax[threadIdx.x] = m;
  ssum[threadIdx.x] = su;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
      ssum[threadIdx.x] += ssum[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    D->gmax = fmax(smax[0], 1e-300);
    D->gmean = fmax(ssum[0] / (double)D->pts, 1e-300);
  }
}

isdf_status launch_diag_stats(hipStream_t s, MlpDomain* doms, int ndom, const double* diag) {
  if (ndom <= 0) return ISDF_OK;
  hipLaunchKernelGGL(diag_stats_kernel, dim3(ndom), dim3(256), 0, s, doms, diag);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// ---------------------------------------------------------------- network
constexpr int NF = 16, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NF, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH;
static_assert(OFF_B3 + 1 == MLP_NPARAM, "parameter packing");

__device__ inline void load_weights(float* w, const float* __restrict__ gw) {
  for (int j = threadIdx.x; j < MLP_NPARAM; j += blockDim.x) w[j] = gw[j];
}

__global__ void __launch_bounds__(256)
mlp_forward_kernel(const float* __restrict__ gw, const float* __restrict__ X, int64_t n,
                   float* __restrict__ zout) {
  __shared__ float w[MLP_NPARAM];
  load_weights(w, gw);
  __syncthreads();
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  float x[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) x[i] = X[p * NF + i];
  float h1[NH];
#pragma unroll 4
  for (int o = 0; o < NH; ++o) {
    float a = w[OFF_B1 + o];
#pragma unroll
    for (int i = 0; i < NF; ++i) a += w[OFF_W1 + o * NF + i] * x[i];
    h1[o] = fmaxf(a, 0.f);
  }
  float z = w[OFF_B3];
  for (int o = 0; o < NH; ++o) {
    float a = w[OFF_B2 + o];
#pragma unroll
    for (int j = 0; j < NH; ++j) a += w[OFF_W2 + o * NH + j] * h1[j];
    z += w[OFF_W3 + o] * fmaxf(a, 0.f);
  }
  zout[p] = z;
}

isdf_status launch_mlp_forward(hipStream_t s, const float* w, const float* X, int64_t n, float* z) {
  if (n <= 0) return ISDF_OK;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, X, n,
                     z);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// One workgroup: 32 points of the (optionally permuted) batch -> partial
// gradient of sum_p l_p / inv_count and the partial loss.
constexpr int PB = 32;
__global__ void __launch_bounds__(256)
mlp_grad_kernel(const float* __restrict__ gw, const float* __restrict__ X,
                const float* __restrict__ Y, const int32_t* __restrict__ perm, int64_t b0,
                int64_t bn, float pw, float inv_count, float* __restrict__ partial,
                float* __restrict__ loss_partial) {
  extern __shared__ float sm[];
  float* w = sm;                       // MLP_NPARAM
  float* xs = w + MLP_NPARAM + 3;      // PB x NF
  float* h1 = xs + PB * NF;            // PB x NH
  float* h2 = h1 + PB * NH;            // PB x NH, later dH1
  float* dh2 = h2 + PB * NH;           // PB x NH
  float* dz = dh2 + PB * NH;           // PB
  float* ls = dz + PB;                 // PB
  const int tid = threadIdx.x;
  load_weights(w, gw);
  const int64_t q0 = (int64_t)blockIdx.x * PB;
  for (int e = tid; e < PB * NF; e += 256) {
    const int p = e / NF, i = e % NF;
    const int64_t q = q0 + p;
    float v = 0.f;
    if (q < bn) {
      const int64_t src = perm ? perm[b0 + q] : b0 + q;
      v = X[src * NF + i];
    }
    xs[e] = v;
  }
  __syncthreads();
  for (int e = tid; e < PB * NH; e += 256) {
    const int p = e / NH, o = e % NH;
    float a = w[OFF_B1 + o];
    for (int i = 0; i < NF; ++i) a += w[OFF_W1 + o * NF + i] * xs[p * NF + i];
    h1[e] = fmaxf(a, 0.f);
  }
  __syncthreads();
  for (int e = tid; e < PB * NH; e += 256) {
    const int p = e / NH, o = e % NH;
    float a = w[OFF_B2 + o];
    for (int j = 0; j < NH; ++j) a += w[OFF_W2 + o * NH + j] * h1[p * NH + j];
    h2[e] = fmaxf(a, 0.f);
  }
  __syncthreads();
  if (tid < PB) {
    const int p = tid;
    const int64_t q = q0 + p;
    float z = w[OFF_B3];
    for (int j = 0; j < NH; ++j) z += w[OFF_W3 + j] * h2[p * NH + j];
    float g = 0.f, l = 0.f;
    if (q < bn) {
      const int64_t src = perm ? perm[b0 + q] : b0 + q;
      const float y = Y[src];
      const float sp_pos = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)));   // softplus(z)
      const float sp_neg = sp_pos - z;                                // softplus(-z)
      l = pw * y * sp_neg + (1.f - y) * sp_pos;
      const float pr = 1.f / (1.f + expf(-z));
      g = (pw * y * (pr - 1.f) + (1.f - y) * pr) * inv_count;
    }
    dz[p] = g;
    ls[p] = l;
  }
  __syncthreads();
  float* gp = partial + (int64_t)blockIdx.x * MLP_NPARAM;
  // dW3, db3, loss
  if (tid < NH) {
    float a = 0.f;
    for (int p = 0; p < PB; ++p) a += dz[p] * h2[p * NH + tid];
    gp[OFF_W3 + tid] = a;
  } else if (tid == NH) {
    float a = 0.f, l = 0.f;
    for (int p = 0; p < PB; ++p) {
      a += dz[p];
      l += ls[p];
    }
    gp[OFF_B3] = a;
    loss_partial[blockIdx.x] = l;
  }
  for (int e = tid; e < PB * NH; e += 256) {
    const int p = e / NH, j = e % NH;
    dh2[e] = h2[e] > 0.f ? dz[p] * w[OFF_W3 + j] : 0.f;
  }
  __syncthreads();
  // dW2[o][j] = sum_p dh2[p][o] h1[p][j]; db2
  for (int e = tid; e < NH * NH; e += 256) {
    const int o = e / NH, j = e % NH;
    float a = 0.f;
    for (int p = 0; p < PB; ++p) a += dh2[p * NH + o] * h1[p * NH + j];
    gp[OFF_W2 + e] = a;
  }
  if (tid < NH) {
    float a = 0.f;
    for (int p = 0; p < PB; ++p) a += dh2[p * NH + tid];
    gp[OFF_B2 + tid] = a;
  }
  // dH1[p][j] = (sum_o W2[o][j] dh2[p][o]) [h1 > 0]  (into h2's storage)
  for (int e = tid; e < PB * NH; e += 256) {
    const int p = e / NH, j = e % NH;
    float a = 0.f;
    for (int o = 0; o < NH; ++o) a += w[OFF_W2 + o * NH + j] * dh2[p * NH + o];
    h2[e] = h1[e] > 0.f ? a : 0.f;
  }
  __syncthreads();
  // dW1[o][i] = sum_p dH1[p][o] x[p][i]; db1
  for (int e = tid; e < NH * NF; e += 256) {
    const int o = e / NF, i = e % NF;
    float a = 0.f;
    for (int p = 0; p < PB; ++p) a += h2[p * NH + o] * xs[p * NF + i];
    gp[OFF_W1 + e] = a;
  }
  if (tid < NH) {
    float a = 0.f;
    for (int p = 0; p < PB; ++p) a += h2[p * NH + tid];
    gp[OFF_B1 + tid] = a;
  }
}

__global__ void __launch_bounds__(256)
grad_reduce_kernel(const float* __restrict__ partial, int nblk, const float* __restrict__ lpart,
                   float* __restrict__ grad, float* __restrict__ loss) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < MLP_NPARAM) {
    float a = 0.f;
    for (int b = 0; b < nblk; ++b) a += partial[(int64_t)b * MLP_NPARAM + j];
    grad[j] = a;
  }
  if (j == MLP_NPARAM) {
    float a = 0.f;
    for (int b = 0; b < nblk; ++b) a += lpart[b];
    *loss = a;
  }
}

__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= MLP_NPARAM) return;
  const float gj = g[j];
  const float mj = b1 * m[j] + (1.f - b1) * gj;
  const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
  m[j] = mj;
  v[j] = vj;
  w[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

size_t mlp_grad_shmem() {
  return sizeof(float) * (MLP_NPARAM + 3 + PB * NF + 3 * PB * NH + 2 * PB);
}

isdf_status launch_mlp_grad(hipStream_t s, const float* w, const float* X, const float* Y,
                            const int32_t* perm, int64_t b0, int64_t bn, float pw,
                            float inv_count, float* partial, float* lpart, float* grad,
                            float* loss) {
  if (bn <= 0) return ISDF_OK;
  const int nblk = (int)((bn + PB - 1) / PB);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(256), mlp_grad_shmem(), s, w, X, Y, perm, b0,
                     bn, pw, inv_count, partial, lpart);
  hipLaunchKernelGGL(grad_reduce_kernel, dim3((MLP_NPARAM + 256) / 256), dim3(256), 0, s, partial,
                     nblk, lpart, grad, loss);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

isdf_status launch_adam(hipStream_t s, float* w, const float* g, float* m, float* v, float lr,
                        float b1, float b2, float eps, int t) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, w, g, m, v, lr,
                     b1, b2, eps, c1, c2);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// --------------------------------------------------------- top-k per domain
// Order-preserving map of a float score to an unsigned key.
__device__ inline uint32_t fkey(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// One workgroup per domain: the largest key t with #{key >= t} >= k, then the
// ascending list of candidates (key >= t).
__global__ void __launch_bounds__(256)
topk_compact_kernel(const CandDomain* __restrict__ doms, const float* __restrict__ z,
                    float zcut, int32_t* __restrict__ cand, int32_t* __restrict__ ncand,
                    uint8_t* __restrict__ flag) {
  const CandDomain D = doms[blockIdx.x];
  __shared__ int s_cnt[256];
  __shared__ uint32_t s_t;
  const int tid = threadIdx.x;
  const float* zz = z + D.pts_off;
  const int k = D.keep < D.pts ? D.keep : D.pts;
  uint32_t t = 0;
  for (int bit = 31; bit >= 0; --bit) {
    const uint32_t trial = t | (1u << bit);
    int c = 0;
    for (int i = tid; i < D.pts; i += 256) c += fkey(zz[i]) >= trial;
    s_cnt[tid] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) s_cnt[tid] += s_cnt[tid + o];
      __syncthreads();
    }
    if (s_cnt[0] >= k) t = trial;
    __syncthreads();
  }
  // candidates: the k best scores and every score above the cutoff
  if (tid == 0) s_t = min(t, fkey(zcut));
  __syncthreads();
  const uint32_t thr = s_t;
  // ordered compaction: chunks of 256 points, block prefix sum per chunk
  __shared__ int s_scan[256];
  __shared__ int s_base;
  if (tid == 0) s_base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < D.pts; c0 += 256) {
    const int i = c0 + tid;
    const int f = (i < D.pts && fkey(zz[i]) >= thr) ? 1 : 0;
    if (i < D.pts) flag[D.pts_off + i] = (uint8_t)f;
    s_scan[tid] = f;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const int v = tid >= o ? s_scan[tid - o] : 0;
      __syncthreads();
      s_scan[tid] += v;
      __syncthreads();
    }
    if (f) cand[D.cand_off + s_base + s_scan[tid] - 1] = i;
    __syncthreads();
    if (tid == 255) s_base += s_scan[255];
    __syncthreads();
  }
  if (tid == 0) ncand[blockIdx.x] = s_base;
}

isdf_status launch_topk_compact(hipStream_t s, const CandDomain* doms, int ndom, const float* z,
                                float zcut, int32_t* cand, int32_t* ncand, uint8_t* flag) {
  if (ndom <= 0) return ISDF_OK;
  hipLaunchKernelGGL(topk_compact_kernel, dim3(ndom), dim3(256), 0, s, doms, z, zcut, cand, ncand,
                     flag);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// Gather candidate rows of Phi (and the diagonal) into compact domains.
__global__ void __launch_bounds__(256)
gather_rows_kernel(const GatherRows* __restrict__ g, const double* __restrict__ phi,
                   const double* __restrict__ diag, const int32_t* __restrict__ cand,
                   double* __restrict__ phic, double* __restrict__ diagc) {
  const GatherRows G = g[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < G.nc; i += gridDim.x * blockDim.x) {
    const int r = cand[G.cand_off + i];
    for (int c = 0; c < G.nG; ++c)
      phic[G.phic_off + (int64_t)c * G.nc + i] = phi[G.phi_off + (int64_t)c * G.pts + r];
    diagc[G.diagc_off + i] = diag[G.diag_off + r];
  }
}

isdf_status launch_gather_rows(hipStream_t s, const GatherRows* g, int ndom, int max_nc,
                               const double* phi, const double* diag, const int32_t* cand,
                               double* phic, double* diagc) {
  if (ndom <= 0 || max_nc <= 0) return ISDF_OK;
  int blocks = (max_nc + 255) / 256;
  if (blocks > 256) blocks = 256;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks, ndom), dim3(256), 0, s, g, phi, diag, cand,
                     phic, diagc);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// Map candidate-local pivots back to domain-local point indices.
__global__ void map_pivots_kernel(const int32_t* __restrict__ cand, int64_t cand_off,
                                  const int32_t* __restrict__ pivc, int32_t* __restrict__ piv, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) piv[k] = cand[cand_off + pivc[k]];
}
isdf_status launch_map_pivots(hipStream_t s, const int32_t* cand, int64_t cand_off,
                              const int32_t* pivc, int32_t* piv, int n) {
  if (n <= 0) return ISDF_OK;
  hipLaunchKernelGGL(map_pivots_kernel, dim3((n + 255) / 256), dim3(256), 0, s, cand, cand_off, pivc,
                     piv, n);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// Fallback check: final residual of every point, d(R) - sum_j F(R,j) Theta(R,j);
// writes the domain maximum.
__global__ void __launch_bounds__(256)
final_residual_kernel(const JudgeDomain* __restrict__ doms, const double* __restrict__ diag,
                      const double* __restrict__ theta, const double* __restrict__ F,
                      double* __restrict__ out) {
  const JudgeDomain D = doms[blockIdx.x];
  __shared__ double sm[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < D.pts; i += 256) {
    double r = diag[D.diag_off + i];
    for (int j = 0; j < D.n; ++j) r -= F[D.th_off + (int64_t)j * D.pts + i] * theta[D.th_off + (int64_t)j * D.pts + i];
    m = fmax(m, r);
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

isdf_status launch_final_residual(hipStream_t s, const JudgeDomain* doms, int ndom,
                                  const double* diag, const double* theta, const double* F,
                                  double* out) {
  if (ndom <= 0) return ISDF_OK;
  hipLaunchKernelGGL(final_residual_kernel, dim3(ndom), dim3(256), 0, s, doms, diag, theta, F, out);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// Largest initial Gram diagonal over the points left out of a domain's
// candidate set (flag 0): if it is below (1 - tau) times the residual of the
// last pivot, no excluded point could ever have entered the tie window, so
// the restricted greedy selection equals the full one.
__global__ void __launch_bounds__(256)
excluded_max_kernel(const JudgeDomain* __restrict__ doms, const double* __restrict__ diag,
                    const uint8_t* __restrict__ flag, double* __restrict__ out) {
  const JudgeDomain D = doms[blockIdx.x];
  __shared__ double sm[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < D.pts; i += 256)
    if (!flag[D.diag_off + i]) m = fmax(m, diag[D.diag_off + i]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

isdf_status launch_excluded_max(hipStream_t s, const JudgeDomain* doms, int ndom,
                                const double* diag, const uint8_t* flag, double* out) {
  if (ndom <= 0) return ISDF_OK;
  hipLaunchKernelGGL(excluded_max_kernel, dim3(ndom), dim3(256), 0, s, doms, diag, flag, out);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

}  // namespace isdf
