// FP64 Cholesky and triangular solves of the interpolation metric, plus small
// elementwise / reduction kernels.
//
// Least squares of Eq. lsqr: F = Theta M_xi^{-1} with M_xi = C C^T (Cholesky),
// i.e. two triangular solves G C^T = Theta, F C = G.  Domains with at most 64
// points are fitted by one fused kernel (factor in LDS, one thread per grid
// row for both substitutions); larger ones go through a blocked path whose
// diagonal 64 x 64 blocks are factored and inverted here and whose updates
// run on the MFMA GEMM.
#include "common.h"

namespace isdf {

// ------------------------------------------------------ 64 x 64 block factor
// LDS Cholesky of the w x w block (w <= 64) of M; writes the lower factor to
// Cf (leading dim ldc) and its inverse to inv (leading dim 64).
__device__ void lds_cholesky(double (*a)[65], int w, int32_t* status) {
  const int tid = threadIdx.x;
  for (int j = 0; j < w; ++j) {
    if (tid == 0) {
      double d = a[j][j];
      if (!(d > 0.0)) {
        atomicOr(status, 1);
        d = 1.0;
      }
      a[j][j] = sqrt(d);
    }
    __syncthreads();
    const double djj = a[j][j];
    for (int i = j + 1 + tid; i < w; i += blockDim.x) a[i][j] /= djj;
    __syncthreads();
    // trailing lower triangle: column j + 1 + (tid mod 64), rows strided by
    // the number of 64-thread groups
    const int c = j + 1 + (tid & 63);
    if (c < w) {
      const double acj = a[c][j];
      for (int r = j + 1 + (tid >> 6); r < w; r += (int)blockDim.x >> 6)
        if (r >= c) a[r][c] -= a[r][j] * acj;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256)
potrf_diag_kernel(double* __restrict__ M, int64_t ldm, double* __restrict__ Cf, int64_t ldc,
                  double* __restrict__ inv, int w, int32_t* status) {
  __shared__ double a[64][65];
  __shared__ double x[64][65];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int i = idx & 63, j = idx >> 6;
    a[i][j] = (i < w && j < w) ? M[i + j * ldm] : 0.0;
  }
  __syncthreads();
  lds_cholesky(a, w, status);
  for (int idx = tid; idx < w * w; idx += 256) {
    const int i = idx % w, j = idx / w;
    Cf[i + j * ldc] = (i >= j) ? a[i][j] : 0.0;
  }
  // inverse of the lower factor: L X = I by forward elimination, the rows
  // below each finished row updated by the whole workgroup
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int i = idx & 63, j = idx >> 6;
    x[i][j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    if (tid <= j) x[j][tid] /= a[j][j];  // row j is final (columns <= j)
    __syncthreads();
    const int c = tid & 63;
    if (c <= j) {
      const double xjc = x[j][c];
      for (int r = j + 1 + (tid >> 6); r < w; r += 4) x[r][c] -= a[r][j] * xjc;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int i = idx & 63, j = idx >> 6;
    inv[i + j * 64] = (i < w && j < w) ? x[i][j] : 0.0;
  }
}

isdf_status launch_potrf_diag(hipStream_t s, double* M, int64_t ldm, double* Cf, int64_t ldc,
                              double* inv, int w, int32_t* status) {
  hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, s, M, ldm, Cf, ldc, inv, w,
                     status);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// ------------------------------------------------------- fused small fit
template <int NMAX>
__global__ void __launch_bounds__(256)
small_fit_kernel(const SmallFitDom* __restrict__ doms, const int32_t* __restrict__ tile_dom,
                 const double* __restrict__ theta, const int32_t* __restrict__ piv,
                 double* __restrict__ F, int32_t* status) {
  __shared__ double a[64][65];
  const int tile = blockIdx.x;
  const SmallFitDom D = doms[tile_dom[tile]];
  const int n = D.n;
  const int64_t P = D.pts;
  const double* th = theta + D.theta_off;
  for (int idx = threadIdx.x; idx < n * n; idx += 256) {
    const int i = idx % n, j = idx / n;
    a[i][j] = th[piv[D.piv_off + i] + j * P];  // M_xi(i, j) = Theta(piv_i, j)
  }
  __syncthreads();
  lds_cholesky(a, n, status);
  const int R = (tile - D.row_tile_off) * 256 + (int)threadIdx.x;
  if (R >= D.pts) return;
  double y[NMAX];
  // G C^T = Theta: forward substitution along the row
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    if (j < n) {
      double s = th[R + j * P];
#pragma unroll
      for (int i = 0; i < j; ++i) s -= y[i] * a[j][i];
      y[j] = s / a[j][j];
    }
  }
  // F C = G: backward substitution
#pragma unroll
  for (int jj = NMAX - 1; jj >= 0; --jj) {
    if (jj < n) {
      double s = y[jj];
#pragma unroll
      for (int i = jj + 1; i < NMAX; ++i)
        if (i < n) s -= y[i] * a[i][jj];
      y[jj] = s / a[jj][jj];
    }
  }
  double* f = F + D.theta_off;
#pragma unroll
  for (int j = 0; j < NMAX; ++j)
    if (j < n) f[R + j * P] = y[j];
}

isdf_status launch_small_fit(hipStream_t s, const SmallFitDom* doms, const int32_t* tile_dom,
                             int ntiles, const double* theta, const int32_t* piv, double* F,
                             int32_t* status, int nmax) {
  if (ntiles <= 0) return ISDF_OK;
  if (nmax <= 16)
    hipLaunchKernelGGL(small_fit_kernel<16>, dim3(ntiles), dim3(256), 0, s, doms, tile_dom, theta,
                       piv, F, status);
  else if (nmax <= 32)
    hipLaunchKernelGGL(small_fit_kernel<32>, dim3(ntiles), dim3(256), 0, s, doms, tile_dom, theta,
                       piv, F, status);
  else
    hipLaunchKernelGGL(small_fit_kernel<64>, dim3(ntiles), dim3(256), 0, s, doms, tile_dom, theta,
                       piv, F, status);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// ------------------------------------------------------------ small helpers
__global__ void fill_kernel(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void narrow_kernel(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
isdf_status launch_narrow(hipStream_t s, const double* x, float* y, int64_t n) {
  if (n <= 0) return ISDF_OK;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, y, n);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

isdf_status launch_fill(hipStream_t s, double* p, int64_t n, double v) {
  if (n <= 0) return ISDF_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// p(i, i) = v for i < n (column-major, leading dimension ld)
__global__ void set_diag_kernel(double* p, int64_t ld, int n, double v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i + (int64_t)i * ld] = v;
}
isdf_status launch_set_diag(hipStream_t s, double* p, int64_t ld, int n, double v) {
  if (n <= 0) return ISDF_OK;
  const int blocks = std::min((n + 255) / 256, 4096);
  hipLaunchKernelGGL(set_diag_kernel, dim3(blocks), dim3(256), 0, s, p, ld, n, v);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// dst(i, c) = alpha src(idx ? idx[i] : i, c), i < rows, c < cols
// (column-major, leading dimensions lds and ldd)
__global__ void __launch_bounds__(256)
scale_rows_kernel(const double* __restrict__ src, int64_t lds, const int32_t* __restrict__ idx, int rows,
                  double alpha, double* __restrict__ dst, int64_t ldd) {
  const int64_t c = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += gridDim.x * blockDim.x)
    dst[i + c * ldd] = alpha * src[(idx ? idx[i] : i) + c * lds];
}
isdf_status launch_scale_rows(hipStream_t s, const double* src, int64_t lds, const int32_t* idx, int rows,
                              int cols, double alpha, double* dst, int64_t ldd) {
  if (rows <= 0 || cols <= 0) return ISDF_OK;
  const int bx = std::min((rows + 255) / 256, 64);
  hipLaunchKernelGGL(scale_rows_kernel, dim3(bx, cols), dim3(256), 0, s, src, lds, idx, rows, alpha, dst, ldd);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// ------------------------------------------------ density screening helpers
// out(b, j) = max over rows r of tile b (block consecutive rows) of |A(r, j)|
// (A column-major m x n, lda; out column-major nt x n)
__global__ void __launch_bounds__(256)
tile_absmax_kernel(const double* __restrict__ A, int64_t lda, int m, int block, int nt,
                   double* __restrict__ out) {
  const int b = blockIdx.x, j = blockIdx.y;
  const int r0 = b * block, r1 = min(m, r0 + block);
  __shared__ double red[256];
  double v = 0.0;
  for (int r = r0 + (int)threadIdx.x; r < r1; r += 256) v = fmax(v, fabs(A[r + (int64_t)j * lda]));
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b + (int64_t)j * nt] = red[0];
}
isdf_status launch_tile_absmax(hipStream_t s, const double* A, int64_t lda, int m, int n, int block,
                               double* out) {
  if (m <= 0 || n <= 0) return ISDF_OK;
  const int nt = (m + block - 1) / block;
  hipLaunchKernelGGL(tile_absmax_kernel, dim3(nt, n), dim3(256), 0, s, A, lda, m, block, nt, out);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// out(b, c) = max |W| over tile (b, c) of a symmetric m x m W (FP64 or FP32)
__global__ void __launch_bounds__(256)
tile_absmax_w_kernel(const double* __restrict__ W, const float* __restrict__ W32, int64_t ld, int m,
                     int block, int nt, double* __restrict__ out) {
  const int b = blockIdx.x, c = blockIdx.y;
  const int r0 = b * block, r1 = min(m, r0 + block), c0 = c * block, c1 = min(m, c0 + block);
  const int h = r1 - r0, w = c1 - c0;
  __shared__ double red[256];
  double v = 0.0;
  for (int e = (int)threadIdx.x; e < h * w; e += 256) {
    const int64_t i = (int64_t)(r0 + e % h) + (int64_t)(c0 + e / h) * ld;
    v = fmax(v, W32 ? fabs((double)W32[i]) : fabs(W[i]));
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b + (int64_t)c * nt] = red[0];
}
isdf_status launch_tile_absmax_w(hipStream_t s, const double* W, const float* W32, int64_t ld, int m, int block,
                                 double* out) {
  if (m <= 0) return ISDF_OK;
  const int nt = (m + block - 1) / block;
  hipLaunchKernelGGL(tile_absmax_w_kernel, dim3(nt, nt), dim3(256), 0, s, W, W32, ld, m, block, nt, out);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// mask[i] = B[i] >= tau
__global__ void __launch_bounds__(256)
mask_ge_kernel(const double* __restrict__ B, int64_t n, double tau, uint8_t* __restrict__ mask) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    mask[i] = B[i] >= tau ? 1 : 0;
}
isdf_status launch_mask_ge(hipStream_t s, const double* B, int64_t n, double tau, uint8_t* mask) {
  if (n <= 0) return ISDF_OK;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(mask_ge_kernel, dim3((unsigned)blocks), dim3(256), 0, s, B, n, tau, mask);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

__global__ void add_kernel(const double* a, const double* b, double* c, int64_t n, double sb) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    c[i] = a[i] + sb * b[i];
}
static isdf_status launch_add_scaled(hipStream_t s, const double* a, const double* b, double* c, int64_t n,
                                     double sb) {
  if (n <= 0) return ISDF_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(add_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, b, c, n, sb);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}
isdf_status launch_add(hipStream_t s, const double* a, const double* b, double* c, int64_t n) {
  return launch_add_scaled(s, a, b, c, n, 1.0);
}
isdf_status launch_sub(hipStream_t s, const double* a, const double* b, double* c, int64_t n) {
  return launch_add_scaled(s, a, b, c, n, -1.0);
}

// C(m, n) = c (c + 2 t) with c = C(m, n) (ldc) and t = T(m, n) (ldt = M;
// t = 0 when T is null): the Hadamard Gram of Eq. M(R,R) from its two parts
// a_L (in C) and a_N (in T).
__global__ void theta_combine_kernel(double* C, int64_t ldc, const double* T, int M, int N) {
  const int64_t n_all = (int64_t)M * N;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n_all;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(t % M), n = (int)(t / M);
    double* c = C + m + (int64_t)n * ldc;
    const double x = *c;
    *c = x * (x + 2.0 * (T ? T[t] : 0.0));
  }
}
isdf_status launch_theta_combine(hipStream_t s, double* C, int64_t ldc, const double* T, int M, int N) {
  const int64_t n_all = (int64_t)M * N;
  if (n_all <= 0) return ISDF_OK;
  const int64_t blocks = std::min<int64_t>((n_all + 255) / 256, 65536);
  hipLaunchKernelGGL(theta_combine_kernel, dim3((unsigned)blocks), dim3(256), 0, s, C, ldc, T, M, N);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// M(i, j) = Theta(piv_i, j), n x n column-major
__global__ void gather_square_kernel(const double* theta, int64_t pts, int n, const int32_t* piv,
                                     double* M) {
  const int j = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += blockDim.x) M[i + (int64_t)j * n] = theta[piv[i] + (int64_t)j * pts];
}
isdf_status launch_gather_square(hipStream_t s, const double* theta, int64_t pts, int n,
                                 const int32_t* piv, double* M) {
  if (n <= 0) return ISDF_OK;
  hipLaunchKernelGGL(gather_square_kernel, dim3(n), dim3(256), 0, s, theta, pts, n, piv, M);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// W symmetrisation: entries of two same-level xi are formed in both orders
// and averaged; a coarser-row entry is mirrored to its finer-row partner.
__global__ void symmetrize_w_kernel(double* W, int64_t nmu, const int8_t* lev, const int32_t* dom) {
  const int64_t j = blockIdx.x;
  for (int64_t i = threadIdx.x; i < j; i += blockDim.x) {
    const int li = lev[i], lj = lev[j];
    double* wij = W + i + j * nmu;
    double* wji = W + j + i * nmu;
    if (li == lj && dom[i] == dom[j]) {  // one domain's block: both orders formed
      const double m = 0.5 * (*wij + *wji);
      *wij = m;
      *wji = m;
    } else if (li <= lj) {  // the row of the lower level (or lower domain) was formed
      *wji = *wij;
    } else {
      *wij = *wji;
    }
  }
}
isdf_status launch_symmetrize_w(hipStream_t s, double* W, int64_t nmu, const int8_t* lev, const int32_t* dom) {
  if (nmu <= 1) return ISDF_OK;
  hipLaunchKernelGGL(symmetrize_w_kernel, dim3((unsigned)nmu), dim3(256), 0, s, W, nmu, lev, dom);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// sum_i a_i b_i with a fixed-order tree (deterministic)
__global__ void dot_partial_kernel(const double* a, const double* b, int64_t n, double* partial) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += a[i] * b[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}
__global__ void dot_final_kernel(const double* partial, int nblk, double* out) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) acc += partial[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}
isdf_status launch_trace_dot(hipStream_t s, const double* a, const double* b, int64_t n,
                             double* partial, int nblk, double* out) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(nblk), dim3(256), 0, s, a, b, n, partial);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(256), 0, s, partial, nblk, out);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

}  // namespace isdf
