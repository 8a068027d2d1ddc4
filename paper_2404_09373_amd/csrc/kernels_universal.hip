// Universal grid with every point as a fitting function: the elementwise
// steps of the occ-RI exchange of its diffuse-diffuse pairs (section
// "Building the exchange matrix"; the sinc functions of the sparse grid in
// the Results section).  The Coulomb operator between grid points is
// applied by the batched FFT Poisson passes of kernels_fft.hip; the two
// products with the basis values run on the FP64 GEMM engine.
//
//   E(R, i)  = sum_nu Phi_U(R, nu) C(nu, i)           (GEMM)
//   rho_p(R) = E(R, a_p) E(R, b_p),  p = (a_p <= b_p) pair_density_kernel
//   V_p      = potential of rho_p                     (FFT Poisson)
//   Z(R, i)  = sum_j E(R, j) V_{pair(i, j)}(R)        z_accumulate_rows_kernel,
//              over tiles of pair rows that bound the potentials held
//   K_UU C   = -dV Phi_U^T Z                          (GEMM, row scatter)
// With atom windows fitted as usual, the universal-window cross terms of the
// same K C run on the GEMM engine and their universal rows join Z here.
#include <algorithm>

#include "common.h"

namespace isdf {

// C0[k + i n0] = C[funcs[k] o + i]: rows of the universal domain's functions
// from the row-major N x o coefficients, as an n0 x o column-major block.
__global__ void gather_rows_t_kernel(const double* C, int o, const int32_t* funcs, int n0, double* C0) {
  const int64_t n = (int64_t)n0 * o;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(t % n0), i = (int)(t / n0);
    C0[t] = C[(int64_t)funcs[k] * o + i];
  }
}

isdf_status launch_gather_rows_t(hipStream_t s, const double* C, int o, const int32_t* funcs, int n0,
                                 double* C0) {
  const int64_t n = (int64_t)n0 * o;
  if (n <= 0) return ISDF_OK;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(gather_rows_t_kernel, dim3((unsigned)blocks), dim3(256), 0, s, C, o, funcs, n0, C0);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// KC[funcs[k] o + i] += KC0[k + i n0] (funcs distinct; other rows untouched).
__global__ void scatter_add_rows_kernel(const double* KC0, int n0, int o, const int32_t* funcs, double* KC) {
  const int64_t n = (int64_t)n0 * o;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(t % n0), i = (int)(t / n0);
    KC[(int64_t)funcs[k] * o + i] += KC0[t];
  }
}

isdf_status launch_scatter_add_rows(hipStream_t s, const double* KC0, int n0, int o, const int32_t* funcs,
                                    double* KC) {
  const int64_t n = (int64_t)n0 * o;
  if (n <= 0) return ISDF_OK;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(scatter_add_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, KC0, n0, o, funcs, KC);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// dst[t] = alpha src[t]
__global__ void scale_copy_kernel(const double* src, double* dst, int64_t n, double alpha) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = alpha * src[t];
}

isdf_status launch_scale_copy(hipStream_t s, const double* src, double* dst, int64_t n, double alpha) {
  if (n <= 0) return ISDF_OK;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(scale_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n, alpha);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// Pair densities of `ncols` consecutive pairs, two per complex array in the
// layout of the batched transforms: z[q][R] = (rho_{2q}(R), rho_{2q+1}(R)),
// the imaginary part zero for an odd last column.  pairs[2 p], pairs[2 p + 1]
// = (a_p, b_p).  Grid: x over points, y over complex arrays.
__global__ void pair_density_kernel(const double* __restrict__ E, int64_t ng, const int32_t* __restrict__ pairs,
                                    int ncols, double2* __restrict__ z) {
  const int q = blockIdx.y;
  const int c0 = 2 * q, c1 = 2 * q + 1;
  const int a0 = pairs[2 * c0], b0 = pairs[2 * c0 + 1];
  const bool has1 = c1 < ncols;
  const int a1 = has1 ? pairs[2 * c1] : 0, b1 = has1 ? pairs[2 * c1 + 1] : 0;
  double2* zq = z + (int64_t)q * ng;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < ng; r += (int64_t)gridDim.x * blockDim.x) {
    double2 v;
    v.x = E[r + a0 * ng] * E[r + b0 * ng];
    v.y = has1 ? E[r + a1 * ng] * E[r + b1 * ng] : 0.0;
    zq[r] = v;
  }
}

isdf_status launch_pair_density(hipStream_t s, const double* E, int64_t ng, const int32_t* pairs, int ncols,
                                double* z) {
  if (ncols <= 0) return ISDF_OK;
  const int nq = (ncols + 1) / 2;
  if (nq > 65535) {
    set_error("universal exchange: too many pair densities in one batch");
    return ISDF_E_ARG;
  }
  const int64_t bx = std::min<int64_t>((ng + 255) / 256, 1024);
  hipLaunchKernelGGL(pair_density_kernel, dim3((unsigned)bx, (unsigned)nq), dim3(256), 0, s, E, ng, pairs, ncols,
                     reinterpret_cast<double2*>(z));
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// Z(R, i) += sum over the pairs (a <= b) of rows a0 <= a < a1 that hold i:
// E(R, b) V_ab(R) where a = i, E(R, a) V_ai(R) where a < i.  The pairs of
// the tile are numbered row by row from (a0, a0): row a starts at
// (a - a0) o - (a (a - 1) - a0 (a0 - 1)) / 2.  One thread per point and a
// block of ZB occupied columns (blockIdx.y); within a tile the sum over the
// partner runs in ascending order, and tiles are added in order, so the
// result does not depend on the launch.  Z starts at zero.
constexpr int ZB = 8;
__global__ void z_accumulate_rows_kernel(const double* __restrict__ E, const double* __restrict__ V, int64_t ng,
                                         int o, int a0, int a1, double* __restrict__ Z) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= ng) return;
  const int i0 = blockIdx.y * ZB;
  auto row0 = [&](int64_t a) -> int64_t {
    return (a - a0) * o - (a * (a - 1) - (int64_t)a0 * (a0 - 1)) / 2;
  };
#pragma unroll
  for (int t = 0; t < ZB; ++t) {
    const int i = i0 + t;
    if (i >= o || i < a0) continue;
    double acc = 0.0;
    const int amax = i < a1 ? i : a1;
    for (int a = a0; a < amax; ++a)  // pairs (a, i), a < i
      acc += E[r + (int64_t)a * ng] * V[(row0(a) + (i - a)) * ng + r];
    if (i < a1) {  // pairs (i, b), b >= i
      const int64_t base = row0(i);
      for (int b = i; b < o; ++b) acc += E[r + (int64_t)b * ng] * V[(base + (b - i)) * ng + r];
    }
    Z[r + (int64_t)i * ng] += acc;
  }
}

isdf_status launch_z_accumulate_rows(hipStream_t s, const double* E, const double* V, int64_t ng, int o, int a0,
                                     int a1, double* Z) {
  if (ng <= 0 || o <= 0 || a1 <= a0) return ISDF_OK;
  const int64_t bx = (ng + 255) / 256;
  const int by = (o + ZB - 1) / ZB;
  if (bx > 0x7fffffff || by > 65535) {
    set_error("universal exchange: grid or occupied count too large");
    return ISDF_E_UNSUPPORTED;
  }
  hipLaunchKernelGGL(z_accumulate_rows_kernel, dim3((unsigned)bx, (unsigned)by), dim3(256), 0, s, E, V, ng, o, a0,
                     a1, Z);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

}  // namespace isdf
