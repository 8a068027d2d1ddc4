// Batched 3D complex FFTs and the FFT Poisson solve of the Coulomb metric
// (Eq. (xi|xi'); "Computational details": one FFT per local fitting function,
// potentials needed on the function's own and on every coarser grid).
//
// Transform: three passes of 1D transforms (x, y, z), each line held in LDS
// and transformed by a Stockham autosort sequence of radix-4/2/3/5 stages
// (compiled per line length for the grids in use, generic otherwise).
// Lines of one workgroup are neighbours along x, so every global access is a
// run of consecutive complex values.  Two real fitting functions travel in
// one complex array (re, im): the Coulomb kernel is real and even in m, so
// the potentials come back as the real and imaginary parts.
//
// Poisson step: a spectrum on grid l' is multiplied by v(m) = 4 pi / |G_m|^2
// on the band J_l = {|m_i| < n_l,i / 2} \ {0} of a grid l <= l' and written
// into grid l's index space (zero elsewhere), ready for the inverse pass.
#include <cmath>

#include <mutex>

#include "common.h"

namespace isdf {

struct FftRadices {
  int32_t n;
  int32_t nrad;
  int32_t r[12];
};

static FftRadices make_radices(int n) {
  FftRadices f{};
  f.n = n;
  int m = n;
  while (m % 4 == 0) { f.r[f.nrad++] = 4; m /= 4; }
  while (m % 2 == 0) { f.r[f.nrad++] = 2; m /= 2; }
  while (m % 3 == 0) { f.r[f.nrad++] = 3; m /= 3; }
  while (m % 5 == 0) { f.r[f.nrad++] = 5; m /= 5; }
  return f;
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// multiply by sign * i
__device__ inline double2 mul_si(double2 a, double sign) { return make_double2(-sign * a.y, sign * a.x); }

template <int R>
__device__ inline void radix_core(const double2* v, double2* y, double sign);

// one radix-R butterfly of a Stockham stage
template <int R>
__device__ inline void butterfly(const double2* src, double2* dst, int n, int j, int Ns,
                                 const double2* tw, double sign) {
  const int k = j % Ns;
  const int stride_in = n / R;
  double2 v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = src[j + r * stride_in];
  const int step = n / (Ns * R);
#pragma unroll
  for (int r = 1; r < R; ++r) {
    double2 w = tw[r * k * step];  // r k step < R Ns n / (Ns R) = n
    if (sign > 0.0) w.y = -w.y;  // the table holds e^{-2 pi i t/n}
    v[r] = cmul(v[r], w);
  }
  double2 y[R];
  radix_core<R>(v, y, sign);
  const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) dst[idxD + r * Ns] = y[r];
}

// the radix-R DFT of v (twiddles applied) into y
template <int R>
__device__ inline void radix_core(const double2* v, double2* y, double sign) {
  if (R == 2) {
    y[0] = cadd(v[0], v[1]);
    y[1] = csub(v[0], v[1]);
  } else if (R == 4) {
    const double2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    const double2 c = cadd(v[1], v[3]), d = mul_si(csub(v[1], v[3]), sign);
    y[0] = cadd(a, c);
    y[2] = csub(a, c);
    y[1] = cadd(b, d);
    y[3] = csub(b, d);
  } else if (R == 3) {
    const double h = 0.86602540378443864676;  // sqrt(3)/2
    const double2 s = cadd(v[1], v[2]);
    const double2 d = mul_si(csub(v[1], v[2]), sign * h);
    const double2 m = make_double2(v[0].x - 0.5 * s.x, v[0].y - 0.5 * s.y);
    y[0] = cadd(v[0], s);
    y[1] = cadd(m, d);
    y[2] = csub(m, d);
  } else if (R == 5) {
    const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;
    const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;
    const double2 p1 = cadd(v[1], v[4]), m1 = csub(v[1], v[4]);
    const double2 p2 = cadd(v[2], v[3]), m2 = csub(v[2], v[3]);
    const double2 a1 = make_double2(v[0].x + c1 * p1.x + c2 * p2.x, v[0].y + c1 * p1.y + c2 * p2.y);
    const double2 a2 = make_double2(v[0].x + c2 * p1.x + c1 * p2.x, v[0].y + c2 * p1.y + c1 * p2.y);
    const double2 b1 = mul_si(make_double2(s1 * m1.x + s2 * m2.x, s1 * m1.y + s2 * m2.y), sign);
    const double2 b2 = mul_si(make_double2(s2 * m1.x - s1 * m2.x, s2 * m1.y - s1 * m2.y), sign);
    y[0] = make_double2(v[0].x + p1.x + p2.x, v[0].y + p1.y + p2.y);
    y[1] = cadd(a1, b1);
    y[4] = csub(a1, b1);
    y[2] = cadd(a2, b2);
    y[3] = csub(a2, b2);
  }
}

__global__ void __launch_bounds__(256)
fft_pass_kernel(double2* __restrict__ z, int batch, int n1, int n2, int n3, int axis, double sign,
                const double2* __restrict__ tw, FftRadices rad, int lpw) {
  extern __shared__ double2 lds[];
  const int n = rad.n;
  double2* bufA = lds;
  double2* bufB = lds + lpw * n;
  const int64_t ng = (int64_t)n1 * n2 * n3;
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  // element (j, i): line j of the group, position i along the axis
  int64_t base;
  int64_t estride;   // stride between positions along the axis
  int64_t lstride;   // stride between lines of the group
  int nlines_here = lpw;
  if (axis == 0) {
    const int64_t nl = (int64_t)n2 * n3 * batch;
    const int64_t L0 = (int64_t)g * lpw;
    if (L0 + lpw > nl) nlines_here = (int)(nl - L0);
    base = L0 * n1;
    estride = 1;
    lstride = n1;
  } else {
    const int groups_x = n1 / lpw;
    const int i10 = (g % groups_x) * lpw;
    const int rest = g / groups_x;
    if (axis == 1) {
      const int i3 = rest % n3, b = rest / n3;
      base = (int64_t)b * ng + i10 + (int64_t)n1 * n2 * i3;
      estride = n1;
    } else {
      const int i2 = rest % n2, b = rest / n2;
      base = (int64_t)b * ng + i10 + (int64_t)n1 * i2;
      estride = (int64_t)n1 * n2;
    }
    lstride = 1;
  }
  const int tot = nlines_here * n;
  if (axis == 0) {
    for (int e = tid; e < tot; e += 256) bufA[e] = z[base + e];
  } else {
    for (int e = tid; e < tot; e += 256) {
      const int j = e % lpw, i = e / lpw;
      bufA[j * n + i] = z[base + j * lstride + i * estride];
    }
  }
  __syncthreads();
  double2* src = bufA;
  double2* dst = bufB;
  int Ns = 1;
  for (int s = 0; s < rad.nrad; ++s) {
    const int R = rad.r[s];
    const int nb = n / R;
    for (int u = tid; u < nlines_here * nb; u += 256) {
      const int line = u / nb, j = u % nb;
      const double2* sl = src + line * n;
      double2* dl = dst + line * n;
      if (R == 4) butterfly<4>(sl, dl, n, j, Ns, tw, sign);
      else if (R == 2) butterfly<2>(sl, dl, n, j, Ns, tw, sign);
      else if (R == 3) butterfly<3>(sl, dl, n, j, Ns, tw, sign);
      else butterfly<5>(sl, dl, n, j, Ns, tw, sign);
    }
    __syncthreads();
    double2* t = src;
    src = dst;
    dst = t;
    Ns *= R;
  }
  if (axis == 0) {
    for (int e = tid; e < tot; e += 256) z[base + e] = src[e];
  } else {
    for (int e = tid; e < tot; e += 256) {
      const int j = e % lpw, i = e / lpw;
      z[base + j * lstride + i * estride] = src[j * n + i];
    }
  }
}

struct PoissonArg {
  int gf[3], gc[3];
  double B[9];   // B[i*3 + j] = component j of reciprocal vector b_i
  double inv_ngf;
};

// v(m) / N_g,f times the fine spectrum at the index of m, for m in the
// band of the coarse grid (m != 0), else 0: the Poisson step of Eq. (xi|xi')
__device__ inline double2 poisson_value(const double2* __restrict__ zf, int64_t fbase, const PoissonArg& a,
                                        int x, int y, int zz) {
  const int j[3] = {x, y, zz};
  int m[3];
  for (int i = 0; i < 3; ++i) {
    m[i] = (j[i] <= (a.gc[i] - 1) / 2) ? j[i] : j[i] - a.gc[i];
    if (2 * abs(m[i]) >= a.gc[i]) return make_double2(0.0, 0.0);
  }
  if ((m[0] | m[1] | m[2]) == 0) return make_double2(0.0, 0.0);
  double G[3];
  for (int c = 0; c < 3; ++c) G[c] = m[0] * a.B[c] + m[1] * a.B[3 + c] + m[2] * a.B[6 + c];
  const double v = 4.0 * 3.14159265358979323846 / (G[0] * G[0] + G[1] * G[1] + G[2] * G[2]) * a.inv_ngf;
  int jf[3];
  for (int i = 0; i < 3; ++i) jf[i] = m[i] < 0 ? m[i] + a.gf[i] : m[i];
  const double2 zv = zf[fbase + jf[0] + (int64_t)a.gf[0] * (jf[1] + (int64_t)a.gf[1] * jf[2])];
  return make_double2(v * zv.x, v * zv.y);
}

// ------------------------------------------------ compile-time line sizes
// The same Stockham sequence with the line length, the radices, the stage
// strides and the lines per workgroup known at compile time: every index
// division becomes a shift or a multiply, which the generic kernel pays for
// at every butterfly.
constexpr int fft_radix(int n, int s) {
  int i = 0;
  while (n % 4 == 0) { if (i == s) return 4; n /= 4; ++i; }
  while (n % 2 == 0) { if (i == s) return 2; n /= 2; ++i; }
  while (n % 3 == 0) { if (i == s) return 3; n /= 3; ++i; }
  while (n % 5 == 0) { if (i == s) return 5; n /= 5; ++i; }
  return 0;
}
constexpr int fft_nstages(int n) {
  int c = 0;
  while (fft_radix(n, c) != 0) ++c;
  return c;
}
constexpr int fft_span(int n, int s) {  // product of the first s radices
  int p = 1;
  for (int i = 0; i < s; ++i) p *= fft_radix(n, i);
  return p;
}

// The Stockham stages of a compiled line length in one LDS buffer: each
// thread reads its butterflies' inputs, the workgroup synchronises, and the
// outputs go back into the same buffer.  Half the LDS of ping-pong buffers,
// so more workgroups (and more lines in flight from HBM) per CU, at two
// barriers a stage instead of one.
template <int N, int S, int NL>
__device__ inline void fft_stages_ip(double2* buf, int nl, const double2* tw, double sign) {
  if constexpr (S < fft_nstages(N)) {
    constexpr int R = fft_radix(N, S), NS = fft_span(N, S), NB = N / R;
    constexpr int UMAX = (NL * NB + 255) / 256;
    constexpr int STEP = N / (NS * R);
    double2 y[UMAX][R];
    int dsto[UMAX];
#pragma unroll
    for (int q = 0; q < UMAX; ++q) {
      const int u = (int)threadIdx.x + 256 * q;
      dsto[q] = -1;
      if (u < nl * NB) {
        const int line = u / NB, j = u % NB, k = j % NS;
        const double2* src = buf + line * N;
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[j + r * NB];
#pragma unroll
        for (int r = 1; r < R; ++r) {
          double2 w = tw[r * k * STEP];
          if (sign > 0.0) w.y = -w.y;
          v[r] = cmul(v[r], w);
        }
        radix_core<R>(v, y[q], sign);
        dsto[q] = line * N + (j / NS) * NS * R + k;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < UMAX; ++q)
      if (dsto[q] >= 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) buf[dsto[q] + r * NS] = y[q][r];
      }
    __syncthreads();
    fft_stages_ip<N, S + 1, NL>(buf, nl, tw, sign);
  }
}

// PLOAD (x pass only): the lines are read from the fine spectrum zf through
// the Poisson step instead of from z.  PSTORE (z pass only): the result is
// written as two real planar columns V[2b], V[2b + 1] of pair b instead of
// back into z (column 2b + 1 only while below ncols).
template <int N, int LPW, bool PLOAD = false, bool PSTORE = false>
__global__ void __launch_bounds__(256)
fft_pass_fixed_kernel(double2* __restrict__ z, int batch, int n1, int n2, int n3, int axis,
                      double sign, const double2* __restrict__ tw,
                      const double2* __restrict__ zf = nullptr, PoissonArg pa = PoissonArg{},
                      double* __restrict__ V = nullptr, int ncols = 0) {
  extern __shared__ double2 lds[];
  double2* bufA = lds;
  const int64_t ng = (int64_t)n1 * n2 * n3;
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  int64_t base, estride, lstride;
  int nl = LPW;
  if (axis == 0) {
    const int64_t nlines = (int64_t)n2 * n3 * batch;
    const int64_t L0 = (int64_t)g * LPW;
    if (L0 + LPW > nlines) nl = (int)(nlines - L0);
    base = L0 * N;
    estride = 1;
    lstride = N;
  } else {
    const int groups_x = n1 / LPW;
    // neighbouring workgroups step along the other strided axis (y for z
    // lines, z for y lines) rather than along x; rest = (that index) +
    // (its extent) * (pair)
    const int nother = axis == 1 ? n3 : n2;
    const int i10 = ((g / nother) % groups_x) * LPW;
    const int rest = (g % nother) + nother * (g / nother / groups_x);
    if (axis == 1) {
      const int i3 = rest % n3, b = rest / n3;
      base = (int64_t)b * ng + i10 + (int64_t)n1 * n2 * i3;
      estride = n1;
    } else {
      const int i2 = rest % n2, b = rest / n2;
      base = (int64_t)b * ng + i10 + (int64_t)n1 * i2;
      estride = (int64_t)n1 * n2;
    }
    lstride = 1;
  }
  const int tot = nl * N;
  if constexpr (PLOAD) {
    const int64_t ngf = (int64_t)pa.gf[0] * pa.gf[1] * pa.gf[2];
    const int64_t L0 = (int64_t)g * LPW;
    for (int e = tid; e < tot; e += 256) {
      const int64_t L = L0 + e / N;  // line (y, z, pair)
      const int y = (int)(L % n2), zz = (int)((L / n2) % n3);
      const int64_t b = L / ((int64_t)n2 * n3);
      bufA[e] = poisson_value(zf, b * ngf, pa, e % N, y, zz);
    }
  } else if (axis == 0) {
    for (int e = tid; e < tot; e += 256) bufA[e] = z[base + e];
  } else {
    for (int e = tid; e < tot; e += 256) {
      const int j = e % LPW, i = e / LPW;
      bufA[j * N + i] = z[base + j * lstride + i * estride];
    }
  }
  __syncthreads();
  fft_stages_ip<N, 0, LPW>(bufA, nl, tw, sign);
  const double2* res = bufA;
  if constexpr (PSTORE) {
    const int b = (g / n2) / (n1 / LPW);
    const int64_t off = base - (int64_t)b * ng;
    double* v0 = V + (int64_t)(2 * b) * ng + off;
    double* v1 = 2 * b + 1 < ncols ? V + (int64_t)(2 * b + 1) * ng + off : nullptr;
    for (int e = tid; e < tot; e += 256) {
      const int j = e % LPW, i = e / LPW;
      const double2 r = res[j * N + i];
      const int64_t o = j * lstride + i * estride;
      v0[o] = r.x;
      if (v1) v1[o] = r.y;
    }
  } else if (axis == 0) {
    for (int e = tid; e < tot; e += 256) z[base + e] = res[e];
  } else {
    for (int e = tid; e < tot; e += 256) {
      const int j = e % LPW, i = e / LPW;
      z[base + j * lstride + i * estride] = res[j * N + i];
    }
  }
}

template <int N>
bool launch_fixed_n(hipStream_t s, double2* z, int batch, int n1, int n2, int n3, int axis,
                    double sign, const double2* tw, int lpw, int64_t groups) {
  const size_t shmem = sizeof(double2) * (size_t)lpw * N;
  if (lpw == 16)
    hipLaunchKernelGGL((fft_pass_fixed_kernel<N, 16>), dim3((unsigned)groups), dim3(256), shmem, s,
                       z, batch, n1, n2, n3, axis, sign, tw);
  else if (lpw == 8)
    hipLaunchKernelGGL((fft_pass_fixed_kernel<N, 8>), dim3((unsigned)groups), dim3(256), shmem, s,
                       z, batch, n1, n2, n3, axis, sign, tw);
  else if (lpw == 4)  // y and z lines of grids whose x extent is 4 mod 8
    hipLaunchKernelGGL((fft_pass_fixed_kernel<N, 4>), dim3((unsigned)groups), dim3(256), shmem, s,
                       z, batch, n1, n2, n3, axis, sign, tw);
  else
    return false;
  return true;
}

// Line lengths with a compiled kernel (the grids of the workloads, and the
// lengths the Fourier-threshold ladders of the diamond cells give).
bool launch_fixed(hipStream_t s, double2* z, int batch, int n1, int n2, int n3, int axis,
                  double sign, const double2* tw, int n, int lpw, int64_t groups) {
  switch (n) {
    case 12: return launch_fixed_n<12>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 18: return launch_fixed_n<18>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 36: return launch_fixed_n<36>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 72: return launch_fixed_n<72>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 100: return launch_fixed_n<100>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 24: return launch_fixed_n<24>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 32: return launch_fixed_n<32>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 40: return launch_fixed_n<40>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 48: return launch_fixed_n<48>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 64: return launch_fixed_n<64>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 80: return launch_fixed_n<80>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 96: return launch_fixed_n<96>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 128: return launch_fixed_n<128>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 144: return launch_fixed_n<144>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 160: return launch_fixed_n<160>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    case 192: return launch_fixed_n<192>(s, z, batch, n1, n2, n3, axis, sign, tw, lpw, groups);
    default: return false;
  }
}

// Line lengths of the fused Poisson / planar passes and of the pruned
// forward transform (every one also has a launch_fixed case).
static bool fused_len(int n) {
  switch (n) {
    case 18: case 24: case 32: case 36: case 40: case 48: case 64: case 72: case 80: case 96: case 128:
    case 144: case 160: case 192:
      return true;
    default:
      return false;
  }
}

static const double2* twiddles(int n);

template <int N>
void launch_poisson_x(hipStream_t s, double2* zc, int batch, const int gc[3], const double2* tw,
                      const double2* zf, const PoissonArg& pa, int64_t groups) {
  hipLaunchKernelGGL((fft_pass_fixed_kernel<N, 8, true, false>), dim3((unsigned)groups), dim3(256),
                     sizeof(double2) * 8 * N, s, zc, batch, gc[0], gc[1], gc[2], 0, 1.0, tw, zf, pa,
                     nullptr, 0);
}
template <int N>
void launch_planar_z(hipStream_t s, double2* zc, int batch, const int gc[3], const double2* tw,
                     double* V, int ncols, int lpw) {
  const int64_t groups = (int64_t)(gc[0] / lpw) * gc[1] * batch;
  if (lpw == 16)
    hipLaunchKernelGGL((fft_pass_fixed_kernel<N, 16, false, true>), dim3((unsigned)groups), dim3(256),
                       sizeof(double2) * 16 * N, s, zc, batch, gc[0], gc[1], gc[2], 2, 1.0, tw, nullptr,
                       PoissonArg{}, V, ncols);
  else
    hipLaunchKernelGGL((fft_pass_fixed_kernel<N, 8, false, true>), dim3((unsigned)groups), dim3(256),
                       sizeof(double2) * 8 * N, s, zc, batch, gc[0], gc[1], gc[2], 2, 1.0, tw, nullptr,
                       PoissonArg{}, V, ncols);
}

// host twiddle tables e^{-2 pi i t / n}, cached per (device, n) for the
// life of the process; a mutex keeps concurrent plans (isdf_fit_batch) safe
struct TwCache {
  int dev = -1, n = 0;
  double2* ptr = nullptr;
};
constexpr int TW_MAX = 128;
static TwCache g_tw[TW_MAX];
static int g_ntw = 0;
static std::mutex g_tw_mu;

static const double2* twiddles(int n) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(g_tw_mu);
  for (int i = 0; i < g_ntw; ++i)
    if (g_tw[i].dev == dev && g_tw[i].n == n) return g_tw[i].ptr;
  if (g_ntw == TW_MAX) return nullptr;
  std::vector<double2> h(n);
  for (int t = 0; t < n; ++t) {
    long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)t / n;
    h[t] = make_double2((double)cosl(ang), (double)sinl(ang));
  }
  double2* d = nullptr;
  if (hipMalloc(&d, sizeof(double2) * n) != hipSuccess) return nullptr;
  if (hipMemcpy(d, h.data(), sizeof(double2) * n, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  g_tw[g_ntw++] = TwCache{dev, n, d};
  return d;
}

isdf_status fft_prepare(int n) {
  if (!twiddles(n)) {
    set_error("fft: twiddle allocation failed");
    return ISDF_E_NOMEM;
  }
  return ISDF_OK;
}

isdf_status fft3d(hipStream_t s, double* zr, int batch, const int grid[3], int sign,
                  const double** /*unused*/) {
  double2* z = reinterpret_cast<double2*>(zr);
  const int n1 = grid[0], n2 = grid[1], n3 = grid[2];
  for (int axis = 0; axis < 3; ++axis) {
    const int n = grid[axis];
    if (n == 1) continue;
    const double2* tw = twiddles(n);
    if (!tw) {
      set_error("fft: twiddle allocation failed");
      return ISDF_E_NOMEM;
    }
    FftRadices rad = make_radices(n);
    int lpw;
    int64_t groups;
    // lines per workgroup: 16 for short lines, 8 from 48 points on (measured
    // on 32^3, 64^3 and 128^3 batches)
    if (axis == 0) {
      lpw = n <= 32 ? 16 : 8;
      const int64_t nl = (int64_t)n2 * n3 * batch;
      groups = (nl + lpw - 1) / lpw;
    } else {
      lpw = (n <= 32 && n1 % 16 == 0) ? 16
            : (n1 % 8 == 0) ? 8 : (n1 % 4 == 0) ? 4 : (n1 % 2 == 0) ? 2 : 1;
      groups = (int64_t)(n1 / lpw) * (axis == 1 ? n3 : n2) * batch;
    }
    if (!launch_fixed(s, z, batch, n1, n2, n3, axis, (double)sign, tw, n, lpw, groups)) {
      const size_t shmem = sizeof(double2) * 2 * (size_t)lpw * n;
      hipLaunchKernelGGL(fft_pass_kernel, dim3((unsigned)groups), dim3(256), shmem, s, z, batch, n1,
                         n2, n3, axis, (double)sign, tw, rad, lpw);
    }
    ISDF_HIP_TRY(hipGetLastError());
  }
  return ISDF_OK;
}

// ---------------------------------------------------------------- Poisson

__global__ void __launch_bounds__(256)
poisson_restrict_kernel(const double2* __restrict__ zf, double2* __restrict__ zc, int batch,
                        PoissonArg a) {
  const int64_t ngc = (int64_t)a.gc[0] * a.gc[1] * a.gc[2];
  const int64_t ngf = (int64_t)a.gf[0] * a.gf[1] * a.gf[2];
  const int b = blockIdx.y;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ngc;
       e += (int64_t)gridDim.x * blockDim.x) {
    int j[3];
    j[0] = (int)(e % a.gc[0]);
    const int64_t r = e / a.gc[0];
    j[1] = (int)(r % a.gc[1]);
    j[2] = (int)(r / a.gc[1]);
    int m[3];
    bool inband = true;
    for (int i = 0; i < 3; ++i) {
      m[i] = (j[i] <= (a.gc[i] - 1) / 2) ? j[i] : j[i] - a.gc[i];
      if (2 * abs(m[i]) >= a.gc[i]) inband = false;
    }
    double2 out = make_double2(0.0, 0.0);
    if (inband && (m[0] | m[1] | m[2]) != 0) {
      double G[3];
      for (int c = 0; c < 3; ++c) G[c] = m[0] * a.B[c] + m[1] * a.B[3 + c] + m[2] * a.B[6 + c];
      const double g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
      const double v = 4.0 * 3.14159265358979323846 / g2 * a.inv_ngf;
      int jf[3];
      for (int i = 0; i < 3; ++i) jf[i] = m[i] < 0 ? m[i] + a.gf[i] : m[i];
      const int64_t f = jf[0] + (int64_t)a.gf[0] * (jf[1] + (int64_t)a.gf[1] * jf[2]);
      const double2 zv = zf[(int64_t)b * ngf + f];
      out = make_double2(v * zv.x, v * zv.y);
    }
    zc[(int64_t)b * ngc + e] = out;
  }
}

isdf_status launch_poisson_restrict(hipStream_t s, const double* zf, const int gf[3], double* zc,
                                    const int gc[3], int batch, const double B[9]) {
  if (batch <= 0) return ISDF_OK;
  PoissonArg a;
  for (int i = 0; i < 3; ++i) {
    a.gf[i] = gf[i];
    a.gc[i] = gc[i];
  }
  for (int i = 0; i < 9; ++i) a.B[i] = B[i];
  a.inv_ngf = 1.0 / ((double)gf[0] * gf[1] * gf[2]);
  const int64_t ngc = (int64_t)gc[0] * gc[1] * gc[2];
  int64_t blocks = (ngc + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(poisson_restrict_kernel, dim3((unsigned)blocks, batch), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(zf), reinterpret_cast<double2*>(zc), batch, a);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// ------------------------------------------------------- scatter / split
__global__ void scatter_cols_kernel(const ScatterCol* __restrict__ cols, double* __restrict__ z,
                                    int64_t ng) {
  const ScatterCol c = cols[blockIdx.y];
  double* zp = z + (int64_t)(c.slot >> 1) * 2 * ng + (c.slot & 1);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < c.n; i += gridDim.x * blockDim.x)
    zp[2 * (int64_t)c.pts[i]] = c.src[i];
}
isdf_status launch_scatter_cols(hipStream_t s, const ScatterCol* cols, int ncols, int max_n,
                                double* z, int64_t ng) {
  if (ncols <= 0) return ISDF_OK;
  int blocks = (max_n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(scatter_cols_kernel, dim3(blocks, ncols), dim3(256), 0, s, cols, z, ng);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

__global__ void split_planar_kernel(const double* __restrict__ z, int64_t ng, int ncols,
                                    double* __restrict__ V) {
  const int c = blockIdx.y;
  const double* zp = z + (int64_t)(c >> 1) * 2 * ng + (c & 1);
  double* vp = V + (int64_t)c * ng;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ng;
       i += (int64_t)gridDim.x * blockDim.x)
    vp[i] = zp[2 * i];
}
isdf_status launch_split_planar(hipStream_t s, const double* z, int64_t ng, int ncols, double* V) {
  if (ncols <= 0) return ISDF_OK;
  int64_t blocks = (ng + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(split_planar_kernel, dim3((unsigned)blocks, ncols), dim3(256), 0, s, z, ng,
                     ncols, V);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// Poisson step + inverse transform on grid gc + planar split, fused into the
// first and last passes where the grid's line lengths have compiled kernels
// (x lines of 8 per workgroup need gc[0] divisible by 8).
isdf_status fft_poisson_inverse(hipStream_t s, const double* zf, const int gf[3], double* zc,
                                const int gc[3], int npairs, const double B[9], double* V,
                                int ncols, bool* done, hipEvent_t* ev) {
  *done = false;
  if (npairs <= 0 || !fused_len(gc[0]) || !fused_len(gc[1]) || !fused_len(gc[2]) || gc[0] % 8) return ISDF_OK;
  PoissonArg a;
  for (int i = 0; i < 3; ++i) {
    a.gf[i] = gf[i];
    a.gc[i] = gc[i];
  }
  for (int i = 0; i < 9; ++i) a.B[i] = B[i];
  a.inv_ngf = 1.0 / ((double)gf[0] * gf[1] * gf[2]);
  double2* z = reinterpret_cast<double2*>(zc);
  const double2* f = reinterpret_cast<const double2*>(zf);
  const double2* tw0 = twiddles(gc[0]);
  const double2* tw1 = twiddles(gc[1]);
  const double2* tw2 = twiddles(gc[2]);
  if (!tw0 || !tw1 || !tw2) {
    set_error("fft: twiddle allocation failed");
    return ISDF_E_NOMEM;
  }
  auto mark = [&](int i) -> isdf_status {
    if (ev) ISDF_HIP_TRY(hipEventRecord(ev[i], s));
    return ISDF_OK;
  };
  isdf_status st;
  // x pass from the fine spectrum
  const int64_t gx = ((int64_t)gc[1] * gc[2] * npairs + 7) / 8;
  if ((st = mark(0)) != ISDF_OK) return st;
  switch (gc[0]) {
    case 24: launch_poisson_x<24>(s, z, npairs, gc, tw0, f, a, gx); break;
    case 32: launch_poisson_x<32>(s, z, npairs, gc, tw0, f, a, gx); break;
    case 40: launch_poisson_x<40>(s, z, npairs, gc, tw0, f, a, gx); break;
    case 48: launch_poisson_x<48>(s, z, npairs, gc, tw0, f, a, gx); break;
    case 64: launch_poisson_x<64>(s, z, npairs, gc, tw0, f, a, gx); break;
    case 80: launch_poisson_x<80>(s, z, npairs, gc, tw0, f, a, gx); break;
    case 96: launch_poisson_x<96>(s, z, npairs, gc, tw0, f, a, gx); break;
    case 72: launch_poisson_x<72>(s, z, npairs, gc, tw0, f, a, gx); break;
    case 128: launch_poisson_x<128>(s, z, npairs, gc, tw0, f, a, gx); break;
    case 144: launch_poisson_x<144>(s, z, npairs, gc, tw0, f, a, gx); break;
    case 160: launch_poisson_x<160>(s, z, npairs, gc, tw0, f, a, gx); break;
    case 192: launch_poisson_x<192>(s, z, npairs, gc, tw0, f, a, gx); break;
    default:
      set_error("fft: no compiled x pass for the Poisson step");
      return ISDF_E_ARG;
  }
  ISDF_HIP_TRY(hipGetLastError());
  if ((st = mark(1)) != ISDF_OK) return st;
  // y pass as usual
  if ((st = mark(2)) != ISDF_OK) return st;
  {
    const int lpw = (gc[1] <= 32 && gc[0] % 16 == 0) ? 16 : 8;
    const int64_t groups = (int64_t)(gc[0] / lpw) * gc[2] * npairs;
    if (!launch_fixed(s, z, npairs, gc[0], gc[1], gc[2], 1, 1.0, tw1, gc[1], lpw, groups)) {
      set_error("fft: no compiled y pass");
      return ISDF_E_ARG;
    }
    ISDF_HIP_TRY(hipGetLastError());
  }
  if ((st = mark(3)) != ISDF_OK) return st;
  // z pass into the planar potentials
  // 16 lines a group where they divide the grid: each strided element of a
  // real plane is then a run of 128 bytes
  const int zlpw = gc[0] % 16 == 0 ? 16 : 8;
  if ((st = mark(4)) != ISDF_OK) return st;
  switch (gc[2]) {
    case 18: launch_planar_z<18>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    case 24: launch_planar_z<24>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    case 36: launch_planar_z<36>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    case 72: launch_planar_z<72>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    case 144: launch_planar_z<144>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    case 192: launch_planar_z<192>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    case 32: launch_planar_z<32>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    case 40: launch_planar_z<40>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    case 48: launch_planar_z<48>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    case 64: launch_planar_z<64>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    case 80: launch_planar_z<80>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    case 96: launch_planar_z<96>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    case 128: launch_planar_z<128>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    case 160: launch_planar_z<160>(s, z, npairs, gc, tw2, V, ncols, zlpw); break;
    default:
      set_error("fft: no compiled z pass for the planar potentials");
      return ISDF_E_ARG;
  }
  ISDF_HIP_TRY(hipGetLastError());
  if ((st = mark(5)) != ISDF_OK) return st;
  *done = true;
  return ISDF_OK;
}

// ------------------------------------------------ pruned forward transform
// A window's fitting function is zero outside the (cyclic) box around its
// points.  Pass x gathers only the lines (y, z) of a pair's box straight
// from the compact column values (no zero fill, no scatter); pass y
// transforms only the box's z planes and reads only its y range (zeros
// elsewhere); pass z reads only the box's z range.  Every value written is
// the exact transform of the zero-padded columns.
__device__ inline bool in_range(int i, int lo, int ext, int n, int* d) {
  int t = i - lo;
  if (t < 0) t += n;
  *d = t;
  return t < ext;
}

__device__ inline double gather_value(const FwdCol& c, int x, int y, int zz, int n1, int n2, int n3) {
  if (!c.src) return 0.0;
  if (!c.map) return c.src[x + (int64_t)n1 * (y + (int64_t)n2 * zz)];
  int dx, dy, dz;
  if (!in_range(x, c.box[0], c.box[3], n1, &dx) || !in_range(y, c.box[1], c.box[4], n2, &dy) ||
      !in_range(zz, c.box[2], c.box[5], n3, &dz))
    return 0.0;
  const int idx = c.map[dx + c.box[3] * (dy + c.box[4] * dz)];
  return idx >= 0 ? c.src[idx] : 0.0;
}

template <int N, int LPW, int AXIS>
__global__ void __launch_bounds__(256)
fft_fwd_pruned_kernel(double2* __restrict__ z, const FwdPair* __restrict__ pairs,
                      const FwdCol* __restrict__ cols, int n1, int n2, int n3,
                      const double2* __restrict__ tw) {
  extern __shared__ double2 lds[];
  double2* bufA = lds;
  const FwdPair P = pairs[blockIdx.y];
  const int64_t ng = (int64_t)n1 * n2 * n3;
  double2* zb = z + (int64_t)blockIdx.y * ng;
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  int nl = LPW;
  int64_t base = 0, estride = 1, lstride = 1;
  if (AXIS == 0) {  // lines (y, z) of the pair's box, LPW per workgroup
    const int nlines = P.box[4] * P.box[5];
    const int t0 = g * LPW;
    if (t0 >= nlines) return;
    nl = min(LPW, nlines - t0);
    const FwdCol c0 = cols[P.c0];
    const FwdCol c1 = P.c1 >= 0 ? cols[P.c1] : FwdCol{};
    for (int e = tid; e < nl * N; e += 256) {
      const int t = t0 + e / N, x = e % N;
      int y = P.box[1] + t % P.box[4], zz = P.box[2] + t / P.box[4];
      if (y >= n2) y -= n2;
      if (zz >= n3) zz -= n3;
      bufA[e] = make_double2(gather_value(c0, x, y, zz, n1, n2, n3), gather_value(c1, x, y, zz, n1, n2, n3));
    }
  } else {
    const int groups_x = n1 / LPW;
    // z lines (groups_x n2 workgroups): neighbouring workgroups step along y,
    // as in the planar z pass; y lines step along x
    const int i10 = (AXIS == 2 ? (g / n2) % groups_x : g % groups_x) * LPW;
    const int q = AXIS == 2 ? g % n2 : g / groups_x;
    if (AXIS == 1) {  // lines (x, z) for z in the box
      if (q >= P.box[5]) return;
      int zz = P.box[2] + q;
      if (zz >= n3) zz -= n3;
      base = i10 + (int64_t)n1 * n2 * zz;
      estride = n1;
      for (int e = tid; e < LPW * N; e += 256) {
        const int j = e % LPW, i = e / LPW;
        int d;
        bufA[j * N + i] = in_range(i, P.box[1], P.box[4], n2, &d) ? zb[base + j + i * estride]
                                                                   : make_double2(0.0, 0.0);
      }
    } else {  // lines (x, y), all of them; z outside the box reads as zero
      base = i10 + (int64_t)n1 * q;
      estride = (int64_t)n1 * n2;
      for (int e = tid; e < LPW * N; e += 256) {
        const int j = e % LPW, i = e / LPW;
        int d;
        bufA[j * N + i] = in_range(i, P.box[2], P.box[5], n3, &d) ? zb[base + j + i * estride]
                                                                   : make_double2(0.0, 0.0);
      }
    }
  }
  __syncthreads();
  fft_stages_ip<N, 0, LPW>(bufA, nl, tw, -1.0);
  const double2* res = bufA;
  if (AXIS == 0) {
    const int t0 = g * LPW;
    for (int e = tid; e < nl * N; e += 256) {
      const int t = t0 + e / N, x = e % N;
      int y = P.box[1] + t % P.box[4], zz = P.box[2] + t / P.box[4];
      if (y >= n2) y -= n2;
      if (zz >= n3) zz -= n3;
      zb[x + (int64_t)n1 * (y + (int64_t)n2 * zz)] = res[e];
    }
  } else {
    for (int e = tid; e < LPW * N; e += 256) {
      const int j = e % LPW, i = e / LPW;
      zb[base + j + i * estride] = res[j * N + i];
    }
  }
}

template <int N, int AXIS>
void launch_fwd_pruned(hipStream_t s, double2* z, const FwdPair* pairs, const FwdCol* cols, int npairs,
                       const int g[3], const double2* tw, int gx) {
  constexpr int LPW = 8;
  hipLaunchKernelGGL((fft_fwd_pruned_kernel<N, LPW, AXIS>), dim3((unsigned)gx, (unsigned)npairs),
                     dim3(256), sizeof(double2) * LPW * N, s, z, pairs, cols, g[0], g[1], g[2], tw);
}

template <int AXIS>
bool fwd_pass(hipStream_t s, double2* z, const FwdPair* pairs, const FwdCol* cols, int npairs,
              const int g[3], const double2* tw, int n, int gx) {
  switch (n) {
    case 18: launch_fwd_pruned<18, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    case 24: launch_fwd_pruned<24, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    case 36: launch_fwd_pruned<36, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    case 72: launch_fwd_pruned<72, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    case 144: launch_fwd_pruned<144, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    case 192: launch_fwd_pruned<192, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    case 32: launch_fwd_pruned<32, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    case 40: launch_fwd_pruned<40, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    case 48: launch_fwd_pruned<48, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    case 64: launch_fwd_pruned<64, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    case 80: launch_fwd_pruned<80, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    case 96: launch_fwd_pruned<96, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    case 128: launch_fwd_pruned<128, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    case 160: launch_fwd_pruned<160, AXIS>(s, z, pairs, cols, npairs, g, tw, gx); return true;
    default: return false;
  }
}

bool fft_forward_pruned_supported(const int g[3]) {
  return fused_len(g[0]) && fused_len(g[1]) && fused_len(g[2]) && g[0] % 8 == 0;
}

isdf_status fft_forward_pruned(hipStream_t s, double* zr, const FwdPair* pairs, const FwdCol* cols,
                               int npairs, const int g[3], int max_yz, int max_z, hipEvent_t* ev) {
  if (npairs <= 0) return ISDF_OK;
  if (!fft_forward_pruned_supported(g)) {
    set_error("fft: pruned forward transform needs compiled line lengths");
    return ISDF_E_ARG;
  }
  double2* z = reinterpret_cast<double2*>(zr);
  const double2* tw0 = twiddles(g[0]);
  const double2* tw1 = twiddles(g[1]);
  const double2* tw2 = twiddles(g[2]);
  if (!tw0 || !tw1 || !tw2) {
    set_error("fft: twiddle allocation failed");
    return ISDF_E_NOMEM;
  }
  if (ev) ISDF_HIP_TRY(hipEventRecord(ev[0], s));
  fwd_pass<0>(s, z, pairs, cols, npairs, g, tw0, g[0], (max_yz + 7) / 8);
  ISDF_HIP_TRY(hipGetLastError());
  if (ev) ISDF_HIP_TRY(hipEventRecord(ev[1], s));
  if (ev) ISDF_HIP_TRY(hipEventRecord(ev[2], s));
  fwd_pass<1>(s, z, pairs, cols, npairs, g, tw1, g[1], (g[0] / 8) * max_z);
  ISDF_HIP_TRY(hipGetLastError());
  if (ev) ISDF_HIP_TRY(hipEventRecord(ev[3], s));
  if (ev) ISDF_HIP_TRY(hipEventRecord(ev[4], s));
  fwd_pass<2>(s, z, pairs, cols, npairs, g, tw2, g[2], (g[0] / 8) * g[1]);
  ISDF_HIP_TRY(hipGetLastError());
  if (ev) ISDF_HIP_TRY(hipEventRecord(ev[5], s));
  return ISDF_OK;
}

}  // namespace isdf
