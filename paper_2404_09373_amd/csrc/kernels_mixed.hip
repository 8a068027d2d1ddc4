// BF16-split GEMM with FP32 accumulation and FP64 carry (mixed precision).
//
// An FP64 operand x is stored as S BF16 planes x = x_0 + x_1 (+ x_2) with
// x_0 = bf16(x), x_1 = bf16(x - x_0), x_2 = bf16(x - x_0 - x_1).  A product
// is formed from the planes whose indices add up to at most S - 1:
//   S = 2 ("x3"): a0 b0 + a0 b1 + a1 b0                 (~16-bit operands)
//   S = 3 ("x6"): the above + a0 b2 + a1 b1 + a2 b0     (~24-bit operands)
// on v_mfma_f32_16x16x32_bf16.  The leading term a0 b0 and the correction
// terms accumulate in separate FP32 registers (the corrections are 2^-8 times
// smaller, so their rounding is negligible) and both are added into FP64
// accumulators every 256 values of k, which bounds the FP32 rounding of the
// leading term.  Used for the Gram, Coulomb-metric and exchange contractions
// when a mixed precision is requested; the interpolation-metric Cholesky and
// triangular solves always stay FP64.
//
// Planes are K-contiguous: A plane p holds element (m, k) at
// A + p * plane_stride + m * lda + k, B plane p holds (k, n) at
// B + p * plane_stride + n * ldb + k, so every MFMA operand is one 16-byte
// LDS read.  Lane layout of v_mfma_f32_16x16x32_bf16 (wave64):
//   operand 1: lane l holds X[i = l % 16][k = 8 (l / 16) + t], t = 0..7
//   operand 2: lane l holds Y[k = 8 (l / 16) + t][j = l % 16]
//   result   : lane l, register v holds D[i = 4 (l / 16) + v][j = l % 16]
// Operand 1 carries B^T and operand 2 A^T, so a lane's results are 16
// consecutive rows of one column of the column-major C.
#include "common.h"

namespace isdf {

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4m __attribute__((ext_vector_type(4)));

namespace {
constexpr int BM = 64, BN = 64, BK = 32, KFLUSH = 256;

// Workgroups go round-robin over the 8 XCDs (each with its own L2): dispatch
// slot b (XCD b % 8) is mapped to a contiguous range of tiles, and within a
// problem the dimension with fewer tiles runs fastest, so the tiles an XCD
// has in flight share blocks of the larger operand in its L2.
constexpr int NXCD = 8;
__device__ inline int xcd_tile(int b, int nb) {
  const int x = b % NXCD, q = b / NXCD, per = nb / NXCD, rem = nb % NXCD;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + q;
}
// Tile order: groups of G row tiles (the problem's tile_group, 8 when
// unset), the row index running fastest within a group.  The workgroups that
// run together on one XCD (consecutive tiles) then share each B column panel
// G ways and keep the group's A row panels in that XCD's L2 across all
// columns; a plain row-major order read every B panel once per row tile from
// HBM (measured: exchange products fetching about 12 times their operand
// bytes).
__device__ inline void tile_coords(int local, int tilesM, int tilesN, int group, int* tm, int* tn) {
  const int G = group > 0 ? group : 8;
  const int per_group = G * tilesN;
  const int g = local / per_group;
  const int rows = min(G, tilesM - g * G);
  const int idx = local - g * per_group;
  *tm = g * G + idx % rows;
  *tn = idx / rows;
}

// Every operand, epilogue input and output lives in device global memory.
// Reaching it through global-address-space pointers makes the compiler emit
// global loads and stores instead of flat ones: a flat access also counts
// against the LDS wait counter, so every wait for LDS fragments would wait
// for the next chunk's operand prefetch from HBM as well.
#define GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ inline const GLOBAL T* gro(const T* q) { return (const GLOBAL T*)q; }
template <class T>
__device__ inline GLOBAL T* grw(T* q) { return (GLOBAL T*)q; }

// Element (m, n) of a Hadamard epilogue's E, held in FP64 or FP32.
__device__ inline double mixed_e(const MixedProblem& p, int m, int n) {
  const int64_t i = (int64_t)m + (int64_t)n * p.lde;
  return p.E32 ? (double)gro(p.E32)[i] : gro(p.E)[i];
}

__device__ inline const MixedProblem* find_mixed(const MixedProblem* probs, int nprob, int tile) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile_start <= tile) lo = mid; else hi = mid - 1;
  }
  return probs + lo;
}
}  // namespace

template <int EPI, int S, int TAG>
__global__ void __launch_bounds__(256)
gemm_mixed_kernel(MixedProblem single, const MixedProblem* __restrict__ probs, int nprob) {
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const MixedProblem* pp = probs ? find_mixed(probs, nprob, tile) : &single;
  const MixedProblem p = *pp;
  int tm, tn;
  tile_coords(tile - p.tile_start, (p.M + BM - 1) / BM, (p.N + BN - 1) / BN, p.tile_group, &tm, &tn);
  const int m0 = tm * BM, n0 = tn * BN;
  if (n0 >= p.N) return;
  if (p.lower && m0 + BM <= n0) return;

  // [plane][row][k], padded by 8 bf16 (16 B) per row against bank conflicts
  __shared__ __attribute__((aligned(16))) __bf16 As[S][BM][BK + 8];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[S][BN][BK + 8];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  f4v hi[2][2], lo[2][2], hiN[2][2], loN[2][2];
  d4m acc[2][2], accN[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      hi[a][b] = lo[a][b] = hiN[a][b] = loN[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
      acc[a][b] = accN[a][b] = d4m{0.0, 0.0, 0.0, 0.0};
    }

  // each thread stages one 16-byte chunk (8 bf16 along k) per plane and operand
  const int lr = tid >> 2;          // row within the tile (0..63)
  const int lk = (tid & 3) * 8;     // k offset within the chunk
  const bool tile_in = m0 + BM <= p.M && n0 + BN <= p.N;
  for (int k0 = 0; k0 < p.K; k0 += BK) {
    bf8v ra[S], rb[S];
    if (tile_in && k0 + BK <= p.K) {  // interior: no bounds tests (see the wide kernel)
#pragma unroll
      for (int s = 0; s < S; ++s) {
        ra[s] = *reinterpret_cast<const GLOBAL bf8v*>(gro(p.A) + s * p.plane_a + (int64_t)(m0 + lr) * p.lda + k0 + lk);
        rb[s] = *reinterpret_cast<const GLOBAL bf8v*>(gro(p.B) + s * p.plane_b + (int64_t)(n0 + lr) * p.ldb + k0 + lk);
      }
    } else {
      const int gm = m0 + lr, gk = k0 + lk;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        bf8v v;
        if (gm < p.M && gk + 8 <= p.K) {
          v = *reinterpret_cast<const GLOBAL bf8v*>(gro(p.A) + s * p.plane_a + (int64_t)gm * p.lda + gk);
        } else {
#pragma unroll
          for (int t = 0; t < 8; ++t)
            v[t] = (gm < p.M && gk + t < p.K) ? gro(p.A)[s * p.plane_a + (int64_t)gm * p.lda + gk + t]
                                               : (__bf16)0.0f;
        }
        ra[s] = v;
      }
      const int gn = n0 + lr;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        bf8v v;
        if (gn < p.N && gk + 8 <= p.K) {
          v = *reinterpret_cast<const GLOBAL bf8v*>(gro(p.B) + s * p.plane_b + (int64_t)gn * p.ldb + gk);
        } else {
#pragma unroll
          for (int t = 0; t < 8; ++t)
            v[t] = (gn < p.N && gk + t < p.K) ? gro(p.B)[s * p.plane_b + (int64_t)gn * p.ldb + gk + t]
                                               : (__bf16)0.0f;
        }
        rb[s] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < S; ++s) {
      *reinterpret_cast<bf8v*>(&As[s][lr][lk]) = ra[s];
      *reinterpret_cast<bf8v*>(&Bs[s][lr][lk]) = rb[s];
    }
    __syncthreads();
    const int kq = 8 * (lane >> 4);
    bf8v xb[S][2], ya[S][2];
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
      for (int b = 0; b < 2; ++b) xb[s][b] = *reinterpret_cast<const bf8v*>(&Bs[s][wn * 32 + b * 16 + (lane & 15)][kq]);
#pragma unroll
      for (int a = 0; a < 2; ++a) ya[s][a] = *reinterpret_cast<const bf8v*>(&As[s][wm * 32 + a * 16 + (lane & 15)][kq]);
    }
    // Theta split: this chunk's k range lies entirely on one side of kL when
    // kL is a multiple of BK (the host pads the L columns to guarantee it)
    const bool toN = (EPI == EPI_THETA) && k0 >= p.kL;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        f4v h = toN ? hiN[a][b] : hi[a][b];
        f4v l = toN ? loN[a][b] : lo[a][b];
        h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb[0][b], ya[0][a], h, 0, 0, 0);
        l = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb[0][b], ya[1][a], l, 0, 0, 0);
        l = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb[1][b], ya[0][a], l, 0, 0, 0);
        if (S == 3) {
          l = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb[0][b], ya[S - 1][a], l, 0, 0, 0);
          l = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb[1][b], ya[1][a], l, 0, 0, 0);
          l = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb[S - 1][b], ya[0][a], l, 0, 0, 0);
        }
        if (toN) {
          hiN[a][b] = h;
          loN[a][b] = l;
        } else {
          hi[a][b] = h;
          lo[a][b] = l;
        }
      }
    if (((k0 + BK) % KFLUSH) == 0 || k0 + BK >= p.K) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            acc[a][b][v] += (double)hi[a][b][v] + (double)lo[a][b][v];
            hi[a][b][v] = lo[a][b][v] = 0.f;
            if (EPI == EPI_THETA) {
              accN[a][b][v] += (double)hiN[a][b][v] + (double)loN[a][b][v];
              hiN[a][b][v] = loN[a][b][v] = 0.f;
            }
          }
    }
  }
  // epilogue: lane holds C(m0 + wm*32 + a*16 + lane%16, n0 + wn*32 + b*16 + 4(lane/16) + v)
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int gm = m0 + wm * 32 + a * 16 + (lane & 15);
    if (gm >= p.M) continue;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gn = n0 + wn * 32 + b * 16 + 4 * (lane >> 4) + v;
        if (gn >= p.N) continue;
        GLOBAL double* cp = grw(p.C) + (int64_t)gm + (int64_t)gn * p.ldc;
        const double x = acc[a][b][v];
        if (EPI == EPI_THETA) {
          *cp = x * (x + 2.0 * accN[a][b][v]);
        } else if (EPI == EPI_HADAMARD) {
          double y = p.alpha * x * mixed_e(p, gm, gn);
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

int mixed_tiles(int M, int N) { return ((M + BM - 1) / BM) * ((N + BN - 1) / BN); }

// ---------------------------------------------------------- wide products
// The same split products for single AXPBY / HADAMARD problems with many
// tiles, on 64 x 128 tiles: four waves of 32 x 64 (2 x 4 MFMA tiles), so a
// k chunk costs 6 S operand reads from LDS for 8 S (S + 1) / 2 MFMAs.  Two
// LDS stages: chunk c + 1 is loaded into registers during chunk c's MFMAs
// and stored into the other stage, one barrier per chunk.  LDS rows are 64
// bytes (four 16-byte units of 8 values of k) without padding; unit u of row
// r sits at position u ^ ((r >> 1) & 3), so that every group of 8 lanes
// touches 8 distinct 16-byte bank groups both when staging (2 rows x 4
// units) and when reading fragments (8 rows, one unit).
namespace {
constexpr int WBM = 64, WBN = 128;
__device__ inline int swz(int r, int u) { return r * BK + ((u ^ ((r >> 1) & 3)) << 3); }
}  // namespace

int mixed_tiles_wide(int M, int N) { return ((M + WBM - 1) / WBM) * ((N + WBN - 1) / WBN); }

template <int EPI, int S, int TAG>
__global__ void __launch_bounds__(256, 2)
gemm_mixed_wide_kernel(MixedProblem single, const MixedProblem* __restrict__ probs, int nprob) {
  // nprob < 0: -nprob problems of one tile grid, interleaved tile by tile
  // (tile t is tile t / -nprob of problem t % -nprob), so the problems'
  // tiles at one position run together on one XCD and share its L2
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const MixedProblem p = !probs ? single : nprob < 0 ? probs[tile % -nprob] : *find_mixed(probs, nprob, tile);
  const int local = !probs ? tile : nprob < 0 ? tile / -nprob : tile - p.tile_start;
  int tm, tn;
  tile_coords(local, (p.M + WBM - 1) / WBM, (p.N + WBN - 1) / WBN, p.tile_group, &tm, &tn);
  const int m0 = tm * WBM, n0 = tn * WBN;

  __shared__ __attribute__((aligned(16))) __bf16 As[2][S][WBM * BK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][S][WBN * BK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;  // wave tile rows wm*32.., columns wn*64..

  f4v hi[2][4], lo[2][4];
  d4m acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      hi[a][b] = lo[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
      acc[a][b] = d4m{0.0, 0.0, 0.0, 0.0};
    }

  // staging: A rows lr (64 rows), B rows lr and lr + 64; unit lu of 8 k values
  const int lr = tid >> 2, lu = tid & 3;
  bf8v ra[S], rb[S][2];
  auto fetch = [&](const GLOBAL __bf16* base, int64_t plane, int64_t ld, int rows, int r, int gk) -> bf8v {
    bf8v v;
    if (r < rows && gk + 8 <= p.K) {
      v = *reinterpret_cast<const GLOBAL bf8v*>(base + plane + (int64_t)r * ld + gk);
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t)
        v[t] = (r < rows && gk + t < p.K) ? base[plane + (int64_t)r * ld + gk + t] : (__bf16)0.0f;
    }
    return v;
  };
  // Interior chunks of interior tiles (a wave-uniform test) load without any
  // bounds test: a guarded load per value would make every load wait for
  // completion at its branch, and the next chunk would no longer be in
  // flight during the MFMAs.
  const bool tile_in = m0 + WBM <= p.M && n0 + WBN <= p.N;
  const GLOBAL __bf16* pa = gro(p.A) + (int64_t)(m0 + lr) * p.lda + lu * 8;
  const GLOBAL __bf16* pb0 = gro(p.B) + (int64_t)(n0 + lr) * p.ldb + lu * 8;
  const GLOBAL __bf16* pb1 = pb0 + (int64_t)64 * p.ldb;
  auto load = [&](int k0) {
    if (tile_in && k0 + BK <= p.K) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        ra[s] = *reinterpret_cast<const GLOBAL bf8v*>(pa + s * p.plane_a + k0);
        rb[s][0] = *reinterpret_cast<const GLOBAL bf8v*>(pb0 + s * p.plane_b + k0);
        rb[s][1] = *reinterpret_cast<const GLOBAL bf8v*>(pb1 + s * p.plane_b + k0);
      }
    } else {
      const int gk = k0 + lu * 8;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        ra[s] = fetch(gro(p.A), s * p.plane_a, p.lda, p.M, m0 + lr, gk);
        rb[s][0] = fetch(gro(p.B), s * p.plane_b, p.ldb, p.N, n0 + lr, gk);
        rb[s][1] = fetch(gro(p.B), s * p.plane_b, p.ldb, p.N, n0 + lr + 64, gk);
      }
    }
  };
  auto store = [&](int st) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      *reinterpret_cast<bf8v*>(&As[st][s][swz(lr, lu)]) = ra[s];
      *reinterpret_cast<bf8v*>(&Bs[st][s][swz(lr, lu)]) = rb[s][0];
      *reinterpret_cast<bf8v*>(&Bs[st][s][swz(lr + 64, lu)]) = rb[s][1];
    }
  };
  load(0);
  store(0);
  __syncthreads();
  const int fu = lane >> 4;  // fragment unit: k = 8 fu .. 8 fu + 7
  // fragment reads and MFMAs of the chunk in stage st; the FP32 sums go into
  // the FP64 accumulators every KFLUSH values of k and after the last chunk
  auto chunk = [&](int k0, int st, bool last) {
    // planes 0 and 1 first; plane 2 (x6) then reuses plane 1's registers
    bf8v x0[4], y0[2], x1[4], y1[2];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      x0[t] = *reinterpret_cast<const bf8v*>(&Bs[st][0][swz(wn * 64 + t * 16 + (lane & 15), fu)]);
      x1[t] = *reinterpret_cast<const bf8v*>(&Bs[st][1][swz(wn * 64 + t * 16 + (lane & 15), fu)]);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      y0[t] = *reinterpret_cast<const bf8v*>(&As[st][0][swz(wm * 32 + t * 16 + (lane & 15), fu)]);
      y1[t] = *reinterpret_cast<const bf8v*>(&As[st][1][swz(wm * 32 + t * 16 + (lane & 15), fu)]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        hi[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0[b], y0[a], hi[a][b], 0, 0, 0);
        f4v l = lo[a][b];
        l = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0[b], y1[a], l, 0, 0, 0);
        l = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1[b], y0[a], l, 0, 0, 0);
        if (S == 3) l = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1[b], y1[a], l, 0, 0, 0);
        lo[a][b] = l;
      }
    if constexpr (S == 3) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
        x1[t] = *reinterpret_cast<const bf8v*>(&Bs[st][2][swz(wn * 64 + t * 16 + (lane & 15), fu)]);
#pragma unroll
      for (int t = 0; t < 2; ++t)
        y1[t] = *reinterpret_cast<const bf8v*>(&As[st][2][swz(wm * 32 + t * 16 + (lane & 15), fu)]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          f4v l = lo[a][b];
          l = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0[b], y1[a], l, 0, 0, 0);
          l = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1[b], y0[a], l, 0, 0, 0);
          lo[a][b] = l;
        }
    }
    if (((k0 + BK) % KFLUSH) == 0 || last) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            acc[a][b][v] += (double)hi[a][b][v] + (double)lo[a][b][v];
            hi[a][b][v] = lo[a][b][v] = 0.f;
          }
    }
  };
  int k0 = 0, st = 0;
  for (; k0 + BK < p.K; k0 += BK, st ^= 1) {
    load(k0 + BK);  // in flight during this chunk's MFMAs
    chunk(k0, st, false);
    store(st ^ 1);  // the other stage: its last readers passed the previous barrier
    __syncthreads();
  }
  // The last chunk (peeled).  With the planes epilogue and E in FP32 the
  // lane's 32 values of E are loaded here, in flight during the chunk's MFMAs,
  // into registers that the staging loads no longer hold; value (a, b, v)
  // is word v of ew[4 a + b].  Outside the problem: a valid address, value 0.
  constexpr bool E_REG = EPI == EPI_HADAMARD_PLANES;
  const bool ereg = E_REG && p.E32 != nullptr;
  f4v ew[8];
  if (ereg) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gm = m0 + wm * 32 + a * 16 + (lane & 15);
          const int gn = n0 + wn * 64 + b * 16 + 4 * (lane >> 4) + v;
          const bool ok = gm < p.M && gn < p.N;
          const float x = gro(p.E32)[ok ? (int64_t)gm + (int64_t)gn * p.lde : 0];
          ew[a * 4 + b][v] = ok ? x : 0.f;
        }
  }
  chunk(k0, st, true);
  __syncthreads();
  // lane holds C(m0 + wm*32 + a*16 + lane%16, n0 + wn*64 + b*16 + 4(lane/16) + v)
  if constexpr (EPI == EPI_HADAMARD_PLANES) {
    // The transposed tile's planes go through LDS (the B stages, free now:
    // S x 128 x 64 values) and out as 16-byte rows of 8 values of m.  Within
    // row r the four 16-value blocks of m are permuted by (r >> 2) & 3, so
    // that the four lane groups of a wave, four rows apart, store into four
    // distinct bank ranges; 8-value runs stay contiguous for the reads.
    __bf16* Ps = &Bs[0][0][0];
    auto pidx = [](int q, int r, int c) { return (q * WBN + r) * WBM + (c ^ (((r >> 2) & 3) << 4)); };
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int cm = wm * 32 + a * 16 + (lane & 15), gm = m0 + cm;
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rn = wn * 64 + b * 16 + 4 * (lane >> 4) + v, gn = n0 + rn;
          double y = 0.0;
          if (gm < p.M && gn < p.N) {
            const double e = ereg ? (double)ew[a * 4 + b][v] : mixed_e(p, gm, gn);
            y = p.alpha * acc[a][b][v] * e;
          }
#pragma unroll
          for (int q = 0; q < S; ++q) {
            const __bf16 h = (__bf16)(float)y;
            Ps[pidx(q, rn, cm)] = h;
            y -= (double)(float)h;
          }
        }
    }
    __syncthreads();
    const bool vec = (p.p_off % 8) == 0 && m0 + WBM <= p.M && n0 + WBN <= p.N;
    if (vec) {
      for (int e = tid; e < S * WBN * (WBM / 8); e += 256) {
        const int q = e / (WBN * (WBM / 8)), r = (e / (WBM / 8)) % WBN, c8 = (e % (WBM / 8)) * 8;
        *reinterpret_cast<GLOBAL bf8v*>(grw(p.P) + q * p.plane_p + (int64_t)(n0 + r) * p.ldp + p.p_off + m0 + c8) =
            *reinterpret_cast<const bf8v*>(&Ps[pidx(q, r, c8)]);
      }
    } else {
      for (int e = tid; e < S * WBN * WBM; e += 256) {
        const int q = e / (WBN * WBM), r = (e / WBM) % WBN, c = e % WBM;
        if (n0 + r < p.N && m0 + c < p.M)
          grw(p.P)[q * p.plane_p + (int64_t)(n0 + r) * p.ldp + p.p_off + m0 + c] = Ps[pidx(q, r, c)];
      }
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int gm = m0 + wm * 32 + a * 16 + (lane & 15);
    if (gm >= p.M) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gn = n0 + wn * 64 + b * 16 + 4 * (lane >> 4) + v;
        if (gn >= p.N) continue;
        const double x = acc[a][b][v];
        GLOBAL double* cp = grw(p.C) + (int64_t)gm + (int64_t)gn * p.ldc;
        double y;
        if (EPI == EPI_HADAMARD)
          y = p.alpha * x * mixed_e(p, gm, gn);
        else
          y = p.alpha * x;
        if (p.beta != 0.0) y += p.beta * *cp;
        *cp = y;
      }
  }
}

template <int S, int TAG>
static void launch_wide_st(hipStream_t s, int epi, const MixedProblem& p, const MixedProblem* probs,
                           int nprob, int tiles) {
  if (epi == EPI_HADAMARD)
    hipLaunchKernelGGL((gemm_mixed_wide_kernel<EPI_HADAMARD, S, TAG>), dim3(tiles), dim3(256), 0, s, p,
                       probs, nprob);
  else if (epi == EPI_HADAMARD_PLANES)
    hipLaunchKernelGGL((gemm_mixed_wide_kernel<EPI_HADAMARD_PLANES, S, TAG>), dim3(tiles), dim3(256), 0, s,
                       p, probs, nprob);
  else
    hipLaunchKernelGGL((gemm_mixed_wide_kernel<EPI_AXPBY, S, TAG>), dim3(tiles), dim3(256), 0, s, p, probs,
                       nprob);
}

template <int S>
static void launch_wide_s(hipStream_t s, int epi, int tag, const MixedProblem& p, const MixedProblem* probs,
                          int nprob, int tiles) {
  switch (tag) {
    case 2: launch_wide_st<S, 2>(s, epi, p, probs, nprob, tiles); break;
    case 3: launch_wide_st<S, 3>(s, epi, p, probs, nprob, tiles); break;
    default: launch_wide_st<S, 4>(s, epi, p, probs, nprob, tiles); break;
  }
}

template <int S, int TAG>
static void launch_st(hipStream_t s, int epi, const MixedProblem& single, const MixedProblem* probs,
                      int nprob, int tiles) {
  if (epi == EPI_THETA)
    hipLaunchKernelGGL((gemm_mixed_kernel<EPI_THETA, S, TAG>), dim3(tiles), dim3(256), 0, s, single,
                       probs, nprob);
  else if (epi == EPI_HADAMARD)
    hipLaunchKernelGGL((gemm_mixed_kernel<EPI_HADAMARD, S, TAG>), dim3(tiles), dim3(256), 0, s,
                       single, probs, nprob);
  else
    hipLaunchKernelGGL((gemm_mixed_kernel<EPI_AXPBY, S, TAG>), dim3(tiles), dim3(256), 0, s, single,
                       probs, nprob);
}

template <int S>
static void launch_s(hipStream_t s, int epi, int tag, const MixedProblem& single,
                     const MixedProblem* probs, int nprob, int tiles) {
  switch (tag) {
    case 2: launch_st<S, 2>(s, epi, single, probs, nprob, tiles); break;
    case 3: launch_st<S, 3>(s, epi, single, probs, nprob, tiles); break;
    default: launch_st<S, 4>(s, epi, single, probs, nprob, tiles); break;
  }
}

isdf_status gemm_mixed(hipStream_t s, int epi, int splits, const MixedProblem& p, int tag) {
  if (p.M <= 0 || p.N <= 0) return ISDF_OK;
  MixedProblem q = p;
  q.tile_start = 0;
  // products with enough 64 x 128 tiles to fill the chip take the wide
  // kernel, and so does the planes epilogue (it exists only there)
  if (epi == EPI_HADAMARD_PLANES ||
      (epi != EPI_THETA && !p.lower && mixed_tiles_wide(p.M, p.N) >= MIXED_WIDE_MIN_TILES)) {
    const int tiles = mixed_tiles_wide(p.M, p.N);
    if (splits == 2) launch_wide_s<2>(s, epi, tag, q, nullptr, 1, tiles);
    else launch_wide_s<3>(s, epi, tag, q, nullptr, 1, tiles);
    ISDF_HIP_TRY(hipGetLastError());
    return ISDF_OK;
  }
  const int tiles = mixed_tiles(p.M, p.N);
  if (splits == 2) launch_s<2>(s, epi, tag, q, nullptr, 1, tiles);
  else launch_s<3>(s, epi, tag, q, nullptr, 1, tiles);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

isdf_status gemm_mixed_wide_grouped(hipStream_t s, int epi, int splits, const MixedProblem* d_probs,
                                    int nprob, int total_tiles, int tag) {
  if (nprob == 0 || total_tiles <= 0) return ISDF_OK;
  if (epi == EPI_THETA) {
    set_error("mixed GEMM: the wide kernel has no Theta epilogue");
    return ISDF_E_ARG;
  }
  MixedProblem dummy{};
  if (splits == 2) launch_wide_s<2>(s, epi, tag, dummy, d_probs, nprob, total_tiles);
  else launch_wide_s<3>(s, epi, tag, dummy, d_probs, nprob, total_tiles);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

__global__ void __launch_bounds__(256)
sum_parts_kernel(const double* __restrict__ parts, int nparts, int64_t count, double* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    double a = 0.0;
    for (int q = 0; q < nparts; ++q) a += parts[(int64_t)q * count + i];
    out[i] = a;
  }
}

isdf_status launch_sum_parts(hipStream_t s, const double* parts, int nparts, int64_t count, double* out) {
  if (count <= 0) return ISDF_OK;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)blocks), dim3(256), 0, s, parts, nparts, count, out);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

isdf_status gemm_mixed_grouped(hipStream_t s, int epi, int splits, const MixedProblem* d_probs,
                               int nprob, int total_tiles, int tag) {
  if (nprob <= 0 || total_tiles <= 0) return ISDF_OK;
  if (epi == EPI_HADAMARD_PLANES) {
    set_error("mixed GEMM: the planes epilogue runs on the wide kernel");
    return ISDF_E_ARG;
  }
  MixedProblem dummy{};
  if (splits == 2) launch_s<2>(s, epi, tag, dummy, d_probs, nprob, total_tiles);
  else launch_s<3>(s, epi, tag, dummy, d_probs, nprob, total_tiles);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

// ------------------------------------------------------------------ split
// Logical operand X (rows x cols, "outer" x "k") read from an FP64 matrix with
// element (o, k) at src[o * so + k * sk]; written as `splits` K-contiguous
// planes dst[p * plane + o * ldd + k] (ldd >= cols).  Optional row gather:
// o_src = gidx ? gidx[o] : o (rows) or k_src = kidx ? kidx[k] : k.
__global__ void __launch_bounds__(256)
split_bf16_kernel(const double* __restrict__ src, int64_t so, int64_t sk,
                  const int32_t* __restrict__ kidx, int rows, int cols, int splits,
                  __bf16* __restrict__ dst, int64_t ldd, int64_t plane, double scale) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    // walk k fastest when the source is k-contiguous, else the outer index
    int64_t o, k;
    if (sk == 1) {
      o = e / cols;
      k = e % cols;
    } else {
      k = e / rows;
      o = e % rows;
    }
    const int64_t ks = kidx ? (int64_t)kidx[k] : k;
    double x = ks >= 0 ? src[o * so + ks * sk] * scale : 0.0;
    __bf16* d = dst + o * ldd + k;
    for (int p = 0; p < splits; ++p) {
      const __bf16 h = (__bf16)(float)x;
      d[p * plane] = h;
      x -= (double)(float)h;
    }
  }
}

// Same for a source whose outer index is the contiguous one (so == 1): a
// 32 x 32 tile is read along o and written along k through LDS.
__global__ void __launch_bounds__(256)
split_bf16_t_kernel(const double* __restrict__ src, int64_t sk, const int32_t* __restrict__ kidx,
                    int rows, int cols, int splits, __bf16* __restrict__ dst, int64_t ldd,
                    int64_t plane, double scale) {
  __shared__ double t[32][33];
  const int o0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int o = o0 + tx, k = k0 + r;
    double v = 0.0;
    if (o < rows && k < cols) {
      const int64_t ks = kidx ? (int64_t)kidx[k] : k;
      v = ks >= 0 ? src[(int64_t)o + ks * sk] * scale : 0.0;
    }
    t[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int o = o0 + r, k = k0 + tx;
    if (o < rows && k < cols) {
      double x = t[tx][r];
      __bf16* d = dst + (int64_t)o * ldd + k;
      for (int q = 0; q < splits; ++q) {
        const __bf16 h = (__bf16)(float)x;
        d[q * plane] = h;
        x -= (double)(float)h;
      }
    }
  }
}

isdf_status launch_split_bf16(hipStream_t s, const double* src, int64_t so, int64_t sk,
                              const int32_t* kidx, int rows, int cols, int splits, __bf16* dst,
                              int64_t ldd, int64_t plane, double scale) {
  const int64_t total = (int64_t)rows * cols;
  if (total <= 0) return ISDF_OK;
  if (so == 1 && sk != 1) {
    hipLaunchKernelGGL(split_bf16_t_kernel, dim3((rows + 31) / 32, (cols + 31) / 32), dim3(256), 0, s,
                       src, sk, kidx, rows, cols, splits, dst, ldd, plane, scale);
    ISDF_HIP_TRY(hipGetLastError());
    return ISDF_OK;
  }
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(split_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, so, sk, kidx,
                     rows, cols, splits, dst, ldd, plane, scale);
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

}  // namespace isdf
