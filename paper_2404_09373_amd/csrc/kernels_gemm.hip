// FP64 GEMM on the CDNA4 matrix cores (v_mfma_f64_16x16x4f64).
//
// One kernel serves every dense contraction of the path: the Hadamard Gram
// Theta = A_L o (A_L + 2 A_N) (Eq. M(R,R) restricted to the pivots), the
// residual updates of the pivoted Cholesky, the triangular-solve updates of
// the least-squares fit (Eq. lsqr), the Coulomb-metric products
// W = dV F^T V (Eq. (xi|xi')) and the exchange products of Eq. ints.
// Problems are column-major; a launch may carry a group of independent
// problems of different sizes (one per domain).
//
// Tiling: a BM x BN output tile per workgroup of WM x WN waves, each wave
// (BM/WM) x (BN/WN) = FM x FN MFMA blocks of 16 x 16 (shapes in kShapes).
// K is staged through two LDS buffers in chunks of 16: the next chunk's
// global loads are issued into registers before the current chunk's MFMAs
// and land in the other buffer afterwards, one barrier per chunk.  The MFMA
// is fed B^T as its first operand and A^T as its second, so a lane's
// accumulators hold 16 consecutive rows of one C column: stores are
// contiguous along the column-major leading dimension.
//
// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2; the flat tile index is remapped so that every XCD walks a contiguous
// range of tiles (neighbouring tiles share A rows or B columns in its L2).
//
// Lane layouts of v_mfma_f64_16x16x4f64 (wave64):
//   operand 1: lane l holds X[i = l % 16][k = l / 16]
//   operand 2: lane l holds Y[k = l / 16][j = l % 16]
//   result   : lane l, register v holds D[i = l / 16 + 4 v][j = l % 16]
#include "common.h"

namespace isdf {

typedef double d4v __attribute__((ext_vector_type(4)));

namespace {
constexpr int BK = 16, PAD = 2, NXCD = 8;

// Loads through global-address-space views: the operands arrive as generic
// pointers inside a problem struct, and generic (flat) loads count against
// the LDS wait counter too, so each wait for an LDS fragment would also wait
// for the next chunk's global loads.
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) double* gdp;
typedef const __attribute__((address_space(1))) dv2* gd2p;
typedef const __attribute__((address_space(1))) int32_t* gip;
typedef const __attribute__((address_space(1))) uint8_t* gbp;
__device__ inline double gld(const double* p) { return *(gdp)p; }
__device__ inline dv2 gld2(const double* p) { return *(gd2p)p; }
__device__ inline int32_t gldi(const int32_t* p) { return *(gip)p; }
__device__ inline uint8_t gldb(const uint8_t* p) { return *(gbp)p; }
}  // namespace

// Loads of the large-tile kernel for elements outside a problem read this
// zero instead: every load is then unconditional (no branch around it and no
// select on the loaded value), so nothing waits for a chunk's loads before
// they are needed.
__device__ const double g_zero_elem = 0.0;

namespace {

__device__ inline const GemmProblem* find_problem(const GemmProblem* probs, int nprob, int tile) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile_start <= tile) lo = mid; else hi = mid - 1;
  }
  return probs + lo;
}

// Bijection of [0, nb): dispatch slot b (XCD b % 8) -> contiguous tile range.
__device__ inline int xcd_tile(int b, int nb) {
  const int x = b % NXCD, q = b / NXCD, per = nb / NXCD, rem = nb % NXCD;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + q;
}

// Per-thread global -> register loads of one K chunk.  Each thread owns
// fixed (row, column) slots of the A and B tiles; their addresses are formed
// once and advanced by a constant stride per chunk.  Interior chunks of
// interior tiles skip all bounds tests.
template <int BM_, int BN_, int NT>
struct TileLoader {
  static constexpr int NA = BM_ * BK / NT, NB = BN_ * BK / NT;
  // A rows: NT % BM_ == 0 for A stored m-fastest; a tile whose rows do not
  // divide the threads (80 or 48 rows) serves only A stored k-fastest
  // (transA), which the host enforces.  Likewise for B: NT % BN_ == 0 for B
  // stored n-fastest, and an 80-column tile takes B stored k-fastest only.
  static constexpr bool A_MFAST = NT % BM_ == 0;
  static constexpr bool B_NFAST = NT % BN_ == 0;
  static_assert((A_MFAST || (NT / BK) * NA == BM_) && (B_NFAST || (NT / BK) * NB == BN_) && NT % BK == 0 &&
                    NA >= 1 && NB >= 1,
                "tile");
  double ra[NA], rb[NB];
  const double* pa;  // slot r = 0 of A at the current chunk
  const double* pb;  // slot r = 0 of B (rows gathered: column base only)
  int64_t sa, sb;    // pointer step between slots r and r + 1
  int64_t ca, cb;    // pointer step per chunk
  int am, ak, bn, bk;  // this thread's tile coordinates of slot 0
  bool a_ok[NA], b_ok[NB];  // row/column inside the problem (slot-wise)
  int32_t nrow;        // gathered B rows: this thread's row of the chunk loaded next

  __device__ void init(const GemmProblem& p, int m0, int n0, int tid) {
    if (!p.transA) {  // A(m, k) at m + k lda: m fastest
      am = A_MFAST ? tid % BM_ : 0;
      ak = A_MFAST ? tid / BM_ : 0;
      pa = p.A + (int64_t)(m0 + am) + (int64_t)ak * p.lda;
      sa = (int64_t)(A_MFAST ? NT / BM_ : 0) * p.lda;
      ca = (int64_t)BK * p.lda;
#pragma unroll
      for (int r = 0; r < NA; ++r) a_ok[r] = A_MFAST && m0 + am < p.M;
    } else {  // A(m, k) at k + m lda: k fastest
      ak = tid % BK;
      am = tid / BK;
      pa = p.A + (int64_t)ak + (int64_t)(m0 + am) * p.lda;
      sa = (int64_t)(NT / BK) * p.lda;
      ca = BK;
#pragma unroll
      for (int r = 0; r < NA; ++r) a_ok[r] = m0 + am + (NT / BK) * r < p.M;
    }
    if (!p.transB) {  // B(k, n) at row(k) + n ldb: k fastest
      bk = tid % BK;
      bn = tid / BK;
      pb = p.B + (int64_t)(n0 + bn) * p.ldb;
      sb = (int64_t)(NT / BK) * p.ldb;
      cb = BK;
#pragma unroll
      for (int r = 0; r < NB; ++r) b_ok[r] = n0 + bn + (NT / BK) * r < p.N;
      nrow = (p.bidx && bk < p.K) ? gldi(p.bidx + bk) : 0;
    } else {  // B(k, n) at n + k ldb: n fastest
      bn = B_NFAST ? tid % BN_ : 0;
      bk = B_NFAST ? tid / BN_ : 0;
      pb = p.B + (int64_t)(n0 + bn) + (int64_t)bk * p.ldb;
      sb = (int64_t)(B_NFAST ? NT / BN_ : 0) * p.ldb;
      cb = (int64_t)BK * p.ldb;
#pragma unroll
      for (int r = 0; r < NB; ++r) b_ok[r] = B_NFAST && n0 + bn < p.N;
    }
  }

  // chunk starting at k0 (the pointers sit at k0)
  __device__ void load(const GemmProblem& p, int k0) {
    const bool kfull = k0 + BK <= p.K;
    if (!p.transA) {
#pragma unroll
      for (int r = 0; r < NA; ++r) {
        const bool ok = a_ok[r] && (kfull || k0 + ak + (A_MFAST ? NT / BM_ : 0) * r < p.K);
        ra[r] = ok ? gld(pa + r * sa) : 0.0;
      }
    } else {
      const bool kok = kfull || k0 + ak < p.K;
#pragma unroll
      for (int r = 0; r < NA; ++r) ra[r] = (a_ok[r] && kok) ? gld(pa + r * sa) : 0.0;
    }
    if (!p.transB) {
      const bool kok = kfull || k0 + bk < p.K;
      int64_t row = k0 + bk;
      if (p.bidx) {
        // the row index was read one chunk ahead, so the value loads below do
        // not wait for an index load; read the next chunk's now
        row = nrow;
        const int kn = k0 + BK + bk;
        nrow = kn < p.K ? gldi(p.bidx + kn) : 0;
      }
#pragma unroll
      for (int r = 0; r < NB; ++r) rb[r] = (b_ok[r] && kok) ? gld(pb + row + r * sb) : 0.0;
    } else {
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        const bool ok = b_ok[r] && (kfull || k0 + bk + (B_NFAST ? NT / BN_ : 0) * r < p.K);
        rb[r] = ok ? gld(pb + r * sb) : 0.0;
      }
    }
  }

  __device__ void advance(const GemmProblem& p) {
    pa += ca;
    if (p.transB) pb += cb;  // gathered rows index from the column base
  }

  __device__ void store(const GemmProblem& p, double (*As)[BM_ + PAD], double (*Bs)[BN_ + PAD]) const {
    if (!p.transA) {
      if constexpr (A_MFAST) {
#pragma unroll
        for (int r = 0; r < NA; ++r) As[ak + (NT / BM_) * r][am] = ra[r];
      }
    } else {
#pragma unroll
      for (int r = 0; r < NA; ++r) As[ak][am + (NT / BK) * r] = ra[r];
    }
    if (!p.transB) {
#pragma unroll
      for (int r = 0; r < NB; ++r) Bs[bk][bn + (NT / BK) * r] = rb[r];
    } else {
      if constexpr (B_NFAST) {
#pragma unroll
        for (int r = 0; r < NB; ++r) Bs[bk + (NT / BN_) * r][bn] = rb[r];
      }
    }
  }
};

// Waves per SIMD that the register allocation must leave room for (the
// second launch-bounds argument): two workgroups per CU of the 512-thread
// AXPBY tile, three of the 256-thread AXPBY tiles and of the 64 x 64 Theta
// tile, one otherwise.  More resident workgroups keep more operand loads in
// flight; these bounds cost no spills (a few outside the main loop for the
// 512-thread tile), tighter ones spill inside it.
template <int EPI, int BM_, int BN_, int WM_, int WN_, int MF4>
constexpr int gemm_min_waves() {
  if (EPI == EPI_AXPBY && WM_ * WN_ == 8) return 4;
  if (BM_ == 80) return 2;  // its 53 KB of LDS allow two workgroups per CU anyway
  if (EPI == EPI_AXPBY && MF4 == 0 && WM_ * WN_ == 4) return 3;
  if (EPI == EPI_THETA && MF4 == 0 && BM_ == 64 && BN_ == 64 && WM_ * WN_ == 4) return 3;
  if (EPI == EPI_THETA && (BN_ == 80 || BN_ == 48)) return 3;
  return 1;
}
}  // namespace

// TAG only separates the instantiations per role (selection Gram, Coulomb
// metric, fit solves, exchange) so that profiles attribute time per role.
template <int EPI, int TAG, int BM_, int BN_, int WM_, int WN_, int MF4 = 0>
__global__ void __launch_bounds__(64 * WM_ * WN_, (gemm_min_waves<EPI, BM_, BN_, WM_, WN_, MF4>()))
gemm_f64_kernel(GemmProblem single, const GemmProblem* __restrict__ probs, int nprob) {
  constexpr int NT = 64 * WM_ * WN_;
  constexpr int TM = BM_ / WM_, TN = BN_ / WN_;  // wave tile
  constexpr int FM = TM / 16, FN = TN / 16;
  constexpr bool TWO = EPI == EPI_THETA;
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const GemmProblem* pp = probs ? find_problem(probs, nprob, tile) : &single;
  const GemmProblem p = *pp;
  const int tilesM = (p.M + BM_ - 1) / BM_;
  const int local = tile - p.tile_start;
  int tm, tn;
  if (BM_ == BN_ && p.lower) {
    // lower triangle of square tiles only, row by row: local = tm (tm + 1) / 2 + tn
    int r = (int)((sqrt(8.0 * (double)local + 1.0) - 1.0) * 0.5);
    while ((int64_t)(r + 1) * (r + 2) / 2 <= local) ++r;
    while ((int64_t)r * (r + 1) / 2 > local) --r;
    tm = r;
    tn = local - r * (r + 1) / 2;
  } else {
    tm = local % tilesM;
    tn = local / tilesM;
  }
  const int m0 = tm * BM_, n0 = tn * BN_;
  if (n0 >= p.N) return;
  if (p.lower && m0 + BM_ <= n0) return;  // tile strictly above the diagonal
  if (p.tmask_mode == 1 && !gldb(p.tmask + (int64_t)tm * p.tm_s0 + (int64_t)tn * p.tm_s1)) {
    // a screened-out tile: C = beta C
    for (int e = (int)threadIdx.x; e < BM_ * BN_; e += 64 * WM_ * WN_) {
      const int r = e % BM_, c = e / BM_;
      if (m0 + r < p.M && n0 + c < p.N) {
        double* cp = p.C + (int64_t)(m0 + r) + (int64_t)(n0 + c) * p.ldc;
        *cp = p.beta == 0.0 ? 0.0 : p.beta * *cp;
      }
    }
    return;
  }
  // mode 2: K ranges of 64 whose A rows of this tile are screened out are
  // neither loaded nor multiplied (the stage they would fill is not read)
  auto live = [&](int k) -> bool {
    return p.tmask_mode != 2 || gldb(p.tmask + (int64_t)tm * p.tm_s0 + (int64_t)(k >> 6) * p.tm_s1) != 0;
  };

  // two LDS stages: chunk c is read from stage c & 1 while chunk c + 1 is
  // written to the other, one barrier per chunk
  __shared__ double As[2][BK][BM_ + PAD];
  __shared__ double Bs[2][BK][BN_ + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM_, wn = wave / WM_;

  d4v acc[FM][FN], accN[TWO ? FM : 1][TWO ? FN : 1];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
  if (TWO) {
#pragma unroll
    for (int a = 0; a < (TWO ? FM : 1); ++a)
#pragma unroll
      for (int b = 0; b < (TWO ? FN : 1); ++b) accN[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
  }

  TileLoader<BM_, BN_, NT> ld;
  ld.init(p, m0, n0, tid);
  if (p.K > 0) {
    if (live(0)) ld.load(p, 0);
    ld.store(p, As[0], Bs[0]);
  }
  __syncthreads();
  int stage = 0;
  for (int k0 = 0; k0 < p.K; k0 += BK) {
    const bool more = k0 + BK < p.K;
    if (more) {
      ld.advance(p);
      if (live(k0 + BK)) ld.load(p, k0 + BK);  // in flight during the MFMAs below
    }
    if (!live(k0)) {
      // screened-out K range: nothing to multiply
    } else if constexpr (MF4) {
      // v_mfma_f64_4x4x4 (4 blocks): one instruction forms rows 0..15 of a
      // 16-row block against 4 columns; its B operand holds those 4 columns
      // once per block (lane 16 k + 4 blk + j: B[k][4 t + j])
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        const int kr = kk * 4 + (lane >> 4);
        double ya[FM], xq[FN][4];
#pragma unroll
        for (int a = 0; a < FM; ++a) ya[a] = As[stage][kr][wm * TM + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
          for (int t = 0; t < 4; ++t) xq[b][t] = Bs[stage][kr][wn * TN + b * 16 + 4 * t + (lane & 3)];
        if constexpr (TWO) {
          const int kb = k0 + kk * 4;
          const bool inL = (kb + (lane >> 4)) < p.kL;
#pragma unroll
          for (int a = 0; a < FM; ++a) {
            const double yL = inL ? ya[a] : 0.0, yN = inL ? 0.0 : ya[a];
#pragma unroll
            for (int b = 0; b < FN; ++b)
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                if (kb < p.kL)
                  acc[a][b][t] = __builtin_amdgcn_mfma_f64_4x4x4f64(yL, xq[b][t], acc[a][b][t], 0, 0, 0);
                if (kb + 4 > p.kL)
                  accN[TWO ? a : 0][TWO ? b : 0][t] = __builtin_amdgcn_mfma_f64_4x4x4f64(
                      yN, xq[b][t], accN[TWO ? a : 0][TWO ? b : 0][t], 0, 0, 0);
              }
          }
        } else {
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b)
#pragma unroll
              for (int t = 0; t < 4; ++t)
                acc[a][b][t] = __builtin_amdgcn_mfma_f64_4x4x4f64(ya[a], xq[b][t], acc[a][b][t], 0, 0, 0);
        }
      }
    } else
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      double xb[FN], ya[FM];
#pragma unroll
      for (int b = 0; b < FN; ++b) xb[b] = Bs[stage][kr][wn * TN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < FM; ++a) ya[a] = As[stage][kr][wm * TM + a * 16 + (lane & 15)];
      if constexpr (TWO) {
        const int kb = k0 + kk * 4;
        if (kb + 4 <= p.kL) {
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[b], ya[a], acc[a][b], 0, 0, 0);
        } else if (kb >= p.kL) {
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b)
              accN[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[b], ya[a], accN[a][b], 0, 0, 0);
        } else {
          const bool inL = (kb + (lane >> 4)) < p.kL;
          double xL[FN], xN[FN];
#pragma unroll
          for (int b = 0; b < FN; ++b) {
            xL[b] = inL ? xb[b] : 0.0;
            xN[b] = inL ? 0.0 : xb[b];
          }
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) {
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xL[b], ya[a], acc[a][b], 0, 0, 0);
              accN[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xN[b], ya[a], accN[a][b], 0, 0, 0);
            }
        }
      } else {
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[b], ya[a], acc[a][b], 0, 0, 0);
      }
    }
    if (more) ld.store(p, As[stage ^ 1], Bs[stage ^ 1]);
    __syncthreads();
    stage ^= 1;
  }
  // ---- epilogue: lane holds C(m0 + wm*TM + a*16 + lane%16, n0 + wn*TN + b*16 + lane/16 + 4v).
  // Per row block a, every read (C when beta != 0, E for the Hadamard) is
  // issued before any store, so the reads overlap instead of each waiting
  // out the previous store.
  const bool rd_c = !TWO && p.beta != 0.0;
  // (with the 4x4x4 instruction: lane holds C(m0 + wm*TM + a*16 + 4*((lane/4)%4) + lane/16,
  //  n0 + wn*TN + b*16 + 4v + lane%4))
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    const int gm = m0 + wm * TM + a * 16 + (MF4 ? 4 * ((lane >> 2) & 3) + (lane >> 4) : (lane & 15));
    if (gm >= p.M) continue;
    double cin[FN][4], ein[EPI == EPI_HADAMARD ? FN : 1][4];
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gn = n0 + wn * TN + b * 16 + (MF4 ? 4 * v + (lane & 3) : (lane >> 4) + 4 * v);
        const bool ok = gn < p.N;
        cin[b][v] = (rd_c && ok) ? p.C[(int64_t)gm + (int64_t)gn * p.ldc] : 0.0;
        if constexpr (EPI == EPI_HADAMARD)
          ein[b][v] = !ok ? 0.0
                          : p.E32 ? (double)p.E32[(int64_t)gm + (int64_t)gn * p.lde]
                                  : p.E[(int64_t)gm + (int64_t)gn * p.lde];
      }
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gn = n0 + wn * TN + b * 16 + (MF4 ? 4 * v + (lane & 3) : (lane >> 4) + 4 * v);
        if (gn >= p.N) continue;
        const double x = acc[a][b][v];
        double y;
        if constexpr (TWO) {
          y = x * (x + 2.0 * accN[TWO ? a : 0][TWO ? b : 0][v]);
        } else if constexpr (EPI == EPI_HADAMARD) {
          y = p.alpha * x * ein[EPI == EPI_HADAMARD ? b : 0][v] + p.beta * cin[b][v];
        } else {
          y = p.alpha * x + p.beta * cin[b][v];
        }
        p.C[(int64_t)gm + (int64_t)gn * p.ldc] = y;
      }
  }
}

// ---------------------------------------------------------------------------
// Large-tile FP64 GEMM on v_mfma_f64_4x4x4 (4 blocks).  On gfx950 this form
// issues at about 75 TFLOP/s in a register-only test, against 36-48 for
// v_mfma_f64_16x16x4, so the large products of the fit (blocked solves,
// Hadamard Grams, selection updates) and of the metric run here.
//
// A 128 x 128 tile per workgroup of 4 waves (2 x 2), 64 x 64 per wave, K in
// chunks of 16 through two LDS stages (one barrier per chunk; the next
// chunk's global loads are in flight during the current chunk's MFMAs).
// One instruction forms a 16 x 4 block (rows from the A operand, one lane
// per row and k; the 4 columns of B repeated in each of its 4 blocks), so a
// wave holds 4 x 16 accumulators and per k step of 4 reads 4 A values and 16
// B values per lane for 64 instructions.  The LDS rows are stored permuted
// so that those reads are contiguous (two and eight 16-byte reads):
//   A tile row r of wave row wm:   position wm 64 + (r % 16) 4 + r / 16
//   B tile column c of wave col wn: position wn 64 + (c % 4) 16 + c / 4
// Global loads move two doubles per request when the operand is 16-byte
// aligned along its contiguous axis (leading dimension even); otherwise one.
// PASS selects the k range: 0 all of K, 1 [0, kL), 2 [kL, K); with
// EPI_THETA the host runs pass 1 with the plain epilogue (C = a_L) and pass 2
// finishes C = c (c + 2 a_N) from the stored c.
namespace {
constexpr int BG = 128, BGPAD = 4;
}  // namespace

// Tile 128 x BGN, NW waves (2 x NW/2), wave tile 64 x (2 BGN / NW); K chunks
// of BKC; TA, TB the operand layouts (transA, transB of the problems).  No
// gathered rows.
template <int EPI, int TAG, int PASS, int NW, int BKC, int TA, int TB, int BGN>
__global__ void __launch_bounds__(64 * NW)
gemm_big_kernel(GemmProblem single, const GemmProblem* __restrict__ probs, int nprob) {
  constexpr int NT = 64 * NW;
  constexpr int WNW = NW / 2;          // waves along N
  constexpr int TN = BGN / WNW;        // wave tile columns (64 or 32)
  constexpr int FT = TN / 4;           // 4-column groups per wave (16 or 8)
  constexpr int NPA = BG * BKC / 2 / NT;   // A pairs per thread per chunk
  constexpr int NPB = BGN * BKC / 2 / NT;  // B pairs per thread per chunk
  constexpr int KH = BKC / 2;
  static_assert(NPA >= 1 && NPB >= 1 && (BG * BKC / 2) % NT == 0 && (BGN * BKC / 2) % NT == 0, "tile");
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const GemmProblem* pp = probs ? find_problem(probs, nprob, tile) : &single;
  const GemmProblem p = *pp;
  const int tilesM = (p.M + BG - 1) / BG;
  const int local = tile - p.tile_start;
  int tm, tn;
  if (p.lower) {
    int r = (int)((sqrt(8.0 * (double)local + 1.0) - 1.0) * 0.5);
    while ((int64_t)(r + 1) * (r + 2) / 2 <= local) ++r;
    while ((int64_t)r * (r + 1) / 2 > local) --r;
    tm = r;
    tn = local - r * (r + 1) / 2;
  } else {
    tm = local % tilesM;
    tn = local / tilesM;
  }
  const int m0 = tm * BG, n0 = tn * BGN;
  if (n0 >= p.N) return;
  // k range of this pass
  const int kL = p.kL < 0 ? 0 : (p.kL > p.K ? p.K : p.kL);
  const int kbeg = PASS == 2 ? kL : 0;
  const int kend = PASS == 1 ? kL : p.K;
  const int KK = kend - kbeg;

  __shared__ __attribute__((aligned(16))) double As[2][BKC][BG + BGPAD];
  __shared__ __attribute__((aligned(16))) double Bs[2][BKC][BGN + BGPAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  // operand geometry at k = kbeg
  const double* A = TA ? p.A + kbeg : p.A + (int64_t)kbeg * p.lda;
  const double* B = TB ? p.B + (int64_t)kbeg * p.ldb : p.B + kbeg;

  // Element e of pair q = tid + NT r of this thread:
  //   A non-trans: m = 2 (q % 64) + e, k = q / 64    A trans: k = 2 (q % KH) + e, m = q / KH
  //   B non-trans: k = 2 (q % KH) + e, n = q / KH
  //   B trans: n = 2 (q % (BGN/2)) + e, k = q / (BGN/2)
  // Every load is issued unconditionally (an element outside the problem
  // reads g_zero_elem), so the chunk's loads stay in flight with no
  // branches or early waits.
  // LDS positions: A row r of wave row wm at wm 64 + (r % 16) 4 + r / 16;
  // B column c of wave column wn at wn TN + (c % 4) FT + c / 4 (within the
  // wave's TN columns)
  auto posA = [](int m) { return (m >> 6) * 64 + (m & 15) * 4 + ((m >> 4) & 3); };
  auto posB = [](int n) { return (n / TN) * TN + (n & 3) * FT + ((n % TN) >> 2); };

  double la[NPA][2], lb[NPB][2];
  auto load = [&](int k0) {  // chunk [k0, k0 + BKC) relative to kbeg
#pragma unroll
    for (int r = 0; r < NPA; ++r) {
      const int q = tid + NT * r;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int m = TA ? q / KH : 2 * (q & 63) + e;
        const int k = TA ? 2 * (q % KH) + e : q >> 6;
        const int gm = m0 + m, gk = k0 + k;
        const bool ok = gm < p.M && gk < KK;
        const int64_t off = TA ? (int64_t)gk + (int64_t)gm * p.lda : (int64_t)gm + (int64_t)gk * p.lda;
        la[r][e] = gld(ok ? A + off : &g_zero_elem);
      }
    }
#pragma unroll
    for (int r = 0; r < NPB; ++r) {
      const int q = tid + NT * r;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int n = TB ? 2 * (q % (BGN / 2)) + e : q / KH;
        const int k = TB ? q / (BGN / 2) : 2 * (q % KH) + e;
        const int gn = n0 + n, gk = k0 + k;
        const bool ok = gn < p.N && gk < KK;
        const int64_t off = TB ? (int64_t)gn + (int64_t)gk * p.ldb : (int64_t)gk + (int64_t)gn * p.ldb;
        lb[r][e] = gld(ok ? B + off : &g_zero_elem);
      }
    }
  };
  auto store = [&](int st) {
#pragma unroll
    for (int r = 0; r < NPA; ++r) {
      const int q = tid + NT * r;
      if (!TA) {
        const int m = 2 * (q & 63), k = q >> 6;
        As[st][k][posA(m)] = la[r][0];
        As[st][k][posA(m + 1)] = la[r][1];
      } else {
        const int k = 2 * (q % KH), m = q / KH;
        As[st][k][posA(m)] = la[r][0];
        As[st][k + 1][posA(m)] = la[r][1];
      }
    }
#pragma unroll
    for (int r = 0; r < NPB; ++r) {
      const int q = tid + NT * r;
      if (!TB) {
        const int k = 2 * (q % KH), n = q / KH;
        Bs[st][k][posB(n)] = lb[r][0];
        Bs[st][k + 1][posB(n)] = lb[r][1];
      } else {
        const int n = 2 * (q % (BGN / 2)), k = q / (BGN / 2);
        Bs[st][k][posB(n)] = lb[r][0];
        Bs[st][k][posB(n + 1)] = lb[r][1];
      }
    }
  };

  double acc[4][FT];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int t = 0; t < FT; ++t) acc[a][t] = 0.0;

  if (KK > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  int stage = 0;
  const int i16 = lane & 15, j4 = lane & 3, kq = lane >> 4;
  for (int k0 = 0; k0 < KK; k0 += BKC) {
    const bool more = k0 + BKC < KK;
    if (more) load(k0 + BKC);
#pragma unroll
    for (int kk = 0; kk < BKC / 4; ++kk) {
      const int kr = kk * 4 + kq;
      const dv2* ap = reinterpret_cast<const dv2*>(&As[stage][kr][wm * 64 + i16 * 4]);
      const dv2* bp = reinterpret_cast<const dv2*>(&Bs[stage][kr][wn * TN + j4 * FT]);
      double av[4], bv[FT];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const dv2 v = ap[h];
        av[2 * h] = v.x;
        av[2 * h + 1] = v.y;
      }
#pragma unroll
      for (int h = 0; h < FT / 2; ++h) {
        const dv2 v = bp[h];
        bv[2 * h] = v.x;
        bv[2 * h + 1] = v.y;
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int t = 0; t < FT; ++t) acc[a][t] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[a], bv[t], acc[a][t], 0, 0, 0);
    }
    if (more) store(stage ^ 1);
    __syncthreads();
    stage ^= 1;
  }
  // epilogue: acc[a][t] is C(m0 + wm 64 + a 16 + 4 ((lane >> 2) & 3) + (lane >> 4),
  //                          n0 + wn TN + 4 t + (lane & 3))
  const int rsub = 4 * ((lane >> 2) & 3) + (lane >> 4);
  const bool rd_c = (PASS == 2) || (EPI != EPI_THETA && p.beta != 0.0);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int gm = m0 + wm * 64 + a * 16 + rsub;
    if (gm >= p.M) continue;
    double cin[FT], ein[EPI == EPI_HADAMARD ? FT : 1];
#pragma unroll
    for (int t = 0; t < FT; ++t) {
      const int gn = n0 + wn * TN + 4 * t + j4;
      const bool ok = gn < p.N;
      cin[t] = (rd_c && ok) ? gld(p.C + (int64_t)gm + (int64_t)gn * p.ldc) : 0.0;
      if constexpr (EPI == EPI_HADAMARD)
        ein[t] = !ok ? 0.0
                     : p.E32 ? (double)p.E32[(int64_t)gm + (int64_t)gn * p.lde]
                             : gld(p.E + (int64_t)gm + (int64_t)gn * p.lde);
    }
#pragma unroll
    for (int t = 0; t < FT; ++t) {
      const int gn = n0 + wn * TN + 4 * t + j4;
      if (gn >= p.N) continue;
      const double x = acc[a][t];
      double y;
      if constexpr (EPI == EPI_THETA) {
        y = PASS == 2 ? cin[t] * (cin[t] + 2.0 * x) : x;  // pass 1 stores a_L
      } else if constexpr (EPI == EPI_HADAMARD) {
        y = p.alpha * x * ein[EPI == EPI_HADAMARD ? t : 0] + p.beta * cin[t];
      } else {
        y = p.alpha * x + p.beta * cin[t];
      }
      p.C[(int64_t)gm + (int64_t)gn * p.ldc] = y;
    }
  }
}

// Tile shapes (BM x BN, waves WM x WN, instruction).  Shape 0 suits skinny
// and grouped window problems; the others trade registers per wave against
// operand reuse; shapes 5-7 use v_mfma_f64_4x4x4 (4 blocks), which issues
// about 1.5 times the FP64 rate of the 16x16x4 form on this chip; shapes 8-11
// are the large-tile kernel above (gemm_big_kernel); shapes 12 and 13 (80
// and 48 rows, one row of four waves) serve A stored k-fastest only: the 65-
// and 45-row windows of the Coulomb metric without the empty rows of a 128-
// or 64-row tile; shapes 14 and 15 (80 and 48 columns, one column of four
// waves) serve B stored k-fastest only: the Theta of windows with 65-80
// fitting functions in one column tile instead of two, and of windows with
// 33-48 in a 48-column tile.
const GemmShape kShapes[GEMM_NSHAPE] = {
    {64, 64, 2, 2, 0},  {128, 64, 2, 2, 0},  {128, 128, 2, 4, 0}, {128, 128, 4, 4, 0},
    {64, 128, 2, 2, 0}, {64, 64, 2, 2, 1},   {128, 128, 4, 4, 1}, {128, 64, 2, 2, 1},
    {128, 64, 2, 2, 2},  {128, 128, 2, 4, 2},  {128, 64, 2, 2, 2},  {128, 128, 2, 2, 2},
    {80, 128, 1, 4, 0}, {48, 128, 1, 4, 0}, {64, 80, 4, 1, 0}, {64, 48, 4, 1, 0}};

namespace {
template <int EPI, int TAG, int SH>
void launch_shape(hipStream_t s, const GemmProblem& single, const GemmProblem* probs, int nprob,
                  int tiles) {
  if constexpr (SH == 0)
    hipLaunchKernelGGL((gemm_f64_kernel<EPI, TAG, 64, 64, 2, 2>), dim3(tiles), dim3(256), 0, s,
                       single, probs, nprob);
  else if constexpr (SH == 1)
    hipLaunchKernelGGL((gemm_f64_kernel<EPI, TAG, 128, 64, 2, 2>), dim3(tiles), dim3(256), 0, s,
                       single, probs, nprob);
  else if constexpr (SH == 2)
    hipLaunchKernelGGL((gemm_f64_kernel<EPI, TAG, 128, 128, 2, 4>), dim3(tiles), dim3(512), 0, s,
                       single, probs, nprob);
  else if constexpr (SH == 3)
    hipLaunchKernelGGL((gemm_f64_kernel<EPI, TAG, 128, 128, 4, 4>), dim3(tiles), dim3(1024), 0, s,
                       single, probs, nprob);
  else if constexpr (SH == 4)
    hipLaunchKernelGGL((gemm_f64_kernel<EPI, TAG, 64, 128, 2, 2>), dim3(tiles), dim3(256), 0, s,
                       single, probs, nprob);
  else if constexpr (SH == 5)
    hipLaunchKernelGGL((gemm_f64_kernel<EPI, TAG, 64, 64, 2, 2, 1>), dim3(tiles), dim3(256), 0, s,
                       single, probs, nprob);
  else if constexpr (SH == 6)
    hipLaunchKernelGGL((gemm_f64_kernel<EPI, TAG, 128, 128, 4, 4, 1>), dim3(tiles), dim3(1024), 0,
                       s, single, probs, nprob);
  else if constexpr (SH == 12)
    hipLaunchKernelGGL((gemm_f64_kernel<EPI, TAG, 80, 128, 1, 4>), dim3(tiles), dim3(256), 0, s,
                       single, probs, nprob);
  else if constexpr (SH == 13)
    hipLaunchKernelGGL((gemm_f64_kernel<EPI, TAG, 48, 128, 1, 4>), dim3(tiles), dim3(256), 0, s,
                       single, probs, nprob);
  else if constexpr (SH == 14)
    hipLaunchKernelGGL((gemm_f64_kernel<EPI, TAG, 64, 80, 4, 1>), dim3(tiles), dim3(256), 0, s,
                       single, probs, nprob);
  else if constexpr (SH == 15)
    hipLaunchKernelGGL((gemm_f64_kernel<EPI, TAG, 64, 48, 4, 1>), dim3(tiles), dim3(256), 0, s,
                       single, probs, nprob);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<EPI, TAG, 128, 64, 2, 2, 1>), dim3(tiles), dim3(256), 0, s,
                       single, probs, nprob);
}

template <int EPI, int TAG, int NW, int BKC, int TA, int TB, int BGN>
void launch_big_t(hipStream_t s, const GemmProblem& single, const GemmProblem* probs, int nprob, int tiles) {
  if constexpr (EPI == EPI_THETA) {
    hipLaunchKernelGGL((gemm_big_kernel<EPI_THETA, TAG, 1, NW, BKC, TA, TB, BGN>), dim3(tiles), dim3(64 * NW), 0,
                       s, single, probs, nprob);
    hipLaunchKernelGGL((gemm_big_kernel<EPI_THETA, TAG, 2, NW, BKC, TA, TB, BGN>), dim3(tiles), dim3(64 * NW), 0,
                       s, single, probs, nprob);
  } else {
    hipLaunchKernelGGL((gemm_big_kernel<EPI, TAG, 0, NW, BKC, TA, TB, BGN>), dim3(tiles), dim3(64 * NW), 0, s,
                       single, probs, nprob);
  }
}

// The operand layouts of a big-tile launch are template arguments: a
// grouped launch passes the layout its problems share (gemm_f64_grouped
// checks), a single problem its own.
template <int EPI, int TAG, int NW, int BKC, int BGN>
void launch_big(hipStream_t s, const GemmProblem& single, const GemmProblem* probs, int nprob, int tiles, int ta,
                int tb) {
  if (ta && tb) launch_big_t<EPI, TAG, NW, BKC, 1, 1, BGN>(s, single, probs, nprob, tiles);
  else if (ta) launch_big_t<EPI, TAG, NW, BKC, 1, 0, BGN>(s, single, probs, nprob, tiles);
  else if (tb) launch_big_t<EPI, TAG, NW, BKC, 0, 1, BGN>(s, single, probs, nprob, tiles);
  else launch_big_t<EPI, TAG, NW, BKC, 0, 0, BGN>(s, single, probs, nprob, tiles);
}

template <int EPI, int TAG>
void launch_epi(hipStream_t s, int shape, const GemmProblem& single, const GemmProblem* probs,
                int nprob, int tiles, int ta, int tb) {
  switch (shape) {
    case 8: launch_big<EPI, TAG, 4, 16, 64>(s, single, probs, nprob, tiles, ta, tb); break;
    case 9: launch_big<EPI, TAG, 8, 16, 128>(s, single, probs, nprob, tiles, ta, tb); break;
    case 10: launch_big<EPI, TAG, 4, 32, 64>(s, single, probs, nprob, tiles, ta, tb); break;
    case 11: launch_big<EPI, TAG, 4, 16, 128>(s, single, probs, nprob, tiles, ta, tb); break;
    case 1: launch_shape<EPI, TAG, 1>(s, single, probs, nprob, tiles); break;
    case 2: launch_shape<EPI, TAG, 2>(s, single, probs, nprob, tiles); break;
    case 3: launch_shape<EPI, TAG, 3>(s, single, probs, nprob, tiles); break;
    case 4: launch_shape<EPI, TAG, 4>(s, single, probs, nprob, tiles); break;
    case 5: launch_shape<EPI, TAG, 5>(s, single, probs, nprob, tiles); break;
    case 6: launch_shape<EPI, TAG, 6>(s, single, probs, nprob, tiles); break;
    case 7: launch_shape<EPI, TAG, 7>(s, single, probs, nprob, tiles); break;
    case 12: launch_shape<EPI, TAG, 12>(s, single, probs, nprob, tiles); break;
    case 13: launch_shape<EPI, TAG, 13>(s, single, probs, nprob, tiles); break;
    case 14: launch_shape<EPI, TAG, 14>(s, single, probs, nprob, tiles); break;
    case 15: launch_shape<EPI, TAG, 15>(s, single, probs, nprob, tiles); break;
    default: launch_shape<EPI, TAG, 0>(s, single, probs, nprob, tiles); break;
  }
}

template <int TAG>
void launch_tag(hipStream_t s, int epi, int shape, const GemmProblem& single,
                const GemmProblem* probs, int nprob, int tiles, int ta, int tb) {
  if (epi == EPI_THETA)
    launch_epi<EPI_THETA, TAG>(s, shape, single, probs, nprob, tiles, ta, tb);
  else if (epi == EPI_HADAMARD)
    launch_epi<EPI_HADAMARD, TAG>(s, shape, single, probs, nprob, tiles, ta, tb);
  else
    launch_epi<EPI_AXPBY, TAG>(s, shape, single, probs, nprob, tiles, ta, tb);
}

isdf_status launch(hipStream_t s, int epi, int tag, int shape, const GemmProblem& single,
                   const GemmProblem* probs, int nprob, int tiles, int ta, int tb) {
  if (tiles <= 0) return ISDF_OK;
  if (epi != EPI_AXPBY && epi != EPI_THETA && epi != EPI_HADAMARD) {
    set_error("gemm: bad epilogue");
    return ISDF_E_ARG;
  }
  if (shape < 0 || shape >= GEMM_NSHAPE) {
    set_error("gemm: bad tile shape");
    return ISDF_E_ARG;
  }
  switch (tag) {
    case 1: launch_tag<1>(s, epi, shape, single, probs, nprob, tiles, ta, tb); break;
    case 2: launch_tag<2>(s, epi, shape, single, probs, nprob, tiles, ta, tb); break;
    case 3: launch_tag<3>(s, epi, shape, single, probs, nprob, tiles, ta, tb); break;
    case 4: launch_tag<4>(s, epi, shape, single, probs, nprob, tiles, ta, tb); break;
    default: launch_tag<0>(s, epi, shape, single, probs, nprob, tiles, ta, tb); break;
  }
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}
}  // namespace

// Measured on MI355X over the path's problem shapes: the 16-wave 128 x 128
// tile wins once there are enough tiles to fill the chip (or a long K keeps
// fewer tiles busy); skinny and mid-sized outputs keep the 64 x 64 tile.
int gemm_default_shape(int epi, int M, int N, int K, bool lower) {
  (void)epi;
  if (lower) return 3;
  const int64_t t128 = (int64_t)((M + 127) / 128) * ((N + 127) / 128);
  if (t128 >= 1024 || (t128 >= 128 && K >= 16384)) return 3;
  return 0;
}

bool gemm_shape_takes_mfast_a(int shape) {
  const GemmShape& g = kShapes[shape < 0 || shape >= GEMM_NSHAPE ? 0 : shape];
  return (64 * g.wm * g.wn) % g.bm == 0;
}

bool gemm_shape_takes_nfast_b(int shape) {
  const GemmShape& g = kShapes[shape < 0 || shape >= GEMM_NSHAPE ? 0 : shape];
  return (64 * g.wm * g.wn) % g.bn == 0;
}

int gemm_tiles(int M, int N, int shape, bool lower) {
  const GemmShape& g = kShapes[shape < 0 || shape >= GEMM_NSHAPE ? 0 : shape];
  if (lower && g.bm == g.bn) {  // square lower-triangle problems list only tiles with tm >= tn
    const int t = (N + g.bn - 1) / g.bn;
    return t * (t + 1) / 2;
  }
  return ((M + g.bm - 1) / g.bm) * ((N + g.bn - 1) / g.bn);
}

isdf_status gemm_f64(hipStream_t s, int epi, const GemmProblem& p, int tag, int shape) {
  if (p.M <= 0 || p.N <= 0) return ISDF_OK;
  GemmProblem q = p;
  q.tile_start = 0;
  // K <= 0 runs the epilogue alone: C = beta C
  if (p.lower && p.M != p.N) {
    set_error("gemm: a lower-triangle update must be square");
    return ISDF_E_ARG;
  }
  if (shape < 0) {
    // plain products with a long K and many rows (the blocked solves and
    // bulk factor columns of the fit) take the large 4x4x4 tile, measured
    // 10-25 % faster than the 64 x 64 tile there; the rest keep the size rule
    if (epi == EPI_AXPBY && !p.lower && !p.bidx && !p.transA && p.K >= 512 && p.M >= 4096 && p.N >= 256)
      shape = 8;
    else
      shape = gemm_default_shape(epi, p.M, p.N, p.K, p.lower != 0);
  }
  if (p.lower && kShapes[shape].bm != kShapes[shape].bn) {
    set_error("gemm: a lower-triangle update needs a square tile shape");
    return ISDF_E_ARG;
  }
  if (kShapes[shape].mf4 == 2 && p.bidx) {
    set_error("gemm: the large-tile shapes take no gathered rows");
    return ISDF_E_ARG;
  }
  if (!p.transA && !gemm_shape_takes_mfast_a(shape)) {
    set_error("gemm: this tile shape takes A stored k-fastest (transA) only");
    return ISDF_E_ARG;
  }
  if (p.transB && !gemm_shape_takes_nfast_b(shape)) {
    set_error("gemm: this tile shape takes B stored k-fastest only");
    return ISDF_E_ARG;
  }
  return launch(s, epi, tag, shape, q, nullptr, 1, gemm_tiles(p.M, p.N, shape, p.lower != 0), p.transA,
                p.transB);
}

isdf_status gemm_f64_grouped(hipStream_t s, int epi, const GemmProblem* d_probs, int nprob,
                             int total_tiles, int tag, int shape, int ta, int tb) {
  if (nprob <= 0) return ISDF_OK;
  if (shape >= 0 && shape < GEMM_NSHAPE && kShapes[shape].mf4 == 2 && (ta < 0 || tb < 0)) {
    set_error("gemm: a grouped large-tile launch needs the problems' shared operand layouts");
    return ISDF_E_ARG;
  }
  if (shape >= 0 && shape < GEMM_NSHAPE && !gemm_shape_takes_mfast_a(shape) && ta != 1) {
    set_error("gemm: a grouped launch of this tile shape needs problems with A stored k-fastest");
    return ISDF_E_ARG;
  }
  if (shape >= 0 && shape < GEMM_NSHAPE && !gemm_shape_takes_nfast_b(shape) && tb != 0) {
    set_error("gemm: a grouped launch of this tile shape needs problems with B stored k-fastest");
    return ISDF_E_ARG;
  }
  GemmProblem dummy{};
  return launch(s, epi, tag, shape, dummy, d_probs, nprob, total_tiles, ta, tb);
}

}  // namespace isdf
