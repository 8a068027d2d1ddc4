// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/isdf.h"

namespace isdf {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
#define ISDF_HIP_TRY(expr)                                                        \
  do {                                                                            \
    hipError_t _e = (expr);                                                       \
    if (_e != hipSuccess) {                                                       \
      ::isdf::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));       \
      return _e == hipErrorOutOfMemory ? ISDF_E_NOMEM : ISDF_E_HIP;               \
    }                                                                             \
  } while (0)

// ------------------------------------------------------------ host plan
struct HostDomain {
  int level = 0;
  int atom = -1;                 // -1: universal domain
  std::vector<int32_t> points;   // ascending flat grid indices
  std::vector<int32_t> funcs;    // L then N, basis order
  int nL = 0, nN = 0, n_mu = 0;
  double r_max = 0.0;
};

struct ShellDev {                // one periodic shell as the basis kernel sees it
  double alpha;
  double norm;
  int32_t l;
  int32_t img_off;
  int32_t img_cnt;
  int32_t pad;
};

struct ColShell {                // a shell occupying columns [col, col + ncomp) of a domain
  int32_t shell;
  int32_t col;
  uint64_t imask;                // bit m: image m of the shell can reach a point of the domain
                                 // (shells with more than 64 images scan them all)
};

struct HostPlan {
  double lattice[9];             // rows a_i
  double inv[9];                 // inverse lattice, frac = r @ inv
  double volume;
  double ln_inv_tau;
  int n_atoms = 0;
  std::vector<double> xyz;
  int n_shells = 0;
  std::vector<int32_t> shell_atom, shell_l, shell_level;
  std::vector<double> shell_alpha;
  std::vector<int32_t> img_off, img_cnt;
  std::vector<double> img_xyz;   // image centres A + T
  int n_basis = 0;
  std::vector<int32_t> f_shell, f_atom, f_comp, f_level;
  int n_levels = 0;
  int grid[8][3];
  std::vector<double> alpha_bound;
  double eps_r, n_mu_ratio, eps_isdf, tie_tol;
  std::vector<HostDomain> domains;
  int domain_mode = 0;
  int64_t n_mu_total = 0;
};

// Builds the plan on the host (validates the system).  Returns ISDF_OK or an
// error status with set_error() called.
isdf_status build_host_plan(const isdf_system* sys, HostPlan& hp);

// Grid ladder for a Fourier threshold eps_K (isdf_grids_for_threshold).
isdf_status threshold_grids(const double* lattice, int n_shells, const double* shell_alpha,
                            int n_levels, const double* alpha_bound, double eps_K, int32_t* out);

// -------------------------------------------------------------- GEMM engine
// Column-major FP64 GEMM problem:  C(m,n) = epi( sum_k opA(m,k) opB(k,n) ).
//   opA(m,k) = transA ? A[k + m*lda] : A[m + k*lda]
//   opB(k,n) = transB ? B[n + k*ldb] : B[(bidx ? bidx[k] : k) + n*ldb]
// Epilogues: EPI_AXPBY  C = alpha*acc + beta*C
//            EPI_THETA  acc split at k = kL: C = aL*(aL + 2*aN)
//            EPI_HADAMARD C = alpha*acc*E(m,n) (+ beta*C)
// EPI_HADAMARD_PLANES (split-BF16 products only): C o E written as the split
// planes of the transposed product, element (m, n) at P + plane_p s + n ldp +
// p_off + m for plane s.
enum { EPI_AXPBY = 0, EPI_THETA = 1, EPI_HADAMARD = 2, EPI_HADAMARD_PLANES = 3 };
struct GemmProblem {
  const double* A;
  const double* B;
  double* C;
  const double* E;
  const int32_t* bidx;
  int64_t lda, ldb, ldc, lde;
  int32_t M, N, K, kL;
  int32_t transA, transB;
  double alpha, beta;
  int32_t tile_start;            // first flat tile of this problem in a grouped launch
  int32_t lower;                 // 1: only tiles touching the lower triangle (m >= n)
  const float* E32;              // EPI_HADAMARD: E held in FP32 (read instead of E when set)
  // Tile masks of density screening (64 x 64 tiles; 64 x 64 tile shape only):
  // mode 1 leaves out output tile (tm, tn) when tmask[tm s0 + tn s1] == 0
  // (C = beta C there); mode 2 leaves out the K range [64 q, 64 q + 64) of
  // output row tile tm when tmask[tm s0 + q s1] == 0 (A is zero there).
  const uint8_t* tmask;
  int64_t tm_s0, tm_s1;
  int32_t tmask_mode;
  int32_t pad_t;
};

// Launch one problem or a group (device array of problems, tile_start
// filled by the caller, total_tiles = sum of tiles).
// tag: 0 generic, 1 selection Gram / residual updates, 2 Coulomb metric,
// 3 fit (Theta, Cholesky, solves), 4 exchange
// Tile shapes of the FP64 GEMM (index into kShapes).  Single problems take
// `shape` < 0 to mean the default for their size; a grouped launch names its
// shape, and its tile_start/total_tiles must be counted with gemm_tiles of
// that shape.
struct GemmShape {
  int bm, bn, wm, wn;
  int mf4;  // 1: v_mfma_f64_4x4x4 (4 blocks), 0: v_mfma_f64_16x16x4, 2: the large-tile
            // 4x4x4 kernel (gemm_big_kernel)
};
constexpr int GEMM_NSHAPE = 16;
extern const GemmShape kShapes[GEMM_NSHAPE];
// False for tile shapes that take A stored k-fastest (transA) only.
bool gemm_shape_takes_mfast_a(int shape);
// False for tile shapes that take B stored k-fastest (not transB) only.
bool gemm_shape_takes_nfast_b(int shape);
isdf_status gemm_f64(hipStream_t s, int epi, const GemmProblem& p, int tag = 0, int shape = -1);
// ta, tb: the operand layouts every problem of the group shares (required by
// the large-tile shapes, whose layouts are compile-time; -1 otherwise).
isdf_status gemm_f64_grouped(hipStream_t s, int epi, const GemmProblem* d_probs, int nprob,
                             int total_tiles, int tag = 0, int shape = 0, int ta = -1, int tb = -1);
int gemm_tiles(int M, int N, int shape = 0, bool lower = false);
int gemm_default_shape(int epi, int M, int N, int K, bool lower = false);

// ------------------------------------------------------------ other kernels
struct BasisTile {
  int32_t domain;
  int32_t start;
};
struct DomainDev {
  int64_t pts_off;               // into the points pool
  int64_t phi_off;               // into the Phi pool (pts x nG, column-major)
  int64_t diag_off;              // into the diag pool
  int32_t pts, nG, nL, n_mu;
  int32_t colshell_off, colshell_cnt;
  int32_t level;
  int32_t pad;
};
struct LatticeArg {
  double a[9];
  double ln_inv_tau;
  int32_t grid[8][3];
};
// aux (optional, 4 per point): a_L, a_N, max_{mu in L} mu^2, sum_{mu in L} mu
isdf_status launch_basis_eval(hipStream_t s, const LatticeArg& lat, const ShellDev* shells,
                              const double* img, const ColShell* colshells,
                              const DomainDev* doms, const int32_t* points,
                              const BasisTile* tiles, int ntiles, double* phi, double* diag,
                              double* aux);

// Selection (pivoted Cholesky) over a batch of domains.
struct SelDomain {
  int64_t phi_off, lfac_off, diag_off, prow_off;
  int32_t pts, nG, nL, n_mu;
  int32_t tile_off, ntiles;
  int32_t piv_off, pad;
};
enum { SEL_END_COUNT = 1, SEL_END_EPS = 2, SEL_END_BLOCK = 3 };
struct SelState {
  double d0max;
  double dpiv;
  int32_t cur;
  int32_t done;
  int32_t count;
  int32_t reason;                // SEL_END_* once done
};
constexpr int SEL_TILE = 64;
isdf_status launch_sel_init(hipStream_t s, const SelDomain* doms, const int32_t* tile_dom,
                            int tile_base, int ntiles, const double* diag, double* tmax,
                            int32_t* tidx, double tau, double* tval = nullptr);
isdf_status launch_sel_select(hipStream_t s, const SelDomain* doms, int dom_base, int ndom,
                              int k, SelState* st, const double* phi, const double* lfac,
                              double* diag, const double* tmax, const int32_t* tidx, double* prow,
                              int32_t* piv, double tau, double eps);
// Left-looking column: from the basis values and all k previous factor columns.
isdf_status launch_sel_column(hipStream_t s, const SelDomain* doms, const int32_t* tile_dom,
                              int tile_base, int ntiles, int k, const SelState* st,
                              const double* phi, double* lfac, double* diag,
                              const double* prow, double* tmax, int32_t* tidx, double tau);

// Gather of the pivot rows of Phi into per-domain X rows and the global
// X^L / X^N (column-major N_mu x N).
struct GatherDom {
  int64_t phi_off;
  int64_t xrow_off;              // into Xrows pool (count x nG, column-major nG x count)
  int32_t pts, nG, nL, count;
  int32_t xoff;                  // first global xi index
  int32_t piv_off;
  int32_t func_off;              // into the per-domain function list pool
  int32_t pad;
};
// ------------------------------------------- candidate-restricted blocks
struct CrbInfo {
  int32_t nc;       // candidates listed
  int32_t nactive;  // points not yet chosen
  double theta;     // largest d outside the candidates (-1: none)
  double dmax;      // largest d
};
isdf_status launch_crb_candidates(hipStream_t s, const double* d, int n, int T, int32_t* cidx,
                                  double* dC, CrbInfo* info);
// A block of greedy steps on the candidates, passed by value to every step:
// step k reads copy k & 1 of the diagonal and tile maxima and writes the
// other.  (One struct argument keeps the launch cost down: the steps are
// bound by it.)
struct CrbBlock {
  const double* R;  // residual R_CC, lower, nc x nc
  double* Lb;       // the block's candidate factor columns, nc x nb
  double* d[2];
  double* t[2];
  int32_t* i[2];
  double* v[2];  // residual at each tile's tie candidate i[c][tile]
  SelState* st;
  int32_t* pivC;  // block pivots, candidate positions
  int32_t nc, nb;
  double tau, eps, dstop, d0max;
};
isdf_status launch_crb_step(hipStream_t s, int k, const CrbBlock& b);
isdf_status launch_crb_gather(hipStream_t s, const double* src, int64_t lds, const int32_t* idx, int nr,
                              int nc, double* dst, int64_t ldd);
isdf_status launch_crb_trsm_block(hipStream_t s, double* X, int64_t ldx, int n, const double* U,
                                  int64_t ldu, int jb, int nb);
isdf_status launch_crb_diag(hipStream_t s, double* d, int n, const double* L, int64_t ldl, int nb,
                            const int32_t* piv);

isdf_status launch_gather_x(hipStream_t s, const GatherDom* doms, int ndom, int max_rows,
                            const double* phi, const int32_t* piv, const int32_t* funcs,
                            double* xrows, double* XL, double* XN, int64_t nmu);

isdf_status launch_fill(hipStream_t s, double* p, int64_t n, double v);
// Density screening: tile maxima of |A| (nt x n, column-major), of |W| over
// tiles (nt x nt), and masks B >= tau.
isdf_status launch_tile_absmax(hipStream_t s, const double* A, int64_t lda, int m, int n, int block,
                               double* out);
isdf_status launch_tile_absmax_w(hipStream_t s, const double* W, const float* W32, int64_t ld, int m, int block,
                                 double* out);
isdf_status launch_mask_ge(hipStream_t s, const double* B, int64_t n, double tau, uint8_t* mask);
// p(i, i) = v for i < n (column-major, leading dimension ld)
isdf_status launch_set_diag(hipStream_t s, double* p, int64_t ld, int n, double v);
// dst(i, c) = alpha src(idx ? idx[i] : i, c) for i < rows, c < cols (column-major)
isdf_status launch_scale_rows(hipStream_t s, const double* src, int64_t lds, const int32_t* idx, int rows,
                              int cols, double alpha, double* dst, int64_t ldd);
// y = (float) x, n values (FP32 storage of an FP64 result).
isdf_status launch_narrow(hipStream_t s, const double* x, float* y, int64_t n);
// C(m, n) = c (c + 2 t), c = C(m, n) (ldc), t = T(m, n) (ldt = M; 0 if T is null)
isdf_status launch_theta_combine(hipStream_t s, double* C, int64_t ldc, const double* T, int M, int N);
isdf_status launch_gather_square(hipStream_t s, const double* theta, int64_t pts, int n,
                                 const int32_t* piv, double* M);
// small domains (n <= 64): Cholesky of M = Theta[piv,:] and F = Theta M^-1 per row
struct SmallFitDom {
  int64_t theta_off;             // Theta and F share the layout (pts x n column-major)
  int32_t pts, n, piv_off, row_tile_off;
};
isdf_status launch_small_fit(hipStream_t s, const SmallFitDom* doms, const int32_t* tile_dom,
                             int ntiles, const double* theta, const int32_t* piv, double* F,
                             int32_t* status, int nmax);
// 64 x 64 diagonal-block Cholesky + inverse of the factor (blocked path)
isdf_status launch_potrf_diag(hipStream_t s, double* M, int64_t ldm, double* Cf, int64_t ldc,
                              double* inv, int w, int32_t* status);

// FFT: batched 3D complex transforms, in place, sign -1 forward / +1 inverse
// (unnormalised).  z holds `batch` complex arrays of n1 n2 n3 (x fastest).
isdf_status fft3d(hipStream_t s, double* z, int batch, const int grid[3], int sign,
                  const double** unused);
// allocate the twiddle table of an axis length ahead of any stream work
isdf_status fft_prepare(int n);
// out[b] (grid gc, complex) = v(m) * zf[b](m) / Ng_fine for m in J_gc \ {0}, else 0;
// B[i*3 + j] = component j of reciprocal vector b_i (a_i . b_j = 2 pi delta_ij)
isdf_status launch_poisson_restrict(hipStream_t s, const double* zf, const int gf[3], double* zc,
                                    const int gc[3], int batch, const double B[9]);
// scatter domain columns into complex pair arrays: z[slot/2][2 pts[i] + slot%2] = src[i]
// Pruned forward transform: one fitting-function column (compact values of
// its domain) and one pair of columns with the cyclic box that holds them.
struct FwdCol {
  const double* src;             // values at the domain's points (nullptr: zero column)
  const int32_t* map;            // box -> local point index (-1 outside); nullptr: src is the whole grid
  int32_t box[6];                // x0, y0, z0, ex, ey, ez (cyclic start and extent per axis)
};
struct FwdPair {
  int32_t c0, c1;                // columns (c1 = -1: none)
  int32_t box[6];                // box holding both columns
};
bool fft_forward_pruned_supported(const int g[3]);
// Forward transforms of npairs column pairs on grid g into z (pair b at
// b * N_g); max_yz / max_z bound the pairs' box lines and planes.  ev (6
// events or null): ev[2 p] and ev[2 p + 1] are recorded around pass p.
isdf_status fft_forward_pruned(hipStream_t s, double* z, const FwdPair* pairs, const FwdCol* cols,
                               int npairs, const int g[3], int max_yz, int max_z,
                               hipEvent_t* ev = nullptr);

struct ScatterCol {
  const double* src;
  const int32_t* pts;
  int32_t n;
  int32_t slot;
};
isdf_status launch_scatter_cols(hipStream_t s, const ScatterCol* cols, int ncols, int max_n,
                                double* z, int64_t ng);
// V[c][R] = component c%2 of z[c/2][R], c < ncols
isdf_status launch_split_planar(hipStream_t s, const double* z, int64_t ng, int ncols, double* V);
// Poisson step from the spectrum on grid gf, inverse transform on grid gc
// and planar split into V in three passes (*done = false: sizes without
// compiled passes, nothing launched; use the three separate steps).  ev as
// for fft_forward_pruned.
isdf_status fft_poisson_inverse(hipStream_t s, const double* zf, const int gf[3], double* zc,
                                const int gc[3], int npairs, const double B[9], double* V,
                                int ncols, bool* done, hipEvent_t* ev = nullptr);
isdf_status launch_symmetrize_w(hipStream_t s, double* W, int64_t nmu, const int8_t* lev, const int32_t* dom);
isdf_status launch_add(hipStream_t s, const double* a, const double* b, double* c, int64_t n);
isdf_status launch_sub(hipStream_t s, const double* a, const double* b, double* c, int64_t n);  // c = a - b
isdf_status launch_trace_dot(hipStream_t s, const double* a, const double* b, int64_t n,
                             double* partial, int nblk, double* out);

// universal grid with every point as a fitting function (kernels_universal.hip)
isdf_status launch_gather_rows_t(hipStream_t s, const double* C, int o, const int32_t* funcs, int n0,
                                 double* C0);
isdf_status launch_scatter_add_rows(hipStream_t s, const double* KC0, int n0, int o, const int32_t* funcs,
                                    double* KC);
isdf_status launch_scale_copy(hipStream_t s, const double* src, double* dst, int64_t n, double alpha);
isdf_status launch_pair_density(hipStream_t s, const double* E, int64_t ng, const int32_t* pairs, int ncols,
                                double* z);
isdf_status launch_z_accumulate_rows(hipStream_t s, const double* E, const double* V, int64_t ng, int o, int a0,
                                     int a1, double* Z);

// ------------------------------------------------------- mixed precision
// BF16-split GEMM problem: A planes hold (m, k) at A + p plane_a + m lda + k,
// B planes hold (k, n) at B + p plane_b + n ldb + k (k-contiguous, lda, ldb,
// plane strides multiples of 8).  Epilogues as for the FP64 engine; with
// EPI_THETA the split point kL must be a multiple of 32.
struct MixedProblem {
  const __bf16* A;
  const __bf16* B;
  double* C;
  const double* E;
  int64_t plane_a, plane_b, lda, ldb, ldc, lde;
  int32_t M, N, K, kL;
  double alpha, beta;
  int32_t tile_start;
  int32_t lower;
  __bf16* P;  // EPI_HADAMARD_PLANES output
  int64_t plane_p, ldp;
  int32_t p_off;
  const float* E32;  // Hadamard epilogues: E held in FP32 (read instead of E when set)
  int32_t tile_group;  // row tiles per group of the tile order (0: 8)
  int32_t pad_g;
};
isdf_status gemm_mixed(hipStream_t s, int epi, int splits, const MixedProblem& p, int tag = 4);
// Grouped problems on the wide-tile kernel (tile_start in units of
// mixed_tiles_wide); epilogues AXPBY, HADAMARD, HADAMARD_PLANES.  nprob < 0:
// -nprob problems with one M x N tile grid, interleaved tile by tile
// (total_tiles = -nprob x tiles of one).
isdf_status gemm_mixed_wide_grouped(hipStream_t s, int epi, int splits, const MixedProblem* d_probs,
                                    int nprob, int total_tiles, int tag = 4);
// out[i] = sum over s of parts[s count + i], s in order (deterministic).
isdf_status launch_sum_parts(hipStream_t s, const double* parts, int nparts, int64_t count, double* out);
isdf_status gemm_mixed_grouped(hipStream_t s, int epi, int splits, const MixedProblem* d_probs,
                               int nprob, int total_tiles, int tag = 4);
int mixed_tiles(int M, int N);
// Single mixed products (not Theta, not lower) with at least this many
// 64 x 128 tiles run on the wide-tile kernel.
#ifndef MIXED_WIDE_MIN_TILES
#define MIXED_WIDE_MIN_TILES 256
#endif
int mixed_tiles_wide(int M, int N);
// planes[p][o][k] (ld ldd, plane stride `plane`) of scale * src[o so + ks sk],
// ks = kidx ? kidx[k] : k (kidx[k] < 0 gives 0)
isdf_status launch_split_bf16(hipStream_t s, const double* src, int64_t so, int64_t sk,
                              const int32_t* kidx, int rows, int cols, int splits, __bf16* dst,
                              int64_t ldd, int64_t plane, double scale);

// ------------------------------------------------------- learned selector
constexpr int MLP_NPARAM = 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1;  // 5313
struct MlpGeom {
  double lat[9];
  double inv[9];
  int32_t n_atoms;
  int32_t n_levels;
};
struct MlpDomain {
  int64_t pts_off;
  int32_t pts, level, atom, nL, n_mu;
  int32_t grid[3];
  double rs, h, gmax, gmean;
};
struct CandDomain {
  int64_t pts_off, cand_off;
  int32_t pts, keep;
};
struct GatherRows {
  int64_t phi_off, diag_off, phic_off, diagc_off, cand_off;
  int32_t pts, nG, nc, pad;
};
struct JudgeDomain {
  int64_t diag_off, th_off;
  int32_t pts, n;
};
isdf_status launch_diag_stats(hipStream_t s, MlpDomain* doms, int ndom, const double* diag);
isdf_status launch_features(hipStream_t s, const MlpGeom& g, const MlpDomain* doms,
                            const int32_t* points, const BasisTile* tiles, int ntiles,
                            const double* aux, const double* diag, const double* atoms,
                            float* feats);
isdf_status launch_mlp_forward(hipStream_t s, const float* w, const float* X, int64_t n, float* z);
size_t mlp_grad_shmem();
// gradient of sum_p l_p * inv_count over batch rows [b0, b0 + bn) (through perm if given)
isdf_status launch_mlp_grad(hipStream_t s, const float* w, const float* X, const float* Y,
                            const int32_t* perm, int64_t b0, int64_t bn, float pw,
                            float inv_count, float* partial, float* lpart, float* grad,
                            float* loss);
isdf_status launch_adam(hipStream_t s, float* w, const float* g, float* m, float* v, float lr,
                        float b1, float b2, float eps, int t);
// candidates = the `keep` best logits of each domain plus every logit >= zcut;
// flag[pts_off + i] = 1 for candidates
isdf_status launch_topk_compact(hipStream_t s, const CandDomain* doms, int ndom, const float* z,
                                float zcut, int32_t* cand, int32_t* ncand, uint8_t* flag);
isdf_status launch_excluded_max(hipStream_t s, const JudgeDomain* doms, int ndom,
                                const double* diag, const uint8_t* flag, double* out);
isdf_status launch_gather_rows(hipStream_t s, const GatherRows* g, int ndom, int max_nc,
                               const double* phi, const double* diag, const int32_t* cand,
                               double* phic, double* diagc);
isdf_status launch_map_pivots(hipStream_t s, const int32_t* cand, int64_t cand_off,
                              const int32_t* pivc, int32_t* piv, int n);
isdf_status launch_final_residual(hipStream_t s, const JudgeDomain* doms, int ndom,
                                  const double* diag, const double* theta, const double* F,
                                  double* out);

}  // namespace isdf
