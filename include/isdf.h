/*
 * isdf.h - C ABI of the MI355X multigrid-ISDF exchange library.
 *
 * Method: Smyser, White, Sharma, "Use of multigrids to reduce the cost of
 * performing interpolative separable density fitting" (arXiv 2404.09373).
 *
 *   isdf_plan      geometry -> grid levels, atom-centred windows and the
 *                  local / global / non-local function sets
 *                  (section "Computational details", Eqs. rcut, Ggrid and
 *                  "mg product density")
 *   isdf_fit       per domain: basis values, pair-density Gram (Eq. M(R,R)),
 *                  pivoted-Cholesky interpolation points, least-squares
 *                  fitting functions (Eq. lsqr); then the Coulomb metric
 *                  (xi|xi') by FFT Poisson solves (Eq. (xi|xi'))
 *   isdf_exchange  the four-term THC exchange matrix (Eq. ints) and
 *                  E_x = tr(D K), once per SCF iteration
 *
 * Conventions
 *   Units: Bohr and Hartree.  Basis functions are ordered atom-major as the
 *   shells are given, p components x, y, z.  Matrices crossing the ABI are
 *   dense FP64; N x N matrices (D, K) are symmetric so row- and column-major
 *   coincide.  Grid points are flat indices i1 + n1 (i2 + n2 i3) of the level
 *   grid.  Domain order: the universal level-0 domain first, then one window
 *   per atom for level 1, level 2, ...; interpolation points xi are ordered
 *   by domain, then by selection order.
 *
 *   Ownership: every array passed in is caller-owned and only read during
 *   the call (isdf_plan copies what it needs).  Handles are library-owned;
 *   destroy fits before their plan.  Device pointers (D, K) must be
 *   allocations on the current HIP device; the library never frees them.
 *
 *   Streams and errors: all device work is ordered on options.stream (a
 *   hipStream_t, NULL for the default stream).  No call throws.  Argument
 *   errors are returned synchronously; errors raised by kernels surface at
 *   the next call that synchronises (isdf_fit, isdf_exchange, isdf_sync and
 *   the copy-out calls all synchronise).  isdf_last_error() gives a message
 *   for the last non-OK status of the calling thread.
 *
 *   Threading: a plan and its fits must not be used from two threads at once.
 */
#ifndef ISDF_H
#define ISDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ISDF_OK = 0,
  ISDF_E_ARG = -1,         /* bad argument (null, NaN, out of range)            */
  ISDF_E_NOMEM = -2,       /* device or host allocation failed                  */
  ISDF_E_HIP = -3,         /* HIP runtime or kernel error                       */
  ISDF_E_NOT_SPD = -4,     /* interpolation metric not positive definite        */
  ISDF_E_RANK = -5,        /* fewer independent points than requested           */
  ISDF_E_STATE = -6,       /* handle used in the wrong state                    */
  ISDF_E_UNSUPPORTED = -7  /* grid or shell outside what the kernels support    */
} isdf_status;

typedef struct isdf_plan_s* isdf_plan_t; /* opaque, library-owned */
typedef struct isdf_fit_s* isdf_fit_t;   /* opaque, library-owned */

/* Precision of the fit / exchange contractions: FP64 MFMA, or BF16-split
 * operands (x = x0 + x1 [+ x2]) multiplied on BF16 MFMA with FP32
 * accumulation carried into FP64 every 256 terms; X3 keeps the 3 leading
 * products of 2-plane operands, X6 the 6 of 3-plane operands.  Cholesky
 * factors and triangular solves of the interpolation metric are FP64 in
 * every mode. */
enum { ISDF_FP64 = 0, ISDF_MIXED_X3 = 1, ISDF_MIXED_X6 = 2 };
enum { ISDF_MIX_THETA = 1, ISDF_MIX_W = 2, ISDF_MIX_EXCHANGE = 4 };
/* Candidate selection before pivoted Cholesky. */
enum { ISDF_SEL_FULL = 0, ISDF_SEL_MLP = 1 };

/* System description (section "Computational details"; the thresholds of
 * its threshold table).  All pointers are host pointers, read only. */
typedef struct {
  double lattice[9];          /* rows a1, a2, a3 (Bohr)                                  */
  int32_t n_atoms;
  const double* xyz;          /* [n_atoms][3] Cartesian positions (Bohr)                 */
  int32_t n_shells;
  const int32_t* shell_atom;  /* [n_shells] atom of each shell, atom-major order         */
  const int32_t* shell_l;     /* [n_shells] 0 (s), 1 (p: x, y, z) or 2 (d: the five real
                                 solid harmonics sqrt3 xy, sqrt3 yz, z^2 - (x^2+y^2)/2,
                                 sqrt3 xz, sqrt3/2 (x^2 - y^2), order m = -2..2);
                                 uncontracted primitives with unit single-centre norm  */
  const double* shell_alpha;  /* [n_shells] exponent (Bohr^-2)                           */
  int32_t n_levels;           /* 1..8                                                     */
  const int32_t* grid;        /* [n_levels][3] points per axis, coarse -> fine, each axis
                                 2^a 3^b 5^c and at most 256                               */
  const double* alpha_bound;  /* [n_levels-1] a shell lives on the coarsest level l with
                                 alpha < alpha_bound[l], else on the finest               */
  double image_tol;           /* periodic-image cutoff tau (e.g. 1e-10)                  */
  double eps_r;               /* window accuracy of Eq. rcut (e.g. 1e-5)                 */
  double n_mu_ratio;          /* points per owned function; <= 0: threshold only, n_mu,d
                                 = min(points, |L|(|L|+1)/2 + |L||N|), the rank bound of
                                 the domain's pair Gram                                   */
  double eps_isdf;            /* relative stop of the pivoted Cholesky (e.g. 1e-14)      */
  double tie_tol;             /* relative tie window of the pivot argmax (e.g. 1e-8)     */
  int32_t domain_mode;        /* 0: universal level-0 domain + one spherical window per
                                 atom on each finer level (section "Computational
                                 details"); 1: one domain per level over the whole level
                                 grid, L = the level's functions, N = all coarser ones  */
  int32_t pad_sys;
} isdf_system;

typedef struct {
  int32_t precision;          /* ISDF_FP64 (default) or a mixed mode                     */
  int32_t selector;           /* ISDF_SEL_FULL (default) or ISDF_SEL_MLP                 */
  double mlp_keep;            /* MLP: at least ceil(mlp_keep * n_mu_d) candidates / domain */
  double mlp_cutoff;          /* MLP: also every point with score >= mlp_cutoff (0..1)    */
  const float* mlp_weights;   /* MLP: host array of ISDF_MLP_NPARAM floats, copied       */
  void* stream;               /* hipStream_t or NULL                                      */
  int32_t w_batch;            /* most fitting functions whose potentials (on every grid)
                                 are held at once, and twice the most Poisson solves per
                                 FFT batch; bounds the Coulomb stage's memory (many plans
                                 fitting at once).  0: as many as 45 % of the free memory
                                 (at most 24 GB) holds                                    */
  int32_t mixed_mask;         /* contractions run in the mixed precision when precision
                                 is ISDF_MIXED_*: bit 0 Theta, bit 1 W (universal rows),
                                 bit 2 exchange; 0 means W and exchange                   */
  int32_t eager_exchange;     /* 0 (default): the exchange of a fit is captured as a HIP
                                 graph on its first call and replayed while the operand
                                 pointers stay the same; 1: always launch kernel by kernel */
  int32_t pad0;
  const char* tune_file;      /* JSON tile-shape table written by isdf_autotune, read at
                                 plan time (copied); NULL: the built-in size rule          */
  int32_t universal_all_points; /* 1: every universal grid point is a fitting function
                                 (the sinc functions of the sparse grid; no selection or
                                 fit there, (R_U|R_U') applied by FFT, never stored);
                                 the exchange is then available as K C only
                                 (isdf_exchange_occ_ri); needs atom windows             */
  int32_t universal_tile_mb;  /* most MB of universal pair potentials held at once (their
                                 pairs go in row tiles); 0: the smaller of 16 GB and 40 %
                                 of the free memory                                       */
  int32_t w_storage;          /* ISDF_W_F64 (default) or ISDF_W_F32: the Coulomb metric
                                 W = (xi|xi') (Eq. (xi|xi')) is formed in FP64 and, with
                                 F32, kept in FP32 after the fit (half the memory and the
                                 exchange's reads of it; entries rounded to 24 bits)      */
  int32_t pad1;
  void* workspace;            /* caller-owned device buffer (e.g. torch.empty), 256-byte
                                 aligned, or NULL: the plan then takes every device buffer
                                 of its fits and exchanges from it (never hipMalloc) and
                                 returns ISDF_E_NOMEM when it runs out; it must outlive the
                                 plan and its fits.  Size it with isdf_plan_workspace_bytes
                                 after a fit and exchange of a plan without one.  (Process-
                                 wide FFT twiddle tables and the 64 MB pinned host staging
                                 ring are not part of it.)                                */
  size_t workspace_bytes;
  int32_t phi_budget_mb;      /* most MB of basis values (Phi of Eq. (Theta)) held at once.
                                 When the domains' Phi exceeds it, the fit runs over
                                 consecutive domain groups that fit it, evaluating the
                                 basis twice (selection pass, then the pass that gathers
                                 X and forms Theta and F) and keeps no Phi afterwards
                                 (ISDF_FIELD_PHI then returns ISDF_E_STATE); the results
                                 are those of the one-pass fit.  0: 40 % of the free
                                 memory                                                   */
  int32_t ri_rows;            /* rows of Q = W o (E E^T) that isdf_exchange_occ_ri holds
                                 at once (row blocks of Z1, Z2; the result does not
                                 depend on it).  0: all N_mu rows when they fit a
                                 quarter of the free memory, else blocks of a multiple
                                 of 256 rows that fit 15 % of it                          */
  double ri_screen_tau;       /* density screening of isdf_exchange_occ_ri (the near-
                                 sightedness of the density matrix, Conclusions): fitting
                                 indices in tiles of 64; a tile (b, c) of Q_ST =
                                 W o (E_S E_T^T) is left out when
                                 max_{b x c}|W| sum_i max_b|E_S(., i)| max_c|E_T(., i)|
                                 is below it (a bound on every |Q| entry of the tile),
                                 skipping its products.  Pays off with localised
                                 occupied orbitals.  0 (default): no screening.  Needs
                                 the FP64 exchange (no mixed bit 2)                       */
} isdf_options;
/* Storage of the Coulomb metric W held by a fit. */
enum { ISDF_W_F64 = 0, ISDF_W_F32 = 1 };

/* Build the multigrid plan (host only, no device work).
 * Reads sys and opts; on success *out owns copies of everything it needs.
 * Errors: ISDF_E_ARG for null pointers, non-positive grids, NaN exponents,
 * domain_mode outside {0, 1}; ISDF_E_UNSUPPORTED for grids that are not
 * 2,3,5-smooth, axes above 256, levels that are not strictly finer, or
 * l > 2. */
isdf_status isdf_plan(const isdf_system* sys, const isdf_options* opts, isdf_plan_t* out);

/* Grid ladder from the Fourier threshold eps_K (Eq. Ggrid; the threshold
 * table of the "Computational details" section).  Host only.
 * For level l, a_l is the largest exponent among the shells living on it
 * (the level rule of isdf_system) and G_max,l = sqrt(-4 a_l ln eps_K).
 * Axis i of level l gets the smallest even 2,3,5-smooth length n whose kept
 * band |m_i| <= n/2 - 1 (the Nyquist plane is not kept) holds the index m_i
 * of every reciprocal vector G = 2 pi sum_j m_j b_j with |G| <= G_max,l;
 * a level is never coarser than the one below it.
 *   lattice      [3][3] host, rows a_i (Bohr)
 *   shell_alpha  [n_shells] host, exponents (Bohr^-2)
 *   alpha_bound  [n_levels-1] host (may be NULL when n_levels == 1)
 *   grid_out     [n_levels][3] host, caller-owned; written on success only
 * Errors: ISDF_E_ARG (null pointers, counts out of range, eps_K outside
 * (0, 1), a non-positive exponent, a level holding no shell, a singular
 * lattice); ISDF_E_UNSUPPORTED when an axis would need more than 256
 * points. */
isdf_status isdf_grids_for_threshold(const double* lattice, int32_t n_shells,
                                     const double* shell_alpha, int32_t n_levels,
                                     const double* alpha_bound, double eps_K, int32_t* grid_out);

/* Device bytes the plan's buffers have needed at once so far (blocks in use
 * plus the plan's block cache, the high-water mark over its fits and
 * exchange builds; 0 before any device work).  After one isdf_fit and the
 * exchange calls of a plan made without a workspace, this is the size of a
 * workspace with which a plan of the same system and options repeats them
 * without allocating. */
isdf_status isdf_plan_workspace_bytes(isdf_plan_t plan, size_t* bytes);

/* Device blocks the plan has taken so far (hipMalloc calls, or carve-outs
 * of the workspace): count, bytes and host milliseconds spent in them.  A
 * plan keeps the blocks its fits and exchanges release and serves later
 * requests of the same size from them, so repeated fits of one plan should
 * add none (any arguments may be NULL). */
isdf_status isdf_plan_alloc_stats(isdf_plan_t plan, int64_t* calls, double* bytes, double* ms);

/* Sizes: number of basis functions N, total requested points N_mu, domains. */
isdf_status isdf_plan_info(isdf_plan_t plan, int64_t* n_basis, int64_t* n_mu, int32_t* n_domains);

/* Domain d: level, centre atom (-1 for the universal domain), point count,
 * |L|, |N| and requested point count n_mu_d. */
isdf_status isdf_plan_domain(isdf_plan_t plan, int32_t d, int32_t* level, int32_t* atom,
                             int64_t* n_points, int32_t* n_L, int32_t* n_N, int32_t* n_mu);

/* Copy domain d's flat grid indices (ascending, n_points entries) and its
 * function indices (n_L local then n_N non-local, basis order) to host
 * arrays of the stated sizes. */
isdf_status isdf_plan_domain_points(isdf_plan_t plan, int32_t d, int64_t* points);
isdf_status isdf_plan_domain_functions(isdf_plan_t plan, int32_t d, int32_t* functions);

/* Fit (interpolative decomposition + Coulomb metric), once per geometry
 * (section "Using multiple grids for exchange", item 1).  Allocates the
 * fit's device buffers, runs every stage on the plan's stream and
 * synchronises.  With n_mu_ratio > 0, a domain whose requested count
 * n_mu_d equals its point count (the cap of the n_mu rule) takes every
 * point, in ascending order, with F_d = I: its pair densities are then
 * exact on the grid, no selection or solve runs and its Theta is not
 * formed (ISDF_FIELD_THETA gives zeros).
 * Errors: ISDF_E_NOMEM, ISDF_E_HIP, ISDF_E_NOT_SPD (a local interpolation
 * metric failed its Cholesky), ISDF_E_RANK (a domain stopped early by
 * eps_isdf while n_mu_ratio > 0; the fit is still usable). */
isdf_status isdf_fit(isdf_plan_t plan, isdf_fit_t* out);

/* Fits of several plans (independent cells of a batch) at once: up to
 * max_concurrent (<= 0: 4) host threads each take the next plan, largest
 * N_mu first, and run isdf_fit on it, so that the cells' kernels and host
 * decisions overlap on the GPU.  Plans made with a NULL stream get a
 * private stream for the duration of the call; give plans their own
 * streams otherwise (fits of plans that share a stream serialise).  The
 * plans must be distinct and must not be used by other threads meanwhile.
 * fits[i] receives the fit of plans[i] (NULL where it failed);
 * statuses[i] (may be NULL) its status.  Returns ISDF_OK or the status of
 * the first failed plan in index order (message names the plan); the
 * caller destroys every non-NULL fit either way.  Results equal those of
 * isdf_fit on each plan alone. */
isdf_status isdf_fit_batch(const isdf_plan_t* plans, int32_t n, int32_t max_concurrent,
                           isdf_fit_t* fits, isdf_status* statuses);

/* Same with the points of every domain given instead of selected:
 * local_points holds, domain after domain, n_mu_d local point indices
 * (positions in the domain's point list).  Duplicate points make the
 * metric singular and return ISDF_E_NOT_SPD. */
isdf_status isdf_fit_with_points(isdf_plan_t plan, const int64_t* local_points, isdf_fit_t* out);

/* Same with the candidate points of every domain given: n_candidates[d]
 * ascending local indices per domain, concatenated in candidates.  The
 * greedy selection then runs over those points only (what the learned
 * selector does with its top-scoring points).  Errors as isdf_fit plus
 * ISDF_E_ARG for counts outside 1..n_points or unsorted lists. */
isdf_status isdf_fit_with_candidates(isdf_plan_t plan, const int64_t* candidates,
                                     const int64_t* n_candidates, isdf_fit_t* out);

/* Selection report per domain (host arrays of n_domains, any may be NULL):
 * candidates the greedy selection ran over, residual of the last pivot,
 * largest initial Gram diagonal among the points left out (candidate modes;
 * when it is below (1 - tie_tol) times the last residual the pivots are
 * those of the full selection), and 1 where that check failed and the
 * domain was refitted with full selection. */
isdf_status isdf_fit_selection(isdf_fit_t fit, int64_t* n_candidates, double* last_residual,
                               double* final_residual, int32_t* fallback);

/* ---- learned candidate selector (not part of the paper's method) ------
 * Network 16 -> 64 -> 64 -> 1 (ReLU, ReLU, sigmoid), FP32, ISDF_MLP_NPARAM
 * parameters packed as W1[64][16], b1[64], W2[64][64], b2[64], w3[64], b3.
 * Loss: mean weighted binary cross-entropy with positive weight pw. */
#define ISDF_MLP_NPARAM 5313
typedef struct {
  int32_t epochs;
  int32_t batch;
  float lr, beta1, beta2, eps;  /* Adam */
  float pos_weight;             /* <= 0: (#negative / #positive) of the labels */
  uint64_t seed;                /* shuffling */
  void* stream;                 /* hipStream_t or NULL */
} isdf_mlp_config;

/* 16 features of every grid point of every domain (domain after domain, in
 * point order) into features_dev [n x 16] float, and labels_dev [n] = 1 for
 * the points a candidate set must keep for the pruned selection to equal the
 * fit's full selection (initial Gram diagonal >= (1 - tie_tol) times the
 * residual of the domain's last pivot), else 0 (labels_dev may be NULL).
 * *n receives the point count; capacity must be at least that.  Device
 * pointers; with features_dev NULL only *n is set. */
isdf_status isdf_fit_features(isdf_fit_t fit, float* features_dev, float* labels_dev,
                              int64_t capacity, int64_t* n);

/* Logits z (score = sigmoid(z)) of n feature rows; weights host, data device. */
isdf_status isdf_mlp_forward(const float* weights, const float* features_dev, int64_t n,
                             float* scores_dev, void* stream);

/* Mean loss and its gradient (host outputs) over n rows. */
isdf_status isdf_mlp_loss_grad(const float* weights, const float* features_dev,
                               const float* labels_dev, int64_t n, float pos_weight, float* grad,
                               float* loss, void* stream);

/* Adam training on the GPU with the library's own forward/backward kernels;
 * weights (host, ISDF_MLP_NPARAM) are read as the start point and receive
 * the result; epoch_loss (host, cfg->epochs, may be NULL) the mean loss of
 * each epoch. */
isdf_status isdf_mlp_train(const float* features_dev, const float* labels_dev, int64_t n,
                           const isdf_mlp_config* cfg, float* weights, float* epoch_loss);

/* Exchange build, once per SCF iteration (Eq. ints):
 *   K = -[X^L'((X^G D X^G') o W)X^L + X^L'((X^G D X^L') o W)X^N
 *         + X^N'((X^L D X^G') o W)X^L + X^N'((X^L D X^L') o W)X^N],
 *   e_x = tr(D K).
 * D_dev, K_dev: device pointers to N x N FP64 (D symmetric, per spin).
 * e_x: host pointer or NULL.  Synchronises the stream.
 * Unless the plan was made with eager_exchange = 1, the first call of a fit
 * captures the kernel sequence as a HIP graph and later calls with the same
 * D_dev/K_dev replay it (the contents of D_dev may change between calls).
 * Errors: ISDF_E_ARG (null D/K, NaN found in D), ISDF_E_STATE (fit not from
 * this plan), ISDF_E_HIP. */
isdf_status isdf_exchange(isdf_plan_t plan, isdf_fit_t fit, const double* D_dev, double* K_dev,
                          double* e_x);

/* The same exchange for a factored density D = C C' (the occupied orbitals of
 * the section on the exchange matrix): the pair products X^S D X^T' are
 * formed as (X^S C)(X^T C)', inner size n_occ instead of N.
 * C_dev: device pointer to N x n_occ FP64, row-major (C[mu * n_occ + i]).
 * K_dev, e_x and errors as isdf_exchange (ISDF_E_ARG also for n_occ < 1). */
isdf_status isdf_exchange_occ(isdf_plan_t plan, isdf_fit_t fit, const double* C_dev,
                              int32_t n_occ, double* K_dev, double* e_x);

/* occ-RI output: K C for D = C C' without forming K (the exchange section's
 * occupied-orbital form, K applied to the occupied orbitals):
 *   K C = -[X^L'(P_GG o W)E_L + X^L'(P_GL o W)E_N + X^N'(P_LG o W)E_L
 *           + X^N'(P_LL o W)E_N],  E_S = X^S C, P_ST = E_S E_T',
 * so every product has an n_occ-wide side (about 14 N_mu^2 n_occ flops
 * against 6 N_mu^2 n_occ + 8 N_mu^2 N for the full K); e_x = tr(C' K C) =
 * tr(D K), the same energy.
 * C_dev: device pointer to N x n_occ FP64, row-major (C[mu * n_occ + i]).
 * KC_dev: device pointer to N x n_occ FP64, row-major, written.
 * e_x, graph capture and errors as isdf_exchange (ISDF_E_ARG also for n_occ
 * outside 1..N).
 * With universal_all_points the result is the method with every universal
 * point a fitting function: the window terms as above (W over window
 * fitting functions), the universal-window cross terms through the stored
 * block W_Uw = (R_U|xi_w) (N_g x N_mu,windows), and the universal-universal
 * term by occ-RI FFT Poisson solves (as isdf_exchange_universal); launched
 * eagerly (no graph), with the memory noted there.  isdf_exchange and
 * isdf_exchange_occ return ISDF_E_UNSUPPORTED for such fits. */
isdf_status isdf_exchange_occ_ri(isdf_plan_t plan, isdf_fit_t fit, const double* C_dev,
                                 int32_t n_occ, double* KC_dev, double* e_x);

/* The occ-RI exchange of isdf_exchange_occ_ri in FP64 without any device
 * allocation, for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, result (K C, e_x = tr(C' K C)) and kernels as the FP64 form of
 * isdf_exchange_occ_ri, whatever the plan's precision; launched kernel by
 * kernel (no graph).  Its workspace (E_G, E_L, E_N, Z1, Z2: N_mu x n_occ;
 * Q_GG, Q_GL, Q_LL: N_mu x N_mu; FP64) lives in a fixed device array of
 * ISDF_NOALLOC_SCRATCH_MB MB built into the library, one per GPU, held until
 * the process ends; every call on a GPU shares it, so calls that overlap on
 * one GPU race (serialise them, e.g. one stream per GPU).  The fit itself
 * is made by isdf_fit as usual.  Synchronises the stream.
 * Errors: ISDF_E_ARG (null pointers, n_occ outside 1..N, a workspace
 * 8 (3 N_mu^2 + 5 N_mu n_occ) bytes, each part rounded up to 256 bytes,
 * above the array, non-finite energy), ISDF_E_STATE (fit not from this
 * plan), ISDF_E_UNSUPPORTED (fits made with universal_all_points),
 * ISDF_E_HIP. */
#define ISDF_NOALLOC_SCRATCH_MB 32
isdf_status isdf_exchange_occ_ri_noalloc(isdf_plan_t plan, isdf_fit_t fit, const double* C_dev,
                                         int32_t n_occ, double* KC_dev, double* e_x);

/* Universal grid with every point as a fitting function (the sinc functions
 * of the sparse grid; sections "Building the exchange matrix" and Results):
 * the exchange of the pairs the universal domain holds (both functions on
 * level 0), applied to the occupied orbitals without interpolation points
 * and without storing the Coulomb operator between grid points:
 *   (K_UU C)(mu, i) = -dV sum_R phi_mu(R) sum_j E(R, j) V[E_j E_i](R),
 *   E = Phi_U C,  V[rho] the potential of a grid density by FFT Poisson
 * solves (band without the Nyquist planes and G = 0, as for W), one per
 * occupied pair i <= j, each SCF iteration (occ-RI).  Rows of functions off
 * the universal grid are zero; e_x = tr(C' K_UU C).  Exact for these pairs
 * (no fitting error); the pairs held by atom windows are not included.
 * C_dev: device pointer to N x n_occ FP64, row-major (C[mu * n_occ + i]).
 * KC_dev: device pointer to N x n_occ FP64, row-major, written.
 * e_x: host pointer or NULL.  Eager launches; synchronises the stream.
 * Device memory: the potentials of the n_occ (n_occ + 1) / 2 pair densities
 * (N_g doubles each; 2.2 GB at a 32^3 grid and 128 orbitals) are held for
 * row tiles of pairs within the plan's universal_tile_mb budget, plus about
 * 2 GB of transform buffers, released on return.
 * Errors: ISDF_E_ARG (null pointers, n_occ outside 1..N, non-finite
 * energy), ISDF_E_STATE (fit not from this plan), ISDF_E_UNSUPPORTED (no
 * universal domain), ISDF_E_NOMEM, ISDF_E_HIP. */
isdf_status isdf_exchange_universal(isdf_plan_t plan, isdf_fit_t fit, const double* C_dev,
                                    int32_t n_occ, double* KC_dev, double* e_x);

/* Tile-shape tuning of the FP64 GEMMs (for callers that set up a plan once
 * and run it many times).  Runs one fit and one dense and one factored
 * exchange (D = I, C = the first n_occ unit vectors) on the plan; every
 * single-problem GEMM class met on the way (epilogue, role, triangle,
 * layouts, accumulation, log2 sizes) is timed with each tile shape, best of
 * `reps` launches, and the fastest is kept in the plan and written to
 * json_out (NULL: kept only).  Results do not depend on the shape; only the
 * speed does.  Load the file into later plans with isdf_options.tune_file.
 * The shapes include the large 128 x 64 / 128 x 128 tiles on
 * v_mfma_f64_4x4x4 (not for gathered-row or non-square triangle problems).
 * Errors: ISDF_E_ARG (n_occ outside 1..N, reps < 1, file not writable),
 * those of isdf_fit and isdf_exchange (ISDF_E_UNSUPPORTED for plans with
 * universal_all_points, whose fits give K C only). */
isdf_status isdf_autotune(isdf_plan_t plan, int32_t n_occ, int32_t reps, const char* json_out);

/* Stage outputs for checks, copied to host (synchronises).
 *   ISDF_FIELD_PHI    domain d: basis values, n_points x (n_L + n_N), column-major
 *   ISDF_FIELD_DIAG   domain d: Gram diagonal, n_points
 *   ISDF_FIELD_POINTS domain d: chosen local point indices (int64), count from COUNT
 *   ISDF_FIELD_COUNT  all: chosen point count per domain (int64, n_domains)
 *   ISDF_FIELD_THETA  domain d: Theta = M(P_d, xi), n_points x n, column-major
 *   ISDF_FIELD_F      domain d: fitting functions, n_points x n, column-major
 *   ISDF_FIELD_XL / ISDF_FIELD_XN  all: N_mu x N column-major
 *   ISDF_FIELD_W      all: N_mu x N_mu column-major (symmetric); FP64 values
 *                     (widened from the stored FP32 when w_storage = ISDF_W_F32)
 * `bytes` must equal the size of the field or ISDF_E_ARG is returned. */
enum {
  ISDF_FIELD_PHI = 0, ISDF_FIELD_DIAG = 1, ISDF_FIELD_POINTS = 2, ISDF_FIELD_COUNT = 3,
  ISDF_FIELD_THETA = 4, ISDF_FIELD_F = 5, ISDF_FIELD_XL = 6, ISDF_FIELD_XN = 7, ISDF_FIELD_W = 8
};
isdf_status isdf_fit_get(isdf_fit_t fit, int32_t field, int32_t d, void* host_out, size_t bytes);

/* Density screening of the fit's last isdf_exchange_occ_ri (ri_screen_tau
 * > 0): the fraction of the 64 x 64 tiles of Q_GG, Q_GL and Q_LL kept
 * (synchronises).  ISDF_E_STATE when no screened exchange has run. */
isdf_status isdf_fit_screen_stats(isdf_fit_t fit, double* kept_fraction);

/* Total fitted points (after any early stop). */
isdf_status isdf_fit_info(isdf_fit_t fit, int64_t* n_mu);

/* Per-stage device times of the last isdf_fit / isdf_exchange (ms), measured
 * with HIP events on the plan's stream:
 *   t[0] basis+diag, t[1] selection, t[2] gather X, t[3] Theta GEMM,
 *   t[4] Cholesky + triangular solves, t[5] Coulomb metric (FFT + GEMM),
 *   t[6] exchange total, t[7] exchange GEMM part. */
isdf_status isdf_stage_times(isdf_plan_t plan, double* t_ms, int32_t n);

/* Per-kernel instrumentation.  isdf_profile(plan, mask) resets the counters
 * and brackets every launch of the kernel families whose bit is set in mask
 * (bit f for family f, ISDF_K_ALL for all, 0 turns it off) with HIP events
 * on the plan's stream; each bracket costs two event records, so profile
 * only the families needed while timing.  With ISDF_K_GEMM_EXCHANGE in the
 * mask the exchange runs eagerly instead of as a replayed graph.
 * isdf_kernel_stats returns, for one family, the summed device time (ms),
 * the launch count and the algorithmic HBM bytes and flops of those launches
 * (what the method must move or compute: basis columns, factor columns and
 * residuals for the selection column kernel; 2 M N K per GEMM, N (N + 1) K
 * for a lower-triangle update).
 *   ISDF_K_SELECT_COLUMN  pivoted-Cholesky column + residual update of the
 *                         windows (batched per level, left-looking)
 *   ISDF_K_SELECT_PICK    tie-rule pivot pick of the windows
 *   ISDF_K_GEMM_SELECT    residual pair Gram and its rank updates (right-looking)
 *   ISDF_K_GEMM_METRIC    W = dV F^T V products
 *   ISDF_K_GEMM_FIT       Theta, blocked Cholesky and triangular-solve products
 *   ISDF_K_GEMM_EXCHANGE  exchange products (Eq. ints)
 *   ISDF_K_FFT            FFT passes of the Poisson solves
 *   ISDF_K_BASIS          basis values + Gram diagonal
 *   ISDF_K_SELECT_BLOCK   candidate-restricted steps of the universal grid's
 *                         selection (pick + column on the candidates, one
 *                         launch per pivot) */
enum {
  ISDF_K_SELECT_COLUMN = 0, ISDF_K_SELECT_PICK = 1, ISDF_K_GEMM_SELECT = 2,
  ISDF_K_GEMM_METRIC = 3, ISDF_K_GEMM_FIT = 4, ISDF_K_GEMM_EXCHANGE = 5, ISDF_K_FFT = 6,
  ISDF_K_BASIS = 7, ISDF_K_SELECT_BLOCK = 8, ISDF_K_NFAMILY = 9, ISDF_K_ALL = (1 << 9) - 1
};
isdf_status isdf_profile(isdf_plan_t plan, int32_t family_mask);
isdf_status isdf_kernel_stats(isdf_plan_t plan, int32_t family, double* ms, int64_t* launches,
                              double* bytes, double* flops);

/* Wait for the plan's stream; report deferred device errors. */
isdf_status isdf_sync(isdf_plan_t plan);

void isdf_fit_destroy(isdf_fit_t fit);
void isdf_plan_destroy(isdf_plan_t plan);

/* Message for the last non-OK status on this thread (never NULL). */
const char* isdf_last_error(void);

/* Library version string. */
const char* isdf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ISDF_H */
