// C ABI and host runtime of the multigrid-ISDF exchange library.
//
// isdf_fit runs, per geometry (section "Using multiple grids for exchange"):
//   1. basis values + Gram diagonal on every domain        (basis_eval)
//   2. pivoted-Cholesky points, one batch per level          (sel_*)
//   3. X rows at the points -> X^L, X^N                      (gather_x)
//   4. Theta = A_L o (A_L + 2 A_N) on MFMA                    (gemm EPI_THETA)
//   5. F = Theta M_xi^{-1}: fused small fit or blocked
//      Cholesky + two triangular solves                     (Eq. lsqr)
//   6. W by FFT Poisson solves, function pairs packed in one
//      complex transform, potentials restricted to every
//      coarser band, W = dV F^T V on MFMA                    (Eq. (xi|xi'))
// isdf_exchange runs the four-term K of Eq. ints as MFMA GEMMs with the
// Hadamard product against W fused into their epilogue, and E_x = tr(D K).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>

#include "common.h"

namespace isdf {
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace isdf

using namespace isdf;

namespace {

constexpr int NSTAGE = 8;
constexpr int RL_MIN_PIVOTS = 128;  // right-looking selection above this many pivots
constexpr int RL_BLOCK = 128;       // pivots between residual (SYRK) updates

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  isdf_status alloc(size_t b) {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = b;
    if (b == 0) return ISDF_OK;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      set_error(std::string("hipMalloc of ") + std::to_string(b) + " bytes: " + hipGetErrorString(e));
      return ISDF_E_NOMEM;
    }
    return ISDF_OK;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

template <class T>
isdf_status upload(DevBuf& b, const std::vector<T>& v) {
  isdf_status st = b.alloc(sizeof(T) * std::max<size_t>(v.size(), 1));
  if (st != ISDF_OK) return st;
  if (!v.empty()) ISDF_HIP_TRY(hipMemcpy(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return ISDF_OK;
}

}  // namespace

struct isdf_plan_s;
namespace {
hipEvent_t prof_event(isdf_plan_s* pl);
}

struct isdf_plan_s {
  HostPlan hp;
  isdf_options opts{};
  hipStream_t stream = nullptr;
  bool uploaded = false;
  // static device tables
  DevBuf d_shells, d_img, d_colshells, d_doms, d_points, d_tiles, d_funcs;
  int ntiles_basis = 0;
  std::vector<int64_t> pts_off, phi_off, func_off;
  int64_t phi_total = 0, pts_total = 0;
  LatticeArg lat{};
  double recip[9];
  hipEvent_t ev[NSTAGE + 1] = {};
  double stage_ms[NSTAGE] = {};
  int fits_alive = 0;
  // per-kernel instrumentation
  struct ProfRec {
    int fam;
    hipEvent_t a, b;
    double bytes, flops;
  };
  bool prof = false;
  std::vector<hipEvent_t> evpool;
  size_t evnext = 0;
  std::vector<ProfRec> pending;
  double kms[ISDF_K_NFAMILY] = {}, kbytes[ISDF_K_NFAMILY] = {}, kflops[ISDF_K_NFAMILY] = {};
  int64_t kn[ISDF_K_NFAMILY] = {};
};

struct isdf_fit_s {
  isdf_plan_s* plan = nullptr;
  DevBuf phi, diag0, dwork, lfac, prow, piv, tmax, tidx, state;
  std::vector<int> count;          // points per domain
  std::vector<int64_t> xoff;       // first xi of each domain
  std::vector<int64_t> lfac_off, th_off, xrow_off, piv_off;
  int64_t nmu = 0;
  DevBuf xrows, XL, XN, XG, theta, F, W, lev;
  // exchange workspace
  DevBuf EG, EL, QGG, QGL, QLL, Y1, Y2, partial, ex_out;
};

namespace {

hipEvent_t prof_event(isdf_plan_s* pl) {
  if (pl->evnext == pl->evpool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pl->evpool.push_back(e);
  }
  return pl->evpool[pl->evnext++];
}

// Brackets one launch (or a short sequence) of a kernel family with events.
struct ProfScope {
  isdf_plan_s* pl;
  int fam;
  double bytes, flops;
  hipEvent_t a = nullptr;
  ProfScope(isdf_plan_s* p, int f, double by, double fl) : pl(p), fam(f), bytes(by), flops(fl) {
    if (pl->prof) {
      a = prof_event(pl);
      if (a) (void)hipEventRecord(a, pl->stream);
    }
  }
  void finish() {
    if (!a) return;
    hipEvent_t b = prof_event(pl);
    if (b) {
      (void)hipEventRecord(b, pl->stream);
      pl->pending.push_back({fam, a, b, bytes, flops});
    }
    a = nullptr;
  }
  ~ProfScope() { finish(); }
};

// Accumulate the finished records (call after the stream has synchronised).
void prof_collect(isdf_plan_s* pl) {
  for (auto& r : pl->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      pl->kms[r.fam] += ms;
      pl->kbytes[r.fam] += r.bytes;
      pl->kflops[r.fam] += r.flops;
      pl->kn[r.fam] += 1;
    }
  }
  pl->pending.clear();
  pl->evnext = 0;
}

double gemm_bytes(const GemmProblem& p) {
  return 8.0 * ((double)p.M * p.K + (double)p.K * p.N + (double)p.M * p.N * (p.beta != 0.0 ? 2 : 1));
}
double gemm_flops(const GemmProblem& p) { return 2.0 * p.M * (double)p.N * p.K; }

isdf_status gemm_prof(isdf_plan_s* pl, int fam, int epi, const GemmProblem& p) {
  ProfScope ps(pl, fam, gemm_bytes(p), gemm_flops(p));
  return gemm_f64(pl->stream, epi, p);
}

isdf_status fft_prof(isdf_plan_s* pl, double* z, int batch, const int grid[3], int sign) {
  int passes = (grid[0] > 1) + (grid[1] > 1) + (grid[2] > 1);
  const double ng = (double)grid[0] * grid[1] * grid[2];
  ProfScope ps(pl, ISDF_K_FFT, 32.0 * ng * batch * passes, 0.0);
  return fft3d(pl->stream, z, batch, grid, sign, nullptr);
}

isdf_status upload_plan(isdf_plan_s* pl) {
  if (pl->uploaded) return ISDF_OK;
  HostPlan& hp = pl->hp;
  std::vector<ShellDev> sh(hp.n_shells);
  for (int s = 0; s < hp.n_shells; ++s) {
    double a = hp.shell_alpha[s];
    double nrm = std::pow(2.0 * a / M_PI, 0.75);
    if (hp.shell_l[s] == 1) nrm *= 2.0 * std::sqrt(a);
    sh[s] = ShellDev{a, nrm, hp.shell_l[s], hp.img_off[s], hp.img_cnt[s], 0};
  }
  std::vector<ColShell> cols;
  std::vector<DomainDev> doms;
  std::vector<int32_t> points, funcs;
  std::vector<BasisTile> tiles;
  pl->pts_off.clear();
  pl->phi_off.clear();
  pl->func_off.clear();
  int64_t phi_off = 0;
  for (size_t d = 0; d < hp.domains.size(); ++d) {
    const HostDomain& D = hp.domains[d];
    DomainDev dd{};
    dd.pts_off = (int64_t)points.size();
    dd.phi_off = phi_off;
    dd.diag_off = dd.pts_off;
    dd.pts = (int)D.points.size();
    dd.nG = (int)D.funcs.size();
    dd.nL = D.nL;
    dd.n_mu = D.n_mu;
    dd.level = D.level;
    dd.colshell_off = (int)cols.size();
    for (int c = 0; c < dd.nG;) {
      int s = hp.f_shell[D.funcs[c]];
      cols.push_back(ColShell{s, c});
      c += hp.shell_l[s] == 1 ? 3 : 1;
    }
    dd.colshell_cnt = (int)cols.size() - dd.colshell_off;
    doms.push_back(dd);
    pl->pts_off.push_back(dd.pts_off);
    pl->phi_off.push_back(phi_off);
    pl->func_off.push_back((int64_t)funcs.size());
    points.insert(points.end(), D.points.begin(), D.points.end());
    funcs.insert(funcs.end(), D.funcs.begin(), D.funcs.end());
    for (int st = 0; st < dd.pts; st += 256) tiles.push_back(BasisTile{(int)d, st});
    phi_off += (int64_t)dd.pts * dd.nG;
  }
  pl->phi_total = phi_off;
  pl->pts_total = (int64_t)points.size();
  pl->ntiles_basis = (int)tiles.size();
  isdf_status st;
  if ((st = upload(pl->d_shells, sh)) != ISDF_OK) return st;
  if ((st = upload(pl->d_img, hp.img_xyz)) != ISDF_OK) return st;
  if ((st = upload(pl->d_colshells, cols)) != ISDF_OK) return st;
  if ((st = upload(pl->d_doms, doms)) != ISDF_OK) return st;
  if ((st = upload(pl->d_points, points)) != ISDF_OK) return st;
  if ((st = upload(pl->d_tiles, tiles)) != ISDF_OK) return st;
  if ((st = upload(pl->d_funcs, funcs)) != ISDF_OK) return st;
  for (int i = 0; i < 9; ++i) pl->lat.a[i] = hp.lattice[i];
  pl->lat.ln_inv_tau = hp.ln_inv_tau;
  for (int l = 0; l < hp.n_levels; ++l)
    for (int i = 0; i < 3; ++i) pl->lat.grid[l][i] = hp.grid[l][i];
  // reciprocal vectors b_i (rows): b_i[j] = 2 pi inv[j][i]
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) pl->recip[i * 3 + j] = 2.0 * M_PI * hp.inv[j * 3 + i];
  for (int l = 0; l < hp.n_levels; ++l)
    for (int i = 0; i < 3; ++i)
      if ((st = fft_prepare(hp.grid[l][i])) != ISDF_OK) return st;
  for (int i = 0; i <= NSTAGE; ++i) ISDF_HIP_TRY(hipEventCreate(&pl->ev[i]));
  pl->uploaded = true;
  return ISDF_OK;
}

inline int64_t level_ng(const HostPlan& hp, int l) {
  return (int64_t)hp.grid[l][0] * hp.grid[l][1] * hp.grid[l][2];
}

// ---------------------------------------------------------------- selection
isdf_status run_selection(isdf_plan_s* pl, isdf_fit_s* f, const int64_t* pinned) {
  HostPlan& hp = pl->hp;
  hipStream_t s = pl->stream;
  const int nd = (int)hp.domains.size();
  std::vector<SelDomain> sd(nd);
  std::vector<int32_t> tile_dom;
  int64_t lf = 0, pr = 0, pv = 0;
  f->lfac_off.assign(nd, 0);
  f->piv_off.assign(nd, 0);
  for (int d = 0; d < nd; ++d) {
    const HostDomain& D = hp.domains[d];
    SelDomain& x = sd[d];
    x.phi_off = pl->phi_off[d];
    x.lfac_off = lf;
    x.diag_off = pl->pts_off[d];
    x.prow_off = pr;
    x.pts = (int)D.points.size();
    x.nG = (int)D.funcs.size();
    x.nL = D.nL;
    x.n_mu = D.n_mu;
    x.tile_off = (int)tile_dom.size();
    x.ntiles = (x.pts + SEL_TILE - 1) / SEL_TILE;
    x.piv_off = (int)pv;
    x.mres_off = -1;
    for (int t = 0; t < x.ntiles; ++t) tile_dom.push_back(d);
    f->lfac_off[d] = lf;
    f->piv_off[d] = pv;
    lf += (int64_t)x.pts * x.n_mu;
    pr += x.nG + x.n_mu;
    pv += x.n_mu;
  }
  isdf_status st;
  if ((st = f->piv.alloc(sizeof(int32_t) * std::max<int64_t>(pv, 1))) != ISDF_OK) return st;
  f->count.assign(nd, 0);
  if (pinned) {
    std::vector<int32_t> hp_piv(pv);
    int64_t o = 0;
    for (int d = 0; d < nd; ++d) {
      const int64_t np = (int64_t)hp.domains[d].points.size();
      std::vector<char> seen(np, 0);
      for (int k = 0; k < hp.domains[d].n_mu; ++k, ++o) {
        const int64_t v = pinned[o];
        if (v < 0 || v >= np) {
          set_error("isdf_fit_with_points: point index outside its domain");
          return ISDF_E_ARG;
        }
        if (seen[v]) {
          set_error("isdf_fit_with_points: duplicate point in a domain");
          return ISDF_E_NOT_SPD;
        }
        seen[v] = 1;
        hp_piv[o] = (int32_t)v;
      }
      f->count[d] = hp.domains[d].n_mu;
    }
    ISDF_HIP_TRY(hipMemcpy(f->piv.p, hp_piv.data(), sizeof(int32_t) * pv, hipMemcpyHostToDevice));
    return ISDF_OK;
  }
  // Large single-domain batches (the universal grid) use the right-looking
  // form: residual Gram kept in HBM, SYRK update every RL_BLOCK pivots.
  size_t free_b = 0, total_b = 0;
  ISDF_HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  std::vector<char> right(nd, 0);
  int64_t mres_max = 0;
  for (int d = 0; d < nd; ++d) {
    const int lev = hp.domains[d].level;
    int nlev = 0;
    for (int e = 0; e < nd; ++e) nlev += hp.domains[e].level == lev;
    const double P = (double)sd[d].pts;
    if (nlev == 1 && sd[d].n_mu > RL_MIN_PIVOTS && P * P * 8.0 <= 0.4 * (double)free_b) {
      right[d] = 1;
      sd[d].mres_off = 0;
      mres_max = std::max<int64_t>(mres_max, (int64_t)sd[d].pts * sd[d].pts);
    }
  }
  DevBuf mres;
  if (mres_max > 0)
    if ((st = mres.alloc(sizeof(double) * mres_max)) != ISDF_OK) return st;
  DevBuf d_sd, d_tile_dom;
  if ((st = upload(d_sd, sd)) != ISDF_OK) return st;
  if ((st = upload(d_tile_dom, tile_dom)) != ISDF_OK) return st;
  const int ntiles = (int)tile_dom.size();
  if ((st = f->lfac.alloc(sizeof(double) * std::max<int64_t>(lf, 1))) != ISDF_OK) return st;
  if ((st = f->prow.alloc(sizeof(double) * std::max<int64_t>(pr, 1))) != ISDF_OK) return st;
  if ((st = f->tmax.alloc(sizeof(double) * ntiles)) != ISDF_OK) return st;
  if ((st = f->tidx.alloc(sizeof(int32_t) * ntiles)) != ISDF_OK) return st;
  if ((st = f->state.alloc(sizeof(SelState) * nd)) != ISDF_OK) return st;
  ISDF_HIP_TRY(hipMemsetAsync(f->state.p, 0, sizeof(SelState) * nd, s));
  const double tau = hp.tie_tol, eps = hp.eps_isdf;
  // one batch per level: domains of a level are contiguous
  int d0 = 0;
  while (d0 < nd) {
    int d1 = d0;
    int kmax = 0;
    while (d1 < nd && hp.domains[d1].level == hp.domains[d0].level) {
      kmax = std::max(kmax, hp.domains[d1].n_mu);
      ++d1;
    }
    const int t0 = sd[d0].tile_off;
    const int t1 = (d1 < nd) ? sd[d1].tile_off : ntiles;
    SelDomain* D = d_sd.as<SelDomain>();
    SelState* S = f->state.as<SelState>();
    if ((st = launch_sel_init(s, D, d_tile_dom.as<int32_t>(), t0, t1 - t0, f->dwork.as<double>(),
                              f->tmax.as<double>(), f->tidx.as<int32_t>(), tau)) != ISDF_OK)
      return st;
    const bool rl = right[d0] != 0;
    const int64_t P = sd[d0].pts;
    if (rl) {
      // residual Gram = full pair Gram A_L o (A_L + 2 A_N), lower triangle
      GemmProblem g{};
      g.A = f->phi.as<double>() + pl->phi_off[d0];
      g.lda = P;
      g.B = g.A;
      g.ldb = P;
      g.transB = 1;
      g.C = mres.as<double>();
      g.ldc = P;
      g.M = (int)P;
      g.N = (int)P;
      g.K = sd[d0].nG;
      g.kL = sd[d0].nL;
      g.lower = 1;
      if ((st = gemm_prof(pl, ISDF_K_GEMM_FIT, EPI_THETA, g)) != ISDF_OK) return st;
    }
    int kb = 0;
    for (int k = 0; k <= kmax; ++k) {
      double col_bytes = 0.0, col_flops = 0.0, pick_bytes = 0.0;
      for (int d = d0; d < d1; ++d) {
        if (sd[d].n_mu <= k) continue;
        col_bytes += 8.0 * sd[d].pts * ((double)sd[d].nG + k + 3.0);
        col_flops += 2.0 * sd[d].pts * ((double)sd[d].nG + k) + 3.0 * sd[d].pts;
        pick_bytes += 12.0 * sd[d].ntiles + 16.0 * (sd[d].nG + k);
      }
      ProfScope ps_pick(pl, ISDF_K_SELECT_PICK, pick_bytes, 0.0);
      if ((st = launch_sel_select(s, D, d0, d1 - d0, k, S, f->phi.as<double>(),
                                  f->lfac.as<double>(), f->dwork.as<double>(),
                                  f->tmax.as<double>(), f->tidx.as<int32_t>(),
                                  f->prow.as<double>(), f->piv.as<int32_t>(), tau, eps)) != ISDF_OK)
        return st;
      ps_pick.finish();
      if (k == kmax) break;
      if (rl) {  // residual column + block columns instead of basis + all columns
        col_bytes = 8.0 * P * ((double)(k - kb) + 4.0);
        col_flops = 2.0 * P * (double)(k - kb);
      }
      {
        ProfScope ps_col(pl, ISDF_K_SELECT_COLUMN, col_bytes, col_flops);
        if ((st = launch_sel_column(s, D, d_tile_dom.as<int32_t>(), t0, t1 - t0, k, rl ? kb : 0, S,
                                    f->phi.as<double>(), mres.as<double>(), f->lfac.as<double>(),
                                    f->dwork.as<double>(), f->prow.as<double>(),
                                    f->tmax.as<double>(), f->tidx.as<int32_t>(), tau)) != ISDF_OK)
          return st;
      }
      if (rl && (k + 1 - kb == RL_BLOCK) && k + 1 < kmax) {
        // Mres -= L[:, kb..k] L[:, kb..k]^T on the lower triangle
        GemmProblem g{};
        g.A = f->lfac.as<double>() + sd[d0].lfac_off + (int64_t)kb * P;
        g.lda = P;
        g.B = g.A;
        g.ldb = P;
        g.transB = 1;
        g.C = mres.as<double>();
        g.ldc = P;
        g.M = (int)P;
        g.N = (int)P;
        g.K = k + 1 - kb;
        g.alpha = -1.0;
        g.beta = 1.0;
        g.lower = 1;
        if ((st = gemm_prof(pl, ISDF_K_GEMM_FIT, EPI_AXPBY, g)) != ISDF_OK) return st;
        kb = k + 1;
      }
    }
    d0 = d1;
  }
  std::vector<SelState> hs(nd);
  ISDF_HIP_TRY(hipMemcpyAsync(hs.data(), f->state.p, sizeof(SelState) * nd, hipMemcpyDeviceToHost, s));
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  for (int d = 0; d < nd; ++d) f->count[d] = hs[d].count;
  return ISDF_OK;
}

// --------------------------------------------------------- blocked fit path
isdf_status blocked_fit(isdf_plan_s* pl, const double* theta, int64_t pts, int n,
                        const int32_t* piv, double* F, int32_t* status) {
  hipStream_t s = pl->stream;
  const int nb = 64;
  const int nblk = (n + nb - 1) / nb;
  DevBuf M, Cf, inv, T, G;
  isdf_status st;
  if ((st = M.alloc(sizeof(double) * n * (int64_t)n)) != ISDF_OK) return st;
  if ((st = Cf.alloc(sizeof(double) * n * (int64_t)n)) != ISDF_OK) return st;
  if ((st = inv.alloc(sizeof(double) * nblk * nb * nb)) != ISDF_OK) return st;
  if ((st = T.alloc(sizeof(double) * pts * n)) != ISDF_OK) return st;
  if ((st = G.alloc(sizeof(double) * pts * n)) != ISDF_OK) return st;
  double* m = M.as<double>();
  double* cf = Cf.as<double>();
  double* iv = inv.as<double>();
  double* t = T.as<double>();
  double* g = G.as<double>();
  if ((st = launch_gather_square(s, theta, pts, n, piv, m)) != ISDF_OK) return st;
  if ((st = launch_fill(s, cf, (int64_t)n * n, 0.0)) != ISDF_OK) return st;
  // Cholesky, left-looking by 64-column blocks
  for (int j = 0; j < nblk; ++j) {
    const int jb = j * nb, w = std::min(nb, n - jb);
    if (jb > 0) {
      GemmProblem p{};
      p.A = cf + jb; p.lda = n;
      p.B = cf + jb; p.ldb = n; p.transB = 1;
      p.C = m + jb + (int64_t)jb * n; p.ldc = n;
      p.M = n - jb; p.N = w; p.K = jb;
      p.alpha = -1.0; p.beta = 1.0;
      if ((st = gemm_prof(pl, ISDF_K_GEMM_FIT, EPI_AXPBY, p)) != ISDF_OK) return st;
    }
    if ((st = launch_potrf_diag(s, m + jb + (int64_t)jb * n, n, cf + jb + (int64_t)jb * n, n,
                                iv + (int64_t)j * nb * nb, w, status)) != ISDF_OK)
      return st;
    if (jb + w < n) {
      GemmProblem p{};
      p.A = m + (jb + w) + (int64_t)jb * n; p.lda = n;
      p.B = iv + (int64_t)j * nb * nb; p.ldb = nb; p.transB = 1;
      p.C = cf + (jb + w) + (int64_t)jb * n; p.ldc = n;
      p.M = n - jb - w; p.N = w; p.K = w;
      p.alpha = 1.0; p.beta = 0.0;
      if ((st = gemm_prof(pl, ISDF_K_GEMM_FIT, EPI_AXPBY, p)) != ISDF_OK) return st;
    }
  }
  // G C^T = Theta
  ISDF_HIP_TRY(hipMemcpyAsync(t, theta, sizeof(double) * pts * n, hipMemcpyDeviceToDevice, s));
  for (int j = 0; j < nblk; ++j) {
    const int jb = j * nb, w = std::min(nb, n - jb);
    if (jb > 0) {
      GemmProblem p{};
      p.A = g; p.lda = pts;
      p.B = cf + jb; p.ldb = n; p.transB = 1;
      p.C = t + (int64_t)jb * pts; p.ldc = pts;
      p.M = (int)pts; p.N = w; p.K = jb;
      p.alpha = -1.0; p.beta = 1.0;
      if ((st = gemm_prof(pl, ISDF_K_GEMM_FIT, EPI_AXPBY, p)) != ISDF_OK) return st;
    }
    GemmProblem p{};
    p.A = t + (int64_t)jb * pts; p.lda = pts;
    p.B = iv + (int64_t)j * nb * nb; p.ldb = nb; p.transB = 1;
    p.C = g + (int64_t)jb * pts; p.ldc = pts;
    p.M = (int)pts; p.N = w; p.K = w;
    p.alpha = 1.0; p.beta = 0.0;
    if ((st = gemm_prof(pl, ISDF_K_GEMM_FIT, EPI_AXPBY, p)) != ISDF_OK) return st;
  }
  // F C = G
  for (int j = nblk - 1; j >= 0; --j) {
    const int jb = j * nb, w = std::min(nb, n - jb);
    if (jb + w < n) {
      GemmProblem p{};
      p.A = F + (int64_t)(jb + w) * pts; p.lda = pts;
      p.B = cf + (jb + w) + (int64_t)jb * n; p.ldb = n;
      p.C = g + (int64_t)jb * pts; p.ldc = pts;
      p.M = (int)pts; p.N = w; p.K = n - jb - w;
      p.alpha = -1.0; p.beta = 1.0;
      if ((st = gemm_prof(pl, ISDF_K_GEMM_FIT, EPI_AXPBY, p)) != ISDF_OK) return st;
    }
    GemmProblem p{};
    p.A = g + (int64_t)jb * pts; p.lda = pts;
    p.B = iv + (int64_t)j * nb * nb; p.ldb = nb;
    p.C = F + (int64_t)jb * pts; p.ldc = pts;
    p.M = (int)pts; p.N = w; p.K = w;
    p.alpha = 1.0; p.beta = 0.0;
    if ((st = gemm_prof(pl, ISDF_K_GEMM_FIT, EPI_AXPBY, p)) != ISDF_OK) return st;
  }
  // the buffers are released when this returns: wait for their users
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  return ISDF_OK;
}

// ------------------------------------------------------------- Coulomb metric
// Columns (fitting functions xi') are processed level by level in chunks.  For
// a chunk on level l' every function is transformed on its own grid, and its
// potential is formed on every grid l <= l' through that grid's band.  The
// potentials of the whole chunk stay in HBM (one slab per grid), so that
// W[rows of level l, chunk] = dV_l F_d^T V_l[P_d, chunk] is one wide grouped
// GEMM per grid.  Chunk widths follow a memory budget; FFT batches follow the
// size of the complex work buffers.
isdf_status run_coulomb(isdf_plan_s* pl, isdf_fit_s* f) {
  HostPlan& hp = pl->hp;
  hipStream_t s = pl->stream;
  const int nd = (int)hp.domains.size();
  const int64_t nmu = f->nmu;
  const int L = hp.n_levels;
  isdf_status st;
  if ((st = f->W.alloc(sizeof(double) * nmu * nmu)) != ISDF_OK) return st;
  if ((st = launch_fill(s, f->W.as<double>(), nmu * nmu, 0.0)) != ISDF_OK) return st;
  // global xi indices are contiguous per level
  std::vector<int64_t> lev_begin(L, -1), lev_end(L, -1);
  std::vector<int> col_dom(nmu), col_j(nmu);
  for (int d = 0; d < nd; ++d) {
    const int l = hp.domains[d].level;
    if (f->count[d] == 0) continue;
    if (lev_begin[l] < 0) lev_begin[l] = f->xoff[d];
    lev_end[l] = f->xoff[d] + f->count[d];
    for (int j = 0; j < f->count[d]; ++j) {
      col_dom[f->xoff[d] + j] = d;
      col_j[f->xoff[d] + j] = j;
    }
  }
  // memory budget for the potential slabs and the complex work buffers
  size_t free_b = 0, total_b = 0;
  ISDF_HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  const double v_budget = std::max(2e9, 0.45 * (double)free_b);
  const double z_budget = std::min(4e9, std::max(2.5e8, 0.05 * (double)free_b));
  struct Chunk {
    int lp;
    int64_t c0, c1;
  };
  std::vector<Chunk> chunks;
  int64_t vmax = 0;  // doubles of V needed by the widest chunk
  for (int lp = 0; lp < L; ++lp) {
    if (lev_begin[lp] < 0) continue;
    double per_col = 0.0;
    for (int l = 0; l <= lp; ++l) per_col += 8.0 * level_ng(hp, l);
    int64_t w = std::max<int64_t>(2, (int64_t)(v_budget / per_col));
    w -= w & 1;
    for (int64_t c0 = lev_begin[lp]; c0 < lev_end[lp]; c0 += w) {
      Chunk c{lp, c0, std::min(c0 + w, lev_end[lp])};
      chunks.push_back(c);
      vmax = std::max<int64_t>(vmax, (int64_t)(per_col / 8.0) * (c.c1 - c.c0));
    }
  }
  // descriptors: scatter per column, GEMM problems per (chunk, row level)
  std::vector<ScatterCol> scat(nmu);
  for (int64_t c = 0; c < nmu; ++c) {
    const int d = col_dom[c];
    const int64_t pts = (int64_t)hp.domains[d].points.size();
    scat[c].src = f->F.as<double>() + f->th_off[d] + (int64_t)col_j[c] * pts;
    scat[c].pts = pl->d_points.as<int32_t>() + pl->pts_off[d];
    scat[c].n = (int)pts;
    scat[c].slot = 0;  // set per batch below
  }
  DevBuf zf, zc, V, d_scat, d_probs;
  int64_t ngz_max = 0;
  for (auto& c : chunks) ngz_max = std::max(ngz_max, level_ng(hp, c.lp));
  int64_t fft_pairs = std::max<int64_t>(1, (int64_t)(z_budget / (16.0 * ngz_max)));
  if ((st = zf.alloc(sizeof(double) * 2 * ngz_max * fft_pairs)) != ISDF_OK) return st;
  if ((st = zc.alloc(sizeof(double) * 2 * ngz_max * fft_pairs)) != ISDF_OK) return st;
  if ((st = V.alloc(sizeof(double) * std::max<int64_t>(vmax, 1))) != ISDF_OK) return st;
  std::vector<GemmProblem> probs;
  struct GemmLaunch {
    int off, cnt, tiles;
    double bytes, flops;
  };
  std::vector<std::vector<GemmLaunch>> glaunch(chunks.size());
  for (size_t ci = 0; ci < chunks.size(); ++ci) {
    const Chunk& ch = chunks[ci];
    int64_t voff = 0;
    for (int l = 0; l <= ch.lp; ++l) {
      GemmLaunch gl{(int)probs.size(), 0, 0, 0.0, 0.0};
      const double dV = hp.volume / (double)level_ng(hp, l);
      for (int d = 0; d < nd; ++d) {
        if (hp.domains[d].level != l || f->count[d] == 0) continue;
        const HostDomain& D = hp.domains[d];
        GemmProblem p{};
        p.A = f->F.as<double>() + f->th_off[d];
        p.lda = (int64_t)D.points.size();
        p.transA = 1;
        p.B = V.as<double>() + voff;
        p.ldb = level_ng(hp, l);
        p.bidx = ((int64_t)D.points.size() == level_ng(hp, l) && D.atom < 0)
                     ? nullptr
                     : pl->d_points.as<int32_t>() + pl->pts_off[d];
        p.C = f->W.as<double>() + f->xoff[d] + ch.c0 * nmu;
        p.ldc = nmu;
        p.M = f->count[d];
        p.N = (int)(ch.c1 - ch.c0);
        p.K = (int)D.points.size();
        p.alpha = dV;
        p.beta = 0.0;
        p.tile_start = gl.tiles;
        gl.tiles += gemm_tiles(p.M, p.N);
        gl.bytes += gemm_bytes(p);
        gl.flops += gemm_flops(p);
        probs.push_back(p);
      }
      gl.cnt = (int)probs.size() - gl.off;
      glaunch[ci].push_back(gl);
      voff += level_ng(hp, l) * (ch.c1 - ch.c0);
    }
  }
  if ((st = upload(d_probs, probs)) != ISDF_OK) return st;
  // the scatter slot of a column is its position within its FFT batch
  for (auto& ch : chunks) {
    const int64_t pairs_max = std::max<int64_t>(1, (ngz_max * fft_pairs) / level_ng(hp, ch.lp));
    const int64_t bw = std::max<int64_t>(2, 2 * pairs_max);
    for (int64_t b0 = ch.c0; b0 < ch.c1; b0 += bw)
      for (int64_t c = b0; c < std::min(b0 + bw, ch.c1); ++c) scat[c].slot = (int)(c - b0);
  }
  if ((st = upload(d_scat, scat)) != ISDF_OK) return st;
  for (size_t ci = 0; ci < chunks.size(); ++ci) {
    const Chunk& ch = chunks[ci];
    const int lp = ch.lp;
    const int64_t ngp = level_ng(hp, lp);
    const int64_t pairs_max = std::max<int64_t>(1, (ngz_max * fft_pairs) / ngp);
    const int64_t bw = std::max<int64_t>(2, 2 * pairs_max);
    for (int64_t b0 = ch.c0; b0 < ch.c1; b0 += bw) {
      const int ncols = (int)std::min<int64_t>(bw, ch.c1 - b0);
      const int npairs = (ncols + 1) / 2;
      int max_n = 0;
      for (int64_t c = b0; c < b0 + ncols; ++c) max_n = std::max(max_n, scat[c].n);
      if ((st = launch_fill(s, zf.as<double>(), 2 * ngp * npairs, 0.0)) != ISDF_OK) return st;
      if ((st = launch_scatter_cols(s, d_scat.as<ScatterCol>() + b0, ncols, max_n, zf.as<double>(),
                                    ngp)) != ISDF_OK)
        return st;
      if ((st = fft_prof(pl, zf.as<double>(), npairs, hp.grid[lp], -1)) != ISDF_OK) return st;
      int64_t voff = 0;
      for (int l = 0; l <= lp; ++l) {
        const int64_t ng = level_ng(hp, l);
        if ((st = launch_poisson_restrict(s, zf.as<double>(), hp.grid[lp], zc.as<double>(),
                                          hp.grid[l], npairs, pl->recip)) != ISDF_OK)
          return st;
        if ((st = fft_prof(pl, zc.as<double>(), npairs, hp.grid[l], +1)) != ISDF_OK) return st;
        if ((st = launch_split_planar(s, zc.as<double>(), ng, ncols,
                                      V.as<double>() + voff + (b0 - ch.c0) * ng)) != ISDF_OK)
          return st;
        voff += ng * (ch.c1 - ch.c0);
      }
    }
    for (int l = 0; l <= lp; ++l) {
      const GemmLaunch& gl = glaunch[ci][l];
      if (gl.cnt == 0) continue;
      ProfScope ps(pl, ISDF_K_GEMM_FIT, gl.bytes, gl.flops);
      if ((st = gemm_f64_grouped(s, EPI_AXPBY, d_probs.as<GemmProblem>() + gl.off, gl.cnt,
                                 gl.tiles)) != ISDF_OK)
        return st;
    }
  }
  // level of each xi, then symmetrise
  std::vector<int8_t> lev(nmu);
  for (int d = 0; d < nd; ++d)
    for (int j = 0; j < f->count[d]; ++j) lev[f->xoff[d] + j] = (int8_t)hp.domains[d].level;
  if ((st = upload(f->lev, lev)) != ISDF_OK) return st;
  if ((st = launch_symmetrize_w(s, f->W.as<double>(), nmu, f->lev.as<int8_t>())) != ISDF_OK)
    return st;
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  return ISDF_OK;
}

isdf_status do_fit(isdf_plan_s* pl, const int64_t* pinned, isdf_fit_t* out) {
  if (!pl || !out) {
    set_error("isdf_fit: null argument");
    return ISDF_E_ARG;
  }
  isdf_status st;
  if ((st = upload_plan(pl)) != ISDF_OK) return st;
  HostPlan& hp = pl->hp;
  hipStream_t s = pl->stream;
  std::unique_ptr<isdf_fit_s> f(new isdf_fit_s());
  f->plan = pl;
  const int nd = (int)hp.domains.size();
  // 1. basis + diagonal
  ISDF_HIP_TRY(hipEventRecord(pl->ev[0], s));
  if ((st = f->phi.alloc(sizeof(double) * std::max<int64_t>(pl->phi_total, 1))) != ISDF_OK) return st;
  if ((st = f->diag0.alloc(sizeof(double) * pl->pts_total)) != ISDF_OK) return st;
  if ((st = f->dwork.alloc(sizeof(double) * pl->pts_total)) != ISDF_OK) return st;
  double basis_bytes = 8.0 * ((double)pl->phi_total + pl->pts_total);
  ProfScope ps_basis(pl, ISDF_K_BASIS, basis_bytes, 0.0);
  if ((st = launch_basis_eval(s, pl->lat, pl->d_shells.as<ShellDev>(), pl->d_img.as<double>(),
                              pl->d_colshells.as<ColShell>(), pl->d_doms.as<DomainDev>(),
                              pl->d_points.as<int32_t>(), pl->d_tiles.as<BasisTile>(),
                              pl->ntiles_basis, f->phi.as<double>(), f->diag0.as<double>())) != ISDF_OK)
    return st;
  ps_basis.finish();
  ISDF_HIP_TRY(hipMemcpyAsync(f->dwork.p, f->diag0.p, sizeof(double) * pl->pts_total,
                              hipMemcpyDeviceToDevice, s));
  ISDF_HIP_TRY(hipEventRecord(pl->ev[1], s));
  // 2. selection
  if ((st = run_selection(pl, f.get(), pinned)) != ISDF_OK) return st;
  ISDF_HIP_TRY(hipEventRecord(pl->ev[2], s));
  bool rank_short = false;
  f->xoff.assign(nd, 0);
  int64_t nmu = 0;
  for (int d = 0; d < nd; ++d) {
    f->xoff[d] = nmu;
    nmu += f->count[d];
    if (f->count[d] < hp.domains[d].n_mu) rank_short = true;
  }
  f->nmu = nmu;
  // 3. gather X
  const int64_t N = hp.n_basis;
  if ((st = f->XL.alloc(sizeof(double) * nmu * N)) != ISDF_OK) return st;
  if ((st = f->XN.alloc(sizeof(double) * nmu * N)) != ISDF_OK) return st;
  if ((st = f->XG.alloc(sizeof(double) * nmu * N)) != ISDF_OK) return st;
  if ((st = launch_fill(s, f->XL.as<double>(), nmu * N, 0.0)) != ISDF_OK) return st;
  if ((st = launch_fill(s, f->XN.as<double>(), nmu * N, 0.0)) != ISDF_OK) return st;
  std::vector<GatherDom> gd(nd);
  f->xrow_off.assign(nd, 0);
  f->th_off.assign(nd, 0);
  int64_t xr = 0, th = 0;
  int max_rows = 0;
  for (int d = 0; d < nd; ++d) {
    const HostDomain& D = hp.domains[d];
    GatherDom& g = gd[d];
    g.phi_off = pl->phi_off[d];
    g.xrow_off = xr;
    g.pts = (int)D.points.size();
    g.nG = (int)D.funcs.size();
    g.nL = D.nL;
    g.count = f->count[d];
    g.xoff = (int)f->xoff[d];
    g.piv_off = (int)f->piv_off[d];
    g.func_off = (int)pl->func_off[d];
    f->xrow_off[d] = xr;
    f->th_off[d] = th;
    xr += (int64_t)g.count * g.nG;
    th += (int64_t)g.count * g.pts;
    max_rows = std::max(max_rows, g.count);
  }
  DevBuf d_gd;
  if ((st = upload(d_gd, gd)) != ISDF_OK) return st;
  if ((st = f->xrows.alloc(sizeof(double) * std::max<int64_t>(xr, 1))) != ISDF_OK) return st;
  if ((st = launch_gather_x(s, d_gd.as<GatherDom>(), nd, max_rows, f->phi.as<double>(),
                            f->piv.as<int32_t>(), pl->d_funcs.as<int32_t>(), f->xrows.as<double>(),
                            f->XL.as<double>(), f->XN.as<double>(), nmu)) != ISDF_OK)
    return st;
  if ((st = launch_add(s, f->XL.as<double>(), f->XN.as<double>(), f->XG.as<double>(), nmu * N)) !=
      ISDF_OK)
    return st;
  ISDF_HIP_TRY(hipEventRecord(pl->ev[3], s));
  // 4. Theta
  if ((st = f->theta.alloc(sizeof(double) * std::max<int64_t>(th, 1))) != ISDF_OK) return st;
  if ((st = f->F.alloc(sizeof(double) * std::max<int64_t>(th, 1))) != ISDF_OK) return st;
  {
    std::vector<GemmProblem> probs;
    int tiles = 0;
    for (int d = 0; d < nd; ++d) {
      if (f->count[d] == 0) continue;
      GemmProblem p{};
      p.A = f->phi.as<double>() + pl->phi_off[d];
      p.lda = gd[d].pts;
      p.B = f->xrows.as<double>() + f->xrow_off[d];
      p.ldb = gd[d].nG;
      p.C = f->theta.as<double>() + f->th_off[d];
      p.ldc = gd[d].pts;
      p.M = gd[d].pts;
      p.N = f->count[d];
      p.K = gd[d].nG;
      p.kL = gd[d].nL;
      p.tile_start = tiles;
      tiles += gemm_tiles(p.M, p.N);
      probs.push_back(p);
    }
    DevBuf d_probs;
    if ((st = upload(d_probs, probs)) != ISDF_OK) return st;
    double by = 0.0, fl = 0.0;
    for (auto& p : probs) {
      by += gemm_bytes(p);
      fl += gemm_flops(p);
    }
    ProfScope ps(pl, ISDF_K_GEMM_FIT, by, fl);
    if ((st = gemm_f64_grouped(s, EPI_THETA, d_probs.as<GemmProblem>(), (int)probs.size(), tiles)) !=
        ISDF_OK)
      return st;
    ISDF_HIP_TRY(hipStreamSynchronize(s));
  }
  ISDF_HIP_TRY(hipEventRecord(pl->ev[4], s));
  // 5. fitting functions
  DevBuf spd;
  if ((st = spd.alloc(sizeof(int32_t))) != ISDF_OK) return st;
  ISDF_HIP_TRY(hipMemsetAsync(spd.p, 0, sizeof(int32_t), s));
  {
    std::vector<SmallFitDom> sf;
    std::vector<int32_t> tile_dom;
    int nmax = 0;
    for (int d = 0; d < nd; ++d) {
      const int n = f->count[d];
      if (n == 0 || n > 64) continue;
      SmallFitDom x{};
      x.theta_off = f->th_off[d];
      x.pts = gd[d].pts;
      x.n = n;
      x.piv_off = (int)f->piv_off[d];
      x.row_tile_off = (int)tile_dom.size();
      for (int t = 0; t < (x.pts + 255) / 256; ++t) tile_dom.push_back((int)sf.size());
      sf.push_back(x);
      nmax = std::max(nmax, n);
    }
    if (!sf.empty()) {
      DevBuf d_sf, d_td;
      if ((st = upload(d_sf, sf)) != ISDF_OK) return st;
      if ((st = upload(d_td, tile_dom)) != ISDF_OK) return st;
      if ((st = launch_small_fit(s, d_sf.as<SmallFitDom>(), d_td.as<int32_t>(), (int)tile_dom.size(),
                                 f->theta.as<double>(), f->piv.as<int32_t>(), f->F.as<double>(),
                                 spd.as<int32_t>(), nmax)) != ISDF_OK)
        return st;
      ISDF_HIP_TRY(hipStreamSynchronize(s));
    }
    for (int d = 0; d < nd; ++d) {
      const int n = f->count[d];
      if (n <= 64) continue;
      if ((st = blocked_fit(pl, f->theta.as<double>() + f->th_off[d], gd[d].pts, n,
                            f->piv.as<int32_t>() + f->piv_off[d], f->F.as<double>() + f->th_off[d],
                            spd.as<int32_t>())) != ISDF_OK)
        return st;
    }
  }
  ISDF_HIP_TRY(hipEventRecord(pl->ev[5], s));
  // 6. Coulomb metric
  if ((st = run_coulomb(pl, f.get())) != ISDF_OK) return st;
  ISDF_HIP_TRY(hipEventRecord(pl->ev[6], s));
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  prof_collect(pl);
  int32_t spd_flag = 0;
  ISDF_HIP_TRY(hipMemcpy(&spd_flag, spd.p, sizeof(int32_t), hipMemcpyDeviceToHost));
  float ms;
  const int map[6] = {0, 1, 2, 3, 4, 5};
  (void)map;
  for (int i = 0; i < 6; ++i) {
    ISDF_HIP_TRY(hipEventElapsedTime(&ms, pl->ev[i], pl->ev[i + 1]));
    pl->stage_ms[i] = ms;
  }
  pl->fits_alive++;
  *out = f.release();
  if (spd_flag) {
    set_error("isdf_fit: an interpolation metric is not positive definite");
    return ISDF_E_NOT_SPD;
  }
  if (rank_short && hp.n_mu_ratio > 0) {
    set_error("isdf_fit: a domain stopped before its requested point count");
    return ISDF_E_RANK;
  }
  return ISDF_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* isdf_last_error(void) { return g_err.c_str(); }
const char* isdf_version(void) { return "isdf-mi355x 0.1 (gfx950)"; }

isdf_status isdf_plan(const isdf_system* sys, const isdf_options* opts, isdf_plan_t* out) {
  if (!out) {
    set_error("isdf_plan: null output handle");
    return ISDF_E_ARG;
  }
  *out = nullptr;
  std::unique_ptr<isdf_plan_s> pl(new isdf_plan_s());
  isdf_status st = build_host_plan(sys, pl->hp);
  if (st != ISDF_OK) return st;
  if (opts) pl->opts = *opts;
  if (pl->opts.precision != ISDF_FP64) {
    set_error("isdf_plan: only ISDF_FP64 is available in this build");
    return ISDF_E_UNSUPPORTED;
  }
  if (pl->opts.selector != ISDF_SEL_FULL) {
    set_error("isdf_plan: only full selection is available in this build");
    return ISDF_E_UNSUPPORTED;
  }
  pl->stream = static_cast<hipStream_t>(pl->opts.stream);
  *out = pl.release();
  return ISDF_OK;
}

isdf_status isdf_plan_info(isdf_plan_t plan, int64_t* n_basis, int64_t* n_mu, int32_t* n_domains) {
  if (!plan) {
    set_error("isdf_plan_info: null plan");
    return ISDF_E_ARG;
  }
  if (n_basis) *n_basis = plan->hp.n_basis;
  if (n_mu) *n_mu = plan->hp.n_mu_total;
  if (n_domains) *n_domains = (int32_t)plan->hp.domains.size();
  return ISDF_OK;
}

isdf_status isdf_plan_domain(isdf_plan_t plan, int32_t d, int32_t* level, int32_t* atom,
                             int64_t* n_points, int32_t* n_L, int32_t* n_N, int32_t* n_mu) {
  if (!plan || d < 0 || d >= (int32_t)plan->hp.domains.size()) {
    set_error("isdf_plan_domain: bad plan or domain index");
    return ISDF_E_ARG;
  }
  const HostDomain& D = plan->hp.domains[d];
  if (level) *level = D.level;
  if (atom) *atom = D.atom;
  if (n_points) *n_points = (int64_t)D.points.size();
  if (n_L) *n_L = D.nL;
  if (n_N) *n_N = D.nN;
  if (n_mu) *n_mu = D.n_mu;
  return ISDF_OK;
}

isdf_status isdf_plan_domain_points(isdf_plan_t plan, int32_t d, int64_t* points) {
  if (!plan || !points || d < 0 || d >= (int32_t)plan->hp.domains.size()) {
    set_error("isdf_plan_domain_points: bad argument");
    return ISDF_E_ARG;
  }
  const HostDomain& D = plan->hp.domains[d];
  for (size_t i = 0; i < D.points.size(); ++i) points[i] = D.points[i];
  return ISDF_OK;
}

isdf_status isdf_plan_domain_functions(isdf_plan_t plan, int32_t d, int32_t* functions) {
  if (!plan || !functions || d < 0 || d >= (int32_t)plan->hp.domains.size()) {
    set_error("isdf_plan_domain_functions: bad argument");
    return ISDF_E_ARG;
  }
  const HostDomain& D = plan->hp.domains[d];
  for (size_t i = 0; i < D.funcs.size(); ++i) functions[i] = D.funcs[i];
  return ISDF_OK;
}

isdf_status isdf_fit(isdf_plan_t plan, isdf_fit_t* out) {
  if (out) *out = nullptr;
  return do_fit(plan, nullptr, out);
}

isdf_status isdf_fit_with_points(isdf_plan_t plan, const int64_t* local_points, isdf_fit_t* out) {
  if (out) *out = nullptr;
  if (!local_points) {
    set_error("isdf_fit_with_points: null points");
    return ISDF_E_ARG;
  }
  return do_fit(plan, local_points, out);
}

isdf_status isdf_fit_info(isdf_fit_t fit, int64_t* n_mu) {
  if (!fit) {
    set_error("isdf_fit_info: null fit");
    return ISDF_E_ARG;
  }
  if (n_mu) *n_mu = fit->nmu;
  return ISDF_OK;
}

isdf_status isdf_fit_get(isdf_fit_t fit, int32_t field, int32_t d, void* host_out, size_t bytes) {
  if (!fit || !host_out) {
    set_error("isdf_fit_get: null argument");
    return ISDF_E_ARG;
  }
  isdf_plan_s* pl = fit->plan;
  const HostPlan& hp = pl->hp;
  const int nd = (int)hp.domains.size();
  const bool per_domain = field == ISDF_FIELD_PHI || field == ISDF_FIELD_DIAG ||
                          field == ISDF_FIELD_POINTS || field == ISDF_FIELD_THETA ||
                          field == ISDF_FIELD_F;
  if (per_domain && (d < 0 || d >= nd)) {
    set_error("isdf_fit_get: domain index out of range");
    return ISDF_E_ARG;
  }
  const void* src = nullptr;
  size_t need = 0;
  std::vector<int64_t> tmp64;
  std::vector<int32_t> tmp32;
  switch (field) {
    case ISDF_FIELD_PHI:
      src = fit->phi.as<double>() + pl->phi_off[d];
      need = sizeof(double) * hp.domains[d].points.size() * hp.domains[d].funcs.size();
      break;
    case ISDF_FIELD_DIAG:
      src = fit->diag0.as<double>() + pl->pts_off[d];
      need = sizeof(double) * hp.domains[d].points.size();
      break;
    case ISDF_FIELD_THETA:
      src = fit->theta.as<double>() + fit->th_off[d];
      need = sizeof(double) * hp.domains[d].points.size() * fit->count[d];
      break;
    case ISDF_FIELD_F:
      src = fit->F.as<double>() + fit->th_off[d];
      need = sizeof(double) * hp.domains[d].points.size() * fit->count[d];
      break;
    case ISDF_FIELD_XL:
      src = fit->XL.p;
      need = sizeof(double) * fit->nmu * hp.n_basis;
      break;
    case ISDF_FIELD_XN:
      src = fit->XN.p;
      need = sizeof(double) * fit->nmu * hp.n_basis;
      break;
    case ISDF_FIELD_W:
      src = fit->W.p;
      need = sizeof(double) * fit->nmu * fit->nmu;
      break;
    case ISDF_FIELD_COUNT: {
      need = sizeof(int64_t) * nd;
      if (bytes != need) break;
      int64_t* o = static_cast<int64_t*>(host_out);
      for (int i = 0; i < nd; ++i) o[i] = fit->count[i];
      return ISDF_OK;
    }
    case ISDF_FIELD_POINTS: {
      need = sizeof(int64_t) * fit->count[d];
      if (bytes != need) break;
      tmp32.resize(std::max(fit->count[d], 1));
      if (fit->count[d] > 0)
        ISDF_HIP_TRY(hipMemcpy(tmp32.data(), fit->piv.as<int32_t>() + fit->piv_off[d],
                               sizeof(int32_t) * fit->count[d], hipMemcpyDeviceToHost));
      int64_t* o = static_cast<int64_t*>(host_out);
      for (int i = 0; i < fit->count[d]; ++i) o[i] = tmp32[i];
      return ISDF_OK;
    }
    default:
      set_error("isdf_fit_get: unknown field");
      return ISDF_E_ARG;
  }
  if (bytes != need) {
    set_error("isdf_fit_get: byte count does not match the field (" + std::to_string(need) + ")");
    return ISDF_E_ARG;
  }
  if (need == 0) return ISDF_OK;
  ISDF_HIP_TRY(hipStreamSynchronize(pl->stream));
  ISDF_HIP_TRY(hipMemcpy(host_out, src, need, hipMemcpyDeviceToHost));
  return ISDF_OK;
}

isdf_status isdf_exchange(isdf_plan_t plan, isdf_fit_t fit, const double* D, double* K,
                          double* e_x) {
  if (!plan || !fit || !D || !K) {
    set_error("isdf_exchange: null argument");
    return ISDF_E_ARG;
  }
  if (fit->plan != plan) {
    set_error("isdf_exchange: fit belongs to another plan");
    return ISDF_E_STATE;
  }
  hipStream_t s = plan->stream;
  const int64_t nmu = fit->nmu, N = plan->hp.n_basis;
  isdf_status st;
  if (!fit->EG.p) {
    if ((st = fit->EG.alloc(sizeof(double) * nmu * N)) != ISDF_OK) return st;
    if ((st = fit->EL.alloc(sizeof(double) * nmu * N)) != ISDF_OK) return st;
    if ((st = fit->Y1.alloc(sizeof(double) * nmu * N)) != ISDF_OK) return st;
    if ((st = fit->Y2.alloc(sizeof(double) * nmu * N)) != ISDF_OK) return st;
    if ((st = fit->QGG.alloc(sizeof(double) * nmu * nmu)) != ISDF_OK) return st;
    if ((st = fit->QGL.alloc(sizeof(double) * nmu * nmu)) != ISDF_OK) return st;
    if ((st = fit->QLL.alloc(sizeof(double) * nmu * nmu)) != ISDF_OK) return st;
    if ((st = fit->partial.alloc(sizeof(double) * 1024)) != ISDF_OK) return st;
    if ((st = fit->ex_out.alloc(sizeof(double))) != ISDF_OK) return st;
  }
  ISDF_HIP_TRY(hipEventRecord(plan->ev[0], s));
  const double* XL = fit->XL.as<double>();
  const double* XN = fit->XN.as<double>();
  const double* XG = fit->XG.as<double>();
  const double* W = fit->W.as<double>();
  double* EG = fit->EG.as<double>();
  double* EL = fit->EL.as<double>();
  double* Y1 = fit->Y1.as<double>();
  double* Y2 = fit->Y2.as<double>();
  double* QGG = fit->QGG.as<double>();
  double* QGL = fit->QGL.as<double>();
  double* QLL = fit->QLL.as<double>();
  auto gemm = [&](int epi, const double* A, int64_t lda, int tA, const double* B, int64_t ldb,
                  int tB, double* C, int64_t ldc, int M, int Nn, int Kk, double alpha, double beta,
                  const double* E) {
    GemmProblem p{};
    p.A = A; p.lda = lda; p.transA = tA;
    p.B = B; p.ldb = ldb; p.transB = tB;
    p.C = C; p.ldc = ldc;
    p.E = E; p.lde = nmu;
    p.M = M; p.N = Nn; p.K = Kk;
    p.alpha = alpha; p.beta = beta;
    return gemm_prof(plan, ISDF_K_GEMM_EXCHANGE, epi, p);
  };
  const int m = (int)nmu, n = (int)N;
  // E_G = X^G D, E_L = X^L D
  if ((st = gemm(EPI_AXPBY, XG, nmu, 0, D, N, 0, EG, nmu, m, n, n, 1.0, 0.0, nullptr)) != ISDF_OK) return st;
  if ((st = gemm(EPI_AXPBY, XL, nmu, 0, D, N, 0, EL, nmu, m, n, n, 1.0, 0.0, nullptr)) != ISDF_OK) return st;
  // Q = (E X^T) o W
  if ((st = gemm(EPI_HADAMARD, EG, nmu, 0, XG, nmu, 1, QGG, nmu, m, m, n, 1.0, 0.0, W)) != ISDF_OK) return st;
  if ((st = gemm(EPI_HADAMARD, EG, nmu, 0, XL, nmu, 1, QGL, nmu, m, m, n, 1.0, 0.0, W)) != ISDF_OK) return st;
  if ((st = gemm(EPI_HADAMARD, EL, nmu, 0, XL, nmu, 1, QLL, nmu, m, m, n, 1.0, 0.0, W)) != ISDF_OK) return st;
  // Y1 = Q_GG X^L + Q_GL X^N ; Y2 = Q_GL^T X^L + Q_LL X^N
  if ((st = gemm(EPI_AXPBY, QGG, nmu, 0, XL, nmu, 0, Y1, nmu, m, n, m, 1.0, 0.0, nullptr)) != ISDF_OK) return st;
  if ((st = gemm(EPI_AXPBY, QGL, nmu, 0, XN, nmu, 0, Y1, nmu, m, n, m, 1.0, 1.0, nullptr)) != ISDF_OK) return st;
  if ((st = gemm(EPI_AXPBY, QGL, nmu, 1, XL, nmu, 0, Y2, nmu, m, n, m, 1.0, 0.0, nullptr)) != ISDF_OK) return st;
  if ((st = gemm(EPI_AXPBY, QLL, nmu, 0, XN, nmu, 0, Y2, nmu, m, n, m, 1.0, 1.0, nullptr)) != ISDF_OK) return st;
  // K = -(X^L^T Y1 + X^N^T Y2)
  if ((st = gemm(EPI_AXPBY, XL, nmu, 1, Y1, nmu, 0, K, N, n, n, m, -1.0, 0.0, nullptr)) != ISDF_OK) return st;
  if ((st = gemm(EPI_AXPBY, XN, nmu, 1, Y2, nmu, 0, K, N, n, n, m, -1.0, 1.0, nullptr)) != ISDF_OK) return st;
  ISDF_HIP_TRY(hipEventRecord(plan->ev[1], s));
  if ((st = launch_trace_dot(s, D, K, N * N, fit->partial.as<double>(), 1024,
                             fit->ex_out.as<double>())) != ISDF_OK)
    return st;
  ISDF_HIP_TRY(hipEventRecord(plan->ev[2], s));
  double ex = 0.0;
  ISDF_HIP_TRY(hipMemcpyAsync(&ex, fit->ex_out.p, sizeof(double), hipMemcpyDeviceToHost, s));
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  prof_collect(plan);
  float ms;
  ISDF_HIP_TRY(hipEventElapsedTime(&ms, plan->ev[0], plan->ev[2]));
  plan->stage_ms[6] = ms;
  ISDF_HIP_TRY(hipEventElapsedTime(&ms, plan->ev[0], plan->ev[1]));
  plan->stage_ms[7] = ms;
  if (e_x) *e_x = ex;
  if (!std::isfinite(ex)) {
    set_error("isdf_exchange: non-finite exchange energy (NaN or Inf in D?)");
    return ISDF_E_ARG;
  }
  return ISDF_OK;
}

isdf_status isdf_stage_times(isdf_plan_t plan, double* t_ms, int32_t n) {
  if (!plan || !t_ms) {
    set_error("isdf_stage_times: null argument");
    return ISDF_E_ARG;
  }
  for (int i = 0; i < n && i < NSTAGE; ++i) t_ms[i] = plan->stage_ms[i];
  return ISDF_OK;
}

isdf_status isdf_profile(isdf_plan_t plan, int32_t enable) {
  if (!plan) {
    set_error("isdf_profile: null plan");
    return ISDF_E_ARG;
  }
  ISDF_HIP_TRY(hipStreamSynchronize(plan->stream));
  prof_collect(plan);
  plan->prof = enable != 0;
  for (int i = 0; i < ISDF_K_NFAMILY; ++i) {
    plan->kms[i] = plan->kbytes[i] = plan->kflops[i] = 0.0;
    plan->kn[i] = 0;
  }
  return ISDF_OK;
}

isdf_status isdf_kernel_stats(isdf_plan_t plan, int32_t family, double* ms, int64_t* launches,
                              double* bytes, double* flops) {
  if (!plan || family < 0 || family >= ISDF_K_NFAMILY) {
    set_error("isdf_kernel_stats: bad plan or family");
    return ISDF_E_ARG;
  }
  if (ms) *ms = plan->kms[family];
  if (launches) *launches = plan->kn[family];
  if (bytes) *bytes = plan->kbytes[family];
  if (flops) *flops = plan->kflops[family];
  return ISDF_OK;
}

isdf_status isdf_sync(isdf_plan_t plan) {
  if (!plan) {
    set_error("isdf_sync: null plan");
    return ISDF_E_ARG;
  }
  ISDF_HIP_TRY(hipStreamSynchronize(plan->stream));
  ISDF_HIP_TRY(hipGetLastError());
  return ISDF_OK;
}

void isdf_fit_destroy(isdf_fit_t fit) {
  if (!fit) return;
  if (fit->plan) {
    (void)hipStreamSynchronize(fit->plan->stream);
    fit->plan->fits_alive--;
  }
  delete fit;
}

void isdf_plan_destroy(isdf_plan_t plan) {
  if (!plan) return;
  (void)hipStreamSynchronize(plan->stream);
  for (int i = 0; i <= NSTAGE; ++i)
    if (plan->ev[i]) (void)hipEventDestroy(plan->ev[i]);
  for (auto e : plan->evpool) (void)hipEventDestroy(e);
  delete plan;
}

}  // extern "C"
