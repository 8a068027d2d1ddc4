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
#include <array>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <chrono>
#include <climits>
#include <map>
#include <set>
#include <sstream>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>


#include "common.h"

namespace isdf {
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace isdf

using namespace isdf;

namespace {

constexpr int NSTAGE = 8;
constexpr int RL_MIN_PIVOTS = 128;  // blocked selection of a lone domain above this many pivots
constexpr int CRB_BLOCK = 512;      // most pivots per block
constexpr int CRB_CANDIDATES = 2048;  // candidates per block to start with
constexpr int CRB_CHUNK = 16;          // greedy-step launches between state checks
constexpr int KSPLIT = 8;              // k ranges of the mixed exchange's final product
constexpr int KSPLIT_RI = 16;          // k ranges of the mixed occ-RI final product
// Columns of the 2 N_mu-long contraction per launch of the mixed occ-RI Z
// products.  A chunk of the second operand (n_occ rows, S planes) then stays
// in the last-level cache while every row tile streams past it; measured on
// 12928 x 768 x 155136 split-BF16 products: 24% of the BF16 issue rate in one
// launch, 32% in chunks of 8192 (29.9% at 32768).
constexpr int RI_Z_KCHUNK = 8192;

// Device memory of one plan.  A block that a buffer gives back is kept and
// handed to a later buffer of the same plan, with no hipFree/hipMalloc (both
// of which stall the host, and freeing multi-GB blocks costs the driver
// hundreds of milliseconds): every kernel and copy of a plan is enqueued on
// the plan's stream, so the stream orders the old uses of a block before the
// new ones.  For the same reason host data reaches the device through a
// pinned staging ring as copies on that stream, never as a synchronous copy
// that could overtake kernels still reading a reused block.
//
// With a caller-owned workspace (isdf_options.workspace) every block comes
// from that buffer instead (first fit over its free ranges, neighbours
// merged on return) and the plan never calls hipMalloc for its buffers.
// `held` counts the device bytes the context holds (blocks in use plus its
// cache) and `peak` their largest value: isdf_plan_workspace_bytes.
struct MemCtx {
  static constexpr size_t STAGE_BYTES = 64u << 20;
  hipStream_t stream = nullptr;
  std::multimap<size_t, void*> free_blocks;
  size_t cached = 0;
  size_t held = 0, peak = 0;
  char* stage = nullptr;
  size_t stage_off = 0;
  char* arena = nullptr;               // caller's workspace, or null
  size_t arena_bytes = 0;
  std::map<size_t, size_t> arena_free;  // offset -> length of each free range

  ~MemCtx() {
    trim();
    if (stage) (void)hipHostFree(stage);
  }
  static size_t round(size_t b) {
    const size_t g = b >= (1u << 20) ? (2u << 20) : 512;
    return (b + g - 1) / g * g;
  }
  void set_arena(void* p, size_t bytes) {
    arena = static_cast<char*>(p);
    arena_bytes = bytes;
    arena_free.clear();
    if (bytes) arena_free[0] = bytes;
  }
  size_t arena_available() const {
    size_t s = 0;
    for (auto& kv : arena_free) s += kv.second;
    return s;
  }
  void* arena_take(size_t r) {
    for (auto it = arena_free.begin(); it != arena_free.end(); ++it) {
      const size_t off = (it->first + 255) / 256 * 256, end = it->first + it->second;
      if (off + r > end) continue;
      const size_t start = it->first;
      arena_free.erase(it);
      if (off > start) arena_free[start] = off - start;
      if (off + r < end) arena_free[off + r] = end - off - r;
      return arena + off;
    }
    return nullptr;
  }
  void arena_give(void* p, size_t r) {
    size_t off = static_cast<char*>(p) - arena, len = r;
    auto next = arena_free.lower_bound(off);
    if (next != arena_free.end() && next->first == off + len) {
      len += next->second;
      next = arena_free.erase(next);
    }
    if (next != arena_free.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        off = prev->first;
        len += prev->second;
        arena_free.erase(prev);
      }
    }
    arena_free[off] = len;
  }
  // new device blocks so far: count, bytes and host time in the allocator
  int64_t n_new = 0;
  double new_bytes = 0.0, new_ms = 0.0;
  void* device_new(size_t r) {
    void* p = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    if (arena) {
      p = arena_take(r);
    } else if (hipMalloc(&p, r) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    new_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (p) {
      held += r;
      peak = std::max(peak, held);
      ++n_new;
      new_bytes += (double)r;
    }
    return p;
  }
  void trim() {
    for (auto& kv : free_blocks) {
      if (arena) arena_give(kv.second, kv.first);
      else (void)hipFree(kv.second);
      held -= kv.first;
    }
    free_blocks.clear();
    cached = 0;
  }
  // Device bytes a new buffer could still take (cached blocks included).
  isdf_status available(double* bytes) {
    if (arena) {
      *bytes = (double)arena_available() + (double)cached;
      return ISDF_OK;
    }
    size_t free_b = 0, total_b = 0;
    ISDF_HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    *bytes = (double)free_b + (double)cached;
    return ISDF_OK;
  }
  // Release one cached block.
  void drop(std::multimap<size_t, void*>::iterator it) {
    if (arena) arena_give(it->second, it->first);
    else (void)hipFree(it->second);
    held -= it->first;
    cached -= it->first;
    free_blocks.erase(it);
  }
  // Release the largest cached block (false when the cache is empty).
  bool drop_largest() {
    if (free_blocks.empty()) return false;
    drop(std::prev(free_blocks.end()));
    return true;
  }
  // A cached block of at least `b` bytes (at most 1/8 larger for big ones),
  // else a new one.  When the device is full, the smallest cached block
  // larger than the request is released first (the blocks of other sizes
  // keep serving the buffers they were made for), then the largest ones
  // until the allocation succeeds.
  void* get(size_t b, size_t* cap) {
    const size_t r = round(b);
    auto it = free_blocks.lower_bound(r);
    if (it != free_blocks.end() && it->first <= r + std::max<size_t>(r / 8, 4096)) {
      void* p = it->second;
      *cap = it->first;
      cached -= it->first;
      free_blocks.erase(it);
      return p;
    }
    void* p = device_new(r);
    if (!p && it != free_blocks.end()) {
      drop(it);
      p = device_new(r);
    }
    while (!p && drop_largest()) p = device_new(r);
    if (!p) return nullptr;
    *cap = r;
    return p;
  }
  void put(void* p, size_t cap) {
    free_blocks.emplace(cap, p);
    cached += cap;
  }
  // Host -> device copy ordered on the plan's stream.
  isdf_status copy_in(void* dst, const void* src, size_t n) {
    if (n == 0) return ISDF_OK;
    if (!stage && hipHostMalloc((void**)&stage, STAGE_BYTES) != hipSuccess) {
      (void)hipGetLastError();
      stage = nullptr;
    }
    if (!stage || n > STAGE_BYTES) {
      ISDF_HIP_TRY(hipStreamSynchronize(stream));
      ISDF_HIP_TRY(hipMemcpy(dst, src, n, hipMemcpyHostToDevice));
      return ISDF_OK;
    }
    if (stage_off + n > STAGE_BYTES) {  // ring full: the earlier copies must have run
      ISDF_HIP_TRY(hipStreamSynchronize(stream));
      stage_off = 0;
    }
    std::memcpy(stage + stage_off, src, n);
    ISDF_HIP_TRY(hipMemcpyAsync(dst, stage + stage_off, n, hipMemcpyHostToDevice, stream));
    stage_off += (n + 255) / 256 * 256;
    return ISDF_OK;
  }
};

// The memory context of the plan whose API call is running on this thread
// (empty outside plan calls: buffers then use hipMalloc/hipFree directly).
thread_local std::shared_ptr<MemCtx> t_mem;

struct MemScope {
  std::shared_ptr<MemCtx> prev;
  explicit MemScope(const std::shared_ptr<MemCtx>& m) : prev(t_mem) { t_mem = m; }
  ~MemScope() { t_mem = prev; }
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0, cap = 0;
  std::shared_ptr<MemCtx> mem;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      if (mem)
        mem->put(p, cap);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    bytes = cap = 0;
    mem.reset();
  }
  isdf_status alloc(size_t b) {
    if (p && mem && mem == t_mem && b <= cap && MemCtx::round(b) + (cap >> 3) >= cap) {
      bytes = b;  // the block held already fits
      return ISDF_OK;
    }
    release();
    bytes = b;
    if (b == 0) return ISDF_OK;
    if (t_mem) {
      p = t_mem->get(b, &cap);
      if (p) mem = t_mem;
    } else if (hipMalloc(&p, b) == hipSuccess) {
      cap = b;
    } else {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (!p) {
      bytes = 0;
      set_error("device allocation of " + std::to_string(b) + " bytes failed");
      return ISDF_E_NOMEM;
    }
    return ISDF_OK;
  }
  // Like alloc, but any block held already that is large enough is kept
  // (work buffers reused across domain groups of varying size).
  isdf_status reserve(size_t b) {
    if (p && mem && mem == t_mem && b <= cap) {
      bytes = b;
      return ISDF_OK;
    }
    return alloc(b);
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// Host -> device copy: stream-ordered through the plan's staging ring inside
// plan calls, synchronous otherwise.
isdf_status copy_in(void* dst, const void* src, size_t n) {
  if (t_mem) return t_mem->copy_in(dst, src, n);
  if (n) ISDF_HIP_TRY(hipMemcpy(dst, src, n, hipMemcpyHostToDevice));
  return ISDF_OK;
}

template <class T>
isdf_status upload(DevBuf& b, const std::vector<T>& v) {
  isdf_status st = b.alloc(sizeof(T) * std::max<size_t>(v.size(), 1));
  if (st != ISDF_OK) return st;
  return copy_in(b.p, v.data(), sizeof(T) * v.size());
}

// BF16 split planes of one logical operand (k-contiguous rows).
struct Planes {
  DevBuf buf;
  int64_t ld = 0, plane = 0;
  int rows = 0, cols = 0;
  const __bf16* p() const { return static_cast<const __bf16*>(buf.p); }
};

isdf_status make_planes(hipStream_t s, int splits, const double* src, int64_t so, int64_t sk,
                        const int32_t* kidx, int rows, int cols, Planes& out, double scale = 1.0) {
  out.rows = rows;
  out.cols = cols;
  out.ld = (cols + 7) / 8 * 8;
  out.plane = (int64_t)rows * out.ld;
  const size_t need = sizeof(__bf16) * (size_t)splits * std::max<int64_t>(out.plane, 8);
  isdf_status st;
  if (out.buf.bytes != need)
    if ((st = out.buf.alloc(need)) != ISDF_OK) return st;
  return launch_split_bf16(s, src, so, sk, kidx, rows, cols, splits, static_cast<__bf16*>(out.buf.p),
                           out.ld, out.plane, scale);
}

// Size the planes of a rows x cols operand without filling them.
isdf_status size_planes(int splits, int rows, int cols, Planes& out) {
  const int64_t ld = (cols + 7) / 8 * 8;
  const size_t need = sizeof(__bf16) * (size_t)splits * std::max<int64_t>((int64_t)rows * ld, 8);
  if (out.buf.bytes == need) return ISDF_OK;
  return out.buf.alloc(need);
}

MixedProblem mixed_problem(const Planes& A, const Planes& B, double* C, int64_t ldc, int M, int N,
                           int K, double alpha, double beta, const double* E, int64_t lde) {
  MixedProblem p{};
  p.A = A.p();
  p.B = B.p();
  p.plane_a = A.plane;
  p.plane_b = B.plane;
  p.lda = A.ld;
  p.ldb = B.ld;
  p.C = C;
  p.ldc = ldc;
  p.E = E;
  p.lde = lde;
  p.M = M;
  p.N = N;
  p.K = K;
  p.alpha = alpha;
  p.beta = beta;
  return p;
}

}  // namespace

struct isdf_plan_s;
namespace {
hipEvent_t prof_event(isdf_plan_s* pl);
}

struct isdf_plan_s {
  HostPlan hp;
  std::shared_ptr<MemCtx> mem;  // device block cache + upload staging
  isdf_options opts{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private non-blocking stream for graph capture
  bool uploaded = false;
  // static device tables
  DevBuf d_shells, d_img, d_colshells, d_doms, d_points, d_tiles, d_funcs, d_mlp_w;
  std::vector<float> mlp_w;
  int ntiles_basis = 0;
  std::vector<int64_t> pts_off, phi_off, func_off;
  std::vector<int> tile_off;  // first basis tile of each domain (n_domains + 1 entries)
  int64_t phi_total = 0, pts_total = 0;
  // per domain: cyclic box of its points on its grid (x0, y0, z0, ex, ey,
  // ez) and the offset of its box -> point map in d_boxmap (-1: all points)
  std::vector<std::array<int32_t, 7>> box;
  DevBuf d_boxmap;
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
  int prof = 0;  // family mask of the bracketed launches
  std::vector<hipEvent_t> evpool;
  size_t evnext = 0;
  std::vector<ProfRec> pending;
  double kms[ISDF_K_NFAMILY] = {}, kbytes[ISDF_K_NFAMILY] = {}, kflops[ISDF_K_NFAMILY] = {};
  int64_t kn[ISDF_K_NFAMILY] = {};
  // GEMM tile shapes per problem class: read from the tune file, or
  // measured while `tuning` (isdf_autotune)
  std::map<std::string, int> tune;
  std::map<std::string, std::vector<float>> tune_us;
  bool tuning = false;
  int tune_reps = 3;
  // universal-grid selection: pinned copies of the block state after the
  // last two chunks of step launches, and the events that mark them
  SelState* crb_host = nullptr;
  hipEvent_t crb_ev[2] = {};
  // device bytes each memory-sized rule assumed available the first time it
  // ran (see plan_available)
  std::map<int, double> avail_memo;
};

struct isdf_fit_s {
  isdf_plan_s* plan = nullptr;
  DevBuf phi, diag0, dwork, aux, piv, cflag;
  std::vector<int> count;          // points per domain
  std::vector<int> ncand;          // candidates the selection ran over
  std::vector<double> dlast;       // residual of the last pivot
  std::vector<double> dfinal;      // largest final residual over the domain (candidate modes)
  std::vector<int> fallback;       // 1: the learned candidates failed the residual check
  std::vector<int> mode;           // selection mode per domain
  std::vector<int64_t> xoff;       // first xi of each domain
  std::vector<int64_t> th_off, xrow_off, piv_off;
  int64_t nmu = 0;
  DevBuf xrows, XL, XN, XG, theta, F, W, lev;
  bool phi_streamed = false;  // basis values evaluated per domain group and not kept
  int groups = 1;
  // w_storage = ISDF_W_F32: W held as FP32 after the fit (W then released)
  DevBuf W32;
  bool w32 = false;
  const double* w64() const { return w32 ? nullptr : W.as<double>(); }
  const float* wf32() const { return w32 ? W32.as<float>() : nullptr; }
  // exchange workspace
  DevBuf EG, EL, QGG, QGL, QLL, Y1, Y2, partial, ex_out;
  // mixed precision: fit-time operand planes and per-exchange planes.
  // xln: row a = [X^L(:, a); X^N(:, a)] (k over 2 N_mu); Q1 = [Q_GG Q_GL] and
  // Q2 = [Q_GL^T Q_LL] as A operands (rows mu, k over 2 N_mu); Y12: row a =
  // [Y1(:, a); Y2(:, a)].  K = -(xln) (Y12)^T runs as KSPLIT partial products.
  Planes xg_row, xl_row, xln;
  Planes Dp, EGp, ELp, Q1, Q2, Y12;
  DevBuf Kpart, d_yprobs, d_kprobs, d_qprobs;
  int ytiles = 0, ktiles = 0, kparts = 0, qprobs_nocc = -1;
  bool ydense = false;  // Y12, Kpart and their problem tables built
  // density screening of the occ-RI exchange: tile maxima of |W| (once per
  // fit), of |E_G| and |E_L|, the tile bounds and masks of Q_GG, Q_GL, Q_LL
  DevBuf s_wt, s_ng, s_nl, s_bgg, s_bgl, s_bll, s_mgg, s_mgl, s_mll;
  int s_nt = 0, s_nocc = -1;
  bool s_ran = false;
  // rows of Q held at once (Q1/Q2 planes or the FP64 Q buffers): N_mu, or a
  // row block of the occ-RI exchange (then QLG holds Q_GL^T's rows)
  int64_t q_rows = 0;
  DevBuf QLG;
  // occ-RI output (K C): E_N = X^N C, Z1 = [Q_GG Q_GL][E_L; E_N],
  // Z2 = [Q_GL^T Q_LL][E_L; E_N] (N_mu x n_occ); mixed: ELN (row i = [E_L(:, i);
  // E_N(:, i)]) and Z12 (row i = [Z1(:, i); Z2(:, i)]) planes, and (K C)^T =
  // -(Z12)(xln)^T as k-range partial products
  DevBuf EN, Z1, Z2, KCpart, d_zprobs, d_kcprobs;
  Planes ELN, Z12;
  int ri_nocc = -1, kcparts = 0, kctiles = 0;
  // factored density: D = C C^T for the energy
  DevBuf Docc;
  // every universal point a fitting function: W_Uw = (R_U | xi_w), N_g x N_mu
  // (the fit's xi are then the window functions only)
  bool all_points = false;
  DevBuf WUw;
  // captured exchange: replayed while (mode, operands, K) stay the same
  hipGraph_t xgraph = nullptr;
  hipGraphExec_t xexec = nullptr;
  const void* xkey_in = nullptr;
  const void* xkey_out = nullptr;
  int xkey_nocc = -1;
  bool xkey_ri = false;
  void drop_graph() {
    if (xexec) (void)hipGraphExecDestroy(xexec);
    if (xgraph) (void)hipGraphDestroy(xgraph);
    xexec = nullptr;
    xgraph = nullptr;
    xkey_in = xkey_out = nullptr;
    xkey_nocc = -1;
  }
  ~isdf_fit_s() { drop_graph(); }
};

namespace {

// Device bytes a buffer-sizing rule of the plan may assume available: free
// memory plus the plan's cached blocks, measured the first time the rule
// asks and kept, so that repeated fits and exchanges of the plan size their
// buffers alike and take them back from its cache (a large allocation costs
// far more than the kernels that fill it).
enum { AVAIL_PHI = 0, AVAIL_COULOMB = 1, AVAIL_RI = 2, AVAIL_UNIVERSAL = 3 };
isdf_status plan_available(isdf_plan_s* pl, int rule, double* bytes) {
  auto it = pl->avail_memo.find(rule);
  if (it != pl->avail_memo.end()) {
    *bytes = it->second;
    return ISDF_OK;
  }
  isdf_status st;
  if ((st = pl->mem->available(bytes)) != ISDF_OK) return st;
  pl->avail_memo[rule] = *bytes;
  return ISDF_OK;
}

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
    if ((pl->prof >> fam) & 1) {
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

// Events around the three passes of one transform call, one record per pass
// (a pass is one kernel launch) when the FFT family is being timed.
struct FftEvents {
  isdf_plan_s* pl;
  hipEvent_t e[6] = {};
  bool on = false;
  explicit FftEvents(isdf_plan_s* p) : pl(p) {
    if (!((pl->prof >> ISDF_K_FFT) & 1)) return;
    on = true;
    for (auto& x : e)
      if (!(x = prof_event(pl))) on = false;
  }
  hipEvent_t* ev() { return on ? e : nullptr; }
  void commit(std::array<double, 3> bytes) {
    if (!on) return;
    for (int p = 0; p < 3; ++p) pl->pending.push_back({ISDF_K_FFT, e[2 * p], e[2 * p + 1], bytes[p], 0.0});
  }
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

// Algorithmic counts; a lower-triangle (symmetric) update counts only the
// N(N+1)/2 entries it has to produce.
double gemm_outputs(const GemmProblem& p) {
  return p.lower ? 0.5 * (double)p.N * (p.N + 1.0) : (double)p.M * p.N;
}
double gemm_bytes(const GemmProblem& p) {
  return 8.0 * ((double)p.M * p.K + (p.lower ? 0.0 : (double)p.K * p.N) +
                gemm_outputs(p) * (p.beta != 0.0 ? 2 : 1));
}
double gemm_flops(const GemmProblem& p) { return 2.0 * gemm_outputs(p) * p.K; }

int mixed_splits(const isdf_plan_s* pl) {
  return pl->opts.precision == ISDF_MIXED_X3 ? 2 : pl->opts.precision == ISDF_MIXED_X6 ? 3 : 0;
}
bool mixed_on(const isdf_plan_s* pl, int bit) {
  if (mixed_splits(pl) == 0) return false;
  // default: the Coulomb metric and the exchange; Theta only on request (its
  // errors are amplified by the conditioning of the interpolation metric)
  const int mask = pl->opts.mixed_mask == 0 ? (ISDF_MIX_W | ISDF_MIX_EXCHANGE) : pl->opts.mixed_mask;
  return (mask & bit) != 0;
}

int family_tag(int fam) {
  switch (fam) {
    case ISDF_K_GEMM_SELECT: return 1;
    case ISDF_K_GEMM_METRIC: return 2;
    case ISDF_K_GEMM_FIT: return 3;
    case ISDF_K_GEMM_EXCHANGE: return 4;
    default: return 0;
  }
}

isdf_status mixed_prof(isdf_plan_s* pl, int fam, int epi, const MixedProblem& p) {
  const int S = mixed_splits(pl);
  ProfScope ps(pl, fam, 2.0 * S * ((double)p.M * p.K + (double)p.K * p.N) + 8.0 * (double)p.M * p.N,
               2.0 * p.M * (double)p.N * p.K);
  return gemm_mixed(pl->stream, epi, S, p, family_tag(fam));
}

// Class of a single GEMM problem for the tile-shape table: epilogue, role,
// triangle, operand layouts, accumulation and log2 buckets of the sizes.
std::string gemm_key(int epi, int tag, const GemmProblem& p) {
  auto lg = [](int x) {
    int b = 0;
    while ((2 << b) <= x) ++b;
    return b;
  };
  char k[160];
  std::snprintf(k, sizeof(k), "e%d t%d l%d a%d b%d c%d g%d m%d n%d k%d", epi, tag, p.lower ? 1 : 0,
                p.transA, p.transB, p.beta != 0.0 ? 1 : 0, p.bidx ? 1 : 0, lg(p.M), lg(p.N),
                lg(std::max(p.K, 1)));
  return k;
}

// Time every valid shape on the problem itself (C saved and restored when
// the update reads it) and keep the fastest; results of all shapes agree
// bit for bit, so the choice changes speed only.
isdf_status tune_problem(isdf_plan_s* pl, int epi, int tag, const GemmProblem& p, const std::string& key) {
  hipStream_t s = pl->stream;
  const bool rd = p.beta != 0.0;
  const size_t cbytes = sizeof(double) * ((size_t)(p.N - 1) * p.ldc + p.M);
  DevBuf save;
  isdf_status st;
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  if (rd) {
    if ((st = save.alloc(cbytes)) != ISDF_OK) return st;
    ISDF_HIP_TRY(hipMemcpyAsync(save.p, p.C, cbytes, hipMemcpyDeviceToDevice, s));
  }
  hipEvent_t a, b;
  ISDF_HIP_TRY(hipEventCreate(&a));
  ISDF_HIP_TRY(hipEventCreate(&b));
  std::vector<float> us(GEMM_NSHAPE, -1.f);
  int best = gemm_default_shape(epi, p.M, p.N, p.K, p.lower != 0);
  float tbest = 0.f;
  for (int sh = 0; sh < GEMM_NSHAPE; ++sh) {
    if (p.lower && kShapes[sh].bm != kShapes[sh].bn) continue;
    if (p.bidx && kShapes[sh].mf4 == 2) continue;  // the large tiles take no gathered rows
    if (!p.transA && !gemm_shape_takes_mfast_a(sh)) continue;
    if (p.transB && !gemm_shape_takes_nfast_b(sh)) continue;
    float tmin = 0.f;
    for (int r = 0; r < pl->tune_reps; ++r) {
      if (rd) ISDF_HIP_TRY(hipMemcpyAsync(p.C, save.p, cbytes, hipMemcpyDeviceToDevice, s));
      ISDF_HIP_TRY(hipEventRecord(a, s));
      if ((st = gemm_f64(s, epi, p, tag, sh)) != ISDF_OK) return st;
      ISDF_HIP_TRY(hipEventRecord(b, s));
      ISDF_HIP_TRY(hipEventSynchronize(b));
      float ms = 0.f;
      ISDF_HIP_TRY(hipEventElapsedTime(&ms, a, b));
      if (r == 0 || ms < tmin) tmin = ms;
    }
    us[sh] = 1e3f * tmin;
    if (us[sh] >= 0.f && (tbest == 0.f || us[sh] < tbest)) {
      tbest = us[sh];
      best = sh;
    }
  }
  if (rd) ISDF_HIP_TRY(hipMemcpyAsync(p.C, save.p, cbytes, hipMemcpyDeviceToDevice, s));
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  pl->tune[key] = best;
  pl->tune_us[key] = us;
  return ISDF_OK;
}

isdf_status gemm_prof(isdf_plan_s* pl, int fam, int epi, const GemmProblem& p) {
  const int tag = family_tag(fam);
  int shape = -1;
  if (p.tmask_mode) {  // screening masks are laid out for 64 x 64 tiles
    ProfScope ps(pl, fam, gemm_bytes(p), gemm_flops(p));
    return gemm_f64(pl->stream, epi, p, tag, 0);
  }
  if (pl->tuning || !pl->tune.empty()) {
    const std::string key = gemm_key(epi, tag, p);
    auto it = pl->tune.find(key);
    if (it == pl->tune.end() && pl->tuning && p.M > 0 && p.N > 0) {
      isdf_status st = tune_problem(pl, epi, tag, p, key);
      if (st != ISDF_OK) return st;
      it = pl->tune.find(key);
    }
    if (it != pl->tune.end()) shape = it->second;
  }
  ProfScope ps(pl, fam, gemm_bytes(p), gemm_flops(p));
  return gemm_f64(pl->stream, epi, p, tag, shape);
}

isdf_status fft_prof(isdf_plan_s* pl, double* z, int batch, const int grid[3], int sign) {
  int passes = (grid[0] > 1) + (grid[1] > 1) + (grid[2] > 1);
  const double ng = (double)grid[0] * grid[1] * grid[2];
  ProfScope ps(pl, ISDF_K_FFT, 32.0 * ng * batch * passes, 0.0);
  return fft3d(pl->stream, z, batch, grid, sign, nullptr);
}

// Centres of the balls a window domain is made of: every point of the window
// of atom A lies within r_max of a translate A + T.  The translates are read
// back from the points (the nearest one to each point, or a neighbour of it),
// so that the basis kernel can skip the images of a shell that are farther
// than r_img + r_max from all of them: those fail the cutoff test at every
// point of the window.  False (every image kept) for the universal domain,
// whole-grid windows, or a point with no translate in reach.
bool window_centres(const HostPlan& hp, const HostDomain& D, std::vector<std::array<double, 3>>& ctr) {
  ctr.clear();
  if (D.atom < 0 || !std::isfinite(D.r_max)) return false;
  const int* g = hp.grid[D.level];
  if ((int64_t)D.points.size() >= (int64_t)g[0] * g[1] * g[2]) return false;
  const double* a = hp.lattice;
  const double* inv = hp.inv;
  const double A[3] = {hp.xyz[3 * D.atom], hp.xyz[3 * D.atom + 1], hp.xyz[3 * D.atom + 2]};
  const double r2 = D.r_max * D.r_max * (1.0 + 1e-12) + 1e-12;
  std::set<std::array<int, 3>> Ts;
  std::array<int, 3> last{INT_MIN, 0, 0};
  for (int32_t flat : D.points) {
    const int i1 = flat % g[0], rem = flat / g[0], i2 = rem % g[1], i3 = rem / g[1];
    const double f[3] = {(double)i1 / g[0], (double)i2 / g[1], (double)i3 / g[2]};
    double dr[3];
    for (int q = 0; q < 3; ++q) dr[q] = f[0] * a[q] + f[1] * a[3 + q] + f[2] * a[6 + q] - A[q];
    auto within = [&](const std::array<int, 3>& T) {
      double s2 = 0.0;
      for (int q = 0; q < 3; ++q) {
        const double v = dr[q] - (T[0] * a[q] + T[1] * a[3 + q] + T[2] * a[6 + q]);
        s2 += v * v;
      }
      return s2 <= r2;
    };
    if (last[0] != INT_MIN && within(last)) continue;  // runs of points share a translate
    std::array<int, 3> base;
    for (int i = 0; i < 3; ++i)
      base[i] = (int)std::lround(dr[0] * inv[i] + dr[1] * inv[3 + i] + dr[2] * inv[6 + i]);
    bool found = false;
    for (int d0 = -1; d0 <= 1 && !found; ++d0)
      for (int d1 = -1; d1 <= 1 && !found; ++d1)
        for (int d2 = -1; d2 <= 1 && !found; ++d2) {
          const std::array<int, 3> T{base[0] + d0, base[1] + d1, base[2] + d2};
          if (within(T)) {
            Ts.insert(T);
            last = T;
            found = true;
          }
        }
    if (!found) return false;
  }
  for (const auto& T : Ts) {
    std::array<double, 3> c;
    for (int q = 0; q < 3; ++q) c[q] = A[q] + T[0] * a[q] + T[1] * a[3 + q] + T[2] * a[6 + q];
    ctr.push_back(c);
  }
  return true;
}


isdf_status upload_plan(isdf_plan_s* pl) {
  if (pl->uploaded) return ISDF_OK;
  HostPlan& hp = pl->hp;
  std::vector<ShellDev> sh(hp.n_shells);
  for (int s = 0; s < hp.n_shells; ++s) {
    double a = hp.shell_alpha[s];
    // unit single-centre norm: N_s = (2a/pi)^(3/4), N_p = N_s 2 sqrt(a),
    // N_d = N_s 4a/sqrt(3) (one factor for all five real solid harmonics)
    double nrm = std::pow(2.0 * a / M_PI, 0.75);
    if (hp.shell_l[s] == 1) nrm *= 2.0 * std::sqrt(a);
    if (hp.shell_l[s] == 2) nrm *= 4.0 * a / std::sqrt(3.0);
    sh[s] = ShellDev{a, nrm, hp.shell_l[s], hp.img_off[s], hp.img_cnt[s], 0};
  }
  std::vector<ColShell> cols;
  std::vector<DomainDev> doms;
  std::vector<int32_t> points, funcs;
  std::vector<BasisTile> tiles;
  pl->pts_off.clear();
  pl->phi_off.clear();
  pl->func_off.clear();
  pl->tile_off.clear();
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
    std::vector<std::array<double, 3>> ctr;
    const bool masked = window_centres(hp, D, ctr);
    for (int c = 0; c < dd.nG;) {
      int s = hp.f_shell[D.funcs[c]];
      const int ni = std::min(hp.img_cnt[s], 64);
      uint64_t mask = ni >= 64 ? ~0ull : (1ull << ni) - 1;  // every image of the shell
      if (masked) {
        mask = 0;
        const double lim = std::sqrt(hp.ln_inv_tau / hp.shell_alpha[s]) + D.r_max + 1e-6;
        for (int m = 0; m < ni; ++m) {
          const double* I = &hp.img_xyz[3 * (size_t)(hp.img_off[s] + m)];
          for (const auto& q : ctr) {
            const double dx = I[0] - q[0], dy = I[1] - q[1], dz = I[2] - q[2];
            if (dx * dx + dy * dy + dz * dz <= lim * lim) {
              mask |= 1ull << m;
              break;
            }
          }
        }
      }
      cols.push_back(ColShell{s, c, mask});
      c += 2 * hp.shell_l[s] + 1;
    }
    dd.colshell_cnt = (int)cols.size() - dd.colshell_off;
    doms.push_back(dd);
    pl->pts_off.push_back(dd.pts_off);
    pl->phi_off.push_back(phi_off);
    pl->func_off.push_back((int64_t)funcs.size());
    points.insert(points.end(), D.points.begin(), D.points.end());
    funcs.insert(funcs.end(), D.funcs.begin(), D.funcs.end());
    pl->tile_off.push_back((int)tiles.size());
    for (int st = 0; st < dd.pts; st += 256) tiles.push_back(BasisTile{(int)d, st});
    phi_off += (int64_t)dd.pts * dd.nG;
  }
  pl->tile_off.push_back((int)tiles.size());
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
  if (!pl->mlp_w.empty())
    if ((st = upload(pl->d_mlp_w, pl->mlp_w)) != ISDF_OK) return st;
  for (int i = 0; i <= NSTAGE; ++i) ISDF_HIP_TRY(hipEventCreate(&pl->ev[i]));
  // cyclic boxes and point maps (pruned forward transforms)
  {
    std::vector<int32_t> maps;
    pl->box.assign(hp.domains.size(), {0, 0, 0, 0, 0, 0, -1});
    for (size_t d = 0; d < hp.domains.size(); ++d) {
      const HostDomain& D = hp.domains[d];
      const int* g = hp.grid[D.level];
      std::array<int32_t, 7>& b = pl->box[d];
      if ((int64_t)D.points.size() == (int64_t)g[0] * g[1] * g[2]) {
        b = {0, 0, 0, g[0], g[1], g[2], -1};
        continue;
      }
      for (int ax = 0; ax < 3; ++ax) {  // smallest cyclic interval holding every coordinate
        std::vector<char> occ(g[ax], 0);
        for (int32_t f : D.points) {
          const int c = ax == 0 ? f % g[0] : ax == 1 ? (f / g[0]) % g[1] : f / (g[0] * g[1]);
          occ[c] = 1;
        }
        int best_len = 0, best_end = 0;
        for (int st0 = 0; st0 < g[ax]; ++st0) {  // longest cyclic run of empty coordinates
          if (occ[st0] || occ[(st0 + g[ax] - 1) % g[ax]] == 0) continue;
          int len = 0;
          while (len < g[ax] && !occ[(st0 + len) % g[ax]]) ++len;
          if (len > best_len) {
            best_len = len;
            best_end = (st0 + len) % g[ax];
          }
        }
        b[ax] = best_len ? best_end : 0;
        b[3 + ax] = g[ax] - best_len;
      }
      b[6] = (int32_t)maps.size();
      maps.resize(maps.size() + (size_t)b[3] * b[4] * b[5], -1);
      for (size_t i = 0; i < D.points.size(); ++i) {
        const int32_t f = D.points[i];
        int c[3] = {f % g[0], (f / g[0]) % g[1], f / (g[0] * g[1])};
        for (int ax = 0; ax < 3; ++ax) c[ax] = (c[ax] - b[ax] + g[ax]) % g[ax];
        maps[b[6] + c[0] + (size_t)b[3] * (c[1] + (size_t)b[4] * c[2])] = (int32_t)i;
      }
    }
    if ((st = upload(pl->d_boxmap, maps)) != ISDF_OK) return st;
  }
  pl->uploaded = true;
  return ISDF_OK;
}

inline int64_t level_ng(const HostPlan& hp, int l) {
  return (int64_t)hp.grid[l][0] * hp.grid[l][1] * hp.grid[l][2];
}

// ---------------------------------------------------------------- selection
// One selection domain: basis values at phi_base + phi_off (column-major,
// leading dimension pts), working diagonal at diag_base + diag_off (consumed).
struct SelSpec {
  int level;
  int pts, nG, nL, n_mu;
  int64_t phi_off, diag_off;
  int lone;  // the plan's only domain on its level (blocked selection above RL_MIN_PIVOTS)
};

// Greedy pivoted Cholesky of every spec domain, one batch per level.  Writes
// pivots (local to the spec domain) to piv_out + piv_off[d], the number found
// to counts[d] and the residual of the last pivot to dlast[d].
// Candidate-restricted blocked selection of one domain (see kernels_crb.hip).
// phi, diag (exact initial diagonal on entry, -1 at chosen points on exit) and
// the factor L (pts x n_mu, all points) are the domain's own; the pivots go to
// piv_out + X.piv_off and the final state to *st (count, last residual).
isdf_status crb_select(isdf_plan_s* pl, const SelDomain& X, const double* phi_base, double* diag_base,
                       double* L, int32_t* piv_out, SelState* st) {
  const HostPlan& hp = pl->hp;
  hipStream_t s = pl->stream;
  const int n = X.pts, nG = X.nG, nL = X.nL, nmu = X.n_mu;
  const double* phi = phi_base + X.phi_off;
  double* d = diag_base + X.diag_off;
  int32_t* piv = piv_out + X.piv_off;
  const double tau = hp.tie_tol, eps = hp.eps_isdf;
  isdf_status e;
  DevBuf cidx, dC, dC2, info, phiC, LC, RCC, LCb, tmaxb, tidxb, tvalb, stb, pivC, tdom, sdb, phiP, LP, Ub;
  const int Tmax = n;
  int T = std::min(n, CRB_CANDIDATES);
  if ((e = cidx.alloc(sizeof(int32_t) * n)) != ISDF_OK) return e;
  if ((e = dC.alloc(sizeof(double) * n)) != ISDF_OK) return e;
  if ((e = info.alloc(sizeof(CrbInfo))) != ISDF_OK) return e;
  if ((e = pivC.alloc(sizeof(int32_t) * CRB_BLOCK)) != ISDF_OK) return e;
  if ((e = stb.alloc(sizeof(SelState))) != ISDF_OK) return e;
  if ((e = sdb.alloc(sizeof(SelDomain))) != ISDF_OK) return e;
  int kb = 0;
  double d0max = -1.0, dlast = 0.0;
  while (kb < nmu) {
    // candidates of this block and the exactness bound
    if ((e = launch_crb_candidates(s, d, n, T, cidx.as<int32_t>(), dC.as<double>(),
                                   info.as<CrbInfo>())) != ISDF_OK)
      return e;
    CrbInfo ci{};
    ISDF_HIP_TRY(hipMemcpyAsync(&ci, info.p, sizeof(CrbInfo), hipMemcpyDeviceToHost, s));
    ISDF_HIP_TRY(hipStreamSynchronize(s));
    if (kb == 0) d0max = ci.dmax;
    if (ci.nactive == 0 || !(ci.dmax > eps * d0max)) break;
    const int nc = ci.nc;
    const int nb = std::min(CRB_BLOCK, nmu - kb);
    // R_CC = M(C, C) - L(C, :kb) L(C, :kb)^T (lower triangle)
    if ((e = phiC.alloc(sizeof(double) * (size_t)nc * nG)) != ISDF_OK) return e;
    if ((e = launch_crb_gather(s, phi, n, cidx.as<int32_t>(), nc, nG, phiC.as<double>(), nc)) != ISDF_OK)
      return e;
    if ((e = RCC.alloc(sizeof(double) * (size_t)nc * nc)) != ISDF_OK) return e;
    {
      GemmProblem g{};
      g.A = phiC.as<double>();
      g.lda = nc;
      g.B = g.A;
      g.ldb = nc;
      g.transB = 1;
      g.C = RCC.as<double>();
      g.ldc = nc;
      g.M = g.N = nc;
      g.K = nG;
      g.kL = nL;
      g.lower = 1;
      if ((e = gemm_prof(pl, ISDF_K_GEMM_SELECT, EPI_THETA, g)) != ISDF_OK) return e;
    }
    if (kb > 0) {
      if ((e = LC.alloc(sizeof(double) * (size_t)nc * kb)) != ISDF_OK) return e;
      if ((e = launch_crb_gather(s, L, n, cidx.as<int32_t>(), nc, kb, LC.as<double>(), nc)) != ISDF_OK)
        return e;
      GemmProblem g{};
      g.A = LC.as<double>();
      g.lda = nc;
      g.B = g.A;
      g.ldb = nc;
      g.transB = 1;
      g.C = RCC.as<double>();
      g.ldc = nc;
      g.M = g.N = nc;
      g.K = kb;
      g.alpha = -1.0;
      g.beta = 1.0;
      g.lower = 1;
      if ((e = gemm_prof(pl, ISDF_K_GEMM_SELECT, EPI_AXPBY, g)) != ISDF_OK) return e;
    }
    // greedy steps on the candidates: right-looking within the block on R_CC
    SelDomain B{};
    B.phi_off = 0;
    B.lfac_off = 0;
    B.diag_off = 0;
    B.prow_off = 0;
    B.pts = nc;
    B.nG = 0;
    B.nL = 0;
    B.n_mu = nb;
    B.tile_off = 0;
    B.ntiles = (nc + SEL_TILE - 1) / SEL_TILE;
    B.piv_off = 0;
    if ((e = copy_in(sdb.p, &B, sizeof(SelDomain))) != ISDF_OK) return e;
    std::vector<int32_t> td(B.ntiles, 0);
    if ((e = upload(tdom, td)) != ISDF_OK) return e;
    if ((e = LCb.alloc(sizeof(double) * (size_t)nc * nb)) != ISDF_OK) return e;
    if ((e = tmaxb.alloc(sizeof(double) * 2 * B.ntiles)) != ISDF_OK) return e;
    if ((e = tidxb.alloc(sizeof(int32_t) * 2 * B.ntiles)) != ISDF_OK) return e;
    if ((e = tvalb.alloc(sizeof(double) * 2 * B.ntiles)) != ISDF_OK) return e;
    if ((e = dC2.alloc(sizeof(double) * (size_t)nc)) != ISDF_OK) return e;
    ISDF_HIP_TRY(hipMemsetAsync(stb.p, 0, sizeof(SelState), s));
    const SelDomain* Dd = sdb.as<SelDomain>();
    const double dstop = ci.theta >= 0.0 ? ci.theta / (1.0 - tau) : 0.0;
    SelState* Sd = stb.as<SelState>();
    if ((e = launch_sel_init(s, Dd, tdom.as<int32_t>(), 0, B.ntiles, dC.as<double>(), tmaxb.as<double>(),
                             tidxb.as<int32_t>(), tau, tvalb.as<double>())) != ISDF_OK)
      return e;
    CrbBlock cb{};
    cb.R = RCC.as<double>();
    cb.Lb = LCb.as<double>();
    cb.d[0] = dC.as<double>();
    cb.d[1] = dC2.as<double>();
    cb.t[0] = tmaxb.as<double>();
    cb.t[1] = tmaxb.as<double>() + B.ntiles;
    cb.i[0] = tidxb.as<int32_t>();
    cb.i[1] = tidxb.as<int32_t>() + B.ntiles;
    cb.v[0] = tvalb.as<double>();
    cb.v[1] = tvalb.as<double>() + B.ntiles;
    cb.st = Sd;
    cb.pivC = pivC.as<int32_t>();
    cb.nc = nc;
    cb.nb = nb;
    cb.tau = tau;
    cb.eps = eps;
    cb.dstop = dstop;
    cb.d0max = d0max;
    // Steps go out in chunks; after each chunk the state is copied to pinned
    // memory, and the copy of the chunk before is checked while this one
    // runs: a block that stopped early (most do, at the theta bound) costs at
    // most two chunks of launches that return at once.
    if (!pl->crb_host) {
      ISDF_HIP_TRY(hipHostMalloc((void**)&pl->crb_host, 2 * sizeof(SelState)));
      for (auto& ev : pl->crb_ev) ISDF_HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    for (int k0 = 0, chunk = 0; k0 <= nb; k0 += CRB_CHUNK, ++chunk) {
      const int k1 = std::min(nb + 1, k0 + CRB_CHUNK);
      for (int k = k0; k < k1; ++k) {
        ProfScope ps(pl, ISDF_K_SELECT_BLOCK, 8.0 * nc * (k + 4.0) + 12.0 * B.ntiles, 2.0 * nc * k);
        if ((e = launch_crb_step(s, k, cb)) != ISDF_OK) return e;
      }
      if (k1 > nb) break;
      const int slot = chunk & 1;
      ISDF_HIP_TRY(hipMemcpyAsync(pl->crb_host + slot, Sd, sizeof(SelState), hipMemcpyDeviceToHost, s));
      ISDF_HIP_TRY(hipEventRecord(pl->crb_ev[slot], s));
      if (chunk > 0) {
        ISDF_HIP_TRY(hipEventSynchronize(pl->crb_ev[slot ^ 1]));
        if (pl->crb_host[slot ^ 1].done) break;
      }
    }
    SelState bs{};
    ISDF_HIP_TRY(hipMemcpyAsync(&bs, stb.p, sizeof(SelState), hipMemcpyDeviceToHost, s));
    ISDF_HIP_TRY(hipStreamSynchronize(s));
    const int sb = bs.count;
    if (sb == 0) {
      if (bs.reason == SEL_END_BLOCK && nc < ci.nactive && T < Tmax) {
        T = std::min(Tmax, 2 * T);  // the cut fell inside a near-tie: widen the candidates
        continue;
      }
      break;
    }
    // the block's pivots and their factor columns over every point
    if ((e = launch_map_pivots(s, cidx.as<int32_t>(), 0, pivC.as<int32_t>(), piv + kb, sb)) != ISDF_OK)
      return e;
    double* Lb = L + (int64_t)kb * n;
    if ((e = phiP.alloc(sizeof(double) * (size_t)sb * nG)) != ISDF_OK) return e;
    if ((e = launch_crb_gather(s, phi, n, piv + kb, sb, nG, phiP.as<double>(), sb)) != ISDF_OK) return e;
    {
      GemmProblem g{};  // M(:, P)
      g.A = phi;
      g.lda = n;
      g.B = phiP.as<double>();
      g.ldb = sb;
      g.transB = 1;
      g.C = Lb;
      g.ldc = n;
      g.M = n;
      g.N = sb;
      g.K = nG;
      g.kL = nL;
      if ((e = gemm_prof(pl, ISDF_K_GEMM_SELECT, EPI_THETA, g)) != ISDF_OK) return e;
    }
    if (kb > 0) {  // - L(:, :kb) L(P, :kb)^T
      if ((e = LP.alloc(sizeof(double) * (size_t)sb * kb)) != ISDF_OK) return e;
      if ((e = launch_crb_gather(s, L, n, piv + kb, sb, kb, LP.as<double>(), sb)) != ISDF_OK) return e;
      GemmProblem g{};
      g.A = L;
      g.lda = n;
      g.B = LP.as<double>();
      g.ldb = sb;
      g.transB = 1;
      g.C = Lb;
      g.ldc = n;
      g.M = n;
      g.N = sb;
      g.K = kb;
      g.alpha = -1.0;
      g.beta = 1.0;
      if ((e = gemm_prof(pl, ISDF_K_GEMM_SELECT, EPI_AXPBY, g)) != ISDF_OK) return e;
    }
    // U = L(P, blk) from the block's candidate factor, then L(:, blk) U^{-T}
    if ((e = Ub.alloc(sizeof(double) * (size_t)sb * sb)) != ISDF_OK) return e;
    if ((e = launch_crb_gather(s, LCb.as<double>(), nc, pivC.as<int32_t>(), sb, sb, Ub.as<double>(), sb)) !=
        ISDF_OK)
      return e;
    for (int jb = 0; jb < sb; jb += 64) {
      const int w = std::min(64, sb - jb);
      if (jb > 0) {
        GemmProblem g{};
        g.A = Lb;
        g.lda = n;
        g.B = Ub.as<double>() + jb;
        g.ldb = sb;
        g.transB = 1;
        g.C = Lb + (int64_t)jb * n;
        g.ldc = n;
        g.M = n;
        g.N = w;
        g.K = jb;
        g.alpha = -1.0;
        g.beta = 1.0;
        if ((e = gemm_prof(pl, ISDF_K_GEMM_SELECT, EPI_AXPBY, g)) != ISDF_OK) return e;
      }
      if ((e = launch_crb_trsm_block(s, Lb, n, n, Ub.as<double>(), sb, jb, w)) != ISDF_OK) return e;
    }
    if ((e = launch_crb_diag(s, d, n, Lb, n, sb, piv + kb)) != ISDF_OK) return e;
    kb += sb;
    dlast = bs.dpiv;
    if (bs.reason == SEL_END_EPS) break;
  }
  SelState fin{};
  fin.d0max = d0max;
  fin.dpiv = dlast;
  fin.done = 1;
  fin.count = kb;
  fin.reason = kb >= nmu ? SEL_END_COUNT : SEL_END_EPS;
  return copy_in(st, &fin, sizeof(SelState));
}

isdf_status select_points(isdf_plan_s* pl, const std::vector<SelSpec>& spec,
                          const double* phi_base, double* diag_base, int32_t* piv_out,
                          const std::vector<int64_t>& piv_off, std::vector<int>& counts,
                          std::vector<double>& dlast) {
  const HostPlan& hp = pl->hp;
  hipStream_t s = pl->stream;
  const int nd = (int)spec.size();
  counts.assign(nd, 0);
  dlast.assign(nd, 0.0);
  if (nd == 0) return ISDF_OK;
  std::vector<SelDomain> sd(nd);
  std::vector<int32_t> tile_dom;
  int64_t lf = 0, pr = 0;
  for (int d = 0; d < nd; ++d) {
    const SelSpec& S = spec[d];
    SelDomain& x = sd[d];
    x.phi_off = S.phi_off;
    x.lfac_off = lf;
    x.diag_off = S.diag_off;
    x.prow_off = pr;
    x.pts = S.pts;
    x.nG = S.nG;
    x.nL = S.nL;
    x.n_mu = S.n_mu;
    x.tile_off = (int)tile_dom.size();
    x.ntiles = (x.pts + SEL_TILE - 1) / SEL_TILE;
    x.piv_off = (int)piv_off[d];
    for (int t = 0; t < x.ntiles; ++t) tile_dom.push_back(d);
    lf += (int64_t)x.pts * x.n_mu;
    pr += x.nG + x.n_mu;
  }
  isdf_status st;
  // A domain alone on its level with many pivots (the universal grid) runs
  // the candidate-restricted blocked selection (crb_select); the others are
  // batched per level, left-looking, one pick and one column launch a step.
  std::vector<char> blocked(nd, 0);
  for (int d = 0; d < nd; ++d) blocked[d] = spec[d].lone && sd[d].n_mu > RL_MIN_PIVOTS;
  DevBuf lfac, prow, tmax, tidx, state, d_sd, d_tile_dom;
  if ((st = upload(d_sd, sd)) != ISDF_OK) return st;
  if ((st = upload(d_tile_dom, tile_dom)) != ISDF_OK) return st;
  const int ntiles = (int)tile_dom.size();
  if ((st = lfac.alloc(sizeof(double) * std::max<int64_t>(lf, 1))) != ISDF_OK) return st;
  if ((st = prow.alloc(sizeof(double) * std::max<int64_t>(pr, 1))) != ISDF_OK) return st;
  if ((st = tmax.alloc(sizeof(double) * std::max(ntiles, 1))) != ISDF_OK) return st;
  if ((st = tidx.alloc(sizeof(int32_t) * std::max(ntiles, 1))) != ISDF_OK) return st;
  if ((st = state.alloc(sizeof(SelState) * nd)) != ISDF_OK) return st;
  ISDF_HIP_TRY(hipMemsetAsync(state.p, 0, sizeof(SelState) * nd, s));
  const double tau = hp.tie_tol, eps = hp.eps_isdf;
  SelDomain* D = d_sd.as<SelDomain>();
  SelState* S = state.as<SelState>();
  // one batch per level (domains of a level are contiguous)
  int d0 = 0;
  while (d0 < nd) {
    int d1 = d0;
    int kmax = 0;
    while (d1 < nd && spec[d1].level == spec[d0].level) {
      kmax = std::max(kmax, spec[d1].n_mu);
      ++d1;
    }
    if (blocked[d0]) {
      if ((st = crb_select(pl, sd[d0], phi_base, diag_base, lfac.as<double>() + sd[d0].lfac_off,
                           piv_out, S + d0)) != ISDF_OK)
        return st;
      d0 = d1;
      continue;
    }
    const int t0 = sd[d0].tile_off;
    const int t1 = (d1 < nd) ? sd[d1].tile_off : ntiles;
    if ((st = launch_sel_init(s, D, d_tile_dom.as<int32_t>(), t0, t1 - t0, diag_base,
                              tmax.as<double>(), tidx.as<int32_t>(), tau)) != ISDF_OK)
      return st;
    for (int k = 0; k <= kmax; ++k) {
      double col_bytes = 0.0, col_flops = 0.0, pick_bytes = 0.0;
      for (int d = d0; d < d1; ++d) {
        if (sd[d].n_mu <= k) continue;
        col_bytes += 8.0 * sd[d].pts * ((double)sd[d].nG + k + 3.0);
        col_flops += 2.0 * sd[d].pts * ((double)sd[d].nG + k) + 3.0 * sd[d].pts;
        pick_bytes += 12.0 * sd[d].ntiles + 16.0 * (sd[d].nG + k);
      }
      ProfScope ps_pick(pl, ISDF_K_SELECT_PICK, pick_bytes, 0.0);
      if ((st = launch_sel_select(s, D, d0, d1 - d0, k, S, phi_base, lfac.as<double>(), diag_base,
                                  tmax.as<double>(), tidx.as<int32_t>(), prow.as<double>(),
                                  piv_out, tau, eps)) != ISDF_OK)
        return st;
      ps_pick.finish();
      if (k == kmax) break;
      {
        ProfScope ps_col(pl, ISDF_K_SELECT_COLUMN, col_bytes, col_flops);
        if ((st = launch_sel_column(s, D, d_tile_dom.as<int32_t>(), t0, t1 - t0, k, S, phi_base,
                                    lfac.as<double>(), diag_base, prow.as<double>(),
                                    tmax.as<double>(), tidx.as<int32_t>(), tau)) != ISDF_OK)
          return st;
      }
    }
    d0 = d1;
  }
  std::vector<SelState> hs(nd);
  ISDF_HIP_TRY(hipMemcpyAsync(hs.data(), state.p, sizeof(SelState) * nd, hipMemcpyDeviceToHost, s));
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  for (int d = 0; d < nd; ++d) {
    counts[d] = hs[d].count;
    dlast[d] = hs[d].dpiv;
  }
  return ISDF_OK;
}

// Features of every point of domains [g0, g1) (learned selector input),
// at their global point offsets in feats (16 per point).
isdf_status compute_features(isdf_plan_s* pl, isdf_fit_s* f, float* feats, int g0 = 0, int g1 = -1) {
  HostPlan& hp = pl->hp;
  hipStream_t s = pl->stream;
  const int nd = (int)hp.domains.size();
  if (g1 < 0) g1 = nd;
  if (g1 <= g0) return ISDF_OK;
  MlpGeom g{};
  for (int i = 0; i < 9; ++i) {
    g.lat[i] = hp.lattice[i];
    g.inv[i] = hp.inv[i];
  }
  g.n_atoms = hp.n_atoms;
  g.n_levels = hp.n_levels;
  std::vector<MlpDomain> md(nd);
  for (int d = 0; d < nd; ++d) {
    const HostDomain& D = hp.domains[d];
    MlpDomain& m = md[d];
    m.pts_off = pl->pts_off[d];
    m.pts = (int)D.points.size();
    m.level = D.level;
    m.atom = D.atom;
    m.nL = D.nL;
    m.n_mu = D.n_mu;
    for (int i = 0; i < 3; ++i) m.grid[i] = hp.grid[D.level][i];
    double h = 0.0;
    for (int i = 0; i < 3; ++i) {
      const double* a = hp.lattice + 3 * i;
      h = std::max(h, std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) / hp.grid[D.level][i]);
    }
    m.h = h;
    if (D.atom >= 0) {
      m.rs = D.r_max;
    } else if (hp.n_levels > 1) {
      m.rs = std::sqrt(-std::log(hp.eps_r) / hp.alpha_bound[0]);
    } else {
      double h0 = 0.0;
      for (int i = 0; i < 3; ++i) {
        const double* a = hp.lattice + 3 * i;
        h0 = std::max(h0, std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) / hp.grid[0][i]);
      }
      m.rs = 10.0 * h0;
    }
  }
  isdf_status st;
  DevBuf d_md, d_atoms;
  if ((st = upload(d_md, md)) != ISDF_OK) return st;
  if ((st = upload(d_atoms, hp.xyz)) != ISDF_OK) return st;
  if ((st = launch_diag_stats(s, d_md.as<MlpDomain>() + g0, g1 - g0, f->diag0.as<double>())) != ISDF_OK)
    return st;
  if ((st = launch_features(s, g, d_md.as<MlpDomain>(), pl->d_points.as<int32_t>(),
                            pl->d_tiles.as<BasisTile>() + pl->tile_off[g0], pl->tile_off[g1] - pl->tile_off[g0],
                            f->aux.as<double>(), f->diag0.as<double>(), d_atoms.as<double>(), feats)) != ISDF_OK)
    return st;
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  return ISDF_OK;
}

// Selection for a fit.  mode[d]: 0 full, 1 candidates from the learned
// scores, 2 candidates given by the caller (cand_in), 3 every point of the
// domain (n_mu_d equals its point count: pivots 0..pts-1, F = I).
// sel_setup sizes the per-domain state and handles what needs no basis
// values (pinned points, all-point domains, the caller's candidate lists);
// sel_group then selects domains [g0, g1) from their basis values at
// phi_base + phi_off[d] (the whole pool, or one domain group of it).
struct SelCtx {
  DevBuf cand;         // candidate lists, at pts_off[d] for domain d
  DevBuf feats, z;     // learned selector: features and scores of every point
  DevBuf phic, diagc, pivc;  // compacted candidate rows of a group (kept across groups)
  std::vector<int32_t> nc_host;
  bool pinned = false, any_cand = false, any_learned = false;
};

int lone_on_level(const HostPlan& hp, int d) {
  int n = 0;
  for (const HostDomain& D : hp.domains) n += D.level == hp.domains[d].level;
  return n == 1;
}

SelSpec full_spec(isdf_plan_s* pl, int d) {
  const HostDomain& D = pl->hp.domains[d];
  return SelSpec{D.level, (int)D.points.size(), (int)D.funcs.size(), D.nL, D.n_mu,
                 pl->phi_off[d], pl->pts_off[d], lone_on_level(pl->hp, d)};
}

isdf_status sel_setup(isdf_plan_s* pl, isdf_fit_s* f, SelCtx& cx, const int64_t* pinned,
                      const std::vector<int>& mode, const int64_t* cand_in, const int64_t* ncand_in) {
  HostPlan& hp = pl->hp;
  hipStream_t s = pl->stream;
  const int nd = (int)hp.domains.size();
  isdf_status st;
  int64_t pv = 0;
  f->piv_off.assign(nd, 0);
  for (int d = 0; d < nd; ++d) {
    f->piv_off[d] = pv;
    pv += hp.domains[d].n_mu;
  }
  if ((st = f->piv.alloc(sizeof(int32_t) * std::max<int64_t>(pv, 1))) != ISDF_OK) return st;
  f->count.assign(nd, 0);
  f->dlast.assign(nd, 0.0);
  f->ncand.assign(nd, 0);
  f->dfinal.assign(nd, 0.0);
  f->fallback.assign(nd, 0);
  if (pinned) {
    cx.pinned = true;
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
    return copy_in(f->piv.p, hp_piv.data(), sizeof(int32_t) * pv);
  }
  // all-point domains: the pivots are the points themselves
  {
    std::vector<int32_t> iota;
    for (int d = 0; d < nd; ++d) {
      if (mode[d] != 3) continue;
      const int np = (int)hp.domains[d].points.size();
      iota.resize(np);
      for (int i = 0; i < np; ++i) iota[i] = i;
      if ((st = copy_in(f->piv.as<int32_t>() + f->piv_off[d], iota.data(), sizeof(int32_t) * np)) != ISDF_OK)
        return st;
      f->count[d] = np;
      f->ncand[d] = np;
    }
  }
  cx.nc_host.assign(nd, 0);
  for (int d = 0; d < nd; ++d) {
    if (mode[d] == 1 || mode[d] == 2) cx.any_cand = true;
    if (mode[d] == 1) cx.any_learned = true;
  }
  if (!cx.any_cand) return ISDF_OK;
  if ((st = cx.cand.alloc(sizeof(int32_t) * std::max<int64_t>(pl->pts_total, 1))) != ISDF_OK) return st;
  if ((st = f->cflag.alloc(std::max<int64_t>(pl->pts_total, 1))) != ISDF_OK) return st;
  ISDF_HIP_TRY(hipMemsetAsync(f->cflag.p, 1, pl->pts_total, s));
  bool any_given = false;
  for (int d = 0; d < nd; ++d) any_given |= mode[d] == 2;
  if (any_given) {
    std::vector<int32_t> hc(std::max<int64_t>(pl->pts_total, 1), 0);
    std::vector<uint8_t> hf(std::max<int64_t>(pl->pts_total, 1), 1);
    int64_t o = 0;
    for (int d = 0; d < nd; ++d) {
      const int64_t n = ncand_in[d];
      const int64_t np = (int64_t)hp.domains[d].points.size();
      if (mode[d] == 2) {
        if (n <= 0 || n > np) {
          set_error("isdf_fit_with_candidates: candidate count outside 1..points");
          return ISDF_E_ARG;
        }
        for (int64_t i = 0; i < np; ++i) hf[pl->pts_off[d] + i] = 0;
        for (int64_t i = 0; i < n; ++i) {
          const int64_t v = cand_in[o + i];
          if (v < 0 || v >= np || (i > 0 && v <= cand_in[o + i - 1])) {
            set_error("isdf_fit_with_candidates: candidates must be ascending local indices");
            return ISDF_E_ARG;
          }
          hc[pl->pts_off[d] + i] = (int32_t)v;
          hf[pl->pts_off[d] + v] = 1;
        }
        cx.nc_host[d] = (int32_t)n;
      }
      o += std::max<int64_t>(n, 0);
    }
    if ((st = copy_in(cx.cand.p, hc.data(), sizeof(int32_t) * hc.size())) != ISDF_OK) return st;
    if ((st = copy_in(f->cflag.p, hf.data(), hf.size())) != ISDF_OK) return st;
  }
  if (cx.any_learned) {
    if ((st = cx.feats.alloc(sizeof(float) * 16 * std::max<int64_t>(pl->pts_total, 1))) != ISDF_OK) return st;
    if ((st = cx.z.alloc(sizeof(float) * std::max<int64_t>(pl->pts_total, 1))) != ISDF_OK) return st;
  }
  return ISDF_OK;
}

isdf_status sel_group(isdf_plan_s* pl, isdf_fit_s* f, SelCtx& cx, const std::vector<int>& mode, int g0, int g1,
                      const double* phi_base) {
  HostPlan& hp = pl->hp;
  hipStream_t s = pl->stream;
  isdf_status st;
  if (cx.pinned) return ISDF_OK;
  // full-mode domains
  std::vector<SelSpec> full;
  std::vector<int> full_id;
  std::vector<int64_t> full_poff;
  for (int d = g0; d < g1; ++d) {
    if (mode[d] != 0 || hp.domains[d].n_mu == 0) continue;  // no points requested: count stays 0
    full.push_back(full_spec(pl, d));
    full_id.push_back(d);
    full_poff.push_back(f->piv_off[d]);
  }
  std::vector<int> cnt;
  std::vector<double> dl;
  if (!full.empty()) {
    if ((st = select_points(pl, full, phi_base, f->dwork.as<double>(), f->piv.as<int32_t>(), full_poff, cnt,
                            dl)) != ISDF_OK)
      return st;
    for (size_t i = 0; i < full.size(); ++i) {
      f->count[full_id[i]] = cnt[i];
      f->dlast[full_id[i]] = dl[i];
      f->ncand[full_id[i]] = full[i].pts;
    }
  }
  // candidate-mode domains
  std::vector<int> cid;
  bool learned = false;
  for (int d = g0; d < g1; ++d)
    if (mode[d] == 1 || mode[d] == 2) {
      cid.push_back(d);
      learned |= mode[d] == 1;
    }
  if (cid.empty()) {
    ISDF_HIP_TRY(hipStreamSynchronize(s));
    return ISDF_OK;
  }
  int32_t* cand = cx.cand.as<int32_t>();
  if (learned) {
    const int64_t p0 = pl->pts_off[g0], p1 = g1 < (int)hp.domains.size() ? pl->pts_off[g1] : pl->pts_total;
    if ((st = compute_features(pl, f, cx.feats.as<float>(), g0, g1)) != ISDF_OK) return st;
    if ((st = launch_mlp_forward(s, pl->d_mlp_w.as<float>(), cx.feats.as<float>() + 16 * p0, p1 - p0,
                                 cx.z.as<float>() + p0)) != ISDF_OK)
      return st;
    std::vector<CandDomain> cd;
    std::vector<int> cd_id;
    for (int d : cid) {
      if (mode[d] != 1) continue;
      CandDomain c{};
      c.pts_off = pl->pts_off[d];
      c.cand_off = pl->pts_off[d];
      c.pts = (int)hp.domains[d].points.size();
      c.keep = std::max(hp.domains[d].n_mu,
                        (int)std::ceil(pl->opts.mlp_keep * (double)hp.domains[d].n_mu));
      c.keep = std::max(1, std::min(c.keep, c.pts));
      cd.push_back(c);
      cd_id.push_back(d);
    }
    DevBuf d_cd, d_nc;
    if ((st = upload(d_cd, cd)) != ISDF_OK) return st;
    if ((st = d_nc.alloc(sizeof(int32_t) * cd.size())) != ISDF_OK) return st;
    const double pc = std::min(std::max(pl->opts.mlp_cutoff, 1e-30), 1.0 - 1e-7);
    const float zcut = (float)std::log(pc / (1.0 - pc));  // logit of the score cutoff
    if ((st = launch_topk_compact(s, d_cd.as<CandDomain>(), (int)cd.size(), cx.z.as<float>(), zcut, cand,
                                  d_nc.as<int32_t>(), f->cflag.as<uint8_t>())) != ISDF_OK)
      return st;
    std::vector<int32_t> nc(cd.size());
    ISDF_HIP_TRY(hipMemcpyAsync(nc.data(), d_nc.p, sizeof(int32_t) * nc.size(), hipMemcpyDeviceToHost, s));
    ISDF_HIP_TRY(hipStreamSynchronize(s));
    for (size_t i = 0; i < cd.size(); ++i) cx.nc_host[cd_id[i]] = nc[i];
  }
  // compact candidate rows, select on them, map pivots back
  std::vector<GatherRows> gr;
  std::vector<SelSpec> cs;
  std::vector<int64_t> cpoff;
  int64_t phic = 0, dgc = 0, pvc = 0;
  int max_nc = 0;
  for (int d : cid) {
    const HostDomain& D = hp.domains[d];
    GatherRows g{};
    g.phi_off = pl->phi_off[d];
    g.diag_off = pl->pts_off[d];
    g.phic_off = phic;
    g.diagc_off = dgc;
    g.cand_off = pl->pts_off[d];
    g.pts = (int)D.points.size();
    g.nG = (int)D.funcs.size();
    g.nc = cx.nc_host[d];
    gr.push_back(g);
    cs.push_back(SelSpec{D.level, g.nc, g.nG, D.nL, std::min(D.n_mu, g.nc), phic, dgc, lone_on_level(hp, d)});
    cpoff.push_back(pvc);
    phic += (int64_t)g.nc * g.nG;
    dgc += g.nc;
    pvc += D.n_mu;
    max_nc = std::max(max_nc, g.nc);
    f->ncand[d] = g.nc;
  }
  DevBuf d_gr;
  DevBuf &phic_b = cx.phic, &diagc_b = cx.diagc, &pivc = cx.pivc;
  if ((st = upload(d_gr, gr)) != ISDF_OK) return st;
  if ((st = phic_b.reserve(sizeof(double) * std::max<int64_t>(phic, 1))) != ISDF_OK) return st;
  if ((st = diagc_b.reserve(sizeof(double) * std::max<int64_t>(dgc, 1))) != ISDF_OK) return st;
  if ((st = pivc.reserve(sizeof(int32_t) * std::max<int64_t>(pvc, 1))) != ISDF_OK) return st;
  if ((st = launch_gather_rows(s, d_gr.as<GatherRows>(), (int)gr.size(), max_nc, phi_base, f->diag0.as<double>(),
                               cand, phic_b.as<double>(), diagc_b.as<double>())) != ISDF_OK)
    return st;
  if ((st = select_points(pl, cs, phic_b.as<double>(), diagc_b.as<double>(), pivc.as<int32_t>(), cpoff, cnt,
                          dl)) != ISDF_OK)
    return st;
  for (size_t i = 0; i < cid.size(); ++i) {
    const int d = cid[i];
    f->count[d] = cnt[i];
    f->dlast[d] = dl[i];
    if ((st = launch_map_pivots(s, cand, pl->pts_off[d], pivc.as<int32_t>() + cpoff[i],
                                f->piv.as<int32_t>() + f->piv_off[d], cnt[i])) != ISDF_OK)
      return st;
  }
  // Exactness check: residual diagonals never grow, so when every point left
  // out has an initial diagonal below (1 - tie_tol) times the residual of the
  // last pivot, none of them could have entered the tie window of any step
  // and the pivots are those of the full selection.  Learned candidate sets
  // that fail (or stop short of n_mu points) are selected again in full.
  std::vector<JudgeDomain> jd;
  for (int d : cid) jd.push_back(JudgeDomain{pl->pts_off[d], 0, (int)hp.domains[d].points.size(), 0});
  DevBuf d_jd, d_out;
  if ((st = upload(d_jd, jd)) != ISDF_OK) return st;
  if ((st = d_out.alloc(sizeof(double) * jd.size())) != ISDF_OK) return st;
  if ((st = launch_excluded_max(s, d_jd.as<JudgeDomain>(), (int)jd.size(), f->diag0.as<double>(),
                                f->cflag.as<uint8_t>(), d_out.as<double>())) != ISDF_OK)
    return st;
  std::vector<double> ho(jd.size());
  ISDF_HIP_TRY(hipMemcpyAsync(ho.data(), d_out.p, sizeof(double) * ho.size(), hipMemcpyDeviceToHost, s));
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  std::vector<SelSpec> redo;
  std::vector<int> redo_id;
  std::vector<int64_t> redo_poff;
  for (size_t i = 0; i < cid.size(); ++i) {
    const int d = cid[i];
    f->dfinal[d] = ho[i];
    const bool exact = ho[i] < (1.0 - hp.tie_tol) * f->dlast[d];
    const bool short_of_points = f->count[d] < hp.domains[d].n_mu;
    if (exact && !short_of_points) continue;
    f->fallback[d] = 1;
    if (mode[d] != 1) continue;  // caller-given candidates: report only
    redo.push_back(full_spec(pl, d));
    redo_id.push_back(d);
    redo_poff.push_back(f->piv_off[d]);
  }
  if (!redo.empty()) {
    // dwork still holds the untouched initial diagonals of these domains
    if ((st = select_points(pl, redo, phi_base, f->dwork.as<double>(), f->piv.as<int32_t>(), redo_poff, cnt,
                            dl)) != ISDF_OK)
      return st;
    for (size_t i = 0; i < redo.size(); ++i) {
      f->count[redo_id[i]] = cnt[i];
      f->dlast[redo_id[i]] = dl[i];
      f->ncand[redo_id[i]] = redo[i].pts;
    }
  }
  ISDF_HIP_TRY(hipStreamSynchronize(s));
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
  // G C^T = Theta, then F C = G, by recursive halving of the column range:
  // each half's update from the other is one wide GEMM, and 64-column
  // diagonal blocks are applied through their inverses.
  ISDF_HIP_TRY(hipMemcpyAsync(t, theta, sizeof(double) * pts * n, hipMemcpyDeviceToDevice, s));
  auto split = [&](int a, int b) { return a + std::max(1, (b - a) / nb / 2) * nb; };  // b - a > nb
  // G[:, a:b] from T[:, a:b]; T[:, b:] is updated by the caller
  std::function<isdf_status(int, int)> fwd = [&](int a, int b) -> isdf_status {
    isdf_status r;
    if (b - a <= nb) {
      GemmProblem p{};
      p.A = t + (int64_t)a * pts; p.lda = pts;
      p.B = iv + (int64_t)(a / nb) * nb * nb; p.ldb = nb; p.transB = 1;
      p.C = g + (int64_t)a * pts; p.ldc = pts;
      p.M = (int)pts; p.N = b - a; p.K = b - a;
      p.alpha = 1.0; p.beta = 0.0;
      return gemm_prof(pl, ISDF_K_GEMM_FIT, EPI_AXPBY, p);
    }
    const int m = split(a, b);
    if ((r = fwd(a, m)) != ISDF_OK) return r;
    GemmProblem p{};  // T[:, m:b] -= G[:, a:m] C[m:b, a:m]^T
    p.A = g + (int64_t)a * pts; p.lda = pts;
    p.B = cf + m + (int64_t)a * n; p.ldb = n; p.transB = 1;
    p.C = t + (int64_t)m * pts; p.ldc = pts;
    p.M = (int)pts; p.N = b - m; p.K = m - a;
    p.alpha = -1.0; p.beta = 1.0;
    if ((r = gemm_prof(pl, ISDF_K_GEMM_FIT, EPI_AXPBY, p)) != ISDF_OK) return r;
    return fwd(m, b);
  };
  // F[:, a:b] from G[:, a:b]; G[:, :a] is updated by the caller
  std::function<isdf_status(int, int)> bwd = [&](int a, int b) -> isdf_status {
    isdf_status r;
    if (b - a <= nb) {
      GemmProblem p{};
      p.A = g + (int64_t)a * pts; p.lda = pts;
      p.B = iv + (int64_t)(a / nb) * nb * nb; p.ldb = nb;
      p.C = F + (int64_t)a * pts; p.ldc = pts;
      p.M = (int)pts; p.N = b - a; p.K = b - a;
      p.alpha = 1.0; p.beta = 0.0;
      return gemm_prof(pl, ISDF_K_GEMM_FIT, EPI_AXPBY, p);
    }
    const int m = split(a, b);
    if ((r = bwd(m, b)) != ISDF_OK) return r;
    GemmProblem p{};  // G[:, a:m] -= F[:, m:b] C[m:b, a:m]
    p.A = F + (int64_t)m * pts; p.lda = pts;
    p.B = cf + m + (int64_t)a * n; p.ldb = n;
    p.C = g + (int64_t)a * pts; p.ldc = pts;
    p.M = (int)pts; p.N = m - a; p.K = b - m;
    p.alpha = -1.0; p.beta = 1.0;
    if ((r = gemm_prof(pl, ISDF_K_GEMM_FIT, EPI_AXPBY, p)) != ISDF_OK) return r;
    return bwd(a, m);
  };
  if ((st = fwd(0, n)) != ISDF_OK) return st;
  if ((st = bwd(0, n)) != ISDF_OK) return st;
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
// scratch (may be null): a device block the caller no longer needs (the
// streamed basis values); when it is large enough it holds the FP64 W of an
// FP32-stored metric, the potential slabs and the FFT work buffers, so that
// none of them is allocated.
isdf_status run_coulomb(isdf_plan_s* pl, isdf_fit_s* f, DevBuf* scratch = nullptr) {
  HostPlan& hp = pl->hp;
  hipStream_t s = pl->stream;
  const int nd = (int)hp.domains.size();
  const int64_t nmu = f->nmu;
  const int L = hp.n_levels;
  isdf_status st;
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
  // (free memory plus the plan's cached blocks, so that repeated fits size
  // their buffers alike and take them back from the cache)
  double avail = 0.0;
  if ((st = plan_available(pl, AVAIL_COULOMB, &avail)) != ISDF_OK) return st;
  const double v_budget = std::min(24e9, std::max(2e9, 0.45 * avail));
  const double z_budget = std::min(4e9, std::max(2.5e8, 0.05 * avail));
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
    if (pl->opts.w_batch > 0) w = std::min<int64_t>(w, std::max(2, pl->opts.w_batch));
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
  if (pl->opts.w_batch > 0) fft_pairs = std::min<int64_t>(fft_pairs, std::max(1, pl->opts.w_batch / 2));
  // W (FP64), V, zf, zc: carved from the scratch block when it holds them
  const bool w_transient = pl->opts.w_storage == ISDF_W_F32;
  auto a256 = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t b_w = sizeof(double) * nmu * nmu, b_z = sizeof(double) * 2 * ngz_max * fft_pairs,
               b_v = sizeof(double) * std::max<int64_t>(vmax, 1);
  const size_t need = (w_transient ? a256(b_w) : 0) + a256(b_v) + 2 * a256(b_z);
  double *Wd = nullptr, *Vd = nullptr, *zfd = nullptr, *zcd = nullptr;
  if (scratch && scratch->p && scratch->cap >= need) {
    char* q = static_cast<char*>(scratch->p);
    if (w_transient) {
      Wd = reinterpret_cast<double*>(q);
      q += a256(b_w);
    }
    Vd = reinterpret_cast<double*>(q);
    q += a256(b_v);
    zfd = reinterpret_cast<double*>(q);
    q += a256(b_z);
    zcd = reinterpret_cast<double*>(q);
  } else {
    if ((st = zf.alloc(b_z)) != ISDF_OK) return st;
    if ((st = zc.alloc(b_z)) != ISDF_OK) return st;
    if ((st = V.alloc(b_v)) != ISDF_OK) return st;
    zfd = zf.as<double>();
    zcd = zc.as<double>();
    Vd = V.as<double>();
  }
  if (!Wd) {
    if ((st = f->W.alloc(b_w)) != ISDF_OK) return st;
    Wd = f->W.as<double>();
  }
  if ((st = launch_fill(s, Wd, nmu * nmu, 0.0)) != ISDF_OK) return st;
  std::vector<GemmProblem> probs;
  struct GemmLaunch {
    int level, off, cnt, tiles, shape;
    double bytes, flops;
  };
  // per chunk: one grouped launch per (row level, tile shape)
  std::vector<std::vector<GemmLaunch>> glaunch(chunks.size());
  for (size_t ci = 0; ci < chunks.size(); ++ci) {
    const Chunk& ch = chunks[ci];
    int64_t voff = 0;
    for (int l = 0; l <= ch.lp; ++l) {
      std::vector<GemmProblem> lp_probs;
      const double dV = hp.volume / (double)level_ng(hp, l);
      for (int d = 0; d < nd; ++d) {
        // all-point domains (F = I) take their rows of the potentials as they are
        if (hp.domains[d].level != l || f->count[d] == 0 || f->mode[d] == 3) continue;
        const HostDomain& D = hp.domains[d];
        // same level: only the columns from the domain's own xi on (each
        // pair of different domains once, mirrored by the symmetrisation)
        const int64_t cs = l == ch.lp ? std::max<int64_t>(ch.c0, f->xoff[d]) : ch.c0;
        if (cs >= ch.c1) continue;
        GemmProblem p{};
        p.A = f->F.as<double>() + f->th_off[d];
        p.lda = (int64_t)D.points.size();
        p.transA = 1;
        p.B = Vd + voff + (cs - ch.c0) * level_ng(hp, l);
        p.ldb = level_ng(hp, l);
        p.bidx = ((int64_t)D.points.size() == level_ng(hp, l) && D.atom < 0)
                     ? nullptr
                     : pl->d_points.as<int32_t>() + pl->pts_off[d];
        p.C = Wd + f->xoff[d] + cs * nmu;
        p.ldc = nmu;
        p.M = f->count[d];
        p.N = (int)(ch.c1 - cs);
        p.K = (int)D.points.size();
        p.alpha = dV;
        p.beta = 0.0;
        lp_probs.push_back(p);
      }
      // window rows (gathered potentials): tiles 128 columns wide, and tall
      // enough for the whole row count up to 128 (48, 64, 80 or 128 rows), so
      // that the gathered rows of V are read once per column tile (they
      // dominate the traffic)
      auto metric_shape = [](const GemmProblem& p) {
        if (!p.bidx) return gemm_default_shape(EPI_AXPBY, p.M, p.N, p.K);
        return p.M <= 48 ? 13 : p.M <= 64 ? 4 : p.M <= 80 ? 12 : p.M <= 128 ? 2
                                                               : gemm_default_shape(EPI_AXPBY, p.M, p.N, p.K);
      };
      for (int shape = 0; shape < GEMM_NSHAPE; ++shape) {
        GemmLaunch gl{l, (int)probs.size(), 0, 0, shape, 0.0, 0.0};
        for (GemmProblem p : lp_probs) {
          if (metric_shape(p) != shape) continue;
          p.tile_start = gl.tiles;
          gl.tiles += gemm_tiles(p.M, p.N, shape);
          gl.bytes += gemm_bytes(p);
          gl.flops += gemm_flops(p);
          probs.push_back(p);
        }
        gl.cnt = (int)probs.size() - gl.off;
        if (gl.cnt > 0) glaunch[ci].push_back(gl);
      }
      voff += level_ng(hp, l) * (ch.c1 - ch.c0);
    }
  }
  if ((st = upload(d_probs, probs)) != ISDF_OK) return st;
  // every universal point a fitting function: W_Uw(R, xi) = dV_0 V_xi(R)
  // straight from the level-0 potentials (F_U = I)
  const int64_t ng0 = level_ng(hp, 0);
  if (f->all_points) {
    if ((st = f->WUw.alloc(sizeof(double) * ng0 * std::max<int64_t>(nmu, 1))) != ISDF_OK) return st;
  }
  // mixed precision for the universal rows (the level-0 row block has one
  // domain whose points are the whole grid, so no row gather is involved)
  const bool w_mixed = mixed_on(pl, ISDF_MIX_W) && nd > 0 && hp.domains[0].atom < 0 &&
                       hp.domains[0].level == 0 && f->count[0] > 0 && f->mode[0] != 3;
  Planes Fp0, Vp0;
  if (w_mixed) {
    const int64_t pts0 = (int64_t)hp.domains[0].points.size();
    if ((st = make_planes(s, mixed_splits(pl), f->F.as<double>() + f->th_off[0], pts0, 1, nullptr,
                          f->count[0], (int)pts0, Fp0)) != ISDF_OK)
      return st;
  }
  // the scatter slot of a column is its position within its FFT batch
  for (auto& ch : chunks) {
    const int64_t pairs_max = std::max<int64_t>(1, (ngz_max * fft_pairs) / level_ng(hp, ch.lp));
    const int64_t bw = std::max<int64_t>(2, 2 * pairs_max);
    for (int64_t b0 = ch.c0; b0 < ch.c1; b0 += bw)
      for (int64_t c = b0; c < std::min(b0 + bw, ch.c1); ++c) scat[c].slot = (int)(c - b0);
  }
  if ((st = upload(d_scat, scat)) != ISDF_OK) return st;
  // pruned forward transforms: one descriptor per column, pairs per batch
  std::vector<FwdCol> fcols(nmu);
  for (int64_t c = 0; c < nmu; ++c) {
    const int d = col_dom[c];
    const std::array<int32_t, 7>& b = pl->box[d];
    fcols[c].src = scat[c].src;
    fcols[c].map = b[6] < 0 ? nullptr : pl->d_boxmap.as<int32_t>() + b[6];
    for (int i = 0; i < 6; ++i) fcols[c].box[i] = b[i];
  }
  auto union_box = [&](const int32_t* a, const int32_t* b, const int* g, int32_t* out) {
    for (int ax = 0; ax < 3; ++ax) {  // cyclic interval holding both (whole axis if unclear)
      const int n = g[ax];
      const int a0 = a[ax], ae = a[3 + ax], b0 = b[ax], be = b[3 + ax];
      int best0 = 0, bestE = n;
      for (int cand : {a0, b0}) {
        const int ea = (a0 - cand + n) % n + ae, eb = (b0 - cand + n) % n + be;
        const int e = std::max(ea, eb);
        if (e < bestE) {
          best0 = cand;
          bestE = e;
        }
      }
      out[ax] = best0;
      out[3 + ax] = std::min(bestE, n);
    }
  };
  std::vector<FwdPair> fpairs;
  std::vector<int64_t> fpair_off;  // per (chunk, batch) in loop order
  for (auto& ch : chunks) {
    const int64_t pairs_max = std::max<int64_t>(1, (ngz_max * fft_pairs) / level_ng(hp, ch.lp));
    const int64_t bw = std::max<int64_t>(2, 2 * pairs_max);
    for (int64_t b0 = ch.c0; b0 < ch.c1; b0 += bw) {
      fpair_off.push_back((int64_t)fpairs.size());
      const int64_t ce = std::min(b0 + bw, ch.c1);
      for (int64_t c = b0; c < ce; c += 2) {
        FwdPair P{};
        P.c0 = (int32_t)c;
        P.c1 = c + 1 < ce ? (int32_t)(c + 1) : -1;
        if (P.c1 < 0 || col_dom[c] == col_dom[c + 1])
          std::copy(fcols[c].box, fcols[c].box + 6, P.box);
        else
          union_box(fcols[c].box, fcols[c + 1].box, hp.grid[ch.lp], P.box);
        fpairs.push_back(P);
      }
    }
  }
  DevBuf d_fcols, d_fpairs;
  if ((st = upload(d_fcols, fcols)) != ISDF_OK) return st;
  if ((st = upload(d_fpairs, fpairs)) != ISDF_OK) return st;
  size_t batch_no = 0;
  for (size_t ci = 0; ci < chunks.size(); ++ci) {
    const Chunk& ch = chunks[ci];
    const int lp = ch.lp;
    const int64_t ngp = level_ng(hp, lp);
    const int64_t pairs_max = std::max<int64_t>(1, (ngz_max * fft_pairs) / ngp);
    const int64_t bw = std::max<int64_t>(2, 2 * pairs_max);
    for (int64_t b0 = ch.c0; b0 < ch.c1; b0 += bw) {
      const int ncols = (int)std::min<int64_t>(bw, ch.c1 - b0);
      const int npairs = (ncols + 1) / 2;
      const int64_t poff = fpair_off[batch_no++];
      if (fft_forward_pruned_supported(hp.grid[lp])) {
        int max_yz = 0, max_z = 0;
        double touched[3] = {0.0, 0.0, 0.0};  // complex points read + written per pass
        const int* g = hp.grid[lp];
        for (int b = 0; b < npairs; ++b) {
          const FwdPair& P = fpairs[poff + b];
          max_yz = std::max(max_yz, P.box[4] * P.box[5]);
          max_z = std::max(max_z, P.box[5]);
          touched[0] += 2.0 * g[0] * P.box[4] * P.box[5];
          touched[1] += 2.0 * g[0] * g[1] * P.box[5];
          touched[2] += (double)g[0] * g[1] * (P.box[5] + g[2]);
        }
        FftEvents fe(pl);
        if ((st = fft_forward_pruned(s, zfd, d_fpairs.as<FwdPair>() + poff,
                                     d_fcols.as<FwdCol>(), npairs, hp.grid[lp], max_yz, max_z, fe.ev())) !=
            ISDF_OK)
          return st;
        fe.commit({16.0 * touched[0], 16.0 * touched[1], 16.0 * touched[2]});
      } else {
        int max_n = 0;
        for (int64_t c = b0; c < b0 + ncols; ++c) max_n = std::max(max_n, scat[c].n);
        if ((st = launch_fill(s, zfd, 2 * ngp * npairs, 0.0)) != ISDF_OK) return st;
        if ((st = launch_scatter_cols(s, d_scat.as<ScatterCol>() + b0, ncols, max_n, zfd,
                                      ngp)) != ISDF_OK)
          return st;
        if ((st = fft_prof(pl, zfd, npairs, hp.grid[lp], -1)) != ISDF_OK) return st;
      }
      int64_t voff = 0;
      for (int l = 0; l <= lp; ++l) {
        const int64_t ng = level_ng(hp, l);
        double* vout = Vd + voff + (b0 - ch.c0) * ng;
        bool fused = false;
        {  // Poisson step, inverse transform and planar split in three passes
          FftEvents fe(pl);
          if ((st = fft_poisson_inverse(s, zfd, hp.grid[lp], zcd, hp.grid[l],
                                        npairs, pl->recip, vout, ncols, &fused, fe.ev())) != ISDF_OK)
            return st;
          const double pass_bytes = 32.0 * (double)ng * npairs;
          if (fused) fe.commit({pass_bytes, pass_bytes, pass_bytes});
        }
        if (!fused) {
          if ((st = launch_poisson_restrict(s, zfd, hp.grid[lp], zcd,
                                            hp.grid[l], npairs, pl->recip)) != ISDF_OK)
            return st;
          if ((st = fft_prof(pl, zcd, npairs, hp.grid[l], +1)) != ISDF_OK) return st;
          if ((st = launch_split_planar(s, zcd, ng, ncols, vout)) != ISDF_OK) return st;
        }
        voff += ng * (ch.c1 - ch.c0);
      }
    }
    if (f->all_points) {  // level-0 potentials of this chunk sit first in V
      if ((st = launch_scale_copy(s, Vd, f->WUw.as<double>() + ch.c0 * ng0, ng0 * (ch.c1 - ch.c0),
                                  hp.volume / (double)ng0)) != ISDF_OK)
        return st;
    }
    {  // rows of all-point domains: W(xi_i, xi') = dV V_xi'(R_i)
      int64_t voff = 0;
      for (int l = 0; l <= lp; ++l) {
        const int64_t ng = level_ng(hp, l);
        for (int d = 0; d < nd; ++d) {
          if (hp.domains[d].level != l || f->count[d] == 0 || f->mode[d] != 3) continue;
          const HostDomain& D = hp.domains[d];
          const bool whole = (int64_t)D.points.size() == ng && D.atom < 0;
          if ((st = launch_scale_rows(s, Vd + voff, ng,
                                      whole ? nullptr : pl->d_points.as<int32_t>() + pl->pts_off[d],
                                      (int)D.points.size(), (int)(ch.c1 - ch.c0), hp.volume / (double)ng,
                                      Wd + f->xoff[d] + ch.c0 * nmu, nmu)) != ISDF_OK)
            return st;
        }
        voff += ng * (ch.c1 - ch.c0);
      }
    }
    for (const GemmLaunch& gl : glaunch[ci]) {
      if (gl.level == 0 && w_mixed) {
        const int w = (int)(ch.c1 - ch.c0);
        if ((st = make_planes(s, mixed_splits(pl), Vd, ng0, 1, nullptr, w, (int)ng0, Vp0)) !=
            ISDF_OK)
          return st;
        MixedProblem mp = mixed_problem(Fp0, Vp0, Wd + f->xoff[0] + ch.c0 * nmu, nmu,
                                        f->count[0], w, (int)ng0, hp.volume / (double)ng0, 0.0,
                                        nullptr, 0);
        if ((st = mixed_prof(pl, ISDF_K_GEMM_METRIC, EPI_AXPBY, mp)) != ISDF_OK) return st;
        continue;
      }
      if (gl.cnt == 1) {  // a lone problem (the universal rows) takes the tuned shape
        if ((st = gemm_prof(pl, ISDF_K_GEMM_METRIC, EPI_AXPBY, probs[gl.off])) != ISDF_OK) return st;
        continue;
      }
      ProfScope ps(pl, ISDF_K_GEMM_METRIC, gl.bytes, gl.flops);
      // every window problem reads F transposed (A k-fastest) and V untransposed
      if ((st = gemm_f64_grouped(s, EPI_AXPBY, d_probs.as<GemmProblem>() + gl.off, gl.cnt,
                                 gl.tiles, family_tag(ISDF_K_GEMM_METRIC), gl.shape, 1, 0)) != ISDF_OK)
        return st;
    }
  }
  // level and domain of each xi, then symmetrise
  std::vector<int8_t> lev(nmu);
  std::vector<int32_t> xdom(nmu);
  for (int d = 0; d < nd; ++d)
    for (int j = 0; j < f->count[d]; ++j) {
      lev[f->xoff[d] + j] = (int8_t)hp.domains[d].level;
      xdom[f->xoff[d] + j] = d;
    }
  DevBuf d_xdom;
  if ((st = upload(f->lev, lev)) != ISDF_OK) return st;
  if ((st = upload(d_xdom, xdom)) != ISDF_OK) return st;
  if ((st = launch_symmetrize_w(s, Wd, nmu, f->lev.as<int8_t>(), d_xdom.as<int32_t>())) !=
      ISDF_OK)
    return st;
  if (pl->opts.w_storage == ISDF_W_F32) {  // keep W in FP32 from here on
    if ((st = f->W32.alloc(sizeof(float) * std::max<int64_t>(nmu * nmu, 1))) != ISDF_OK) return st;
    if ((st = launch_narrow(s, Wd, f->W32.as<float>(), nmu * nmu)) != ISDF_OK) return st;
    ISDF_HIP_TRY(hipStreamSynchronize(s));
    f->W.release();  // (nothing held when W sat in the scratch block)
    f->w32 = true;
  }
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  return ISDF_OK;
}

// Stage clock of a fit: event pairs per stage segment, summed after the
// final synchronisation (a streamed fit visits the stages once per group).
struct StageClock {
  std::vector<std::pair<int, std::array<hipEvent_t, 2>>> segs;
  hipStream_t s = nullptr;
  int open_stage = -1;
  ~StageClock() {
    for (auto& x : segs)
      for (hipEvent_t e : x.second) (void)hipEventDestroy(e);
  }
  isdf_status begin(int stage) {
    std::array<hipEvent_t, 2> e{};
    ISDF_HIP_TRY(hipEventCreate(&e[0]));
    ISDF_HIP_TRY(hipEventCreate(&e[1]));
    segs.push_back({stage, e});
    ISDF_HIP_TRY(hipEventRecord(e[0], s));
    open_stage = stage;
    return ISDF_OK;
  }
  isdf_status end() {
    ISDF_HIP_TRY(hipEventRecord(segs.back().second[1], s));
    open_stage = -1;
    return ISDF_OK;
  }
  isdf_status next(int stage) {
    isdf_status st;
    if (open_stage >= 0 && (st = end()) != ISDF_OK) return st;
    return begin(stage);
  }
  isdf_status collect(double* ms_out, int n) {
    for (int i = 0; i < n; ++i) ms_out[i] = 0.0;
    for (auto& x : segs) {
      float ms = 0.f;
      ISDF_HIP_TRY(hipEventElapsedTime(&ms, x.second[0], x.second[1]));
      if (x.first < n) ms_out[x.first] += ms;
    }
    return ISDF_OK;
  }
};

// Consecutive domain groups whose basis values fit the budget (a domain
// larger than the budget is a group of its own).
std::vector<std::pair<int, int>> phi_groups(isdf_plan_s* pl, double budget_bytes) {
  const int nd = (int)pl->hp.domains.size();
  std::vector<std::pair<int, int>> g;
  int g0 = 0;
  double acc = 0.0;
  for (int d = 0; d < nd; ++d) {
    const double b = 8.0 * (double)pl->hp.domains[d].points.size() * pl->hp.domains[d].funcs.size();
    if (d > g0 && acc + b > budget_bytes) {
      g.push_back({g0, d});
      g0 = d;
      acc = 0.0;
    }
    acc += b;
  }
  g.push_back({g0, nd});
  return g;
}

isdf_status do_fit(isdf_plan_s* pl, const int64_t* pinned, const int64_t* cand_in,
                   const int64_t* ncand_in, const std::vector<int>* force_full, isdf_fit_t* out) {
  if (!pl || !out) {
    set_error("isdf_fit: null argument");
    return ISDF_E_ARG;
  }
  MemScope mscope(pl->mem);
  isdf_status st;
  if ((st = upload_plan(pl)) != ISDF_OK) return st;
  HostPlan& hp = pl->hp;
  hipStream_t s = pl->stream;
  std::unique_ptr<isdf_fit_s> f(new isdf_fit_s());
  f->plan = pl;
  const int nd = (int)hp.domains.size();
  StageClock clk;
  clk.s = s;
  // domain groups by the basis-value budget
  double budget = 0.0;
  if (pl->opts.phi_budget_mb > 0) {
    budget = 1048576.0 * pl->opts.phi_budget_mb;
  } else {
    double avail = 0.0;
    if ((st = plan_available(pl, AVAIL_PHI, &avail)) != ISDF_OK) return st;
    budget = 0.4 * avail;
  }
  const std::vector<std::pair<int, int>> groups =
      8.0 * (double)pl->phi_total > budget ? phi_groups(pl, budget) : std::vector<std::pair<int, int>>{{0, nd}};
  const bool streamed = groups.size() > 1;
  int64_t phi_cap = pl->phi_total;
  if (streamed) {
    phi_cap = 0;
    for (auto& g : groups) {
      const int64_t e = (g.second < nd ? pl->phi_off[g.second] : pl->phi_total) - pl->phi_off[g.first];
      phi_cap = std::max(phi_cap, e);
    }
  }
  f->phi_streamed = streamed;
  auto grp_pts = [&](const std::pair<int, int>& g, int64_t* p0) {
    *p0 = pl->pts_off[g.first];
    return (g.second < nd ? pl->pts_off[g.second] : pl->pts_total) - *p0;
  };
  // basis values (and diagonal, aux) of one group; phi_base + phi_off[d]
  // addresses domain d of the group
  auto basis = [&](const std::pair<int, int>& g, double** phi_base) -> isdf_status {
    *phi_base = f->phi.as<double>() - (streamed ? pl->phi_off[g.first] : 0);
    const int t0 = pl->tile_off[g.first], t1 = pl->tile_off[g.second];
    int64_t p0;
    const int64_t np = grp_pts(g, &p0);
    const int64_t e = (g.second < nd ? pl->phi_off[g.second] : pl->phi_total) - pl->phi_off[g.first];
    ProfScope ps_basis(pl, ISDF_K_BASIS, 8.0 * ((double)e + np), 0.0);
    return launch_basis_eval(s, pl->lat, pl->d_shells.as<ShellDev>(), pl->d_img.as<double>(),
                             pl->d_colshells.as<ColShell>(), pl->d_doms.as<DomainDev>(), pl->d_points.as<int32_t>(),
                             pl->d_tiles.as<BasisTile>() + t0, t1 - t0, *phi_base, f->diag0.as<double>(),
                             f->aux.as<double>());
  };
  // 1-2. basis values, then selection, per group
  if ((st = f->phi.alloc(sizeof(double) * std::max<int64_t>(phi_cap, 1))) != ISDF_OK) return st;
  if ((st = f->diag0.alloc(sizeof(double) * pl->pts_total)) != ISDF_OK) return st;
  if ((st = f->dwork.alloc(sizeof(double) * pl->pts_total)) != ISDF_OK) return st;
  if ((st = f->aux.alloc(sizeof(double) * 4 * pl->pts_total)) != ISDF_OK) return st;
  f->mode.assign(nd, 0);
  f->all_points = pl->opts.universal_all_points != 0;
  for (int d = 0; d < nd; ++d) {
    const int pts = (int)hp.domains[d].points.size();
    if (hp.domains[d].n_mu == 0) continue;  // nothing to select
    if (!pinned && hp.n_mu_ratio > 0 && hp.domains[d].n_mu >= pts) {
      f->mode[d] = 3;  // count-driven and capped at the point count: every point, F = I
    } else if (cand_in) {
      f->mode[d] = 2;
    } else if (pl->opts.selector == ISDF_SEL_MLP && !(force_full && (*force_full)[d])) {
      const int keep = (int)std::ceil(pl->opts.mlp_keep * (double)hp.domains[d].n_mu);
      f->mode[d] = keep < pts ? 1 : 0;
    }
  }
  SelCtx cx;
  if ((st = sel_setup(pl, f.get(), cx, pinned, f->mode, cand_in, ncand_in)) != ISDF_OK) return st;
  for (const auto& g : groups) {
    double* phi_base = nullptr;
    if ((st = clk.next(0)) != ISDF_OK) return st;
    if ((st = basis(g, &phi_base)) != ISDF_OK) return st;
    int64_t p0;
    const int64_t np = grp_pts(g, &p0);
    ISDF_HIP_TRY(hipMemcpyAsync(f->dwork.as<double>() + p0, f->diag0.as<double>() + p0, sizeof(double) * np,
                                hipMemcpyDeviceToDevice, s));
    if ((st = clk.next(1)) != ISDF_OK) return st;
    if ((st = sel_group(pl, f.get(), cx, f->mode, g.first, g.second, phi_base)) != ISDF_OK) return st;
  }
  if ((st = clk.end()) != ISDF_OK) return st;
  for (DevBuf* b : {&cx.cand, &cx.feats, &cx.z, &cx.phic, &cx.diagc, &cx.pivc}) b->release();  // no longer needed
  bool rank_short = false;
  f->xoff.assign(nd, 0);
  int64_t nmu = 0;
  for (int d = 0; d < nd; ++d) {
    f->xoff[d] = nmu;
    nmu += f->count[d];
    if (f->count[d] < hp.domains[d].n_mu) rank_short = true;
  }
  f->nmu = nmu;
  // 3-5 per group: gather X, Theta, fitting functions
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
  }
  DevBuf d_gd;
  if ((st = upload(d_gd, gd)) != ISDF_OK) return st;
  if ((st = f->xrows.alloc(sizeof(double) * std::max<int64_t>(xr, 1))) != ISDF_OK) return st;
  if ((st = f->theta.alloc(sizeof(double) * std::max<int64_t>(th, 1))) != ISDF_OK) return st;
  if ((st = f->F.alloc(sizeof(double) * std::max<int64_t>(th, 1))) != ISDF_OK) return st;
  DevBuf spd;
  if ((st = spd.alloc(sizeof(int32_t))) != ISDF_OK) return st;
  ISDF_HIP_TRY(hipMemsetAsync(spd.p, 0, sizeof(int32_t), s));
  // all-point domains: F = I, Theta not formed (zeros)
  for (int d = 0; d < nd; ++d) {
    if (f->mode[d] != 3) continue;
    const int64_t np = gd[d].pts;
    if ((st = launch_fill(s, f->F.as<double>() + f->th_off[d], np * np, 0.0)) != ISDF_OK) return st;
    if ((st = launch_set_diag(s, f->F.as<double>() + f->th_off[d], np, (int)np, 1.0)) != ISDF_OK) return st;
    if ((st = launch_fill(s, f->theta.as<double>() + f->th_off[d], np * np, 0.0)) != ISDF_OK) return st;
  }
  auto fitted = [&](int d) { return f->count[d] > 0 && f->mode[d] != 3; };
  for (const auto& g : groups) {
    const int g0 = g.first, g1 = g.second;
    double* phi_base = f->phi.as<double>();
    if (streamed) {
      if ((st = clk.next(0)) != ISDF_OK) return st;
      if ((st = basis(g, &phi_base)) != ISDF_OK) return st;
    }
    if ((st = clk.next(2)) != ISDF_OK) return st;
    int max_rows = 0;
    for (int d = g0; d < g1; ++d) max_rows = std::max(max_rows, gd[d].count);
    if ((st = launch_gather_x(s, d_gd.as<GatherDom>() + g0, g1 - g0, max_rows, phi_base, f->piv.as<int32_t>(),
                              pl->d_funcs.as<int32_t>(), f->xrows.as<double>(), f->XL.as<double>(),
                              f->XN.as<double>(), nmu)) != ISDF_OK)
      return st;
    // Theta
    if ((st = clk.next(3)) != ISDF_OK) return st;
    std::vector<GemmProblem> probs;
    for (int d = g0; d < g1; ++d) {
      if (!fitted(d)) continue;
      GemmProblem p{};
      p.A = phi_base + pl->phi_off[d];
      p.lda = gd[d].pts;
      p.B = f->xrows.as<double>() + f->xrow_off[d];
      p.ldb = gd[d].nG;
      p.C = f->theta.as<double>() + f->th_off[d];
      p.ldc = gd[d].pts;
      p.M = gd[d].pts;
      p.N = f->count[d];
      p.K = gd[d].nG;
      p.kL = gd[d].nL;
      probs.push_back(p);
    }
    if (mixed_on(pl, ISDF_MIX_THETA)) {
      // per domain: planes of Phi_d and of its pivot rows with the L columns
      // padded to a multiple of 32 so that no k chunk straddles the L/N split
      const int S = mixed_splits(pl);
      Planes Ap, Bp;
      DevBuf kx;
      for (int d = g0; d < g1; ++d) {
        if (!fitted(d)) continue;
        const int nL = gd[d].nL, nG = gd[d].nG, padL = (nL + 31) / 32 * 32;
        std::vector<int32_t> kidx(padL + (nG - nL));
        for (int c = 0; c < padL; ++c) kidx[c] = c < nL ? c : -1;
        for (int c = nL; c < nG; ++c) kidx[padL + c - nL] = c;
        if ((st = upload(kx, kidx)) != ISDF_OK) return st;
        const int Kp = (int)kidx.size();
        if ((st = make_planes(s, S, phi_base + pl->phi_off[d], 1, gd[d].pts, kx.as<int32_t>(), gd[d].pts, Kp,
                              Ap)) != ISDF_OK)
          return st;
        if ((st = make_planes(s, S, f->xrows.as<double>() + f->xrow_off[d], nG, 1, kx.as<int32_t>(), f->count[d],
                              Kp, Bp)) != ISDF_OK)
          return st;
        MixedProblem mp = mixed_problem(Ap, Bp, f->theta.as<double>() + f->th_off[d], gd[d].pts, gd[d].pts,
                                        f->count[d], Kp, 1.0, 0.0, nullptr, 0);
        mp.kL = padL;
        if ((st = mixed_prof(pl, ISDF_K_GEMM_FIT, EPI_THETA, mp)) != ISDF_OK) return st;
        ISDF_HIP_TRY(hipStreamSynchronize(s));  // planes and index are reused
      }
    } else {
      // one grouped launch per tile shape (the universal domain is big, the
      // windows are skinny)
      std::vector<GemmProblem> grouped;
      int tiles[GEMM_NSHAPE] = {}, first[GEMM_NSHAPE] = {}, cnt[GEMM_NSHAPE] = {};
      double by[GEMM_NSHAPE] = {}, fl[GEMM_NSHAPE] = {};
      // windows with 65-80 fitting functions take the 80-column tile (one
      // column tile instead of two), those with 33-48 the 48-column one; the
      // rest the size rule
      auto theta_shape = [](const GemmProblem& p) {
        if (!p.transA && !p.transB && p.N > 64 && p.N <= 80) return 14;
        if (!p.transA && !p.transB && p.N > 32 && p.N <= 48) return 15;
        return gemm_default_shape(EPI_THETA, p.M, p.N, p.K);
      };
      for (int shape = 0; shape < GEMM_NSHAPE; ++shape) {
        first[shape] = (int)grouped.size();
        for (GemmProblem p : probs) {
          if (theta_shape(p) != shape) continue;
          p.tile_start = tiles[shape];
          tiles[shape] += gemm_tiles(p.M, p.N, shape);
          by[shape] += gemm_bytes(p);
          fl[shape] += gemm_flops(p);
          grouped.push_back(p);
        }
        cnt[shape] = (int)grouped.size() - first[shape];
      }
      DevBuf d_probs;
      if ((st = upload(d_probs, grouped)) != ISDF_OK) return st;
      for (int shape = 0; shape < GEMM_NSHAPE; ++shape) {
        if (cnt[shape] == 1) {  // a lone problem (the universal domain) takes the tuned shape
          if ((st = gemm_prof(pl, ISDF_K_GEMM_FIT, EPI_THETA, grouped[first[shape]])) != ISDF_OK) return st;
        } else if (cnt[shape] > 1) {
          ProfScope ps(pl, ISDF_K_GEMM_FIT, by[shape], fl[shape]);
          // every problem: Phi m-fastest (A), pivot rows k-fastest (B)
          if ((st = gemm_f64_grouped(s, EPI_THETA, d_probs.as<GemmProblem>() + first[shape], cnt[shape],
                                     tiles[shape], family_tag(ISDF_K_GEMM_FIT), shape, 0, 0)) != ISDF_OK)
            return st;
        }
      }
      ISDF_HIP_TRY(hipStreamSynchronize(s));  // the problem table is released
    }
    // fitting functions
    if ((st = clk.next(4)) != ISDF_OK) return st;
    std::vector<SmallFitDom> sf;
    std::vector<int32_t> tile_dom;
    int nmax = 0;
    for (int d = g0; d < g1; ++d) {
      const int n = f->count[d];
      if (!fitted(d) || n > 64) continue;
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
                                 f->theta.as<double>(), f->piv.as<int32_t>(), f->F.as<double>(), spd.as<int32_t>(),
                                 nmax)) != ISDF_OK)
        return st;
      ISDF_HIP_TRY(hipStreamSynchronize(s));
    }
    for (int d = g0; d < g1; ++d) {
      const int n = f->count[d];
      if (!fitted(d) || n <= 64) continue;
      if ((st = blocked_fit(pl, f->theta.as<double>() + f->th_off[d], gd[d].pts, n,
                            f->piv.as<int32_t>() + f->piv_off[d], f->F.as<double>() + f->th_off[d],
                            spd.as<int32_t>())) != ISDF_OK)
        return st;
    }
  }
  if ((st = clk.next(2)) != ISDF_OK) return st;
  if ((st = launch_add(s, f->XL.as<double>(), f->XN.as<double>(), f->XG.as<double>(), nmu * N)) != ISDF_OK)
    return st;
  // 6. Coulomb metric (a streamed fit keeps no basis values: their block
  // serves as the metric's work space and is released afterwards)
  if ((st = clk.next(5)) != ISDF_OK) return st;
  if ((st = run_coulomb(pl, f.get(), streamed ? &f->phi : nullptr)) != ISDF_OK) return st;
  if ((st = clk.end()) != ISDF_OK) return st;
  if (streamed) {
    ISDF_HIP_TRY(hipStreamSynchronize(s));
    f->phi.release();
  }
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  prof_collect(pl);
  int32_t spd_flag = 0;
  ISDF_HIP_TRY(hipMemcpy(&spd_flag, spd.p, sizeof(int32_t), hipMemcpyDeviceToHost));
  if ((st = clk.collect(pl->stage_ms, 6)) != ISDF_OK) return st;
  f->groups = (int)groups.size();
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

// ------------------------------------------------------------ tune file
// {"arch": "...", "entries": [{"key": "<class>", "shape": s, "us": [...]}, ...]}
// Only the key/shape pairs are read back; times are for the reader.
isdf_status read_tune_file(const char* path, std::map<std::string, int>& out) {
  std::ifstream f(path);
  if (!f) {
    set_error(std::string("tune file: cannot open ") + path);
    return ISDF_E_ARG;
  }
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t pos = 0;
  int n = 0;
  while ((pos = t.find("\"key\"", pos)) != std::string::npos) {
    const size_t q0 = t.find('"', t.find(':', pos) + 1);
    const size_t q1 = q0 == std::string::npos ? q0 : t.find('"', q0 + 1);
    const size_t sp = q1 == std::string::npos ? q1 : t.find("\"shape\"", q1);
    if (sp == std::string::npos) break;
    const size_t c = t.find(':', sp);
    const int shape = c == std::string::npos ? -1 : std::atoi(t.c_str() + c + 1);
    if (shape < 0 || shape >= GEMM_NSHAPE) {
      set_error(std::string("tune file: bad shape in ") + path);
      return ISDF_E_ARG;
    }
    out[t.substr(q0 + 1, q1 - q0 - 1)] = shape;
    pos = c;
    ++n;
  }
  if (n == 0 && t.find("\"entries\"") == std::string::npos) {
    set_error(std::string("tune file: no entries in ") + path);
    return ISDF_E_ARG;
  }
  return ISDF_OK;
}

isdf_status write_tune_file(const isdf_plan_s* pl, const char* path) {
  std::ofstream f(path);
  if (!f) {
    set_error(std::string("tune file: cannot write ") + path);
    return ISDF_E_ARG;
  }
  int dev = 0;
  hipDeviceProp_t pr{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess)
    std::snprintf(pr.gcnArchName, sizeof(pr.gcnArchName), "unknown");
  f << "{\n  \"arch\": \"" << pr.gcnArchName << "\",\n  \"shapes\": [";
  for (int i = 0; i < GEMM_NSHAPE; ++i)
    f << (i ? ", " : "") << "\"" << kShapes[i].bm << "x" << kShapes[i].bn << " w" << kShapes[i].wm
      << "x" << kShapes[i].wn << "\"";
  f << "],\n  \"entries\": [";
  bool first = true;
  for (const auto& kv : pl->tune) {
    f << (first ? "\n" : ",\n") << "    {\"key\": \"" << kv.first << "\", \"shape\": " << kv.second;
    auto it = pl->tune_us.find(kv.first);
    if (it != pl->tune_us.end()) {
      f << ", \"us\": [";
      for (size_t i = 0; i < it->second.size(); ++i) {
        char b[32];
        std::snprintf(b, sizeof(b), "%.1f", it->second[i]);
        f << (i ? ", " : "") << b;
      }
      f << "]";
    }
    f << "}";
    first = false;
  }
  f << "\n  ]\n}\n";
  return f ? ISDF_OK : ISDF_E_ARG;
}

// ------------------------------------------------------------- exchange
// Workspace of the exchange (n_occ = 0: dense D, else the factored form).
// Everything the kernel sequence touches is sized here, so that the
// sequence itself allocates nothing and can be captured as a graph.
// Rows of Q held at once by the occ-RI exchange: all N_mu when the full Q
// buffers fit a quarter of the free memory, else row blocks (multiples of
// 256) that fit 15 % of it (the fit's own blocks stay cached beside them).
// The dense exchange always holds all rows.
isdf_status ri_q_rows(isdf_plan_s* plan, isdf_fit_s* fit, bool mixed, int64_t* rows) {
  const int64_t m = fit->nmu;
  if (plan->opts.ri_rows > 0) {
    *rows = std::min<int64_t>(m, plan->opts.ri_rows);
    return ISDF_OK;
  }
  double avail = 0.0;
  isdf_status st;
  if ((st = plan_available(plan, AVAIL_RI, &avail)) != ISDF_OK) return st;
  const double ld2 = (double)((2 * m + 7) / 8 * 8);
  const double full = mixed ? 2.0 * mixed_splits(plan) * m * ld2 * 2.0 : 3.0 * 8.0 * m * m;
  const double per_row = mixed ? 2.0 * mixed_splits(plan) * ld2 * 2.0 : 4.0 * 8.0 * m;
  if (full <= 0.25 * avail) {
    *rows = m;
    return ISDF_OK;
  }
  int64_t r = (int64_t)(0.15 * avail / per_row) / 256 * 256;
  *rows = std::min<int64_t>(m, std::max<int64_t>(256, r));
  return ISDF_OK;
}

isdf_status exchange_prepare(isdf_plan_s* plan, isdf_fit_s* fit, int n_occ, bool ri) {
  const int64_t nmu = fit->nmu, N = plan->hp.n_basis;
  const int64_t ec = n_occ > 0 ? n_occ : N;  // columns of E_G, E_L
  isdf_status st;
  const bool mixed = mixed_on(plan, ISDF_MIX_EXCHANGE);
  if (!ri && !fit->Y1.p) {  // dense K only
    if ((st = fit->Y1.alloc(sizeof(double) * nmu * N)) != ISDF_OK) return st;
    if ((st = fit->Y2.alloc(sizeof(double) * nmu * N)) != ISDF_OK) return st;
  }
  if (!fit->partial.p) {
    if ((st = fit->partial.alloc(sizeof(double) * 1024)) != ISDF_OK) return st;
    if ((st = fit->ex_out.alloc(sizeof(double))) != ISDF_OK) return st;
  }
  // rows of Q: the dense exchange needs all, occ-RI may run in row blocks
  // (whole 64-index screening tiles when screening)
  int64_t need_rows = nmu;
  if (ri && fit->q_rows < nmu && (st = ri_q_rows(plan, fit, mixed, &need_rows)) != ISDF_OK) return st;
  if (ri && plan->opts.ri_screen_tau > 0.0 && need_rows < nmu) need_rows = std::max<int64_t>(64, need_rows / 64 * 64);
  const bool new_q = fit->q_rows < need_rows;
  if (new_q) {
    fit->q_rows = need_rows;
    fit->drop_graph();  // a captured exchange would read the old buffers
  }
  const int64_t qr = fit->q_rows;
  if (!mixed && (new_q || !fit->QGG.p)) {  // the mixed path writes Q straight into split planes
    for (DevBuf* q : {&fit->QGG, &fit->QGL, &fit->QLL})
      if ((st = q->alloc(sizeof(double) * qr * nmu)) != ISDF_OK) return st;
    if (qr < nmu) {
      if ((st = fit->QLG.alloc(sizeof(double) * qr * nmu)) != ISDF_OK) return st;
    } else {
      fit->QLG.release();
    }
  }
  if (fit->EG.bytes < sizeof(double) * nmu * ec) {
    if ((st = fit->EG.alloc(sizeof(double) * nmu * ec)) != ISDF_OK) return st;
    if ((st = fit->EL.alloc(sizeof(double) * nmu * ec)) != ISDF_OK) return st;
  }
  if (!ri && n_occ > 0 && !fit->Docc.p)
    if ((st = fit->Docc.alloc(sizeof(double) * N * N)) != ISDF_OK) return st;
  if (mixed) {
    const int S = mixed_splits(plan);
    const int m = (int)nmu, n = (int)N;
    hipStream_t s = plan->stream;
    if (!fit->xg_row.buf.p) {  // fit-time operands, built once
      if ((st = make_planes(s, S, fit->XG.as<double>(), 1, nmu, nullptr, m, n, fit->xg_row)) != ISDF_OK)
        return st;
      if ((st = make_planes(s, S, fit->XL.as<double>(), 1, nmu, nullptr, m, n, fit->xl_row)) != ISDF_OK)
        return st;
      if ((st = size_planes(S, n, 2 * m, fit->xln)) != ISDF_OK) return st;
      fit->xln.rows = n;
      fit->xln.cols = 2 * m;
      fit->xln.ld = (2 * m + 7) / 8 * 8;
      fit->xln.plane = (int64_t)n * fit->xln.ld;
      __bf16* xb = static_cast<__bf16*>(fit->xln.buf.p);
      if ((st = launch_split_bf16(s, fit->XL.as<double>(), nmu, 1, nullptr, n, m, S, xb, fit->xln.ld,
                                  fit->xln.plane, 1.0)) != ISDF_OK)
        return st;
      if ((st = launch_split_bf16(s, fit->XN.as<double>(), nmu, 1, nullptr, n, m, S, xb + m, fit->xln.ld,
                                  fit->xln.plane, 1.0)) != ISDF_OK)
        return st;
    }
    if (new_q || !fit->Q1.buf.p) {  // Q1 = [Q_GG Q_GL], Q2 = [Q_GL^T Q_LL]: q_rows rows of 2 N_mu
      for (Planes* q : {&fit->Q1, &fit->Q2}) {
        if ((st = size_planes(S, (int)qr, 2 * m, *q)) != ISDF_OK) return st;
        q->rows = (int)qr;
        q->cols = 2 * m;
        q->ld = (2 * m + 7) / 8 * 8;
        q->plane = qr * q->ld;
      }
      fit->qprobs_nocc = -1;  // problem tables point at the planes
      fit->ri_nocc = -1;
      fit->ydense = false;
    }
    if (!ri && !fit->ydense) {  // dense K: Y12 planes and the Y and K problem tables
      if ((st = size_planes(S, n, 2 * m, fit->Y12)) != ISDF_OK) return st;
      fit->Y12.rows = n;
      fit->Y12.cols = 2 * m;
      fit->Y12.ld = (2 * m + 7) / 8 * 8;
      fit->Y12.plane = (int64_t)n * fit->Y12.ld;
      // Y1 = Q1 xln^T and Y2 = Q2 xln^T, one grouped launch
      std::vector<MixedProblem> yp(2);
      int tiles = 0;
      for (int i = 0; i < 2; ++i) {
        yp[i] = mixed_problem(i == 0 ? fit->Q1 : fit->Q2, fit->xln, (i == 0 ? fit->Y1 : fit->Y2).as<double>(),
                              nmu, m, n, 2 * m, 1.0, 0.0, nullptr, 0);
        yp[i].tile_start = tiles;
        tiles += mixed_tiles_wide(m, n);
      }
      fit->ytiles = tiles;
      if ((st = upload(fit->d_yprobs, yp)) != ISDF_OK) return st;
      // K = -(xln)(Y12)^T over k ranges of KSPLIT_CHUNK, partials summed in order
      const int kc = std::max(32, (2 * m + KSPLIT - 1) / KSPLIT / 32 * 32);
      std::vector<MixedProblem> kp;
      tiles = 0;
      for (int k0 = 0; k0 < 2 * m; k0 += kc) {
        MixedProblem q = mixed_problem(fit->xln, fit->Y12, nullptr, N, n, n, std::min(kc, 2 * m - k0), -1.0,
                                       0.0, nullptr, 0);
        q.A += k0;
        q.B += k0;
        q.tile_start = tiles;
        tiles += mixed_tiles(n, n);
        kp.push_back(q);
      }
      fit->kparts = (int)kp.size();
      fit->ktiles = tiles;
      if ((st = fit->Kpart.alloc(sizeof(double) * (size_t)fit->kparts * n * n)) != ISDF_OK) return st;
      for (int i = 0; i < fit->kparts; ++i) kp[i].C = fit->Kpart.as<double>() + (int64_t)i * n * n;
      if ((st = upload(fit->d_kprobs, kp)) != ISDF_OK) return st;
      fit->ydense = true;
    }
    if ((st = size_planes(S, n_occ > 0 ? n_occ : n, n, fit->Dp)) != ISDF_OK) return st;
    if ((st = size_planes(S, m, (int)ec, fit->EGp)) != ISDF_OK) return st;
    if ((st = size_planes(S, m, (int)ec, fit->ELp)) != ISDF_OK) return st;
    if (fit->qprobs_nocc != n_occ) {
      // Q_ST = P_ST o W with P_ST = E_S B_T^T, B = E (factored) or X (dense).
      // The product C(i, j) = (B_T E_S^T)(i, j) W(i, j) = Q_ST(j, i) (W is
      // symmetric) lands transposed, at row j and column i of the A operand,
      // so each block of Q1 = [Q_GG Q_GL] and Q2 = [Q_GL^T Q_LL] is one
      // product whose planes the epilogue writes; the four share W's tiles.
      // Row block [r0, r1) of Q1 and Q2: rows r0.. of the second operand
      // and columns r0.. of W, written from row 0 of the planes.
      fit->EGp.rows = fit->ELp.rows = m;
      fit->EGp.cols = fit->ELp.cols = (int)ec;
      fit->EGp.ld = fit->ELp.ld = (ec + 7) / 8 * 8;
      fit->EGp.plane = fit->ELp.plane = (int64_t)m * fit->EGp.ld;
      const Planes& BG = n_occ > 0 ? fit->EGp : fit->xg_row;
      const Planes& BL = n_occ > 0 ? fit->ELp : fit->xl_row;
      const Planes* ops[4][2] = {{&BG, &fit->EGp}, {&BL, &fit->EGp}, {&fit->EGp, &BL}, {&BL, &fit->ELp}};
      Planes* dst[4] = {&fit->Q1, &fit->Q1, &fit->Q2, &fit->Q2};
      const int off[4] = {0, m, 0, m};
      std::vector<MixedProblem> qp;
      for (int64_t r0 = 0; r0 < nmu; r0 += qr) {
        const int rb = (int)std::min<int64_t>(qr, nmu - r0);
        for (int i = 0; i < 4; ++i) {
          MixedProblem q = mixed_problem(*ops[i][0], *ops[i][1], nullptr, 0, m, rb, (int)ec, 1.0, 0.0,
                                         fit->w64() ? fit->w64() + r0 * nmu : nullptr, nmu);
          q.B += r0 * ops[i][1]->ld;
          q.E32 = fit->wf32() ? fit->wf32() + r0 * nmu : nullptr;
          q.P = static_cast<__bf16*>(dst[i]->buf.p);
          q.plane_p = dst[i]->plane;
          q.ldp = dst[i]->ld;
          q.p_off = off[i];
          q.tile_group = 16;  // measured on the 384-atom Q products: 42.6 ms against 44.0 with 8
          qp.push_back(q);
        }
      }
      if ((st = upload(fit->d_qprobs, qp)) != ISDF_OK) return st;
      fit->qprobs_nocc = n_occ;
    }
  }
  if (ri && plan->opts.ri_screen_tau > 0.0 && !mixed && fit->s_nocc != n_occ) {
    // density screening: tile maxima of |W| once per fit, the rest per n_occ
    const int64_t nt = (nmu + 63) / 64;
    if (!fit->s_wt.p) {
      if ((st = fit->s_wt.alloc(sizeof(double) * nt * nt)) != ISDF_OK) return st;
      if ((st = launch_tile_absmax_w(plan->stream, fit->w64(), fit->wf32(), nmu, (int)nmu, 64, fit->s_wt.as<double>())) !=
          ISDF_OK)
        return st;
    }
    for (DevBuf* d : {&fit->s_ng, &fit->s_nl})
      if ((st = d->alloc(sizeof(double) * nt * std::max(n_occ, 1))) != ISDF_OK) return st;
    for (DevBuf* d : {&fit->s_bgg, &fit->s_bgl, &fit->s_bll})
      if ((st = d->alloc(sizeof(double) * nt * nt)) != ISDF_OK) return st;
    for (DevBuf* d : {&fit->s_mgg, &fit->s_mgl, &fit->s_mll})
      if ((st = d->alloc(nt * nt)) != ISDF_OK) return st;
    fit->s_nt = (int)nt;
    fit->s_nocc = n_occ;
    fit->drop_graph();
  }
  if (ri && fit->ri_nocc != n_occ) {
    const int m = (int)nmu, n = (int)N, o = n_occ;
    for (DevBuf* b : {&fit->EN, &fit->Z1, &fit->Z2})
      if ((st = b->alloc(sizeof(double) * nmu * o)) != ISDF_OK) return st;
    if (mixed) {
      const int S = mixed_splits(plan);
      for (Planes* q : {&fit->ELN, &fit->Z12}) {
        if ((st = size_planes(S, o, 2 * m, *q)) != ISDF_OK) return st;
        q->rows = o;
        q->cols = 2 * m;
        q->ld = (2 * m + 7) / 8 * 8;
        q->plane = (int64_t)o * q->ld;
      }
      // per row block: Z1 = Q1 ELN^T, Z2 = Q2 ELN^T, one grouped launch per
      // range of RI_Z_KCHUNK columns of the 2 N_mu-long contraction, the
      // first with beta = 0 and the rest accumulating (beta = 1)
      std::vector<MixedProblem> zp;
      for (int64_t r0 = 0; r0 < nmu; r0 += qr) {
        const int rb = (int)std::min<int64_t>(qr, nmu - r0);
        for (int k0 = 0; k0 < 2 * m; k0 += RI_Z_KCHUNK) {
          int tiles = 0;
          for (int i = 0; i < 2; ++i) {
            MixedProblem z = mixed_problem(i == 0 ? fit->Q1 : fit->Q2, fit->ELN,
                                           (i == 0 ? fit->Z1 : fit->Z2).as<double>() + r0, nmu, rb, o,
                                           std::min(RI_Z_KCHUNK, 2 * m - k0), 1.0, k0 ? 1.0 : 0.0, nullptr, 0);
            z.A += k0;
            z.B += k0;
            z.tile_group = 2;  // measured on the 384-atom Z chunks: 22.7 ms against 23.5 with 8
            z.tile_start = tiles;
            tiles += mixed_tiles_wide(rb, o);
            zp.push_back(z);
          }
        }
      }
      if ((st = upload(fit->d_zprobs, zp)) != ISDF_OK) return st;
      // (K C)^T = -(Z12)(xln)^T over k ranges on the wide-tile kernel,
      // partials summed in order
      const int kc = std::max(32, (2 * m + KSPLIT_RI - 1) / KSPLIT_RI / 32 * 32);
      std::vector<MixedProblem> kp;
      int tiles = 0;
      for (int k0 = 0; k0 < 2 * m; k0 += kc) {
        MixedProblem q = mixed_problem(fit->Z12, fit->xln, nullptr, o, o, n, std::min(kc, 2 * m - k0), -1.0,
                                       0.0, nullptr, 0);
        q.A += k0;
        q.B += k0;
        q.tile_start = tiles;
        tiles += mixed_tiles_wide(o, n);
        kp.push_back(q);
      }
      fit->kcparts = (int)kp.size();
      fit->kctiles = tiles;
      if ((st = fit->KCpart.alloc(sizeof(double) * (size_t)fit->kcparts * o * n)) != ISDF_OK) return st;
      for (int i = 0; i < fit->kcparts; ++i) kp[i].C = fit->KCpart.as<double>() + (int64_t)i * o * n;
      if ((st = upload(fit->d_kcprobs, kp)) != ISDF_OK) return st;
    }
    fit->ri_nocc = n_occ;
  }
  return ISDF_OK;
}

// The kernel sequence of one exchange on plan->stream: no allocation, no
// synchronisation.  in = D (n_occ = 0) or C_occ (row-major N x n_occ).
isdf_status exchange_enqueue(isdf_plan_s* plan, isdf_fit_s* fit, const double* in, int n_occ,
                             double* K, bool stage_event) {
  hipStream_t s = plan->stream;
  const int64_t nmu = fit->nmu, N = plan->hp.n_basis;
  const int m = (int)nmu, n = (int)N, ec = n_occ > 0 ? n_occ : n;
  const double* XL = fit->XL.as<double>();
  const double* XN = fit->XN.as<double>();
  const double* XG = fit->XG.as<double>();
  const double* W = fit->w64();
  double* EG = fit->EG.as<double>();
  double* EL = fit->EL.as<double>();
  double* Y1 = fit->Y1.as<double>();
  double* Y2 = fit->Y2.as<double>();
  double* QGG = fit->QGG.as<double>();
  double* QGL = fit->QGL.as<double>();
  double* QLL = fit->QLL.as<double>();
  isdf_status st;
  auto gemm = [&](int epi, const double* A, int64_t lda, int tA, const double* B, int64_t ldb,
                  int tB, double* C, int64_t ldc, int M, int Nn, int Kk, double alpha, double beta,
                  const double* E) {
    GemmProblem p{};
    p.A = A; p.lda = lda; p.transA = tA;
    p.B = B; p.ldb = ldb; p.transB = tB;
    p.C = C; p.ldc = ldc;
    p.E = E; p.lde = nmu;
    if (epi == EPI_HADAMARD) p.E32 = fit->wf32();  // every Hadamard factor here is W
    p.M = M; p.N = Nn; p.K = Kk;
    p.alpha = alpha; p.beta = beta;
    return gemm_prof(plan, ISDF_K_GEMM_EXCHANGE, epi, p);
  };
  if (mixed_on(plan, ISDF_MIX_EXCHANGE)) {
    const int S = mixed_splits(plan);
    auto mg = [&](int epi, const Planes& A, const Planes& B, double* C, int64_t ldc, int M, int Nn,
                  int Kk, double alpha, double beta) {
      return mixed_prof(plan, ISDF_K_GEMM_EXCHANGE, epi,
                        mixed_problem(A, B, C, ldc, M, Nn, Kk, alpha, beta, W, nmu));
    };
    // B operand of E = X D (k = nu): rows lam of D, or rows i of C_occ
    if (n_occ > 0) {
      if ((st = make_planes(s, S, in, 1, n_occ, nullptr, n_occ, n, fit->Dp)) != ISDF_OK) return st;
    } else {
      if ((st = make_planes(s, S, in, N, 1, nullptr, n, n, fit->Dp)) != ISDF_OK) return st;
    }
    if ((st = mg(EPI_AXPBY, fit->xg_row, fit->Dp, EG, nmu, m, ec, n, 1.0, 0.0)) != ISDF_OK) return st;
    if ((st = mg(EPI_AXPBY, fit->xl_row, fit->Dp, EL, nmu, m, ec, n, 1.0, 0.0)) != ISDF_OK) return st;
    if ((st = make_planes(s, S, EG, 1, nmu, nullptr, m, ec, fit->EGp)) != ISDF_OK) return st;
    if ((st = make_planes(s, S, EL, 1, nmu, nullptr, m, ec, fit->ELp)) != ISDF_OK) return st;
    {  // the four Q blocks (exchange_prepare), interleaved tile by tile
      ProfScope ps(plan, ISDF_K_GEMM_EXCHANGE,
                   4.0 * (2.0 * S * 2.0 * m * (double)ec + 2.0 * S * (double)m * m) + 8.0 * (double)m * m,
                   4.0 * 2.0 * m * (double)m * ec);
      if ((st = gemm_mixed_wide_grouped(s, EPI_HADAMARD_PLANES, S, fit->d_qprobs.as<MixedProblem>(), -4,
                                        4 * mixed_tiles_wide(m, m), family_tag(ISDF_K_GEMM_EXCHANGE))) != ISDF_OK)
        return st;
    }
    {  // Y1 = Q1 xln^T, Y2 = Q2 xln^T
      ProfScope ps(plan, ISDF_K_GEMM_EXCHANGE, 2.0 * (2.0 * S * (2.0 * m * m + 2.0 * m * n) + 8.0 * m * n),
                   2.0 * (2.0 * m * (double)n * 2.0 * m));
      if ((st = gemm_mixed_wide_grouped(s, EPI_AXPBY, S, fit->d_yprobs.as<MixedProblem>(), 2, fit->ytiles,
                                        family_tag(ISDF_K_GEMM_EXCHANGE))) != ISDF_OK)
        return st;
    }
    __bf16* yb = static_cast<__bf16*>(fit->Y12.buf.p);
    if ((st = launch_split_bf16(s, Y1, nmu, 1, nullptr, n, m, S, yb, fit->Y12.ld, fit->Y12.plane, 1.0)) !=
        ISDF_OK)
      return st;
    if ((st = launch_split_bf16(s, Y2, nmu, 1, nullptr, n, m, S, yb + m, fit->Y12.ld, fit->Y12.plane, 1.0)) !=
        ISDF_OK)
      return st;
    {  // K = -(xln)(Y12)^T: partial products over k ranges, then their ordered sum
      ProfScope ps(plan, ISDF_K_GEMM_EXCHANGE, 2.0 * S * (4.0 * m * n) + 8.0 * fit->kparts * n * (double)n,
                   2.0 * n * (double)n * 2.0 * m);
      if ((st = gemm_mixed_grouped(s, EPI_AXPBY, S, fit->d_kprobs.as<MixedProblem>(), fit->kparts,
                                   fit->ktiles, family_tag(ISDF_K_GEMM_EXCHANGE))) != ISDF_OK)
        return st;
    }
    if ((st = launch_sum_parts(s, fit->Kpart.as<double>(), fit->kparts, (int64_t)n * n, K)) != ISDF_OK)
      return st;
  } else {
    if (n_occ > 0) {
      // E_G = X^G C, E_L = X^L C; Q_ST = (E_S E_T^T) o W
      if ((st = gemm(EPI_AXPBY, XG, nmu, 0, in, n_occ, 1, EG, nmu, m, ec, n, 1.0, 0.0, nullptr)) != ISDF_OK) return st;
      if ((st = gemm(EPI_AXPBY, XL, nmu, 0, in, n_occ, 1, EL, nmu, m, ec, n, 1.0, 0.0, nullptr)) != ISDF_OK) return st;
      if ((st = gemm(EPI_HADAMARD, EG, nmu, 0, EG, nmu, 1, QGG, nmu, m, m, ec, 1.0, 0.0, W)) != ISDF_OK) return st;
      if ((st = gemm(EPI_HADAMARD, EG, nmu, 0, EL, nmu, 1, QGL, nmu, m, m, ec, 1.0, 0.0, W)) != ISDF_OK) return st;
      if ((st = gemm(EPI_HADAMARD, EL, nmu, 0, EL, nmu, 1, QLL, nmu, m, m, ec, 1.0, 0.0, W)) != ISDF_OK) return st;
    } else {
      // E_G = X^G D, E_L = X^L D; Q = (E X^T) o W
      if ((st = gemm(EPI_AXPBY, XG, nmu, 0, in, N, 0, EG, nmu, m, n, n, 1.0, 0.0, nullptr)) != ISDF_OK) return st;
      if ((st = gemm(EPI_AXPBY, XL, nmu, 0, in, N, 0, EL, nmu, m, n, n, 1.0, 0.0, nullptr)) != ISDF_OK) return st;
      if ((st = gemm(EPI_HADAMARD, EG, nmu, 0, XG, nmu, 1, QGG, nmu, m, m, n, 1.0, 0.0, W)) != ISDF_OK) return st;
      if ((st = gemm(EPI_HADAMARD, EG, nmu, 0, XL, nmu, 1, QGL, nmu, m, m, n, 1.0, 0.0, W)) != ISDF_OK) return st;
      if ((st = gemm(EPI_HADAMARD, EL, nmu, 0, XL, nmu, 1, QLL, nmu, m, m, n, 1.0, 0.0, W)) != ISDF_OK) return st;
    }
    // Y1 = Q_GG X^L + Q_GL X^N ; Y2 = Q_GL^T X^L + Q_LL X^N
    if ((st = gemm(EPI_AXPBY, QGG, nmu, 0, XL, nmu, 0, Y1, nmu, m, n, m, 1.0, 0.0, nullptr)) != ISDF_OK) return st;
    if ((st = gemm(EPI_AXPBY, QGL, nmu, 0, XN, nmu, 0, Y1, nmu, m, n, m, 1.0, 1.0, nullptr)) != ISDF_OK) return st;
    if ((st = gemm(EPI_AXPBY, QGL, nmu, 1, XL, nmu, 0, Y2, nmu, m, n, m, 1.0, 0.0, nullptr)) != ISDF_OK) return st;
    if ((st = gemm(EPI_AXPBY, QLL, nmu, 0, XN, nmu, 0, Y2, nmu, m, n, m, 1.0, 1.0, nullptr)) != ISDF_OK) return st;
    // K = -(X^L^T Y1 + X^N^T Y2)
    if ((st = gemm(EPI_AXPBY, XL, nmu, 1, Y1, nmu, 0, K, N, n, n, m, -1.0, 0.0, nullptr)) != ISDF_OK) return st;
    if ((st = gemm(EPI_AXPBY, XN, nmu, 1, Y2, nmu, 0, K, N, n, n, m, -1.0, 1.0, nullptr)) != ISDF_OK) return st;
  }
  if (stage_event) ISDF_HIP_TRY(hipEventRecord(plan->ev[1], s));
  const double* Dm = in;
  if (n_occ > 0) {  // D = C C^T for e_x = tr(D K)
    if ((st = gemm(EPI_AXPBY, in, n_occ, 1, in, n_occ, 0, fit->Docc.as<double>(), N, n, n, n_occ, 1.0,
                   0.0, nullptr)) != ISDF_OK)
      return st;
    Dm = fit->Docc.as<double>();
  }
  return launch_trace_dot(s, Dm, K, N * N, fit->partial.as<double>(), 1024, fit->ex_out.as<double>());
}

// occ-RI output on plan->stream (no allocation, no synchronisation):
// KC = K C (N x n_occ, row-major like C) for D = C C^T, without forming K:
// E_L = X^L C, E_N = X^N C, Z1 = Q_GG E_L + Q_GL E_N, Z2 = Q_GL^T E_L +
// Q_LL E_N, K C = -(X^L' Z1 + X^N' Z2); e_x = sum(C o KC) = tr(D K).
// Workspace of the FP64 occ-RI products: E_G, E_L, E_N, Z1, Z2 (N_mu x n_occ)
// and the three Hadamard blocks Q_GG, Q_GL, Q_LL (N_mu x N_mu), column-major.
struct RiBuffers {
  double *EG, *EL, *EN, *QGG, *QGL, *QLL, *Z1, *Z2;
  // row blocks: qrows rows per block in QGG, QGL, QLG, QLL (qrows x N_mu
  // each); 0 or N_mu: one block, no QLG
  double* QLG;
  int64_t qrows;
  // density screening (tau > 0; FP64 path): tile maxima and bounds, masks
  double tau;
  const double *wt;
  double *ng, *nl, *bgg, *bgl, *bll;
  uint8_t *mgg, *mgl, *mll;
};

// FP64 occ-RI products into the given workspace (no allocation):
//   E_G = X^G C, E_L = X^L C, E_N = E_G - E_L,
//   Q_ST = W o (E_S E_T^T), Z1 = Q_GG E_L + Q_GL E_N, Z2 = Q_GL^T E_L + Q_LL E_N,
//   (K C)^T = -(Z1^T X^L + Z2^T X^N)   (n_occ x N column-major = K C row-major).
// With row blocks, rows [r0, r1) of Z1 and Z2 come from the same rows of
// Q_GG, Q_GL, Q_LL and Q_LG = Q_GL^T (W symmetric: Q_LG(r, :) is
// W(r, :) o (E_L(r, :) E_G^T)), so no N_mu x N_mu buffer is held.
isdf_status ri_fp64_products(isdf_plan_s* plan, isdf_fit_s* fit, const double* Cin, int o, double* KC,
                             const RiBuffers& b) {
  hipStream_t s = plan->stream;
  const int64_t nmu = fit->nmu;
  const int m = (int)nmu, n = (int)plan->hp.n_basis;
  const double* XL = fit->XL.as<double>();
  const double* XN = fit->XN.as<double>();
  const double* XG = fit->XG.as<double>();
  const double* W = fit->w64();
  const float* W32 = fit->wf32();
  const bool scr = b.tau > 0.0;
  const int64_t nt = (nmu + 63) / 64;
  // mask of a product: base, strides of (row tile, column or K tile), mode
  struct Mask {
    const uint8_t* base;
    int64_t s0, s1;
    int mode;
  };
  const Mask none{nullptr, 0, 0, 0};
  auto gemm = [&](int epi, const double* A, int64_t lda, int tA, const double* B, int64_t ldb, int tB,
                  double* C, int64_t ldc, int M, int Nn, int Kk, double alpha, double beta, int64_t e_row,
                  const Mask& mk) {
    GemmProblem p{};
    p.A = A; p.lda = lda; p.transA = tA;
    p.B = B; p.ldb = ldb; p.transB = tB;
    p.C = C; p.ldc = ldc;
    if (epi == EPI_HADAMARD) {  // the Hadamard factor is W, from row e_row on
      p.E = W ? W + e_row : nullptr;
      p.E32 = W32 ? W32 + e_row : nullptr;
    }
    p.lde = nmu;
    p.M = M; p.N = Nn; p.K = Kk;
    p.alpha = alpha; p.beta = beta;
    if (scr && mk.mode) {
      p.tmask = mk.base;
      p.tm_s0 = mk.s0;
      p.tm_s1 = mk.s1;
      p.tmask_mode = mk.mode;
    }
    return gemm_prof(plan, ISDF_K_GEMM_EXCHANGE, epi, p);
  };
  isdf_status st;
  if ((st = gemm(EPI_AXPBY, XG, nmu, 0, Cin, o, 1, b.EG, nmu, m, o, n, 1.0, 0.0, 0, none)) != ISDF_OK) return st;
  if ((st = gemm(EPI_AXPBY, XL, nmu, 0, Cin, o, 1, b.EL, nmu, m, o, n, 1.0, 0.0, 0, none)) != ISDF_OK) return st;
  if ((st = launch_sub(s, b.EG, b.EL, b.EN, nmu * o)) != ISDF_OK) return st;
  if (scr) {
    // tile bounds B_ST = Wt o (N_S N_T^T), N_S(b, i) = max over tile b of
    // |E_S(., i)|, and the masks of the tiles at or above tau
    if ((st = launch_tile_absmax(s, b.EG, nmu, m, o, 64, b.ng)) != ISDF_OK) return st;
    if ((st = launch_tile_absmax(s, b.EL, nmu, m, o, 64, b.nl)) != ISDF_OK) return st;
    const double* NS[3] = {b.ng, b.ng, b.nl};
    const double* NT[3] = {b.ng, b.nl, b.nl};
    double* BB[3] = {b.bgg, b.bgl, b.bll};
    uint8_t* MM[3] = {b.mgg, b.mgl, b.mll};
    for (int t = 0; t < 3; ++t) {
      GemmProblem p{};
      p.A = NS[t]; p.lda = nt;
      p.B = NT[t]; p.ldb = nt; p.transB = 1;
      p.C = BB[t]; p.ldc = nt;
      p.E = b.wt; p.lde = nt;
      p.M = (int)nt; p.N = (int)nt; p.K = o;
      p.alpha = 1.0;
      if ((st = gemm_prof(plan, ISDF_K_GEMM_EXCHANGE, EPI_HADAMARD, p)) != ISDF_OK) return st;
      if ((st = launch_mask_ge(s, BB[t], nt * nt, b.tau, MM[t])) != ISDF_OK) return st;
    }
  }
  // masks: output tiles (mode 1) of the Q products, K ranges (mode 2) of Z
  auto out_mask = [&](const uint8_t* mk, int64_t row_tile0) { return Mask{mk + row_tile0, 1, nt, 1}; };
  auto k_mask = [&](const uint8_t* mk, int64_t row_tile0) { return Mask{mk + row_tile0, 1, nt, 2}; };
  if (b.qrows <= 0 || b.qrows >= nmu) {
    if ((st = gemm(EPI_HADAMARD, b.EG, nmu, 0, b.EG, nmu, 1, b.QGG, nmu, m, m, o, 1.0, 0.0, 0, out_mask(b.mgg, 0))) !=
        ISDF_OK)
      return st;
    if ((st = gemm(EPI_HADAMARD, b.EG, nmu, 0, b.EL, nmu, 1, b.QGL, nmu, m, m, o, 1.0, 0.0, 0, out_mask(b.mgl, 0))) !=
        ISDF_OK)
      return st;
    if ((st = gemm(EPI_HADAMARD, b.EL, nmu, 0, b.EL, nmu, 1, b.QLL, nmu, m, m, o, 1.0, 0.0, 0, out_mask(b.mll, 0))) !=
        ISDF_OK)
      return st;
    if ((st = gemm(EPI_AXPBY, b.QGG, nmu, 0, b.EL, nmu, 0, b.Z1, nmu, m, o, m, 1.0, 0.0, 0, k_mask(b.mgg, 0))) !=
        ISDF_OK)
      return st;
    if ((st = gemm(EPI_AXPBY, b.QGL, nmu, 0, b.EN, nmu, 0, b.Z1, nmu, m, o, m, 1.0, 1.0, 0, k_mask(b.mgl, 0))) !=
        ISDF_OK)
      return st;
    // Q_GL^T: its row tile r, K tile q is Q_GL's tile (q, r)
    if ((st = gemm(EPI_AXPBY, b.QGL, nmu, 1, b.EL, nmu, 0, b.Z2, nmu, m, o, m, 1.0, 0.0, 0,
                   Mask{b.mgl, nt, 1, 2})) != ISDF_OK)
      return st;
    if ((st = gemm(EPI_AXPBY, b.QLL, nmu, 0, b.EN, nmu, 0, b.Z2, nmu, m, o, m, 1.0, 1.0, 0, k_mask(b.mll, 0))) !=
        ISDF_OK)
      return st;
  } else {
    for (int64_t r0 = 0; r0 < nmu; r0 += b.qrows) {
      const int rb = (int)std::min<int64_t>(b.qrows, nmu - r0);
      const int64_t q = b.qrows;  // leading dimension of the block buffers
      const int64_t t0 = r0 / 64;  // first row tile (row blocks start on tile boundaries)
      // Q_XY(r, :) = W(r, :) o (E_X(r, :) E_Y^T): rows r0.. of W are W + r0 (lde N_mu)
      if ((st = gemm(EPI_HADAMARD, b.EG + r0, nmu, 0, b.EG, nmu, 1, b.QGG, q, rb, m, o, 1.0, 0.0, r0,
                     out_mask(b.mgg, t0))) != ISDF_OK)
        return st;
      if ((st = gemm(EPI_HADAMARD, b.EG + r0, nmu, 0, b.EL, nmu, 1, b.QGL, q, rb, m, o, 1.0, 0.0, r0,
                     out_mask(b.mgl, t0))) != ISDF_OK)
        return st;
      // Q_LG = Q_GL^T: its tile (r, c) is Q_GL's tile (c, r)
      if ((st = gemm(EPI_HADAMARD, b.EL + r0, nmu, 0, b.EG, nmu, 1, b.QLG, q, rb, m, o, 1.0, 0.0, r0,
                     Mask{b.mgl + t0 * nt, nt, 1, 1})) != ISDF_OK)
        return st;
      if ((st = gemm(EPI_HADAMARD, b.EL + r0, nmu, 0, b.EL, nmu, 1, b.QLL, q, rb, m, o, 1.0, 0.0, r0,
                     out_mask(b.mll, t0))) != ISDF_OK)
        return st;
      if ((st = gemm(EPI_AXPBY, b.QGG, q, 0, b.EL, nmu, 0, b.Z1 + r0, nmu, rb, o, m, 1.0, 0.0, 0,
                     k_mask(b.mgg, t0))) != ISDF_OK)
        return st;
      if ((st = gemm(EPI_AXPBY, b.QGL, q, 0, b.EN, nmu, 0, b.Z1 + r0, nmu, rb, o, m, 1.0, 1.0, 0,
                     k_mask(b.mgl, t0))) != ISDF_OK)
        return st;
      if ((st = gemm(EPI_AXPBY, b.QLG, q, 0, b.EL, nmu, 0, b.Z2 + r0, nmu, rb, o, m, 1.0, 0.0, 0,
                     Mask{b.mgl + t0 * nt, nt, 1, 2})) != ISDF_OK)
        return st;
      if ((st = gemm(EPI_AXPBY, b.QLL, q, 0, b.EN, nmu, 0, b.Z2 + r0, nmu, rb, o, m, 1.0, 1.0, 0,
                     k_mask(b.mll, t0))) != ISDF_OK)
        return st;
    }
  }
  if ((st = gemm(EPI_AXPBY, b.Z1, nmu, 1, XL, nmu, 0, KC, o, o, n, m, -1.0, 0.0, 0, none)) != ISDF_OK) return st;
  return gemm(EPI_AXPBY, b.Z2, nmu, 1, XN, nmu, 0, KC, o, o, n, m, -1.0, 1.0, 0, none);
}

isdf_status exchange_enqueue_ri(isdf_plan_s* plan, isdf_fit_s* fit, const double* Cin, int n_occ, double* KC,
                                bool stage_event) {
  hipStream_t s = plan->stream;
  const int64_t nmu = fit->nmu, N = plan->hp.n_basis;
  const int m = (int)nmu, n = (int)N, o = n_occ;
  double* EG = fit->EG.as<double>();
  double* EL = fit->EL.as<double>();
  double* EN = fit->EN.as<double>();
  double* Z1 = fit->Z1.as<double>();
  double* Z2 = fit->Z2.as<double>();
  isdf_status st;
  if (mixed_on(plan, ISDF_MIX_EXCHANGE)) {
    const int S = mixed_splits(plan);
    if ((st = make_planes(s, S, Cin, 1, o, nullptr, o, n, fit->Dp)) != ISDF_OK) return st;
    for (int t = 0; t < 2; ++t) {
      MixedProblem q = mixed_problem(t == 0 ? fit->xg_row : fit->xl_row, fit->Dp, t == 0 ? EG : EL, nmu, m, o, n,
                                     1.0, 0.0, nullptr, 0);
      if ((st = mixed_prof(plan, ISDF_K_GEMM_EXCHANGE, EPI_AXPBY, q)) != ISDF_OK) return st;
    }
    if ((st = launch_sub(s, EG, EL, EN, nmu * o)) != ISDF_OK) return st;
    if ((st = make_planes(s, S, EG, 1, nmu, nullptr, m, o, fit->EGp)) != ISDF_OK) return st;
    if ((st = make_planes(s, S, EL, 1, nmu, nullptr, m, o, fit->ELp)) != ISDF_OK) return st;
    __bf16* eb = static_cast<__bf16*>(fit->ELN.buf.p);
    if ((st = launch_split_bf16(s, EL, nmu, 1, nullptr, o, m, S, eb, fit->ELN.ld, fit->ELN.plane, 1.0)) != ISDF_OK)
      return st;
    if ((st = launch_split_bf16(s, EN, nmu, 1, nullptr, o, m, S, eb + m, fit->ELN.ld, fit->ELN.plane, 1.0)) !=
        ISDF_OK)
      return st;
    // per row block of Q (all N_mu rows at once unless memory asks for blocks)
    int blk = 0;
    for (int64_t r0 = 0; r0 < nmu; r0 += fit->q_rows, ++blk) {
      const int rb = (int)std::min<int64_t>(fit->q_rows, nmu - r0);
      {  // rows r0.. of Q1 = [Q_GG Q_GL], Q2 = [Q_GL^T Q_LL] as split planes (exchange_prepare)
        ProfScope ps(plan, ISDF_K_GEMM_EXCHANGE,
                     4.0 * (2.0 * S * (m + (double)rb) * o + 2.0 * S * (double)rb * m) + 8.0 * (double)rb * m,
                     4.0 * 2.0 * rb * (double)m * o);
        if ((st = gemm_mixed_wide_grouped(s, EPI_HADAMARD_PLANES, S, fit->d_qprobs.as<MixedProblem>() + 4 * blk, -4,
                                          4 * mixed_tiles_wide(m, rb), family_tag(ISDF_K_GEMM_EXCHANGE))) !=
            ISDF_OK)
          return st;
      }
      // rows r0.. of Z1 = Q1 ELN^T, Z2 = Q2 ELN^T, by K chunk (exchange_prepare)
      const int nkz = (2 * m + RI_Z_KCHUNK - 1) / RI_Z_KCHUNK;
      for (int c = 0; c < nkz; ++c) {
        const double kc = std::min(RI_Z_KCHUNK, 2 * m - c * RI_Z_KCHUNK);
        ProfScope ps(plan, ISDF_K_GEMM_EXCHANGE,
                     2.0 * (2.0 * S * (rb + (double)o) * kc + (c ? 16.0 : 8.0) * rb * o),
                     2.0 * (2.0 * rb * (double)o * kc));
        if ((st = gemm_mixed_wide_grouped(s, EPI_AXPBY, S, fit->d_zprobs.as<MixedProblem>() + 2 * (blk * nkz + c), 2,
                                          2 * mixed_tiles_wide(rb, o), family_tag(ISDF_K_GEMM_EXCHANGE))) != ISDF_OK)
          return st;
      }
    }
    __bf16* zb = static_cast<__bf16*>(fit->Z12.buf.p);
    if ((st = launch_split_bf16(s, Z1, nmu, 1, nullptr, o, m, S, zb, fit->Z12.ld, fit->Z12.plane, 1.0)) != ISDF_OK)
      return st;
    if ((st = launch_split_bf16(s, Z2, nmu, 1, nullptr, o, m, S, zb + m, fit->Z12.ld, fit->Z12.plane, 1.0)) !=
        ISDF_OK)
      return st;
    {  // (K C)^T = -(Z12)(xln)^T: partial products over k ranges, then their ordered sum
      ProfScope ps(plan, ISDF_K_GEMM_EXCHANGE, 2.0 * S * (2.0 * m * (o + n)) + 8.0 * fit->kcparts * o * (double)n,
                   2.0 * o * (double)n * 2.0 * m);
      if ((st = gemm_mixed_wide_grouped(s, EPI_AXPBY, S, fit->d_kcprobs.as<MixedProblem>(), fit->kcparts,
                                        fit->kctiles, family_tag(ISDF_K_GEMM_EXCHANGE))) != ISDF_OK)
        return st;
    }
    if ((st = launch_sum_parts(s, fit->KCpart.as<double>(), fit->kcparts, (int64_t)o * n, KC)) != ISDF_OK)
      return st;
  } else {
    RiBuffers b{EG, EL, EN, fit->QGG.as<double>(), fit->QGL.as<double>(), fit->QLL.as<double>(),
                Z1, Z2, fit->QLG.as<double>(), fit->q_rows};
    if (plan->opts.ri_screen_tau > 0.0) {
      b.tau = plan->opts.ri_screen_tau;
      b.wt = fit->s_wt.as<double>();
      b.ng = fit->s_ng.as<double>();
      b.nl = fit->s_nl.as<double>();
      b.bgg = fit->s_bgg.as<double>();
      b.bgl = fit->s_bgl.as<double>();
      b.bll = fit->s_bll.as<double>();
      b.mgg = fit->s_mgg.as<uint8_t>();
      b.mgl = fit->s_mgl.as<uint8_t>();
      b.mll = fit->s_mll.as<uint8_t>();
      fit->s_ran = true;
    }
    if ((st = ri_fp64_products(plan, fit, Cin, o, KC, b)) != ISDF_OK) return st;
  }
  if (stage_event) ISDF_HIP_TRY(hipEventRecord(plan->ev[1], s));
  return launch_trace_dot(s, Cin, KC, N * o, fit->partial.as<double>(), 1024, fit->ex_out.as<double>());
}

// C (M x N, column-major, ldc = M) = alpha op(A) op(B), plus the old C when
// `accumulate`, with K cut into slices whose products run as one grouped
// launch and are summed in order (skinny products with a long K: a 64 x 64
// tile grid of tens of tiles would leave most of the chip idle).
isdf_status gemm_split_k(isdf_plan_s* pl, const double* A, int64_t lda, int tA, const double* B, int64_t ldb,
                         int tB, double* C, int64_t M, int64_t N, int64_t K, double alpha, bool accumulate) {
  hipStream_t s = pl->stream;
  if (M <= 0 || N <= 0) return ISDF_OK;
  const int tiles1 = gemm_tiles((int)M, (int)N, 0);
  const int parts = (int)std::max<int64_t>(1, std::min<int64_t>((512 + tiles1 - 1) / tiles1, K / 256));
  const int slot0 = accumulate ? 1 : 0;
  isdf_status st;
  DevBuf part, dprobs;
  if ((st = part.alloc(sizeof(double) * (parts + slot0) * M * N)) != ISDF_OK) return st;
  if (accumulate)
    ISDF_HIP_TRY(hipMemcpyAsync(part.p, C, sizeof(double) * M * N, hipMemcpyDeviceToDevice, s));
  std::vector<GemmProblem> probs;
  const int64_t kc = (K + parts - 1) / parts;
  int tiles = 0;
  for (int q = 0; q < parts; ++q) {
    const int64_t k0 = q * kc, k1 = std::min(K, k0 + kc);
    if (k1 <= k0) break;
    GemmProblem p{};
    p.A = tA ? A + k0 : A + k0 * lda;
    p.lda = lda;
    p.transA = tA;
    p.B = tB ? B + k0 * ldb : B + k0;
    p.ldb = ldb;
    p.transB = tB;
    p.C = part.as<double>() + (slot0 + probs.size()) * M * N;
    p.ldc = M;
    p.M = (int)M;
    p.N = (int)N;
    p.K = (int)(k1 - k0);
    p.alpha = alpha;
    p.beta = 0.0;
    p.tile_start = tiles;
    tiles += tiles1;
    probs.push_back(p);
  }
  if ((st = upload(dprobs, probs)) != ISDF_OK) return st;
  {
    ProfScope ps(pl, ISDF_K_GEMM_EXCHANGE, 8.0 * (double)K * (M + N) + 8.0 * probs.size() * M * N,
                 2.0 * (double)M * N * K);
    if ((st = gemm_f64_grouped(s, EPI_AXPBY, dprobs.as<GemmProblem>(), (int)probs.size(), tiles,
                               family_tag(ISDF_K_GEMM_EXCHANGE), 0)) != ISDF_OK)
      return st;
  }
  return launch_sum_parts(s, part.as<double>(), (int)probs.size() + slot0, M * N, C);
}

// Universal-grid terms of K C (row-major N x o), added into KC on the plan's
// stream.  The universal domain takes every grid point as a fitting
// function (F = I), E_U = Phi_U C.
//   universal-universal: -dV Phi_U^T Z, Z(R, i) = sum_j E_U(R, j) V[E_j E_i](R),
//     the potentials by batched FFT Poisson solves of the n_occ (n_occ + 1) / 2
//     pair densities (the operator between grid points is never formed);
//   cross (fits made with universal_all_points; W_Uw = (R_U | xi_w) stored):
//     A1 = W_Uw o (E_U E_G^T), A2 = W_Uw o (E_U E_L^T) over the window xi,
//     universal rows -Phi_U^T (A1 E_L + A2 E_N), window rows
//     -(X^L' A1' E_U + X^N' A2' E_U) (the four-term exchange with the
//     universal block of X^N empty).
// Synchronises the stream before returning (its buffers are released).
isdf_status universal_terms(isdf_plan_s* pl, isdf_fit_s* f, const double* C, int o, double* KC, bool cross) {
  HostPlan& hp = pl->hp;
  if (hp.domains.empty() || hp.domains[0].atom >= 0 || hp.domains[0].level != 0 ||
      hp.domains[0].nN != 0) {
    set_error("universal exchange: the plan has no universal domain");
    return ISDF_E_UNSUPPORTED;
  }
  if (f->plan != pl) {
    set_error("universal exchange: fit belongs to another plan");
    return ISDF_E_STATE;
  }
  hipStream_t s = pl->stream;
  const HostDomain& U = hp.domains[0];
  const int64_t ng = level_ng(hp, 0);
  const int n0 = U.nL;
  const int64_t N = hp.n_basis;
  if ((int64_t)U.points.size() != ng || (int64_t)U.funcs.size() != n0) {
    set_error("universal exchange: universal domain does not cover its grid");
    return ISDF_E_STATE;
  }
  const double* Phi = f->phi.as<double>() + pl->phi_off[0];  // ng x n0, column-major
  const int32_t* funcs = pl->d_funcs.as<int32_t>() + pl->func_off[0];
  const int64_t P = (int64_t)o * (o + 1) / 2;
  const int64_t m = f->nmu;
  cross = cross && m > 0;
  // pair potentials are held for tiles of pair rows [a0, a1) within a
  // budget (universal_tile_mb, else the smaller of 16 GB and 40 % of the
  // free memory); a tile holds at least one row
  double avail = 0.0;
  {
    const isdf_status sa = plan_available(pl, AVAIL_UNIVERSAL, &avail);
    if (sa != ISDF_OK) return sa;
  }
  const double v_budget = pl->opts.universal_tile_mb > 0 ? (double)pl->opts.universal_tile_mb * (1 << 20)
                                                         : std::min(16e9, 0.4 * avail);
  std::vector<std::pair<int, int>> tiles;
  int64_t tile_max = 0;
  for (int a0 = 0; a0 < o;) {
    int a1 = a0;
    int64_t np = 0;
    while (a1 < o && (a1 == a0 || (double)(np + (o - a1)) * ng * 8.0 <= v_budget)) np += o - a1++;
    tiles.emplace_back(a0, a1);
    tile_max = std::max(tile_max, np);
    a0 = a1;
  }
  // pair densities per FFT batch: complex work arrays of at most ~1 GB each
  const int64_t per_pair = 16 * ng;
  int64_t ncb = 2 * std::max<int64_t>(1, std::min<int64_t>(65535, (int64_t)1e9 / per_pair));
  ncb = std::min<int64_t>(ncb, tile_max + (tile_max & 1));
  isdf_status st;
  DevBuf C0, E, V, Z, KC0, zf, zc, dpairs, A1, A2, Z1U, Z1w, Z2w;
  if ((st = C0.alloc(sizeof(double) * n0 * o)) != ISDF_OK || (st = E.alloc(sizeof(double) * ng * o)) != ISDF_OK ||
      (st = Z.alloc(sizeof(double) * ng * o)) != ISDF_OK || (st = KC0.alloc(sizeof(double) * n0 * o)) != ISDF_OK ||
      (st = V.alloc(sizeof(double) * tile_max * ng)) != ISDF_OK ||
      (st = zf.alloc(sizeof(double) * ng * ncb)) != ISDF_OK || (st = zc.alloc(sizeof(double) * ng * ncb)) != ISDF_OK)
    return st;
  if (cross && ((st = A1.alloc(sizeof(double) * ng * m)) != ISDF_OK ||
                (st = A2.alloc(sizeof(double) * ng * m)) != ISDF_OK ||
                (st = Z1U.alloc(sizeof(double) * ng * o)) != ISDF_OK ||
                (st = Z1w.alloc(sizeof(double) * m * o)) != ISDF_OK ||
                (st = Z2w.alloc(sizeof(double) * m * o)) != ISDF_OK))
    return st;
  std::vector<int32_t> pairs((size_t)(2 * P));
  for (int64_t a = 0, p = 0; a < o; ++a)
    for (int64_t b = a; b < o; ++b, ++p) {
      pairs[2 * p] = (int32_t)a;
      pairs[2 * p + 1] = (int32_t)b;
    }
  if ((st = upload(dpairs, pairs)) != ISDF_OK) return st;  // all pairs, row by row
  auto gemm = [&](int epi, const double* A, int64_t lda, int tA, const double* B, int64_t ldb, int tB, double* Cm,
                  int64_t ldc, int64_t M, int64_t Nn, int64_t Kk, double alpha, double beta, const double* Ep,
                  int64_t lde) {
    GemmProblem p{};
    p.A = A; p.lda = lda; p.transA = tA;
    p.B = B; p.ldb = ldb; p.transB = tB;
    p.C = Cm; p.ldc = ldc;
    p.E = Ep; p.lde = lde;
    p.M = (int)M; p.N = (int)Nn; p.K = (int)Kk;
    p.alpha = alpha; p.beta = beta;
    return gemm_prof(pl, ISDF_K_GEMM_EXCHANGE, epi, p);
  };
  // E_U = Phi_U C(funcs, :)
  if ((st = launch_gather_rows_t(s, C, o, funcs, n0, C0.as<double>())) != ISDF_OK) return st;
  if ((st = gemm(EPI_AXPBY, Phi, ng, 0, C0.as<double>(), n0, 0, E.as<double>(), ng, ng, o, n0, 1.0, 0.0, nullptr,
                 0)) != ISDF_OK)
    return st;
  if (cross) {
    const double* EG = f->EG.as<double>();
    const double* EL = f->EL.as<double>();
    const double* EN = f->EN.as<double>();
    const double* W = f->WUw.as<double>();
    if ((st = gemm(EPI_HADAMARD, E.as<double>(), ng, 0, EG, m, 1, A1.as<double>(), ng, ng, m, o, 1.0, 0.0, W,
                   ng)) != ISDF_OK ||
        (st = gemm(EPI_HADAMARD, E.as<double>(), ng, 0, EL, m, 1, A2.as<double>(), ng, ng, m, o, 1.0, 0.0, W,
                   ng)) != ISDF_OK)
      return st;
    if ((st = gemm(EPI_AXPBY, A1.as<double>(), ng, 0, EL, m, 0, Z1U.as<double>(), ng, ng, o, m, 1.0, 0.0, nullptr,
                   0)) != ISDF_OK ||
        (st = gemm(EPI_AXPBY, A2.as<double>(), ng, 0, EN, m, 0, Z1U.as<double>(), ng, ng, o, m, 1.0, 1.0, nullptr,
                   0)) != ISDF_OK)
      return st;
    if ((st = gemm_split_k(pl, A1.as<double>(), ng, 1, E.as<double>(), ng, 0, Z1w.as<double>(), m, o, ng, 1.0,
                           false)) != ISDF_OK ||
        (st = gemm_split_k(pl, A2.as<double>(), ng, 1, E.as<double>(), ng, 0, Z2w.as<double>(), m, o, ng, 1.0,
                           false)) != ISDF_OK)
      return st;
    // (K C)^T += -(Z1w' X^L + Z2w' X^N): window rows of the cross terms
    if ((st = gemm_split_k(pl, Z1w.as<double>(), m, 1, f->XL.as<double>(), m, 0, KC, o, N, m, -1.0, true)) !=
            ISDF_OK ||
        (st = gemm_split_k(pl, Z2w.as<double>(), m, 1, f->XN.as<double>(), m, 0, KC, o, N, m, -1.0, true)) !=
            ISDF_OK)
      return st;
  }
  // per tile of pair rows: potentials of its pair densities, batch by
  // batch, into V (column q = the tile's pair q), then their part of Z
  const int* g0 = hp.grid[0];
  if ((st = launch_fill(s, Z.as<double>(), ng * o, 0.0)) != ISDF_OK) return st;
  for (const auto& t : tiles) {
    const int a0 = t.first, a1 = t.second;
    const int64_t first = (int64_t)a0 * o - (int64_t)a0 * (a0 - 1) / 2;  // pair index of (a0, a0)
    const int64_t np = (int64_t)(a1 - a0) * o - ((int64_t)a1 * (a1 - 1) - (int64_t)a0 * (a0 - 1)) / 2;
    for (int64_t q0 = 0; q0 < np; q0 += ncb) {
      const int nc = (int)std::min<int64_t>(ncb, np - q0);
      const int npc = (nc + 1) / 2;
      double* vout = V.as<double>() + q0 * ng;
      if ((st = launch_pair_density(s, E.as<double>(), ng, dpairs.as<int32_t>() + 2 * (first + q0), nc,
                                    zf.as<double>())) != ISDF_OK)
        return st;
      if ((st = fft_prof(pl, zf.as<double>(), npc, g0, -1)) != ISDF_OK) return st;
      bool fused = false;
      if ((st = fft_poisson_inverse(s, zf.as<double>(), g0, zc.as<double>(), g0, npc, pl->recip, vout, nc,
                                    &fused)) != ISDF_OK)
        return st;
      if (!fused) {
        if ((st = launch_poisson_restrict(s, zf.as<double>(), g0, zc.as<double>(), g0, npc, pl->recip)) != ISDF_OK)
          return st;
        if ((st = fft_prof(pl, zc.as<double>(), npc, g0, +1)) != ISDF_OK) return st;
        if ((st = launch_split_planar(s, zc.as<double>(), ng, nc, vout)) != ISDF_OK) return st;
      }
    }
    if ((st = launch_z_accumulate_rows(s, E.as<double>(), V.as<double>(), ng, o, a0, a1, Z.as<double>())) !=
        ISDF_OK)
      return st;
  }
  // universal rows: -Phi_U^T (dV Z_UU + A1 E_L + A2 E_N)
  const double dV = hp.volume / (double)ng;
  if ((st = launch_scale_copy(s, Z.as<double>(), Z.as<double>(), ng * o, dV)) != ISDF_OK) return st;
  if (cross && (st = launch_add(s, Z.as<double>(), Z1U.as<double>(), Z.as<double>(), ng * o)) != ISDF_OK) return st;
  if ((st = gemm_split_k(pl, Phi, ng, 1, Z.as<double>(), ng, 0, KC0.as<double>(), n0, o, ng, -1.0, false)) !=
      ISDF_OK)
    return st;
  if ((st = launch_scatter_add_rows(s, KC0.as<double>(), n0, o, funcs, KC)) != ISDF_OK) return st;
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  return ISDF_OK;
}

// isdf_exchange_universal: the universal-universal block alone.
isdf_status universal_exchange(isdf_plan_s* pl, isdf_fit_s* f, const double* C, int o, double* KC,
                               double* e_x) {
  MemScope mscope(pl->mem);
  hipStream_t s = pl->stream;
  const int64_t N = pl->hp.n_basis;
  isdf_status st;
  DevBuf partial, out;
  if ((st = partial.alloc(sizeof(double) * 1024)) != ISDF_OK || (st = out.alloc(sizeof(double))) != ISDF_OK)
    return st;
  if ((st = launch_fill(s, KC, N * o, 0.0)) != ISDF_OK) return st;
  if ((st = universal_terms(pl, f, C, o, KC, false)) != ISDF_OK) return st;
  if ((st = launch_trace_dot(s, C, KC, N * o, partial.as<double>(), 1024, out.as<double>())) != ISDF_OK) return st;
  double ex = 0.0;
  ISDF_HIP_TRY(hipMemcpyAsync(&ex, out.p, sizeof(double), hipMemcpyDeviceToHost, s));
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  if (e_x) *e_x = ex;
  if (!std::isfinite(ex)) {
    set_error("isdf_exchange_universal: non-finite energy (NaN or Inf in C?)");
    return ISDF_E_ARG;
  }
  return ISDF_OK;
}

// ri: occ-RI output (exchange_enqueue_ri), else the full K.
isdf_status exchange_run(isdf_plan_s* plan, isdf_fit_s* fit, const double* in, int n_occ, double* K,
                         double* e_x, bool ri = false) {
  if (fit->plan != plan) {
    set_error("isdf_exchange: fit belongs to another plan");
    return ISDF_E_STATE;
  }
  if (fit->all_points && !ri) {
    set_error("isdf_exchange: a fit with every universal point a fitting function gives K C only "
              "(isdf_exchange_occ_ri)");
    return ISDF_E_UNSUPPORTED;
  }
  MemScope mscope(plan->mem);
  hipStream_t s = plan->stream;
  isdf_status st;
  if ((st = exchange_prepare(plan, fit, n_occ, ri)) != ISDF_OK) return st;
  auto enqueue = [&](bool stage_event) {
    return ri ? exchange_enqueue_ri(plan, fit, in, n_occ, K, stage_event)
              : exchange_enqueue(plan, fit, in, n_occ, K, stage_event);
  };
  const bool graph = plan->opts.eager_exchange == 0 && !((plan->prof >> ISDF_K_GEMM_EXCHANGE) & 1) &&
                     !plan->tuning && !fit->all_points;
  if (graph && (!fit->xexec || fit->xkey_in != in || fit->xkey_out != K || fit->xkey_nocc != n_occ ||
                fit->xkey_ri != ri)) {
    fit->drop_graph();
    if (!plan->cap_stream)
      ISDF_HIP_TRY(hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking));
    // recorded on the private stream (capture needs a non-null one), replayed on the plan's
    ISDF_HIP_TRY(hipStreamSynchronize(s));
    plan->stream = plan->cap_stream;
    hipError_t e = hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
      plan->stream = s;
      set_error(std::string("isdf_exchange: graph capture: ") + hipGetErrorString(e));
      return ISDF_E_HIP;
    }
    st = enqueue(false);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(plan->cap_stream, &g);
    plan->stream = s;
    if (st != ISDF_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      if (st == ISDF_OK) {
        set_error(std::string("isdf_exchange: graph capture: ") + hipGetErrorString(e));
        st = ISDF_E_HIP;
      }
      return st;
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      set_error(std::string("isdf_exchange: graph instantiate: ") + hipGetErrorString(e));
      return ISDF_E_HIP;
    }
    fit->xgraph = g;
    fit->xexec = x;
    fit->xkey_in = in;
    fit->xkey_out = K;
    fit->xkey_nocc = n_occ;
    fit->xkey_ri = ri;
  }
  ISDF_HIP_TRY(hipEventRecord(plan->ev[0], s));
  if (graph) {
    ISDF_HIP_TRY(hipGraphLaunch(fit->xexec, s));
  } else {
    if ((st = enqueue(true)) != ISDF_OK) return st;
    if (fit->all_points) {  // the window terms are in K C: add the universal ones
      if ((st = universal_terms(plan, fit, in, n_occ, K, true)) != ISDF_OK) return st;
      if ((st = launch_trace_dot(s, in, K, plan->hp.n_basis * n_occ, fit->partial.as<double>(), 1024,
                                 fit->ex_out.as<double>())) != ISDF_OK)
        return st;
    }
  }
  ISDF_HIP_TRY(hipEventRecord(plan->ev[2], s));
  double ex = 0.0;
  ISDF_HIP_TRY(hipMemcpyAsync(&ex, fit->ex_out.p, sizeof(double), hipMemcpyDeviceToHost, s));
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  prof_collect(plan);
  float ms;
  ISDF_HIP_TRY(hipEventElapsedTime(&ms, plan->ev[0], plan->ev[2]));
  plan->stage_ms[6] = ms;
  if (!graph) ISDF_HIP_TRY(hipEventElapsedTime(&ms, plan->ev[0], plan->ev[1]));
  plan->stage_ms[7] = ms;  // with a graph: the whole exchange
  if (e_x) *e_x = ex;
  if (!std::isfinite(ex)) {
    set_error("isdf_exchange: non-finite exchange energy (NaN or Inf in the density?)");
    return ISDF_E_ARG;
  }
  return ISDF_OK;
}

}  // namespace

// ====================================================================== C ABI
// ---------------------------------------------------------------------------
// Exchange with no device allocation (isdf_exchange_occ_ri_noalloc): the
// FP64 occ-RI workspace lives in this file-scope array, one copy per GPU,
// held until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is a stand-in, not a device address): each device's
// address comes from hipGetSymbolAddress, taken once with that device
// current, and only that address is used.  Every call on a GPU shares its
// array, so calls that overlap on one GPU race.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(ISDF_NOALLOC_SCRATCH_MB) << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;  // device -> address of its copy of `scratch`

isdf_status scratch_address(void** out) {
  int dev = -1;
  ISDF_HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it == g_scratch_addr.end()) {
    void* p = nullptr;
    ISDF_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("isdf_exchange_occ_ri_noalloc: no device address for the scratch array");
      return ISDF_E_HIP;
    }
    it = g_scratch_addr.emplace(dev, p).first;
  }
  *out = it->second;
  return ISDF_OK;
}

// Bytes of the FP64 occ-RI workspace for N_mu points and n_occ orbitals
// (every part rounded up to 256 bytes).
size_t noalloc_bytes(int64_t nmu, int64_t o) {
  auto r = [](size_t b) { return (b + 255) / 256 * 256; };
  return 5 * r(sizeof(double) * nmu * o) + 3 * r(sizeof(double) * nmu * nmu) + r(sizeof(double) * 1024) +
         r(sizeof(double));
}

extern "C" {

const char* isdf_last_error(void) { return g_err.c_str(); }
const char* isdf_version(void) { return "isdf-mi355x 0.1 (gfx950)"; }

isdf_status isdf_grids_for_threshold(const double* lattice, int32_t n_shells,
                                     const double* shell_alpha, int32_t n_levels,
                                     const double* alpha_bound, double eps_K, int32_t* grid_out) {
  return threshold_grids(lattice, n_shells, shell_alpha, n_levels, alpha_bound, eps_K, grid_out);
}

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
  if (pl->opts.precision != ISDF_FP64 && pl->opts.precision != ISDF_MIXED_X3 &&
      pl->opts.precision != ISDF_MIXED_X6) {
    set_error("isdf_plan: unknown precision");
    return ISDF_E_ARG;
  }
  if (pl->opts.universal_tile_mb < 0) {
    set_error("isdf_plan: universal_tile_mb must not be negative");
    return ISDF_E_ARG;
  }
  if (!(pl->opts.ri_screen_tau >= 0.0)) {
    set_error("isdf_plan: ri_screen_tau must be >= 0");
    return ISDF_E_ARG;
  }
  if (pl->opts.ri_screen_tau > 0.0 && pl->opts.precision != ISDF_FP64 &&
      (pl->opts.mixed_mask == 0 || (pl->opts.mixed_mask & ISDF_MIX_EXCHANGE))) {
    set_error("isdf_plan: ri_screen_tau needs the FP64 exchange (a mixed plan without mixed_mask bit 2)");
    return ISDF_E_UNSUPPORTED;
  }
  if (pl->opts.phi_budget_mb < 0 || pl->opts.ri_rows < 0) {
    set_error("isdf_plan: phi_budget_mb and ri_rows must not be negative");
    return ISDF_E_ARG;
  }
  if (pl->opts.w_storage != ISDF_W_F64 && pl->opts.w_storage != ISDF_W_F32) {
    set_error("isdf_plan: w_storage must be ISDF_W_F64 or ISDF_W_F32");
    return ISDF_E_ARG;
  }
  if (pl->opts.mixed_mask < 0 || pl->opts.mixed_mask > 7) {
    set_error("isdf_plan: mixed_mask must be within 0..7");
    return ISDF_E_ARG;
  }
  if (pl->opts.selector == ISDF_SEL_MLP) {
    if (!pl->opts.mlp_weights || !(pl->opts.mlp_keep >= 1.0)) {
      set_error("isdf_plan: the learned selector needs weights and mlp_keep >= 1");
      return ISDF_E_ARG;
    }
    pl->mlp_w.assign(pl->opts.mlp_weights, pl->opts.mlp_weights + MLP_NPARAM);
    for (float v : pl->mlp_w)
      if (!std::isfinite(v)) {
        set_error("isdf_plan: non-finite network weight");
        return ISDF_E_ARG;
      }
    pl->opts.mlp_weights = nullptr;
  } else if (pl->opts.selector != ISDF_SEL_FULL) {
    set_error("isdf_plan: unknown selector");
    return ISDF_E_ARG;
  }
  if (pl->opts.tune_file) {
    if ((st = read_tune_file(pl->opts.tune_file, pl->tune)) != ISDF_OK) return st;
    pl->opts.tune_file = nullptr;  // not kept: the caller owns the string
  }
  if (pl->opts.universal_all_points) {
    HostPlan& hp = pl->hp;
    if (hp.domain_mode != 0 || hp.domains.size() < 2 || hp.domains[0].atom >= 0 ||
        hp.domains[0].level != 0) {
      set_error("isdf_plan: universal_all_points needs a universal domain and atom windows "
                "(a one-level plan: isdf_exchange_universal)");
      return ISDF_E_UNSUPPORTED;
    }
    hp.n_mu_total -= hp.domains[0].n_mu;
    hp.domains[0].n_mu = 0;  // no interpolation points: every grid point is a fitting function
  }
  pl->stream = static_cast<hipStream_t>(pl->opts.stream);
  pl->mem = std::make_shared<MemCtx>();
  pl->mem->stream = pl->stream;
  if (pl->opts.workspace || pl->opts.workspace_bytes) {
    if (!pl->opts.workspace || pl->opts.workspace_bytes < 4096 ||
        (reinterpret_cast<uintptr_t>(pl->opts.workspace) & 255)) {
      set_error("isdf_plan: a workspace needs a 256-byte aligned pointer and at least 4096 bytes");
      return ISDF_E_ARG;
    }
    pl->mem->set_arena(pl->opts.workspace, pl->opts.workspace_bytes);
  }
  *out = pl.release();
  return ISDF_OK;
}

isdf_status isdf_plan_workspace_bytes(isdf_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) {
    set_error("isdf_plan_workspace_bytes: null argument");
    return ISDF_E_ARG;
  }
  *bytes = plan->mem ? plan->mem->peak : 0;
  return ISDF_OK;
}

isdf_status isdf_plan_alloc_stats(isdf_plan_t plan, int64_t* calls, double* bytes, double* ms) {
  if (!plan) {
    set_error("isdf_plan_alloc_stats: null plan");
    return ISDF_E_ARG;
  }
  if (calls) *calls = plan->mem->n_new;
  if (bytes) *bytes = plan->mem->new_bytes;
  if (ms) *ms = plan->mem->new_ms;
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
  return do_fit(plan, nullptr, nullptr, nullptr, nullptr, out);
}

isdf_status isdf_fit_batch(const isdf_plan_t* plans, int32_t n, int32_t max_concurrent,
                           isdf_fit_t* fits, isdf_status* statuses) {
  if (!plans || !fits || n < 0) {
    set_error("isdf_fit_batch: null plans/fits or n < 0");
    return ISDF_E_ARG;
  }
  for (int i = 0; i < n; ++i) {
    fits[i] = nullptr;
    if (statuses) statuses[i] = ISDF_OK;
  }
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) {
      set_error("isdf_fit_batch: null plan " + std::to_string(i));
      return ISDF_E_ARG;
    }
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) {
        set_error("isdf_fit_batch: plan " + std::to_string(i) + " appears twice");
        return ISDF_E_ARG;
      }
  }
  if (n == 0) return ISDF_OK;
  int dev = 0;
  ISDF_HIP_TRY(hipGetDevice(&dev));
  // plans on the null stream get a private stream for the call (the null
  // stream would serialise them)
  std::vector<hipStream_t> own(n, nullptr);
  for (int i = 0; i < n; ++i)
    if (!plans[i]->stream) {
      hipError_t e = hipStreamCreateWithFlags(&own[i], hipStreamNonBlocking);
      if (e != hipSuccess) {
        for (int j = 0; j < i; ++j)
          if (own[j]) {
            plans[j]->stream = nullptr;
            plans[j]->mem->stream = nullptr;
            (void)hipStreamDestroy(own[j]);
          }
        set_error(std::string("isdf_fit_batch: stream: ") + hipGetErrorString(e));
        return ISDF_E_HIP;
      }
      plans[i]->stream = own[i];
      plans[i]->mem->stream = own[i];
    }
  // largest first, so that the long fits start early
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return plans[a]->hp.n_mu_total > plans[b]->hp.n_mu_total;
  });
  std::vector<isdf_status> sts(n, ISDF_OK);
  std::vector<std::string> msg(n);
  std::atomic<int> next(0);
  auto worker = [&]() {
    // a worker that cannot select the caller's device takes no plan (the
    // others take them all; if none can, every plan reports the error)
    const hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return;
    }
    for (int k; (k = next.fetch_add(1)) < n;) {
      const int i = order[k];
      sts[i] = do_fit(plans[i], nullptr, nullptr, nullptr, nullptr, &fits[i]);
      if (sts[i] != ISDF_OK) msg[i] = g_err;
    }
  };
  const int nt = std::max(1, std::min(n, max_concurrent > 0 ? (int)max_concurrent : 4));
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
  for (int k = next.load(); k < n; ++k) {  // never started: no worker could select the device
    const int i = order[k];
    sts[i] = ISDF_E_HIP;
    msg[i] = "no worker thread could select device " + std::to_string(dev);
  }
  for (int i = 0; i < n; ++i)
    if (own[i]) {
      (void)hipStreamSynchronize(own[i]);
      plans[i]->stream = nullptr;
      plans[i]->mem->stream = nullptr;
      (void)hipStreamDestroy(own[i]);
    }
  isdf_status first = ISDF_OK;
  for (int i = 0; i < n; ++i) {
    if (statuses) statuses[i] = sts[i];
    if (sts[i] != ISDF_OK && first == ISDF_OK) {
      first = sts[i];
      set_error("isdf_fit_batch: plan " + std::to_string(i) + ": " + msg[i]);
    }
  }
  return first;
}

isdf_status isdf_fit_with_points(isdf_plan_t plan, const int64_t* local_points, isdf_fit_t* out) {
  if (out) *out = nullptr;
  if (!local_points) {
    set_error("isdf_fit_with_points: null points");
    return ISDF_E_ARG;
  }
  return do_fit(plan, local_points, nullptr, nullptr, nullptr, out);
}

isdf_status isdf_fit_with_candidates(isdf_plan_t plan, const int64_t* candidates,
                                     const int64_t* n_candidates, isdf_fit_t* out) {
  if (out) *out = nullptr;
  if (!candidates || !n_candidates) {
    set_error("isdf_fit_with_candidates: null candidates");
    return ISDF_E_ARG;
  }
  return do_fit(plan, nullptr, candidates, n_candidates, nullptr, out);
}

isdf_status isdf_fit_selection(isdf_fit_t fit, int64_t* n_candidates, double* last_residual,
                               double* final_residual, int32_t* fallback) {
  if (!fit) {
    set_error("isdf_fit_selection: null fit");
    return ISDF_E_ARG;
  }
  const size_t nd = fit->count.size();
  for (size_t d = 0; d < nd; ++d) {
    if (n_candidates) n_candidates[d] = fit->ncand.size() == nd ? fit->ncand[d] : 0;
    if (last_residual) last_residual[d] = fit->dlast.size() == nd ? fit->dlast[d] : 0.0;
    if (final_residual) final_residual[d] = fit->dfinal.size() == nd ? fit->dfinal[d] : 0.0;
    if (fallback) fallback[d] = fit->fallback.size() == nd ? fit->fallback[d] : 0;
  }
  return ISDF_OK;
}

isdf_status isdf_fit_features(isdf_fit_t fit, float* features_dev, float* labels_dev,
                              int64_t capacity, int64_t* n) {
  if (!fit) {
    set_error("isdf_fit_features: null fit");
    return ISDF_E_ARG;
  }
  isdf_plan_s* pl = fit->plan;
  if (n) *n = pl->pts_total;
  if (!features_dev) return ISDF_OK;  // size query
  MemScope mscope(pl->mem);
  if (capacity < pl->pts_total) {
    set_error("isdf_fit_features: capacity below the number of points");
    return ISDF_E_ARG;
  }
  isdf_status st = compute_features(pl, fit, features_dev);
  if (st != ISDF_OK) return st;
  if (labels_dev) {
    std::vector<float> lab(pl->pts_total, 0.f);
    const int nd = (int)pl->hp.domains.size();
    // needed set: initial diagonal >= (1 - tie_tol) x residual of the last pivot
    std::vector<double> dg(pl->pts_total);
    ISDF_HIP_TRY(hipStreamSynchronize(pl->stream));
    ISDF_HIP_TRY(hipMemcpy(dg.data(), fit->diag0.p, sizeof(double) * pl->pts_total, hipMemcpyDeviceToHost));
    for (int d = 0; d < nd; ++d) {
      const double thr = (1.0 - pl->hp.tie_tol) * fit->dlast[d];
      const int64_t np = (int64_t)pl->hp.domains[d].points.size();
      for (int64_t i = 0; i < np; ++i) lab[pl->pts_off[d] + i] = dg[pl->pts_off[d] + i] >= thr ? 1.f : 0.f;
    }
    ISDF_HIP_TRY(hipMemcpy(labels_dev, lab.data(), sizeof(float) * lab.size(), hipMemcpyHostToDevice));
  }
  return ISDF_OK;
}

isdf_status isdf_mlp_forward(const float* weights, const float* features_dev, int64_t n,
                             float* scores_dev, void* stream) {
  if (!weights || !features_dev || !scores_dev || n < 0) {
    set_error("isdf_mlp_forward: bad argument");
    return ISDF_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBuf w;
  isdf_status st;
  if ((st = upload(w, std::vector<float>(weights, weights + MLP_NPARAM))) != ISDF_OK) return st;
  if ((st = launch_mlp_forward(s, w.as<float>(), features_dev, n, scores_dev)) != ISDF_OK) return st;
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  return ISDF_OK;
}

isdf_status isdf_mlp_loss_grad(const float* weights, const float* features_dev,
                               const float* labels_dev, int64_t n, float pos_weight, float* grad,
                               float* loss, void* stream) {
  if (!weights || !features_dev || !labels_dev || n <= 0) {
    set_error("isdf_mlp_loss_grad: bad argument");
    return ISDF_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  isdf_status st;
  DevBuf w, part, lpart, g, l;
  const int64_t nblk = (n + 31) / 32;
  if ((st = upload(w, std::vector<float>(weights, weights + MLP_NPARAM))) != ISDF_OK) return st;
  if ((st = part.alloc(sizeof(float) * nblk * MLP_NPARAM)) != ISDF_OK) return st;
  if ((st = lpart.alloc(sizeof(float) * nblk)) != ISDF_OK) return st;
  if ((st = g.alloc(sizeof(float) * MLP_NPARAM)) != ISDF_OK) return st;
  if ((st = l.alloc(sizeof(float))) != ISDF_OK) return st;
  if ((st = launch_mlp_grad(s, w.as<float>(), features_dev, labels_dev, nullptr, 0, n, pos_weight,
                            1.0f / (float)n, part.as<float>(), lpart.as<float>(), g.as<float>(),
                            l.as<float>())) != ISDF_OK)
    return st;
  float lh = 0.f;
  if (grad) ISDF_HIP_TRY(hipMemcpyAsync(grad, g.p, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, s));
  ISDF_HIP_TRY(hipMemcpyAsync(&lh, l.p, sizeof(float), hipMemcpyDeviceToHost, s));
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  if (loss) *loss = lh / (float)n;
  return ISDF_OK;
}

isdf_status isdf_mlp_train(const float* features_dev, const float* labels_dev, int64_t n,
                           const isdf_mlp_config* cfg, float* weights, float* epoch_loss) {
  if (!features_dev || !labels_dev || !cfg || !weights || n <= 0 || cfg->epochs <= 0 ||
      cfg->batch <= 0) {
    set_error("isdf_mlp_train: bad argument");
    return ISDF_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(cfg->stream);
  isdf_status st;
  float pw = cfg->pos_weight;
  if (!(pw > 0.f)) {
    std::vector<float> lab(n);
    ISDF_HIP_TRY(hipMemcpy(lab.data(), labels_dev, sizeof(float) * n, hipMemcpyDeviceToHost));
    double pos = 0.0;
    for (float v : lab) pos += v;
    pw = pos > 0.0 ? (float)((n - pos) / pos) : 1.f;
  }
  const int64_t B = std::min<int64_t>(cfg->batch, n);
  const int64_t nblk = (B + 31) / 32;
  const int64_t nbatch = (n + B - 1) / B;
  DevBuf w, m, v, g, part, lpart, lbuf, perm;
  if ((st = upload(w, std::vector<float>(weights, weights + MLP_NPARAM))) != ISDF_OK) return st;
  if ((st = upload(m, std::vector<float>(MLP_NPARAM, 0.f))) != ISDF_OK) return st;
  if ((st = upload(v, std::vector<float>(MLP_NPARAM, 0.f))) != ISDF_OK) return st;
  if ((st = g.alloc(sizeof(float) * MLP_NPARAM)) != ISDF_OK) return st;
  if ((st = part.alloc(sizeof(float) * nblk * MLP_NPARAM)) != ISDF_OK) return st;
  if ((st = lpart.alloc(sizeof(float) * nblk)) != ISDF_OK) return st;
  if ((st = lbuf.alloc(sizeof(float) * nbatch)) != ISDF_OK) return st;
  if ((st = perm.alloc(sizeof(int32_t) * n)) != ISDF_OK) return st;
  std::vector<int32_t> hp(n);
  uint64_t state = 0x9E3779B97F4A7C15ull ^ (uint64_t)cfg->seed;
  auto next = [&]() {  // splitmix64
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  int t = 0;
  std::vector<float> lb(nbatch);
  for (int ep = 0; ep < cfg->epochs; ++ep) {
    for (int64_t i = 0; i < n; ++i) hp[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) std::swap(hp[i], hp[(int64_t)(next() % (uint64_t)(i + 1))]);
    ISDF_HIP_TRY(hipMemcpyAsync(perm.p, hp.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    for (int64_t b = 0; b < nbatch; ++b) {
      const int64_t b0 = b * B, bn = std::min(B, n - b0);
      if ((st = launch_mlp_grad(s, w.as<float>(), features_dev, labels_dev, perm.as<int32_t>(), b0, bn,
                                pw, 1.0f / (float)bn, part.as<float>(), lpart.as<float>(),
                                g.as<float>(), lbuf.as<float>() + b)) != ISDF_OK)
        return st;
      if ((st = launch_adam(s, w.as<float>(), g.as<float>(), m.as<float>(), v.as<float>(), cfg->lr,
                            cfg->beta1, cfg->beta2, cfg->eps, ++t)) != ISDF_OK)
        return st;
    }
    ISDF_HIP_TRY(hipMemcpyAsync(lb.data(), lbuf.p, sizeof(float) * nbatch, hipMemcpyDeviceToHost, s));
    ISDF_HIP_TRY(hipStreamSynchronize(s));
    double tot = 0.0;
    for (float x : lb) tot += x;
    if (epoch_loss) epoch_loss[ep] = (float)(tot / (double)n);
  }
  ISDF_HIP_TRY(hipMemcpy(weights, w.p, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost));
  return ISDF_OK;
}

isdf_status isdf_fit_screen_stats(isdf_fit_t fit, double* kept_fraction) {
  if (!fit || !kept_fraction) {
    set_error("isdf_fit_screen_stats: null argument");
    return ISDF_E_ARG;
  }
  if (!fit->s_ran || fit->s_nt <= 0) {
    set_error("isdf_fit_screen_stats: no screened exchange has run on this fit");
    return ISDF_E_STATE;
  }
  const size_t nn = (size_t)fit->s_nt * fit->s_nt;
  std::vector<uint8_t> h(nn);
  ISDF_HIP_TRY(hipStreamSynchronize(fit->plan->stream));
  size_t kept = 0;
  for (DevBuf* d : {&fit->s_mgg, &fit->s_mgl, &fit->s_mll}) {
    ISDF_HIP_TRY(hipMemcpy(h.data(), d->p, nn, hipMemcpyDeviceToHost));
    for (uint8_t v : h) kept += v;
  }
  *kept_fraction = (double)kept / (3.0 * (double)nn);
  return ISDF_OK;
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
      if (fit->phi_streamed) {
        set_error("isdf_fit_get: the fit streamed its basis values by domain group and kept none");
        return ISDF_E_STATE;
      }
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
      need = sizeof(double) * fit->nmu * fit->nmu;
      if (fit->w32) {  // widen the stored FP32 values
        if (bytes != need) break;
        std::vector<float> t((size_t)(fit->nmu * fit->nmu));
        ISDF_HIP_TRY(hipStreamSynchronize(pl->stream));
        if (!t.empty())
          ISDF_HIP_TRY(hipMemcpy(t.data(), fit->W32.p, sizeof(float) * t.size(), hipMemcpyDeviceToHost));
        double* o = static_cast<double*>(host_out);
        for (size_t i = 0; i < t.size(); ++i) o[i] = t[i];
        return ISDF_OK;
      }
      src = fit->W.p;
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
      ISDF_HIP_TRY(hipStreamSynchronize(pl->stream));
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
  return exchange_run(plan, fit, D, 0, K, e_x);
}

isdf_status isdf_exchange_occ(isdf_plan_t plan, isdf_fit_t fit, const double* C_occ, int32_t n_occ,
                              double* K, double* e_x) {
  if (!plan || !fit || !C_occ || !K || n_occ < 1) {
    set_error("isdf_exchange_occ: null argument or n_occ < 1");
    return ISDF_E_ARG;
  }
  return exchange_run(plan, fit, C_occ, n_occ, K, e_x);
}

isdf_status isdf_exchange_occ_ri(isdf_plan_t plan, isdf_fit_t fit, const double* C_occ, int32_t n_occ,
                                 double* KC, double* e_x) {
  if (!plan || !fit || !C_occ || !KC || n_occ < 1) {
    set_error("isdf_exchange_occ_ri: null argument or n_occ < 1");
    return ISDF_E_ARG;
  }
  if (n_occ > plan->hp.n_basis) {
    set_error("isdf_exchange_occ_ri: n_occ above the basis size");
    return ISDF_E_ARG;
  }
  return exchange_run(plan, fit, C_occ, n_occ, KC, e_x, true);
}

isdf_status isdf_exchange_occ_ri_noalloc(isdf_plan_t plan, isdf_fit_t fit, const double* C_occ,
                                         int32_t n_occ, double* KC, double* e_x) {
  if (!plan || !fit || !C_occ || !KC || n_occ < 1) {
    set_error("isdf_exchange_occ_ri_noalloc: null argument or n_occ < 1");
    return ISDF_E_ARG;
  }
  if (n_occ > plan->hp.n_basis) {
    set_error("isdf_exchange_occ_ri_noalloc: n_occ above the basis size");
    return ISDF_E_ARG;
  }
  if (fit->plan != plan) {
    set_error("isdf_exchange_occ_ri_noalloc: fit belongs to another plan");
    return ISDF_E_STATE;
  }
  if (fit->all_points) {
    set_error("isdf_exchange_occ_ri_noalloc: fits with every universal point a fitting function "
              "need the allocating isdf_exchange_occ_ri");
    return ISDF_E_UNSUPPORTED;
  }
  const int64_t nmu = fit->nmu, o = n_occ;
  const size_t need = noalloc_bytes(nmu, o);
  if (need > NOALLOC_SCRATCH_BYTES) {
    set_error("isdf_exchange_occ_ri_noalloc: workspace of " + std::to_string(need) +
              " bytes (3 N_mu^2 + 5 N_mu n_occ doubles) exceeds the fixed " +
              std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte scratch array");
    return ISDF_E_ARG;
  }
  void* base = nullptr;
  isdf_status st;
  if ((st = scratch_address(&base)) != ISDF_OK) return st;
  char* p = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    double* q = reinterpret_cast<double*>(p);
    p += (bytes + 255) / 256 * 256;
    return q;
  };
  RiBuffers b{};
  b.EG = take(sizeof(double) * nmu * o);
  b.EL = take(sizeof(double) * nmu * o);
  b.EN = take(sizeof(double) * nmu * o);
  b.Z1 = take(sizeof(double) * nmu * o);
  b.Z2 = take(sizeof(double) * nmu * o);
  b.QGG = take(sizeof(double) * nmu * nmu);
  b.QGL = take(sizeof(double) * nmu * nmu);
  b.QLL = take(sizeof(double) * nmu * nmu);
  double* partial = take(sizeof(double) * 1024);
  double* ex_out = take(sizeof(double));
  hipStream_t s = plan->stream;
  ISDF_HIP_TRY(hipEventRecord(plan->ev[0], s));
  // every buffer is written before it is read (beta = 0 first, the partial
  // sums by the reduction itself), so nothing needs clearing
  if ((st = ri_fp64_products(plan, fit, C_occ, n_occ, KC, b)) != ISDF_OK) return st;
  if ((st = launch_trace_dot(s, C_occ, KC, plan->hp.n_basis * o, partial, 1024, ex_out)) != ISDF_OK) return st;
  ISDF_HIP_TRY(hipEventRecord(plan->ev[2], s));
  double ex = 0.0;
  ISDF_HIP_TRY(hipMemcpyAsync(&ex, ex_out, sizeof(double), hipMemcpyDeviceToHost, s));
  ISDF_HIP_TRY(hipStreamSynchronize(s));
  prof_collect(plan);
  float ms = 0.f;
  ISDF_HIP_TRY(hipEventElapsedTime(&ms, plan->ev[0], plan->ev[2]));
  plan->stage_ms[6] = plan->stage_ms[7] = ms;
  if (e_x) *e_x = ex;
  if (!std::isfinite(ex)) {
    set_error("isdf_exchange_occ_ri_noalloc: non-finite exchange energy (NaN or Inf in C?)");
    return ISDF_E_ARG;
  }
  return ISDF_OK;
}

isdf_status isdf_exchange_universal(isdf_plan_t plan, isdf_fit_t fit, const double* C_occ, int32_t n_occ,
                                    double* KC, double* e_x) {
  if (!plan || !fit || !C_occ || !KC || n_occ < 1) {
    set_error("isdf_exchange_universal: null argument or n_occ < 1");
    return ISDF_E_ARG;
  }
  if (n_occ > plan->hp.n_basis) {
    set_error("isdf_exchange_universal: n_occ above the basis size");
    return ISDF_E_ARG;
  }
  return universal_exchange(plan, fit, C_occ, n_occ, KC, e_x);
}

isdf_status isdf_autotune(isdf_plan_t plan, int32_t n_occ, int32_t reps, const char* json_out) {
  if (!plan || n_occ < 1 || reps < 1) {
    set_error("isdf_autotune: null plan, n_occ < 1 or reps < 1");
    return ISDF_E_ARG;
  }
  const int64_t N = plan->hp.n_basis;
  if (n_occ > N) {
    set_error("isdf_autotune: n_occ above the basis size");
    return ISDF_E_ARG;
  }
  isdf_status st = ISDF_OK;
  plan->tuning = true;
  plan->tune_reps = reps;
  isdf_fit_t fit = nullptr;
  {
    // operands of the exchange shapes: D = I, C = the first n_occ unit vectors
    std::vector<double> hD((size_t)(N * N), 0.0), hC((size_t)(N * n_occ), 0.0);
    for (int64_t i = 0; i < N; ++i) hD[i * N + i] = 1.0;
    for (int64_t i = 0; i < n_occ; ++i) hC[i * n_occ + i] = 1.0;
    DevBuf dD, dC, dK;
    MemScope mscope(plan->mem);
    st = do_fit(plan, nullptr, nullptr, nullptr, nullptr, &fit);
    if (st == ISDF_OK && (st = upload(dD, hD)) == ISDF_OK && (st = upload(dC, hC)) == ISDF_OK &&
        (st = dK.alloc(sizeof(double) * N * N)) == ISDF_OK) {
      st = exchange_run(plan, fit, dD.as<double>(), 0, dK.as<double>(), nullptr);
      if (st == ISDF_OK) st = exchange_run(plan, fit, dC.as<double>(), n_occ, dK.as<double>(), nullptr);
    }
    if (fit) isdf_fit_destroy(fit);
  }
  plan->tuning = false;
  if (st != ISDF_OK) return st;
  if (json_out) return write_tune_file(plan, json_out);
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

isdf_status isdf_profile(isdf_plan_t plan, int32_t family_mask) {
  if (!plan) {
    set_error("isdf_profile: null plan");
    return ISDF_E_ARG;
  }
  ISDF_HIP_TRY(hipStreamSynchronize(plan->stream));
  prof_collect(plan);
  plan->prof = family_mask & ISDF_K_ALL;
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
  for (auto e : plan->crb_ev)
    if (e) (void)hipEventDestroy(e);
  if (plan->crb_host) (void)hipHostFree(plan->crb_host);
  if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
  delete plan;
}

}  // extern "C"
