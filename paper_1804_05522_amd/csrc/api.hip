// Host side of the C ABI: planning of the HODLR trees, device memory,
// kernel launches, refinement policy and the graph-captured time loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <array>
#include <cstdlib>
#include <string>
#include <vector>
#include <map>
#include <mutex>
#include <map>
#include <mutex>
#include <tuple>
#include <functional>



using namespace hfde;

// Per-kernel timing for measurement runs: when a context has timing on,
// every kernel launched through it is bracketed by two HIP events on the
// context's stream, and counts and durations accumulate per kernel until
// read or reset.  The events are resolved when the entry point returns.
struct KTimer {
  hipStream_t stream = nullptr;
  struct Pend {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Pend> pend;
  std::vector<hipEvent_t> pool;
  std::vector<std::string> names;
  std::vector<int64_t> counts;
  std::vector<double> ms;
  hipEvent_t ev() {
    if (pool.empty()) {
      hipEvent_t e = nullptr;
      (void)hipEventCreate(&e);
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  int kind(const char* n) {
    for (size_t i = 0; i < names.size(); ++i)
      if (names[i] == n) return int(i);
    names.emplace_back(n);
    counts.push_back(0);
    ms.push_back(0.0);
    return int(names.size()) - 1;
  }
  void flush() {
    if (pend.empty()) return;
    (void)hipEventSynchronize(pend.back().b);
    for (const Pend& q : pend) {
      float t = 0.0f;
      (void)hipEventElapsedTime(&t, q.a, q.b);
      counts[q.kind] += 1;
      ms[q.kind] += t;
      pool.push_back(q.a);
      pool.push_back(q.b);
    }
    pend.clear();
  }
  void reset() {
    flush();
    names.clear();
    counts.clear();
    ms.clear();
  }
  ~KTimer() {
    flush();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

struct hodlr_ctx_s {
  hipStream_t stream = nullptr;
  int last_arg = 0;
  bool timing = false;
  KTimer timer;
};

static thread_local KTimer* g_timer = nullptr;

// Launch, bracketed by timing events when the calling entry point's context
// has timing on.  Kernel names are the launch expressions.
#define HFDE_LAUNCH(K, ...)                                   \
  do {                                                        \
    KTimer* t_ = g_timer;                                     \
    hipEvent_t a_ = nullptr, b_ = nullptr;                    \
    if (t_) {                                                 \
      a_ = t_->ev();                                          \
      b_ = t_->ev();                                          \
      (void)hipEventRecord(a_, t_->stream);                   \
    }                                                         \
    hipLaunchKernelGGL(K, __VA_ARGS__);                       \
    if (t_) {                                                 \
      (void)hipEventRecord(b_, t_->stream);                   \
      t_->pend.push_back(KTimer::Pend{t_->kind(#K), a_, b_}); \
    }                                                         \
  } while (0)

// Makes the context's timer current for the duration of an entry point.
struct TimerScope {
  KTimer* prev;
  explicit TimerScope(hodlr_ctx c) : prev(g_timer) {
    g_timer = (c && c->timing) ? &c->timer : nullptr;
    if (g_timer) g_timer->stream = c->stream;
  }
  ~TimerScope() {
    if (g_timer) g_timer->flush();
    g_timer = prev;
  }
};

// Transform scratch of hodlr_toeplitz_matvec_noalloc, for callers that cannot
// allocate device memory: one packed column of 2M complex values per problem
// (at most kNoallocScratchBytes in all).  Every GPU the library runs on holds
// its own copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoallocScratchBytes = size_t(16) << 20;
static __device__ __align__(256) double2 scratch[kNoallocScratchBytes / sizeof(double2)];

namespace {

constexpr int kNCF = 16;     // columns per FFT launch group
constexpr int kNCS = 16;     // columns per column block of a multi-column solve launch
constexpr int kNCB = 2;      // column blocks per launch (grid y): 32 columns in one set of launches
constexpr int kFftSmallMax = 13;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct hodlr_mat_s {
  hodlr_ctx ctx = nullptr;
  hodlr_opts opts{};
  int batch = 0;
  int b = 0;
  int Lmax = 0;
  int64_t total_n = 0;
  int64_t total_leaves = 0;
  int64_t total_nodes = 0;
  std::vector<Item> items;
  std::vector<Node> nodes;
  std::vector<WorkUnit> wu_h;
  std::vector<NodeUnit> nu_h;
  DevPtrs P{};
  std::vector<void*> allocs;
  std::vector<size_t> alloc_bytes;
  size_t bytes_device = 0;
  WorkUnit* wu = nullptr;
  NodeUnit* nu = nullptr;
  int nwu = 0, nnu = 0;
  // FFT work lists per column count
  std::vector<int> small_items, big_items;
  FftUnit* fft_small_units = nullptr;   // (item, col) for col < kNCF
  int n_fft_small = 0;
  FftUnit* fft_p1_units = nullptr;
  int n_fft_p1 = 0;
  FftUnit* fft_p2_units = nullptr;
  int n_fft_p2 = 0;
  FftUnit* fft_row_units = nullptr;
  int n_fft_rows = 0;
  size_t fft4_lds = 0;
  int64_t fws_packed = 0;     // complex values of the packed single-column transform scratch (sum of 2M)
  // solve scratch
  double* partL = nullptr;
  double* partU = nullptr;
  double* zL = nullptr;
  double* zU = nullptr;
  double* ytmp = nullptr;     // total_n x (kNCS kNCB)
  int64_t part_block = 0;     // doubles between the column blocks of partL / partU
  int64_t z_block = 0;        // and of zL / zU
  double* rbuf = nullptr;     // total_n x kNCS
  double* dbuf = nullptr;
  double* bbuf = nullptr;
  double* norms = nullptr;    // batch x kNCS x 2
  // per-step convergence check of the time loop
  double* ukeep = nullptr;    // total_n: u at the start of a run of steps (restored on fallback)
  double2* step_part = nullptr;   // batch x step_slices partial sums (d^2, u^2)
  double* step_worst = nullptr;   // batch: worst relative correction of the steps since the last clear
  double* host_worst = nullptr;   // pinned host copy of step_worst
  int step_slices = 0;
  bool has_mass = false;         // some problem is a finite-element operator (E != I)
  // GMRES-IR (opts.gmres_m > 0): basis V (total_n x (kGmMax + 1)), preconditioned
  // vectors Z (total_n x kGmMax), per-problem small arrays
  double* gmV = nullptr;
  double* gmZ = nullptr;
  GmState gms{};
  bool factored = false;
  int max_rank_factors = 0;
  int max_rank_A = 0;
  bool capped_A = false;      // the Hankel compression of some problem hit the rank cap above its tolerance
  // caller-owned device memory (hodlr_build_ws): every buffer is carved from it
  char* ws = nullptr;
  size_t ws_bytes = 0, ws_used = 0;
  size_t ws_sched = 0;        // start of the factorisation schedule's region (re-planned in place)
  bool sizing = false;        // hodlr_workspace_size: buffers are counted, not allocated
  // low precision copies
  float* IL32 = nullptr;
  float* IU32 = nullptr;
  float* LUinv32 = nullptr;
  bf16* IL16 = nullptr;
  bf16* IU16 = nullptr;
  // multi-work-group factorisation schedule
  bool mwg_planned = false;
  int core_threads = kCoreWG;                // launch shapes of the factorisation (tunable)
  int leaf_threads = 512;
  int gram_rows = kGramRows;
  int fuse_rows = kFuseRows;                 // phase A of nodes with children up to this many rows: fused kernels
  int fuse_used = kFuseRows;                 // the threshold the current schedule was planned with
  std::vector<int> mwg_kind;                 // launch kind per record
  std::vector<int> mwg_grid;                 // grid size
  std::vector<int64_t> mwg_off;              // offset into the unit array of its kind
  std::vector<int64_t> mwg_off2;             // secondary offset (tasks / jobs)
  NodeTask* d_tasks = nullptr;
  GramUnit* d_gram = nullptr;
  ReduceUnit* d_red = nullptr;
  int2* d_core = nullptr;
  FormUnit* d_form = nullptr;
  ProdJob* d_jobs = nullptr;
  ProdUnit* d_punits = nullptr;
  double* d_gpart = nullptr;
  double* d_gpart_side = nullptr;            // Gram partials of the second stream's recompressions
  std::vector<char> mwg_side;                // record runs on the second stream
  hipStream_t side = nullptr;                // second stream of the factorisation (default priority)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double* d_G = nullptr;
  double* d_M = nullptr;
  double* d_ppart = nullptr;
  double* d_pz = nullptr;
  // graph of one time step
  hipGraphExec_t step_graph = nullptr;
  const double* graph_u = nullptr;
  const double* graph_f = nullptr;
  int graph_sweeps = -1;
  double graph_fscale = 0.0;
};

constexpr int kLrSlots = 22;   // low-rank work slots of a 2D plan (Grams, transfer matrices, unit lists)

struct fde2d_plan_s {
  hodlr_ctx ctx = nullptr;
  hodlr_mat mat = nullptr;      // 2J shifted problems: x_j = A + q_j I (items 0..J-1), y_j = B + p_j I (J..2J-1)
  hodlr_mat exact = nullptr;    // the unshifted A and B (exact products for the residual)
  int J = 0;
  std::vector<double> p, q;
  std::vector<int> order;   // application order of the shift pairs (interleaved)
  int64_t nx = 0, ny = 0;
  double shift_x = 0.5, shift_y = 0.5;
  double bound_x = 1.0, bound_y = 1.0;   // lower bounds of ||A||_2, ||B||_2: the largest diagonal entries
  // Finite elements: A X E_y + E_x X B^T = C (eq. (sylv-timestepping-fe)),
  // E = mass (I + mc (S + S^T)); mass = 1, mc = 0 for an identity E.
  bool fe = false;
  double mass_x = 1.0, mass_y = 1.0, mc_x = 0.0, mc_y = 0.0;
  double* cz = nullptr;         // E_x [Z_m, F_Z] and E_y [W_m, F_W] (finite elements), (kMaxCat + kRS) columns
  double* cw = nullptr;
  double* ex_mass = nullptr;    // E applied to the exact products' inputs, layout of ex_in
  fde2d_opts opts{};
  std::vector<int> pwu_off, pwu_cnt, pnu_off, pnu_cnt;
  WorkUnit* pair_wu = nullptr;
  NodeUnit* pair_nu = nullptr;
  double* G = nullptr;          // residual factors (nx x 64 / ny x 64)
  double* H = nullptr;
  double* G0 = nullptr;         // right-hand side factors of the current sweep
  double* H0 = nullptr;
  double* Zx[2] = {nullptr, nullptr};   // solution factors, main term (ping-pong)
  double* Zc[2] = {nullptr, nullptr};   // solution factors, sum of the corrections (ping-pong)
  double* Wc[2] = {nullptr, nullptr};
  double* counters = nullptr;   // device: algorithmic flops of the recompression cores (k_lr_core)
  double lrs_flops = 0.0;       // host: algorithmic flops of the dense residual sums (k_lrs_dense)
  double* lrs_cpart = nullptr;  // slice partials of the factored sketch products
  double* lrs_t = nullptr;      // their sums
  double* lrs_part = nullptr;   // per-tile sums of squares of a dense low-rank sum
  double* dnorm = nullptr;      // their total
  double* om = nullptr;         // dense compression: sketch matrix (ny x kSketch)
  double* sk_y = nullptr;       //   sketch X Om (nx x kSketch)
  double* sk_q1 = nullptr;      //   first orthonormal basis
  double* sk_q2 = nullptr;      //   second orthonormal basis
  double* sk_b = nullptr;       //   X^T Q2 (ny x kSketch)
  double* eye = nullptr;        //   kSketch x kSketch identity
  double* sk_junk = nullptr;    //   unused right factor of the orthonormalising passes
  double* Wx[2] = {nullptr, nullptr};
  double* Zd[2] = {nullptr, nullptr};   // correction factors (even shift pairs of a sweep, then the merge)
  double* Ze[2] = {nullptr, nullptr};   // correction factors of the odd shift pairs
  double* We[2] = {nullptr, nullptr};
  double* Wd[2] = {nullptr, nullptr};
  double* R1 = nullptr;         // residual recompression temporaries
  double* R1w = nullptr;
  double* xin = nullptr;        // (total rows of mat) x 64 solve workspace
  double* ex_in = nullptr;      // (nx + ny) x 64 for the exact products
  double* ex_out = nullptr;
  int32_t* ranks = nullptr;     // device ranks, see kR_* below
  hipGraphExec_t blk_graph[2][16] = {};   // sweep blocks of four shift pairs, by solve width (16 / 32 columns)
  hipGraphExec_t d_graph[2][16] = {};     // their accumulation chains (even and odd shift pairs)
  hipStream_t side[2] = {nullptr, nullptr};   // streams of the two accumulation chains
  hipEvent_t ev_blk = nullptr, ev_done[2] = {nullptr, nullptr};
  int32_t* host_ranks = nullptr;          // pinned host memory: ranks (32 ints), then the norm read-back
  double* host_frob = nullptr;
  LrUnit* units = nullptr;      // per work slot: gram, reduce and form units
  char* ws = nullptr;            // caller workspace (fde2d_plan_create_ws): plan arrays carved from it
  size_t ws_bytes = 0, ws_used = 0;
  bool sizing = false;          // fde2d_plan_workspace_size: arrays counted, not allocated
  int64_t unit_rows[kLrSlots][2] = {};   // row counts the slot's unit lists were built for (-1: none)
  double* gpart = nullptr;
  double* grams = nullptr;
  double* mbuf = nullptr;
  double* frob = nullptr;
  int cap_gram = 0;             // gram units per job slot
  int slot_units = 0;           // LrUnit entries per job slot
  // extended Krylov solver (arrays allocated on its first use)
  bool ek_ready = false;
  bool use_ek = false;          // the current step solves by extended Krylov instead of fADI sweeps
  char* ek_ws = nullptr;        // caller workspace of the solver's arrays (fde2d_ek_attach_workspace)
  int ek_last[2] = {2, 2};      // iterations the last extended Krylov solves took (first solve, correction)
  double ek_gemm_flops = 0.0;   // host: 2 M N K over the solver's k_ek_gemm launches (N before device clipping)
  double iv[4] = {0, 0, 0, 0};  // spectral intervals [iv0, iv1] of A, [iv2, iv3] of B (the shifts' problem)
  int ek_J = 0;                 // shift pairs of the projected fADI (reaching opts.tol / 10 on the intervals)
  std::vector<double> ek_p, ek_q;
  double* ekU = nullptr;        // nx x kEkMax orthonormal basis of the A side
  double* ekAU = nullptr;       // A times it (exact products)
  double* ekV = nullptr;        // ny x kEkMax basis of the B side
  double* ekBV = nullptr;       // B times it
  double* ekTA = nullptr;       // kEkMax x kEkMax projected U^T A U
  double* ekTB = nullptr;       // kEkMax x kEkMax projected V^T B V
  double* ekW = nullptr;        // max(nx, ny) x kRS candidate block
  double* ekO = nullptr;        // max(nx, ny) x kRS its first orthonormalisation
  double* ekS = nullptr;        // kEkMax x kRS Gram-Schmidt coefficients
  double* ekPart = nullptr;     // split-K partial products
  double* ekShift = nullptr;    // device shifts: q_0 .. q_{J-1}, p_0 .. p_{J-1}
  double* ekLU = nullptr;       // 2J shifted projected matrices, LU factors
  double* ekInv = nullptr;      // their inverses
  int32_t* ekPiv = nullptr;     // 2J x kEkMax pivot rows
  int32_t* ekFlag = nullptr;    // 2J zero-pivot flags
  double* ekG[2] = {nullptr, nullptr};   // projected right-hand side factors (kEkMax x kRS, ping-pong)
  double* ekH[2] = {nullptr, nullptr};
  double* ekKZ = nullptr;       // kEkMax x (64 kRS) projected fADI factors
  double* ekKY = nullptr;
  double* ekY = nullptr;        // kEkMax x kEkMax projected solution
  double* ekOm = nullptr;       // kEkMax x kEkSk sketch of its columns
  double* ekYs = nullptr;       // kEkMax x kEkSk: Y Om, then its orthonormal bases, then Y^T Q
  double* ekQ1 = nullptr;
  double* ekQ2 = nullptr;
  double* ekBt = nullptr;
  double* ekEye = nullptr;      // kEkSk x kEkSk identity
  double* ekZf = nullptr;       // nx x kRS, ny x kRS: U Q and V Y^T Q
  double* ekWf = nullptr;
  double* ekJunk = nullptr;     // kEkSk x kRS unused right factor of the orthonormalising passes
  double* ekG0 = nullptr;       // kEkMax x kRS projected right-hand side factors U^T G, V^T H
  double* ekH0 = nullptr;
  double* ekR = nullptr;        // max(nx, ny) x kEkMax residual blocks (A U Y - U T_A Y, ...)
  double* ekY1 = nullptr;       // kEkMax x kEkMax products with the projected matrices
  double* ekRs = nullptr;       // kEkMax x kEkMax projected residual
  double* ekNrm = nullptr;      // device: sums of squares of the three residual terms
  double* ekPivX = nullptr;     // finite elements: pivots of the mass matrices' tridiagonal LU (nx, ny)
  double* ekPivY = nullptr;
  double* ekGt = nullptr;       // finite elements: E_x^-1 G, E_y^-1 H (kRS columns)
  double* ekHt = nullptr;
  std::vector<void*> allocs;
};

namespace {

hodlr_status set_arg(hodlr_ctx ctx, int idx) {
  if (ctx) ctx->last_arg = idx;
  return HODLR_EINVAL;
}

#define HIP_TRY(expr)                                 \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) {                           \
      fprintf(stderr, "hodlr_fde: %s failed: %s\n", #expr, hipGetErrorString(e_)); \
      return HODLR_EHIP;                              \
    }                                                 \
  } while (0)

// Device blocks released by destroyed matrices, per device, handed to later
// matrices that ask for exactly the same sizes: a loop that builds a matrix
// of the same shape again and again (a serving loop, a benchmark) then maps
// no new memory, which for tens of GB costs about a second.  At most kPoolMax
// bytes are kept; an allocation that fails releases the pool and tries again.
struct BlockPool {
  std::mutex mu;
  std::map<int, std::multimap<size_t, void*>> blocks;   // device -> (bytes, block)
  std::map<int, size_t> held;
};
BlockPool& block_pool() {
  static BlockPool* p = new BlockPool;   // never destroyed: no HIP calls during process exit
  return *p;
}
constexpr size_t kPoolMax = size_t(160) << 30;

void* pool_take(size_t bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  BlockPool& P = block_pool();
  std::lock_guard<std::mutex> g(P.mu);
  auto& mm = P.blocks[dev];
  auto it = mm.find(bytes);
  if (it == mm.end()) return nullptr;
  void* q = it->second;
  mm.erase(it);
  P.held[dev] -= bytes;
  return q;
}

void pool_give(void* q, size_t bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipFree(q);
    return;
  }
  BlockPool& P = block_pool();
  std::lock_guard<std::mutex> g(P.mu);
  if (P.held[dev] + bytes > kPoolMax) {
    (void)hipFree(q);
    return;
  }
  P.blocks[dev].emplace(bytes, q);
  P.held[dev] += bytes;
}

void pool_release() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  BlockPool& P = block_pool();
  std::lock_guard<std::mutex> g(P.mu);
  for (auto& kv : P.blocks[dev]) (void)hipFree(kv.second);
  P.blocks[dev].clear();
  P.held[dev] = 0;
}

// The block pool is opt-in (HODLR_POOL=1): by default a destroyed matrix
// frees its blocks.
bool pool_enabled() {
  static const bool on = getenv("HODLR_POOL") && getenv("HODLR_POOL")[0] == '1';
  return on;
}

template <typename T>
hodlr_status dalloc(hodlr_mat m, T** p, size_t count) {
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  if (m->sizing || m->ws) {
    const size_t off = (m->ws_used + 255) & ~size_t(255);
    if (m->sizing) {
      m->ws_used = off + bytes;
      *p = nullptr;
      return HODLR_OK;
    }
    if (off + bytes > m->ws_bytes) return HODLR_EWORKSPACE;
    m->ws_used = off + bytes;
    m->bytes_device += bytes;
    *p = reinterpret_cast<T*>(m->ws + off);
    return HODLR_OK;
  }
  void* q = pool_enabled() ? pool_take(bytes) : nullptr;
  if (!q && hipMalloc(&q, bytes) != hipSuccess) {
    (void)hipGetLastError();
    pool_release();
    q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return HODLR_ENOMEM;
    }
  }
  m->allocs.push_back(q);
  m->alloc_bytes.push_back(bytes);
  // HODLR_POISON=1 fills new device memory with NaN bytes, so that a read of
  // memory no kernel has written shows up in the results
  static const bool poison = getenv("HODLR_POISON") && getenv("HODLR_POISON")[0] == '1';
  if (poison && hipMemset(q, 0xff, bytes) != hipSuccess) return HODLR_EHIP;
  m->bytes_device += bytes;
  *p = static_cast<T*>(q);
  return HODLR_OK;
}

#define TRY(expr)                      \
  do {                                 \
    hodlr_status s_ = (expr);          \
    if (s_ != HODLR_OK) return s_;     \
  } while (0)

int levels_for(int64_t n, int b) {
  int L = 0;
  while ((n + (int64_t(1) << L) - 1) >> L > b) ++L;
  return L;
}

void build_nodes(int64_t n, int L, std::vector<Node>& out) {
  size_t base = out.size();
  out.resize(base + ((size_t(1) << (L + 1)) - 1));
  out[base] = Node{0, int32_t(n)};
  for (int d = 0; d < L; ++d) {
    for (int64_t j = 0; j < (int64_t(1) << d); ++j) {
      const Node p = out[base + ((size_t(1) << d) - 1) + j];
      const int32_t n1 = p.size / 2;
      out[base + ((size_t(1) << (d + 1)) - 1) + 2 * j] = Node{p.start, n1};
      out[base + ((size_t(1) << (d + 1)) - 1) + 2 * j + 1] = Node{p.start + n1, p.size - n1};
    }
  }
}

// Work-groups go to the eight XCDs round-robin by index, and each XCD has an
// L2 of its own.  The strided four-step passes read and write short segments
// whose cache lines neighbouring tiles share, so a unit list is reordered to
// give every XCD a contiguous run of each column's tiles.
constexpr int kXcds = 8;
void xcd_order(std::vector<FftUnit>& u, size_t per_col) {
  if (per_col == 0) return;
  std::vector<FftUnit> out(u.size());
  for (size_t c0 = 0; c0 < u.size(); c0 += per_col) {
    size_t k = c0;
    for (size_t x = 0; x < size_t(kXcds); ++x)
      for (size_t b = c0; b < c0 + per_col; ++b)
        if (b % kXcds == x) out[b] = u[k++];
  }
  u.swap(out);
}

// y = M x (+ b - 2 M x when b is given: the residual b - M x) through the
// near band and the circulant far field.  P supplies the transform scratch:
// the handle's own (columns in groups of kNCF) or, with P.fws_compact, a
// packed buffer for one column at a time.
void launch_fft_matvec_p(hodlr_mat m, const DevPtrs& P, const double* x, int64_t ldx, double* y, int64_t ldy,
                         const double* b, int64_t ldb, int nc, hipStream_t s) {
  const int group = P.fws_compact ? 1 : kNCF;
  for (int c0 = 0; c0 < nc; c0 += group) {
    const int cn = std::min(group, nc - c0);
    const double* xc = x + int64_t(c0) * ldx;
    double* yc = y + int64_t(c0) * ldy;
    const double* bc = b ? b + int64_t(c0) * ldb : nullptr;
    if (m->n_fft_small) {
      // units are laid out column-major: first all items for col 0, then col 1 ...
      int cnt = int(m->small_items.size()) * cn;
      size_t lds = 0;
      int maxlog = 0;
      for (int i : m->small_items) maxlog = std::max(maxlog, m->items[i].fftlog);
      lds = (size_t(1) << maxlog) * sizeof(double2);
      HFDE_LAUNCH(k_fft_small, dim3(cnt), dim3(512), lds, s, P, m->fft_small_units, 1, xc, ldx, yc,
                         ldy, bc, ldb);
    }
    if (m->n_fft_p1) {
      const int per_col1 = m->n_fft_p1 / kNCF, per_col2 = m->n_fft_p2 / kNCF;
      const size_t lds = m->fft4_lds;
      HFDE_LAUNCH(k_fft4_pass1, dim3(per_col1 * cn), dim3(kFft4WG), lds, s, P, m->fft_p1_units, 1, false,
                         xc, ldx);
      HFDE_LAUNCH(k_fft4_pass2, dim3(per_col2 * cn), dim3(kFft4WG), lds, s, P, m->fft_p2_units, 1, false,
                         xc, ldx, yc, ldy, bc, ldb);
      HFDE_LAUNCH(k_fft4_pass1, dim3(per_col1 * cn), dim3(kFft4WG), lds, s, P, m->fft_p1_units, 1, true,
                         xc, ldx);
      HFDE_LAUNCH(k_fft4_pass2, dim3(per_col2 * cn), dim3(kFft4WG), lds, s, P, m->fft_p2_units, 1, true,
                         xc, ldx, yc, ldy, bc, ldb);
    }
    if (m->n_fft_rows) {
      const int per_colr = m->n_fft_rows / kNCF;
      HFDE_LAUNCH(k_exact_rows, dim3(per_colr * cn), dim3(kExactRowsWG), 0, s, P, m->fft_row_units, xc, ldx, yc,
                         ldy, bc, ldb);
    }
  }
}

void launch_fft_matvec(hodlr_mat m, const double* x, int64_t ldx, double* y, int64_t ldy, const double* b,
                       int64_t ldb, int nc, hipStream_t s) {
  launch_fft_matvec_p(m, m->P, x, ldx, y, ldy, b, ldb, nc, s);
}

template <typename TF, typename TL, int NC>
void launch_solve_t(hodlr_mat m, SolveFactors<TF, TL> F, const WorkUnit* wu, int nwu, const NodeUnit* nu, int nnu,
                    const double* x, int64_t ldx, double* y, int64_t ldy, int nc, hipStream_t s) {
  const TF* IL = F.IL;
  const int64_t lv = m->total_leaves;
  if (NC == 1) {                        // one right-hand side: row-per-lane kernels
    HFDE_LAUNCH((k_project1<TF>), dim3(nwu), dim3(256), kSolve1Lds, s, m->P, wu, 0, IL, x, m->partL, lv);
    if (nnu) HFDE_LAUNCH(k_reduce, dim3(nnu), dim3(256), 0, s, m->P, nu, 0, 1, m->partL, m->zL, lv, 1,
                         int64_t(0), int64_t(0));
    HFDE_LAUNCH((k_expand1<TF, TL>), dim3(nwu), dim3(256), kSolve1Lds, s, m->P, F, wu, 0, x, m->ytmp, m->zL,
                       m->partU, lv, m->b);
    if (nnu) HFDE_LAUNCH(k_reduce, dim3(nnu), dim3(256), 0, s, m->P, nu, 1, 1, m->partU, m->zU, lv, 1,
                         int64_t(0), int64_t(0));
    HFDE_LAUNCH((k_expand1<TF, TL>), dim3(nwu), dim3(256), 0, s, m->P, F, wu, 1, m->ytmp, y, m->zU,
                       (double*)nullptr, lv, m->b);
    (void)ldx;
    (void)ldy;
    return;
  }
  // nc <= kNCB * NC columns in kNCB column blocks (grid y), each with its own
  // regions of the partials, node sums and ytmp
  const unsigned nb = unsigned((nc + NC - 1) / NC);
  const int64_t ps = m->part_block, zs = m->z_block;
  HFDE_LAUNCH((k_project<TF, NC>), dim3(nwu, nb), dim3(256), 0, s, m->P, wu, 0, IL, x, ldx, nc, m->partL, lv, ps);
  if (nnu) HFDE_LAUNCH(k_reduce, dim3(nnu, nb), dim3(256), 0, s, m->P, nu, 0, nc, m->partL, m->zL, lv, NC, ps, zs);
  HFDE_LAUNCH((k_expand<TF, TL, NC>), dim3(nwu, nb), dim3(256), 0, s, m->P, F, wu, 0, x, ldx, m->ytmp,
                     m->total_n, nc, m->zL, m->partU, lv, m->b, ps, zs);
  if (nnu) HFDE_LAUNCH(k_reduce, dim3(nnu, nb), dim3(256), 0, s, m->P, nu, 1, nc, m->partU, m->zU, lv, NC, ps, zs);
  HFDE_LAUNCH((k_expand<TF, TL, NC>), dim3(nwu, nb), dim3(256), 0, s, m->P, F, wu, 1, m->ytmp, m->total_n, y,
                     ldy, nc, m->zU, (double*)nullptr, lv, m->b, ps, zs);
}

// y <- M_low^{-1} x at precision `prec` (x and y may alias: the first
// expansion writes ytmp, the second reads only ytmp), over the problems whose
// leaves / nodes are listed (all by default).
void launch_solve_units(hodlr_mat m, int prec, const WorkUnit* wu, int nwu, const NodeUnit* nu, int nnu,
                        const double* x, int64_t ldx, double* y, int64_t ldy, int nc, hipStream_t s) {
  for (int c0 = 0; c0 < nc; c0 += kNCS * kNCB) {
    const int cn = std::min(kNCS * kNCB, nc - c0);
    const double* xc = x + int64_t(c0) * ldx;
    double* yc = y + int64_t(c0) * ldy;
    if (prec == HODLR_MIXED_FP32) {
      SolveFactors<float, float> F{m->IL32, m->IU32, m->LUinv32};
      if (cn == 1) launch_solve_t<float, float, 1>(m, F, wu, nwu, nu, nnu, xc, ldx, yc, ldy, cn, s);
      else launch_solve_t<float, float, kNCS>(m, F, wu, nwu, nu, nnu, xc, ldx, yc, ldy, cn, s);
    } else if (prec == HODLR_MIXED_BF16) {
      SolveFactors<bf16, float> F{m->IL16, m->IU16, m->LUinv32};
      if (cn == 1) launch_solve_t<bf16, float, 1>(m, F, wu, nwu, nu, nnu, xc, ldx, yc, ldy, cn, s);
      else launch_solve_t<bf16, float, kNCS>(m, F, wu, nwu, nu, nnu, xc, ldx, yc, ldy, cn, s);
    } else {
      SolveFactors<double, double> F{m->P.IL, m->P.IU, m->P.LUinv};
      if (cn == 1) launch_solve_t<double, double, 1>(m, F, wu, nwu, nu, nnu, xc, ldx, yc, ldy, cn, s);
      else launch_solve_t<double, double, kNCS>(m, F, wu, nwu, nu, nnu, xc, ldx, yc, ldy, cn, s);
    }
  }
}

void launch_solve(hodlr_mat m, int prec, const double* x, int64_t ldx, double* y, int64_t ldy, int nc,
                  hipStream_t s) {
  launch_solve_units(m, prec, m->wu, m->nwu, m->nu, m->nnu, x, ldx, y, ldy, nc, s);
}

void launch_norms(hodlr_mat m, const double* v, int64_t ld, int nc, double* out, hipStream_t s) {
  HFDE_LAUNCH(k_item_norms, dim3(m->batch, nc), dim3(256), 0, s, m->P, v, ld, nc, out);
}

void launch_axpby(int64_t nrows, int nc, double a, const double* x, int64_t ldx, double bco, const double* y,
                  int64_t ldy, double* z, int64_t ldz, hipStream_t s) {
  const int64_t tot = nrows * nc;
  const int blocks = int(std::min<int64_t>((tot + 255) / 256, 65535));
  HFDE_LAUNCH(k_axpby, dim3(blocks), dim3(256), 0, s, nrows, nc, a, x, ldx, bco, y, ldy, z, ldz);
}

}  // namespace


// ------------------------------------------------------------------
// Multi-work-group factorisation: host schedule (post-order, lock-step
// over the problems of the batch, which must share one tree shape).
enum MwgKind { KL_LEAF = 0, KL_GRAM, KL_REDUCE, KL_CORE, KL_FORM, KL_SPP, KL_SPR, KL_SPE, KL_NODE_REC, KL_NODE_PEND,
               KL_FORK, KL_JOIN_MARK, KL_JOIN_WAIT };

static int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return v ? atoi(v) : dflt;
}

static hodlr_status plan_mwg(hodlr_mat m) {
  if (m->mwg_planned) return HODLR_OK;
  const int B = m->batch;
  std::vector<NodeTask> tasks;
  std::vector<GramUnit> grams;
  std::vector<ReduceUnit> reds;
  std::vector<int2> cores;
  std::vector<FormUnit> forms;
  std::vector<ProdJob> jobs;
  std::vector<ProdUnit> punits;
  size_t max_gpart = 1, max_ppart = 1, max_pz = 1;
  bool on_side = false;                      // records go to the second stream
  auto rec = [&](int kind, int grid, int64_t off, int64_t off2) {
    m->mwg_side.push_back(on_side ? 1 : 0);
    m->mwg_kind.push_back(kind);
    m->mwg_grid.push_back(grid);
    m->mwg_off.push_back(off);
    m->mwg_off2.push_back(off2);
  };
  // Events of a problem's post-order walk.  type 0: leaf; 3: recompression
  // of the off-diagonal blocks S12, S21 (with the pending update) of every
  // internal node on the left spine that starts at (d, j): a node's blocks
  // and pending update are known once the spine's head has its pending
  // update (a left child inherits its parent's), so the spine is recompressed
  // in one step before its leftmost leaf; 1: phase A after the left child
  // (subtree products, C, W and the pending update of the right child, whose
  // spine follows); 2: phase B after the right child.
  struct Ev { int type, d; int64_t j; };
  std::vector<std::vector<Ev>> evs(B);
  for (int i = 0; i < B; ++i) {
    const int L = m->items[i].L;
    std::vector<int> state(L + 2, 0);
    int d = 0;
    int64_t j = 0;
    if (L > 0) evs[i].push_back(Ev{3, 0, 0});
    for (;;) {
      if (d == L) {
        evs[i].push_back(Ev{0, d, j});
        if (d == 0) break;
        --d; j >>= 1;
        continue;
      }
      if (state[d] == 0) { state[d] = 1; state[d + 1] = 0; ++d; j = 2 * j; continue; }
      if (state[d] == 1) {
        evs[i].push_back(Ev{1, d, j});
        if (d + 1 < L) evs[i].push_back(Ev{3, d + 1, 2 * j + 1});
        state[d] = 2; state[d + 1] = 0; ++d; j = 2 * j + 1;
        continue;
      }
      evs[i].push_back(Ev{2, d, j});
      if (d == 0) break;
      --d; j >>= 1;
    }
  }
  size_t steps = 0;
  for (auto& e : evs) steps = std::max(steps, e.size());
  const int fuse_rows = env_int("HODLR_FUSE_ROWS", m->fuse_rows);
  m->fuse_used = fuse_rows;
  bool side_open = false;
  struct TaskSpec { int item, d; int64_t j; int64_t n1, n2; };
  size_t max_step_tasks = 1;
  auto add_tasks = [&](const std::vector<TaskSpec>& ts) {
    max_step_tasks = std::max(max_step_tasks, ts.size());
    const int64_t t0 = int64_t(tasks.size());
    for (size_t k = 0; k < ts.size(); ++k) tasks.push_back(NodeTask{ts[k].item, ts[k].d, int32_t(ts[k].j), int32_t(k)});
    return t0;
  };
  auto rows_of = [](const TaskSpec& t, int type) { return (type == 0 || type == 3 || type == 4 || type == 7) ? t.n1 : t.n2; };
  auto add_grams = [&](int64_t t0, const std::vector<TaskSpec>& ts, std::vector<std::array<int, 3>> pairs) {
    const int64_t g0 = int64_t(grams.size()), r0 = int64_t(reds.size());
    int32_t outi = 0;
    for (size_t k = 0; k < ts.size(); ++k)
      for (auto& p : pairs) {
        const int chunks = int((rows_of(ts[k], p[0]) + m->gram_rows - 1) / m->gram_rows);
        reds.push_back(ReduceUnit{outi, std::max(chunks, 1), int32_t(k * 9 + p[2]), 0});
        for (int c = 0; c < std::max(chunks, 1); ++c)
          grams.push_back(GramUnit{int32_t(k), int16_t(p[0]), int16_t(p[1]), c, outi++});
      }
    max_gpart = std::max(max_gpart, size_t(outi));
    rec(KL_GRAM, int(grams.size() - g0), g0, t0);
    rec(KL_REDUCE, int(reds.size() - r0), r0, t0);
  };
  auto add_core = [&](int64_t t0, size_t nt, std::vector<int> whiches) {
    const int64_t c0 = int64_t(cores.size());
    for (size_t k = 0; k < nt; ++k)
      for (int w : whiches) cores.push_back(make_int2(int(k), w));
    rec(KL_CORE, int(cores.size() - c0), c0, t0);
  };
  auto add_form = [&](int64_t t0, const std::vector<TaskSpec>& ts, std::vector<int> outs) {
    const int64_t f0 = int64_t(forms.size());
    static const int src_type[7] = {0, 1, 2, 3, 8, 5, 6};
    for (size_t k = 0; k < ts.size(); ++k)
      for (int o : outs) {
        const int64_t rows = rows_of(ts[k], src_type[o]);
        for (int64_t c = 0; c < (rows + 255) / 256; ++c) forms.push_back(FormUnit{int32_t(k), o, int32_t(c), 0});
      }
    rec(KL_FORM, int(forms.size() - f0), f0, t0);
  };
  struct Spec { int child, which, trans, xarr, yarr, rk; double sign; };
  auto add_prods = [&](const std::vector<TaskSpec>& ts, std::vector<Spec> specs) {
    const int64_t j0i = int64_t(jobs.size());
    std::vector<ProdUnit> leafu, nodeu;
    for (const TaskSpec& t : ts) {
      const int L = m->items[t.item].L;
      for (auto& sp : specs) {
        ProdJob jb{};
        jb.item = t.item;
        jb.d0 = int16_t(t.d + 1);
        jb.j0 = int32_t(2 * t.j + sp.child);
        jb.which = int16_t(sp.which);
        jb.trans = int16_t(sp.trans);
        jb.xarr = int8_t(sp.xarr);
        jb.yarr = int8_t(sp.yarr);
        jb.xlev = int16_t(t.d);
        jb.ylev = int16_t(t.d);
        jb.rd = int16_t(t.d);
        jb.rj = int32_t(t.j);
        jb.rk = int16_t(sp.rk);
        jb.sign = sp.sign;
        jb.unit0 = int32_t(leafu.size());
        jb.node0 = int32_t(nodeu.size());
        const int jid = int(jobs.size() - j0i);
        const int64_t lo = int64_t(jb.j0) << (L - jb.d0), cnt = int64_t(1) << (L - jb.d0);
        for (int64_t l = 0; l < cnt; ++l) leafu.push_back(ProdUnit{jid, int32_t(lo + l), 0, 0});
        for (int dd = jb.d0; dd < L; ++dd)
          for (int64_t q = 0; q < (int64_t(1) << (dd - jb.d0)); ++q)
            nodeu.push_back(ProdUnit{jid, dd, int32_t((int64_t(jb.j0) << (dd - jb.d0)) + q), 0});
        jobs.push_back(jb);
      }
    }
    const int64_t lu0 = int64_t(punits.size());
    punits.insert(punits.end(), leafu.begin(), leafu.end());
    const int64_t nu0 = int64_t(punits.size());
    punits.insert(punits.end(), nodeu.begin(), nodeu.end());
    max_ppart = std::max(max_ppart, leafu.size());
    max_pz = std::max(max_pz, nodeu.size());
    // subtrees that are single leaves have no levels to project onto
    bool levels = false;
    for (int64_t q = j0i; q < int64_t(jobs.size()); ++q) levels = levels || jobs[q].d0 < m->items[jobs[q].item].L;
    if (levels) rec(KL_SPP, int(leafu.size()), lu0, j0i);
    if (!nodeu.empty()) rec(KL_SPR, int(nodeu.size()), nu0, j0i);
    rec(KL_SPE, int(leafu.size()), lu0, j0i);
  };
  for (size_t g = 0; g < steps; ++g) {
    std::vector<TaskSpec> lt, at, bt, st;
    for (int i = 0; i < B; ++i) {
      if (g >= evs[i].size()) continue;
      const Ev e = evs[i][g];
      if (e.type == 3) {                 // every internal node of the spine
        const int L = m->items[i].L;
        for (int dd = e.d; dd < L; ++dd) {
          const int64_t jj = e.j << (dd - e.d);
          const Node nd = m->nodes[node_index(m->items[i], dd, jj)];
          st.push_back(TaskSpec{i, dd, jj, nd.size / 2, nd.size - nd.size / 2});
        }
        continue;
      }
      const Node nd = m->nodes[node_index(m->items[i], e.d, e.j)];
      TaskSpec t{i, e.d, e.j, nd.size / 2, nd.size - nd.size / 2};
      (e.type == 0 ? lt : (e.type == 1 ? at : bt)).push_back(t);
    }
    // nodes whose children fit the fused single-work-group kernels, and the rest
    auto split = [&](const std::vector<TaskSpec>& ts, std::vector<TaskSpec>& small, std::vector<TaskSpec>& big) {
      for (const TaskSpec& t : ts) (std::max(t.n1, t.n2) <= fuse_rows ? small : big).push_back(t);
    };
    if (!lt.empty()) {
      const int64_t t0 = add_tasks(lt);
      rec(KL_LEAF, int(lt.size()), t0, t0);
    }
    if (!st.empty()) {
      // the spine's recompressions run on the second stream, concurrently with
      // the leaves that follow; phase A waits for them (join)
      rec(KL_FORK, 1, 0, 0);
      on_side = true;
      std::vector<TaskSpec> small, big;
      split(st, small, big);
      if (!small.empty()) {
        const int64_t t0 = add_tasks(small);
        rec(KL_NODE_REC, int(2 * small.size()), t0, t0);
      }
      if (!big.empty()) {
        const int64_t t0 = add_tasks(big);
        add_grams(t0, big, {{0, 0, 0}, {1, 1, 1}, {2, 2, 2}, {3, 3, 3}});
        add_core(t0, big.size(), {0, 1});
        add_form(t0, big, {0, 1, 2, 3});
      }
      rec(KL_JOIN_MARK, 1, 0, 0);
      on_side = false;
      side_open = true;
    }
    if (!at.empty()) {
      if (side_open) rec(KL_JOIN_WAIT, 1, 0, 0);
      side_open = false;
      add_prods(at, {{0, 0, 0, A_T1, A_FU, 0, 1.0}, {0, 1, 1, A_T2, A_FL, 1, 1.0}});
      std::vector<TaskSpec> small, big;
      split(at, small, big);
      if (!small.empty()) {
        const int64_t t0 = add_tasks(small);
        rec(KL_NODE_PEND, int(small.size()), t0, t0);
      }
      if (!big.empty()) {
        const int64_t t0 = add_tasks(big);
        add_grams(t0, big, {{4, 7, 4}});
        add_form(t0, big, {4});
        add_grams(t0, big, {{5, 5, 5}, {6, 6, 6}});
        add_core(t0, big.size(), {2});
        add_form(t0, big, {5, 6});
      }
    }
    if (!bt.empty())
      add_prods(bt, {{1, 0, 0, A_FL, A_IL, 1, -1.0}, {0, 0, 1, A_FL, A_IL, 1, 1.0},
                     {0, 1, 0, A_FU, A_IU, 0, -1.0}, {1, 1, 1, A_FU, A_IU, 0, 1.0}});
  }
  if (side_open) rec(KL_JOIN_WAIT, 1, 0, 0);
  const int Lmax = std::max(1, m->Lmax);
  if (m->ws && !m->sizing) {
    // a workspace holds one schedule: a new one replaces the last in place,
    // once no factorisation that reads it can still run
    if (m->ws_used > m->ws_sched) HIP_TRY(hipDeviceSynchronize());
    m->ws_used = m->ws_sched;
  }
  TRY(dalloc(m, &m->d_tasks, tasks.size()));
  TRY(dalloc(m, &m->d_gram, grams.size()));
  TRY(dalloc(m, &m->d_red, reds.size()));
  TRY(dalloc(m, &m->d_core, cores.size()));
  TRY(dalloc(m, &m->d_form, forms.size()));
  TRY(dalloc(m, &m->d_jobs, jobs.size()));
  TRY(dalloc(m, &m->d_punits, punits.size()));
  TRY(dalloc(m, &m->d_gpart, max_gpart * kG2));
  TRY(dalloc(m, &m->d_gpart_side, max_gpart * kG2));
  TRY(dalloc(m, &m->d_G, max_step_tasks * 9 * kG2));
  TRY(dalloc(m, &m->d_M, max_step_tasks * 3 * 2 * kMaxCat * kRS));
  TRY(dalloc(m, &m->d_ppart, max_ppart * Lmax * kRS * kPNC));
  TRY(dalloc(m, &m->d_pz, max_pz * kRS * kPNC));
  if (m->sizing) return HODLR_OK;
  auto up = [](void* dst, const void* src, size_t bytes) -> hodlr_status {
    if (bytes) HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return HODLR_OK;
  };
  TRY(up(m->d_tasks, tasks.data(), tasks.size() * sizeof(NodeTask)));
  TRY(up(m->d_gram, grams.data(), grams.size() * sizeof(GramUnit)));
  TRY(up(m->d_red, reds.data(), reds.size() * sizeof(ReduceUnit)));
  TRY(up(m->d_core, cores.data(), cores.size() * sizeof(int2)));
  TRY(up(m->d_form, forms.data(), forms.size() * sizeof(FormUnit)));
  TRY(up(m->d_jobs, jobs.data(), jobs.size() * sizeof(ProdJob)));
  TRY(up(m->d_punits, punits.data(), punits.size() * sizeof(ProdUnit)));
  m->mwg_planned = true;
  return HODLR_OK;
}

// Launch shapes chosen by hodlr_autotune, per tree signature (batch, total
// rows, depth, leaf size), applied to matrices built later in the process.
struct TuneKey {
  int batch;
  int64_t total_n;
  int levels, leaf;
  bool operator<(const TuneKey& o) const {
    return std::tie(batch, total_n, levels, leaf) < std::tie(o.batch, o.total_n, o.levels, o.leaf);
  }
};
struct TuneVal {
  int core_threads, leaf_threads, gram_rows, fuse_rows;
};
static std::map<TuneKey, TuneVal> g_tuned;
static std::mutex g_tuned_mu;

static TuneKey tune_key(hodlr_mat m) { return TuneKey{m->batch, m->total_n, m->Lmax, m->b}; }


static void enqueue_mwg(hodlr_mat m, hipStream_t s) {
  const DevPtrs& P = m->P;
  // block sizes of the latency-bound single-group kernels (512 measured fastest);
  // the leaf kernel splits its dot products over blockDim/128 threads, so it needs >= 128
  auto pick = [](int v) { return v >= 512 ? 512 : (v >= 256 ? 256 : 128); };
  const int core_threads = kCoreWG;   // fixed by the cores' launch bounds (register-held columns)
  const int leaf_threads = std::max(256, pick(env_int("HODLR_LEAF_THREADS", m->leaf_threads)));
  const int Lmax = std::max(1, m->Lmax);
  // second stream for the spine recompressions; timed runs (events on the
  // context's stream around every launch) keep everything on one stream
  bool two = g_timer == nullptr;
  if (two && !m->side) {
    two = hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking) == hipSuccess &&
          hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming) == hipSuccess &&
          hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming) == hipSuccess;
  }
  const hipStream_t main_s = s;
  for (size_t q = 0; q < m->mwg_kind.size(); ++q) {
    const int g = m->mwg_grid[q];
    if (g <= 0) continue;
    const int64_t off = m->mwg_off[q], off2 = m->mwg_off2[q];
    const bool on_side = m->mwg_side[q] != 0;
    s = (two && on_side) ? m->side : main_s;
    double* gpart = on_side ? m->d_gpart_side : m->d_gpart;
    switch (m->mwg_kind[q]) {
      case KL_FORK:
        if (two) {
          (void)hipEventRecord(m->ev_fork, main_s);
          (void)hipStreamWaitEvent(m->side, m->ev_fork, 0);
        }
        break;
      case KL_JOIN_MARK:
        if (two) (void)hipEventRecord(m->ev_join, m->side);
        break;
      case KL_JOIN_WAIT:
        if (two) (void)hipStreamWaitEvent(main_s, m->ev_join, 0);
        break;
      case KL_LEAF:
        HFDE_LAUNCH(k_leaf_task, dim3(g), dim3(leaf_threads), kFactorLdsBytes, s, P, m->d_tasks + off, m->b);
        break;
      case KL_GRAM:
        HFDE_LAUNCH(k_gram_partial, dim3(g), dim3(256), 0, s, P, m->d_tasks + off2, m->d_gram + off, gpart,
                    m->gram_rows);
        break;
      case KL_REDUCE:
        HFDE_LAUNCH(k_gram_reduce, dim3(g), dim3(256), 0, s, m->d_red + off, gpart, m->d_G);
        break;
      case KL_CORE:
        HFDE_LAUNCH(k_core, dim3(g), dim3(core_threads), kFactorLdsBytes, s, P, m->d_tasks + off2, m->d_core + off, m->d_G,
                           m->d_M, m->opts.max_rank);
        break;
      case KL_FORM:
        HFDE_LAUNCH(k_form, dim3(g), dim3(256), 0, s, P, m->d_tasks + off2, m->d_form + off, m->d_G, m->d_M);
        break;
      case KL_SPP:
        HFDE_LAUNCH(k_sp_project, dim3(g), dim3(256), kSpProjLds, s, P, m->d_jobs + off2, m->d_punits + off, m->d_ppart, Lmax);
        break;
      case KL_SPR:
        HFDE_LAUNCH(k_sp_reduce, dim3(g), dim3(256), 0, s, P, m->d_jobs + off2, m->d_punits + off, m->d_ppart,
                           m->d_pz, Lmax);
        break;
      case KL_NODE_REC:
        HFDE_LAUNCH(k_node_recompress, dim3(g), dim3(core_threads), kFactorLdsBytes, s, P, m->d_tasks + off,
                    m->opts.max_rank);
        break;
      case KL_NODE_PEND:
        HFDE_LAUNCH(k_node_pending, dim3(g), dim3(core_threads), kFactorLdsBytes, s, P, m->d_tasks + off);
        break;
      default:
        HFDE_LAUNCH(k_sp_expand, dim3(g), dim3(256), kSpExpLds, s, P, m->d_jobs + off2, m->d_punits + off, m->d_pz, m->b);
        break;
    }
  }
}

// ===================================================================== ABI
extern "C" {

const char* hodlr_status_string(hodlr_status s) {
  switch (s) {
    case HODLR_OK: return "ok";
    case HODLR_EINVAL: return "invalid argument";
    case HODLR_ENOMEM: return "device allocation failed";
    case HODLR_EHIP: return "HIP runtime error";
    case HODLR_ESTATE: return "call out of order";
    case HODLR_EWORKSPACE: return "caller workspace too small";
    case HODLR_ESINGULAR: return "singular leaf pivot";
    case HODLR_ENOCONV: return "refinement did not converge (FP64 fallback used)";
    case HODLR_ERANK: return "rank cap reached above tolerance";
  }
  return "unknown status";
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
static hodlr_status scratch_address(void** out) {
  static std::mutex mu;
  static void* addr[256] = {};
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 256) return HODLR_EHIP;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      fprintf(stderr, "hodlr_fde: hipGetSymbolAddress(scratch) failed on device %d: %s\n", dev,
              hipGetErrorString(e));
      return HODLR_EHIP;
    }
    addr[dev] = p;
  }
  *out = addr[dev];
  return HODLR_OK;
}

hodlr_status hodlr_ctx_create(hodlr_ctx* ctx, void* hip_stream) {
  if (!ctx) return HODLR_EINVAL;
  void* sp = nullptr;
  TRY(scratch_address(&sp));   // the no-allocation entry point's scratch on this device
  hodlr_ctx c = new (std::nothrow) hodlr_ctx_s;
  if (!c) return HODLR_ENOMEM;
  c->stream = static_cast<hipStream_t>(hip_stream);
  *ctx = c;
  return HODLR_OK;
}

void hodlr_ctx_destroy(hodlr_ctx ctx) { delete ctx; }

int hodlr_last_arg(hodlr_ctx ctx) { return ctx ? ctx->last_arg : 0; }

hodlr_status hodlr_ctx_set_timing(hodlr_ctx ctx, int enable) {
  if (!ctx) return HODLR_EINVAL;
  ctx->timer.flush();
  ctx->timing = enable != 0;
  return HODLR_OK;
}

int hodlr_ctx_timing_count(hodlr_ctx ctx) { return ctx ? int(ctx->timer.names.size()) : 0; }

hodlr_status hodlr_ctx_timing_entry(hodlr_ctx ctx, int i, const char** name, int64_t* launches, double* total_ms) {
  if (!ctx) return HODLR_EINVAL;
  if (i < 0 || i >= int(ctx->timer.names.size())) return set_arg(ctx, 2);
  if (name) *name = ctx->timer.names[i].c_str();
  if (launches) *launches = ctx->timer.counts[i];
  if (total_ms) *total_ms = ctx->timer.ms[i];
  return HODLR_OK;
}

void hodlr_ctx_timing_reset(hodlr_ctx ctx) {
  if (ctx) ctx->timer.reset();
}

hodlr_status hodlr_default_opts(hodlr_opts* o) {
  if (!o) return HODLR_EINVAL;
  o->leaf = 64;
  o->tol = 1e-10;
  o->prec = HODLR_FP64;
  o->max_rank = 32;
  o->refine_max = 0;
  o->rtol = 1e-12;
  o->gmres_m = 0;
  return HODLR_OK;
}

void hodlr_destroy(hodlr_mat m) {
  if (!m) return;
  if (m->step_graph) (void)hipGraphExecDestroy(m->step_graph);
  if (m->side) {
    (void)hipStreamSynchronize(m->side);
    (void)hipStreamDestroy(m->side);
  }
  if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
  if (m->ev_join) (void)hipEventDestroy(m->ev_join);
  // no kernel may still use a block when it goes back to the pool
  (void)hipDeviceSynchronize();
  for (size_t i = 0; i < m->allocs.size(); ++i) {
    if (pool_enabled()) pool_give(m->allocs[i], m->alloc_bytes[i]);
    else (void)hipFree(m->allocs[i]);
  }
  if (m->host_worst) (void)hipHostFree(m->host_worst);
  delete m;
}

static hodlr_status set_lds_limits() {
  static bool done = false;
  if (done) return HODLR_OK;
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_factor),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(kFactorLdsBytes)));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_leaf_task),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(kFactorLdsBytes)));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_core),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(kFactorLdsBytes)));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_node_recompress),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(kFactorLdsBytes)));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_node_pending),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(kFactorLdsBytes)));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sp_project),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(kSpProjLds)));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sp_expand),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(kSpExpLds)));
#define HFDE_LDS1(kern) HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&kern), \
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(kSolve1Lds)))
  HFDE_LDS1(k_project1<double>);
  HFDE_LDS1(k_project1<float>);
  HFDE_LDS1(k_project1<bf16>);
  HFDE_LDS1((k_expand1<double, double>));
  HFDE_LDS1((k_expand1<float, float>));
  HFDE_LDS1((k_expand1<bf16, float>));
#undef HFDE_LDS1
  const int fl = int(size_t(kFftLds) * sizeof(double2));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_small),
                              hipFuncAttributeMaxDynamicSharedMemorySize, fl));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft4_pass1),
                              hipFuncAttributeMaxDynamicSharedMemorySize, fl));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft4_pass2),
                              hipFuncAttributeMaxDynamicSharedMemorySize, fl));
  done = true;
  return HODLR_OK;
}

// Reads the compression's status bits (after the stream has drained): a
// Hankel compression stopped by the rank cap is remembered and reported by
// the next hodlr_factor as HODLR_ERANK.
static hodlr_status read_capped_A(hodlr_mat m) {
  std::vector<int32_t> st(m->batch);
  HIP_TRY(hipMemcpy(st.data(), m->P.status, m->batch * sizeof(int32_t), hipMemcpyDeviceToHost));
  m->capped_A = false;
  for (int32_t v : st) m->capped_A |= (v & 4) != 0;
  return HODLR_OK;
}

// The reduced-precision copies of the solve's factors (FP32 leaf inverses and
// low-rank factors; BF16 low-rank factors as well for HODLR_MIXED_BF16).
static hodlr_status alloc_lowprec(hodlr_mat m) {
  if (m->opts.prec == HODLR_FP64) return HODLR_OK;
  int64_t nlvl = 0;
  for (const Item& it : m->items) nlvl += int64_t(it.L + 1) * it.n * kRS;
  const int64_t nleafv = m->total_leaves * m->b * m->b;
  TRY(dalloc(m, &m->LUinv32, nleafv));
  TRY(dalloc(m, &m->IL32, nlvl));
  TRY(dalloc(m, &m->IU32, nlvl));
  if (m->opts.prec == HODLR_MIXED_BF16) {
    TRY(dalloc(m, &m->IL16, nlvl));
    TRY(dalloc(m, &m->IU16, nlvl));
  }
  return HODLR_OK;
}

// Host plan, device buffers and device construction of a batch of
// operators.  Three modes: library-allocated (ws == nullptr), carved from a
// caller's workspace (ws != nullptr), or sizing only (need != nullptr: every
// buffer is counted, nothing is allocated or launched, and *need receives the
// workspace the matrix would use, including the factorisation schedule at
// every launch shape the autotuner tries).
static hodlr_status build_impl(hodlr_ctx ctx, const fde_operator* ops, int batch, const hodlr_opts* opts,
                               void* ws, size_t ws_bytes, hodlr_mat* out, size_t* need) {
  const bool sizing = need != nullptr;
  if (!ops) return set_arg(ctx, 2);
  if (batch < 1) return set_arg(ctx, 3);
  if (!opts) return set_arg(ctx, 4);
  if (!sizing && !out) return set_arg(ctx, 7);
  if (opts->leaf < 16 || opts->leaf > kMaxLeaf) return set_arg(ctx, 4);
  if (!(opts->tol > 0.0) || opts->max_rank < 1 || opts->max_rank > kRS) return set_arg(ctx, 4);
  if (opts->prec < HODLR_FP64 || opts->prec > HODLR_MIXED_BF16) return set_arg(ctx, 4);
  if (opts->gmres_m < 0 || opts->gmres_m > kGmMax) return set_arg(ctx, 4);
  for (int i = 0; i < batch; ++i) {
    const fde_operator& o = ops[i];
    // the solve and product kernels address a level's factor block (n x 32
    // values) with 32-bit byte offsets that must stay below the out-of-range
    // sentinel kOob, so n x 32 x 8 < 2^31 - 16
    if (o.n < 1 || o.n >= (int64_t(1) << 23) || !(o.alpha >= 1.0 && o.alpha <= 2.0) || !(o.dt > 0.0) ||
        !(o.dx > 0.0) || !(o.shift > 0.0) || (!sizing && (!o.d_plus || !o.d_minus)) ||
        (o.discretization != FDE_FD && o.discretization != FDE_FE))
      return set_arg(ctx, 2);
  }
  if (!sizing) TRY(set_lds_limits());
  hodlr_mat m = new (std::nothrow) hodlr_mat_s;
  if (!m) return HODLR_ENOMEM;
  m->ctx = ctx;
  m->opts = *opts;
  m->batch = batch;
  m->b = opts->leaf;
  m->sizing = sizing;
  m->ws = static_cast<char*>(ws);
  m->ws_bytes = ws_bytes;
  hipStream_t s = ctx ? ctx->stream : nullptr;
  // ---- plan
  int64_t row0 = 0, leaf0 = 0, node0 = 0, lvl0 = 0, g0 = 0, w0 = 0, z0 = 0, tw0 = 0, ws0 = 0, wsc0 = 0;
  for (int i = 0; i < batch; ++i) {
    const fde_operator& o = ops[i];
    Item it{};
    it.n = o.n;
    it.row0 = row0;
    it.L = levels_for(o.n, m->b);
    it.leaf0 = leaf0;
    it.node0 = node0;
    it.lvl0 = lvl0;
    it.g0 = g0;
    it.nh = (o.n + 1) / 2;
    it.w0 = w0;
    it.z0 = z0;
    it.alpha = o.alpha;
    it.nu = o.dt / std::pow(o.dx, o.alpha);
    it.shift = o.shift;
    it.kind = o.discretization;
    it.mass = o.discretization == FDE_FE ? 2.0 / 3.0 : 1.0;
    it.mc = o.discretization == FDE_FE ? 0.25 : 0.0;
    if (o.discretization == FDE_FE) {   // 1/Gamma(4 - alpha) in extended precision, split hi + lo
      const long double ig = 1.0L / std::tgamma(4.0L - static_cast<long double>(o.alpha));
      it.fig = static_cast<double>(ig);
      it.fig_lo = static_cast<double>(ig - static_cast<long double>(it.fig));
    }
    m->has_mass |= o.discretization == FDE_FE;
    int flog = 1;
    while ((int64_t(1) << flog) < 2 * o.n - 1) ++flog;
    it.fftlog = flog;
    it.band = int(std::min<int64_t>(64, o.n - 1));
    it.tw0 = tw0;
    it.mu0 = tw0;   // mu shares the offsets of the twiddle table (separate array)
    it.ws0 = ws0;
    it.wsc0 = wsc0;
    m->items.push_back(it);
    build_nodes(o.n, it.L, m->nodes);
    row0 += o.n;
    leaf0 += int64_t(1) << it.L;
    node0 += (int64_t(1) << (it.L + 1)) - 1;
    lvl0 += int64_t(it.L + 1) * o.n * kRS;
    g0 += o.n + 8;
    w0 += it.nh * kRS;
    z0 += (int64_t(1) << it.L) * kRS * 64;
    tw0 += int64_t(1) << flog;
    ws0 += 2 * (int64_t(1) << flog) * kNCF;
    wsc0 += 2 * (int64_t(1) << flog);
    m->Lmax = std::max(m->Lmax, it.L);
  }
  m->total_n = row0;
  m->fws_packed = wsc0;
  m->total_leaves = leaf0;
  m->total_nodes = node0;
  std::vector<int32_t> rowleaf(row0);
  for (int i = 0; i < batch; ++i) {
    const Item& it = m->items[i];
    for (int64_t l = 0; l < (int64_t(1) << it.L); ++l) {
      const Node nd = m->nodes[node_index(it, it.L, l)];
      for (int32_t r = 0; r < nd.size; ++r) rowleaf[it.row0 + nd.start + r] = int32_t(l);
      m->wu_h.push_back(WorkUnit{i, int32_t(l), nd.start, nd.size, it.row0, it.lvl0, it.n, it.leaf0 + l, it.node0,
                                 it.L, 0});
    }
    for (int d = 0; d < it.L; ++d)
      for (int64_t j = 0; j < (int64_t(1) << d); ++j) m->nu_h.push_back(NodeUnit{i, d, int32_t(j), 0});
  }
  m->nwu = int(m->wu_h.size());
  m->nnu = int(m->nu_h.size());
  const int b = m->b;
  // FFT work lists
  std::vector<FftUnit> us, u1, u2, ur;
  for (int i = 0; i < batch; ++i) {
    if (m->items[i].fftlog <= kFftSmallMax) m->small_items.push_back(i);
    else m->big_items.push_back(i);
  }
  for (int c = 0; c < kNCF; ++c)
    for (int i : m->small_items) us.push_back(FftUnit{i, c, 0, 0});
  for (int c = 0; c < kNCF; ++c)
    for (int i : m->big_items) {
      const int lg = m->items[i].fftlog;
      const int l2 = lg / 2, l1 = lg - l2;
      int T = std::min(kFftTileMax, kFftLds >> l1);
      m->fft4_lds = std::max(m->fft4_lds, size_t(T) * (size_t(1) << l1) * sizeof(double2));
      for (int t = 0; t < (1 << l1) / T; ++t) u1.push_back(FftUnit{i, c, t, 0});
      for (int t = 0; t < (1 << l2) / T; ++t) u2.push_back(FftUnit{i, c, t, 0});
    }
  // near-band rows of every item (after either transform path)
  for (int c = 0; c < kNCF; ++c)
    for (int i = 0; i < m->batch; ++i) {
      constexpr int kRowsPerUnit = kExactRowsWG / 4;   // rows of one k_exact_rows work-group
      for (int64_t t = 0; t < (m->items[i].n + kRowsPerUnit - 1) / kRowsPerUnit; ++t)
        ur.push_back(FftUnit{i, c, int32_t(t), 0});
    }
  xcd_order(u1, u1.size() / kNCF);
  xcd_order(u2, u2.size() / kNCF);
  m->n_fft_small = int(m->small_items.size());
  m->n_fft_p1 = int(u1.size());
  m->n_fft_p2 = int(u2.size());
  m->n_fft_rows = int(ur.size());
  // ---- device buffers
  DevPtrs& P = m->P;
  hodlr_status st;
#define ALLOC(ptr, cnt)                                   \
  do {                                                    \
    st = dalloc(m, &(ptr), (cnt));                        \
    if (st != HODLR_OK) { hodlr_destroy(m); return st == HODLR_EWORKSPACE ? set_arg(ctx, 6) : st; } \
  } while (0)
  ALLOC(P.items, batch);
  ALLOC(P.nodes, m->nodes.size());
  ALLOC(P.rowleaf, row0);
  ALLOC(P.g, g0);
  ALLOC(P.W, w0);
  ALLOC(P.dplus, row0);
  ALLOC(P.dminus, row0);
  const size_t leafsz = size_t(leaf0) * b * b;
  ALLOC(P.Aleaf, leafsz);
  ALLOC(P.LU, leafsz);
  ALLOC(P.LUinv, leafsz);
  ALLOC(P.perm, size_t(leaf0) * b);
  ALLOC(P.perminv, size_t(leaf0) * b);
  ALLOC(P.XL, lvl0);
  ALLOC(P.XR, lvl0);
  ALLOC(P.FL, lvl0);
  ALLOC(P.FU, lvl0);
  ALLOC(P.IL, lvl0);
  ALLOC(P.IU, lvl0);
  ALLOC(P.T1, std::max<int64_t>(lvl0, w0));
  ALLOC(P.T2, lvl0);
  ALLOC(P.PP, lvl0);
  ALLOC(P.PQ, lvl0);
  ALLOC(P.Z, z0);
  ALLOC(P.rankL, node0);
  ALLOC(P.rankU, node0);
  ALLOC(P.rankP, node0);
  ALLOC(P.tw, tw0);
  ALLOC(P.mu, tw0);
  ALLOC(P.fws, ws0);
  ALLOC(P.status, batch);
  ALLOC(P.diag, 4 * batch);
  ALLOC(m->wu, m->nwu);
  ALLOC(m->nu, m->nnu);
  // the solve's work arrays hold kNCB column blocks of kNCS columns
  const int64_t part_sz = leaf0 * std::max(1, m->Lmax) * kRS * kNCS;
  m->part_block = part_sz;
  m->z_block = node0 * kRS * kNCS;
  ALLOC(m->partL, part_sz * kNCB);
  ALLOC(m->partU, part_sz * kNCB);
  ALLOC(m->zL, std::max(2, kNCB) * node0 * kRS * kNCS);   // the operator matvec stores two sides per node
  ALLOC(m->zU, std::max(2, kNCB) * node0 * kRS * kNCS);
  ALLOC(m->ytmp, row0 * kNCS * kNCB);
  ALLOC(m->rbuf, row0 * kNCS);
  ALLOC(m->dbuf, row0 * kNCS);
  ALLOC(m->bbuf, row0 * kNCS);
  ALLOC(m->norms, batch * kNCS * 4);
  {
    int64_t nmax = 1;
    for (const Item& it : m->items) nmax = std::max(nmax, it.n);
    m->step_slices = int((nmax + kStepRows - 1) / kStepRows);
  }
  ALLOC(m->ukeep, row0);
  ALLOC(m->step_part, size_t(batch) * m->step_slices);
  ALLOC(m->step_worst, batch);
  if (opts->gmres_m > 0) {
    static_assert(kGmRows == kStepRows, "GMRES row kernels share the step kernels' slices");
    GmState& G = m->gms;
    G.slices = m->step_slices;
    ALLOC(m->gmV, row0 * (kGmMax + 1));
    ALLOC(m->gmZ, row0 * kGmMax);
    ALLOC(G.H, size_t(batch) * (kGmMax + 1) * kGmMax);
    ALLOC(G.g, size_t(batch) * (kGmMax + 1));
    ALLOC(G.cs, size_t(batch) * kGmMax);
    ALLOC(G.sn, size_t(batch) * kGmMax);
    ALLOC(G.y, size_t(batch) * kGmMax);
    ALLOC(G.h1, size_t(G.slices) * batch * (kGmMax + 1));
    ALLOC(G.h2, size_t(G.slices) * batch * (kGmMax + 1));
    ALLOC(G.nrm, size_t(G.slices) * batch);
  }
  ALLOC(m->fft_row_units, ur.size());
  ALLOC(m->fft_small_units, us.size());
  ALLOC(m->fft_p1_units, u1.size());
  ALLOC(m->fft_p2_units, u2.size());
  if (m->ws || sizing) {
    // in a workspace the reduced-precision factor copies sit before the
    // factorisation schedule, which is re-planned in place when the launch
    // shapes change and so comes last
    st = alloc_lowprec(m);
    if (st != HODLR_OK) { hodlr_destroy(m); return st == HODLR_EWORKSPACE ? set_arg(ctx, 6) : st; }
    m->ws_sched = (m->ws_used + 255) & ~size_t(255);
  }
#undef ALLOC
  if (sizing) {
    // the schedule at the shapes the autotuner tries and at the ones this
    // process has tuned for the tree signature
    std::vector<std::pair<int, int>> shapes;
    for (int g : {128, 256, 512})
      for (int f : {0, 128, 256, 512, 1024}) shapes.emplace_back(g, f);
    shapes.emplace_back(m->gram_rows, m->fuse_rows);
    {
      std::lock_guard<std::mutex> lk(g_tuned_mu);
      auto f = g_tuned.find(tune_key(m));
      if (f != g_tuned.end()) shapes.emplace_back(f->second.gram_rows, f->second.fuse_rows);
    }
    size_t most = 0;
    for (auto& gf : shapes) {
      m->gram_rows = gf.first;
      m->fuse_rows = gf.second;
      m->mwg_planned = false;
      m->mwg_kind.clear();
      m->mwg_side.clear();
      m->mwg_grid.clear();
      m->mwg_off.clear();
      m->mwg_off2.clear();
      m->ws_used = m->ws_sched;
      st = plan_mwg(m);
      if (st != HODLR_OK) { delete m; return st; }
      most = std::max(most, m->ws_used - m->ws_sched);
    }
    *need = m->ws_sched + most + 256;   // + alignment of the workspace's own start
    delete m;
    return HODLR_OK;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&m->host_worst), batch * sizeof(double), hipHostMallocDefault) !=
      hipSuccess) {
    (void)hipGetLastError();
    m->host_worst = nullptr;
    hodlr_destroy(m);
    return HODLR_ENOMEM;
  }
  auto up = [&](void* dst, const void* src, size_t bytes) -> hodlr_status {
    if (bytes) HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return HODLR_OK;
  };
  TRY(up(m->fft_row_units, ur.data(), ur.size() * sizeof(FftUnit)));
  TRY(up(m->fft_small_units, us.data(), us.size() * sizeof(FftUnit)));
  TRY(up(m->fft_p1_units, u1.data(), u1.size() * sizeof(FftUnit)));
  TRY(up(m->fft_p2_units, u2.data(), u2.size() * sizeof(FftUnit)));
  TRY(up(P.items, m->items.data(), batch * sizeof(Item)));
  TRY(up(P.nodes, m->nodes.data(), m->nodes.size() * sizeof(Node)));
  TRY(up(P.rowleaf, rowleaf.data(), row0 * sizeof(int32_t)));
  TRY(up(m->wu, m->wu_h.data(), m->nwu * sizeof(WorkUnit)));
  TRY(up(m->nu, m->nu_h.data(), m->nnu * sizeof(NodeUnit)));
  HIP_TRY(hipMemsetAsync(P.status, 0, batch * sizeof(int32_t), s));
  HIP_TRY(hipMemsetAsync(P.diag, 0, 4 * batch * sizeof(int32_t), s));
  HIP_TRY(hipMemsetAsync(P.rankL, 0, node0 * sizeof(int32_t), s));
  HIP_TRY(hipMemsetAsync(P.rankU, 0, node0 * sizeof(int32_t), s));
  HIP_TRY(hipMemsetAsync(P.rankP, 0, node0 * sizeof(int32_t), s));
  for (int i = 0; i < batch; ++i) {
    const Item& it = m->items[i];
    HIP_TRY(hipMemcpyAsync(P.dplus + it.row0, ops[i].d_plus, it.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(P.dminus + it.row0, ops[i].d_minus, it.n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  // ---- device construction
  HFDE_LAUNCH(k_gl_weights, dim3(batch), dim3(1024), 0, s, P);
  HFDE_LAUNCH(k_hankel_aca, dim3(batch), dim3(512), 0, s, P, opts->tol);
  HFDE_LAUNCH(k_hankel_truncate, dim3(batch), dim3(256), 0, s, P);
  for (int i = 0; i < batch; ++i) {
    const Item& it = m->items[i];
    if (it.L > 0)
      HFDE_LAUNCH(k_assemble_bases, dim3(unsigned((it.n + 255) / 256), it.L), dim3(256), 0, s, P, i);
    HFDE_LAUNCH(k_assemble_leaves, dim3(unsigned(int64_t(1) << it.L)), dim3(256), 0, s, P, i, b);
    HFDE_LAUNCH(k_twiddles, dim3(unsigned(std::min<int64_t>(((int64_t(1) << it.fftlog) + 255) / 256, 4096))),
                       dim3(256), 0, s, P, i);
  }
  // far-field multipliers mu = FFT(c_far) -> lambda + i conj(lambda)
  if (m->n_fft_small) {
    int maxlog = 0;
    for (int i : m->small_items) maxlog = std::max(maxlog, m->items[i].fftlog);
    HFDE_LAUNCH(k_fft_small, dim3(m->n_fft_small), dim3(512), (size_t(1) << maxlog) * sizeof(double2), s,
                       P, m->fft_small_units, 0, (const double*)nullptr, 0, (double*)nullptr, 0,
                       (const double*)nullptr, 0);
  }
  if (m->n_fft_p1) {
    const size_t lds = m->fft4_lds;
    HFDE_LAUNCH(k_fft4_pass1, dim3(m->n_fft_p1 / kNCF), dim3(kFft4WG), lds, s, P, m->fft_p1_units, 0, false,
                       (const double*)nullptr, 0);
    HFDE_LAUNCH(k_fft4_pass2, dim3(m->n_fft_p2 / kNCF), dim3(kFft4WG), lds, s, P, m->fft_p2_units, 0, false,
                       (const double*)nullptr, 0, (double*)nullptr, 0, (const double*)nullptr, 0);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(m->items.data(), P.items, batch * sizeof(Item), hipMemcpyDeviceToHost));
  for (const Item& it : m->items) m->max_rank_A = std::max(m->max_rank_A, it.r);
  TRY(read_capped_A(m));
  {  // launch shapes tuned earlier in the process for this tree signature
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    auto f = g_tuned.find(tune_key(m));
    if (f != g_tuned.end()) {
      m->core_threads = f->second.core_threads;
      m->leaf_threads = f->second.leaf_threads;
      m->gram_rows = f->second.gram_rows;
      m->fuse_rows = f->second.fuse_rows;
    }
  }
  *out = m;
  return HODLR_OK;
}

hodlr_status hodlr_build(hodlr_ctx ctx, const fde_operator* ops, int batch, const hodlr_opts* opts,
                         hodlr_mat* out) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!out) return set_arg(ctx, 5);
  return build_impl(ctx, ops, batch, opts, nullptr, 0, out, nullptr);
}

// Workspace sizes already computed in this process, by the arguments that
// determine them (sizes, leaf, precision and the launch shapes tuned for the
// tree, if any): the sizing pass plans the factorisation schedule at every
// shape the autotuner tries, which costs milliseconds of host time for large
// batches, and a loop that builds matrices of one shape asks again and again.
static std::map<std::vector<int64_t>, size_t> g_ws_sizes;
static std::mutex g_ws_mu;

static hodlr_status workspace_size_cached(const fde_operator* ops, int batch, const hodlr_opts* opts,
                                          size_t* bytes) {
  if (!ops || batch < 1 || !opts) return build_impl(nullptr, ops, batch, opts, nullptr, 0, nullptr, bytes);
  std::vector<int64_t> key{batch, opts->leaf, opts->prec, env_int("HODLR_FUSE_ROWS", -1)};
  int64_t total = 0, Lmax = 0;
  for (int i = 0; i < batch; ++i) {
    key.push_back(ops[i].n);
    total += ops[i].n;
    Lmax = std::max<int64_t>(Lmax, levels_for(ops[i].n, std::max(1, opts->leaf)));
  }
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    auto f = g_tuned.find(TuneKey{batch, total, int(Lmax), opts->leaf});
    key.push_back(f != g_tuned.end() ? f->second.gram_rows : -1);
    key.push_back(f != g_tuned.end() ? f->second.fuse_rows : -1);
  }
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto f = g_ws_sizes.find(key);
    if (f != g_ws_sizes.end()) {
      *bytes = f->second;
      return HODLR_OK;
    }
  }
  size_t need = 0;
  const hodlr_status st = build_impl(nullptr, ops, batch, opts, nullptr, 0, nullptr, &need);
  if (st != HODLR_OK) return st;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  g_ws_sizes[key] = need;
  *bytes = need;
  return HODLR_OK;
}

hodlr_status hodlr_workspace_size(const fde_operator* ops, int batch, const hodlr_opts* opts, size_t* bytes) {
  if (!bytes) return HODLR_EINVAL;
  return workspace_size_cached(ops, batch, opts, bytes);
}

hodlr_status hodlr_build_ws(hodlr_ctx ctx, const fde_operator* ops, int batch, const hodlr_opts* opts,
                            void* workspace, size_t ws_bytes, hodlr_mat* out) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!workspace) return set_arg(ctx, 5);
  if (!out) return set_arg(ctx, 7);
  size_t need = 0;
  hodlr_status st = workspace_size_cached(ops, batch, opts, &need);
  if (st == HODLR_EINVAL) st = build_impl(ctx, ops, batch, opts, nullptr, 0, nullptr, &need);   // names the argument
  if (st != HODLR_OK) return st;
  // the workspace's own start may be unaligned: carve from the first 256-byte boundary
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(workspace);
  const uintptr_t a1 = (a0 + 255) & ~uintptr_t(255);
  if (ws_bytes < need || ws_bytes < (a1 - a0)) return set_arg(ctx, 6);
  return build_impl(ctx, ops, batch, opts, reinterpret_cast<void*>(a1), ws_bytes - (a1 - a0), out, nullptr);
}

hodlr_status hodlr_update_coefficients(hodlr_ctx ctx, hodlr_mat m, const fde_operator* ops) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!m) return set_arg(ctx, 2);
  if (!ops) return set_arg(ctx, 3);
  for (int i = 0; i < m->batch; ++i) {
    const fde_operator& o = ops[i];
    const Item& it = m->items[i];
    const double nu = (o.dt > 0.0 && o.dx > 0.0) ? o.dt / std::pow(o.dx, o.alpha) : -1.0;
    if (o.n != it.n || o.alpha != it.alpha || o.shift != it.shift || !(std::fabs(nu - it.nu) <= 1e-14 * it.nu) ||
        !o.d_plus || !o.d_minus || o.discretization != it.kind)
      return set_arg(ctx, 3);
  }
  hipStream_t s = ctx->stream;
  DevPtrs& P = m->P;
  const int batch = m->batch;
  for (int i = 0; i < batch; ++i) {
    const Item& it = m->items[i];
    HIP_TRY(hipMemcpyAsync(P.dplus + it.row0, ops[i].d_plus, it.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(P.dminus + it.row0, ops[i].d_minus, it.n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(hipMemsetAsync(P.status, 0, batch * sizeof(int32_t), s));
  HIP_TRY(hipMemsetAsync(P.diag, 0, 4 * batch * sizeof(int32_t), s));
  HIP_TRY(hipMemsetAsync(P.rankL, 0, m->total_nodes * sizeof(int32_t), s));
  HIP_TRY(hipMemsetAsync(P.rankU, 0, m->total_nodes * sizeof(int32_t), s));
  HIP_TRY(hipMemsetAsync(P.rankP, 0, m->total_nodes * sizeof(int32_t), s));
  HFDE_LAUNCH(k_hankel_aca, dim3(batch), dim3(512), 0, s, P, m->opts.tol);
  HFDE_LAUNCH(k_hankel_truncate, dim3(batch), dim3(256), 0, s, P);
  for (int i = 0; i < batch; ++i) {
    const Item& it = m->items[i];
    if (it.L > 0)
      HFDE_LAUNCH(k_assemble_bases, dim3(unsigned((it.n + 255) / 256), it.L), dim3(256), 0, s, P, i);
    HFDE_LAUNCH(k_assemble_leaves, dim3(unsigned(int64_t(1) << it.L)), dim3(256), 0, s, P, i, m->b);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(m->items.data(), P.items, batch * sizeof(Item), hipMemcpyDeviceToHost));
  m->max_rank_A = 0;
  for (const Item& it : m->items) m->max_rank_A = std::max(m->max_rank_A, it.r);
  TRY(read_capped_A(m));
  m->factored = false;
  return HODLR_OK;
}

// Algorithmic FP64 flops of the factorisation of Sec. 3.5 as carried out
// (ranks read back from the device): per internal node the two
// recompressions of the off-diagonal Schur blocks and the one of the pending
// update (Gram matrices 2 m R^2, factor formation 2 m R r), the projections
// that form U~12, V~21 and the four inverse-factor blocks (one HODLR product
// of a child subtree on r columns each: 2 r (n b + 2 n sum of child ranks)),
// C and W (2 n1 r^2, 2 n2 r^2); per leaf the Schur update 2 m^2 rp, the LU
// (2/3) m^3 and the two triangular inverses (2/3) m^3.
struct FlopSplit {
  double total = 0.0;   // whole factorisation
  double core = 0.0;    // recompression cores (k_core): per recompression of R columns to rank r,
                        // two pivoted Cholesky ~2 R^3, K ~2 R^3, QRCP ~4 R^2 r, Q 4 R r^2, M_U, M_V ~R r^2 + 2 R^2 r
  double gram = 0.0;    // Gram matrices (k_gram_partial): 2 rows x cols x cols each
  double leaf = 0.0;    // leaves (k_leaf_task): pending update, LU, both inverses
  double node_rec = 0.0;   // fused phase A, first part (k_node_recompress): Grams, cores, forms of S12, S21
  double node_pend = 0.0;  // fused phase A, last part (k_node_pending): C, W, pending Grams, core, forms
  double sp_expand = 0.0;  // subtree products (U~12, V~21, inverse blocks): leaf blocks + half the levels (k_sp_expand)
  double sp_project = 0.0; // subtree products: the other half of the levels, the projections (k_sp_project)
};

static FlopSplit factor_flop_split(hodlr_mat m);

static double factor_flop_model(hodlr_mat m) { return factor_flop_split(m).total; }

static FlopSplit factor_flop_split(hodlr_mat m) {
  FlopSplit out;
  std::vector<int32_t> rl(m->total_nodes), ru(m->total_nodes), rp(m->total_nodes);
  (void)hipMemcpy(rl.data(), m->P.rankL, rl.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
  (void)hipMemcpy(ru.data(), m->P.rankU, ru.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
  (void)hipMemcpy(rp.data(), m->P.rankP, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
  double fl = 0.0;
  for (const Item& it : m->items) {
    // subtree product cost per column: leaves (m^2) + 2 * rows * rank per level below
    // (the projection and the expansion each), kept as the leaf part and the level part
    std::vector<double> sub(size_t(1) << (it.L + 1), 0.0);   // per node (depth-major index)
    std::vector<double> subl(size_t(1) << (it.L + 1), 0.0);  // its leaf part
    auto idx = [&](int d, int64_t j) { return size_t((int64_t(1) << d) - 1 + j); };
    for (int d = it.L; d >= 0; --d)
      for (int64_t j = 0; j < (int64_t(1) << d); ++j) {
        const Node nd = m->nodes[node_index(it, d, j)];
        if (d == it.L) { sub[idx(d, j)] = subl[idx(d, j)] = double(nd.size) * nd.size; continue; }
        const int64_t ni = node_index(it, d, j);
        const double rr = 0.5 * (rl[ni] + ru[ni]);
        sub[idx(d, j)] = sub[idx(d + 1, 2 * j)] + sub[idx(d + 1, 2 * j + 1)] + 4.0 * nd.size * rr;
        subl[idx(d, j)] = subl[idx(d + 1, 2 * j)] + subl[idx(d + 1, 2 * j + 1)];
      }
    for (int d = 0; d <= it.L; ++d)
      for (int64_t j = 0; j < (int64_t(1) << d); ++j) {
        const int64_t ni = node_index(it, d, j);
        const Node nd = m->nodes[ni];
        const double n = nd.size, pr = rp[ni];
        if (d == it.L) {
          fl += 2.0 * n * n * pr + (4.0 / 3.0) * n * n * n;
          out.leaf += 2.0 * n * n * pr + (4.0 / 3.0) * n * n * n;
          continue;
        }
        const double n1 = double(nd.size / 2), n2 = n - n1;
        const double r = it.r, R = r + pr, r12 = ru[ni], r21 = rl[ni];
        auto core = [](double Rc, double rc) { return 4.0 * Rc * Rc * Rc + 6.0 * Rc * Rc * rc + 5.0 * Rc * rc * rc; };
        const double rpc = rp[node_index(it, d + 1, 2 * j + 1)], Rp = pr + r12;
        if (std::max(n1, n2) <= double(m->fuse_used)) {
          out.node_rec += core(R, r12) + core(R, r21) + 4.0 * n * R * R + 2.0 * n * R * (r12 + r21);
          out.node_pend += 2.0 * n1 * r21 * r12 + 2.0 * n2 * r21 * r12 + core(Rp, rpc) + 4.0 * n2 * Rp * Rp +
                           4.0 * n2 * Rp * rpc;
        } else {
          out.core += core(R, r12) + core(R, r21) + core(Rp, rpc);
          out.gram += 4.0 * n * R * R + 2.0 * n1 * r21 * r12 + 4.0 * n2 * Rp * Rp;
        }
        fl += 2 * (2.0 * n * R * R) + 2.0 * n * R * (r12 + r21);              // S12, S21 recompression
        fl += 2.0 * n2 * (pr + r12) * (pr + r12) * 2 + 2.0 * n2 * (pr + r12) * r12;  // pending recompression
        fl += 2.0 * n1 * r12 * r21 + 2.0 * n2 * r21 * r12;                      // C and W
        const double s1 = sub[idx(d + 1, 2 * j)], s2 = sub[idx(d + 1, 2 * j + 1)];
        fl += 2.0 * (r12 + r21) * s1;                                           // U~12, V~21
        fl += 2.0 * r21 * (s1 + s2) + 2.0 * r12 * (s1 + s2);                    // inverse blocks
        const double l1 = subl[idx(d + 1, 2 * j)], l2 = subl[idx(d + 1, 2 * j + 1)];
        const double leafpart = 2.0 * (r12 + r21) * l1 + 2.0 * (r21 + r12) * (l1 + l2);
        const double levelpart = 2.0 * (r12 + r21) * (s1 - l1) + 2.0 * (r21 + r12) * (s1 + s2 - l1 - l2);
        out.sp_expand += leafpart + 0.5 * levelpart;
        out.sp_project += 0.5 * levelpart;
      }
  }
  out.total = fl;
  return out;
}

hodlr_status hodlr_get_info(hodlr_mat m, hodlr_mat_info* info) {
  if (!m || !info) return HODLR_EINVAL;
  info->batch = m->batch;
  info->leaf = m->b;
  info->max_levels = m->Lmax;
  info->total_n = m->total_n;
  info->max_rank_A = m->max_rank_A;
  info->max_rank_factors = m->max_rank_factors;
  // bytes of one single-RHS solve: leaf inverses (both triangles) + both
  // families of off-diagonal factors at their actual ranks
  size_t bytes = 0;
  if (m->factored) {
    std::vector<int32_t> rl(m->total_nodes), ru(m->total_nodes);
    (void)hipMemcpy(rl.data(), m->P.rankL, rl.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
    (void)hipMemcpy(ru.data(), m->P.rankU, ru.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
    const size_t fb = m->opts.prec == HODLR_FP64 ? 8 : (m->opts.prec == HODLR_MIXED_FP32 ? 4 : 4);
    for (const Item& it : m->items) {
      for (int d = 0; d < it.L; ++d)
        for (int64_t j = 0; j < (int64_t(1) << d); ++j) {
          const Node nd = m->nodes[node_index(it, d, j)];
          const int64_t idx = node_index(it, d, j);
          bytes += size_t(nd.size) * (rl[idx] + ru[idx]) * fb;
        }
      for (int64_t l = 0; l < (int64_t(1) << it.L); ++l) {
        const Node nd = m->nodes[node_index(it, it.L, l)];
        bytes += size_t(nd.size) * nd.size * fb;
      }
    }
  }
  info->bytes_factors = bytes;
  info->bytes_device = m->bytes_device;
  const FlopSplit fs = m->factored ? factor_flop_split(m) : FlopSplit{};
  info->factor_flops = fs.total;
  info->core_flops = fs.core;
  info->gram_flops = fs.gram;
  info->leaf_flops = fs.leaf;
  info->node_rec_flops = fs.node_rec;
  info->node_pend_flops = fs.node_pend;
  info->sp_expand_flops = fs.sp_expand;
  info->sp_project_flops = fs.sp_project;
  return HODLR_OK;
}

hodlr_status hodlr_matvec(hodlr_ctx ctx, hodlr_mat m, const double* x, double* y, int nrhs, int64_t ld) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!m) return set_arg(ctx, 2);
  if (!x) return set_arg(ctx, 3);
  if (!y) return set_arg(ctx, 4);
  if (nrhs < 1) return set_arg(ctx, 5);
  if (ld < m->total_n) return set_arg(ctx, 6);
  hipStream_t s = ctx->stream;
  for (int c0 = 0; c0 < nrhs; c0 += kNCS) {
    const int cn = std::min(kNCS, nrhs - c0);
    const double* xc = x + int64_t(c0) * ld;
    double* yc = y + int64_t(c0) * ld;
    HFDE_LAUNCH(k_hmatvec_A_project, dim3(m->nwu), dim3(64), 0, s, m->P, m->wu, xc, ld, cn, m->partL,
                       m->Lmax);
    if (m->nnu)
      HFDE_LAUNCH(k_hmatvec_A_reduce, dim3(m->nnu), dim3(64), 0, s, m->P, m->nu, cn, m->partL, m->zL,
                         m->Lmax);
    HFDE_LAUNCH(k_hmatvec_A_expand, dim3(m->nwu), dim3(64), 0, s, m->P, m->wu, xc, ld, yc, ld, cn, m->zL,
                       m->b);
  }
  HIP_TRY(hipGetLastError());
  return HODLR_OK;
}

hodlr_status hodlr_get_weights(hodlr_ctx ctx, hodlr_mat m, int item, double* out, int64_t count) {
  if (!ctx) return HODLR_EINVAL;
  if (!m || m->sizing) return set_arg(ctx, 2);
  if (item < 0 || item >= m->batch) return set_arg(ctx, 3);
  if (!out) return set_arg(ctx, 4);
  const Item& it = m->items[item];
  if (count < 0 || count > it.n + 3) return set_arg(ctx, 5);
  if (count == 0) return HODLR_OK;
  hipStream_t s = ctx->stream;
  HIP_TRY(hipMemcpyAsync(out, m->P.g + it.g0, count * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return HODLR_OK;
}

hodlr_status hodlr_toeplitz_matvec(hodlr_ctx ctx, hodlr_mat m, const double* x, double* y, int nrhs, int64_t ld) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!m) return set_arg(ctx, 2);
  if (!x) return set_arg(ctx, 3);
  if (!y) return set_arg(ctx, 4);
  if (nrhs < 1) return set_arg(ctx, 5);
  if (ld < m->total_n) return set_arg(ctx, 6);
  if (x == y) return set_arg(ctx, 4);
  launch_fft_matvec(m, x, ld, y, ld, nullptr, 0, nrhs, ctx->stream);
  HIP_TRY(hipGetLastError());
  return HODLR_OK;
}

hodlr_status hodlr_toeplitz_matvec_noalloc(hodlr_ctx ctx, hodlr_mat m, const double* x, double* y, int nrhs,
                                           int64_t ld) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!m) return set_arg(ctx, 2);
  if (!x) return set_arg(ctx, 3);
  if (!y) return set_arg(ctx, 4);
  if (nrhs < 1) return set_arg(ctx, 5);
  if (ld < m->total_n) return set_arg(ctx, 6);
  if (x == y) return set_arg(ctx, 4);
  if (size_t(m->fws_packed) * sizeof(double2) > kNoallocScratchBytes) {
    fprintf(stderr, "hodlr_fde: hodlr_toeplitz_matvec_noalloc: the matrix needs %lld bytes of transform scratch, "
                    "above the static maximum of %zu\n",
            (long long)(size_t(m->fws_packed) * sizeof(double2)), kNoallocScratchBytes);
    return set_arg(ctx, 2);
  }
  void* sp = nullptr;
  TRY(scratch_address(&sp));
  DevPtrs Ps = m->P;
  Ps.fws = static_cast<double2*>(sp);
  Ps.fws_compact = 1;
  launch_fft_matvec_p(m, Ps, x, ld, y, ld, nullptr, 0, nrhs, ctx->stream);
  HIP_TRY(hipGetLastError());
  return HODLR_OK;
}

hodlr_status hodlr_set_tuning(hodlr_ctx ctx, hodlr_mat m, const hodlr_tuning* t) {
  if (!ctx) return HODLR_EINVAL;
  if (!m) return set_arg(ctx, 2);
  if (!t || t->core_threads != kCoreWG || (t->leaf_threads != 256 && t->leaf_threads != 512) ||
      t->gram_rows < 32 || t->gram_rows > 65536 || t->gram_rows % 32 != 0 || t->fuse_rows < 0)
    return set_arg(ctx, 3);
  if (t->gram_rows != m->gram_rows || t->fuse_rows != m->fuse_rows) {
    m->gram_rows = t->gram_rows;
    m->fuse_rows = t->fuse_rows;
    m->mwg_planned = false;
    m->mwg_kind.clear();
    m->mwg_side.clear();
    m->mwg_grid.clear();
    m->mwg_off.clear();
    m->mwg_off2.clear();
  }
  m->core_threads = t->core_threads;
  m->leaf_threads = t->leaf_threads;
  return HODLR_OK;
}

hodlr_status hodlr_autotune(hodlr_ctx ctx, hodlr_mat m, hodlr_tuning* best) {
  if (!ctx) return HODLR_EINVAL;
  if (!m) return set_arg(ctx, 2);
  hipStream_t s = ctx->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  auto replan = [&](int g, int f) -> hodlr_status {
    if (g == m->gram_rows && f == m->fuse_rows && m->mwg_planned) return HODLR_OK;
    m->gram_rows = g;
    m->fuse_rows = f;
    m->mwg_planned = false;
    m->mwg_kind.clear();
    m->mwg_side.clear();
    m->mwg_grid.clear();
    m->mwg_off.clear();
    m->mwg_off2.clear();
    return plan_mwg(m);
  };
  // factorisation time of one launch-shape choice: best of two runs
  auto trial = [&](const TuneVal& v, double& ms) -> hodlr_status {
    TRY(replan(v.gram_rows, v.fuse_rows));
    m->core_threads = v.core_threads;
    m->leaf_threads = v.leaf_threads;
    ms = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
      HIP_TRY(hipEventRecord(e0, s));
      enqueue_mwg(m, s);
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      float t = 0.0f;
      HIP_TRY(hipEventElapsedTime(&t, e0, e1));
      ms = std::min(ms, double(t));
    }
    return HODLR_OK;
  };
  // coordinate search: fused-node threshold, then Gram chunk rows, then the
  // work-group sizes of the cores and leaves
  TuneVal bestv{kCoreWG, m->leaf_threads, m->gram_rows, m->fuse_rows};
  double best_ms = 1e300;
  auto consider = [&](TuneVal v) -> hodlr_status {
    double ms = 0.0;
    TRY(trial(v, ms));
    if (ms < best_ms) {
      best_ms = ms;
      bestv = v;
    }
    return HODLR_OK;
  };
  for (int f : {0, 128, 256, 512, 1024}) TRY(consider(TuneVal{bestv.core_threads, bestv.leaf_threads, bestv.gram_rows, f}));
  for (int g : {128, 256, 512})
    if (g != bestv.gram_rows) TRY(consider(TuneVal{bestv.core_threads, bestv.leaf_threads, g, bestv.fuse_rows}));
  const TuneVal base = bestv;
  for (int lt : {256, 512})
    if (lt != base.leaf_threads) TRY(consider(TuneVal{kCoreWG, lt, base.gram_rows, base.fuse_rows}));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  TRY(replan(bestv.gram_rows, bestv.fuse_rows));
  m->core_threads = bestv.core_threads;
  m->leaf_threads = bestv.leaf_threads;
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    g_tuned[tune_key(m)] = bestv;
  }
  if (best) {
    best->core_threads = bestv.core_threads;
    best->leaf_threads = bestv.leaf_threads;
    best->gram_rows = bestv.gram_rows;
    best->fuse_rows = bestv.fuse_rows;
    best->factor_ms = best_ms;
  }
  HIP_TRY(hipGetLastError());
  return HODLR_OK;
}

hodlr_status hodlr_factor(hodlr_ctx ctx, hodlr_mat m, hodlr_info* info) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!m) return set_arg(ctx, 2);
  hipStream_t s = ctx->stream;
  const size_t lds = kFactorLdsBytes;
  HIP_TRY(hipMemsetAsync(m->P.status, 0, m->batch * sizeof(int32_t), s));
  HIP_TRY(hipMemsetAsync(m->P.diag, 0, 4 * m->batch * sizeof(int32_t), s));
  const char* env = getenv("HODLR_FACTOR_PATH");
  const bool single = (env && env[0] == 's');
  if (single) {
    HFDE_LAUNCH(k_factor, dim3(m->batch), dim3(kWG), lds, s, m->P, m->b, m->opts.max_rank);
  } else {
    TRY(plan_mwg(m));
    enqueue_mwg(m, s);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<int32_t> stv(m->batch), dg(4 * m->batch);
  HIP_TRY(hipMemcpy(stv.data(), m->P.status, m->batch * sizeof(int32_t), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(dg.data(), m->P.diag, 4 * m->batch * sizeof(int32_t), hipMemcpyDeviceToHost));
  hodlr_status res = HODLR_OK;
  int maxr = 0, badp = -1, badl = -1;
  for (int i = 0; i < m->batch; ++i) {
    maxr = std::max(maxr, dg[4 * i + 1]);
    if ((stv[i] & 1) && badp < 0) { badp = i; badl = dg[4 * i]; }
    if (stv[i] & 1) res = HODLR_ESINGULAR;
    else if ((stv[i] & 4) && res == HODLR_OK) res = HODLR_ERANK;
  }
  if (m->capped_A && res == HODLR_OK) res = HODLR_ERANK;
  m->max_rank_factors = maxr;
  m->factored = true;
  // low precision copies
  if (m->opts.prec != HODLR_FP64) {
    const int64_t lvl = int64_t(m->allocs.size());
    (void)lvl;
    int64_t nlvl = 0;
    for (const Item& it : m->items) nlvl += int64_t(it.L + 1) * it.n * kRS;
    const int64_t nleafv = m->total_leaves * m->b * m->b;
    if (!m->LUinv32) TRY(alloc_lowprec(m));
    HFDE_LAUNCH(k_convert<float>, dim3(4096), dim3(256), 0, s, m->P.LUinv, m->LUinv32, nleafv);
    HFDE_LAUNCH(k_convert<float>, dim3(4096), dim3(256), 0, s, m->P.IL, m->IL32, nlvl);
    HFDE_LAUNCH(k_convert<float>, dim3(4096), dim3(256), 0, s, m->P.IU, m->IU32, nlvl);
    if (m->opts.prec == HODLR_MIXED_BF16) {
      HFDE_LAUNCH(k_convert<bf16>, dim3(4096), dim3(256), 0, s, m->P.IL, m->IL16, nlvl);
      HFDE_LAUNCH(k_convert<bf16>, dim3(4096), dim3(256), 0, s, m->P.IU, m->IU16, nlvl);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (info) {
    memset(info, 0, sizeof(*info));
    info->status = res;
    info->max_rank = maxr;
    info->leaf = badp;
    info->row = badl;
  }
  return res;
}

// One GMRES-IR cycle for one column: d (into m->dbuf) from gmres_m
// iterations on M d = b - M x, right-preconditioned by the solve with the
// factors of precision p; the exact residual and products in FP64.
static void gmres_cycle(hodlr_mat m, int p, const double* b, const double* x, hipStream_t s) {
  const int64_t tn = m->total_n;
  const int M = m->opts.gmres_m, B = m->batch;
  const dim3 grid(m->step_slices, B), one(unsigned((B + 255) / 256));
  GmState& G = m->gms;
  double* V = m->gmV;
  double* Z = m->gmZ;
  launch_fft_matvec(m, x, tn, m->rbuf, tn, b, tn, 1, s);                      // r = b - M x
  HFDE_LAUNCH(k_gm_norm2, grid, dim3(256), 0, s, m->P, m->rbuf, G, B);
  HFDE_LAUNCH(k_gm_normalize, grid, dim3(256), 0, s, m->P, m->rbuf, V, G, B, -1);
  for (int j = 0; j < M; ++j) {
    double* vj = V + int64_t(j) * tn;
    double* zj = Z + int64_t(j) * tn;
    launch_solve(m, p, vj, tn, zj, tn, 1, s);                                  // z_j = M_low^{-1} v_j
    launch_fft_matvec(m, zj, tn, m->dbuf, tn, nullptr, 0, 1, s);               // w = M z_j
    HFDE_LAUNCH(k_gm_dots, grid, dim3(256), 0, s, m->P, V, tn, j, m->dbuf, G.h1, B);
    HFDE_LAUNCH(k_gm_subtract, grid, dim3(256), 0, s, m->P, V, tn, j, m->dbuf, G.h1, G, B);
    HFDE_LAUNCH(k_gm_dots, grid, dim3(256), 0, s, m->P, V, tn, j, m->dbuf, G.h2, B);
    HFDE_LAUNCH(k_gm_subtract, grid, dim3(256), 0, s, m->P, V, tn, j, m->dbuf, G.h2, G, B);
    HFDE_LAUNCH(k_gm_norm2, grid, dim3(256), 0, s, m->P, m->dbuf, G, B);
    HFDE_LAUNCH(k_gm_normalize, grid, dim3(256), 0, s, m->P, m->dbuf, V + int64_t(j + 1) * tn, G, B, j);
    HFDE_LAUNCH(k_gm_givens, one, dim3(256), 0, s, G, B, j);
  }
  HFDE_LAUNCH(k_gm_solve_y, one, dim3(256), 0, s, G, B, M);
  HFDE_LAUNCH(k_gm_combine, grid, dim3(256), 0, s, m->P, Z, tn, M, G, m->dbuf);  // d = Z y
}

// x <- M_p^{-1} b (b in m->bbuf, cn columns), then FP64 refinement sweeps
// r = b - M x (exact), d = M_p^{-1} r, x += d, until ||d|| <= rtol ||x|| for
// every problem and column (the correction estimates the forward error; the
// residual of a stiff M floors near u ||M|| ||x||), or the correction stalls
// (shrinks by less than 10%), or maxsw sweeps.  1: converged, 0: not, negative:
// a HIP error status.  rel_r, rel_d: worst ||r||/||b|| and ||d||/||x||.
static int sweep_solve(hodlr_mat m, int p, int maxsw, double* xc, int64_t ld, int cn, hipStream_t s,
                       double& rel_r, double& rel_d, int& iters) {
  const int64_t tn = m->total_n;
  const int nb_off = m->batch * kNCS;
  double* nrm = m->norms;   // [0]: ||r||^2  [1]: ||b||^2  [2]: ||d||^2  [3]: ||x||^2 (each batch x kNCS)
  launch_norms(m, m->bbuf, tn, cn, nrm + nb_off, s);
  launch_solve(m, p, m->bbuf, tn, xc, ld, cn, s);
  double prev = 1e300;
  std::vector<double> h(4 * nb_off);
  rel_r = rel_d = 1e300;
  const bool gm = m->opts.gmres_m > 0 && cn == 1;
  for (int sweep = 0; sweep < maxsw; ++sweep) {
    if (gm) {
      gmres_cycle(m, p, m->bbuf, xc, s);                          // d in dbuf, r in rbuf
    } else {
      launch_fft_matvec(m, xc, ld, m->rbuf, tn, m->bbuf, tn, cn, s);
      launch_solve(m, p, m->rbuf, tn, m->dbuf, tn, cn, s);
    }
    launch_axpby(tn, cn, 1.0, xc, ld, 1.0, m->dbuf, tn, xc, ld, s);
    launch_norms(m, m->rbuf, tn, cn, nrm, s);
    launch_norms(m, m->dbuf, tn, cn, nrm + 2 * nb_off, s);
    launch_norms(m, xc, ld, cn, nrm + 3 * nb_off, s);
    if (hipMemcpyAsync(h.data(), nrm, h.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return HODLR_EHIP;
    rel_r = rel_d = 0.0;
    for (int q = 0; q < m->batch * cn; ++q) {
      const double bq = h[nb_off + q], xq = h[3 * nb_off + q];
      rel_r = std::max(rel_r, bq > 0 ? std::sqrt(h[q] / bq) : 0.0);
      rel_d = std::max(rel_d, xq > 0 ? std::sqrt(h[2 * nb_off + q] / xq) : 0.0);
    }
    iters = std::max(iters, sweep + 1);
    if (!(rel_d == rel_d)) return 0;   // NaN
    if (rel_d <= m->opts.rtol) return 1;
    if (rel_d > 0.9 * prev) return 0;  // stalled or diverging
    prev = rel_d;
  }
  return 0;
}

hodlr_status hodlr_solve(hodlr_ctx ctx, hodlr_mat m, double* x, int nrhs, int64_t ld, hodlr_info* info) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!m) return set_arg(ctx, 2);
  if (!x) return set_arg(ctx, 3);
  if (nrhs < 1) return set_arg(ctx, 4);
  if (ld < m->total_n) return set_arg(ctx, 5);
  if (!m->factored) return HODLR_ESTATE;
  hipStream_t s = ctx->stream;
  const int prec = m->opts.prec;
  hodlr_status res = HODLR_OK;
  int iters = 0;
  double worst = 0.0, worst_d = 0.0;
  bool fallback = false;
  // GMRES-IR refines one column at a time, in place in a total_n-row copy
  const int group = m->opts.gmres_m > 0 && m->opts.refine_max > 0 ? 1 : kNCS;
  for (int c0 = 0; c0 < nrhs; c0 += group) {
    const int cn = std::min(group, nrhs - c0);
    double* xc = x + int64_t(c0) * ld;
    const int64_t tn = m->total_n;
    if (m->opts.refine_max <= 0) {
      launch_solve(m, prec, xc, ld, xc, ld, cn, s);
      continue;
    }
    // keep b, then the refined solve at the stored precision; a low-precision
    // solve that does not converge is redone from b with the FP64 factors
    HIP_TRY(hipMemcpy2DAsync(m->bbuf, tn * sizeof(double), xc, ld * sizeof(double), tn * sizeof(double), cn,
                             hipMemcpyDeviceToDevice, s));
    double rr = 0, rd = 0;
    int conv = sweep_solve(m, prec, m->opts.refine_max, xc, ld, cn, s, rr, rd, iters);
    if (conv < 0) return hodlr_status(conv);
    if (!conv && prec != HODLR_FP64) {
      fallback = true;
      conv = sweep_solve(m, HODLR_FP64, std::max(4, m->opts.refine_max), xc, ld, cn, s, rr, rd, iters);
      if (conv < 0) return hodlr_status(conv);
    }
    if (!conv) res = HODLR_ENOCONV;
    worst = std::max(worst, rr);
    worst_d = std::max(worst_d, rd);
  }
  HIP_TRY(hipGetLastError());
  if (info) {
    memset(info, 0, sizeof(*info));
    info->status = res;
    info->refine_iters = iters;
    info->rel_residual = worst;
    info->max_rank = m->max_rank_factors;
    info->leaf = -1;
    info->row = -1;
    info->used_fallback = fallback ? 1 : 0;
    info->rel_correction = worst_d;
  }
  return res;
}

// One implicit Euler step at the stored precision with a fixed number of
// refinement sweeps: b = u + fscale f, u = M_low^{-1} b, then `sweeps` times
// r = b - M u (exact), d = M_low^{-1} r (or a GMRES-IR cycle), u += d.  With sweeps > 0 the last
// update also folds the step's ||d||/||u|| into m->step_worst.  No host
// synchronisation: the sequence is what a time-step graph captures.
// Right-hand side of an implicit Euler step into m->bbuf: b = u + fscale f,
// or E (u + fscale f) for finite-element problems (E = P1 mass / h; Sec. 2.2.2).
static void launch_step_rhs(hodlr_mat m, const double* u, const double* f, double fscale, hipStream_t s) {
  const int64_t tn = m->total_n;
  if (m->has_mass) {
    HFDE_LAUNCH(k_step_rhs, dim3(m->step_slices, m->batch), dim3(256), 0, s, m->P, u, f, fscale, m->bbuf);
    return;
  }
  if (f) launch_axpby(tn, 1, 1.0, u, tn, fscale, f, tn, m->bbuf, tn, s);
  else launch_axpby(tn, 1, 1.0, u, tn, 0.0, u, tn, m->bbuf, tn, s);
}

static void record_step(hodlr_mat m, double* u, const double* f, double fscale, int sweeps, hipStream_t s) {
  const int64_t tn = m->total_n;
  const int prec = m->opts.prec;
  launch_step_rhs(m, u, f, fscale, s);
  launch_solve(m, prec, m->bbuf, tn, u, tn, 1, s);
  for (int q = 0; q < sweeps; ++q) {
    if (m->opts.gmres_m > 0) {
      gmres_cycle(m, prec, m->bbuf, u, s);     // d in dbuf
    } else {
      launch_fft_matvec(m, u, tn, m->rbuf, tn, m->bbuf, tn, 1, s);
      launch_solve(m, prec, m->rbuf, tn, m->dbuf, tn, 1, s);
    }
    if (q + 1 < sweeps) {
      launch_axpby(tn, 1, 1.0, u, tn, 1.0, m->dbuf, tn, u, tn, s);
    } else {
      HFDE_LAUNCH(k_step_update, dim3(m->step_slices, m->batch), dim3(256), 0, s, m->P, u, m->dbuf,
                  m->step_part, m->step_slices);
      HFDE_LAUNCH(k_step_check, dim3(1), dim3(256), 0, s, m->batch, m->step_part, m->step_slices,
                  m->step_worst);
    }
  }
}

// Steps between two convergence checks of the time loop.
constexpr int kCheckSteps = 32;

hodlr_status hodlr_time_steps(hodlr_ctx ctx, hodlr_mat m, double* u, const double* f, double fscale, int steps,
                              hodlr_info* info) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!m) return set_arg(ctx, 2);
  if (!u) return set_arg(ctx, 3);
  if (steps < 0) return set_arg(ctx, 5);
  if (!m->factored) return HODLR_ESTATE;
  hipStream_t s = ctx->stream;
  const int64_t tn = m->total_n;
  const int sweeps = m->opts.refine_max;
  const bool direct = (s == nullptr || ctx->timing);
  if (!direct && (!m->step_graph || m->graph_u != u || m->graph_f != f || m->graph_sweeps != sweeps ||
                  m->graph_fscale != fscale)) {
    // the legacy null stream cannot be captured, and timed runs bracket every
    // launch with events: those launch the steps directly
    if (m->step_graph) {
      (void)hipGraphExecDestroy(m->step_graph);
      m->step_graph = nullptr;
    }
    hipGraph_t g;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    record_step(m, u, f, fscale, sweeps, s);
    HIP_TRY(hipStreamEndCapture(s, &g));
    HIP_TRY(hipGraphInstantiate(&m->step_graph, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    m->graph_u = u;
    m->graph_f = f;
    m->graph_sweeps = sweeps;
    m->graph_fscale = fscale;
  }
  // Runs of kCheckSteps steps.  With refinement, each run starts from a copy
  // of u and ends with one read-back of the worst correction of its steps; a
  // run in which any step of any problem missed rtol (or went non-finite) is
  // restored and redone step by step on the FP64 factors, each step refined
  // until it converges or stalls.
  const bool check = sweeps > 0;
  bool fallback = false, unconv = false;
  double worst_all = 0.0;
  int iters = sweeps;
  for (int k0 = 0; k0 < steps; k0 += (check ? kCheckSteps : steps)) {
    const int kc = check ? std::min(kCheckSteps, steps - k0) : steps;
    if (check) {
      HIP_TRY(hipMemcpyAsync(m->ukeep, u, tn * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIP_TRY(hipMemsetAsync(m->step_worst, 0, m->batch * sizeof(double), s));
    }
    for (int k = 0; k < kc; ++k) {
      if (direct) record_step(m, u, f, fscale, sweeps, s);
      else HIP_TRY(hipGraphLaunch(m->step_graph, s));
    }
    if (!check) break;
    HIP_TRY(hipMemcpyAsync(m->host_worst, m->step_worst, m->batch * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double w = 0.0;
    for (int q = 0; q < m->batch; ++q) w = std::max(w, m->host_worst[q]);
    if (w <= m->opts.rtol) {
      worst_all = std::max(worst_all, w);
      continue;
    }
    fallback = true;
    HIP_TRY(hipMemcpyAsync(u, m->ukeep, tn * sizeof(double), hipMemcpyDeviceToDevice, s));
    for (int k = 0; k < kc; ++k) {
      launch_step_rhs(m, u, f, fscale, s);
      double rr = 0, rd = 0;
      const int conv = sweep_solve(m, HODLR_FP64, std::max(4, sweeps), u, tn, 1, s, rr, rd, iters);
      if (conv < 0) return hodlr_status(conv);
      if (!conv) unconv = true;
      worst_all = std::max(worst_all, rd);
    }
  }
  HIP_TRY(hipGetLastError());
  const hodlr_status res = unconv ? HODLR_ENOCONV : HODLR_OK;
  if (info) {
    memset(info, 0, sizeof(*info));
    info->refine_iters = iters;
    info->max_rank = m->max_rank_factors;
    info->leaf = -1;
    info->row = -1;
    info->used_fallback = fallback ? 1 : 0;
    // residual of the last step against its right-hand side (still in bbuf)
    info->rel_residual = 0.0;
    if (steps > 0) {
      launch_fft_matvec(m, u, tn, m->rbuf, tn, m->bbuf, tn, 1, s);
      launch_norms(m, m->rbuf, tn, 1, m->norms, s);
      launch_norms(m, m->bbuf, tn, 1, m->norms + m->batch * kNCS, s);
      std::vector<double> nr(m->batch), nb(m->batch);
      HIP_TRY(hipMemcpyAsync(nr.data(), m->norms, nr.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(nb.data(), m->norms + m->batch * kNCS, nb.size() * sizeof(double),
                             hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      double rel = 0.0;
      for (int q = 0; q < m->batch; ++q) rel = std::max(rel, nb[q] > 0 ? std::sqrt(nr[q] / nb[q]) : 0.0);
      info->rel_residual = rel;
    }
    // worst relative correction over every step of every problem (0 without refinement)
    info->rel_correction = worst_all;
    info->status = res;
  }
  return res;
}

// ---- 2D (factored ADI): implemented in adi.hip
}  // extern "C"
