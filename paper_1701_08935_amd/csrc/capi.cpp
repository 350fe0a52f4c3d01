// C ABI and host orchestration of the hot path on one GPU.
//
//   zolo_pencil_create : CSR upload + nested dissection + symbolic analysis
//   zolo_factor        : numeric LDL^T of K_j = A - sigma_hat_j B (Algorithm 2, lines 5-6)
//   zolo_apply_G       : G V of eq. (solve)
//   zolo_filter_apply  : multi-shift block GMRES on G + weighted sum (Algorithm 2, lines 8-9)
//   zolo_solve         : Algorithm 1 (subspace iteration + Rayleigh-Ritz)
//
// Internally every N x p block lives in the nested-dissection ordering, so a
// front's own rows are contiguous; blocks are permuted at the ABI boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <complex>
#include <type_traits>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "front.h"
#include "gemm.h"
#include "krylov.h"
#include "sparse.h"
#include "zolo_internal.h"

using namespace zolo;

namespace zolo {
static thread_local std::string g_err;
// shifts one zolo_inertia call factors together at most (0 = as many as 80% of
// the free device memory holds); a serving worker sets it so that its share of
// the device stays within what admission reserved for it
static thread_local int g_inertia_cap = 0;
void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}
}  // namespace zolo

#define HIPC(x)                                                                     \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      zolo::set_error("%s failed: %s (%s:%d)", #x, hipGetErrorString(e_), __FILE__, __LINE__); \
      return ZOLO_EDEVICE;                                                          \
    }                                                                               \
  } while (0)

#define CHK(x)                  \
  do {                          \
    int rc_ = (x);              \
    if (rc_ != ZOLO_OK) return (zolo_status)rc_; \
  } while (0)

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device memory cache.  Blocks released by arenas are kept, after a device
// synchronization (what hipFree would imply), and handed out again to later
// allocations of about the same size, so that repeated queries do not pay for
// hipMalloc / hipFree of their multi-gigabyte factors.  When hipMalloc fails
// the cached blocks are freed and the allocation is tried once more.  The
// cache is never destroyed (it lives until the process ends).
// The stream a released block was used on and an event recorded there at its
// release: the block is handed out again only once the event has completed,
// whatever the new owner does with it first (kernels on any stream, or
// synchronous copies and clears).
struct ReleaseMark {
  hipEvent_t ev = nullptr;
  hipStream_t stream = nullptr;
  ~ReleaseMark() {
    if (ev) (void)hipEventDestroy(ev);
  }
};

// Streams whose release events the pool may query later: the null stream and
// the streams the library creates itself (serving workers), which retire
// through retire_stream before they are destroyed.  An event recorded on a
// stream the caller may destroy at any time is not queried; arenas on such
// streams synchronize the device when they release.
std::mutex g_streams_m;
std::set<hipStream_t> g_owned_streams;
bool stream_marks_ok(hipStream_t s) {
  if (!s) return true;
  std::lock_guard<std::mutex> lk(g_streams_m);
  return g_owned_streams.count(s) != 0;
}

class DevicePool {
 public:
  static DevicePool& get() {
    static DevicePool* p = new DevicePool();
    return *p;
  }
  // rounded request: 1 MiB granules from 1 MiB up, powers of two below
  static size_t round(size_t bytes) {
    if (bytes >= (1u << 20)) return (bytes + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1);
    size_t r = 256;
    while (r < bytes) r <<= 1;
    return r;
  }
  // a cached block of [bytes, 9/8 bytes] on device dev that is free of pending
  // work: released after a device synchronization, or whose release event has
  // completed
  void* take(size_t bytes, int dev) {
    std::lock_guard<std::mutex> lk(m_);
    auto it = free_.lower_bound(bytes);
    for (; it != free_.end() && it->first <= bytes + bytes / 8; ++it) {
      const Cached& c = it->second;
      if (c.dev != dev) continue;
      if (c.mark && !mark_done(*c.mark)) continue;
      void* p = c.p;
      cached_ -= it->first;
      free_.erase(it);
      return p;
    }
    return nullptr;
  }
  // the blocks released on stream s no longer wait for their events (the
  // stream has been synchronized and is about to be destroyed)
  void drop_marks(hipStream_t s) {
    std::lock_guard<std::mutex> lk(m_);
    for (auto& kv : free_)
      if (kv.second.mark && kv.second.mark->stream == s) kv.second.mark.reset();
  }
  // whether a release event has completed; a pending query result (not ready)
  // is taken off the thread's last-error state, which the caller's own launch
  // checks read, unless an error was already pending there
  static bool mark_done(const ReleaseMark& m) {
    if (hipPeekAtLastError() != hipSuccess) return false;
    const hipError_t e = hipEventQuery(m.ev);
    if (e == hipSuccess) return true;
    (void)hipGetLastError();
    return false;
  }
  // keeps the block for reuse while the cache stays under its cap, three
  // quarters of the device's memory (a block that would exceed it is freed;
  // the caller has synchronized the device).  Mapping fresh device memory
  // costs about 45 GB/s, so a query that reallocates its ~100 GB of factors
  // pays seconds; allocations that find too little free memory empty the
  // cache first (DevArena::alloc).
  void give(void* p, size_t bytes, int dev, const std::shared_ptr<ReleaseMark>& mark) {
    std::lock_guard<std::mutex> lk(m_);
    if (cap_ == 0) {
      size_t fr = 0, tot = 0;
      cap_ = hipMemGetInfo(&fr, &tot) == hipSuccess ? tot / 4 * 3 : ((size_t)48 << 30);
    }
    if (cached_ + bytes > cap_) {
      if (mark) (void)hipEventSynchronize(mark->ev);
      (void)hipFree(p);
      return;
    }
    free_.insert({bytes, Cached{dev, p, mark}});
    cached_ += bytes;
  }
  // Device-memory budget per device (0 = none): blocks handed out to arenas
  // and not yet released count against it.
  bool charge(int dev, size_t bytes) {
    std::lock_guard<std::mutex> lk(m_);
    if (dev < 0 || dev >= kDev) return true;
    if (budget_[dev] && in_use_[dev] + bytes > budget_[dev]) return false;
    in_use_[dev] += bytes;
    return true;
  }
  void uncharge(int dev, size_t bytes) {
    std::lock_guard<std::mutex> lk(m_);
    if (dev >= 0 && dev < kDev) in_use_[dev] -= std::min(bytes, in_use_[dev]);
  }
  void set_budget(int dev, size_t bytes) {
    std::lock_guard<std::mutex> lk(m_);
    if (dev >= 0 && dev < kDev) budget_[dev] = bytes;
  }
  size_t budget(int dev) {
    std::lock_guard<std::mutex> lk(m_);
    return (dev >= 0 && dev < kDev) ? budget_[dev] : 0;
  }
  size_t cached(int dev) {
    std::lock_guard<std::mutex> lk(m_);
    size_t c = 0;
    for (const auto& kv : free_)
      if (kv.second.dev == dev) c += kv.first;
    return c;
  }
  size_t in_use(int dev) {
    std::lock_guard<std::mutex> lk(m_);
    return (dev >= 0 && dev < kDev) ? in_use_[dev] : 0;
  }
  void trim() {
    std::lock_guard<std::mutex> lk(m_);
    if (free_.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto& kv : free_) (void)hipFree(kv.second.p);
    free_.clear();
    cached_ = 0;
  }
  // frees cached blocks of device dev, largest first, until `need` bytes are
  // released (the rest of the cache stays for the next queries)
  void trim_for(size_t need, int dev) {
    std::lock_guard<std::mutex> lk(m_);
    if (free_.empty()) return;
    (void)hipDeviceSynchronize();
    size_t got = 0;
    for (auto it = free_.end(); it != free_.begin() && got < need;) {
      --it;
      if (it->second.dev != dev) continue;
      (void)hipFree(it->second.p);
      got += it->first;
      cached_ -= it->first;
      it = free_.erase(it);
    }
  }

 private:
  static constexpr int kDev = 64;
  std::mutex m_;
  struct Cached {
    int dev;
    void* p;
    std::shared_ptr<ReleaseMark> mark;  // null: released after a device synchronization
  };
  std::multimap<size_t, Cached> free_;  // block size -> block
  size_t cached_ = 0;
  size_t cap_ = 0;  // set at the first release
  size_t budget_[kDev] = {};
  size_t in_use_[kDev] = {};
};

// RAII owner of device allocations (through the cache above)
constexpr size_t kReserve = (size_t)8 << 30;
struct DevArena {
  struct Block {
    void* p;
    size_t bytes;
    int dev;
  };
  std::vector<Block> ptrs;
  // An arena whose blocks are used on one stream only (set_stream) hands them
  // back with an event recorded on that stream, so its release waits for
  // nothing; otherwise the release synchronizes the device first.
  bool ordered = false;
  hipStream_t stream = nullptr;
  void set_stream(hipStream_t s) {
    ordered = true;
    stream = s;
  }
  ~DevArena() { release(); }
  void release() {
    if (ptrs.empty()) return;
    std::shared_ptr<ReleaseMark> mark;
    if (ordered && stream_marks_ok(stream)) {
      mark = std::make_shared<ReleaseMark>();
      mark->stream = stream;
      if (hipEventCreateWithFlags(&mark->ev, hipEventDisableTiming) != hipSuccess ||
          hipEventRecord(mark->ev, stream) != hipSuccess)
        mark.reset();
    }
    if (!mark) (void)hipDeviceSynchronize();  // no kernel may still use a block handed out again
    for (const Block& b : ptrs) {
      DevicePool::get().give(b.p, b.bytes, b.dev, mark);
      DevicePool::get().uncharge(b.dev, b.bytes);
    }
    ptrs.clear();
  }
  template <typename T>
  int alloc(T** out, size_t count) {
    const size_t bytes = DevicePool::round(std::max<size_t>(count, 1) * sizeof(T));
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (!DevicePool::get().charge(dev, bytes)) {
      set_error("device memory budget of %zu bytes exceeded (%zu in use, %zu more requested)",
                DevicePool::get().budget(dev), DevicePool::get().in_use(dev), bytes);
      return ZOLO_ENOMEM;
    }
    void* p = DevicePool::get().take(bytes, dev);
    if (!p) {
      // keep room for the runtime's own allocations (kernel scratch, queues): when
      // a new block would leave less than kReserve free, return cached blocks first
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess && fr < bytes + kReserve)
        DevicePool::get().trim_for(bytes + kReserve - fr, dev);
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        DevicePool::get().trim();
        e = hipMalloc(&p, bytes);
      }
      if (e != hipSuccess) {
        DevicePool::get().uncharge(dev, bytes);
        set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        return ZOLO_ENOMEM;
      }
    }
    ptrs.push_back({p, bytes, dev});
    *out = (T*)p;
    return ZOLO_OK;
  }
  template <typename T>
  int upload(T** out, const T* host, size_t count) {
    CHK(alloc(out, count));
    if (count) {
      hipError_t e = hipMemcpy(*out, host, count * sizeof(T), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        set_error("hipMemcpy failed: %s", hipGetErrorString(e));
        return ZOLO_EDEVICE;
      }
    }
    return ZOLO_OK;
  }
};

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// splitmix64 + Box-Muller Gaussian start block (used when none is passed in)
struct GemmLaunch {
  int off = 0, cnt = 0, tiles = 0;
  int maxM = 0, maxN = 0;  // bounds over the launch's products (GEMM launches)
  int max_split = 1;       // largest inner-dimension split of its products
  int grid_tiles = 0;      // workgroups per split the launch needs (0: tiles of maxM x maxN)
  double flops = 0.0, bytes = 0.0;  // algorithmic work of the launch
};

// ---- per-kernel-class timing with HIP events on the launching stream ----
namespace prof {
bool on = false;
struct Pend {
  hipEvent_t a, b;
  int cls;
  double flops, bytes;
};
std::vector<Pend> pend;
std::vector<hipEvent_t> pool;
double ms[ZOLO_PROF_COUNT], fl[ZOLO_PROF_COUNT], by[ZOLO_PROF_COUNT];
long long cnt[ZOLO_PROF_COUNT];
hipEvent_t get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}
void resolve() {
  for (Pend& p : pend) {
    float t = 0.0f;
    (void)hipEventSynchronize(p.b);
    if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) ms[p.cls] += t;
    fl[p.cls] += p.flops;
    by[p.cls] += p.bytes;
    cnt[p.cls] += 1;
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pend.clear();
}
void reset() {
  resolve();
  for (int i = 0; i < ZOLO_PROF_COUNT; ++i) ms[i] = fl[i] = by[i] = 0.0, cnt[i] = 0;
}
struct Scope {
  bool act;
  Pend p;
  hipStream_t s;
  Scope(int cls, double flops, double bytes, hipStream_t st) : act(on), s(st) {
    if (!act) return;
    p.a = get_event();
    p.b = get_event();
    p.cls = cls;
    p.flops = flops;
    p.bytes = bytes;
    (void)hipEventRecord(p.a, s);
  }
  ~Scope() {
    if (!act) return;
    (void)hipEventRecord(p.b, s);
    pend.push_back(p);
    if (pend.size() > 20000) resolve();
  }
};
}  // namespace prof

}  // namespace

// ===========================================================================
// handles
// ===========================================================================
struct zolo_ctx {
  int device = 0;
};

struct zolo_pencil {
  zolo_ctx* ctx = nullptr;
  int64_t n = 0, nnz = 0;
  int scalar = 0;
  Symbolic S;
  DevArena mem;
  int64_t* prow = nullptr;
  int32_t* pcol = nullptr;
  double* pa = nullptr;  // real pencils: permuted CSR values
  double* pb = nullptr;
  zd* za = nullptr;      // complex Hermitian pencils: permuted CSR values
  zd* zb = nullptr;
  int32_t* perm = nullptr;   // perm[new] = old
  int32_t* iperm = nullptr;  // iperm[old] = new
  int32_t* struct_rows = nullptr;
  int32_t* pmap = nullptr;
  double normA = 0.0, normB = 0.0;
  double t_symbolic = 0.0;
  // sigma-independent numeric layout
  std::vector<int> lvl_order;       // fronts ordered by level
  std::vector<int64_t> panel_off, inv_off, upd_off;
  std::vector<int64_t> lvl_panel_begin, lvl_panel_end, lvl_inv_begin, lvl_inv_end, lvl_upd_begin, lvl_upd_end;
  int64_t panel_total = 0, inv_total = 0, upd_total = 0;  // upd_total: the level-scoped update pool
  int64_t upd_sum = 0;                                     // all fronts' update blocks together
  int64_t* asm_dst = nullptr;
  int64_t* asm_src = nullptr;
  int64_t* asm_src_t = nullptr;  // complex pencils: the CSR entry transposed to asm_src's
  std::vector<int64_t> lvl_asm_begin, lvl_asm_end;
  ExtDesc* ext = nullptr;
  std::vector<std::vector<GemmLaunch>> lvl_ext;  // per level per slot: off/cnt/max_nb (tiles)
  DiagDesc* diag = nullptr;
  std::vector<int> lvl_diag_off, lvl_diag_cnt;
  std::vector<std::vector<int>> lvl_diag_nJ, lvl_trsm_rows;  // per level per step
  int64_t inv_scratch = 0;   // L11 inverse temporaries of one level (recursive doubling, per side)
  int64_t conv_scratch = 0;  // -L21 X of one level's fronts before stacking (per side)
  // forward-solve right-hand sides, in rows (independent of the block width):
  // per row of a level's stacked front blocks, the right-hand-side row it starts
  // from (-1: a border row) and, in fill_cidx[fill_cbeg[r] .. fill_cbeg[r+1]), the
  // rows of the children's update blocks added to it, in child order
  int32_t* fill_own = nullptr;
  int32_t* fill_cbeg = nullptr;
  int32_t* fill_cidx = nullptr;
  std::vector<int64_t> lvl_fill_off, lvl_fill_rows;
  // per level, for the byte counts of the solves' gathers: contribution rows
  // added by the fill, rows taken from the right-hand side, and sum of k
  std::vector<int64_t> lvl_fill_adds, lvl_fill_src, lvl_k;
  bool cplx() const { return scalar == ZOLO_COMPLEX128; }
};

// One factored pole.  Real pencils: complex-symmetric LDL^T (panel = L,
// inv = L11^-1 blocks).  Complex Hermitian pencils: LU = L D U with the U
// factor stored transposed (upanel = U^T, uinv = (U11^T)^-1 blocks) and
// dconj = conj(D) for the solves with K^-H.
template <typename T>
struct PoleMF {
  T* panel = nullptr;
  T* inv = nullptr;
  T* dvec = nullptr;
  T* upanel = nullptr;
  T* uinv = nullptr;
  T* dconj = nullptr;
};

template <typename T>
struct SolveProg {
  int p = 0;
  DevArena mem;
  T* W = nullptr;  // per level: each front's k x p right-hand side (forward, then backward)
  T* U = nullptr;  // each front's nb x p contribution to its parent (forward)
  T* Y = nullptr;  // forward solution, N x p per solve
  T* X = nullptr;  // solution, N x p per solve
  SolveDesc* sd = nullptr;
  std::vector<int> lvl_sd_off, lvl_sd_cnt, lvl_maxk;
  // forward right-hand sides: per row of a level's W (levels one after the other),
  // the right-hand-side row it starts from (-1: none) and, in cidx[cbeg[r] ..
  // cbeg[r+1]), the rows of U (children's updates) added to it, in child order
  const int32_t* own = nullptr;  // the pencil's tables (zolo_pencil::fill_*)
  const int32_t* cbeg = nullptr;
  const int32_t* cidx = nullptr;
  std::vector<int64_t> lvl_row_off, lvl_rows;
  int64_t wstride = 0, ustride = 0;  // elements between the solves' W and U regions
  int np = 0;                        // poles solved together
  int64_t xstride = 0;                           // elements between poles' X (and Y) blocks
  GemmDesc<T>* gd = nullptr;                     // all poles, per level
  std::vector<GemmLaunch> fw, bw;                // [level]: forward, backward products
};

// Krylov-side buffers.  Blocks hold real values for real pencils and complex
// values for complex Hermitian pencils (ef = 2 doubles per entry); they are
// typed double* and read through the block scalar type where used.
struct Workspace {
  DevArena mem;
  int p = 0, mmax = 0, nshift = 0, ef = 1;
  int64_t n = 0;
  double* Vb = nullptr;   // N x Mp
  double* W = nullptr;    // N x p
  double* T1 = nullptr;   // N x p
  double* Tb = nullptr;   // N x p (B V)
  zd* Xc = nullptr;       // N x p complex (pole solution)
  zd* Rc = nullptr;       // N x p complex (refinement residual)
  zd* Dc = nullptr;       // N x p complex (refinement correction)
  double* H = nullptr;    // ldh x mmax p
  int64_t ldh = 0;
  double* hbuf = nullptr; // (mmax+1)p x p
  double* partial = nullptr;
  int64_t partial_len = 0;
  double* G = nullptr;    // p x p
  double* R1 = nullptr;
  double* R1i = nullptr;
  double* R2 = nullptr;
  double* R2i = nullptr;
  double* R0 = nullptr;
  double* Rk = nullptr;
  int* flag = nullptr;
  double* res = nullptr;  // nshift x p
  double* coef = nullptr;
  double* shift_im = nullptr;
  double* Cm = nullptr;   // mmax p x p
  zd* Ys = nullptr;       // nshift x (mmax p) x p
  HlsState hls{};
  void* gdesc = nullptr;  // room for gdesc_cap + 4 descriptors of either scalar type
  int gdesc_cap = 0;
  double* cn_partial = nullptr;
  double* cn_out = nullptr;
};

struct zolo_factors {
  zolo_pencil* P = nullptr;
  zolo_filter_coeffs co{};
  int precision = 0;
  DevArena mem;
  std::vector<PoleMF<zd>> pd;
  std::vector<PoleMF<zf>> pf;
  std::vector<PoleMF<double>> pr;  // real LDL^T (inertia counts of real pencils at real shifts)
  std::map<int, std::unique_ptr<SolveProg<zd>>> prog_d;
  std::map<int, std::unique_ptr<SolveProg<zf>>> prog_f;
  std::unique_ptr<Workspace> ws;
  double t_factor = 0.0;
  int max_refine = 8;
  double tol_refine = 1e-13;  // zolo_factor: pole solves refined to FP64 accuracy; zolo_solve sets its own
  long long n_refine = 0;
  int refine_sweeps_max = 0;  // most corrections one refinement took
  int refine_missed = 0;      // refinements that stopped above their target
  double refine_worst = 0.0;  // largest relative residual such a refinement left
  long long n_solv = 0;
  int64_t bytes = 0;
};

struct zolo_result {
  int64_t n = 0, count = 0;
  int ef = 1;  // doubles per vector entry: 1 real, 2 complex (interleaved)
  std::vector<double> eig;
  DevArena mem;
  double* vec = nullptr;  // N x count row-major, original ordering
  zolo_stats st{};
};

// ===========================================================================
// small helpers
// ===========================================================================
namespace {

template <typename T>
int upload_gemm(DevArena& mem, const std::vector<GemmDesc<T>>& h, GemmDesc<T>** d) {
  return mem.upload(d, h.data(), h.size());
}

template <typename T>
void run_gemm(const GemmDesc<T>* base, const GemmLaunch& L, hipStream_t s, int tag) {
  if (L.cnt <= 0 || L.maxM <= 0 || L.maxN <= 0) return;
  prof::Scope ps(tag == 0 ? ZOLO_PROF_GEMM_FACTOR : tag == 1 ? ZOLO_PROF_GEMM_SOLVE : ZOLO_PROF_GEMM_KRYLOV, L.flops,
                 L.bytes, s);
  gemm_batched<T>(base + L.off, L.cnt, L.maxM, L.maxN, s, tag, L.max_split, L.grid_tiles);
}

// Inner-dimension splits of the products of GEMM launches (GemmDesc::splitk).
// A launch with fewer tiles than kSplitBelow workgroups splits each product
// whose inner loop has at least 2 * kMinSplitChunks chunks, aiming at about
// kSplitTarget workgroups.  Launches run one after another on a stream, so
// they share one partial buffer and one tile-counter array, sized for the
// largest launch; patch_split fills in the pointers once they exist.
constexpr int kSplitBelow = 256, kSplitTarget = 512, kMinSplitChunks = 8, kMaxSplit = 16;
struct SplitPlan {
  std::vector<std::pair<int, std::pair<int64_t, int64_t>>> at;  // descriptor -> (part offset, counter offset)
  int64_t part = 0, cnt = 0;                                    // sizes (real scalars, counters)
};
template <typename T>
void plan_split(std::vector<GemmDesc<T>>& gd, GemmLaunch& g, SplitPlan* sp, int tag) {
  if (g.cnt <= 0 || g.maxM <= 0 || g.maxN <= 0) return;
  const int tk = gemm_tile_k(g.maxM, g.maxN, tag);
  // longest products first, so that the launch's last workgroups are short ones
  // (the products of a launch are independent; their order is free)
  std::stable_sort(gd.begin() + g.off, gd.begin() + g.off + g.cnt, [&](const GemmDesc<T>& x, const GemmDesc<T>& y) {
    return (double)gemm_desc_tiles(x.M, x.N, x.flags, x.tri_off, g.maxM, g.maxN, tag) * x.K >
           (double)gemm_desc_tiles(y.M, y.N, y.flags, y.tri_off, g.maxM, g.maxN, tag) * y.K;
  });
  int64_t total = 0;
  g.grid_tiles = 0;
  for (int i = g.off; i < g.off + g.cnt; ++i) {
    const int t = gemm_desc_tiles(gd[i].M, gd[i].N, gd[i].flags, gd[i].tri_off, g.maxM, g.maxN, tag);
    g.grid_tiles = std::max(g.grid_tiles, t);
    total += t;
  }
  if (total >= kSplitBelow) return;
  const int goal = (int)std::min<int64_t>(kMaxSplit, (kSplitTarget + total - 1) / std::max<int64_t>(total, 1));
  const int64_t pe = gemm_part_elems(g.maxM, g.maxN, tag, ST<T>::cplx);
  int64_t po = 0, co = 0;
  for (int i = g.off; i < g.off + g.cnt; ++i) {
    GemmDesc<T>& d = gd[i];
    const int chunks = (d.K + tk - 1) / tk;
    const int S = std::min(goal, chunks / kMinSplitChunks);
    if (S < 2) continue;
    // tiles of this product in the launch's tile shape (the counter and
    // partial-sum slots its splits index)
    const int64_t t = gemm_desc_tiles(d.M, d.N, 0, 0, g.maxM, g.maxN, tag);
    d.splitk = S;
    sp->at.push_back({i, {po, co}});
    po += (int64_t)S * t * pe;
    co += t;
    g.max_split = std::max(g.max_split, S);
  }
  sp->part = std::max(sp->part, po);
  sp->cnt = std::max(sp->cnt, co);
}
template <typename T>
void patch_split(std::vector<GemmDesc<T>>& gd, const SplitPlan& sp, typename ST<T>::real* part, int* cnt) {
  for (const auto& a : sp.at) {
    gd[a.first].part = part + a.second.first;
    gd[a.first].cnt = cnt + a.second.second;
  }
}

// out (m x n, col-major ld ldo) [+]= X^H Y with X: N x m row-major (ld ldx), Y: N x n row-major (ld ldy)
template <typename VT>
int gemm_tn(Workspace& ws, const VT* X, int64_t ldx, const VT* Y, int64_t ldy, int64_t N, int m, int n, VT* out,
            int64_t ldo, bool add, hipStream_t s) {
  // row chunks: about 2048 workgroups (eight per CU) of at least 256 rows each,
  // so that the long inner loops of these tall products keep the chip busy
  int tiles = gemm_tiles(m, n, 2);
  int64_t S = std::max<int64_t>(1, std::min<int64_t>((2048 + tiles - 1) / tiles, N / 256));
  // partial_len counts entries of the workspace's own block type (ef doubles)
  const int64_t cap = ws.partial_len * ws.ef / (ST<VT>::cplx ? 2 : 1);
  while (S * (int64_t)m * n > cap && S > 1) S /= 2;
  if (S * (int64_t)m * n > cap) {
    set_error("gemm_tn: partial buffer too small");
    return ZOLO_ENOMEM;
  }
  if (S > ws.gdesc_cap) S = ws.gdesc_cap;
  const int64_t chunk = (N + S - 1) / S;
  const int cnt = chunk > 0 ? (int)((N + chunk - 1) / chunk) : 0;  // chunks that hold rows
  VT* partial = (VT*)ws.partial;
  // chunk q: rows [q chunk, min(N, (q + 1) chunk)) of X and Y into partial q
  GemmDesc<VT> d{};
  d.A = X;
  d.lda = ldx;
  d.B = Y;
  d.ldb = ldy;
  d.C = partial;
  d.ldc = m;
  d.M = m;
  d.N = n;
  d.K = (int)chunk;
  d.flags = GF_TRANSB | (ST<VT>::cplx ? GF_CONJA : 0);
  d.alpha = ST<VT>::one();
  d.beta = ST<VT>::zero();
  GemmDesc<VT>* dg = (GemmDesc<VT>*)ws.gdesc;
  gemm_desc_series<VT>(d, cnt, chunk * ldx, chunk * ldy, (int64_t)m * n, chunk, N, dg, s);
  {
    double fl = 0.0, by = 0.0;
    for (int q = 0; q < cnt; ++q) {
      d.K = (int)std::min<int64_t>(chunk, N - q * chunk);
      gemm_work(d, &fl, &by);
    }
    prof::Scope ps(ZOLO_PROF_GEMM_KRYLOV, fl, by, s);
    gemm_batched<VT>(dg, cnt, m, n, s, 2);
  }
  {
    prof::Scope ps(ZOLO_PROF_ELEMWISE, 0.0, (double)sizeof(VT) * m * n * (cnt + 1), s);
    reduce_partials<VT>(out, ldo, partial, cnt, m, n, add, s);
  }
  return ZOLO_OK;
}

// C^T (p x N col-major view of row-major C, ld ldc) = beta C^T + alpha opA(Msmall) Bv^T
// Used for W -= V h and V_new = W R^-1 style updates: C_rm = beta C_rm + alpha Bv_rm opA^T
template <typename VT>
int gemm_nt_big(Workspace& ws, VT* C, int64_t ldc, const VT* Cin, int64_t ldcin, double beta, double alpha,
                const VT* Msmall, int64_t ldm, bool transM, const VT* Bv, int64_t ldb, int64_t N, int p, int K,
                hipStream_t s) {
  GemmDesc<VT> d{};
  d.C = C;
  d.ldc = ldc;
  d.Cin = Cin;
  d.ldcin = ldcin;
  d.beta = cvt<VT, double>(beta);
  d.alpha = cvt<VT, double>(alpha);
  d.K = K;
  // A block of 65 to 96 columns is computed as C_rm = Bv opM^T (row-major C,
  // N rows): one 96-column tile per 64 rows of Bv, so Bv is read once and no
  // tile is padded, where p x N in 64 x 64 tiles pads p to 128 and reads each
  // slab of Bv twice.
  const bool rows = p > 64 && p <= 96;
  if (rows) {
    d.A = Bv;
    d.lda = ldb;
    d.B = Msmall;
    d.ldb = ldm;
    d.flags = GF_TRANSA | GF_TRANSC | (transM ? 0 : GF_TRANSB);
    d.M = (int)N;
    d.N = p;
  } else {
    d.A = Msmall;
    d.lda = ldm;
    d.flags = transM ? GF_TRANSA : 0;
    d.B = Bv;
    d.ldb = ldb;
    d.M = p;
    d.N = (int)N;
  }
  GemmDesc<VT>* dg = (GemmDesc<VT>*)ws.gdesc + ws.gdesc_cap;
  gemm_desc_series<VT>(d, 1, 0, 0, 0, K, K, dg, s);
  {
    double fl = 0.0, by = 0.0;
    gemm_work(d, &fl, &by);
    prof::Scope ps(ZOLO_PROF_GEMM_KRYLOV, fl, by, s);
    gemm_batched<VT>(dg, 1, d.M, d.N, s, 2);
  }
  return ZOLO_OK;
}

}  // namespace

// ===========================================================================
// pencil
// ===========================================================================
extern "C" const char* zolo_last_error(void) { return zolo::g_err.c_str(); }
extern "C" const char* zolo_version(void) { return "zolo-mi355x 0.1"; }

extern "C" zolo_status zolo_opts_default(zolo_opts* o) {
  if (!o) {
    set_error("null opts");
    return ZOLO_EINVAL;
  }
  std::memset(o, 0, sizeof(*o));
  o->a_minus = o->a_plus = o->b_minus = o->b_plus = NAN;
  o->r1 = 2;
  o->r2 = 0;
  o->filter_eps = 1e-10;
  o->n_ss = 0;
  o->max_subspace_iter = 6;
  o->max_gmres_iter = 60;
  o->tol_resid = 1e-8;
  o->tol_gmres = 1e-10;
  o->precision = ZOLO_PREC_FP64;
  o->seed = 2;
  o->max_refine = 8;
  o->tol_refine = 1e-8;
  o->block_cols = 0;
  o->filter_kind = ZOLO_FILTER_HYBRID;
  o->gmres_restart = 30;
  return ZOLO_OK;
}

// ---------------------------------------------------------------------------
// Static device scratch for zolo_residuals_noalloc: the partial sums of the
// fused residual kernel (kResidGroups workgroups x 2 sums x at most
// kResidMaxCols columns, 4 MiB).  Each GPU holds its own copy for the life of
// the process.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in): the device address of each GPU's copy is looked
// up once, with that device current, and kept in g_scratch_dev.  The array has
// external linkage: with internal linkage the compiler keeps it a local symbol
// of the device code object, which the loader cannot resolve by name, and the
// runtime's symbol lookup then fails.
__device__ __align__(256) double zolo_noalloc_scratch[(size_t)kResidGroups * 2 * kResidMaxCols];
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// device address of `scratch` on device dev (which must be current)
zolo_status scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d devices the static scratch table holds", dev, kMaxDevices);
    return ZOLO_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev]) return ZOLO_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(zolo_noalloc_scratch));
  if (e != hipSuccess || !ptr) {
    set_error("hipGetSymbolAddress of the static scratch failed on device %d: %s", dev, hipGetErrorString(e));
    return ZOLO_EDEVICE;
  }
  g_scratch_dev[dev] = (double*)ptr;
  return ZOLO_OK;
}
}  // namespace

extern "C" zolo_status zolo_ctx_create(int dev, zolo_ctx** out) {
  if (!out) {
    set_error("null output");
    return ZOLO_EINVAL;
  }
  int nd = 0;
  HIPC(hipGetDeviceCount(&nd));
  if (dev < 0 || dev >= nd) {
    set_error("device %d out of range (%d devices)", dev, nd);
    return ZOLO_EINVAL;
  }
  HIPC(hipSetDevice(dev));
  CHK(scratch_setup(dev));
  auto* c = new zolo_ctx();
  c->device = dev;
  *out = c;
  return ZOLO_OK;
}

extern "C" zolo_status zolo_ctx_set_hbm_budget(zolo_ctx* c, size_t bytes) {
  if (!c) {
    set_error("zolo_ctx_set_hbm_budget: null context");
    return ZOLO_EINVAL;
  }
  DevicePool::get().set_budget(c->device, bytes);
  return ZOLO_OK;
}

extern "C" zolo_status zolo_ctx_hbm_in_use(const zolo_ctx* c, size_t* bytes) {
  if (!c || !bytes) {
    set_error("zolo_ctx_hbm_in_use: null argument");
    return ZOLO_EINVAL;
  }
  *bytes = DevicePool::get().in_use(c->device);
  return ZOLO_OK;
}

extern "C" void zolo_ctx_destroy(zolo_ctx* c) {
  delete c;
  DevicePool::get().trim();  // return cached device memory
}

static // Forward-solve fill tables (zolo_pencil::fill_*), by counting: the rows of
// the update blocks are numbered over all fronts in level order, as the solve
// program lays its update buffer out.
zolo_status build_fill(zolo_pencil* P) {
  const Symbolic& S = P->S;
  const int nl = (int)S.levels.size();
  std::vector<int64_t> urow(S.fronts.size(), 0);
  int64_t ur = 0;
  for (int L = 0; L < nl; ++L)
    for (int f : S.levels[L]) {
      urow[f] = ur;
      ur += S.fronts[f].nb;
    }
  if (ur >= INT32_MAX) {
    set_error("pencil too large for the solve tables");
    return ZOLO_EINVAL;
  }
  std::vector<int32_t> own, cbeg, cidx, cnt;
  P->lvl_fill_off.assign(nl, 0);
  P->lvl_fill_rows.assign(nl, 0);
  P->lvl_fill_adds.assign(nl, 0);
  P->lvl_fill_src.assign(nl, 0);
  P->lvl_k.assign(nl, 0);
  for (int L = 0; L < nl; ++L) {
    P->lvl_fill_off[L] = (int64_t)own.size();
    const int64_t adds0 = (int64_t)cidx.size();
    for (int f : S.levels[L]) {
      const Front& Fr = S.fronts[f];
      const int k = Fr.ns + Fr.nb;
      cnt.assign(k + 1, 0);
      for (int slot = 0; slot < Fr.child_count; ++slot) {
        const Front& C = S.fronts[S.children[Fr.child_begin + slot]];
        for (int i = 0; i < C.nb; ++i) ++cnt[S.parent_map[C.struct_off + i] + 1];
      }
      const int64_t base = (int64_t)cidx.size();
      for (int r = 0; r < k; ++r) {
        cnt[r + 1] += cnt[r];
        own.push_back(r < Fr.ns ? Fr.first + r : -1);
        cbeg.push_back((int32_t)(base + cnt[r]));
      }
      cidx.resize(base + cnt[k]);
      for (int slot = 0; slot < Fr.child_count; ++slot) {  // child order within each row
        const int ch = S.children[Fr.child_begin + slot];
        const Front& C = S.fronts[ch];
        for (int i = 0; i < C.nb; ++i) cidx[base + cnt[S.parent_map[C.struct_off + i]]++] = (int32_t)(urow[ch] + i);
      }
    }
    P->lvl_fill_rows[L] = (int64_t)own.size() - P->lvl_fill_off[L];
    P->lvl_fill_adds[L] = (int64_t)cidx.size() - adds0;
    for (int f : S.levels[L]) {
      P->lvl_fill_src[L] += S.fronts[f].ns;
      P->lvl_k[L] += S.fronts[f].ns + S.fronts[f].nb;
    }
  }
  cbeg.push_back((int32_t)cidx.size());
  if (own.empty()) own.push_back(-1);
  if (cidx.empty()) cidx.push_back(0);
  CHK(P->mem.upload(&P->fill_own, own.data(), own.size()));
  CHK(P->mem.upload(&P->fill_cbeg, cbeg.data(), cbeg.size()));
  CHK(P->mem.upload(&P->fill_cidx, cidx.data(), cidx.size()));
  return ZOLO_OK;
}

zolo_status build_layout(zolo_pencil* P) {
  const Symbolic& S = P->S;
  const int nf = (int)S.fronts.size();
  const int nl = (int)S.levels.size();
  P->panel_off.assign(nf, 0);
  P->inv_off.assign(nf, 0);
  P->upd_off.assign(nf, 0);
  P->lvl_order.clear();
  P->lvl_panel_begin.assign(nl, 0);
  P->lvl_panel_end.assign(nl, 0);
  P->lvl_inv_begin.assign(nl, 0);
  P->lvl_inv_end.assign(nl, 0);
  int64_t po = 0, io = 0, uo = 0;
  P->inv_scratch = 0;
  P->conv_scratch = 0;
  for (int L = 0; L < nl; ++L) {
    P->lvl_panel_begin[L] = po;
    P->lvl_inv_begin[L] = io;
    int64_t scr = 0;
    for (int f : S.levels[L]) {
      const Front& F = S.fronts[f];
      int64_t k = (int64_t)F.ns + F.nb;
      P->panel_off[f] = po;
      po += k * F.ns;
      P->inv_off[f] = io;
      io += (int64_t)F.ns * F.ns;
      P->upd_off[f] = uo;  // within the level's range for now (placed below)
      uo += (int64_t)F.nb * F.nb;
      P->lvl_order.push_back(f);
    }
    // recursive doubling of the inverse: at block size s every block holds an h2 x h
    // temporary (h = s / 2); the level needs the largest sum over its fronts at one s
    for (int64_t sz = 2 * FB;; sz *= 2) {
      const int64_t h = sz / 2;
      int64_t tot = 0;
      bool any = false;
      for (int f : S.levels[L]) {
        const int64_t ns = S.fronts[f].ns;
        for (int64_t r0 = 0; r0 + h < ns; r0 += sz) {
          tot += std::min(h, ns - r0 - h) * h;
          any = true;
        }
      }
      if (!any) break;
      scr = std::max(scr, tot);
    }
    int64_t cv = 0;
    for (int f : S.levels[L]) cv += (int64_t)S.fronts[f].nb * S.fronts[f].ns;
    P->inv_scratch = std::max(P->inv_scratch, scr);
    P->conv_scratch = std::max(P->conv_scratch, cv);
    P->lvl_panel_end[L] = po;
    P->lvl_inv_end[L] = io;
  }
  P->panel_total = po;
  P->inv_total = io;
  P->upd_sum = uo;
  // Update-block pool.  The update block of a front of level L is written at
  // level L (the extend-add scatters into it, then the Schur update adds to it)
  // and read at its parent's level, after which it is dead.  Each level gets one
  // contiguous range (cleared when the level starts), placed first-fit among
  // the ranges still live, and released after the last level that reads any of
  // its blocks, so the pool holds a few levels' blocks instead of all of them.
  {
    struct Rng {
      int64_t off, len;
      int last;
    };
    std::vector<Rng> live;
    int64_t pool = 0;
    P->lvl_upd_begin.assign(nl, 0);
    P->lvl_upd_end.assign(nl, 0);
    for (int L = 0; L < nl; ++L) {
      int64_t len = 0;
      int last = L;
      for (int f : S.levels[L]) {
        len += (int64_t)S.fronts[f].nb * S.fronts[f].nb;
        if (S.fronts[f].parent >= 0) last = std::max(last, (int)S.fronts[S.fronts[f].parent].level);
      }
      live.erase(std::remove_if(live.begin(), live.end(), [L](const Rng& r) { return r.last < L; }), live.end());
      std::sort(live.begin(), live.end(), [](const Rng& x, const Rng& y) { return x.off < y.off; });
      int64_t base = 0;
      for (const Rng& r : live) {
        if (r.off - base >= len) break;
        base = std::max(base, r.off + r.len);
      }
      const int64_t lvl0 = P->upd_off[S.levels[L].empty() ? 0 : S.levels[L][0]];
      for (int f : S.levels[L]) P->upd_off[f] = P->upd_off[f] - lvl0 + base;
      P->lvl_upd_begin[L] = base;
      P->lvl_upd_end[L] = base + len;
      if (len > 0) live.push_back({base, len, last});
      pool = std::max(pool, base + len);
    }
    P->upd_total = pool;
  }
  // assembly lists in level order
  std::vector<int64_t> dst, src;
  P->lvl_asm_begin.assign(nl, 0);
  P->lvl_asm_end.assign(nl, 0);
  for (int L = 0; L < nl; ++L) {
    P->lvl_asm_begin[L] = (int64_t)dst.size();
    for (int f : S.levels[L]) {
      const Front& F = S.fronts[f];
      for (int64_t e = F.asm_begin; e < F.asm_end; ++e) {
        dst.push_back(P->panel_off[f] + S.asm_pos[e]);
        src.push_back(S.asm_entry[e]);
      }
    }
    P->lvl_asm_end[L] = (int64_t)dst.size();
  }
  CHK(P->mem.upload(&P->asm_dst, dst.data(), dst.size()));
  CHK(P->mem.upload(&P->asm_src, src.data(), src.size()));
  if (P->cplx()) {
    // LU fronts need both triangles: the CSR entry transposed to each
    // assembly entry (the permuted CSR has sorted columns)
    std::vector<int64_t> srct(src.size());
    for (size_t q = 0; q < src.size(); ++q) {
      const int64_t e = src[q];
      const int32_t j = S.pcol[e];
      const int64_t i = std::upper_bound(S.prow.begin(), S.prow.end(), e) - S.prow.begin() - 1;
      const int32_t* lo = S.pcol.data() + S.prow[j];
      const int32_t* hi = S.pcol.data() + S.prow[j + 1];
      srct[q] = std::lower_bound(lo, hi, (int32_t)i) - S.pcol.data();
    }
    CHK(P->mem.upload(&P->asm_src_t, srct.data(), srct.size()));
  }
  // extend-add descriptors: per parent level, per child slot
  std::vector<ExtDesc> ext;
  P->lvl_ext.assign(nl, {});
  for (int L = 0; L < nl; ++L) {
    int maxc = 0;
    for (int f : S.levels[L]) maxc = std::max(maxc, S.fronts[f].child_count);
    for (int slot = 0; slot < maxc; ++slot) {
      GemmLaunch g;
      g.off = (int)ext.size();
      int maxnb = 0;
      for (int f : S.levels[L]) {
        const Front& F = S.fronts[f];
        if (slot >= F.child_count) continue;
        int c = S.children[F.child_begin + slot];
        const Front& C = S.fronts[c];
        if (C.nb == 0) continue;
        ExtDesc d{};
        d.child_upd = P->upd_off[c];
        d.pmap = C.struct_off;
        d.par_panel = P->panel_off[f];
        d.par_upd = P->upd_off[f];
        d.nb_c = C.nb;
        d.k_p = F.ns + F.nb;
        d.ns_p = F.ns;
        ext.push_back(d);
        maxnb = std::max(maxnb, C.nb);
      }
      g.cnt = (int)ext.size() - g.off;
      g.tiles = maxnb;
      P->lvl_ext[L].push_back(g);
    }
  }
  CHK(P->mem.upload(&P->ext, ext.data(), ext.size()));
  // diagonal-block descriptors, per level sorted by ns descending
  std::vector<DiagDesc> dg;
  P->lvl_diag_off.assign(nl, 0);
  P->lvl_diag_cnt.assign(nl, 0);
  P->lvl_diag_nJ.assign(nl, {});
  P->lvl_trsm_rows.assign(nl, {});
  for (int L = 0; L < nl; ++L) {
    std::vector<int> fs = S.levels[L];
    std::stable_sort(fs.begin(), fs.end(), [&](int a, int b) { return S.fronts[a].ns > S.fronts[b].ns; });
    P->lvl_diag_off[L] = (int)dg.size();
    int maxns = 0;
    for (int f : fs) {
      const Front& F = S.fronts[f];
      DiagDesc d{};
      d.panel = P->panel_off[f];
      d.inv = P->inv_off[f];
      d.k = F.ns + F.nb;
      d.ns = F.ns;
      d.first = F.first;
      dg.push_back(d);
      maxns = std::max(maxns, F.ns);
    }
    P->lvl_diag_cnt[L] = (int)fs.size();
    for (int J = 0; J < maxns; J += FB) {
      int cnt = 0, rows = 0;
      for (int f : fs) {
        const Front& F = S.fronts[f];
        if (F.ns <= J) break;
        ++cnt;
        int jb = std::min(FB, F.ns - J);
        rows = std::max(rows, F.ns + F.nb - J - jb);
      }
      P->lvl_diag_nJ[L].push_back(cnt);
      P->lvl_trsm_rows[L].push_back(rows);
    }
  }
  CHK(P->mem.upload(&P->diag, dg.data(), dg.size()));
  return ZOLO_OK;
}

extern "C" zolo_status zolo_pencil_create(zolo_ctx* ctx, int64_t n, const int64_t* rowptr, const int32_t* colind,
                                          const void* a_vals, const void* b_vals, int scalar, const int32_t* grid,
                                          int leaf_size, zolo_pencil** out) {
  if (!ctx || !rowptr || !colind || !a_vals || !b_vals || !out || n <= 0) {
    set_error("zolo_pencil_create: null argument or n <= 0");
    return ZOLO_EINVAL;
  }
  if (scalar != ZOLO_REAL64 && scalar != ZOLO_COMPLEX128) {
    set_error("zolo_pencil_create: unknown scalar type %d", scalar);
    return ZOLO_EINVAL;
  }
  if (n > INT32_MAX) {
    set_error("n too large");
    return ZOLO_EINVAL;
  }
  const int64_t nnz = rowptr[n];
  if (rowptr[0] != 0 || nnz < n) {
    set_error("CSR: rowptr[0] must be 0 and the diagonal stored");
    return ZOLO_EINVAL;
  }
  const bool cx = scalar == ZOLO_COMPLEX128;
  // value e of A or B as (re, im)
  const double* av = (const double*)a_vals;
  const double* bv = (const double*)b_vals;
  auto aval = [&](int64_t e) { return cx ? zd{av[2 * e], av[2 * e + 1]} : zd{av[e], 0.0}; };
  auto bval = [&](int64_t e) { return cx ? zd{bv[2 * e], bv[2 * e + 1]} : zd{bv[e], 0.0}; };
  // validate: sorted columns in range, diagonal present, symmetric pattern, Hermitian values
  for (int64_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] < rowptr[i]) {
      set_error("CSR: rowptr not monotone at row %lld", (long long)i);
      return ZOLO_EINVAL;
    }
    bool diag = false;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      int32_t j = colind[e];
      if (j < 0 || j >= n || (e > rowptr[i] && colind[e - 1] >= j)) {
        set_error("CSR: column indices must be in range and strictly increasing (row %lld)", (long long)i);
        return ZOLO_EINVAL;
      }
      if (j == i) diag = true;
    }
    if (!diag) {
      set_error("CSR: diagonal entry missing in row %lld", (long long)i);
      return ZOLO_EINVAL;
    }
  }
  double na = 0.0, nb = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double ra = 0.0, rb = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      int32_t j = colind[e];
      const zd ae = aval(e), be = bval(e);
      ra += std::sqrt(abs2(ae));
      rb += std::sqrt(abs2(be));
      const int32_t* lo = colind + rowptr[j];
      const int32_t* hi = colind + rowptr[j + 1];
      const int32_t* it = std::lower_bound(lo, hi, (int32_t)i);
      if (it == hi || *it != i) {
        set_error("CSR: pattern not symmetric at (%lld, %d)", (long long)i, (int)j);
        return ZOLO_ENOTHERM;
      }
      const int64_t et = it - colind;
      const zd at = aval(et), bt = bval(et);
      const double sa = std::max(1.0, std::sqrt(abs2(ae))), sb = std::max(1.0, std::sqrt(abs2(be)));
      if (std::fabs(at.re - ae.re) > 1e-14 * sa || std::fabs(at.im + ae.im) > 1e-14 * sa ||
          std::fabs(bt.re - be.re) > 1e-14 * sb || std::fabs(bt.im + be.im) > 1e-14 * sb) {
        set_error("A or B not Hermitian at (%lld, %d)", (long long)i, (int)j);
        return ZOLO_ENOTHERM;
      }
      if (j == i && !(be.re > 0.0)) {  // a Hermitian positive definite B has a positive diagonal
        set_error("B is not positive definite: B(%lld, %lld) = %g", (long long)i, (long long)i, be.re);
        return ZOLO_EINVAL;
      }
    }
    na = std::max(na, ra);
    nb = std::max(nb, rb);
  }
  HIPC(hipSetDevice(ctx->device));
  std::unique_ptr<zolo_pencil> P(new zolo_pencil());
  P->ctx = ctx;
  P->n = n;
  P->nnz = nnz;
  P->scalar = scalar;
  P->normA = na;
  P->normB = nb;
  double t0 = now_s();
  CHK(symbolic_analyze(n, rowptr, colind, grid, leaf_size, &P->S));
  P->t_symbolic = now_s() - t0;
  const Symbolic& S = P->S;
  CHK(P->mem.upload(&P->prow, S.prow.data(), S.prow.size()));
  CHK(P->mem.upload(&P->pcol, S.pcol.data(), S.pcol.size()));
  if (cx) {
    std::vector<zd> pa(nnz), pb(nnz);
    for (int64_t e = 0; e < nnz; ++e) {
      pa[e] = aval(S.psrc[e]);
      pb[e] = bval(S.psrc[e]);
    }
    CHK(P->mem.upload(&P->za, pa.data(), pa.size()));
    CHK(P->mem.upload(&P->zb, pb.data(), pb.size()));
  } else {
    std::vector<double> pa(nnz), pb(nnz);
    for (int64_t e = 0; e < nnz; ++e) {
      pa[e] = av[S.psrc[e]];
      pb[e] = bv[S.psrc[e]];
    }
    CHK(P->mem.upload(&P->pa, pa.data(), pa.size()));
    CHK(P->mem.upload(&P->pb, pb.data(), pb.size()));
  }
  CHK(P->mem.upload(&P->perm, S.perm.data(), S.perm.size()));
  CHK(P->mem.upload(&P->iperm, S.iperm.data(), S.iperm.size()));
  CHK(P->mem.upload(&P->struct_rows, S.struct_rows.data(), S.struct_rows.size()));
  CHK(P->mem.upload(&P->pmap, S.parent_map.data(), S.parent_map.size()));
  CHK(build_layout(P.get()));
  CHK(build_fill(P.get()));
  *out = P.release();
  return ZOLO_OK;
}

extern "C" void zolo_pencil_free(zolo_pencil* p) { delete p; }

extern "C" zolo_status zolo_pencil_info(const zolo_pencil* p, int64_t* n_fronts, int64_t* n_levels, int64_t* nnz_l,
                                        double* flops, int64_t* max_front) {
  if (!p) {
    set_error("null pencil");
    return ZOLO_EINVAL;
  }
  if (n_fronts) *n_fronts = (int64_t)p->S.fronts.size();
  if (n_levels) *n_levels = (int64_t)p->S.levels.size();
  if (nnz_l) *nnz_l = p->S.panel_entries + p->S.inv_entries;
  if (flops) *flops = p->S.flops;
  if (max_front) *max_front = p->S.max_front;
  return ZOLO_OK;
}

extern "C" zolo_status zolo_symbolic(int64_t n, const int64_t* rowptr, const int32_t* colind, const int32_t* grid,
                                     int leaf_size, int32_t* perm, double* info) {
  if (n <= 0 || !rowptr || !colind || n > INT32_MAX) {
    set_error("zolo_symbolic: invalid argument");
    return ZOLO_EINVAL;
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
      if (colind[e] < 0 || colind[e] >= n) {
        set_error("zolo_symbolic: column index out of range in row %lld", (long long)i);
        return ZOLO_EINVAL;
      }
  Symbolic S;
  CHK(symbolic_analyze(n, rowptr, colind, grid, leaf_size, &S));
  if (perm) std::memcpy(perm, S.perm.data(), sizeof(int32_t) * n);
  if (info) {
    info[0] = (double)S.fronts.size();
    info[1] = (double)S.levels.size();
    info[2] = (double)S.panel_entries;
    info[3] = (double)S.inv_entries;
    info[4] = (double)S.update_entries;
    info[5] = (double)S.max_front;
    info[6] = (double)S.struct_total;
    info[7] = S.flops;
  }
  return ZOLO_OK;
}

extern "C" zolo_status zolo_pencil_memory(const zolo_pencil* p, int64_t* out) {
  if (!p || !out) {
    set_error("zolo_pencil_memory: null argument");
    return ZOLO_EINVAL;
  }
  out[0] = p->panel_total;
  out[1] = p->inv_total;
  out[2] = p->upd_total;
  out[3] = p->upd_sum;
  out[4] = p->inv_scratch;
  out[5] = p->conv_scratch;
  return ZOLO_OK;
}

extern "C" zolo_status zolo_pencil_flops(const zolo_pencil* p, double* out) {
  if (!p || !out) {
    set_error("zolo_pencil_flops: null argument");
    return ZOLO_EINVAL;
  }
  const double lu = p->cplx() ? 2.0 : 1.0;
  int64_t nnzl = 0;
  for (const Front& F : p->S.fronts) nnzl += ((int64_t)F.ns + F.nb) * F.ns;
  out[0] = lu * p->S.elim_flops;
  out[1] = lu * p->S.flops;
  out[2] = lu * 16.0 * (double)nnzl;
  return ZOLO_OK;
}

extern "C" zolo_status zolo_pencil_perm(const zolo_pencil* p, int32_t* perm) {
  if (!p || !perm) {
    set_error("null argument");
    return ZOLO_EINVAL;
  }
  std::memcpy(perm, p->S.perm.data(), sizeof(int32_t) * p->n);
  return ZOLO_OK;
}

extern "C" zolo_status zolo_filter_plan(double am, double ap, double bm, double bp, int r1, int r2, double eps,
                                        zolo_filter_coeffs* out) {
  if (!out) {
    set_error("null output");
    return ZOLO_EINVAL;
  }
  char err[256] = {0};
  int rc = plan_filter(am, ap, bm, bp, r1, r2, eps > 0 ? eps : 1e-10, out, err, sizeof(err));
  if (rc != ZOLO_OK) set_error("%s", err);
  return (zolo_status)rc;
}

extern "C" zolo_status zolo_filter_plan_kind(int kind, double a, double b, double am, double ap, double bm,
                                             double bp, int r, double eps, zolo_filter_coeffs* out) {
  if (!out) {
    set_error("null output");
    return ZOLO_EINVAL;
  }
  char err[256] = {0};
  int rc;
  if (kind == ZOLO_FILTER_HYBRID || kind == ZOLO_FILTER_ZOLO) {
    rc = plan_filter(am, ap, bm, bp, r, kind == ZOLO_FILTER_ZOLO ? 1 : 0, eps > 0 ? eps : 1e-10, out, err, sizeof(err));
    if (rc == ZOLO_OK) out->kind = kind;
  } else if (kind == ZOLO_FILTER_TRAPEZOID || kind == ZOLO_FILTER_GAUSS) {
    rc = plan_contour(kind, a, b, r, out, err, sizeof(err));
  } else {
    snprintf(err, sizeof(err), "unknown filter kind %d", kind);
    rc = ZOLO_EINVAL;
  }
  if (rc != ZOLO_OK) set_error("%s", err);
  return (zolo_status)rc;
}

// ===========================================================================
// numeric factorization
// ===========================================================================
namespace {

// Numeric factorization of one pole in two phases: factor_plan allocates the
// factor and its temporaries and uploads the program's GEMM descriptors
// (synchronous host work); factor_step only enqueues kernels on a stream, a
// few launches at a time, so several poles run concurrently on their own streams.
struct FactorLevelG {
  std::vector<GemmLaunch> trsm;       // per step J: panel rows below the diagonal block
  std::vector<GemmLaunch> trail;      // per step J: columns up to the end of its outer block
  std::vector<GemmLaunch> trail_out;  // per step J: at an outer block's end, the columns after it
  GemmLaunch schur;
  std::vector<GemmLaunch> inv1, inv2;  // per block row I >= 1
  GemmLaunch conv;                     // -L21 L11^-1 of every front (solve panel, lower part)
  int stk_off = 0, stk_cnt = 0;        // stacking of the solve panels
  int64_t stk_max = 0;                 // largest ns (panel columns) of the level
};
// one pole's temporaries
template <typename T>
struct FactorWork {
  DevArena tmp;
  T* upd = nullptr;
  T* scratch = nullptr;
  T* ctmp = nullptr;  // -L21 L11^-1 of one level's fronts before stacking
  int* flag = nullptr;
};
// The factorization program of all poles: every launch runs one step of every
// pole (the GEMM launches hold all poles' products, the front kernels take the
// pole as a grid dimension), on one stream.
template <typename T>
struct FactorProg {
  DevArena mem;
  GemmDesc<T>* dgd = nullptr;
  StackDesc<T>* dstk = nullptr;
  PoleBase<T>* dpb = nullptr;
  std::vector<FactorLevelG> lg;
  int np = 0;
  bool pivots_only = false;  // inertia counts: D alone, no L11^-1 blocks or solve panels
};

template <typename T>
zolo_status factor_plan(zolo_factors* F, zolo_pencil* P, const zolo_filter_coeffs* co_, std::vector<PoleMF<T>>& poles,
                        std::vector<std::unique_ptr<FactorWork<T>>>& fws, FactorProg<T>* prog) {
  const Symbolic& S = P->S;
  const int nl = (int)S.levels.size();
  const bool lu = P->cplx();
  const int np = (int)poles.size();
  std::vector<PoleBase<T>> pb(np);
  for (int jp = 0; jp < np; ++jp) {
    PoleMF<T>* pole = &poles[jp];
    FactorWork<T>* fw = fws[jp].get();
    CHK(F->mem.alloc(&pole->panel, P->panel_total));
    CHK(F->mem.alloc(&pole->inv, P->inv_total));
    CHK(F->mem.alloc(&pole->dvec, P->n));
    F->bytes += (int64_t)sizeof(T) * (P->panel_total + P->inv_total + P->n);
    if (lu) {
      CHK(F->mem.alloc(&pole->upanel, P->panel_total));
      CHK(F->mem.alloc(&pole->uinv, P->inv_total));
      CHK(F->mem.alloc(&pole->dconj, P->n));
      F->bytes += (int64_t)sizeof(T) * (P->panel_total + P->inv_total + P->n);
    }
    DevArena& tmp = fw->tmp;
    CHK(tmp.alloc(&fw->upd, P->upd_total));
    CHK(tmp.alloc(&fw->scratch, std::max<int64_t>(P->inv_scratch * (lu ? 2 : 1), 1)));
    CHK(tmp.alloc(&fw->ctmp, std::max<int64_t>(P->conv_scratch * (lu ? 2 : 1), 1)));
    CHK(tmp.alloc(&fw->flag, 1));
    pb[jp] = PoleBase<T>{pole->panel, pole->upanel, pole->inv, pole->uinv, pole->dvec, fw->upd, fw->flag,
                         co_->sigma_hat_re[jp], co_->sigma_hat_im[jp]};
  }
  // GEMM descriptors of the whole program: every launch holds the products of
  // all poles (each pole's descriptors point into its own arrays)
  std::vector<GemmDesc<T>> gd;
  std::vector<StackDesc<T>> stk;
  std::vector<FactorLevelG>& lg = prog->lg;
  lg.assign(nl, FactorLevelG());
  const T one = ST<T>::one(), mone = neg(ST<T>::one()), zero = ST<T>::zero();
  for (int L = 0; L < nl; ++L) {
    std::vector<int> fs = S.levels[L];
    lg[L].stk_off = (int)stk.size();
    int maxns = 0;
    for (int f : fs) maxns = std::max(maxns, S.fronts[f].ns);
    // panel solves, per step J: rows r >= J + jb of the block column,
    //   L(r, c) = sum_t P(r, t) X(c, t) / d(c)   (X: inverse of the unit diagonal block),
    // computed transposed (c x r) so that the 1/d(c) scale is a row scale of the product; the
    // panel rows are read and overwritten by the same tile.  LU: L rows with (U^T)^-1 blocks,
    // U^T rows with L^-1 blocks.
    for (int J = 0; J < maxns; J += FB) {
      GemmLaunch g;
      g.off = (int)gd.size();
      for (int jp = 0; jp < np; ++jp)
      for (int f : fs) {
        const PoleMF<T>* pole = &poles[jp];
        const Front& Fr = S.fronts[f];
        if (Fr.ns <= J) continue;
        const int jb = std::min(FB, Fr.ns - J);
        const int64_t k = (int64_t)Fr.ns + Fr.nb;
        const int rows = (int)(k - J - jb);
        if (rows <= 0) continue;
        for (int side = 0; side < (lu ? 2 : 1); ++side) {
          T* Pn = (side == 0 ? pole->panel : pole->upanel) + P->panel_off[f];
          const T* Xi = (lu ? (side == 0 ? pole->uinv : pole->inv) : pole->inv) + P->inv_off[f];
          GemmDesc<T> d{};
          d.A = Xi + J + (int64_t)J * Fr.ns;
          d.lda = Fr.ns;
          d.B = Pn + (J + jb) + (int64_t)J * k;
          d.ldb = k;
          d.C = Pn + (J + jb) + (int64_t)J * k;
          d.ldc = k;
          d.crs = pole->dvec + Fr.first + J;
          d.M = jb;
          d.N = rows;
          d.K = jb;
          d.flags = GF_TRANSB | GF_TRANSC | GF_CRS | GF_CRS_INV | GF_CRS_ACC;
          d.alpha = one;
          d.beta = zero;
          gd.push_back(d);
          gemm_work(d, &g.flops, &g.bytes);
          g.maxM = std::max(g.maxM, d.M);
          g.maxN = std::max(g.maxN, d.N);
        }
      }
      g.cnt = (int)gd.size() - g.off;
      lg[L].trsm.push_back(g);
    }
    // trailing updates inside the panel, per step J, blocked in two levels: step
    // J updates only the columns of its outer block of FOB columns, and the
    // last step of an outer block updates every column after it with the
    // whole outer block at once (inner dimension FOB instead of FB)
    auto trail_desc = [&](const PoleMF<T>* pole, const Front& Fr, int f, int side, int c0, int kc, int c1,
                          GemmLaunch* g) {
      // rows and columns from c0 on, columns below c1, rank kc from columns c0 - kc
      const int64_t k = (int64_t)Fr.ns + Fr.nb;
      T* Pn = pole->panel + P->panel_off[f];
      T* Un = lu ? pole->upanel + P->panel_off[f] : Pn;
      // LDL^T: L(r0:, r0:) -= L(r0:, J) D L(r0:, J)^T; LU: the same for L with U^T
      // on the right, and for U^T with L on the right
      T* Cb = side == 0 ? Pn : Un;
      T* Bb = side == 0 ? Un : Pn;
      const int J = c0 - kc;
      GemmDesc<T> d{};
      d.C = Cb + c0 + (int64_t)c0 * k;
      d.Cin = d.C;
      d.ldc = d.ldcin = k;
      d.A = Cb + c0 + (int64_t)J * k;
      d.lda = k;
      d.B = Bb + c0 + (int64_t)J * k;
      d.ldb = k;
      d.dk = pole->dvec + Fr.first + J;
      d.M = (int)(k - c0);
      d.N = c1 - c0;
      d.K = kc;
      d.flags = GF_TRANSB | GF_TRI;
      d.tri_off = 0;
      d.alpha = mone;
      d.beta = one;
      gd.push_back(d);
      gemm_work(d, &g->flops, &g->bytes);
      g->maxM = std::max(g->maxM, d.M);
      g->maxN = std::max(g->maxN, d.N);
    };
    for (int J = 0; J < maxns; J += FB) {
      const int Jo = J / FOB * FOB;
      GemmLaunch g, go;
      g.off = (int)gd.size();
      for (int jp = 0; jp < np; ++jp)
        for (int f : fs) {
          const Front& Fr = S.fronts[f];
          const int jb = std::min(FB, Fr.ns - J);
          if (Fr.ns <= J + jb) continue;
          const int r0 = J + jb, c1 = std::min(Fr.ns, Jo + FOB);
          if (c1 > r0)
            for (int side = 0; side < (lu ? 2 : 1); ++side) trail_desc(&poles[jp], Fr, f, side, r0, jb, c1, &g);
        }
      g.cnt = (int)gd.size() - g.off;
      go.off = (int)gd.size();
      for (int jp = 0; jp < np; ++jp)
        for (int f : fs) {
          const Front& Fr = S.fronts[f];
          const int jb = std::min(FB, Fr.ns - J);
          if (Fr.ns <= J + jb || J + jb != Jo + FOB) continue;  // only at the end of a full outer block
          for (int side = 0; side < (lu ? 2 : 1); ++side)
            trail_desc(&poles[jp], Fr, f, side, Jo + FOB, FOB, Fr.ns, &go);
        }
      go.cnt = (int)gd.size() - go.off;
      lg[L].trail.push_back(g);
      lg[L].trail_out.push_back(go);
    }
    // Schur complement update U -= L21 D L21^T (lower)
    {
      GemmLaunch g;
      g.off = (int)gd.size();
      for (int jp = 0; jp < np; ++jp)
      for (int f : fs) {
        const PoleMF<T>* pole = &poles[jp];
        T* upd = fws[jp]->upd;
        const Front& Fr = S.fronts[f];
        if (Fr.nb == 0) continue;
        int64_t k = (int64_t)Fr.ns + Fr.nb;
        T* Pn = pole->panel + P->panel_off[f];
        GemmDesc<T> d{};
        d.C = upd + P->upd_off[f];
        d.Cin = d.C;
        d.ldc = d.ldcin = Fr.nb;
        d.A = Pn + Fr.ns;
        d.lda = k;
        d.B = (lu ? pole->upanel + P->panel_off[f] : Pn) + Fr.ns;  // LU: full update L21 D U12
        d.ldb = k;
        d.dk = pole->dvec + Fr.first;
        d.M = Fr.nb;
        d.N = Fr.nb;
        d.K = Fr.ns;
        d.flags = lu ? GF_TRANSB : (GF_TRANSB | GF_TRI);
        d.tri_off = 0;
        d.alpha = mone;
        d.beta = one;
        gd.push_back(d);
        gemm_work(d, &g.flops, &g.bytes);
        g.maxM = std::max(g.maxM, d.M);
        g.maxN = std::max(g.maxN, d.N);
      }
      g.cnt = (int)gd.size() - g.off;
      lg[L].schur = g;
    }
    // Inverse of L11 (LU: also of U11^T) from its 64 x 64 diagonal-block inverses by
    // recursive doubling: at block size s = 128, 256, ... every block [X1 0; L21 X2] with
    // inverted halves X1 = L1^-1, X2 = L2^-1 gets its lower-left quarter
    //   X21 = -X2 (L21 X1)
    // (T = L21 X1 with X1 lower triangular, then -X2 T with X2 lower triangular); all blocks
    // of one size, over every front and side, are one launch each.
    for (int64_t sz = 2 * FB;; sz *= 2) {
      const int64_t h = sz / 2;
      GemmLaunch g1, g2;
      g1.off = (int)gd.size();
      std::vector<GemmDesc<T>> second;
      for (int jp = 0; jp < np; ++jp)
      for (int side = 0; side < (lu ? 2 : 1); ++side) {
        const PoleMF<T>* pole = &poles[jp];
        T* scratch = fws[jp]->scratch;
        int64_t so = 0;
        for (int f : fs) {
          const Front& Fr = S.fronts[f];
          const int64_t k = (int64_t)Fr.ns + Fr.nb;
          const T* Pn = (side ? pole->upanel : pole->panel) + P->panel_off[f];
          T* X = (side ? pole->uinv : pole->inv) + P->inv_off[f];
          for (int64_t r0 = 0; r0 + h < Fr.ns; r0 += sz) {
            const int64_t h2 = std::min(h, (int64_t)Fr.ns - r0 - h);
            T* Tb = scratch + side * P->inv_scratch + so;
            so += h2 * h;
            GemmDesc<T> d{};
            d.C = Tb;  // T = L21 X1 (h2 x h)
            d.ldc = h2;
            d.A = Pn + (r0 + h) + r0 * k;
            d.lda = k;
            d.B = X + r0 + r0 * Fr.ns;
            d.ldb = Fr.ns;
            d.M = (int)h2;
            d.N = (int)h;
            d.K = (int)h;
            d.flags = GF_BLOW;
            d.alpha = one;
            d.beta = zero;
            gd.push_back(d);
            gemm_work(d, &g1.flops, &g1.bytes);
            g1.maxM = std::max(g1.maxM, d.M);
            g1.maxN = std::max(g1.maxN, d.N);
            GemmDesc<T> e{};
            e.C = X + (r0 + h) + r0 * Fr.ns;  // X21 = -X2 T
            e.ldc = Fr.ns;
            e.A = X + (r0 + h) + (r0 + h) * Fr.ns;
            e.lda = Fr.ns;
            e.B = Tb;
            e.ldb = h2;
            e.M = (int)h2;
            e.N = (int)h;
            e.K = (int)h2;
            e.flags = GF_ALOW;
            e.alpha = mone;
            e.beta = zero;
            second.push_back(e);
          }
        }
      }
      g1.cnt = (int)gd.size() - g1.off;
      if (g1.cnt == 0) break;
      g2.off = (int)gd.size();
      for (const GemmDesc<T>& e : second) {
        gd.push_back(e);
        gemm_work(e, &g2.flops, &g2.bytes);
        g2.maxM = std::max(g2.maxM, e.M);
        g2.maxN = std::max(g2.maxN, e.N);
      }
      g2.cnt = (int)gd.size() - g2.off;
      lg[L].inv1.push_back(g1);
      lg[L].inv2.push_back(g2);
    }
    // Solve panels.  Once the level is factored, each front's panel is replaced
    // by [X; -L21 X] with X = L11^-1 (LU: the U^T panel likewise with
    // (U11^T)^-1), so that a supernodal solve step is one product per front:
    // forward y1 = X w1, w2 -= L21 X w1; backward x1 = X^T D^-1 y1 - (L21 X)^T x2.
    {
      GemmLaunch g;
      g.off = (int)gd.size();
      for (int jp = 0; jp < np; ++jp) {
      const PoleMF<T>* pole = &poles[jp];
      FactorWork<T>* fw = fws[jp].get();
      int64_t co = 0;
      for (int side = 0; side < (lu ? 2 : 1); ++side)
        for (int f : fs) {
          const Front& Fr = S.fronts[f];
          const int64_t k = (int64_t)Fr.ns + Fr.nb;
          T* Pn = (side ? pole->upanel : pole->panel) + P->panel_off[f];
          T* X = (side ? pole->uinv : pole->inv) + P->inv_off[f];
          if (Fr.ns > 0) {
            StackDesc<T> sdsc{Pn, X, fw->ctmp + co, Fr.ns, Fr.nb};
            stk.push_back(sdsc);
            lg[L].stk_max = std::max<int64_t>(lg[L].stk_max, Fr.ns);
          }
          if (Fr.nb == 0 || Fr.ns == 0) continue;
          GemmDesc<T> d{};
          d.C = fw->ctmp + co;
          d.ldc = Fr.nb;
          d.A = Pn + Fr.ns;
          d.lda = k;
          d.B = X;
          d.ldb = Fr.ns;
          d.M = Fr.nb;
          d.N = Fr.ns;
          d.K = Fr.ns;
          d.flags = GF_BLOW;
          d.alpha = mone;
          d.beta = zero;
          gd.push_back(d);
          gemm_work(d, &g.flops, &g.bytes);
          g.maxM = std::max(g.maxM, d.M);
          g.maxN = std::max(g.maxN, d.N);
          co += (int64_t)Fr.nb * Fr.ns;
        }
      }
      g.cnt = (int)gd.size() - g.off;
      lg[L].conv = g;
      lg[L].stk_cnt = (int)stk.size() - lg[L].stk_off;
    }
  }
  // inner-dimension splits of launches with few tiles
  SplitPlan sp;
  for (FactorLevelG& l : lg) {
    for (GemmLaunch& g : l.trsm) plan_split(gd, g, &sp, 0);
    for (GemmLaunch& g : l.trail) plan_split(gd, g, &sp, 0);
    for (GemmLaunch& g : l.trail_out) plan_split(gd, g, &sp, 0);
    plan_split(gd, l.schur, &sp, 0);
    for (GemmLaunch& g : l.inv1) plan_split(gd, g, &sp, 0);
    for (GemmLaunch& g : l.inv2) plan_split(gd, g, &sp, 0);
    plan_split(gd, l.conv, &sp, 0);
  }
  DevArena& tmp = prog->mem;
  if (!sp.at.empty()) {
    typename ST<T>::real* part = nullptr;
    int* cnt = nullptr;
    CHK(tmp.alloc(&part, sp.part));
    CHK(tmp.alloc(&cnt, sp.cnt));
    HIPC(hipMemset(cnt, 0, sizeof(int) * sp.cnt));
    patch_split(gd, sp, part, cnt);
  }
  CHK(tmp.upload(&prog->dgd, gd.data(), gd.size()));
  CHK(tmp.upload(&prog->dstk, stk.data(), stk.size()));
  CHK(tmp.upload(&prog->dpb, pb.data(), pb.size()));
  prog->np = np;
  return ZOLO_OK;
}

// Where the factorization program stands: level L, and within it the stage
// (0 assembly and extend-add, 1 diagonal-block chain, 2 Schur update, 3
// inverse doubling, 4 conversion and panel stacking) and the index inside a
// multi-launch stage.
struct FactorCursor {
  int L = -1;  // -1: buffers not cleared yet
  int stage = 0;
  size_t idx = 0;
  bool done = false;
};

// Enqueue the next short group of launches of the program on s and advance
// the cursor.
template <typename T>
zolo_status factor_step(zolo_pencil* P, std::vector<PoleMF<T>>& poles, std::vector<std::unique_ptr<FactorWork<T>>>& fws,
                        const FactorProg<T>& prog, hipStream_t s, FactorCursor* c) {
  const Symbolic& S = P->S;
  const int nl = (int)S.levels.size();
  const int np = prog.np;
  const GemmDesc<T>* dgd = prog.dgd;
  const std::vector<FactorLevelG>& lg = prog.lg;
  const bool lu = P->cplx();
  if (c->done) return ZOLO_OK;
  if (c->L < 0) {
    for (int j = 0; j < np; ++j) {
      const PoleMF<T>& pole = poles[j];
      HIPC(hipMemsetAsync(fws[j]->flag, 0, sizeof(int), s));
      HIPC(hipMemsetAsync(pole.panel, 0, sizeof(T) * P->panel_total, s));
      HIPC(hipMemsetAsync(pole.inv, 0, sizeof(T) * P->inv_total, s));
      if (lu) {
        HIPC(hipMemsetAsync(pole.upanel, 0, sizeof(T) * P->panel_total, s));
        HIPC(hipMemsetAsync(pole.uinv, 0, sizeof(T) * P->inv_total, s));
      }
    }
    c->L = 0;
    c->stage = 0;
    c->idx = 0;
    if (nl == 0) c->done = true;
    return ZOLO_OK;
  }
  const int L = c->L;
  switch (c->stage) {
    case 0: {
      prof::Scope ps(ZOLO_PROF_FRONT_OTHER, 0.0, 0.0, s);
      const int64_t na = P->lvl_asm_end[L] - P->lvl_asm_begin[L];
      if (P->lvl_upd_end[L] > P->lvl_upd_begin[L])  // this level's update blocks start from zero
        for (int j = 0; j < np; ++j)
          HIPC(hipMemsetAsync(fws[j]->upd + P->lvl_upd_begin[L], 0,
                              sizeof(T) * (P->lvl_upd_end[L] - P->lvl_upd_begin[L]), s));
      if (lu) {
        // asm_src holds the CSR entry (j, i) for the lower position (i, j) (equal for symmetric
        // matrices); the L panel takes (i, j) itself, the transposed U panel takes (j, i)
        front_assemble_cplx<T>(prog.dpb, np, false, P->asm_dst + P->lvl_asm_begin[L],
                               P->asm_src_t + P->lvl_asm_begin[L], na, P->za, P->zb, s);
        front_assemble_cplx<T>(prog.dpb, np, true, P->asm_dst + P->lvl_asm_begin[L], P->asm_src + P->lvl_asm_begin[L],
                               na, P->za, P->zb, s);
        for (const GemmLaunch& g : P->lvl_ext[L])
          front_extend_add_lu<T>(prog.dpb, np, P->pmap, P->ext + g.off, g.cnt, g.tiles, s);
      } else {
        front_assemble<T>(prog.dpb, np, P->asm_dst + P->lvl_asm_begin[L], P->asm_src + P->lvl_asm_begin[L], na, P->pa,
                          P->pb, s);
        for (const GemmLaunch& g : P->lvl_ext[L]) front_extend_add<T>(prog.dpb, np, P->pmap, P->ext + g.off, g.cnt, g.tiles, s);
      }
      c->stage = 1;
      c->idx = 0;
      break;
    }
    case 1: {
      const size_t jj = c->idx;
      if (jj < P->lvl_diag_nJ[L].size()) {
        const DiagDesc* dd = P->diag + P->lvl_diag_off[L];
        const int J = (int)jj * FB;
        const int nd = P->lvl_diag_nJ[L][jj];
        {
          prof::Scope ps(ZOLO_PROF_FRONT_OTHER, 0.0, 0.0, s);
          if (lu)
            front_diag_block_lu<T>(prog.dpb, np, dd, nd, J, s);
          else
            front_diag_block<T>(prog.dpb, np, dd, nd, J, s);
        }
        // LDL^T: L21 = F21 L11^-T D^-1; LU: L21 = F21 U11^-1 D^-1 and U12^T = F12^T L11^-T D^-1
        run_gemm<T>(dgd, lg[L].trsm[jj], s, 0);
        run_gemm<T>(dgd, lg[L].trail[jj], s, 0);
        run_gemm<T>(dgd, lg[L].trail_out[jj], s, 0);
        ++c->idx;
      }
      if (c->idx >= P->lvl_diag_nJ[L].size()) {
        c->stage = 2;
        c->idx = 0;
      }
      break;
    }
    case 2:
      run_gemm<T>(dgd, lg[L].schur, s, 0);
      c->stage = 3;
      c->idx = 0;
      if (prog.pivots_only) {  // the next level needs only the update blocks
        c->stage = 0;
        if (++c->L >= nl) c->done = true;
      }
      break;
    case 3: {
      const size_t I = c->idx;
      if (I < lg[L].inv1.size()) {
        run_gemm<T>(dgd, lg[L].inv1[I], s, 0);
        run_gemm<T>(dgd, lg[L].inv2[I], s, 0);
        ++c->idx;
      }
      if (c->idx >= lg[L].inv1.size()) {
        c->stage = 4;
        c->idx = 0;
      }
      break;
    }
    default: {
      run_gemm<T>(dgd, lg[L].conv, s, 0);
      {
        prof::Scope ps(ZOLO_PROF_FRONT_OTHER, 0.0, 0.0, s);
        front_stack<T>(prog.dstk + lg[L].stk_off, lg[L].stk_cnt, lg[L].stk_max, s);
      }
      c->stage = 0;
      c->idx = 0;
      if (++c->L >= nl) {
        if (lu)
          for (int j = 0; j < np; ++j) conj_copy(poles[j].dconj, poles[j].dvec, P->n, s);
        c->done = true;
      }
      break;
    }
  }
  HIPC(hipGetLastError());
  return ZOLO_OK;
}

// all poles: one program whose launches run every pole, on the caller's
// stream; wait, check pivots
template <typename T>
zolo_status factor_all(zolo_factors* F, zolo_pencil* P, const zolo_filter_coeffs* co, std::vector<PoleMF<T>>* poles,
                       hipStream_t s, bool pivots_only = false) {
  const int np = co->r1;
  poles->assign(np, PoleMF<T>());
  std::vector<std::unique_ptr<FactorWork<T>>> fw(np);
  for (int j = 0; j < np; ++j) {
    fw[j].reset(new FactorWork<T>());
    fw[j]->tmp.set_stream(s);
  }
  FactorProg<T> prog;
  prog.mem.set_stream(s);
  prog.pivots_only = pivots_only;
  CHK(factor_plan<T>(F, P, co, *poles, fw, &prog));
  FactorCursor cur;
  while (!cur.done) CHK(factor_step<T>(P, *poles, fw, prog, s, &cur));
  const hipError_t se = hipStreamSynchronize(s);
  if (se != hipSuccess) {
    set_error("HIP error in the factorization: %s", hipGetErrorString(se));
    return ZOLO_EDEVICE;
  }
  for (int j = 0; j < np; ++j) {
    int hflag = 0;
    HIPC(hipMemcpy(&hflag, fw[j]->flag, sizeof(int), hipMemcpyDeviceToHost));
    if (hflag) {
      set_error("zero pivot in the LDL^T of A - sigma B (pole %d)", j);
      return ZOLO_EBREAKDOWN;
    }
  }
  return ZOLO_OK;
}

}  // namespace

extern "C" zolo_status zolo_factor(zolo_ctx* ctx, zolo_pencil* P, const zolo_filter_coeffs* co, int precision,
                                   void* stream, zolo_factors** out) {
  if (!ctx || !P || !co || !out) {
    set_error("zolo_factor: null argument");
    return ZOLO_EINVAL;
  }
  if (co->r1 < 1 || co->r1 > ZOLO_MAX_R || co->r2 < 1 || co->r2 > ZOLO_MAX_R) {
    set_error("zolo_factor: coefficients not planned (r1=%d, r2=%d)", co->r1, co->r2);
    return ZOLO_EINVAL;
  }
  if (co->kind < ZOLO_FILTER_HYBRID || co->kind > ZOLO_FILTER_GAUSS) {
    set_error("zolo_factor: unknown filter kind %d", co->kind);
    return ZOLO_EINVAL;
  }
  if (precision != ZOLO_PREC_FP64 && precision != ZOLO_PREC_MIXED) {
    set_error("zolo_factor: unknown precision %d", precision);
    return ZOLO_EINVAL;
  }
  HIPC(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  std::unique_ptr<zolo_factors> F(new zolo_factors());
  F->P = P;
  F->co = *co;
  F->precision = precision;
  double t0 = now_s();
  if (precision == ZOLO_PREC_FP64)
    CHK(factor_all<zd>(F.get(), P, co, &F->pd, s));
  else
    CHK(factor_all<zf>(F.get(), P, co, &F->pf, s));
  F->t_factor = now_s() - t0;
  *out = F.release();
  return ZOLO_OK;
}

extern "C" void zolo_factors_free(zolo_factors* f) { delete f; }

// Sylvester inertia on the device: for real shifts sigma_k, K = A - sigma_k B
// is Hermitian (real symmetric for real pencils), its unpivoted LDL^T (LU =
// L D L^H for complex pencils) in the nested-dissection order is a congruence,
// so the number of negative pivots of D is the number of eigenvalues of (A, B)
// below sigma_k.  All shifts of a call are factored concurrently (one stream
// each), in complex128 with zero imaginary shift.
extern "C" zolo_status zolo_inertia(zolo_ctx* ctx, zolo_pencil* P, const double* sigmas, int nshift,
                                    int64_t* counts, void* stream) {
  if (!ctx || !P || !sigmas || !counts || nshift < 1 || nshift > ZOLO_MAX_R) {
    set_error("zolo_inertia: invalid argument (1 <= nshift <= %d)", ZOLO_MAX_R);
    return ZOLO_EINVAL;
  }
  for (int k = 0; k < nshift; ++k)
    if (!std::isfinite(sigmas[k])) {
      set_error("zolo_inertia: shift %d is not finite", k);
      return ZOLO_EINVAL;
    }
  HIPC(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  // shifts factored together: as many as 80% of the free device memory holds
  const int64_t lu = P->cplx() ? 2 : 1;
  const int64_t per_shift =
      (int64_t)(P->cplx() ? sizeof(zd) : sizeof(double)) * (lu * (P->panel_total + P->inv_total + P->n) +
                                                              P->upd_total + lu * (P->inv_scratch + P->conv_scratch));
  size_t free_b = 0, total_b = 0;
  HIPC(hipMemGetInfo(&free_b, &total_b));
  int group = (int)std::max<int64_t>(1, std::min<int64_t>(nshift, (int64_t)(0.8 * (double)free_b) / per_shift));
  if (g_inertia_cap > 0) group = std::min(group, g_inertia_cap);
  std::vector<zd> d(P->cplx() ? P->n : 0);
  std::vector<double> dr(P->cplx() ? 0 : P->n);
  for (int k0 = 0; k0 < nshift; k0 += group) {
    const int ng = std::min(group, nshift - k0);
    zolo_filter_coeffs co{};
    co.r1 = ng;
    co.r2 = 1;
    for (int k = 0; k < ng; ++k) co.sigma_hat_re[k] = sigmas[k0 + k];
    std::unique_ptr<zolo_factors> F(new zolo_factors());
    F->P = P;
    F->co = co;
    F->precision = ZOLO_PREC_FP64;
    // real pencils at real shifts: a real symmetric LDL^T; complex Hermitian
    // pencils: LDL^H in complex arithmetic (D real up to rounding)
    zolo_status rc = P->cplx() ? factor_all<zd>(F.get(), P, &co, &F->pd, s, true)
                               : factor_all<double>(F.get(), P, &co, &F->pr, s, true);
    if (rc == ZOLO_EBREAKDOWN) {
      set_error("zolo_inertia: zero pivot (a shift is numerically an eigenvalue); move the shift slightly");
      return rc;
    }
    CHK(rc);
    for (int k = 0; k < ng; ++k) {
      int64_t neg = 0;
      if (P->cplx()) {
        HIPC(hipMemcpy(d.data(), F->pd[k].dvec, sizeof(zd) * P->n, hipMemcpyDeviceToHost));
        for (const zd& v : d) neg += v.re < 0.0;
      } else {
        HIPC(hipMemcpy(dr.data(), F->pr[k].dvec, sizeof(double) * P->n, hipMemcpyDeviceToHost));
        for (double v : dr) neg += v < 0.0;
      }
      counts[k0 + k] = neg;
    }
  }
  return ZOLO_OK;
}

// ===========================================================================
// supernodal solves
// ===========================================================================
namespace {

template <typename T>
zolo_status build_solve_prog(zolo_factors* F, int p, SolveProg<T>* G, const std::vector<PoleMF<T>>& poles) {
  // One program solves all r1 poles at once: every launch of a level covers the
  // level's fronts for every pole, with per-pole buffer regions.
  zolo_pencil* P = F->P;
  const Symbolic& S = P->S;
  const int nl = (int)S.levels.size();
  // Solves of one program ("virtual poles").  LDL^T: K_j^-1 for every pole.
  // LU (complex Hermitian pencils): K_j^-1 = U^-1 D^-1 L^-1, then
  // K_j^-H = L^-H conj(D)^-1 U^-H, whose triangles are the conjugates of the
  // stored U^T and L factors: the forward pass runs on (U^T, its inverse
  // blocks), the backward pass on (L, its inverse blocks), all conjugated.
  // Each front's solve panel is [X; -L21 X] (k x ns, ld k) with X = L11^-1.
  struct Role {
    const T *fp, *bp, *dv;
    int cj;
  };
  const bool lu = P->cplx();
  std::vector<Role> roles;
  for (const PoleMF<T>& pm : poles) roles.push_back({pm.panel, lu ? pm.upanel : pm.panel, pm.dvec, 0});
  if (lu)
    for (const PoleMF<T>& pm : poles) roles.push_back({pm.upanel, pm.panel, pm.dconj, GF_CONJA});
  const int np = (int)roles.size();
  G->p = p;
  G->np = np;
  int64_t wmax = 0;
  std::vector<int64_t> uoff(S.fronts.size(), 0);
  int64_t utot = 0;
  for (int L = 0; L < nl; ++L) {
    int64_t w = 0;
    for (int f : S.levels[L]) {
      const Front& Fr = S.fronts[f];
      w += (int64_t)(Fr.ns + Fr.nb) * p;
      uoff[f] = utot;
      utot += (int64_t)Fr.nb * p;
    }
    wmax = std::max(wmax, w);
  }
  const int64_t npx = P->n * p;
  G->xstride = npx;
  CHK(G->mem.alloc(&G->W, wmax * np));
  CHK(G->mem.alloc(&G->U, utot * np));
  CHK(G->mem.alloc(&G->Y, npx * np));
  CHK(G->mem.alloc(&G->X, npx * np));
  std::vector<SolveDesc> sd;
  G->lvl_sd_off.assign(nl, 0);
  G->lvl_sd_cnt.assign(nl, 0);
  G->lvl_maxk.assign(nl, 0);
  // per level, per front (level order): offsets within one pole's regions
  std::vector<std::vector<int64_t>> woff(nl);
  for (int L = 0; L < nl; ++L) {
    int64_t w = 0;
    for (int f : S.levels[L]) {
      const Front& Fr = S.fronts[f];
      woff[L].push_back(w);
      w += (int64_t)(Fr.ns + Fr.nb) * p;
      G->lvl_maxk[L] = std::max(G->lvl_maxk[L], Fr.ns + Fr.nb);
    }
    G->lvl_sd_off[L] = (int)sd.size();
    for (int j = 0; j < np; ++j) {
      size_t i = 0;
      for (int f : S.levels[L]) {
        const Front& Fr = S.fronts[f];
        SolveDesc d{};
        d.dv = roles[j].dv;
        d.w = j * wmax + woff[L][i];
        d.u = j * utot + uoff[f];
        d.srow = Fr.struct_off;
        d.xo = j * npx;
        d.first = Fr.first;
        d.ns = Fr.ns;
        d.nb = Fr.nb;
        d.k = Fr.ns + Fr.nb;
        sd.push_back(d);
        ++i;
      }
    }
    G->lvl_sd_cnt[L] = (int)sd.size() - G->lvl_sd_off[L];
  }
  G->own = P->fill_own;
  G->cbeg = P->fill_cbeg;
  G->cidx = P->fill_cidx;
  G->lvl_row_off = P->lvl_fill_off;
  G->lvl_rows = P->lvl_fill_rows;
  G->wstride = wmax;
  G->ustride = utot;
  CHK(G->mem.upload(&G->sd, sd.data(), sd.size()));
  const T one = ST<T>::one(), mone = neg(ST<T>::one()), zero = ST<T>::zero();
  G->fw.assign(nl, GemmLaunch());
  G->bw.assign(nl, GemmLaunch());
  std::vector<GemmDesc<T>> gd;
  for (int L = 0; L < nl; ++L) {
    const std::vector<int>& fs = S.levels[L];
    auto add = [&](GemmLaunch& g, const GemmDesc<T>& d) {
      gd.push_back(d);
      gemm_work(d, &g.flops, &g.bytes);
      g.maxM = std::max(g.maxM, d.M);
      g.maxN = std::max(g.maxN, d.N);
    };
    // forward: Y[first:first+ns] = X W[0:ns] and U = W[ns:k] + (-L21 X) W[0:ns],
    // both reading only W, so one launch per level
    GemmLaunch& gf = G->fw[L];
    gf.off = (int)gd.size();
    for (int j = 0; j < np; ++j)
      for (size_t i = 0; i < fs.size(); ++i) {
        const Front& Fr = S.fronts[fs[i]];
        if (Fr.ns == 0) continue;
        const int64_t k = (int64_t)Fr.ns + Fr.nb;
        const T* Pn = roles[j].fp + P->panel_off[fs[i]];
        const T* Wf = G->W + j * wmax + woff[L][i];
        GemmDesc<T> d{};
        d.C = G->Y + j * npx + (int64_t)Fr.first * p;
        d.ldc = p;
        d.A = Pn;
        d.lda = k;
        d.B = Wf;
        d.ldb = p;
        d.M = Fr.ns;
        d.N = p;
        d.K = Fr.ns;
        d.flags = GF_TRANSB | GF_TRANSC | GF_ALOW | roles[j].cj;
        d.alpha = one;
        d.beta = zero;
        add(gf, d);
        if (Fr.nb == 0) continue;
        GemmDesc<T> e{};
        e.C = G->U + j * utot + uoff[fs[i]];
        e.ldc = p;
        e.Cin = Wf + (int64_t)Fr.ns * p;
        e.ldcin = p;
        e.A = Pn + Fr.ns;
        e.lda = k;
        e.B = Wf;
        e.ldb = p;
        e.M = Fr.nb;
        e.N = p;
        e.K = Fr.ns;
        e.flags = GF_TRANSB | GF_TRANSC | roles[j].cj;
        e.alpha = one;
        e.beta = one;
        add(gf, e);
      }
    gf.cnt = (int)gd.size() - gf.off;
    // backward: X[first:first+ns] = [X; -L21 X]^T [D^-1 y1; x2], with the
    // stacked right-hand side gathered into W (X^T is upper triangular)
    GemmLaunch& gb = G->bw[L];
    gb.off = (int)gd.size();
    for (int j = 0; j < np; ++j)
      for (size_t i = 0; i < fs.size(); ++i) {
        const Front& Fr = S.fronts[fs[i]];
        if (Fr.ns == 0) continue;
        const int64_t k = (int64_t)Fr.ns + Fr.nb;
        GemmDesc<T> d{};
        d.C = G->X + j * npx + (int64_t)Fr.first * p;
        d.ldc = p;
        d.A = roles[j].bp + P->panel_off[fs[i]];
        d.lda = k;
        d.B = G->W + j * wmax + woff[L][i];
        d.ldb = p;
        d.M = Fr.ns;
        d.N = p;
        d.K = (int)k;
        d.flags = GF_TRANSA | GF_TRANSB | GF_TRANSC | GF_AUP | roles[j].cj;
        d.alpha = one;
        d.beta = zero;
        add(gb, d);
      }
    gb.cnt = (int)gd.size() - gb.off;
  }
  // inner-dimension splits of launches with few tiles (the top levels)
  SplitPlan sp;
  for (int L = 0; L < nl; ++L) {
    plan_split(gd, G->fw[L], &sp, 1);
    plan_split(gd, G->bw[L], &sp, 1);
  }
  if (!sp.at.empty()) {
    typename ST<T>::real* part = nullptr;
    int* cnt = nullptr;
    CHK(G->mem.alloc(&part, sp.part));
    CHK(G->mem.alloc(&cnt, sp.cnt));
    HIPC(hipMemset(cnt, 0, sizeof(int) * sp.cnt));
    patch_split(gd, sp, part, cnt);
  }
  CHK(G->mem.upload(&G->gd, gd.data(), gd.size()));
  return ZOLO_OK;
}

template <typename T>
SolveProg<T>* get_prog(zolo_factors* F, int p);
template <>
SolveProg<zd>* get_prog<zd>(zolo_factors* F, int p) {
  auto it = F->prog_d.find(p);
  if (it != F->prog_d.end()) return it->second.get();
  std::unique_ptr<SolveProg<zd>> G(new SolveProg<zd>());
  if (build_solve_prog<zd>(F, p, G.get(), F->pd) != ZOLO_OK) return nullptr;
  SolveProg<zd>* r = G.get();
  F->prog_d[p] = std::move(G);
  return r;
}
template <>
SolveProg<zf>* get_prog<zf>(zolo_factors* F, int p) {
  auto it = F->prog_f.find(p);
  if (it != F->prog_f.end()) return it->second.get();
  std::unique_ptr<SolveProg<zf>> G(new SolveProg<zf>());
  if (build_solve_prog<zf>(F, p, G.get(), F->pf) != ZOLO_OK) return nullptr;
  SolveProg<zf>* r = G.get();
  F->prog_f[p] = std::move(G);
  return r;
}

// X_j (in G->X + j xstride, new ordering, N x p) = K_j^-1 src_j for all poles j.
// src: N x p row-major (new ordering); src_stride = 0 shares one right-hand
// side, otherwise pole j reads src + j * src_stride.
// per_pole: pole j reads its right-hand side at src + j * xstride (ld p)
template <typename Ts, typename T>
void run_solve(zolo_factors* F, SolveProg<T>* G, const Ts* src, int64_t lds, bool per_pole, hipStream_t s) {
  zolo_pencil* P = F->P;
  const int nl = (int)P->S.levels.size();
  const int p = G->p;
  // algorithmic bytes of the gathers: every row written once, every row read
  // once (the shared right-hand side once for all poles), the index tables
  const double vt = sizeof(T), vs = sizeof(Ts), npd = G->np;
  for (int L = 0; L < nl; ++L) {
    {
      const double by = npd * p * vt * (P->lvl_fill_rows[L] + P->lvl_fill_adds[L]) +
                        (per_pole ? npd : 1.0) * p * vs * P->lvl_fill_src[L] +
                        4.0 * (2.0 * P->lvl_fill_rows[L] + P->lvl_fill_adds[L]);
      prof::Scope ps(ZOLO_PROF_SOLVE_GATHER, 0.0, by, s);
      solve_fill<Ts, T>(G->W, G->wstride, src, lds, per_pole ? G->xstride : 0, G->U, G->ustride,
                        G->own + G->lvl_row_off[L], G->cbeg + G->lvl_row_off[L], G->cidx, G->lvl_rows[L], p, G->np, s);
    }
    run_gemm<T>(G->gd, G->fw[L], s, 1);
  }
  for (int L = nl - 1; L >= 0; --L) {
    {
      const double by = 2.0 * npd * p * vt * P->lvl_k[L];  // each row of W written, its source row read
      prof::Scope ps(ZOLO_PROF_SOLVE_GATHER, 0.0, by, s);
      solve_gather_back<T>(G->W, G->Y, G->X, P->struct_rows, G->sd + G->lvl_sd_off[L], G->lvl_sd_cnt[L], p,
                           G->lvl_maxk[L], s);
    }
    run_gemm<T>(G->gd, G->bw[L], s, 1);
  }
}

int ensure_ws(zolo_factors* F, int p, int mmax) {
  Workspace* ws = F->ws.get();
  const bool cx = F->P->cplx();
  const int nshift = F->co.r2 * (cx ? 2 : 1);  // complex pencils: +i sqrt(c_j) and -i sqrt(c_j)
  if (ws && ws->p >= p && ws->mmax >= mmax && ws->nshift == nshift) return ZOLO_OK;
  F->ws.reset(new Workspace());
  ws = F->ws.get();
  const int64_t n = F->P->n;
  const int ef = cx ? 2 : 1;
  ws->p = p;
  ws->mmax = mmax;
  ws->nshift = nshift;
  ws->ef = ef;
  ws->n = n;
  const int64_t Mp = (int64_t)(mmax + 1) * p;
  CHK(ws->mem.alloc(&ws->Vb, n * Mp * ef));
  CHK(ws->mem.alloc(&ws->W, n * p * ef));
  CHK(ws->mem.alloc(&ws->T1, n * p * ef));
  CHK(ws->mem.alloc(&ws->Tb, n * p * ef));
  const int np = F->co.r1 * (cx ? 2 : 1);
  CHK(ws->mem.alloc(&ws->Xc, n * p * np));
  CHK(ws->mem.alloc(&ws->Rc, n * p * np));
  CHK(ws->mem.alloc(&ws->Dc, 1));
  ws->ldh = Mp;
  CHK(ws->mem.alloc(&ws->H, Mp * (int64_t)mmax * p * ef));
  CHK(ws->mem.alloc(&ws->hbuf, Mp * p * ef));
  // gemm_tn's row-chunk partial sums: about 2048 tiles of at most 64 x 96
  ws->partial_len = std::max<int64_t>({Mp * p * 8, (int64_t)p * p * 256, (int64_t)2048 * 64 * 96});
  CHK(ws->mem.alloc(&ws->partial, ws->partial_len * ef));
  for (double** q : {&ws->G, &ws->R1, &ws->R1i, &ws->R2, &ws->R2i, &ws->R0, &ws->Rk})
    CHK(ws->mem.alloc(q, (size_t)p * p * ef));
  CHK(ws->mem.alloc(&ws->flag, 4));
  CHK(ws->mem.alloc(&ws->res, (size_t)nshift * p));
  CHK(ws->mem.alloc(&ws->coef, nshift));
  CHK(ws->mem.alloc(&ws->shift_im, nshift));
  CHK(ws->mem.alloc(&ws->Cm, (size_t)mmax * p * p * ef));
  CHK(ws->mem.alloc(&ws->Ys, (size_t)nshift * mmax * p * p));
  ws->gdesc_cap = 1024;
  char* gd = nullptr;
  CHK(ws->mem.alloc(&gd, sizeof(GemmDesc<zd>) * (ws->gdesc_cap + 4)));
  ws->gdesc = gd;
  CHK(ws->mem.alloc(&ws->cn_partial, (size_t)colnorm_partials(n) * p * np + 16));
  CHK(ws->mem.alloc(&ws->cn_out, (size_t)p * np));
  HlsState& h = ws->hls;
  h.ldr = Mp;
  h.mmax = mmax;
  h.p = p;
  h.nshift = nshift;
  CHK(ws->mem.alloc(&h.R, (size_t)nshift * Mp * mmax * p));
  CHK(ws->mem.alloc(&h.refl, (size_t)nshift * mmax * p * (p + 1)));
  CHK(ws->mem.alloc(&h.tau, (size_t)nshift * mmax * p));
  CHK(ws->mem.alloc(&h.g, (size_t)nshift * Mp * p));
  // Corollary 1: Z_2r2(g) = (M/2) sum_j a_j [(g + i sqrt c_j)^-1 + (g - i sqrt c_j)^-1], so the
  // filter is Y = V/2 + sum over shifts of (M a_j / 4) (G + s)^-1 V.  Real pencils solve only
  // s = +i sqrt c_j and take twice the real part.
  std::vector<double> sh(nshift), cf(nshift);
  for (int q = 0; q < nshift; ++q) {
    const int j = q % F->co.r2;
    sh[q] = (q < F->co.r2 ? 1.0 : -1.0) * std::sqrt(F->co.c[j]);
    cf[q] = (cx ? 0.25 : 0.5) * F->co.M * F->co.a[j];
  }
  HIPC(hipMemcpy(ws->shift_im, sh.data(), sizeof(double) * nshift, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ws->coef, cf.data(), sizeof(double) * nshift, hipMemcpyHostToDevice));
  h.shift_im = ws->shift_im;
  return ZOLO_OK;
}

// X_j (zd, N x p, new ordering, at X + j n p) = K_j^{-1} T for every pole j
// (T of the block scalar type, new ordering, ld p).  Complex Hermitian pencils
// also solve the conjugate poles: X_{r1+j} = K_j^-H T = (A - conj(sigma_j) B)^-1 T.
// FP64 factors: one supernodal solve of all poles.  Mixed precision: complex64
// factors, then iterative refinement against FP64 residuals
// R_j = T - (A - sigma_j B) X_j, all poles per sweep with one host
// synchronization, until max_j,c ||R_j,c|| / ||T_c|| <= tol_inner, or until a
// sweep gains less than a factor 2 (the FP64 residual floor of an
// ill-conditioned pole), or after max_refine corrections.
// Xres (optional): where the solutions are left.  FP64 factors: the solve
// program's own buffer (valid until its next solve), so nothing is copied to X.
template <typename VT>
zolo_status poles_solve_all(zolo_factors* F, const VT* T, int p, zd* X, double tol_inner, hipStream_t s,
                            const zd** Xres = nullptr) {
  zolo_pencil* P = F->P;
  const int64_t n = P->n;
  const int r1 = F->co.r1;
  const int np = r1 * (P->cplx() ? 2 : 1);
  const int64_t npx = n * p;
  if (F->precision == ZOLO_PREC_FP64) {
    SolveProg<zd>* G = get_prog<zd>(F, p);
    if (!G) return ZOLO_ENOMEM;
    run_solve<VT, zd>(F, G, T, p, false, s);
    if (Xres)
      *Xres = G->X;
    else
      HIPC(hipMemcpyAsync(X, G->X, sizeof(zd) * npx * np, hipMemcpyDeviceToDevice, s));
    F->n_solv += (long long)p * np;
    return ZOLO_OK;
  }
  SolveProg<zf>* G = get_prog<zf>(F, p);
  if (!G) return ZOLO_ENOMEM;
  Workspace& ws = *F->ws;
  run_solve<VT, zf>(F, G, T, p, false, s);
  set_lowp(X, G->X, npx * np, s);
  F->n_solv += (long long)p * np;
  const int64_t cnp = (int64_t)colnorm_partials(n) * p;
  std::vector<double> tn(p), rn((size_t)np * p);
  if constexpr (ST<VT>::cplx)
    colnorm2_cplx(T, n, p, ws.cn_partial, ws.cn_out, s);
  else
    colnorm2_real(T, p, n, p, ws.cn_partial, ws.cn_out, s);
  HIPC(hipMemcpyAsync(tn.data(), ws.cn_out, sizeof(double) * p, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  for (double& v : tn) v = std::sqrt(std::max(v, 1e-300));
  double prev = HUGE_VAL, worst = HUGE_VAL;
  int sweeps = 0;
  for (;;) {
    for (int j = 0; j < np; ++j) {
      const int q = j % r1;
      const double sr = F->co.sigma_hat_re[q], si = (j < r1 ? 1.0 : -1.0) * F->co.sigma_hat_im[q];
      {
        prof::Scope ps(ZOLO_PROF_SPMM, 8.0 * P->nnz * p, (ST<VT>::cplx ? 36.0 : 20.0) * P->nnz + 48.0 * n * p, s);
        if constexpr (ST<VT>::cplx)
          spmm_shift_resid(n, P->prow, P->pcol, P->za, P->zb, sr, si, X + j * npx, T, p, p, ws.Rc + j * npx, s);
        else
          spmm_shift_resid(n, P->prow, P->pcol, P->pa, P->pb, sr, si, X + j * npx, T, p, p, ws.Rc + j * npx, s);
      }
      prof::Scope ps(ZOLO_PROF_ELEMWISE, 0.0, 16.0 * n * p, s);
      colnorm2_cplx(ws.Rc + j * npx, n, p, ws.cn_partial + j * cnp, ws.cn_out + (int64_t)j * p, s);
    }
    HIPC(hipMemcpyAsync(rn.data(), ws.cn_out, sizeof(double) * np * p, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    worst = 0.0;
    for (int j = 0; j < np; ++j)
      for (int c = 0; c < p; ++c) worst = std::max(worst, std::sqrt(rn[(size_t)j * p + c]) / tn[c]);
    if (worst <= tol_inner || sweeps >= F->max_refine || worst > 0.5 * prev) break;
    run_solve<zd, zf>(F, G, ws.Rc, p, true, s);
    add_lowp(X, G->X, npx * np, s);
    F->n_refine += (long long)p * np;
    ++sweeps;
    prev = worst;
  }
  F->refine_sweeps_max = std::max(F->refine_sweeps_max, sweeps);
  if (worst > tol_inner) {
    ++F->refine_missed;
    F->refine_worst = std::max(F->refine_worst, worst);
  }
  if (Xres) *Xres = X;
  return ZOLO_OK;
}

// W (N x p, ld ldw) = G V (V: N x p new ordering, ld ldv).  Proposition 2:
// G V = M_hat [c0 V + sum_j (w_hat_j K_j^-1 + conj(w_hat_j) conj-pole solve) B V];
// for real pencils the conjugate-pole solve is conj(K_j^-1 B V).
template <typename VT>
zolo_status apply_G_new(zolo_factors* F, const VT* V, int64_t ldv, int p, VT* W, int64_t ldw, double tol_inner,
                        hipStream_t s) {
  zolo_pencil* P = F->P;
  const int64_t n = P->n;
  Workspace& ws = *F->ws;
  const zolo_filter_coeffs& co = F->co;
  VT* Tb = (VT*)ws.Tb;
  // T = B V
  {
    prof::Scope ps(ZOLO_PROF_SPMM, 2.0 * P->nnz * p * (ST<VT>::cplx ? 4 : 1),
                   (ST<VT>::cplx ? 20.0 : 12.0) * P->nnz + 8.0 * (n + 1) + 2.0 * sizeof(VT) * n * p, s);
    if constexpr (ST<VT>::cplx)
      spmm_cplx(n, P->prow, P->pcol, P->zb, nullptr, V, ldv, p, Tb, p, nullptr, 0, s);
    else
      spmm_real(n, P->prow, P->pcol, P->pb, nullptr, V, ldv, p, Tb, p, nullptr, 0, s);
  }
  const zd* Xs = nullptr;  // the poles' solutions, N x p each, pole j at Xs + j n p
  if constexpr (ST<VT>::cplx) {
    {
      prof::Scope ps(ZOLO_PROF_ELEMWISE, 0.0, 2.0 * sizeof(VT) * n * p, s);
      scale_copy(W, ldw, V, ldv, co.M_hat * co.c0, n, p, s);
    }
    CHK(poles_solve_all<VT>(F, Tb, p, ws.Xc, tol_inner, s, &Xs));
    for (int j = 0; j < co.r1; ++j) {
      prof::Scope ps(ZOLO_PROF_ELEMWISE, 0.0, 48.0 * n * p, s);
      axpy_pair(W, ldw, Xs + (int64_t)j * n * p, Xs + (int64_t)(co.r1 + j) * n * p, co.M_hat * co.w_hat_re[j],
                co.M_hat * co.w_hat_im[j], n, p, s);
    }
  } else {
    // W = M c0 V + sum_j 2 Re(M w_j X_j) in one pass over V, the X_j and W
    CHK(poles_solve_all<VT>(F, Tb, p, ws.Xc, tol_inner, s, &Xs));
    GCombineCoef wc{};
    for (int j = 0; j < co.r1; ++j) {
      wc.wr[j] = co.M_hat * co.w_hat_re[j];
      wc.wi[j] = co.M_hat * co.w_hat_im[j];
    }
    prof::Scope ps(ZOLO_PROF_ELEMWISE, 0.0, (16.0 + 16.0 * co.r1) * n * p, s);
    g_combine_real(W, ldw, (const double*)V, ldv, co.M_hat * co.c0, Xs, n * p, wc, co.r1, n, p, s);
  }
  return ZOLO_OK;
}

// CholQR2 of Win (N x p row-major, ld ldin) into Qout (ld ldq); R (p x p) = R2 R1 into ws.Rk
template <typename VT>
zolo_status cholqr2(zolo_factors* F, const VT* Win, int64_t ldin, VT* Qout, int64_t ldq, int p, bool* breakdown,
                    hipStream_t s) {
  Workspace& ws = *F->ws;
  const int64_t n = F->P->n;
  VT *G = (VT*)ws.G, *R1 = (VT*)ws.R1, *R1i = (VT*)ws.R1i, *R2 = (VT*)ws.R2, *R2i = (VT*)ws.R2i, *T1 = (VT*)ws.T1;
  int hf[2] = {0, 0};
  HIPC(hipMemsetAsync(ws.flag, 0, sizeof(int) * 4, s));
  CHK(gemm_tn<VT>(ws, Win, ldin, Win, ldin, n, p, p, G, p, false, s));
  chol_upper_inv<VT>(G, p, 1e-15, R1, R1i, ws.flag, s);
  CHK(gemm_nt_big<VT>(ws, T1, p, nullptr, 0, 0.0, 1.0, R1i, p, true, Win, ldin, n, p, p, s));
  CHK(gemm_tn<VT>(ws, T1, p, T1, p, n, p, p, G, p, false, s));
  chol_upper_inv<VT>(G, p, 0.0, R2, R2i, ws.flag + 1, s);
  CHK(gemm_nt_big<VT>(ws, Qout, ldq, nullptr, 0, 0.0, 1.0, R2i, p, true, T1, p, n, p, p, s));
  upper_mul<VT>(R2, R1, (VT*)ws.Rk, p, s);
  HIPC(hipMemcpyAsync(hf, ws.flag, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  *breakdown = hf[0] || hf[1];
  return ZOLO_OK;
}

// W (b x nrhs, col-major) = T^-1 W for a b x b col-major T, Gaussian
// elimination with partial pivoting on the host; false if T is singular
bool dense_solve_host(std::vector<std::complex<double>>& T, std::vector<std::complex<double>>& W, int b, int nrhs) {
  for (int k = 0; k < b; ++k) {
    int piv = k;
    for (int i = k + 1; i < b; ++i)
      if (std::abs(T[i + (size_t)k * b]) > std::abs(T[piv + (size_t)k * b])) piv = i;
    if (T[piv + (size_t)k * b] == std::complex<double>(0.0, 0.0)) return false;
    if (piv != k) {
      for (int j = 0; j < b; ++j) std::swap(T[k + (size_t)j * b], T[piv + (size_t)j * b]);
      for (int j = 0; j < nrhs; ++j) std::swap(W[k + (size_t)j * b], W[piv + (size_t)j * b]);
    }
    const std::complex<double> d = T[k + (size_t)k * b];
    for (int i = k + 1; i < b; ++i) {
      const std::complex<double> l = T[i + (size_t)k * b] / d;
      if (l == std::complex<double>(0.0, 0.0)) continue;
      for (int j = k + 1; j < b; ++j) T[i + (size_t)j * b] -= l * T[k + (size_t)j * b];
      for (int j = 0; j < nrhs; ++j) W[i + (size_t)j * b] -= l * W[k + (size_t)j * b];
    }
  }
  for (int j = 0; j < nrhs; ++j)
    for (int k = b - 1; k >= 0; --k) {
      std::complex<double> v = W[k + (size_t)j * b];
      for (int t = k + 1; t < b; ++t) v -= T[k + (size_t)t * b] * W[t + (size_t)j * b];
      W[k + (size_t)j * b] = v / T[k + (size_t)k * b];
    }
  return true;
}

// Thin QR of a rows x p col-major complex matrix on the host by Householder
// reflections: A = Q R, Q rows x p with orthonormal columns (whatever the rank
// of A), R p x p upper triangular.
void householder_qr_host(const std::vector<std::complex<double>>& A, int64_t rows, int p,
                         std::vector<std::complex<double>>* Q, std::vector<std::complex<double>>* R) {
  using cd = std::complex<double>;
  std::vector<cd> W(A);
  std::vector<std::vector<cd>> vs(p);
  std::vector<double> taus(p, 0.0);
  for (int k = 0; k < p; ++k) {
    cd* col = W.data() + (size_t)k * rows;
    double nrm2 = 0.0;
    for (int64_t i = k; i < rows; ++i) nrm2 += std::norm(col[i]);
    const double nrm = std::sqrt(nrm2), a0 = std::abs(col[k]);
    const cd ph = a0 > 0.0 ? col[k] / a0 : cd(1.0, 0.0);
    std::vector<cd> v(col + k, col + rows);
    v[0] += ph * nrm;
    double vn2 = 0.0;
    for (const cd& x : v) vn2 += std::norm(x);
    const double t = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
    for (int j = k; j < p; ++j) {  // columns k.. of W: x -= t v (v^H x)
      cd* x = W.data() + (size_t)j * rows + k;
      cd d(0.0, 0.0);
      for (size_t i = 0; i < v.size(); ++i) d += std::conj(v[i]) * x[i];
      d *= t;
      for (size_t i = 0; i < v.size(); ++i) x[i] -= d * v[i];
    }
    vs[k] = std::move(v);
    taus[k] = t;
  }
  R->assign((size_t)p * p, cd(0.0, 0.0));
  for (int j = 0; j < p; ++j)
    for (int i = 0; i <= j; ++i) (*R)[i + (size_t)j * p] = W[i + (size_t)j * rows];
  // Q = H_0 ... H_{p-1} [I; 0]
  Q->assign((size_t)rows * p, cd(0.0, 0.0));
  for (int j = 0; j < p; ++j) (*Q)[j + (size_t)j * rows] = cd(1.0, 0.0);
  for (int k = p - 1; k >= 0; --k) {
    const std::vector<cd>& v = vs[k];
    for (int j = 0; j < p; ++j) {
      cd* x = Q->data() + (size_t)j * rows + k;
      cd d(0.0, 0.0);
      for (size_t i = 0; i < v.size(); ++i) d += std::conj(v[i]) * x[i];
      d *= taus[k];
      for (size_t i = 0; i < v.size(); ++i) x[i] -= d * v[i];
    }
  }
}

// Internal status (never returned through the ABI): the complex64 factors'
// refinement diverges (relative residual above 1 after the sweeps: kappa u_32
// beyond 1 for poles this close to the spectrum), so the query must be run
// again with FP64 factors.
constexpr int kNeedFP64 = 100;
bool refinement_diverged(const zolo_factors* F) { return F->precision == ZOLO_PREC_MIXED && F->refine_worst > 1.0; }

// State of a restarted multi-shift block GMRES run across its cycles
struct GmresRun {
  int total = 0, restarts = 0;
  double worst = 1.0;
  bool exhausted = false, done = false;
  std::vector<std::complex<double>> G0;  // per-shift right-hand sides of the next cycle (p x p each)
  // complex pencils restart the - shifts after the + shifts: their start block
  // (N x p), right-hand sides and residual while they wait
  DevArena mem;
  zd* pend_start = nullptr;
  std::vector<std::complex<double>> pend_G0;
  bool pending = false;
  double pend_worst = 0.0;
};

// One cycle of multi-shift block GMRES on blocks of scalar KT (the pencil's
// type in the first cycle, complex after a restart), then either the final
// minimal-residual updates or a collinear restart (see filter_apply_new).
template <typename VT, typename KT>
zolo_status gmres_cycle(zolo_factors* F, const VT* V, int64_t ldv, int p, VT* Y, int64_t ldy, double tol, int mr,
                        int maxit, bool first, const std::vector<double>& r0n, GmresRun& run, hipStream_t s) {
  using cd = std::complex<double>;
  constexpr bool same = std::is_same<VT, KT>::value;  // false: a real pencil on a complex basis
  DevArena rmem;  // this cycle's restart buffers
  rmem.set_stream(s);
  Workspace& ws = *F->ws;
  const int64_t n = F->P->n;
  const int64_t Mp = same ? ws.ldh : ws.ldh / 2;  // ld of the basis and rows of H, in KT
  const int ns = ws.nshift;
  KT *Vb = (KT*)ws.Vb, *W = (KT*)ws.W, *H = (KT*)ws.H, *hbuf = (KT*)ws.hbuf;
  ws.hls.p = p;
  ws.hls.ldr = (int64_t)(ws.mmax + 1) * p;
  if (first) {
    hls_init<KT>(ws.hls, (const KT*)ws.R0, s);
  } else {
    zd* g0 = nullptr;
    CHK(rmem.alloc(&g0, run.G0.size()));
    HIPC(hipMemcpyAsync(g0, run.G0.data(), sizeof(zd) * run.G0.size(), hipMemcpyHostToDevice, s));
    hls_init_multi(ws.hls, g0, s);
  }
  HIPC(hipMemsetAsync(H, 0, sizeof(KT) * Mp * (int64_t)mr * p, s));
  std::vector<double> res((size_t)ns * p), wq(ns, 0.0);
  bool bd = false;
  int m = 0;
  for (int k = 0; k < mr && run.total < maxit; ++k) {
    // inexact inner solves (mixed precision): the tolerance grows as the outer
    // residual falls, tol_refine / ||r_{k-1}|| capped at 1e-2
    const double tol_inner = std::min(1e-2, F->tol_refine / std::max(run.worst, 1e-300));
    if constexpr (same)
      CHK(apply_G_new<VT>(F, Vb + (int64_t)k * p, Mp, p, W, p, tol_inner, s));
    else  // G is real: the complex block is the real block of its 2p interleaved columns
      CHK(apply_G_new<double>(F, (const double*)(Vb + (int64_t)k * p), 2 * Mp, 2 * p, (double*)W, 2 * p, tol_inner,
                              s));
    if (refinement_diverged(F)) {
      set_error("complex64 factors: the refinement of the pole solves diverges (relative residual %.1e)",
                F->refine_worst);
      return (zolo_status)kNeedFP64;
    }
    const int kp1 = (k + 1) * p;
    for (int pass = 0; pass < 2; ++pass) {
      CHK(gemm_tn<KT>(ws, Vb, Mp, W, p, n, kp1, p, hbuf, kp1, false, s));
      CHK(gemm_nt_big<KT>(ws, W, p, W, p, 1.0, -1.0, hbuf, kp1, true, Vb, Mp, n, p, kp1, s));
      reduce_partials<KT>(H + (int64_t)k * p * Mp, Mp, hbuf, 1, kp1, p, true, s);
    }
    CHK(cholqr2<KT>(F, W, p, Vb + (int64_t)kp1, Mp, p, &bd, s));
    put_block<KT>(H, Mp, kp1, (int64_t)k * p, (const KT*)ws.Rk, p, s);
    {
      prof::Scope ps(ZOLO_PROF_HLS, 0.0, 0.0, s);
      hls_step<KT>(ws.hls, H, Mp, k, ws.res, s);
    }
    HIPC(hipMemcpyAsync(res.data(), ws.res, sizeof(double) * ns * p, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    HIPC(hipGetLastError());
    run.worst = 0.0;
    for (int q = 0; q < ns; ++q) {
      wq[q] = 0.0;
      for (int c = 0; c < p; ++c) wq[q] = std::max(wq[q], res[(size_t)q * p + c] / std::max(r0n[c], 1e-300));
      run.worst = std::max(run.worst, wq[q]);
    }
    m = k + 1;
    ++run.total;
    if (bd) run.exhausted = true;
    if (run.worst <= tol || run.exhausted) {
      run.done = true;
      break;
    }
  }
  const bool restart = !run.done && run.total < maxit;
  const int64_t rows = (int64_t)(m + 1) * p, mp = (int64_t)m * p;
  const HlsState& hs = ws.hls;
  // shift groups with a base each: one group, or at a complex pencil's first
  // restart the + shifts [0, r2) and the - shifts [r2, 2 r2), which continue
  // one after the other (a - shift's residual is not a multiple of a + shift's)
  const bool split = ST<VT>::cplx && restart && run.restarts == 0 && ns >= 2;
  const int ngroups = split ? 2 : 1;
  auto group_of = [&](int q) { return split && q >= ns / 2 ? 1 : 0; };
  zd* E[2] = {nullptr, nullptr};  // orthonormal bases Q_Z of the bases' residual blocks, rows x p
  int base[2] = {-1, -1};
  std::vector<cd> wsol, rz[2];
  if (restart) {
    ++run.restarts;
    for (int g = 0; g < ngroups; ++g) {
      double best = -1.0;
      for (int q = 0; q < ns; ++q)
        if (group_of(q) == g && wq[q] > best) {
          best = wq[q];
          base[g] = q;
        }
      if (g == 1) run.pend_worst = best;
    }
    // Z = Q_base [0; g_base(mp:(m+1)p, :)]: a base's residual block in the
    // basis; Z = Q_Z R_Z on the host (Householder: Q_Z orthonormal at any rank)
    zd *Z = nullptr, *T = nullptr, *Wd = nullptr;
    CHK(rmem.alloc(&Z, (size_t)rows * p));
    CHK(rmem.alloc(&T, (size_t)ns * rows * p));
    CHK(rmem.alloc(&Wd, (size_t)ns * p * p));
    for (int g = 0; g < ngroups; ++g) {
      CHK(rmem.alloc(&E[g], (size_t)rows * p));
      HIPC(hipMemsetAsync(Z, 0, sizeof(zd) * rows * p, s));
      HIPC(hipMemcpy2DAsync(Z + mp, sizeof(zd) * rows, hs.g + (int64_t)base[g] * hs.ldr * p + mp,
                            sizeof(zd) * hs.ldr, sizeof(zd) * p, p, hipMemcpyDeviceToDevice, s));
      hls_apply_q(hs, base[g], m, Z, rows, 0, p, false, s);
      std::vector<cd> zh((size_t)rows * p), qz;
      HIPC(hipMemcpyAsync(zh.data(), Z, sizeof(zd) * zh.size(), hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      householder_qr_host(zh, rows, p, &qz, &rz[g]);
      HIPC(hipMemcpyAsync(E[g], qz.data(), sizeof(zd) * qz.size(), hipMemcpyHostToDevice, s));
    }
    // T_s = Q_s^H Q_Z(group of s) for every shift; W_s = T_s,bot^-1 g_s,bot on
    // the host: shift s's residual becomes V_{m+1} Q_Z W_s (bases and shifts
    // with no right-hand side keep W_s = 0)
    for (int q = 0; q < ns; ++q)
      HIPC(hipMemcpyAsync(T + (int64_t)q * rows * p, E[group_of(q)], sizeof(zd) * rows * p, hipMemcpyDeviceToDevice,
                          s));
    hls_apply_q(hs, -1, m, T, rows, rows * p, p, true, s);
    std::vector<cd> tb((size_t)ns * p * p), gb((size_t)ns * p * p);
    for (int q = 0; q < ns; ++q) {
      HIPC(hipMemcpy2DAsync(tb.data() + (size_t)q * p * p, sizeof(zd) * p, T + (int64_t)q * rows * p + mp,
                            sizeof(zd) * rows, sizeof(zd) * p, p, hipMemcpyDeviceToHost, s));
      HIPC(hipMemcpy2DAsync(gb.data() + (size_t)q * p * p, sizeof(zd) * p, hs.g + (int64_t)q * hs.ldr * p + mp,
                            sizeof(zd) * hs.ldr, sizeof(zd) * p, p, hipMemcpyDeviceToHost, s));
    }
    HIPC(hipStreamSynchronize(s));
    wsol.assign((size_t)ns * p * p, cd(0.0, 0.0));
    for (int q = 0; q < ns; ++q) {
      if (q == base[0] || q == base[1]) continue;
      std::vector<cd> Wq(gb.begin() + (size_t)q * p * p, gb.begin() + (size_t)(q + 1) * p * p);
      bool any = false;
      for (const cd& x : Wq) any = any || x != cd(0.0, 0.0);
      if (!any) continue;
      std::vector<cd> Tq(tb.begin() + (size_t)q * p * p, tb.begin() + (size_t)(q + 1) * p * p);
      if (!dense_solve_host(Tq, Wq, p, p)) {
        set_error("block GMRES restart: singular collinearity system for shift %d", q);
        return ZOLO_EBREAKDOWN;
      }
      std::copy(Wq.begin(), Wq.end(), wsol.begin() + (size_t)q * p * p);
    }
    HIPC(hipMemcpyAsync(Wd, wsol.data(), sizeof(zd) * wsol.size(), hipMemcpyHostToDevice, s));
    hls_collinear_rhs(hs, m, T, rows * p, Wd, -1, s);
  }
  // the cycle's updates (after a restart: the base's minimal residual, the
  // others' collinear ones), Y = V/2 + V_m C or Y += V_m C
  hls_backsolve(hs, m, ws.Ys, s);
  if constexpr (same) {
    hls_combine(ws.Ys, m, p, ns, ws.coef, (VT*)ws.Cm, s);
    if (first)
      CHK(gemm_nt_big<VT>(ws, Y, ldy, V, ldv, 0.5, 1.0, (VT*)ws.Cm, mp, true, Vb, Mp, n, p, (int)mp, s));
    else
      CHK(gemm_nt_big<VT>(ws, Y, ldy, Y, ldy, 1.0, 1.0, (VT*)ws.Cm, mp, true, Vb, Mp, n, p, (int)mp, s));
  } else {
    // real pencil, complex basis: Y += Re(V_m C) = [Re V_m, Im V_m] [Re C; -Im C],
    // the interleaved real view of V_m times that of conj(C)
    hls_combine(ws.Ys, m, p, ns, ws.coef, (zd*)ws.Cm, s);
    conj_copy<zd>((zd*)ws.Cm, (const zd*)ws.Cm, mp * p, s);
    CHK(gemm_nt_big<double>(ws, (double*)Y, ldy, (const double*)Y, ldy, 1.0, 1.0, (const double*)ws.Cm, 2 * mp, true,
                            (const double*)Vb, 2 * Mp, n, p, (int)(2 * mp), s));
  }
  if (!restart) return ZOLO_OK;
  // next start block V_{m+1} Q_Z, orthonormal (complex; for a real pencil's
  // first cycle the real basis times the interleaved real columns of Q_Z); a
  // waiting group's start block is kept beside it
  zd* Bn = nullptr;
  CHK(rmem.alloc(&Bn, (size_t)n * p));
  if constexpr (std::is_same<KT, double>::value) {
    double* Er = nullptr;
    CHK(rmem.alloc(&Er, (size_t)rows * 2 * p));
    cols_re_im(E[0], rows, rows, p, Er, s);
    CHK(gemm_nt_big<double>(ws, (double*)Bn, 2 * p, nullptr, 0, 0.0, 1.0, Er, rows, true, Vb, Mp, n, 2 * p, (int)rows,
                            s));
  } else {
    CHK(gemm_nt_big<zd>(ws, Bn, p, nullptr, 0, 0.0, 1.0, E[0], rows, true, Vb, Mp, n, p, (int)rows, s));
    if (split) {
      CHK(run.mem.alloc(&run.pend_start, (size_t)n * p));
      CHK(gemm_nt_big<zd>(ws, run.pend_start, p, nullptr, 0, 0.0, 1.0, E[1], rows, true, Vb, Mp, n, p, (int)rows, s));
    }
  }
  // a real pencil's workspace grows to hold complex blocks (2p real columns)
  if (!ST<VT>::cplx && F->ws->p < 2 * p) CHK(ensure_ws(F, 2 * p, mr));
  Workspace& wn = *F->ws;
  const int64_t Mn = ST<VT>::cplx ? wn.ldh : wn.ldh / 2;
  HIPC(hipMemcpy2DAsync(wn.Vb, sizeof(zd) * Mn, Bn, sizeof(zd) * p, sizeof(zd) * p, n, hipMemcpyDeviceToDevice, s));
  // next right-hand sides: a base's residual is V_1' R_Z, shift s's V_1' W_s;
  // shifts of the other group get none
  run.G0.assign((size_t)ns * p * p, cd(0.0, 0.0));
  if (split) run.pend_G0.assign((size_t)ns * p * p, cd(0.0, 0.0));
  for (int q = 0; q < ns; ++q) {
    const int g = group_of(q);
    const cd* src = q == base[g] ? rz[g].data() : wsol.data() + (size_t)q * p * p;
    std::copy(src, src + (size_t)p * p, (g == 0 ? run.G0 : run.pend_G0).begin() + (size_t)q * p * p);
  }
  if (split) run.pending = true;
  HIPC(hipStreamSynchronize(s));
  return ZOLO_OK;
}

// Y (ld ldy) = R_ab(B^-1 A) V, everything in the new ordering: multi-shift
// block GMRES on G (eq. solve2, Corollary 1) over the outer shifts, every
// shift's least-squares problem on one shared block Krylov basis (shift
// invariance of the Krylov space), Y = V/2 + sum_s coef_s X_s.
//
// Restarts (every `restart` steps, 0 = none): after a cycle of m steps the
// shift with the largest residual (the base) takes its minimal-residual
// update, whose residual is V_{m+1} Z with Z = Q_base [0; g_base,bot].  Every
// other shift s takes the update that makes its residual a multiple of the
// same block: [H_s, Z] [y_s; W_s] = E1 S M_s, square, solved through shift
// s's own QR of H_s (T = Q_s^H Z; W_s = T_bot^-1 g_s,bot;
// y_s = R_s^-1 (g_s,top - T_top W_s)).  The next cycle starts from the
// orthonormalized block V_{m+1} Z = V1' S' and gives shift s the right-hand
// side E1 S' W_s, so all shifts still share one Krylov basis (collinear
// restarts of shifted GMRES, Frommer and Glaessner, 1998, in block form).
// The base residual of a real pencil is complex: its later cycles run on a
// complex basis (G applied to the 2p interleaved real columns), solving only
// the + shifts, Y += Re(V_m C).
template <typename VT>
zolo_status filter_apply_new(zolo_factors* F, const VT* V, int64_t ldv, int p, VT* Y, int64_t ldy, double tol,
                             int maxit, int restart, zolo_filter_stats* st, hipStream_t s) {
  const int mr = restart > 0 && restart < maxit ? restart : maxit;
  CHK(ensure_ws(F, p, mr));
  bool bd = false;
  {
    Workspace& ws = *F->ws;
    // V = V0 R0
    CHK(cholqr2<VT>(F, V, ldv, (VT*)ws.Vb, ws.ldh, p, &bd, s));
    if (bd) {
      set_error("filter: input block is rank deficient");
      return ZOLO_EBREAKDOWN;
    }
    HIPC(hipMemcpyAsync(ws.R0, ws.Rk, sizeof(VT) * p * p, hipMemcpyDeviceToDevice, s));
  }
  std::vector<VT> r0((size_t)p * p);
  std::vector<double> r0n(p, 0.0);
  HIPC(hipMemcpyAsync(r0.data(), F->ws->R0, sizeof(VT) * p * p, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  for (int c = 0; c < p; ++c)
    for (int i = 0; i <= c; ++i) r0n[c] += abs2(r0[i + c * p]);
  for (int c = 0; c < p; ++c) r0n[c] = std::sqrt(r0n[c]);
  GmresRun run;
  run.mem.set_stream(s);
  CHK((gmres_cycle<VT, VT>(F, V, ldv, p, Y, ldy, tol, mr, maxit, true, r0n, run, s)));
  while (run.total < maxit) {
    if (run.done) {
      if (!run.pending) break;
      // the + shifts have converged: the - shifts continue from their own block
      Workspace& ws = *F->ws;
      HIPC(hipMemcpy2DAsync(ws.Vb, sizeof(zd) * ws.ldh, run.pend_start, sizeof(zd) * p, sizeof(zd) * p, F->P->n,
                            hipMemcpyDeviceToDevice, s));
      run.G0.swap(run.pend_G0);
      run.pending = run.done = run.exhausted = false;
      run.worst = run.pend_worst;
    }
    CHK((gmres_cycle<VT, zd>(F, V, ldv, p, Y, ldy, tol, mr, maxit, false, r0n, run, s)));
  }
  if (run.pending) run.worst = std::max(run.worst, run.pend_worst);
  HIPC(hipStreamSynchronize(s));
  if (st) {
    st->n_gmres = run.total;
    st->worst_resid = run.worst;
    st->breakdown = run.exhausted ? 1 : 0;
    st->restarts = run.restarts;
  }
  if (run.worst > tol && !run.exhausted) {
    set_error("block GMRES reached %d steps (%d restarts) with relative residual %.3e > %.3e", run.total,
              run.restarts, run.worst, tol);
    return ZOLO_ENOCONV;
  }
  return ZOLO_OK;
}

// Y = R(B^-1 A) V for a one-stage filter (kind != 0): R = s0 + s1 g with g in
// the pole form of G (Zolo(r): (g + 1)/2; contour rules: g itself), one pole
// solve per pole, no outer Krylov stage.
template <typename VT>
zolo_status rational_apply_new(zolo_factors* F, const VT* V, int64_t ldv, int p, VT* Y, int64_t ldy, hipStream_t s) {
  CHK(ensure_ws(F, p, 1));
  CHK(apply_G_new<VT>(F, V, ldv, p, Y, ldy, F->tol_refine, s));
  if (refinement_diverged(F)) {
    set_error("complex64 factors: the refinement of the pole solves diverges (relative residual %.1e)",
              F->refine_worst);
    return (zolo_status)kNeedFP64;
  }
  if (F->co.kind == ZOLO_FILTER_ZOLO) axpby_rows<VT>(Y, ldy, V, ldv, 0.5, 0.5, F->P->n, p, s);
  return ZOLO_OK;
}

}  // namespace

// ===========================================================================
// ABI entry points on blocks in the original ordering
// ===========================================================================
namespace {
// the ABI block entry points, on blocks of the pencil's scalar type
template <typename VT>
zolo_status spmm_abi(zolo_pencil* P, int which, const VT* d_X, int64_t ldx, int ncols, VT* d_Y, int64_t ldy,
                     hipStream_t s) {
  DevArena tmp;
  tmp.set_stream(s);
  VT *xn = nullptr, *yn = nullptr;
  const int64_t n = P->n;
  CHK(tmp.alloc(&xn, n * ncols));
  CHK(tmp.alloc(&yn, n * ncols));
  rows_gather<VT>(xn, ncols, d_X, ldx, P->perm, n, ncols, s);
  if constexpr (ST<VT>::cplx)
    spmm_cplx(n, P->prow, P->pcol, which == 0 ? P->za : P->zb, nullptr, xn, ncols, ncols, yn, ncols, nullptr, 0, s);
  else
    spmm_real(n, P->prow, P->pcol, which == 0 ? P->pa : P->pb, nullptr, xn, ncols, ncols, yn, ncols, nullptr, 0, s);
  rows_scatter<VT>(d_Y, ldy, yn, ncols, P->perm, n, ncols, s);
  HIPC(hipStreamSynchronize(s));
  HIPC(hipGetLastError());
  return ZOLO_OK;
}

template <typename VT>
zolo_status pole_solve_abi(zolo_factors* F, int j, const VT* d_T, int64_t ldt, int ncols, zd* d_X, int64_t ldx,
                           hipStream_t s) {
  CHK(ensure_ws(F, ncols, F->ws ? std::max(F->ws->mmax, 1) : 1));
  const int64_t n = F->P->n;
  DevArena tmp;
  tmp.set_stream(s);
  VT* tn = nullptr;
  CHK(tmp.alloc(&tn, n * ncols));
  rows_gather<VT>(tn, ncols, d_T, ldt, F->P->perm, n, ncols, s);
  CHK(poles_solve_all<VT>(F, tn, ncols, F->ws->Xc, F->tol_refine, s));
  rows_scatter<zd>(d_X, ldx, F->ws->Xc + (int64_t)j * n * ncols, ncols, F->P->perm, n, ncols, s);
  HIPC(hipStreamSynchronize(s));
  HIPC(hipGetLastError());
  return ZOLO_OK;
}

template <typename VT>
zolo_status apply_G_abi(zolo_factors* F, const VT* d_V, int64_t ldv, int ncols, VT* d_W, int64_t ldw, hipStream_t s) {
  CHK(ensure_ws(F, ncols, F->ws ? std::max(F->ws->mmax, 1) : 1));
  const int64_t n = F->P->n;
  DevArena tmp;
  tmp.set_stream(s);
  VT *vn = nullptr, *wn = nullptr;
  CHK(tmp.alloc(&vn, n * ncols));
  CHK(tmp.alloc(&wn, n * ncols));
  rows_gather<VT>(vn, ncols, d_V, ldv, F->P->perm, n, ncols, s);
  CHK(apply_G_new<VT>(F, vn, ncols, ncols, wn, ncols, F->tol_refine, s));
  rows_scatter<VT>(d_W, ldw, wn, ncols, F->P->perm, n, ncols, s);
  HIPC(hipStreamSynchronize(s));
  HIPC(hipGetLastError());
  return ZOLO_OK;
}

template <typename VT>
zolo_status filter_apply_abi(zolo_factors* F, const VT* d_V, int64_t ldv, int ncols, VT* d_Y, int64_t ldy, double tol,
                             int maxit, int restart, zolo_filter_stats* st, hipStream_t s) {
  const int64_t n = F->P->n;
  DevArena tmp;
  tmp.set_stream(s);
  VT *vn = nullptr, *yn = nullptr;
  CHK(tmp.alloc(&vn, n * ncols));
  CHK(tmp.alloc(&yn, n * ncols));
  rows_gather<VT>(vn, ncols, d_V, ldv, F->P->perm, n, ncols, s);
  zolo_status rc = ZOLO_OK;
  if (F->co.kind == ZOLO_FILTER_HYBRID) {
    rc = filter_apply_new<VT>(F, vn, ncols, ncols, yn, ncols, tol, maxit, restart, st, s);
  } else {
    rc = rational_apply_new<VT>(F, vn, ncols, ncols, yn, ncols, s);
    if (st) *st = zolo_filter_stats{0, 0.0, 0, 0};
  }
  if (rc == kNeedFP64) return ZOLO_ENOCONV;  // the message says why; factor in FP64
  if (rc != ZOLO_OK && rc != ZOLO_ENOCONV) return rc;
  rows_scatter<VT>(d_Y, ldy, yn, ncols, F->P->perm, n, ncols, s);
  HIPC(hipStreamSynchronize(s));
  HIPC(hipGetLastError());
  return rc;
}
}  // namespace

extern "C" zolo_status zolo_spmm(zolo_pencil* P, int which, const void* d_X, int64_t ldx, int ncols, void* d_Y,
                                 int64_t ldy, void* stream) {
  if (!P || !d_X || !d_Y || ncols <= 0 || ldx < ncols || ldy < ncols || (which != 0 && which != 1)) {
    set_error("zolo_spmm: invalid argument");
    return ZOLO_EINVAL;
  }
  hipStream_t s = as_stream(stream);
  if (P->cplx()) return spmm_abi<zd>(P, which, (const zd*)d_X, ldx, ncols, (zd*)d_Y, ldy, s);
  return spmm_abi<double>(P, which, (const double*)d_X, ldx, ncols, (double*)d_Y, ldy, s);
}

namespace {
zolo_status residuals_check(const zolo_pencil* P, const void* d_X, int64_t ldx, int ncols, const double* d_lambda,
                            const double* d_out, const char* who) {
  if (!P || ncols < 0 || (ncols > 0 && (!d_X || !d_lambda || !d_out || ldx < ncols))) {
    set_error("%s: invalid argument", who);
    return ZOLO_EINVAL;
  }
  if (ncols > kResidMaxCols) {
    set_error("%s: %d columns exceed the limit of %d", who, ncols, kResidMaxCols);
    return ZOLO_EINVAL;
  }
  return ZOLO_OK;
}

zolo_status residuals_run(zolo_pencil* P, const void* d_X, int64_t ldx, int ncols, const double* d_lambda,
                          double* d_out, double* partial, hipStream_t s) {
  if (P->cplx())
    eig_resid_norms<zd>(P->n, P->prow, P->pcol, P->za, P->zb, P->perm, (const zd*)d_X, ldx, ncols, d_lambda,
                        P->normA, P->normB, partial, d_out, s);
  else
    eig_resid_norms<double>(P->n, P->prow, P->pcol, P->pa, P->pb, P->perm, (const double*)d_X, ldx, ncols, d_lambda,
                            P->normA, P->normB, partial, d_out, s);
  HIPC(hipGetLastError());
  return ZOLO_OK;
}
}  // namespace

extern "C" zolo_status zolo_residuals(zolo_pencil* P, const void* d_X, int64_t ldx, int ncols, const double* d_lambda,
                                      double* d_out, void* stream) {
  CHK(residuals_check(P, d_X, ldx, ncols, d_lambda, d_out, "zolo_residuals"));
  if (ncols == 0) return ZOLO_OK;
  hipStream_t s = as_stream(stream);
  DevArena tmp;  // released on return, ordered after this call's kernels on s
  tmp.set_stream(s);
  double* partial = nullptr;
  CHK(tmp.alloc(&partial, (size_t)kResidGroups * 2 * ncols));
  return residuals_run(P, d_X, ldx, ncols, d_lambda, d_out, partial, s);
}

extern "C" zolo_status zolo_residuals_noalloc(zolo_pencil* P, const void* d_X, int64_t ldx, int ncols,
                                              const double* d_lambda, double* d_out, void* stream) {
  CHK(residuals_check(P, d_X, ldx, ncols, d_lambda, d_out, "zolo_residuals_noalloc"));
  if (ncols == 0) return ZOLO_OK;
  const int dev = P->ctx->device;
  double* ptr = (dev >= 0 && dev < kMaxDevices) ? g_scratch_dev[dev] : nullptr;
  if (!ptr) {
    int cur = 0;
    HIPC(hipGetDevice(&cur));
    if (cur != dev) {
      set_error("zolo_residuals_noalloc: device %d is not current (and its scratch is not set up)", dev);
      return ZOLO_EDEVICE;
    }
    CHK(scratch_setup(dev));
    ptr = g_scratch_dev[dev];
  }
  // every workgroup overwrites its 2 * ncols partial sums, so nothing needs clearing
  return residuals_run(P, d_X, ldx, ncols, d_lambda, d_out, ptr, as_stream(stream));
}

extern "C" zolo_status zolo_pole_solve(zolo_factors* F, int j, const double* d_T, int64_t ldt, int ncols, void* d_X,
                                       int64_t ldx, void* stream) {
  const int nj = F ? F->co.r1 * (F->P->cplx() ? 2 : 1) : 0;
  if (!F || !d_T || !d_X || j < 0 || j >= nj || ncols <= 0 || ldt < ncols || ldx < ncols) {
    set_error("zolo_pole_solve: invalid argument");
    return ZOLO_EINVAL;
  }
  hipStream_t s = as_stream(stream);
  if (F->P->cplx()) return pole_solve_abi<zd>(F, j, (const zd*)d_T, ldt, ncols, (zd*)d_X, ldx, s);
  return pole_solve_abi<double>(F, j, d_T, ldt, ncols, (zd*)d_X, ldx, s);
}

extern "C" zolo_status zolo_apply_G(zolo_factors* F, const double* d_V, int64_t ldv, int ncols, double* d_W,
                                    int64_t ldw, void* stream) {
  if (!F || !d_V || !d_W || ncols <= 0 || ldv < ncols || ldw < ncols) {
    set_error("zolo_apply_G: invalid argument");
    return ZOLO_EINVAL;
  }
  hipStream_t s = as_stream(stream);
  if (F->P->cplx()) return apply_G_abi<zd>(F, (const zd*)d_V, ldv, ncols, (zd*)d_W, ldw, s);
  return apply_G_abi<double>(F, d_V, ldv, ncols, d_W, ldw, s);
}

extern "C" zolo_status zolo_filter_apply(zolo_factors* F, const double* d_V, int64_t ldv, int ncols, double* d_Y,
                                         int64_t ldy, double tol, int maxit, int restart, zolo_filter_stats* st,
                                         void* stream) {
  if (!F || !d_V || !d_Y || ncols <= 0 || ldv < ncols || ldy < ncols || restart < 0) {
    set_error("zolo_filter_apply: invalid argument");
    return ZOLO_EINVAL;
  }
  if (tol <= 0) tol = 1e-10;
  if (maxit <= 0) maxit = 60;
  hipStream_t s = as_stream(stream);
  if (F->P->cplx())
    return filter_apply_abi<zd>(F, (const zd*)d_V, ldv, ncols, (zd*)d_Y, ldy, tol, maxit, restart, st, s);
  return filter_apply_abi<double>(F, d_V, ldv, ncols, d_Y, ldy, tol, maxit, restart, st, s);
}

// ===========================================================================
// Algorithm 1
// ===========================================================================
namespace {
// Algorithm 1 on blocks of scalar VT (double: real pencils, zd: complex Hermitian pencils)
// Eigengaps when the caller gives none (Alg. 2, line 1; the paper leaves the
// estimate open).  Inertia counts nu(x) (eigenvalues below x) find
// eigenvalue-free intervals on each side of a and of b separately:
// (a - l, a) is free when nu(a - l) = nu(a), (a, a + u) when nu(a + u) = nu(a),
// and likewise at b.  Each half-width starts at half the mean eigenvalue
// spacing in (a, b) (from the count nu(b) - nu(a), taken first) and is halved
// (and counted again) while its side holds an eigenvalue, at most 10 times;
// all pending sides are counted together.  No
// eigenvalue below a - l makes a_- = -inf, none above b + u makes b_+ = +inf.
// Gaps narrower than the true ones are safe (the filter is planned on a wider
// transition band); they only raise the filter degree.
struct GapInfo {
  int64_t count = -1;  // eigenvalues in (a, b) by inertia, -1 if not computed
  double t_gaps = 0.0;
};

zolo_status estimate_gaps(zolo_ctx* ctx, zolo_pencil* P, double a, double b, int n_est, zolo_opts* o, GapInfo* gi,
                          hipStream_t s) {
  const double t0 = now_s();
  // the count in (a, b) first: it sets the mean spacing the searches start from
  int64_t nu_a = -1, nu_b = -1;
  {
    double ab[2] = {a, b};
    int64_t nu[2];
    CHK(zolo_inertia(ctx, P, ab, 2, nu, s));
    nu_a = nu[0];
    nu_b = nu[1];
  }
  const double spacing = (b - a) / (double)std::max<int64_t>(nu_b - nu_a, 1);
  (void)n_est;
  // sides: 0 = below a, 1 = above a, 2 = below b, 3 = above b
  double hw[4] = {0.5 * spacing, 0.5 * spacing, 0.5 * spacing, 0.5 * spacing};
  bool ok[4] = {false, false, false, false};
  int64_t nu_side[4] = {0, 0, 0, 0};
  for (int round = 0; round < 11 && !(ok[0] && ok[1] && ok[2] && ok[3]); ++round) {
    std::vector<double> sh;
    std::vector<int> who;
    for (int q = 0; q < 4; ++q)
      if (!ok[q]) {
        const double x = (q < 2 ? a : b) + (q % 2 ? hw[q] : -hw[q]);
        sh.push_back(x);
        who.push_back(q);
      }
    std::vector<int64_t> cnt(sh.size());
    CHK(zolo_inertia(ctx, P, sh.data(), (int)sh.size(), cnt.data(), s));
    for (size_t i = 0; i < sh.size(); ++i) {
      if (who[i] == -1) nu_a = cnt[i];
      if (who[i] == -2) nu_b = cnt[i];
    }
    for (size_t i = 0; i < sh.size(); ++i) {
      const int q = who[i];
      if (q < 0) continue;
      const int64_t ref = q < 2 ? nu_a : nu_b;
      if (cnt[i] == ref) {
        ok[q] = true;
        nu_side[q] = cnt[i];
      } else {
        hw[q] *= 0.5;
      }
    }
  }
  for (int q = 0; q < 4; ++q)
    if (!ok[q]) {
      set_error("eigengap estimate: an eigenvalue lies within %.3g of %s", hw[q], q < 2 ? "a" : "b");
      return ZOLO_EGAP;
    }
  o->a_minus = nu_side[0] == 0 ? -INFINITY : a - hw[0];
  o->a_plus = a + hw[1];
  o->b_minus = b - hw[2];
  o->b_plus = nu_side[3] == P->n ? INFINITY : b + hw[3];
  if (std::isinf(o->a_minus) && std::isinf(o->b_plus)) o->b_plus = b + hw[3];  // at most one infinite end
  gi->count = nu_b - nu_a;
  gi->t_gaps = now_s() - t0;
  return ZOLO_OK;
}

// r1 = 0 (Remark after Alg. 2 leaves the split open): the fewest inner poles
// (factorizations, at most 4) whose inner error delta_1 leaves the outer modulus
// l2 = (1 - delta_1)/(1 + delta_1) >= kMinL2.  Fewer poles are often faster on
// this GPU (a factorization and a pole solve of the block cost more than the
// extra block GMRES steps: grid7 64^3 window of 64, block 96, r1 = 1, 2, 3 take
// 9, 7, 7 steps and 0.24, 0.32, 0.44 s per query), but at l2 near 0.01 the step
// count can also run past the GMRES limit (complex 7 x 8 x 6 pencil sliced into
// windows of 40: 60 steps, residual 5e-2), so the automatic choice keeps the
// outer systems well separated.  At most as many poles as leave the free device
// memory (cached blocks counted as free) to the solves and the Krylov basis.
constexpr double kMinL2 = 0.2;
zolo_status choose_r1(const zolo_pencil* P, zolo_opts* o, int nss) {
  size_t free_b = 0, total_b = 0;
  int r_mem = 4;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    free_b += DevicePool::get().cached(dev);
    const int maxit = o->max_gmres_iter > 0 ? o->max_gmres_iter : 60;
    while (r_mem > 1 &&
           query_bytes_estimate(P, r_mem, nss, maxit, o->gmres_restart, o->precision, o->block_cols) >
               (int64_t)(0.9 * (double)free_b))
      --r_mem;
  }
  for (int r1 = 1; r1 <= r_mem; ++r1) {
    zolo_filter_coeffs co;
    CHK(zolo_filter_plan(o->a_minus, o->a_plus, o->b_minus, o->b_plus, r1, o->r2, o->filter_eps, &co));
    if (co.l2 >= kMinL2 || r1 == r_mem) {
      o->r1 = r1;
      return ZOLO_OK;
    }
  }
  return ZOLO_OK;
}

template <typename VT>
zolo_status solve_impl(zolo_ctx* ctx, zolo_pencil* P, double a, double b, int n_lambda_est, zolo_opts o,
                       const double* d_Q0, void* stream, zolo_result** out, const GapInfo& gi,
                       zolo_factors* F_in = nullptr, zolo_factors** F_keep = nullptr) {
  hipStream_t s = as_stream(stream);
  const double t_start = now_s() - gi.t_gaps;
  const int64_t n = P->n;
  // with an exact count from the inertia, the subspace follows it
  const int n_for_ss = gi.count >= 0 ? (int)gi.count : n_lambda_est;
  int nss = o.n_ss > 0 ? o.n_ss : (int)std::max<int64_t>((int64_t)std::ceil(1.5 * std::max(n_for_ss, 1)), n_for_ss + 8);
  nss = (int)std::min<int64_t>(nss, n);
  if (nss > 512) {
    set_error("zolo_solve: subspace size %d above 512", nss);
    return ZOLO_EINVAL;
  }
  std::unique_ptr<zolo_result> R(new zolo_result());
  R->n = n;
  R->ef = ST<VT>::cplx ? 2 : 1;
  zolo_stats& st = R->st;
  double t0 = now_s();
  zolo_filter_coeffs co;
  if (o.filter_kind == ZOLO_FILTER_HYBRID)
    CHK(zolo_filter_plan(o.a_minus, o.a_plus, o.b_minus, o.b_plus, o.r1, o.r2, o.filter_eps, &co));
  else
    CHK(zolo_filter_plan_kind(o.filter_kind, a, b, o.a_minus, o.a_plus, o.b_minus, o.b_plus, o.r1, o.filter_eps, &co));
  st.t_plan = now_s() - t0;
  st.t_gaps = gi.t_gaps;
  st.inertia_count = gi.count;
  st.a_minus = o.a_minus;
  st.a_plus = o.a_plus;
  st.b_minus = o.b_minus;
  st.b_plus = o.b_plus;
  st.t_symbolic = P->t_symbolic;
  st.r1 = co.r1;
  st.r2 = co.r2;
  st.l1 = co.l1;
  st.l2 = co.l2;
  st.delta0 = co.delta0;
  st.norm_a = P->normA;
  st.norm_b = P->normB;
  t0 = now_s();
  // resident factors of the same filter (serving) or a new factorization
  std::unique_ptr<zolo_factors> F_own;
  zolo_factors* Fu = F_in;
  if (Fu && (Fu->P != P || Fu->precision != o.precision || Fu->co.kind != co.kind || Fu->co.r1 != co.r1 ||
             Fu->co.r2 != co.r2 || Fu->co.sigma_hat_re[0] != co.sigma_hat_re[0] ||
             Fu->co.a_minus != co.a_minus || Fu->co.a_plus != co.a_plus || Fu->co.b_minus != co.b_minus ||
             Fu->co.b_plus != co.b_plus))
    Fu = nullptr;  // not this query's filter: factor anew
  if (!Fu) {
    zolo_factors* Fp = nullptr;
    CHK(zolo_factor(ctx, P, &co, o.precision, stream, &Fp));
    F_own.reset(Fp);
    Fu = Fp;
  } else {
    st.factors_reused = 1;
  }
  Fu->n_solv = Fu->n_refine = 0;
  Fu->refine_sweeps_max = Fu->refine_missed = 0;
  Fu->refine_worst = 0.0;
  struct Keep {
    std::unique_ptr<zolo_factors>& own;
    zolo_factors** keep;
    ~Keep() {
      if (keep && own) *keep = own.release();
    }
  } keep_guard{F_own, F_keep};
  zolo_factors* const F_ptr = Fu;
  struct FRef {
    zolo_factors* p;
    zolo_factors* get() const { return p; }
    zolo_factors* operator->() const { return p; }
  } F{F_ptr};
  F->max_refine = o.max_refine > 0 ? o.max_refine : 8;
  F->tol_refine = o.tol_refine > 0 ? o.tol_refine : 1e-8;
  st.t_factor = st.factors_reused ? 0.0 : now_s() - t0;
  st.factor_bytes = F->bytes;
  st.nnz_l = P->S.panel_entries + P->S.inv_entries;
  st.factor_flops = P->S.flops;
  const int maxit = o.max_gmres_iter > 0 ? o.max_gmres_iter : 60;
  const double tol_g = o.tol_gmres > 0 ? o.tol_gmres : 1e-10;
  // Column sub-blocks of the filter (block GMRES over pb columns at a time):
  // the filter acts column by column, so splitting the block changes only how
  // the Krylov spaces are shared, and the basis needs pb, not nss, columns.
  const int nsub = o.block_cols > 0 ? (nss + o.block_cols - 1) / o.block_cols : 1;
  const int pb = (nss + nsub - 1) / nsub;
  CHK(ensure_ws(F.get(), pb, o.gmres_restart > 0 && o.gmres_restart < maxit ? o.gmres_restart : maxit));
  // products of the Rayleigh-Ritz step: partial sums and descriptors only
  Workspace ws;
  ws.mem.set_stream(s);
  ws.ef = ST<VT>::cplx ? 2 : 1;
  ws.partial_len = std::max<int64_t>((int64_t)nss * nss * 256, 1 << 20);
  CHK(ws.mem.alloc(&ws.partial, ws.partial_len * (ST<VT>::cplx ? 2 : 1)));
  ws.gdesc_cap = 1024;
  {
    char* gd = nullptr;
    CHK(ws.mem.alloc(&gd, sizeof(GemmDesc<zd>) * (ws.gdesc_cap + 4)));
    ws.gdesc = gd;
  }
  // subspace buffers (new ordering)
  DevArena mem;
  mem.set_stream(s);
  VT *Q, *Y, *AY, *BY, *X, *AX, *BX, *At, *Bt, *Cm, *work, *Gx;
  double *theta, *rp, *rn;
  int* kdev;
  CHK(mem.alloc(&Q, n * nss));
  CHK(mem.alloc(&Y, n * nss));
  CHK(mem.alloc(&AY, n * nss));
  CHK(mem.alloc(&BY, n * nss));
  CHK(mem.alloc(&X, n * nss));
  CHK(mem.alloc(&AX, n * nss));
  CHK(mem.alloc(&BX, n * nss));
  CHK(mem.alloc(&At, (size_t)nss * nss));
  CHK(mem.alloc(&Bt, (size_t)nss * nss));
  CHK(mem.alloc(&Gx, (size_t)nss * nss));
  CHK(mem.alloc(&theta, nss));
  CHK(mem.alloc(&Cm, (size_t)nss * nss));
  CHK(mem.alloc(&work, (size_t)7 * nss * nss + 8 * nss + 64));  // 6 n^2 values + 2 n doubles + 2 n ints
  CHK(mem.alloc(&rp, (size_t)((n + 511) / 512) * 3 * nss + 16));
  CHK(mem.alloc(&rn, (size_t)3 * nss));
  CHK(mem.alloc(&kdev, 1));
  if (d_Q0) {
    rows_gather<VT>(Q, nss, (const VT*)d_Q0, nss, P->perm, n, nss, s);
  } else {
    // seeded Gaussian start block (complex pencils: independent real and imaginary
    // parts), drawn on the device into X as staging
    gaussian_fill(o.seed, (int64_t)n * nss * (ST<VT>::cplx ? 2 : 1), (double*)X, s);
    HIPC(hipGetLastError());
    rows_gather<VT>(Q, nss, X, nss, P->perm, n, nss, s);
  }
  t0 = now_s();
  std::vector<double> th(nss), rnh(3 * nss);
  std::vector<int> sel;
  int k = 0;
  int empty_runs = 0;
  bool converged = false;
  zolo_status frc = ZOLO_OK;
  for (int it = 1; it <= std::max(1, o.max_subspace_iter); ++it) {
    frc = ZOLO_OK;
    st.n_gmres_last = 0;
    st.gmres_resid = 0.0;
    for (int b0 = 0; b0 < nss; b0 += pb) {
      zolo_filter_stats fs{};
      const int pc = std::min(pb, nss - b0);
      zolo_status rc = ZOLO_OK;
      if (co.kind == ZOLO_FILTER_HYBRID)
        rc = filter_apply_new<VT>(F.get(), Q + b0, nss, pc, Y + b0, nss, tol_g, maxit, o.gmres_restart, &fs, s);
      else
        rc = rational_apply_new<VT>(F.get(), Q + b0, nss, pc, Y + b0, nss, s);
      if (rc != ZOLO_OK && rc != ZOLO_ENOCONV) return rc;
      if (rc == ZOLO_ENOCONV) frc = rc;
      st.n_gmres_total += fs.n_gmres;
      st.n_gmres_last = std::max(st.n_gmres_last, fs.n_gmres);
      st.gmres_resid = std::max(st.gmres_resid, fs.worst_resid);
      st.n_restart += fs.restarts;
    }
    st.n_iter = it;
    // Rayleigh-Ritz
    {
      prof::Scope ps(ZOLO_PROF_SPMM, 4.0 * P->nnz * nss * (ST<VT>::cplx ? 4 : 1),
                     (ST<VT>::cplx ? 36.0 : 20.0) * P->nnz + 8.0 * (n + 1) + 3.0 * sizeof(VT) * n * nss, s);
      if constexpr (ST<VT>::cplx)
        spmm_cplx(n, P->prow, P->pcol, P->za, P->zb, Y, nss, nss, AY, nss, BY, nss, s);
      else
        spmm_real(n, P->prow, P->pcol, P->pa, P->pb, Y, nss, nss, AY, nss, BY, nss, s);
    }
    CHK(gemm_tn<VT>(ws, Y, nss, AY, nss, n, nss, nss, At, nss, false, s));
    CHK(gemm_tn<VT>(ws, Y, nss, BY, nss, n, nss, nss, Bt, nss, false, s));
    {
      prof::Scope ps(ZOLO_PROF_RR, 0.0, 0.0, s);
      rr_reduce<VT>(At, Bt, nss, 1e-12, theta, Cm, kdev, work, s);
    }
    HIPC(hipMemcpyAsync(&k, kdev, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    HIPC(hipGetLastError());
    if (k < 0) {
      set_error("Rayleigh-Ritz: a Hermitian eigensolve did not converge");
      return ZOLO_EBREAKDOWN;
    }
    if (k == 0) {
      set_error("Rayleigh-Ritz: filtered block has rank 0");
      return ZOLO_EBREAKDOWN;
    }
    // X = Y C, AX = AY C, BX = BY C  (row-major N x k)
    CHK(gemm_nt_big<VT>(ws, X, k, nullptr, 0, 0.0, 1.0, Cm, nss, true, Y, nss, n, k, nss, s));
    CHK(gemm_nt_big<VT>(ws, AX, k, nullptr, 0, 0.0, 1.0, Cm, nss, true, AY, nss, n, k, nss, s));
    CHK(gemm_nt_big<VT>(ws, BX, k, nullptr, 0, 0.0, 1.0, Cm, nss, true, BY, nss, n, k, nss, s));
    resid_norms<VT>(AX, BX, X, theta, n, k, rp, rn, s);
    HIPC(hipMemcpyAsync(th.data(), theta, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(rnh.data(), rn, sizeof(double) * 3 * k, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    sel.clear();
    double worst = 0.0;
    for (int c = 0; c < k; ++c) {
      if (!(th[c] > a && th[c] < b)) continue;
      sel.push_back(c);
      double r = std::sqrt(rnh[3 * c]) / ((P->normA + std::fabs(th[c]) * P->normB) * std::sqrt(rnh[3 * c + 1]));
      worst = std::max(worst, r);
    }
    st.max_resid = worst;
    // next block: Ritz vectors, padded with the previous block's columns
    HIPC(hipMemcpy2DAsync(Q, sizeof(VT) * nss, X, sizeof(VT) * k, sizeof(VT) * k, n, hipMemcpyDeviceToDevice, s));
    if (!sel.empty() && worst <= o.tol_resid) {
      converged = true;
      break;
    }
    // An interval with no eigenvalue: after two filtered iterations any
    // eigenvector inside (a, b) present in the start block would dominate the
    // subspace, so two empty selections in a row mean the count is zero.
    if (sel.empty()) {
      if (++empty_runs >= 2) {
        converged = true;
        break;
      }
    } else {
      empty_runs = 0;
    }
  }
  // Ritz values that have converged inside a stated eigengap (a_-, a_+) or
  // (b_-, b_+), away from its ends, contradict the caller's gaps
  int in_gap = 0;
  double gap_theta = 0.0;
  if (converged) {
    const double gl[2] = {o.a_minus, o.b_minus}, gh[2] = {o.a_plus, o.b_plus};
    for (int c = 0; c < k; ++c) {
      const double r = std::sqrt(rnh[3 * c]) / ((P->normA + std::fabs(th[c]) * P->normB) * std::sqrt(rnh[3 * c + 1]));
      if (!(r <= o.tol_resid)) continue;
      for (int g = 0; g < 2; ++g) {
        double m = 1e-9 * std::max({1.0, std::fabs(th[c]), std::isfinite(gl[g]) ? std::fabs(gl[g]) : 0.0,
                                     std::isfinite(gh[g]) ? std::fabs(gh[g]) : 0.0});
        if (th[c] > gl[g] + m && th[c] < gh[g] - m) {
          ++in_gap;
          gap_theta = th[c];
        }
      }
    }
  }
  st.t_iter = now_s() - t0;
  st.n_solv = F->n_solv;
  st.n_refine = F->n_refine;
  st.refine_sweeps_max = F->refine_sweeps_max;
  st.refine_missed = F->refine_missed;
  st.refine_worst = F->refine_worst;
  // results: selected pairs, original ordering
  const int cnt = (int)sel.size();
  R->count = cnt;
  R->eig.resize(cnt);
  double emax = 0.0;
  for (int i = 0; i < cnt; ++i) {
    int c = sel[i];
    R->eig[i] = th[c];
    emax = std::max(emax, std::sqrt(rnh[3 * c]) / (std::max(std::fabs(a), std::fabs(b)) * std::sqrt(rnh[3 * c + 2])));
  }
  st.e_lambda_x = emax;
  st.n_found = cnt;
  if (cnt > 0) {
    VT* vec = nullptr;
    CHK(R->mem.alloc(&vec, n * cnt));
    R->vec = (double*)vec;
    VT* tmpv = nullptr;
    CHK(mem.alloc(&tmpv, n * cnt));
    int c0 = sel[0];
    // selected Ritz values are consecutive in the ascending order
    HIPC(hipMemcpy2DAsync(tmpv, sizeof(VT) * cnt, X + c0, sizeof(VT) * k, sizeof(VT) * cnt, n, hipMemcpyDeviceToDevice,
                          s));
    rows_scatter<VT>(vec, cnt, tmpv, cnt, P->perm, n, cnt, s);
    // B-orthonormality of the returned vectors: X^H B X - I
    if constexpr (ST<VT>::cplx)
      spmm_cplx(n, P->prow, P->pcol, P->zb, nullptr, tmpv, cnt, cnt, AX, cnt, nullptr, 0, s);
    else
      spmm_real(n, P->prow, P->pcol, P->pb, nullptr, tmpv, cnt, cnt, AX, cnt, nullptr, 0, s);
    CHK(gemm_tn<VT>(ws, tmpv, cnt, AX, cnt, n, cnt, cnt, Gx, cnt, false, s));
    std::vector<VT> gx((size_t)cnt * cnt);
    HIPC(hipMemcpyAsync(gx.data(), Gx, sizeof(VT) * cnt * cnt, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    double bo = 0.0;
    for (int i = 0; i < cnt; ++i)
      for (int j2 = 0; j2 < cnt; ++j2)
        bo = std::max(bo, std::sqrt(abs2(sub(gx[i + (size_t)j2 * cnt], cvt<VT, double>(i == j2 ? 1.0 : 0.0)))));
    st.b_orth = bo;
  }
  st.t_total = now_s() - t_start;
  *out = R.release();
  // A subspace (nearly) filled by converged pairs cannot tell whether more lie
  // in (a, b): then the inertia count decides (computed here when the caller
  // gave the eigengaps).
  if (cnt >= nss - 1) {
    int64_t count = gi.count;
    if (count < 0) {
      double ab[2] = {a, b};
      int64_t nu[2];
      CHK(zolo_inertia(ctx, P, ab, 2, nu, stream));
      count = nu[1] - nu[0];
      (*out)->st.inertia_count = count;
    }
    if (count != cnt) {
      set_error("found %d eigenpairs with a subspace of %d, inertia counts %lld: estimate too small", cnt, nss,
                (long long)count);
      return ZOLO_ESUBSPACE;
    }
  }
  if (!converged) {
    set_error("subspace iteration did not reach tol_resid (worst %.3e)", st.max_resid);
    return ZOLO_ENOCONV;
  }
  if (in_gap) {
    set_error("%d converged Ritz value(s) inside a stated eigengap (e.g. %.15g): the eigengaps are wrong", in_gap,
              gap_theta);
    return ZOLO_EGAP;
  }
  return frc == ZOLO_ENOCONV ? ZOLO_ENOCONV : ZOLO_OK;
}
}  // namespace

namespace zolo {
zolo_status solve_resident(zolo_ctx* ctx, zolo_pencil* P, double a, double b, int n_lambda_est,
                           const zolo_opts* opts_in, const double* d_Q0, void* stream, zolo_factors* F_in,
                           zolo_factors** F_keep, zolo_result** out) {
  if (!ctx || !P || !out || !(a < b) || n_lambda_est < 0) {
    set_error("zolo_solve: invalid argument");
    return ZOLO_EINVAL;
  }
  zolo_opts o;
  if (opts_in)
    o = *opts_in;
  else
    zolo_opts_default(&o);
  if (o.filter_kind < ZOLO_FILTER_HYBRID || o.filter_kind > ZOLO_FILTER_GAUSS) {
    set_error("zolo_solve: unknown filter kind %d", o.filter_kind);
    return ZOLO_EINVAL;
  }
  HIPC(hipSetDevice(ctx->device));
  GapInfo gi;
  if (o.filter_kind == ZOLO_FILTER_TRAPEZOID || o.filter_kind == ZOLO_FILTER_GAUSS) {
    // contour rules need no eigengaps; the count sizes the subspace when the
    // caller gives no estimate
    if (o.r1 == 0) o.r1 = 8;
    if (n_lambda_est == 0 && o.n_ss <= 0) {
      double ab[2] = {a, b};
      int64_t nu[2];
      CHK(zolo_inertia(ctx, P, ab, 2, nu, stream));
      gi.count = nu[1] - nu[0];
    }
    if (P->cplx()) return solve_impl<zd>(ctx, P, a, b, n_lambda_est, o, d_Q0, stream, out, gi, F_in, F_keep);
    return solve_impl<double>(ctx, P, a, b, n_lambda_est, o, d_Q0, stream, out, gi, F_in, F_keep);
  }
  const int n_nan = std::isnan(o.a_minus) + std::isnan(o.a_plus) + std::isnan(o.b_minus) + std::isnan(o.b_plus);
  if (n_nan != 0 && n_nan != 4) {
    set_error("zolo_solve: give all four eigengap ends, or none (NaN) to have them estimated");
    return ZOLO_EINVAL;
  }
  if (n_nan == 4) CHK(estimate_gaps(ctx, P, a, b, n_lambda_est, &o, &gi, as_stream(stream)));
  if (!(o.a_minus < a && a < o.a_plus && o.b_minus < b && b < o.b_plus)) {
    set_error("zolo_solve: need a in (a_minus, a_plus) and b in (b_minus, b_plus)");
    return ZOLO_EINVAL;
  }
  if (o.r1 == 0 && o.filter_kind == ZOLO_FILTER_ZOLO) o.r1 = 4;
  if (o.r1 == 0) {
    const int n_for_ss = gi.count >= 0 ? (int)gi.count : n_lambda_est;
    const int nss = o.n_ss > 0 ? o.n_ss : (int)std::max<int64_t>((int64_t)std::ceil(1.5 * std::max(n_for_ss, 1)), n_for_ss + 8);
    CHK(choose_r1(P, &o, (int)std::min<int64_t>(nss, P->n)));
  }
  auto run = [&](zolo_factors* fin) {
    return P->cplx() ? solve_impl<zd>(ctx, P, a, b, n_lambda_est, o, d_Q0, stream, out, gi, fin, F_keep)
                     : solve_impl<double>(ctx, P, a, b, n_lambda_est, o, d_Q0, stream, out, gi, fin, F_keep);
  };
  zolo_status rc = run(F_in);
  if ((int)rc == kNeedFP64) {
    // complex64 factors useless for these poles: the same query with FP64 factors
    if (F_keep && *F_keep) {
      zolo_factors_free(*F_keep);
      *F_keep = nullptr;
    }
    o.precision = ZOLO_PREC_FP64;
    rc = run(nullptr);
    if (*out) (*out)->st.precision_fallback = 1;
  }
  return rc;
}

const zolo_filter_coeffs* factors_coeffs(const zolo_factors* F) { return &F->co; }
void set_inertia_cap(int shifts) { g_inertia_cap = shifts; }
void factors_keep_only(zolo_factors* F) {
  F->ws.reset();
  F->prog_d.clear();
  F->prog_f.clear();
}
int64_t inertia_shift_bytes(const zolo_pencil* P) {
  const int64_t lu = P->cplx() ? 2 : 1;
  return (int64_t)(P->cplx() ? sizeof(zd) : sizeof(double)) *
         (lu * (P->panel_total + P->inv_total + P->n) + P->upd_total + lu * (P->inv_scratch + P->conv_scratch));
}
int64_t factors_bytes(const zolo_factors* F) { return F->bytes; }
}  // namespace zolo

extern "C" zolo_status zolo_solve(zolo_ctx* ctx, zolo_pencil* P, double a, double b, int n_lambda_est,
                                  const zolo_opts* opts_in, const double* d_Q0, void* stream, zolo_result** out) {
  return zolo::solve_resident(ctx, P, a, b, n_lambda_est, opts_in, d_Q0, stream, nullptr, nullptr, out);
}

// Spectrum slicing (Sec. 1: the eigenpairs of a long interval, computed as
// many adjacent intervals, each its own filter; independent, so the natural
// unit of parallel work): (lo, hi) is cut into n_slices slices of equal width
// whose inner ends are moved off eigenvalues (an inner end x is kept when
// (x - d, x + d) holds no eigenvalue by inertia, d a tenth of the mean spacing;
// else it moves by a third of the spacing, up to 8 tries), every slice is one
// zolo_solve with its eigengaps and count estimated by inertia, all sharing the
// pencil's ordering and symbolic analysis, and the results are joined in
// ascending order.
extern "C" zolo_status zolo_slice(zolo_ctx* ctx, zolo_pencil* P, double lo, double hi, int n_slices,
                                  const zolo_opts* opts_in, void* stream, zolo_result** out) {
  if (!ctx || !P || !out || !(lo < hi) || n_slices < 1 || n_slices > 4096) {
    set_error("zolo_slice: invalid argument");
    return ZOLO_EINVAL;
  }
  HIPC(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  zolo_opts base;
  if (opts_in)
    base = *opts_in;
  else
    zolo_opts_default(&base);
  base.a_minus = base.a_plus = base.b_minus = base.b_plus = NAN;
  base.n_ss = 0;
  int64_t ends[2];
  double lh[2] = {lo, hi};
  CHK(zolo_inertia(ctx, P, lh, 2, ends, stream));
  const int64_t total = ends[1] - ends[0];
  const double spacing = (hi - lo) / (double)std::max<int64_t>(total, 1);
  std::vector<double> x(n_slices + 1);
  for (int k = 0; k <= n_slices; ++k) x[k] = lo + (hi - lo) * k / n_slices;
  x[n_slices] = hi;
  // inner ends off the eigenvalues
  std::vector<int> pending;
  for (int k = 1; k < n_slices; ++k) pending.push_back(k);
  const double d = 0.1 * spacing;
  for (int attempt = 0; attempt < 8 && !pending.empty(); ++attempt) {
    std::vector<double> sh;
    for (int k : pending) {
      sh.push_back(x[k] - d);
      sh.push_back(x[k] + d);
    }
    std::vector<int64_t> c(sh.size());
    for (size_t q0 = 0; q0 < sh.size(); q0 += ZOLO_MAX_R) {
      const int nq = (int)std::min<size_t>(ZOLO_MAX_R, sh.size() - q0);
      CHK(zolo_inertia(ctx, P, sh.data() + q0, nq, c.data() + q0, stream));
    }
    std::vector<int> still;
    for (size_t i = 0; i < pending.size(); ++i)
      if (c[2 * i] != c[2 * i + 1]) {
        const int k = pending[i];
        x[k] += (attempt % 2 ? -1.0 : 1.0) * (attempt + 1) * spacing / 3.0;
        still.push_back(k);
      }
    pending.swap(still);
  }
  for (int k = 1; k <= n_slices; ++k)
    if (!(x[k] > x[k - 1]) || (k < n_slices && !(x[k] < hi))) {
      set_error("zolo_slice: slices too narrow for the eigenvalue spacing (use fewer slices)");
      return ZOLO_EINVAL;
    }
  if (!pending.empty()) {
    set_error("zolo_slice: could not place a slice end away from the eigenvalues");
    return ZOLO_EGAP;
  }
  std::unique_ptr<zolo_result> R(new zolo_result());
  R->n = P->n;
  R->ef = P->cplx() ? 2 : 1;
  std::vector<std::unique_ptr<zolo_result>> parts;
  zolo_status worst_rc = ZOLO_OK;
  zolo_stats& st = R->st;
  const double t0 = now_s();
  for (int k = 0; k < n_slices; ++k) {
    double xx[2] = {x[k], x[k + 1]};
    int64_t cc[2];
    CHK(zolo_inertia(ctx, P, xx, 2, cc, stream));
    if (cc[1] == cc[0]) continue;  // an empty slice
    zolo_result* r = nullptr;
    zolo_status rc = zolo_solve(ctx, P, x[k], x[k + 1], (int)(cc[1] - cc[0]), &base, nullptr, stream, &r);
    if (!r) return rc;
    if (rc != ZOLO_OK) worst_rc = rc;
    st.n_iter = std::max(st.n_iter, r->st.n_iter);
    st.n_gmres_total += r->st.n_gmres_total;
    st.n_solv += r->st.n_solv;
    st.n_refine += r->st.n_refine;
    st.max_resid = std::max(st.max_resid, r->st.max_resid);
    st.e_lambda_x = std::max(st.e_lambda_x, r->st.e_lambda_x);
    st.b_orth = std::max(st.b_orth, r->st.b_orth);
    st.t_factor += r->st.t_factor;
    st.t_iter += r->st.t_iter;
    st.t_gaps += r->st.t_gaps;
    st.r1 = std::max(st.r1, r->st.r1);
    st.r2 = std::max(st.r2, r->st.r2);
    R->count += r->count;
    parts.emplace_back(r);
  }
  st.inertia_count = total;
  st.n_found = (int)R->count;
  st.norm_a = P->normA;
  st.norm_b = P->normB;
  st.t_symbolic = P->t_symbolic;
  if (R->count > 0) {
    CHK(R->mem.alloc(&R->vec, (size_t)P->n * R->count * R->ef));
    const size_t e = sizeof(double) * R->ef;
    int64_t c0 = 0;
    for (auto& r : parts) {
      if (r->count == 0) continue;
      HIPC(hipMemcpy2DAsync(R->vec + c0 * R->ef, e * R->count, r->vec, e * r->count, e * r->count, P->n,
                            hipMemcpyDeviceToDevice, s));
      R->eig.insert(R->eig.end(), r->eig.begin(), r->eig.end());
      c0 += r->count;
    }
    HIPC(hipStreamSynchronize(s));
  }
  st.t_total = now_s() - t0;
  *out = R.release();
  if (worst_rc != ZOLO_OK) return worst_rc;
  if ((*out)->count != total) {
    set_error("zolo_slice: found %lld eigenpairs, inertia counts %lld", (long long)(*out)->count, (long long)total);
    return ZOLO_ENOCONV;
  }
  return ZOLO_OK;
}

extern "C" zolo_status zolo_profile_enable(int on) {
  prof::reset();
  prof::on = on != 0;
  return ZOLO_OK;
}

extern "C" zolo_status zolo_profile_query(int cls, zolo_kernel_profile* out) {
  if (!out || cls < 0 || cls >= ZOLO_PROF_COUNT) {
    set_error("zolo_profile_query: invalid argument");
    return ZOLO_EINVAL;
  }
  prof::resolve();
  out->launches = prof::cnt[cls];
  out->ms = prof::ms[cls];
  out->flops = prof::fl[cls];
  out->bytes = prof::by[cls];
  return ZOLO_OK;
}

extern "C" int64_t zolo_result_count(const zolo_result* r) { return r ? r->count : 0; }
extern "C" const double* zolo_result_eigenvalues(const zolo_result* r) { return r ? r->eig.data() : nullptr; }
extern "C" zolo_status zolo_result_copy_vectors(const zolo_result* r, void* d_dst, int64_t ld, void* stream) {
  if (!r || !d_dst || ld < r->count) {
    set_error("zolo_result_copy_vectors: invalid argument");
    return ZOLO_EINVAL;
  }
  if (r->count == 0) return ZOLO_OK;
  hipStream_t s = as_stream(stream);
  const size_t e = sizeof(double) * r->ef;
  HIPC(hipMemcpy2DAsync(d_dst, e * ld, r->vec, e * r->count, e * r->count, r->n, hipMemcpyDeviceToDevice, s));
  HIPC(hipStreamSynchronize(s));
  return ZOLO_OK;
}
extern "C" zolo_status zolo_result_copy_vectors_host(const zolo_result* r, void* h_dst, int64_t ld) {
  if (!r || !h_dst || ld < r->count) {
    set_error("zolo_result_copy_vectors_host: invalid argument");
    return ZOLO_EINVAL;
  }
  if (r->count == 0) return ZOLO_OK;
  const size_t e = sizeof(double) * r->ef;
  HIPC(hipMemcpy2D(h_dst, e * ld, r->vec, e * r->count, e * r->count, r->n, hipMemcpyDeviceToHost));
  return ZOLO_OK;
}
extern "C" const void* zolo_result_device_vectors(const zolo_result* r, int64_t* ld) {
  if (ld) *ld = r ? r->count : 0;
  return (r && r->count > 0) ? (const void*)r->vec : nullptr;
}
extern "C" zolo_status zolo_result_stats(const zolo_result* r, zolo_stats* out) {
  if (!r || !out) {
    set_error("null argument");
    return ZOLO_EINVAL;
  }
  *out = r->st;
  return ZOLO_OK;
}
extern "C" void zolo_result_free(zolo_result* r) { delete r; }

// ===========================================================================
// internal helpers for the serving loop (serve.cpp)
// ===========================================================================
namespace zolo {

int64_t query_bytes_estimate(const zolo_pencil* P, int r1, int nss, int maxit, int restart, int precision,
                             int block_cols) {
  const int64_t n = P->n;
  const int64_t elem = precision == ZOLO_PREC_FP64 ? 16 : 8;
  const int64_t lu = P->cplx() ? 2 : 1;  // LU: two panels and inverses; K^-1 and K^-H solves
  const int64_t vb = P->cplx() ? 16 : 8;  // bytes per block entry
  const int64_t factors = (int64_t)r1 * lu * (P->panel_total + P->inv_total + n) * elem;
  const int64_t factor_tmp = (int64_t)r1 * (P->upd_total + lu * (P->inv_scratch + P->conv_scratch)) * elem;
  // the filter runs on column sub-blocks of p columns; the basis holds mmax
  // blocks, and a restarted real pencil continues on 2p columns (with a
  // second solve program)
  const int64_t nsub = block_cols > 0 ? (nss + block_cols - 1) / block_cols : 1;
  const int64_t p = (nss + nsub - 1) / nsub;
  const bool restarts = restart > 0 && restart < maxit;
  const int64_t mmax = restarts ? restart : maxit;
  const int64_t pk = restarts && !P->cplx() ? 2 * p : p;
  const int64_t solve = (int64_t)r1 * lu * (6 * n * (p + (pk > p ? pk : 0))) * elem;  // W, U, Xb, t, Y, X
  const int64_t krylov = ((mmax + 2) * n * pk + 3 * n * pk) * vb                      // basis, W, T1, Tb
                         + 2 * (int64_t)r1 * lu * n * pk * 16                         // pole solutions, residuals
                         + (int64_t)2048 * 64 * 96 * vb;                              // Gram partial sums
  const int64_t subspace = 8 * n * (int64_t)nss * vb;  // Q, Y, AY, BY, X, AX, BX, result
  const int64_t total = factors + std::max(factor_tmp, solve + krylov) + subspace;
  return total + total / 10 + ((int64_t)64 << 20);
}

int64_t pencil_n(const zolo_pencil* P) { return P->n; }
bool pencil_cplx(const zolo_pencil* P) { return P->cplx(); }

zolo_result* result_clone(const zolo_result* r) {
  std::unique_ptr<zolo_result> c(new zolo_result());
  c->n = r->n;
  c->count = r->count;
  c->ef = r->ef;
  c->eig = r->eig;
  c->st = r->st;
  if (r->count > 0) {
    if (c->mem.alloc(&c->vec, r->n * r->count * r->ef) != ZOLO_OK) return nullptr;
    if (hipMemcpy(c->vec, r->vec, sizeof(double) * r->n * r->count * r->ef, hipMemcpyDeviceToDevice) != hipSuccess)
      return nullptr;
  }
  return c.release();
}

int64_t result_bytes(const zolo_result* r) { return (int64_t)sizeof(double) * r->n * r->count * r->ef; }

zolo_status result_verify(zolo_pencil* P, const zolo_result* r, void* stream, double* worst) {
  *worst = 0.0;
  if (r->count == 0) return ZOLO_OK;
  hipStream_t s = as_stream(stream);
  DevArena tmp;
  tmp.set_stream(s);
  double *dl = nullptr, *dout = nullptr;
  CHK(tmp.alloc(&dl, r->count));
  CHK(tmp.alloc(&dout, r->count));
  HIPC(hipMemcpyAsync(dl, r->eig.data(), sizeof(double) * r->count, hipMemcpyHostToDevice, s));
  for (int64_t c0 = 0; c0 < r->count; c0 += 512)  // the residual call's column limit
    CHK(zolo_residuals(P, r->vec + c0 * r->ef, r->count, (int)std::min<int64_t>(512, r->count - c0), dl + c0,
                       dout + c0, s));
  std::vector<double> h(r->count);
  HIPC(hipMemcpyAsync(h.data(), dout, sizeof(double) * r->count, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  for (double x : h) *worst = std::max(*worst, x);
  return ZOLO_OK;
}

void result_mark_reused(zolo_result* r, double max_resid, double t_check) {
  r->st.subspace_reused = 1;
  r->st.max_resid = max_resid;
  r->st.t_total = t_check;
}

void register_stream(void* s) {
  std::lock_guard<std::mutex> lk(g_streams_m);
  g_owned_streams.insert((hipStream_t)s);
}

void retire_stream(void* s) {
  (void)hipStreamSynchronize((hipStream_t)s);
  {
    std::lock_guard<std::mutex> lk(g_streams_m);
    g_owned_streams.erase((hipStream_t)s);
  }
  DevicePool::get().drop_marks((hipStream_t)s);
}

void gaussian_device(uint64_t seed, int64_t n, double* d_out, void* stream) {
  gaussian_fill(seed, n, d_out, as_stream(stream));
}

}  // namespace zolo
