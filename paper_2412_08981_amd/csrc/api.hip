// Driver and C ABI of the nnms library: device upload of a hierarchy,
// numeric setup per parameter (assembly, extraction, batched LU), batched
// solve plans (descriptor tables, triangular-solve task order, a HIP graph
// of one Arnoldi step) and the single-operation entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "devtypes.h"
#include "kernels.h"
#include "nnms_internal.h"

namespace nnms {

static thread_local std::string g_last_error;
void set_last_error(const std::string& m) { g_last_error = m; }
static std::atomic<int64_t> g_bytes{0};

#define HIP_CHECK(x)                                                                                 \
  do {                                                                                               \
    hipError_t e_ = (x);                                                                             \
    if (e_ != hipSuccess) throw Error(NNMS_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// device memory: the caller's allocator or hipMalloc; freed together
// ---------------------------------------------------------------------------

// Batch plans own only small buffers (descriptors, task lists, counters).
// They are recycled per device and power-of-two size class instead of
// freed, because hipFree waits for the whole device: dropping a plan would
// otherwise wait for unrelated work on other streams (the factorisation of
// a newly admitted request in the serving loop).  At most kDevCacheCap
// bytes are kept; buffers beyond that are freed.
static constexpr size_t kDevCacheCap = size_t(64) << 20;
struct DevCache {
  std::mutex mu;
  std::map<std::pair<int, int>, std::vector<void*>> free;  // (device, log2 size)
  size_t cached = 0;
};
static DevCache& dev_cache() {
  static DevCache* c = new DevCache();  // never destroyed: outlives every plan
  return *c;
}

struct Arena {
  nnms_allocator a{};
  bool has = false;
  bool pooled = false;  // small buffers of a plan: recycled through dev_cache
  int dev = -1;
  std::vector<std::pair<void*, size_t>> bufs;
  size_t total = 0;
  Arena() = default;
  explicit Arena(const nnms_allocator* al) {
    if (al && al->alloc && al->free) a = *al, has = true;
  }
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  void* raw(size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    void* p = nullptr;
    if (pooled && !has) {
      int c = 12;
      while ((size_t(1) << c) < bytes) ++c;
      bytes = size_t(1) << c;
      if (dev < 0) HIP_CHECK(hipGetDevice(&dev));
      std::lock_guard<std::mutex> g(dev_cache().mu);
      auto& v = dev_cache().free[{dev, c}];
      if (!v.empty()) {
        p = v.back();
        v.pop_back();
        dev_cache().cached -= bytes;
      }
    }
    if (p) {
    } else if (has) {
      p = a.alloc(bytes, a.ctx);
      if (!p) throw Error(NNMS_ERR_OUT_OF_MEMORY, "device allocator returned null for " + std::to_string(bytes) + " bytes");
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(NNMS_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                                hipGetErrorName(e));
      }
    }
    bufs.emplace_back(p, bytes);
    total += bytes;
    g_bytes += int64_t(bytes);
    return p;
  }
  template <typename T>
  T* alloc(size_t n, hipStream_t s, bool zero = true) {
    T* p = (T*)raw(n * sizeof(T));
    if (zero) HIP_CHECK(hipMemsetAsync(p, 0, std::max<size_t>(n * sizeof(T), 1), s));
    return p;
  }
  template <typename T>
  T* upload(const std::vector<T>& v, hipStream_t s) {
    T* p = (T*)raw(v.size() * sizeof(T));
    if (!v.empty()) HIP_CHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return p;
  }
  void release() {
    for (auto& b : bufs) {
      bool kept = false;
      if (pooled && !has) {
        int c = 12;
        while ((size_t(1) << c) < b.second) ++c;
        std::lock_guard<std::mutex> g(dev_cache().mu);
        if (dev_cache().cached + b.second <= kDevCacheCap) {
          dev_cache().free[{dev, c}].push_back(b.first);
          dev_cache().cached += b.second;
          kept = true;
        }
      }
      if (kept) {
      } else if (has)
        a.free(b.first, a.ctx);
      else
        (void)hipFree(b.first);
      g_bytes -= int64_t(b.second);
    }
    bufs.clear();
    total = 0;
  }
  ~Arena() { release(); }
};

struct DevLevel {
  int32_t *rp = nullptr, *col = nullptr, *cptr = nullptr, *citem = nullptr, *vptr = nullptr, *vitem = nullptr,
          *tets = nullptr;
  double* xyz = nullptr;
  uint8_t* dmask = nullptr;
  int32_t *gidx = nullptr, *ext_rs = nullptr, *ext_lc = nullptr;
  int32_t *sell_off = nullptr, *sell_col = nullptr, *sell_src = nullptr;
  int32_t* p_idx = nullptr;
  double* p_w64 = nullptr;
  float* p_w32 = nullptr;
  int32_t *pt_rp = nullptr, *pt_col = nullptr;
  double* pt_w64 = nullptr;
  float* pt_w32 = nullptr;
  int32_t *pts_off = nullptr, *pts_col = nullptr;  // P^T in sliced ELL layout
  double* pts_w64 = nullptr;
  float* pts_w32 = nullptr;
  // P^T in column-sorted slices (null where a slice does not fit the keys)
  int32_t *ptc_key = nullptr, *ptc_base = nullptr;
  double* ptc_w64 = nullptr;
  float* ptc_w32 = nullptr;
  int32_t ptc_cap = 0;
  int32_t *pn_off = nullptr, *pn_col = nullptr;  // MLS: -P in sliced ELL layout
  double* pn_w64 = nullptr;
  float* pn_w32 = nullptr;
  int32_t transfer = NNMS_TRANSFER_BARYCENTRIC;
  // ILU subdomain solver (subsolver == NNMS_SUBSOLVER_ILU)
  int32_t subsolver = NNMS_SUBSOLVER_LU;
  int32_t *ilu_rp = nullptr, *ilu_col = nullptr, *ilu_asrc = nullptr, *ilu_dpos = nullptr, *ilu_gid = nullptr;
  int32_t *ilu_fmeta = nullptr, *ilu_bmeta = nullptr, *ilu_flev = nullptr, *ilu_blev = nullptr;
};

}  // namespace nnms

using namespace nnms;

struct nnms_hierarchy {
  HostHierarchy host;
  bool on_device = false;
  std::unique_ptr<Arena> mem;
  std::vector<DevLevel> dev;
  std::atomic<int> systems{0};
  nnms_allocator alloc{};
  bool has_alloc = false;
  nnms_tuning tune{};
};

namespace nnms {

struct SysLevel {
  double* val64 = nullptr;
  float* val32 = nullptr;
  double* ell64 = nullptr;  // the values in the sliced ELL layout of the pattern
  float* ell32 = nullptr;
  void* fac = nullptr;  // factor tiles (float in mixed smoothed levels, else double)
  void* yx = nullptr;   // triangular-solve workspace (factor type)
  void* r = nullptr;    // level vectors, working precision
  void* z = nullptr;
  void* t = nullptr;
  void* ilu_val = nullptr;  // ILU factor values (factor type), ILU levels only
  void* xinv = nullptr;     // inverse panels X_p (factor type), NNMS_APPLY_INVERSE only
  void* xpart = nullptr;    // their smoother's partial sums (factor type)
};

struct Plan;

}  // namespace nnms

struct nnms_system {
  nnms_hierarchy* h = nullptr;
  int prec = NNMS_FP64;
  int dev = -1;  // device the system was assembled on
  std::unique_ptr<Arena> mem;
  std::vector<SysLevel> lev;
  double* b0 = nullptr;  // assembled load vector
  // solve workspace
  double *V = nullptr, *Z = nullptr, *w = nullptr, *x = nullptr, *bw = nullptr;
  double *part1 = nullptr, *part2 = nullptr, *partn = nullptr, *partr = nullptr;
  KState* st = nullptr;
  int restart_cap = 0;
  int nblk = 0, nblkr = 0;
  std::unique_ptr<Plan> solo;   // single-slot solve plan
  std::unique_ptr<Plan> apply;  // stateless plan for single operator applications
  hipStream_t stream = nullptr;
  ~nnms_system();
};

namespace nnms {

constexpr int SPMV_G_A = 16;   // lanes per row of the level operators
constexpr int SPMV_G_PT = 32;  // lanes per row of P^T
static int ras_grid_default() {
  static int g = [] {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
      hipDeviceProp_t p;
      if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    }
    return cus * 4;
  }();
  return g;
}

// blocks of one SpMV launch: G lanes per CSR row, or the sliced ELL layout:
// G = 0 four 64-row slices per block, G = 1 one slice per block (its steps
// split over the four waves)
// G = 2 (P^T only) the column-sorted slices, one slice per block
static bool is_sell(int G) { return G == 0 || G == 1; }
constexpr int SPMV_CSORT = 2;
static int spmv_blocks(int64_t n, int G) {
  if (G == 0) return int((n + 255) / 256);
  if (G == 1 || G == SPMV_CSORT) return int((n + 63) / 64);
  return int((n + (256 / G) - 1) / (256 / G));
}
static int vec_blocks(int64_t n) { return int((n + VBLK - 1) / VBLK); }

// ---------------------------------------------------------------------------
// a batch plan: descriptor tables for every launch of one Arnoldi step
// ---------------------------------------------------------------------------
// One SpMV launch per lanes-per-row choice among the systems of a plan: the
// choice fixes the summation order, so every system keeps the one of its own
// hierarchy's tuning and gives the same bits alone and in any batch.
struct SpmvGroup {
  SpmvDesc* d = nullptr;
  int nd = 0, blocks = 0, g = 16;
  int cap = 0;  // column-sorted slices: most entries of one slice
};

// items: (lanes per row, descriptor); blk0 is counted inside each group
static std::vector<SpmvGroup> spmv_groups(Arena& mem, const std::vector<std::pair<int, SpmvDesc>>& items,
                                          hipStream_t s) {
  std::vector<int> gs;
  for (const auto& it : items)
    if (std::find(gs.begin(), gs.end(), it.first) == gs.end()) gs.push_back(it.first);
  std::vector<SpmvGroup> out;
  for (int g : gs) {
    std::vector<SpmvDesc> v;
    int b = 0, cap = 0;
    for (const auto& it : items)
      if (it.first == g) {
        SpmvDesc d = it.second;
        d.blk0 = b;
        b += spmv_blocks(d.n, g);
        cap = std::max(cap, d.cap);
        v.push_back(d);
      }
    SpmvGroup G;
    G.d = mem.upload(v, s), G.nd = int(v.size()), G.blocks = b, G.g = g, G.cap = cap;
    out.push_back(G);
  }
  return out;
}

template <typename T>
static hipError_t launch_spmv_groups(const std::vector<SpmvGroup>& gs, hipStream_t s) {
  for (const SpmvGroup& G : gs) {
    const hipError_t e = G.g == SPMV_CSORT ? launch_csort<T>(G.d, G.nd, G.blocks, G.cap, s)
                         : is_sell(G.g)      ? launch_sell<T>(G.d, G.nd, G.blocks, G.g, s)
                                             : launch_spmv<T>(G.d, G.nd, G.blocks, G.g, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One smoother launch pair per blocks-per-work-item choice among the
// systems of a plan (one- and two-block items round differently): every
// system keeps its own hierarchy's choice, alone and in any batch.
struct RasGroup {
  RasLaunch r{}, t{};  // input r_l (write) / t_l (add)
  int grid = 0;
};

template <typename F, typename V>
static hipError_t launch_ras_groups(const std::vector<RasGroup>& gs, bool add, hipStream_t s) {
  for (const RasGroup& G : gs) {
    const hipError_t e = launch_ras<F, V>(add ? G.t : G.r, G.grid, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ILU smoother launch of one level over the ILU systems of a plan that share
// a lanes-per-row choice (it fixes the summation order, so every system
// keeps its own alone and in any batch): input r_l (write) / t_l (add), one
// work-group per subdomain
struct IluGroup {
  IluDesc *r = nullptr, *t = nullptr;
  int nd = 0, maxn = 0, lanes = 4;
};

struct LevelPlan {
  std::vector<SpmvGroup> res, rst;
  ProlongDesc* pro = nullptr;  // barycentric systems (four entries per row)
  int pro_blocks = 0;
  std::vector<SpmvGroup> prom;  // MLS systems: z_f - (-P) z_c, sliced ELL
  std::vector<RasGroup> ras;    // systems with dense subdomain LU
  std::vector<IluGroup> ilu;    // systems with ILU subdomain solves, per lanes choice
  int nd = 0;  // descriptors in pro
};

// z_f += P_l z_c for every system of a level plan
template <typename T>
static hipError_t launch_prolong_level(const LevelPlan& LP, hipStream_t s) {
  if (LP.pro_blocks) {
    const hipError_t e = launch_prolong<T>(LP.pro, LP.nd, LP.pro_blocks, s);
    if (e != hipSuccess) return e;
  }
  return launch_spmv_groups<T>(LP.prom, s);
}

// one smoother application on a smoothed level: z = B^{-1} r_l (add false)
// or z += B^{-1} t_l (add true), dense-LU and ILU systems alike
template <typename T>
static hipError_t launch_smoother_level(const LevelPlan& LP, bool add, hipStream_t s) {
  hipError_t e = launch_ras_groups<T, T>(LP.ras, add, s);
  if (e != hipSuccess) return e;
  for (const IluGroup& G : LP.ilu)
    if ((e = launch_ilu_apply<T>(add ? G.t : G.r, G.nd, G.maxn, G.lanes, add ? 1 : 0, s)) != hipSuccess) return e;
  return hipSuccess;
}

// Streams and pinned host words of plans are recycled instead of destroyed:
// hipStreamDestroy and hipHostFree wait for the device, which would make
// dropping a batch plan wait for unrelated work on other streams (the
// factorisation of a newly admitted request in the serving loop).  A
// recycled stream keeps its order: work of the next plan queues behind the
// last one's.
struct PlanPools {
  std::mutex mu;
  std::vector<hipStream_t> streams;
  std::vector<int*> words;
};
static PlanPools& plan_pools() {
  static PlanPools* p = new PlanPools();  // never destroyed: outlives every plan
  return *p;
}
static hipStream_t pool_stream() {
  {
    std::lock_guard<std::mutex> g(plan_pools().mu);
    auto& v = plan_pools().streams;
    if (!v.empty()) {
      hipStream_t st = v.back();
      v.pop_back();
      return st;
    }
  }
  hipStream_t st = nullptr;
  HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  return st;
}
static int* pool_word() {
  {
    std::lock_guard<std::mutex> g(plan_pools().mu);
    auto& v = plan_pools().words;
    if (!v.empty()) {
      int* w = v.back();
      v.pop_back();
      return w;
    }
  }
  int* w = nullptr;
  HIP_CHECK(hipHostMalloc((void**)&w, sizeof(int), hipHostMallocDefault));
  return w;
}

struct Plan {
  std::vector<nnms_system*> sys;
  int L = 0, prec = NNMS_FP64, its = 3;
  bool with_state = true;
  Arena mem;
  std::vector<LevelPlan> lev;  // smoothed levels
  std::vector<RasGroup> coarse;  // the coarsest direct solve (write launches)
  int nd = 0;
  KrylovDesc* kd = nullptr;
  std::vector<KrylovDesc> kd_host;
  int kblocks = 0;
  std::vector<SpmvGroup> wspmv, rspmv;
  int* d_active = nullptr;
  int* h_active = nullptr;
  hipStream_t stream = nullptr;
  hipGraphExec_t graph = nullptr;  // one Arnoldi step, captured on first use
  bool use_graph = true;
  // Arnoldi steps the plan's last solve took: the next solve enqueues that
  // many steps before it reads the active count
  int expect = 0;
  std::vector<int32_t*> counters;
  Plan() = default;
  ~Plan() {
    // this plan's own work is done before its graph and descriptors go (a
    // stream synchronisation: other streams are not waited for)
    if (stream) (void)hipStreamSynchronize(stream);
    if (graph) (void)hipGraphExecDestroy(graph);
    std::lock_guard<std::mutex> g(plan_pools().mu);
    if (h_active) plan_pools().words.push_back(h_active);
    if (stream) plan_pools().streams.push_back(stream);
  }
};

template <typename T>
static const void* val_of(const SysLevel& sl) {
  if (std::is_same<T, float>::value) return sl.val32;
  return sl.val64;
}

template <typename T>
static const void* ell_of(const SysLevel& sl) {
  if (std::is_same<T, float>::value) return sl.ell32;
  return sl.ell64;
}

// task list of one restricted additive Schwarz launch over subdomains with
// N[q] blocks: forward block i at step i, backward block i at step 2N-1-i,
// ordered by (step, subdomain) so that every dependency has a lower ticket.
// The backward sweep of subdomain q starts at the work item holding block
// B0[q] (the first owned one): the rows before it are not owned, and with
// them last in the sweep nothing after them depends on them.
static std::vector<int32_t> ras_tasks(const std::vector<int32_t>& N, const std::vector<int32_t>& B0, int K) {
  // counting sort by key = step + 4 (NBmax - NB): a subdomain with fewer work
  // items enters the order later, so the longest chains start first and the
  // launch's tail shortens (fine level 0.317 -> 0.306 ms FP32, second level
  // 0.139 -> 0.135 ms FP64; larger head starts starve the small subdomains).
  // Inside a subdomain the order stays that of its steps, a dependency
  // order, so no work item waits on one drawn after it.  Inside a key,
  // subdomains stay in ascending order.
  int nbmax = 0;
  for (int32_t n : N) nbmax = std::max(nbmax, (n + K - 1) / K);
  auto shift = [&](int NB) { return 4 * (nbmax - NB); };
  int steps = 0;
  for (int32_t n : N) {
    const int NB = (n + K - 1) / K;
    steps = std::max(steps, 2 * NB + shift(NB));
  }
  std::vector<int32_t> cnt(size_t(steps) + 1, 0);
  for (size_t q = 0; q < N.size(); ++q) {
    const int NB = (N[q] + K - 1) / K, I0 = std::min(B0[q] / K, NB - 1);
    for (int s = 0; s < 2 * NB - I0; ++s) cnt[s + shift(NB) + 1]++;
  }
  for (int s = 0; s < steps; ++s) cnt[s + 1] += cnt[s];
  std::vector<int32_t> out(cnt[steps]);
  for (size_t q = 0; q < N.size(); ++q) {
    const int NB = (N[q] + K - 1) / K, I0 = std::min(B0[q] / K, NB - 1);
    const int sh = shift(NB);
    for (int i = 0; i < NB; ++i) {
      out[cnt[i + sh]++] = int32_t((q << 16) | i);
      if (i >= I0) out[cnt[2 * NB - 1 - i + sh]++] = int32_t((q << 16) | (1 << 15) | i);
    }
  }
  return out;
}

// work items of an inverse-panel launch: per subdomain q and owned tile
// column b, the overlap part (Nv tiles, when there are overlap rows) and the
// owned part (No - b tiles): (q << 16) | (owned << 15) | b.  Ordered by
// decreasing tile count (ties by subdomain, then column), so the long items
// start first and the launch's tail is short.
static std::vector<int32_t> xpanel_tasks(const std::vector<SubDesc>& subs) {
  std::vector<std::pair<int, int32_t>> items;  // (-tiles, code)
  for (size_t q = 0; q < subs.size(); ++q) {
    const int No = (subs[q].no + TILE - 1) / TILE, Nv = (subs[q].nv + TILE - 1) / TILE;
    for (int b = 0; b < No; ++b) {
      if (Nv > 0) items.emplace_back(-Nv, int32_t((q << 16) | b));
      items.emplace_back(-(No - b), int32_t((q << 16) | (1 << 15) | b));
    }
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const std::pair<int, int32_t>& x, const std::pair<int, int32_t>& y) { return x.first < y.first; });
  std::vector<int32_t> out;
  for (auto& it : items) out.push_back(it.second);
  return out;
}

// smoother work-item kind of a system's level: blocks per triangular-sweep
// work item (the hierarchy's tuning), or 0 for inverse panels
static int ras_kind(const nnms_system* x, int l) {
  return x->h->host.lev[l].xinv ? 0 : x->h->tune.ras_blocks[l];
}

// The two smoother launches of level l over a set of systems (input r_l with
// z written, input t_l with z added), for work items of K blocks; flags,
// tasks and the ticket counter are allocated in `mem`.
// subdomain descriptors of level l over a set of systems: input r_l (subs_r)
// and t_l (subs_t), and the block count of every subdomain
static void ras_subdescs(const std::vector<nnms_system*>& sys, int l, bool coarse, int prec, bool with_state,
                         std::vector<SubDesc>& subs_r, std::vector<SubDesc>& subs_t, std::vector<int32_t>& Ns,
                         std::vector<int32_t>& B0s) {
  for (auto* x : sys) {
    const HostLevel& hl = x->h->host.lev[l];
    if (!coarse && hl.subsolver == NNMS_SUBSOLVER_ILU)
      throw Error(NNMS_ERR_INVALID_ARG, "dense smoother launch requested on an ILU level");
    const DevLevel& dl = x->h->dev[l];
    const SysLevel& sl = x->lev[l];
    const size_t fsz = (coarse || prec == NNMS_FP64) ? sizeof(double) : sizeof(float);
    for (int p = 0; p < hl.nparts; ++p) {
      SubDesc d{};
      if (hl.xinv) {
        d.fac = (const char*)sl.xinv + size_t(hl.xs_off[p]) * fsz;
        d.part = (char*)sl.xpart + size_t(hl.xp_off[p]) * fsz;
      }
      else
        d.fac = (const char*)sl.fac + size_t(hl.fac_off[p]) * fsz;
      d.gidx = dl.gidx + hl.g_off[p];
      d.no = hl.nown[p];
      d.nv = int32_t(hl.s_ptr[p + 1] - hl.s_ptr[p]) - hl.nown[p];
      d.yx = (char*)sl.yx + size_t(hl.g_off[p]) * 16;
      d.rin = sl.r;
      d.zout = sl.z;
      d.st = with_state ? x->st : nullptr;
      d.N = hl.nblk[p];
      subs_r.push_back(d);
      d.rin = sl.t;
      subs_t.push_back(d);
      Ns.push_back(hl.nblk[p]);
      B0s.push_back(hl.bwd0.empty() ? 0 : hl.bwd0[p]);
    }
  }
  if (subs_r.size() > 32767) throw Error(NNMS_ERR_INVALID_ARG, "too many subdomains in one batch");
}

static void build_ras_pair(Arena& mem, std::vector<int32_t*>& counters, const std::vector<nnms_system*>& sys, int l,
                           bool coarse, int prec, bool with_state, int K, hipStream_t s, RasLaunch& rr, RasLaunch& rt) {
  std::vector<SubDesc> subs_r, subs_t;
  std::vector<int32_t> Ns, B0s;
  ras_subdescs(sys, l, coarse, prec, with_state, subs_r, subs_t, Ns, B0s);
  std::vector<int32_t> tasks = K == 0 ? xpanel_tasks(subs_r) : ras_tasks(Ns, B0s, K);
  int32_t* counter = mem.alloc<int32_t>(4, s);
  HIP_CHECK(launch_ras_seed(counter, s));
  counters.push_back(counter);
  rr = RasLaunch{};
  rr.subs = mem.upload(subs_r, s);
  rr.tasks = mem.upload(tasks, s);
  rr.counter = counter;
  rr.ntasks = int(tasks.size());
  rr.add = 0;
  rr.group = K;
  for (int32_t n : Ns) rr.max_tiles = std::max(rr.max_tiles, n);
  rt = rr;
  rt.subs = mem.upload(subs_t, s);
  rt.add = 1;
}

static std::vector<IluDesc> ilu_descs(const nnms_system& x, int l, bool with_state) {
  const HostLevel& hl = x.h->host.lev[l];
  const DevLevel& dl = x.h->dev[l];
  const SysLevel& sl = x.lev[l];
  std::vector<IluDesc> v;
  for (int p = 0; p < hl.nparts; ++p) {
    const int64_t base = hl.s_ptr[p];
    IluDesc d{};
    d.rp = dl.ilu_rp + base, d.dpos = dl.ilu_dpos + base, d.col = dl.ilu_col;
    d.fmeta = dl.ilu_fmeta + base * 4, d.flev = dl.ilu_flev + hl.ilu_flev_off[p];
    d.bmeta = dl.ilu_bmeta + base * 4, d.blev = dl.ilu_blev + hl.ilu_blev_off[p];
    d.gid = dl.ilu_gid + base, d.val = sl.ilu_val;
    d.rin = sl.r, d.zout = sl.z, d.st = with_state ? x.st : nullptr;
    d.n = int32_t(hl.s_ptr[p + 1] - base);
    d.nfl = int32_t(hl.ilu_flev_off[p + 1] - hl.ilu_flev_off[p]) - 1;
    d.nbl = int32_t(hl.ilu_blev_off[p + 1] - hl.ilu_blev_off[p]) - 1;
    v.push_back(d);
  }
  return v;
}

static std::vector<IluGroup> ilu_groups_of(Arena& mem, const std::vector<nnms_system*>& sys, int l, bool with_state,
                                           hipStream_t s) {
  std::vector<int> gs;
  for (auto* x : sys) {
    const HostLevel& hl = x->h->host.lev[l];
    if (hl.subsolver == NNMS_SUBSOLVER_ILU && std::find(gs.begin(), gs.end(), hl.ilu_lanes) == gs.end())
      gs.push_back(hl.ilu_lanes);
  }
  std::vector<IluGroup> out;
  for (int g : gs) {
    std::vector<IluDesc> r, t;
    IluGroup G;
    G.lanes = g;
    for (auto* x : sys) {
      const HostLevel& hl = x->h->host.lev[l];
      if (hl.subsolver != NNMS_SUBSOLVER_ILU || hl.ilu_lanes != g) continue;
      for (IluDesc d : ilu_descs(*x, l, with_state)) {
        G.maxn = std::max(G.maxn, int(d.n));
        r.push_back(d);
        d.rin = x->lev[l].t;
        t.push_back(d);
      }
    }
    G.r = mem.upload(r, s);
    G.t = mem.upload(t, s);
    G.nd = int(r.size());
    out.push_back(G);
  }
  return out;
}

template <typename T>
static void build_plan(Plan& P, const std::vector<nnms_system*>& sys, bool with_state, hipStream_t s) {
  P.sys = sys;
  P.with_state = with_state;
  nnms_hierarchy* h0 = sys[0]->h;
  P.L = h0->host.L;
  P.prec = sys[0]->prec;
  P.its = h0->host.opts.its;
  const int L = P.L;
  P.nd = int(sys.size());
  if (sys.size() > 32767) throw Error(NNMS_ERR_INVALID_ARG, "too many systems in one batch");
  for (auto* x : sys)
    if (x->h->host.L != L || x->prec != P.prec || x->h->host.opts.its != P.its)
      throw Error(NNMS_ERR_INVALID_ARG, "batched systems must share level count, precision and smoothing steps");
  P.lev.resize(std::max(0, L - 1));
  // smoother launches of level l, one per blocks-per-item value (the launch
  // grid, which changes no arithmetic, from the group's first system)
  auto dense_at = [&](const nnms_system* x, int l, bool coarse) {
    return coarse || x->h->host.lev[l].subsolver != NNMS_SUBSOLVER_ILU;
  };
  auto ras_groups_of = [&](int l, bool coarse) {
    std::vector<int> ks;
    for (auto* x : sys)
      if (dense_at(x, l, coarse) && std::find(ks.begin(), ks.end(), ras_kind(x, l)) == ks.end())
        ks.push_back(ras_kind(x, l));
    std::vector<RasGroup> out;
    for (int K : ks) {
      std::vector<nnms_system*> sub;
      for (auto* x : sys)
        if (dense_at(x, l, coarse) && ras_kind(x, l) == K) sub.push_back(x);
      RasGroup G;
      const int g = sub[0]->h->tune.ras_groups[l];
      G.grid = g > 0 ? g : ras_grid_default();
      build_ras_pair(P.mem, P.counters, sub, l, coarse, P.prec, with_state, K, s, G.r, G.t);
      out.push_back(G);
    }
    return out;
  };
  for (int l = 0; l < L - 1; ++l) {
    LevelPlan& LP = P.lev[l];
    std::vector<std::pair<int, SpmvDesc>> res, rst;
    std::vector<ProlongDesc> pro;
    std::vector<std::pair<int, SpmvDesc>> prom;
    int bp = 0;
    for (auto* x : sys) {
      const HostLevel& hl = x->h->host.lev[l];
      const HostLevel& hc = x->h->host.lev[l + 1];
      const DevLevel& dl = x->h->dev[l];
      const SysLevel& sl = x->lev[l];
      const SysLevel& sc = x->lev[l + 1];
      const KState* st = with_state ? x->st : nullptr;
      SpmvDesc d{};
      const int ga = x->h->tune.spmv_lanes[l];
      if (is_sell(ga))
        d.rp = dl.sell_off, d.col = dl.sell_col, d.val = ell_of<T>(sl);
      else
        d.rp = dl.rp, d.col = dl.col, d.val = val_of<T>(sl);
      d.x = sl.z, d.r = sl.r, d.y = sl.t;
      d.st = st, d.n = int(hl.nv), d.when = WHEN_RUNNING;
      res.emplace_back(ga, d);
      SpmvDesc e{};
      const int gp = x->h->tune.pt_lanes[l];
      if (gp == SPMV_CSORT) {
        e.rp = dl.pt_rp, e.col = dl.ptc_key, e.base = dl.ptc_base, e.cap = dl.ptc_cap;
        e.val = std::is_same<T, float>::value ? (const void*)dl.ptc_w32 : (const void*)dl.ptc_w64;
      } else if (is_sell(gp)) {
        e.rp = dl.pts_off, e.col = dl.pts_col;
        e.val = std::is_same<T, float>::value ? (const void*)dl.pts_w32 : (const void*)dl.pts_w64;
      } else {
        e.rp = dl.pt_rp, e.col = dl.pt_col;
        e.val = std::is_same<T, float>::value ? (const void*)dl.pt_w32 : (const void*)dl.pt_w64;
      }
      e.x = sl.t, e.r = nullptr, e.y = sc.r, e.st = st, e.n = int(hc.nv), e.when = WHEN_RUNNING;
      rst.emplace_back(gp, e);
      if (dl.transfer == NNMS_TRANSFER_MLS) {
        SpmvDesc m{};
        m.rp = dl.pn_off, m.col = dl.pn_col;
        m.val = std::is_same<T, float>::value ? (const void*)dl.pn_w32 : (const void*)dl.pn_w64;
        m.x = sc.z, m.r = sl.z, m.y = sl.z, m.st = st, m.n = int(hl.nv), m.when = WHEN_RUNNING;
        prom.emplace_back(0, m);
        continue;
      }
      ProlongDesc pd{};
      pd.idx = dl.p_idx;
      pd.w = std::is_same<T, float>::value ? (const void*)dl.p_w32 : (const void*)dl.p_w64;
      pd.zc = sc.z, pd.zf = sl.z, pd.st = st, pd.n = int(hl.nv), pd.blk0 = bp;
      pro.push_back(pd);
      bp += int((hl.nv + 255) / 256);
    }
    LP.res = spmv_groups(P.mem, res, s);
    LP.rst = spmv_groups(P.mem, rst, s);
    if (!pro.empty()) LP.pro = P.mem.upload(pro, s);
    LP.pro_blocks = bp;
    LP.nd = int(pro.size());
    LP.prom = spmv_groups(P.mem, prom, s);
    LP.ras = ras_groups_of(l, false);
    LP.ilu = ilu_groups_of(P.mem, sys, l, with_state, s);
  }
  P.coarse = ras_groups_of(L - 1, true);
  // Krylov descriptors
  if (with_state) {
    std::vector<std::pair<int, SpmvDesc>> wd, rd;
    int kb = 0;
    for (auto* x : sys) {
      const HostLevel& h0l = x->h->host.lev[0];
      const DevLevel& d0 = x->h->dev[0];
      KrylovDesc k{};
      k.V = x->V, k.Z = x->Z, k.w = x->w, k.x = x->x, k.b = x->bw, k.dmask = d0.dmask;
      k.part1 = x->part1, k.part2 = x->part2, k.partn = x->partn, k.partr = x->partr, k.st = x->st;
      k.r0 = x->lev[0].r, k.z0 = x->lev[0].z;
      const int gw = x->h->tune.krylov_lanes;
      k.n = int(h0l.nv), k.blk0 = kb, k.nblk = x->nblk, k.nblkr = spmv_blocks(h0l.nv, gw);
      if (k.nblkr > x->nblkr) throw Error(NNMS_ERR_INVALID_ARG, "residual partials exceed their buffer");
      P.kd_host.push_back(k);
      kb += x->nblk;
      SpmvDesc d{};
      if (is_sell(gw))
        d.rp = d0.sell_off, d.col = d0.sell_col, d.val = x->lev[0].ell64;
      else
        d.rp = d0.rp, d.col = d0.col, d.val = x->lev[0].val64;
      d.x = x->Z, d.x_jstride = h0l.nv, d.r = nullptr;
      d.y = x->w, d.st = x->st, d.n = int(h0l.nv), d.when = WHEN_RUNNING;
      wd.emplace_back(gw, d);
      d.x = x->x, d.x_jstride = 0, d.r = x->bw, d.nrm = x->partr, d.when = WHEN_CYCLE_END;
      rd.emplace_back(gw, d);
    }
    P.kd = P.mem.upload(P.kd_host, s);
    P.kblocks = kb;
    P.wspmv = spmv_groups(P.mem, wd, s);
    P.rspmv = spmv_groups(P.mem, rd, s);
    P.d_active = P.mem.alloc<int>(1, s);
    P.h_active = pool_word();
  }
  HIP_CHECK(hipStreamSynchronize(s));
}

static void check_counters(Plan& P, hipStream_t s) {
  for (int32_t* c : P.counters) {
    int32_t v[4];
    HIP_CHECK(hipMemcpyAsync(v, c, sizeof v, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (v[2]) {
      // reported once: later calls through the same plan report only their own failures
      HIP_CHECK(hipMemsetAsync(c + 2, 0, sizeof(int32_t), s));
      HIP_CHECK(hipStreamSynchronize(s));
      throw Error(NNMS_ERR_DEVICE, "triangular-solve wait limit exceeded (error bits " + std::to_string(v[2]) + ")");
    }
  }
}

template <typename T>
static void enqueue_vcycle(Plan& P, hipStream_t s) {
  const int L = P.L, its = P.its;
  for (int l = 0; l < L - 1; ++l) {
    LevelPlan& LP = P.lev[l];
    HIP_CHECK(launch_smoother_level<T>(LP, false, s));
    for (int k = 1; k < its; ++k) {
      HIP_CHECK(launch_spmv_groups<T>(LP.res, s));
      HIP_CHECK(launch_smoother_level<T>(LP, true, s));
    }
    HIP_CHECK(launch_spmv_groups<T>(LP.res, s));
    HIP_CHECK(launch_spmv_groups<T>(LP.rst, s));
  }
  HIP_CHECK((launch_ras_groups<double, T>(P.coarse, false, s)));
  for (int l = L - 2; l >= 0; --l) {
    LevelPlan& LP = P.lev[l];
    HIP_CHECK(launch_prolong_level<T>(LP, s));
    for (int k = 0; k < its; ++k) {
      HIP_CHECK(launch_spmv_groups<T>(LP.res, s));
      HIP_CHECK(launch_smoother_level<T>(LP, true, s));
    }
  }
}

template <typename T>
static void enqueue_step(Plan& P, hipStream_t s) {
  HIP_CHECK(launch_krylov_cast_in<T>(P.kd, P.nd, P.kblocks, s));
  enqueue_vcycle<T>(P, s);
  HIP_CHECK(launch_krylov_cast_out<T>(P.kd, P.nd, P.kblocks, s));
  HIP_CHECK(launch_spmv_groups<double>(P.wspmv, s));
  HIP_CHECK(launch_krylov_dots1(P.kd, P.nd, P.kblocks, s));
  HIP_CHECK(launch_krylov_upd1(P.kd, P.nd, P.kblocks, s));
  HIP_CHECK(launch_krylov_upd2(P.kd, P.nd, P.kblocks, s));
  HIP_CHECK(launch_krylov_givens(P.kd, P.nd, s));
  HIP_CHECK(launch_krylov_normalize(P.kd, P.nd, P.kblocks, s));
  HIP_CHECK(launch_krylov_xupd(P.kd, P.nd, P.kblocks, s));
  HIP_CHECK(launch_spmv_groups<double>(P.rspmv, s));
  HIP_CHECK(launch_krylov_cycle(P.kd, P.nd, s));
}

// K consecutive Arnoldi steps enqueued back to back: K replays of the
// plan's one-step graph (captured once, on first use: a capture in progress
// makes other threads' legacy-stream calls fail, so none happens per solve),
// or the launches themselves with NNMS_NO_GRAPH.  Steps after a slot has
// converged leave it unchanged (every kernel skips finished slots).
static void plan_steps(Plan& P, int K) {
  hipStream_t s = P.stream;
  auto enqueue = [&]() {
    if (P.prec == NNMS_MIXED)
      enqueue_step<float>(P, s);
    else
      enqueue_step<double>(P, s);
  };
  if (!P.use_graph) {
    for (int k = 0; k < K; ++k) enqueue();
    return;
  }
  if (!P.graph) {
    hipGraph_t g;
    HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      enqueue();
    } catch (...) {
      hipGraph_t junk;
      (void)hipStreamEndCapture(s, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      throw;
    }
    HIP_CHECK(hipStreamEndCapture(s, &g));
    hipError_t e = hipGraphInstantiate(&P.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_CHECK(e);
  }
  for (int k = 0; k < K; ++k) HIP_CHECK(hipGraphLaunch(P.graph, s));
}

static void plan_step(Plan& P) { plan_steps(P, 1); }

static int plan_active(Plan& P) {
  HIP_CHECK(launch_count_active(P.kd, P.nd, P.d_active, P.stream));
  HIP_CHECK(hipMemcpyAsync(P.h_active, P.d_active, sizeof(int), hipMemcpyDeviceToHost, P.stream));
  HIP_CHECK(hipStreamSynchronize(P.stream));
  return *P.h_active;
}

static void plan_start_slot(Plan& P, int k, const double* b_dev, const nnms_solve_opts& o) {
  nnms_system* x = P.sys[k];
  const int64_t n = x->h->host.lev[0].nv;
  if (b_dev != x->bw) HIP_CHECK(hipMemcpyAsync(x->bw, b_dev, n * sizeof(double), hipMemcpyDeviceToDevice, P.stream));
  const KrylovDesc& kd = P.kd_host[k];
  HIP_CHECK(launch_krylov_init_slot(P.kd, P.nd, kd.blk0, kd.nblk, P.stream));
  HIP_CHECK(launch_krylov_start_slot(P.kd + k, o.rtol, o.restart, o.max_it, P.stream));
}

template <typename T>
static std::unique_ptr<Plan> make_plan(const std::vector<nnms_system*>& sys, bool with_state) {
  auto P = std::make_unique<Plan>();
  P->mem.pooled = true;
  P->stream = pool_stream();
  build_plan<T>(*P, sys, with_state, P->stream);
  return P;
}

static std::unique_ptr<Plan> make_plan_any(const std::vector<nnms_system*>& sys, bool with_state) {
  if (sys[0]->prec == NNMS_MIXED) return make_plan<float>(sys, with_state);
  return make_plan<double>(sys, with_state);
}

// order the plan's internal stream after the caller's stream
static void join_in(hipStream_t user, hipStream_t inner) {
  hipEvent_t ev;
  HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  HIP_CHECK(hipEventRecord(ev, user));
  HIP_CHECK(hipStreamWaitEvent(inner, ev, 0));
  (void)hipEventDestroy(ev);
}

static void validate_solve_opts(const nnms_solve_opts& o) {
  if (o.restart < 1 || o.restart > NNMS_MAX_RESTART || !(o.rtol > 0) || o.max_it < 1)
    throw Error(NNMS_ERR_INVALID_ARG, "bad solve options");
}

// a system keeps Krylov bases of restart_cap columns
static void check_restart(const std::vector<nnms_system*>& sys, const nnms_solve_opts& o) {
  for (auto* s : sys)
    if (o.restart > s->restart_cap)
      throw Error(NNMS_ERR_INVALID_ARG, "restart " + std::to_string(o.restart) + " exceeds the system's restart_cap " +
                                            std::to_string(s->restart_cap));
}

}  // namespace nnms

nnms_system::~nnms_system() {
  solo.reset();
  apply.reset();
  mem.reset();
  if (h) h->systems--;
}

// ===========================================================================
// C ABI
// ===========================================================================
#define ABI_BEGIN try {
#define ABI_END                                      \
  }                                                  \
  catch (const nnms::Error& e) {                     \
    nnms::set_last_error(e.what());                  \
    return e.code;                                   \
  }                                                  \
  catch (const std::bad_alloc&) {                    \
    nnms::set_last_error("host out of memory");      \
    return NNMS_ERR_OUT_OF_MEMORY;                   \
  }                                                  \
  catch (const std::exception& e) {                  \
    nnms::set_last_error(e.what());                  \
    return NNMS_ERR_INVALID_ARG;                     \
  }

extern "C" const char* nnms_last_error(void) { return nnms::g_last_error.c_str(); }
extern "C" int64_t nnms_device_bytes_in_use(void) { return nnms::g_bytes.load(); }

static void default_tuning(nnms_tuning& t) {
  std::memset(&t, 0, sizeof t);
  for (int l = 0; l < NNMS_MAX_LEVELS; ++l)
    t.spmv_lanes[l] = SPMV_G_A, t.pt_lanes[l] = SPMV_G_PT, t.ras_groups[l] = 0, t.ras_blocks[l] = 1;
  t.krylov_lanes = SPMV_G_A;
  t.tuned = 0;
}

static void build_host(const nnms_mesh* const* levels, int32_t L, const nnms_setup_opts* opts, HostHierarchy& H) {
  if (!levels || L < 1 || L > NNMS_MAX_LEVELS || !opts) throw Error(NNMS_ERR_INVALID_ARG, "bad hierarchy arguments");
  if (opts->overlap < 0 || opts->its < 1 || (opts->precision != NNMS_FP64 && opts->precision != NNMS_MIXED) ||
      (opts->transfer != NNMS_TRANSFER_BARYCENTRIC && opts->transfer != NNMS_TRANSFER_MLS) ||
      (opts->transfer == NNMS_TRANSFER_MLS && !(opts->mls_alpha > 0)) ||
      (opts->subsolver != NNMS_SUBSOLVER_LU && opts->subsolver != NNMS_SUBSOLVER_ILU) ||
      (opts->ncomp != 0 && opts->ncomp != 1 && opts->ncomp != 3) || (opts->mls_clip != 0 && opts->mls_clip != 1) ||
      (opts->dense_apply != NNMS_APPLY_SWEEPS && opts->dense_apply != NNMS_APPLY_INVERSE))
    throw Error(NNMS_ERR_INVALID_ARG, "bad setup options");
  const int K = opts->ncomp ? opts->ncomp : 1;
  H.L = L;
  H.opts = *opts;
  H.opts.ncomp = K;
  H.lev.resize(L);
  for (int l = 0; l < L; ++l) {
    if (!levels[l]) throw Error(NNMS_ERR_INVALID_ARG, "null mesh");
    HostLevel& lv = H.lev[l];
    lv.nv = levels[l]->nv, lv.nt = levels[l]->nt;
    lv.xyz = levels[l]->xyz;
    lv.tets = levels[l]->tets;
    lv.dir = levels[l]->dir;
    build_pattern(lv);
    build_sell(lv);
    const bool direct = (l == L - 1);
    int np = direct ? 1 : opts->nparts[l];
    if (!direct && np == 0) np = default_nparts(lv.nv * K);
    H.opts.nparts[l] = np;
    lv.owned_last = !direct && opts->subsolver == NNMS_SUBSOLVER_LU;
    lv.xinv = opts->dense_apply == NNMS_APPLY_INVERSE && (direct || opts->subsolver == NNMS_SUBSOLVER_LU);
    build_partition(lv, np, opts->overlap, direct);
  }
  // transfers between the vertex-level meshes, then every level carried to
  // K unknowns per vertex (field splitting: each component is a field)
  for (int l = 0; l + 1 < L; ++l) {
    if (opts->transfer == NNMS_TRANSFER_MLS)
      build_transfer_mls(H.lev[l], H.lev[l + 1], opts->mls_alpha, opts->mls_restrict != 0,
                         opts->mls_clip ? H.opts.nparts[l] : 0, opts->overlap);
    else
      build_transfer(H.lev[l], H.lev[l + 1]);
  }
  for (int l = 0; l < L; ++l) expand_fields(H.lev[l], K);
  for (int l = 0; l + 1 < L; ++l) {
    HostLevel& lv = H.lev[l];
    if (opts->subsolver == NNMS_SUBSOLVER_ILU) {
      if (opts->ilu_fill[l] < 0) throw Error(NNMS_ERR_INVALID_ARG, "ILU fill level must be >= 0");
      const size_t vsz = opts->precision == NNMS_FP64 ? sizeof(double) : sizeof(float);
      for (int p = 0; p < lv.nparts; ++p)
        if (size_t(lv.s_ptr[p + 1] - lv.s_ptr[p]) * vsz > ILU_MAX_LDS)
          throw Error(NNMS_ERR_INVALID_ARG, "subdomain too large for the ILU smoother (" +
                                                std::to_string(lv.s_ptr[p + 1] - lv.s_ptr[p]) + " rows)");
      build_ilu(lv, opts->ilu_fill[l]);
    }
  }
}

extern "C" nnms_status nnms_hierarchy_setup_host(const nnms_mesh* const* levels, int32_t L, const nnms_setup_opts* opts,
                                                 nnms_hierarchy** out) {
  ABI_BEGIN
  if (!out) throw Error(NNMS_ERR_INVALID_ARG, "null output");
  *out = nullptr;
  auto h = std::make_unique<nnms_hierarchy>();
  build_host(levels, L, opts, h->host);
  default_tuning(h->tune);
  *out = h.release();
  return NNMS_OK;
  ABI_END
}

template <typename A, typename B>
static std::vector<B> convert(const std::vector<A>& v) {
  return std::vector<B>(v.begin(), v.end());
}

extern "C" nnms_status nnms_hierarchy_setup(const nnms_mesh* const* levels, int32_t L, const nnms_setup_opts* opts,
                                            const nnms_allocator* alloc, void* stream, nnms_hierarchy** out) {
  ABI_BEGIN
  if (!out) throw Error(NNMS_ERR_INVALID_ARG, "null output");
  *out = nullptr;
  auto h = std::make_unique<nnms_hierarchy>();
  build_host(levels, L, opts, h->host);
  default_tuning(h->tune);
  hipStream_t s = (hipStream_t)stream;
  h->mem = std::make_unique<Arena>(alloc);
  if (alloc && alloc->alloc && alloc->free) h->alloc = *alloc, h->has_alloc = true;
  h->dev.resize(L);
  Arena& A = *h->mem;
  for (int l = 0; l < L; ++l) {
    const HostLevel& hl = h->host.lev[l];
    DevLevel& d = h->dev[l];
    d.rp = A.upload(hl.rp, s);
    d.col = A.upload(hl.col, s);
    d.cptr = A.upload(hl.cptr, s);
    d.citem = A.upload(hl.citem, s);
    d.vptr = A.upload(hl.vptr, s);
    d.vitem = A.upload(hl.vitem, s);
    d.tets = A.upload(hl.tets, s);
    d.xyz = A.upload(hl.xyz, s);
    d.dmask = A.upload(hl.dir, s);
    d.gidx = A.upload(hl.gidx, s);
    d.ext_rs = A.upload(hl.ext_rs, s);
    d.ext_lc = A.upload(hl.ext_lc, s);
    d.sell_off = A.upload(hl.sell_off, s);
    d.sell_col = A.upload(hl.sell_col, s);
    d.sell_src = A.upload(hl.sell_src, s);
    if (l + 1 < L) {
      d.p_idx = A.upload(hl.p_idx, s);
      d.p_w64 = A.upload(hl.p_w, s);
      d.p_w32 = A.upload(convert<double, float>(hl.p_w), s);
      d.pt_rp = A.upload(hl.pt_rp, s);
      d.pt_col = A.upload(hl.pt_col, s);
      d.pt_w64 = A.upload(hl.pt_w, s);
      d.pt_w32 = A.upload(convert<double, float>(hl.pt_w), s);
      d.pts_off = A.upload(hl.pts_off, s);
      d.pts_col = A.upload(hl.pts_col, s);
      d.pts_w64 = A.upload(hl.pts_w, s);
      d.pts_w32 = A.upload(convert<double, float>(hl.pts_w), s);
      {
        std::vector<int32_t> key, base, src;
        if (build_csort_layout(hl.pt_rp, hl.pt_col, int64_t(hl.pt_rp.size()) - 1, key, base, src, d.ptc_cap) &&
            d.ptc_cap > 0) {
          std::vector<double> w(src.size());
          for (size_t e = 0; e < src.size(); ++e) w[e] = hl.pt_w[src[e]];
          d.ptc_key = A.upload(key, s);
          d.ptc_base = A.upload(base, s);
          d.ptc_w64 = A.upload(w, s);
          d.ptc_w32 = A.upload(convert<double, float>(w), s);
        } else {
          d.ptc_cap = 0;
        }
      }
      d.transfer = hl.transfer;
      if (hl.transfer == NNMS_TRANSFER_MLS) {
        d.pn_off = A.upload(hl.pn_off, s);
        d.pn_col = A.upload(hl.pn_col, s);
        d.pn_w64 = A.upload(hl.pn_w, s);
        d.pn_w32 = A.upload(convert<double, float>(hl.pn_w), s);
      }
      d.subsolver = hl.subsolver;
      if (hl.subsolver == NNMS_SUBSOLVER_ILU) {
        d.ilu_rp = A.upload(hl.ilu_rp, s);
        d.ilu_col = A.upload(hl.ilu_col, s);
        d.ilu_asrc = A.upload(hl.ilu_asrc, s);
        d.ilu_dpos = A.upload(hl.ilu_dpos, s);
        d.ilu_gid = A.upload(hl.ilu_gid, s);
        d.ilu_fmeta = A.upload(hl.ilu_fmeta, s);
        d.ilu_bmeta = A.upload(hl.ilu_bmeta, s);
        d.ilu_flev = A.upload(hl.ilu_flev, s);
        d.ilu_blev = A.upload(hl.ilu_blev, s);
      }
    }
  }
  HIP_CHECK(hipStreamSynchronize(s));
  h->on_device = true;
  *out = h.release();
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_hierarchy_destroy(nnms_hierarchy* h) {
  if (!h) return NNMS_OK;
  if (h->systems.load() > 0) {
    nnms::set_last_error("hierarchy still has live systems");
    return NNMS_ERR_IN_USE;
  }
  delete h;
  return NNMS_OK;
}

extern "C" nnms_status nnms_hierarchy_level_info(const nnms_hierarchy* h, int32_t level, nnms_level_info* o) {
  ABI_BEGIN
  if (!h || !o || level < 0 || level >= h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad level");
  const HostLevel& lv = h->host.lev[level];
  std::memset(o, 0, sizeof *o);
  o->nv = lv.nvert, o->nt = lv.nt, o->ninterior = lv.nint / lv.ncomp, o->nnz = int64_t(lv.col.size());
  o->ncomp = lv.ncomp, o->ndof = lv.nv;
  o->dense_apply = lv.xinv ? NNMS_APPLY_INVERSE : NNMS_APPLY_SWEEPS;
  o->nparts = lv.nparts;
  int mx = 0, mn = INT32_MAX;
  for (int p = 0; p < lv.nparts; ++p) {
    int n = int(lv.s_ptr[p + 1] - lv.s_ptr[p]);
    mx = std::max(mx, n), mn = std::min(mn, n);
  }
  o->max_block = mx, o->min_block = lv.nparts ? mn : 0;
  o->s_total = int64_t(lv.s_idx.size());
  o->factor_elems = lv.fac_elems;
  o->transfer = lv.transfer;
  o->subsolver = lv.subsolver;
  o->ilu_nnz = int64_t(lv.ilu_col.size());
  o->mls_restrict = lv.mls_restrict;
  o->p_nnz = int64_t(lv.p_col.size());
  o->r_nnz = int64_t(lv.pt_col.size());
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_hierarchy_csr(const nnms_hierarchy* h, int32_t level, int32_t* rp, int32_t* col) {
  ABI_BEGIN
  if (!h || !rp || !col || level < 0 || level >= h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  const HostLevel& lv = h->host.lev[level];
  std::memcpy(rp, lv.rp.data(), lv.rp.size() * sizeof(int32_t));
  std::memcpy(col, lv.col.data(), lv.col.size() * sizeof(int32_t));
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_hierarchy_partition(const nnms_hierarchy* h, int32_t level, int32_t* owner, int64_t* s_ptr,
                                                int32_t* s_idx) {
  ABI_BEGIN
  if (!h || !owner || !s_ptr || !s_idx || level < 0 || level >= h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  const HostLevel& lv = h->host.lev[level];
  std::memcpy(owner, lv.owner.data(), lv.owner.size() * sizeof(int32_t));
  std::memcpy(s_ptr, lv.s_ptr.data(), lv.s_ptr.size() * sizeof(int64_t));
  std::memcpy(s_idx, lv.s_idx.data(), lv.s_idx.size() * sizeof(int32_t));
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_hierarchy_transfer(const nnms_hierarchy* h, int32_t level, int32_t* idx, double* w) {
  ABI_BEGIN
  if (!h || !idx || !w || level < 0 || level + 1 >= h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  const HostLevel& lv = h->host.lev[level];
  if (lv.transfer != NNMS_TRANSFER_BARYCENTRIC)
    throw Error(NNMS_ERR_INVALID_ARG, "four-entry form exists for the barycentric transfer only");
  std::memcpy(idx, lv.p_idx.data(), lv.p_idx.size() * sizeof(int32_t));
  std::memcpy(w, lv.p_w.data(), lv.p_w.size() * sizeof(double));
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_hierarchy_transfer_csr(const nnms_hierarchy* h, int32_t level, int32_t* rp, int32_t* col,
                                                   double* w) {
  ABI_BEGIN
  if (!h || !rp || !col || !w || level < 0 || level + 1 >= h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  const HostLevel& lv = h->host.lev[level];
  std::memcpy(rp, lv.p_rp.data(), lv.p_rp.size() * sizeof(int32_t));
  std::memcpy(col, lv.p_col.data(), lv.p_col.size() * sizeof(int32_t));
  std::memcpy(w, lv.p_val.data(), lv.p_val.size() * sizeof(double));
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_hierarchy_restriction_csr(const nnms_hierarchy* h, int32_t level, int32_t* rp,
                                                      int32_t* col, double* w) {
  ABI_BEGIN
  if (!h || !rp || !col || !w || level < 0 || level + 1 >= h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  const HostLevel& lv = h->host.lev[level];
  std::memcpy(rp, lv.pt_rp.data(), lv.pt_rp.size() * sizeof(int32_t));
  std::memcpy(col, lv.pt_col.data(), lv.pt_col.size() * sizeof(int32_t));
  std::memcpy(w, lv.pt_w.data(), lv.pt_w.size() * sizeof(double));
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_hierarchy_ilu_pattern(const nnms_hierarchy* h, int32_t level, int32_t* rp, int32_t* col) {
  ABI_BEGIN
  if (!h || !rp || !col || level < 0 || level + 1 >= h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  const HostLevel& lv = h->host.lev[level];
  if (lv.subsolver != NNMS_SUBSOLVER_ILU) throw Error(NNMS_ERR_INVALID_ARG, "the level has no ILU subdomain solver");
  std::memcpy(rp, lv.ilu_rp.data(), lv.ilu_rp.size() * sizeof(int32_t));
  std::memcpy(col, lv.ilu_col.data(), lv.ilu_col.size() * sizeof(int32_t));
  return NNMS_OK;
  ABI_END
}

// Device memory of one assembly, allocation by allocation (each rounded up to
// 256 bytes, as the arena does): `resident` stays with the system,
// `transient` is held only while the assembly runs.  kappa_kind / rhs_kind
// select the per-tetrahedron and load arrays the assembly uploads.
struct SysLayout {
  int64_t resident = 0, transient = 0;
};
static int64_t round256(int64_t b) { return ((b ? b : 1) + 255) & ~int64_t(255); }

static SysLayout system_layout(const HostHierarchy& H, int prec, int cap, int kappa_kind, int rhs_kind) {
  SysLayout o;
  auto R = [&](int64_t b) { o.resident += round256(b); };
  auto T = [&](int64_t b) { o.transient += round256(b); };
  int64_t max_nt = 0;
  for (int l = 0; l < H.L; ++l) max_nt = std::max(max_nt, H.lev[l].nt);
  const int64_t K = H.opts.ncomp;
  T(max_nt * (16 * K * K + 1) * 8);  // element matrices and volumes
  T(sizeof(int));      // pivot error flag
  const int64_t tsz = prec == NNMS_FP64 ? 8 : 4;
  for (int l = 0; l < H.L; ++l) {
    const HostLevel& lv = H.lev[l];
    const bool coarse = (l == H.L - 1);
    const int64_t fsz = (coarse || prec == NNMS_FP64) ? 8 : 4;
    const int64_t nnz = int64_t(lv.col.size()), nell = int64_t(lv.sell_off.back());
    R(nnz * 8);
    if (prec == NNMS_MIXED) R(nnz * 4);
    R(nell * 8);
    if (prec == NNMS_MIXED) R(nell * 4);
    if (!coarse && lv.subsolver == NNMS_SUBSOLVER_ILU) {
      R(256), R(256), R(std::max<int64_t>(int64_t(lv.ilu_col.size()) * fsz, 256));
      T(int64_t(lv.nparts) * int64_t(sizeof(IluDesc)));
    } else {
      R(std::max<int64_t>(lv.fac_elems * fsz, 256)), R(lv.g_total * 16);
      if (lv.xinv) R(lv.xs_elems * fsz), R(lv.xp_elems * fsz), T(lv.x_elems * fsz);
      T(int64_t(lv.nparts) * int64_t(sizeof(FacDesc)));
    }
    R(lv.nv * tsz), R(lv.nv * tsz), R(lv.nv * tsz);
    if (l == 0) R(lv.nv * 8);  // load vector
    if (kappa_kind == 2) T(lv.nt * 8);
  }
  const int64_t n0 = H.lev[0].nv, nt0 = H.lev[0].nt;
  if (rhs_kind == 1) T(nt0 * K * 8);
  if (rhs_kind == 2) T(n0 * 8);
  const int64_t nblk = (n0 + VBLK - 1) / VBLK, nblkr = (n0 + 3) / 4;
  R(n0 * (cap + 1) * 8), R(n0 * cap * 8);  // Krylov bases V, Z
  R(n0 * 8), R(n0 * 8), R(n0 * 8);          // w, x, b
  R(nblk * (MMAX + 1) * 8), R(nblk * MMAX * 8), R(nblk * 8), R(nblkr * 8);
  R(int64_t(sizeof(KState)));
  return o;
}

extern "C" int64_t nnms_hierarchy_system_bytes(const nnms_hierarchy* h, int32_t restart) {
  if (!h || restart < 0 || restart > NNMS_MAX_RESTART) return -1;
  const HostHierarchy& H = h->host;
  // the larger of the two per-element-array choices of the load: per tetrahedron
  const SysLayout o = system_layout(H, H.opts.precision, restart ? restart : NNMS_MAX_RESTART, 2,
                                    H.lev[0].nt * H.opts.ncomp >= H.lev[0].nv ? 1 : 2);
  return o.resident + o.transient;
}

// Dense subdomain matrices of one level and their factorisation: zero fill
// of the tile storage, extraction of A[S_p, S_p], blocked LU.
struct FactorJob {
  std::vector<FacDesc> host;  // source of the upload, kept alive with the job
  FacDesc* d = nullptr;       // device array, one per subdomain
  int nd = 0, maxn = 0, maxN = 0;
  bool f64 = true;
  void* fac = nullptr;
  int64_t elems = 0;
  // inverse panels: X_p from the factors (forward steps over the owned tile
  // rows' span, then backward steps over all tile rows)
  void* x = nullptr;
  int64_t x_elems = 0;
  int maxNo = 0, fsteps = 0, bsteps = 0, maxPacked = 0;
};

static FactorJob factor_job(const nnms_system& sys, int l, Arena& mem, hipStream_t s) {
  const HostLevel& hl = sys.h->host.lev[l];
  if (l < sys.h->host.L - 1 && hl.subsolver == NNMS_SUBSOLVER_ILU)
    throw Error(NNMS_ERR_INVALID_ARG, "dense factorisation requested on an ILU level");
  const DevLevel& dl = sys.h->dev[l];
  const SysLevel& sl = sys.lev[l];
  FactorJob job;
  job.f64 = (l == sys.h->host.L - 1) || sys.prec == NNMS_FP64;
  const size_t fsz = job.f64 ? 8 : 4;
  // the full inverse panels exist only while the packed form is made
  void* xfull = hl.xinv ? mem.raw(size_t(hl.x_elems) * fsz) : nullptr;
  std::vector<FacDesc>& fd = job.host;
  for (int p = 0; p < hl.nparts; ++p) {
    FacDesc d{};
    d.fac = (char*)sl.fac + size_t(hl.fac_off[p]) * fsz;
    d.gidx = dl.gidx + hl.g_off[p];
    d.ext_rs = dl.ext_rs + hl.s_ptr[p];
    d.ext_lc = dl.ext_lc;
    d.rp = dl.rp;
    d.val = sl.val64;
    d.n = int(hl.s_ptr[p + 1] - hl.s_ptr[p]);
    d.N = hl.nblk[p];
    job.maxn = std::max(job.maxn, d.n), job.maxN = std::max(job.maxN, d.N);
    if (hl.xinv) {
      d.X = (char*)xfull + size_t(hl.x_off[p]) * fsz;
      d.Xs = (char*)sl.xinv + size_t(hl.xs_off[p]) * fsz;
      d.nv = d.n - hl.nown[p];
      d.No = (hl.nown[p] + TILE - 1) / TILE;
      job.maxNo = std::max(job.maxNo, d.No);
      job.fsteps = std::max(job.fsteps, d.N - d.nv / TILE);
      job.bsteps = std::max(job.bsteps, d.N);
      const int Nv = (d.nv + TILE - 1) / TILE;
      job.maxPacked = std::max(job.maxPacked, Nv * d.No + d.No * (d.No + 1) / 2);
    }
    fd.push_back(d);
  }
  if (hl.xinv) job.x = xfull, job.x_elems = hl.x_elems;
  job.d = mem.upload(fd, s);
  job.nd = int(fd.size());
  job.fac = sl.fac;
  job.elems = hl.fac_elems;
  return job;
}

template <typename F>
static hipError_t enqueue_factor_t(const FactorJob& j, int* err, hipStream_t s) {
  hipError_t e;
  if ((e = launch_fill<F>((F*)j.fac, j.elems, F(0), s)) != hipSuccess) return e;
  if ((e = launch_extract<F>(j.d, j.nd, j.maxn, s)) != hipSuccess) return e;
  if ((e = launch_lu<F>(j.d, j.nd, j.maxN, err, s)) != hipSuccess) return e;
  if (!j.x) return hipSuccess;
  if ((e = launch_fill<F>((F*)j.x, j.x_elems, F(0), s)) != hipSuccess) return e;
  if ((e = launch_xinv<F>(j.d, j.nd, j.maxNo, j.fsteps, j.bsteps, s)) != hipSuccess) return e;
  return launch_xpack<F>(j.d, j.nd, j.maxPacked, s);
}

static hipError_t enqueue_factor(const FactorJob& j, int* err, hipStream_t s) {
  return j.f64 ? enqueue_factor_t<double>(j, err, s) : enqueue_factor_t<float>(j, err, s);
}

// ILU factors of one level: values from the level's CSR (0 on fill), then
// the level-scheduled factorisation, one work-group per subdomain.
struct IluJob {
  std::vector<IluDesc> host;
  IluDesc* d = nullptr;
  int nd = 0, lanes = 4;
  bool f64 = true;
  const int32_t* asrc = nullptr;
  const double* a = nullptr;
  void* val = nullptr;
  int64_t nnz = 0;
};

static IluJob ilu_job(const nnms_system& sys, int l, Arena& mem, hipStream_t s) {
  IluJob job;
  job.f64 = sys.prec == NNMS_FP64;
  job.host = ilu_descs(sys, l, false);
  job.d = mem.upload(job.host, s);
  job.nd = int(job.host.size());
  job.asrc = sys.h->dev[l].ilu_asrc;
  job.a = sys.lev[l].val64;
  job.val = sys.lev[l].ilu_val;
  job.nnz = int64_t(sys.h->host.lev[l].ilu_col.size());
  job.lanes = sys.h->host.lev[l].ilu_lanes;
  return job;
}

static hipError_t enqueue_ilu(const IluJob& j, int* err, hipStream_t s) {
  hipError_t e;
  if (j.f64) {
    if ((e = launch_ilu_extract<double>(j.asrc, j.a, (double*)j.val, j.nnz, s)) != hipSuccess) return e;
    return launch_ilu_factor<double>(j.d, j.nd, j.lanes, err, s);
  }
  if ((e = launch_ilu_extract<float>(j.asrc, j.a, (float*)j.val, j.nnz, s)) != hipSuccess) return e;
  return launch_ilu_factor<float>(j.d, j.nd, j.lanes, err, s);
}

// Per-device stream on which assemblies run their coarse levels'
// factorisations beside the fine level's (created once, never destroyed:
// destroying a stream waits for the device).  Only ever waits on events
// recorded before, so assemblies on several threads may share it.
static hipStream_t assembly_side_stream() {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Error(NNMS_ERR_INVALID_ARG, "device id out of range");
  std::lock_guard<std::mutex> g(mu);
  if (!streams[dev]) HIP_CHECK(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
  return streams[dev];
}

static bool all_finite(const double* v, int64_t n, bool positive) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i]) || (positive && !(v[i] > 0))) return false;
  return true;
}

extern "C" nnms_status nnms_assemble_ex(nnms_hierarchy* h, const nnms_assemble_opts* o, void* stream,
                                        nnms_system** out) {
  ABI_BEGIN
  if (!h || !o || !o->kappa || !out) throw Error(NNMS_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (!h->on_device) throw Error(NNMS_ERR_INVALID_ARG, "hierarchy was set up without a device");
  const nnms_kappa* k = o->kappa;
  const HostHierarchy& H = h->host;
  const int L = H.L, prec = H.opts.precision;
  KappaDev kd{};
  kd.kind = k->kind;
  if (k->kind == 0) {
    if (!(k->value > 0) || !std::isfinite(k->value)) throw Error(NNMS_ERR_INVALID_ARG, "kappa must be positive");
    kd.value = k->value;
  } else if (k->kind == 1) {
    if (k->ncentres < 0 || k->ncentres > MAXC || !(k->width > 0) || (k->ncentres && (!k->centres || !k->mu)))
      throw Error(NNMS_ERR_INVALID_ARG, "bad log-Gaussian kappa");
    kd.nc = k->ncentres, kd.width = k->width, kd.value = 1.0;
    for (int c = 0; c < kd.nc; ++c) {
      for (int a = 0; a < 3; ++a) kd.c[3 * c + a] = k->centres[3 * c + a];
      kd.mu[c] = k->mu[c];
    }
  } else if (k->kind == 2) {
    if (!k->per_tet) throw Error(NNMS_ERR_INVALID_ARG, "per-tetrahedron kappa needs one array per level");
    for (int l = 0; l < L; ++l)
      if (!k->per_tet[l] || !all_finite(k->per_tet[l], H.lev[l].nt, true))
        throw Error(NNMS_ERR_INVALID_ARG, "per-tetrahedron kappa of level " + std::to_string(l) +
                                              " must be finite and positive");
  } else {
    throw Error(NNMS_ERR_INVALID_ARG, "unknown kappa kind");
  }
  nnms_rhs rhs{};
  rhs.kind = 0, rhs.value = 1.0;
  if (o->rhs) rhs = *o->rhs;
  if (rhs.kind == 0) {
    if (!std::isfinite(rhs.value)) throw Error(NNMS_ERR_INVALID_ARG, "the load must be finite");
  } else if (rhs.kind == 1 || rhs.kind == 2) {
    const int64_t n = rhs.kind == 1 ? H.lev[0].nt * H.opts.ncomp : H.lev[0].nv;
    if (!rhs.values || !all_finite(rhs.values, n, false))
      throw Error(NNMS_ERR_INVALID_ARG, "load values missing or not finite");
  } else {
    throw Error(NNMS_ERR_INVALID_ARG, "unknown load kind");
  }
  const int K = H.opts.ncomp;
  if (K == 3 && !(o->poisson_ratio >= 0.0 && o->poisson_ratio < 0.5))
    throw Error(NNMS_ERR_INVALID_ARG, "Poisson's ratio must lie in [0, 0.5)");
  if (rhs.kind == 0 && K == 3 && !all_finite(rhs.vector, 3, false))
    throw Error(NNMS_ERR_INVALID_ARG, "the body force must be finite");
  const int cap = o->restart_cap ? o->restart_cap : NNMS_MAX_RESTART;
  if (cap < 1 || cap > NNMS_MAX_RESTART) throw Error(NNMS_ERR_INVALID_ARG, "restart_cap out of range");
  if (o->max_device_bytes < 0) throw Error(NNMS_ERR_INVALID_ARG, "negative device-memory budget");
  if (o->max_device_bytes > 0) {
    const int64_t need = nnms_hierarchy_system_bytes(h, cap);
    if (need > o->max_device_bytes)
      throw Error(NNMS_ERR_BUDGET, "the assembly needs up to " + std::to_string(need) +
                                       " device bytes, the budget is " + std::to_string(o->max_device_bytes));
  }
  hipStream_t s = (hipStream_t)stream;
  auto sys = std::unique_ptr<nnms_system>(new nnms_system);
  sys->h = h;
  h->systems++;
  sys->prec = prec;
  HIP_CHECK(hipGetDevice(&sys->dev));
  sys->mem = std::make_unique<Arena>(h->has_alloc ? &h->alloc : nullptr);
  Arena& A = *sys->mem;
  sys->lev.resize(L);
  const size_t tsz = prec == NNMS_FP64 ? 8 : 4;
  int64_t max_nt = 0;
  for (int l = 0; l < L; ++l) max_nt = std::max(max_nt, H.lev[l].nt);
  Arena scratch(h->has_alloc ? &h->alloc : nullptr);
  std::vector<FactorJob> fac_jobs;
  std::vector<IluJob> ilu_jobs;
  std::vector<int> job_level;
  double* elem = scratch.alloc<double>(size_t(max_nt) * (16 * K * K + 1), s, false);
  int* err = scratch.alloc<int>(1, s);
  const double* fval = nullptr;
  if (rhs.kind != 0) {
    const int64_t n = rhs.kind == 1 ? H.lev[0].nt * K : H.lev[0].nv;
    fval = scratch.upload(std::vector<double>(rhs.values, rhs.values + n), s);
  }
  for (int l = 0; l < L; ++l) {
    const HostLevel& hl = H.lev[l];
    const DevLevel& dl = h->dev[l];
    SysLevel& sl = sys->lev[l];
    const bool coarse = (l == L - 1);
    const size_t fsz = (coarse || prec == NNMS_FP64) ? 8 : 4;
    sl.val64 = A.alloc<double>(hl.col.size(), s, false);
    if (prec == NNMS_MIXED) sl.val32 = A.alloc<float>(hl.col.size(), s, false);
    const int64_t nell = int64_t(hl.sell_off.back());
    sl.ell64 = A.alloc<double>(nell, s, false);
    if (prec == NNMS_MIXED) sl.ell32 = A.alloc<float>(nell, s, false);
    const bool ilu = !coarse && hl.subsolver == NNMS_SUBSOLVER_ILU;
    if (ilu) {
      sl.fac = A.raw(256);
      sl.yx = A.raw(256);
      sl.ilu_val = A.raw(std::max<size_t>(hl.ilu_col.size() * fsz, 256));
    } else {
      sl.fac = A.raw(std::max<size_t>(size_t(hl.fac_elems) * fsz, 256));
      sl.yx = A.alloc<char>(size_t(hl.g_total) * 16, s);  // tagged block results: 16 bytes per value
      if (hl.xinv) sl.xinv = A.raw(size_t(hl.xs_elems) * fsz), sl.xpart = A.raw(size_t(hl.xp_elems) * fsz);
    }
    sl.r = A.alloc<char>(hl.nv * tsz, s);
    sl.z = A.alloc<char>(hl.nv * tsz, s);
    sl.t = A.alloc<char>(hl.nv * tsz, s);
    AsmDesc ad{};
    ad.xyz = dl.xyz, ad.tets = dl.tets, ad.cptr = dl.cptr, ad.citem = dl.citem, ad.rp = dl.rp;
    ad.vptr = dl.vptr, ad.vitem = dl.vitem, ad.dmask = dl.dmask, ad.elem = elem;
    ad.val64 = sl.val64, ad.val32 = sl.val32, ad.nt = hl.nt, ad.nv = hl.nv;
    ad.ncomp = K, ad.nu = o->poisson_ratio;
    for (int c = 0; c < 3; ++c) ad.fvec[c] = rhs.vector[c];
    if (k->kind == 2) ad.kappa_tet = scratch.upload(std::vector<double>(k->per_tet[l], k->per_tet[l] + hl.nt), s);
    if (l == 0) {
      sys->b0 = A.alloc<double>(hl.nv, s, false);
      ad.b = sys->b0;
      ad.fkind = rhs.kind;
      ad.fval = fval;
    }
    HIP_CHECK(launch_assemble(ad, kd, rhs.value, s));
    HIP_CHECK(launch_gather_ell<double>(dl.sell_src, sl.val64, sl.ell64, nell, s));
    if (sl.ell32) HIP_CHECK(launch_gather_ell<float>(dl.sell_src, sl.val64, sl.ell32, nell, s));
    if (ilu)
      ilu_jobs.push_back(ilu_job(*sys, l, scratch, s));  // ILU(k) values and factorisation
    else
      fac_jobs.push_back(factor_job(*sys, l, scratch, s));  // dense subdomain matrices and factors
    job_level.push_back(l);
  }
  // The levels' factorisations are independent: the finest on `s`, the
  // coarser ones on the library's side stream beside it (their launches are
  // short and latency-bound and fill gaps of the fine level's), joined back
  // into `s` before the system is handed out.
  {
    hipStream_t side = assembly_side_stream();
    hipEvent_t assembled, factored;
    HIP_CHECK(hipEventCreateWithFlags(&assembled, hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&factored, hipEventDisableTiming));
    HIP_CHECK(hipEventRecord(assembled, s));
    HIP_CHECK(hipStreamWaitEvent(side, assembled, 0));
    size_t fi = 0, ii = 0;
    for (int l : job_level) {
      const bool ilu = l < L - 1 && H.lev[l].subsolver == NNMS_SUBSOLVER_ILU;
      hipStream_t st = l == 0 ? s : side;
      if (ilu)
        HIP_CHECK(enqueue_ilu(ilu_jobs[ii++], err, st));
      else
        HIP_CHECK(enqueue_factor(fac_jobs[fi++], err, st));
    }
    HIP_CHECK(hipEventRecord(factored, side));
    HIP_CHECK(hipStreamWaitEvent(s, factored, 0));
    (void)hipEventDestroy(assembled);
    (void)hipEventDestroy(factored);
  }
  // solve workspace: Krylov bases of restart_cap columns
  const int64_t n0 = H.lev[0].nv;
  sys->restart_cap = cap;
  sys->nblk = vec_blocks(n0);
  sys->nblkr = spmv_blocks(n0, 64);  // most blocks of any lanes-per-row choice (4 rows per block)
  sys->V = A.alloc<double>(size_t(n0) * (cap + 1), s, false);
  sys->Z = A.alloc<double>(size_t(n0) * cap, s, false);
  sys->w = A.alloc<double>(n0, s);
  sys->x = A.alloc<double>(n0, s);
  sys->bw = A.alloc<double>(n0, s);
  sys->part1 = A.alloc<double>(size_t(sys->nblk) * (MMAX + 1), s);
  sys->part2 = A.alloc<double>(size_t(sys->nblk) * MMAX, s);
  sys->partn = A.alloc<double>(sys->nblk, s);
  sys->partr = A.alloc<double>(sys->nblkr, s);
  sys->st = (KState*)A.alloc<char>(sizeof(KState), s);
  {
    const int32_t idle = ST_IDLE;
    HIP_CHECK(hipMemcpyAsync(&sys->st->status, &idle, sizeof idle, hipMemcpyHostToDevice, s));
  }
  int herr = 0;
  HIP_CHECK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  if (herr) throw Error(NNMS_ERR_SINGULAR, "non-positive pivot in a subdomain or coarse factorisation");
  *out = sys.release();
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_assemble(nnms_hierarchy* h, const nnms_kappa* k, double f, void* stream, nnms_system** out) {
  nnms_rhs rhs{};
  rhs.kind = 0, rhs.value = f;
  rhs.vector[0] = rhs.vector[1] = rhs.vector[2] = f;
  nnms_assemble_opts o{};
  o.kappa = k, o.rhs = &rhs, o.poisson_ratio = 0.3;
  return nnms_assemble_ex(h, &o, stream, out);
}

extern "C" nnms_status nnms_system_destroy(nnms_system* s) {
  delete s;
  return NNMS_OK;
}

extern "C" int64_t nnms_system_device_bytes(const nnms_system* s) { return s && s->mem ? int64_t(s->mem->total) : 0; }

extern "C" nnms_status nnms_system_rhs(const nnms_system* s, double* b) {
  ABI_BEGIN
  if (!s || !b) throw Error(NNMS_ERR_INVALID_ARG, "null argument");
  HIP_CHECK(hipMemcpy(b, s->b0, s->h->host.lev[0].nv * sizeof(double), hipMemcpyDeviceToHost));
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_system_matrix(const nnms_system* s, int32_t level, double* val) {
  ABI_BEGIN
  if (!s || !val || level < 0 || level >= s->h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  HIP_CHECK(hipMemcpy(val, s->lev[level].val64, s->h->host.lev[level].col.size() * sizeof(double), hipMemcpyDeviceToHost));
  return NNMS_OK;
  ABI_END
}

// ---------------------------------------------------------------------------
// single operator applications (host vectors, FP64 at the boundary)
// ---------------------------------------------------------------------------
static Plan& apply_plan(nnms_system* s) {
  if (!s->apply) s->apply = make_plan_any({s}, false);
  return *s->apply;
}

static void put_vec(nnms_system* s, void* dst, const double* src, int64_t n, hipStream_t st) {
  if (s->prec == NNMS_FP64) {
    HIP_CHECK(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, st));
  } else {
    std::vector<float> tmp(src, src + n);
    HIP_CHECK(hipMemcpyAsync(dst, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
    HIP_CHECK(hipStreamSynchronize(st));
  }
}
static void get_vec(nnms_system* s, double* dst, const void* src, int64_t n, hipStream_t st) {
  if (s->prec == NNMS_FP64) {
    HIP_CHECK(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
  } else {
    std::vector<float> tmp(n);
    HIP_CHECK(hipMemcpyAsync(tmp.data(), src, n * sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; ++i) dst[i] = tmp[i];
  }
}
static size_t tsize(const nnms_system* s) { return s->prec == NNMS_FP64 ? 8 : 4; }

extern "C" nnms_status nnms_apply_operator(nnms_system* s, int32_t level, const double* x, double* y, void* stream) {
  ABI_BEGIN
  if (!s || !x || !y || level < 0 || level >= s->h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  Plan& P = apply_plan(s);
  join_in((hipStream_t)stream, P.stream);
  const int64_t n = s->h->host.lev[level].nv;
  SysLevel& sl = s->lev[level];
  const DevLevel& dl = s->h->dev[level];
  put_vec(s, sl.z, x, n, P.stream);
  SpmvDesc d{};
  d.rp = dl.rp, d.col = dl.col, d.x = sl.z, d.y = sl.t, d.n = int(n), d.blk0 = 0, d.when = WHEN_RUNNING;
  d.val = s->prec == NNMS_FP64 ? (const void*)sl.val64 : (const void*)sl.val32;
  Arena tmp;
  std::vector<SpmvDesc> v{d};
  SpmvDesc* dd = tmp.upload(v, P.stream);
  if (s->prec == NNMS_FP64)
    HIP_CHECK(launch_spmv<double>(dd, 1, spmv_blocks(n, SPMV_G_A), SPMV_G_A, P.stream));
  else
    HIP_CHECK(launch_spmv<float>(dd, 1, spmv_blocks(n, SPMV_G_A), SPMV_G_A, P.stream));
  get_vec(s, y, sl.t, n, P.stream);
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_apply_smoother(nnms_system* s, int32_t level, const double* r, double* z, void* stream) {
  ABI_BEGIN
  if (!s || !r || !z || level < 0 || level >= s->h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  Plan& P = apply_plan(s);
  join_in((hipStream_t)stream, P.stream);
  const int64_t n = s->h->host.lev[level].nv;
  SysLevel& sl = s->lev[level];
  put_vec(s, sl.r, r, n, P.stream);
  HIP_CHECK(hipMemsetAsync(sl.z, 0, n * tsize(s), P.stream));
  if (level == s->h->host.L - 1) {
    if (s->prec == NNMS_FP64)
      HIP_CHECK((launch_ras_groups<double, double>(P.coarse, false, P.stream)));
    else
      HIP_CHECK((launch_ras_groups<double, float>(P.coarse, false, P.stream)));
  } else {
    if (s->prec == NNMS_FP64)
      HIP_CHECK(launch_smoother_level<double>(P.lev[level], false, P.stream));
    else
      HIP_CHECK(launch_smoother_level<float>(P.lev[level], false, P.stream));
  }
  get_vec(s, z, sl.z, n, P.stream);
  check_counters(P, P.stream);
  return NNMS_OK;
  ABI_END
}

// ---------------------------------------------------------------------------
// smoother application for callers that cannot allocate device memory
// ---------------------------------------------------------------------------
// The tables of one smoother launch (counter words, subdomain or ILU
// descriptors, task list) live in this file-scope array instead of memory the
// library allocates: one copy per GPU, held until the process ends.  Host code
// never uses the array's name as an address: each device's address comes
// from hipGetSymbolAddress, with that device current, on its first use.
static __device__ __align__(256) unsigned char scratch[NNMS_NOALLOC_SCRATCH_BYTES];

namespace nnms {
constexpr int kMaxDevices = 64;
constexpr size_t kScratchTables = 256;  // offset of the descriptors (counter words first)
struct ScratchTable {
  std::mutex mu;
  char* ptr[kMaxDevices] = {};
};
static ScratchTable& scratch_table() {
  static ScratchTable* t = new ScratchTable();  // never destroyed: outlives every call
  return *t;
}

// device address of this device's `scratch`; on the first call per device its
// counter words are zeroed and given the first launch epoch
static char* scratch_on(int dev, hipStream_t s) {
  if (dev < 0 || dev >= kMaxDevices) throw Error(NNMS_ERR_INVALID_ARG, "device id out of range");
  ScratchTable& T = scratch_table();
  std::lock_guard<std::mutex> g(T.mu);
  if (!T.ptr[dev]) {
    void* p = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    HIP_CHECK(launch_ras_seed((int32_t*)p, s));
    HIP_CHECK(hipStreamSynchronize(s));
    T.ptr[dev] = (char*)p;
  }
  return T.ptr[dev];
}

template <typename T>
static void noalloc_smoother(nnms_system* s, int level, const double* r, double* z, hipStream_t st) {
  const HostHierarchy& H = s->h->host;
  const HostLevel& hl = H.lev[level];
  const bool coarse = level == H.L - 1;
  const bool ilu = !coarse && hl.subsolver == NNMS_SUBSOLVER_ILU;
  SysLevel& sl = s->lev[level];
  const int64_t n = hl.nv;
  // host images of the launch's tables, sized against the scratch array
  // before any device work
  std::vector<SubDesc> subs, unused;
  std::vector<IluDesc> ilus;
  std::vector<int32_t> Ns, B0s, tasks;
  const int K = ras_kind(s, level);
  size_t desc_bytes = 0;
  if (ilu) {
    ilus = ilu_descs(*s, level, false);
    desc_bytes = ilus.size() * sizeof(IluDesc);
  } else {
    ras_subdescs({s}, level, coarse, s->prec, false, subs, unused, Ns, B0s);
    tasks = K == 0 ? xpanel_tasks(subs) : ras_tasks(Ns, B0s, K);
    desc_bytes = subs.size() * sizeof(SubDesc);
  }
  const size_t task_off = kScratchTables + ((desc_bytes + 255) & ~size_t(255));
  const size_t need = task_off + tasks.size() * sizeof(int32_t);
  if (need > NNMS_NOALLOC_SCRATCH_BYTES)
    throw Error(NNMS_ERR_INVALID_ARG, "the level's smoother tables need " + std::to_string(need) +
                                          " bytes of scratch, the maximum is " +
                                          std::to_string(size_t(NNMS_NOALLOC_SCRATCH_BYTES)));
  char* sp = scratch_on(s->dev, st);
  int32_t* counter = (int32_t*)sp;
  // input in the level's working precision, output zeroed (Dirichlet rows stay 0)
  if (std::is_same<T, double>::value)
    HIP_CHECK(hipMemcpyAsync(sl.r, r, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  else
    HIP_CHECK(launch_cast_d2f(r, (float*)sl.r, n, st));
  HIP_CHECK(launch_fill<T>((T*)sl.z, n, T(0), st));
  if (ilu) {
    int maxn = 0;
    for (const IluDesc& d : ilus) maxn = std::max(maxn, int(d.n));
    HIP_CHECK(hipMemcpyAsync(sp + kScratchTables, ilus.data(), desc_bytes, hipMemcpyHostToDevice, st));
    HIP_CHECK(launch_ilu_apply<T>((const IluDesc*)(sp + kScratchTables), int(ilus.size()), maxn, hl.ilu_lanes, 0, st));
  } else {
    HIP_CHECK(hipMemcpyAsync(sp + kScratchTables, subs.data(), desc_bytes, hipMemcpyHostToDevice, st));
    HIP_CHECK(hipMemcpyAsync(sp + task_off, tasks.data(), tasks.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    RasLaunch rl{};
    rl.subs = (const SubDesc*)(sp + kScratchTables);
    rl.tasks = (const int32_t*)(sp + task_off);
    rl.counter = counter;
    rl.ntasks = int(tasks.size());
    rl.add = 0;
    rl.group = K;
    for (int32_t nb : Ns) rl.max_tiles = std::max(rl.max_tiles, nb);
    const int g = s->h->tune.ras_groups[level];
    if (coarse)
      HIP_CHECK((launch_ras<double, T>(rl, g > 0 ? g : ras_grid_default(), st)));
    else
      HIP_CHECK((launch_ras<T, T>(rl, g > 0 ? g : ras_grid_default(), st)));
  }
  if (std::is_same<T, double>::value)
    HIP_CHECK(hipMemcpyAsync(z, sl.z, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  else
    HIP_CHECK(launch_cast_f2d((const float*)sl.z, z, n, st));
  int32_t werr = 0;
  HIP_CHECK(hipMemcpyAsync(&werr, counter + 2, sizeof werr, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  if (werr) {
    HIP_CHECK(launch_ras_seed(counter, st));  // clears the error word for later calls
    HIP_CHECK(hipStreamSynchronize(st));
    throw Error(NNMS_ERR_DEVICE, "triangular-solve wait limit exceeded (error bits " + std::to_string(werr) + ")");
  }
}
}  // namespace nnms

extern "C" nnms_status nnms_apply_smoother_noalloc(nnms_system* s, int32_t level, const double* r_dev, double* z_dev,
                                                   void* stream) {
  ABI_BEGIN
  if (!s || !r_dev || !z_dev || level < 0 || level >= s->h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  int dev = -1;
  HIP_CHECK(hipGetDevice(&dev));
  if (dev != s->dev) throw Error(NNMS_ERR_INVALID_ARG, "the current device is not the system's");
  if (s->prec == NNMS_FP64)
    noalloc_smoother<double>(s, level, r_dev, z_dev, (hipStream_t)stream);
  else
    noalloc_smoother<float>(s, level, r_dev, z_dev, (hipStream_t)stream);
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_apply_prolong(nnms_system* s, int32_t level, const double* x, double* y, void* stream) {
  ABI_BEGIN
  if (!s || !x || !y || level < 0 || level + 1 >= s->h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  Plan& P = apply_plan(s);
  join_in((hipStream_t)stream, P.stream);
  const int64_t nf = s->h->host.lev[level].nv, nc = s->h->host.lev[level + 1].nv;
  put_vec(s, s->lev[level + 1].z, x, nc, P.stream);
  HIP_CHECK(hipMemsetAsync(s->lev[level].z, 0, nf * tsize(s), P.stream));
  if (s->prec == NNMS_FP64)
    HIP_CHECK(launch_prolong_level<double>(P.lev[level], P.stream));
  else
    HIP_CHECK(launch_prolong_level<float>(P.lev[level], P.stream));
  get_vec(s, y, s->lev[level].z, nf, P.stream);
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_apply_restrict(nnms_system* s, int32_t level, const double* x, double* y, void* stream) {
  ABI_BEGIN
  if (!s || !x || !y || level < 0 || level + 1 >= s->h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  Plan& P = apply_plan(s);
  join_in((hipStream_t)stream, P.stream);
  const int64_t nf = s->h->host.lev[level].nv, nc = s->h->host.lev[level + 1].nv;
  put_vec(s, s->lev[level].t, x, nf, P.stream);
  if (s->prec == NNMS_FP64)
    HIP_CHECK(launch_spmv_groups<double>(P.lev[level].rst, P.stream));
  else
    HIP_CHECK(launch_spmv_groups<float>(P.lev[level].rst, P.stream));
  get_vec(s, y, s->lev[level + 1].r, nc, P.stream);
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_apply_vcycle(nnms_system* s, const double* r, double* z, void* stream) {
  ABI_BEGIN
  if (!s || !r || !z) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  Plan& P = apply_plan(s);
  join_in((hipStream_t)stream, P.stream);
  const int64_t n = s->h->host.lev[0].nv;
  put_vec(s, s->lev[0].r, r, n, P.stream);
  for (int l = 0; l < s->h->host.L; ++l) HIP_CHECK(hipMemsetAsync(s->lev[l].z, 0, s->h->host.lev[l].nv * tsize(s), P.stream));
  if (s->prec == NNMS_FP64)
    enqueue_vcycle<double>(P, P.stream);
  else
    enqueue_vcycle<float>(P, P.stream);
  get_vec(s, z, s->lev[0].z, n, P.stream);
  check_counters(P, P.stream);
  return NNMS_OK;
  ABI_END
}

// ---------------------------------------------------------------------------
// solves
// ---------------------------------------------------------------------------
extern "C" nnms_status nnms_solve_opts_default(nnms_solve_opts* o) {
  if (!o) return NNMS_ERR_INVALID_ARG;
  std::memset(o, 0, sizeof *o);
  o->restart = 30;
  o->max_it = 1000;
  o->rtol = 1e-8;
  return NNMS_OK;
}

struct nnms_batch {
  std::unique_ptr<Plan> plan;
  nnms_solve_opts opts{};
  hipStream_t user = nullptr;  // the caller's stream: start and result are ordered with its work
};

// Steps until no slot is running: first as many as the plan's last solve
// took (at most MAX_GRAPH_STEPS), back to back with one host read of the
// active count (parametric solves of one system take about the same number),
// then one at a time.
constexpr int MAX_GRAPH_STEPS = 64;
static void run_plan(Plan& P, int max_steps) {
  int k = 0;
  int K = std::max(1, std::min({P.expect, max_steps, MAX_GRAPH_STEPS}));
  while (k < max_steps) {
    plan_steps(P, K);
    k += K;
    if (plan_active(P) == 0) return;
    K = 1;
  }
}

static nnms_solve_info read_info(nnms_system* s, hipStream_t st) {
  KState ks;
  HIP_CHECK(hipMemcpyAsync(&ks, s->st, sizeof(KState), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  nnms_solve_info in{};
  in.iterations = ks.its;
  in.cycles = ks.cycles;
  in.relres = ks.relres;
  in.status = ks.status == ST_CONVERGED ? NNMS_OK : NNMS_ERR_NOT_CONVERGED;
  in.running = ks.status == ST_RUNNING ? 1 : 0;
  return in;
}

static nnms_status solve_many(nnms_system* const* systems, int32_t nb, const double* const* b, double* const* x,
                              const nnms_solve_opts* opts, nnms_solve_info* infos, void* stream, bool use_solo) {
  nnms_solve_opts o;
  if (opts)
    o = *opts;
  else
    nnms_solve_opts_default(&o);
  validate_solve_opts(o);
  if (!systems || nb < 1 || !b || !x) throw Error(NNMS_ERR_INVALID_ARG, "null argument");
  std::vector<nnms_system*> sys(systems, systems + nb);
  for (auto* s : sys)
    if (!s) throw Error(NNMS_ERR_INVALID_ARG, "null system");
  check_restart(sys, o);
  std::unique_ptr<Plan> local;
  Plan* P;
  if (use_solo) {
    if (!sys[0]->solo) sys[0]->solo = make_plan_any(sys, true);
    P = sys[0]->solo.get();
  } else {
    local = make_plan_any(sys, true);
    P = local.get();
  }
  P->use_graph = !(o.flags & NNMS_NO_GRAPH);
  hipStream_t user = (hipStream_t)stream;
  join_in(user, P->stream);
  const bool dev = (o.flags & NNMS_DEVICE_PTRS) != 0;
  for (int k = 0; k < nb; ++k) {
    nnms_system* s = sys[k];
    const int64_t n = s->h->host.lev[0].nv;
    if (dev) {
      plan_start_slot(*P, k, b[k], o);
    } else {
      HIP_CHECK(hipMemcpyAsync(s->bw, b[k], n * sizeof(double), hipMemcpyHostToDevice, P->stream));
      HIP_CHECK(hipStreamSynchronize(P->stream));
      plan_start_slot(*P, k, s->bw, o);
    }
  }
  // with an expected step count the first read is skipped: steps leave
  // slots that are not running (a zero right-hand side) unchanged
  if (P->expect > 0 || plan_active(*P) > 0) run_plan(*P, o.max_it + 1);
  check_counters(*P, P->stream);
  nnms_status worst = NNMS_OK;
  int most_its = 0;
  for (int k = 0; k < nb; ++k) {
    nnms_system* s = sys[k];
    const int64_t n = s->h->host.lev[0].nv;
    HIP_CHECK(hipMemcpyAsync(x[k], s->x, n * sizeof(double), dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             P->stream));
    nnms_solve_info in = read_info(s, P->stream);
    if (infos) infos[k] = in;
    if (in.status != NNMS_OK) worst = NNMS_ERR_NOT_CONVERGED;
    most_its = std::max(most_its, int(in.iterations));
  }
  HIP_CHECK(hipStreamSynchronize(P->stream));
  P->expect = most_its;
  if (worst != NNMS_OK) nnms::set_last_error("iteration limit reached before the tolerance");
  return worst;
}

extern "C" nnms_status nnms_solve(nnms_system* s, const double* b, double* x, const nnms_solve_opts* opts,
                                  nnms_solve_info* info, void* stream) {
  ABI_BEGIN
  if (!s || !b || !x) throw Error(NNMS_ERR_INVALID_ARG, "null argument");
  return solve_many(&s, 1, &b, &x, opts, info, stream, true);
  ABI_END
}

extern "C" nnms_status nnms_solve_batch(nnms_system* const* systems, int32_t nb, const double* const* b, double* const* x,
                                        const nnms_solve_opts* opts, nnms_solve_info* infos, void* stream) {
  ABI_BEGIN
  return solve_many(systems, nb, b, x, opts, infos, stream, false);
  ABI_END
}

extern "C" nnms_status nnms_batch_create(nnms_system* const* systems, int32_t nb, const nnms_solve_opts* opts,
                                         void* stream, nnms_batch** out) {
  ABI_BEGIN
  if (!systems || nb < 1 || !out) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  *out = nullptr;
  auto bt = std::make_unique<nnms_batch>();
  if (opts)
    bt->opts = *opts;
  else
    nnms_solve_opts_default(&bt->opts);
  validate_solve_opts(bt->opts);
  std::vector<nnms_system*> sys(systems, systems + nb);
  for (auto* s : sys)
    if (!s) throw Error(NNMS_ERR_INVALID_ARG, "null system");
  check_restart(sys, bt->opts);
  bt->plan = make_plan_any(sys, true);
  bt->plan->use_graph = !(bt->opts.flags & NNMS_NO_GRAPH);
  bt->user = (hipStream_t)stream;
  join_in(bt->user, bt->plan->stream);
  // slots keep their systems' solve state: a freshly assembled system is
  // idle, a system still iterating in an earlier batch goes on here
  HIP_CHECK(hipStreamSynchronize(bt->plan->stream));
  *out = bt.release();
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_batch_start(nnms_batch* bt, int32_t slot, const double* b_dev) {
  ABI_BEGIN
  if (!bt || !b_dev || slot < 0 || slot >= bt->plan->nd) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  join_in(bt->user, bt->plan->stream);  // b as the caller's stream has it now
  plan_start_slot(*bt->plan, slot, b_dev, bt->opts);
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_batch_step(nnms_batch* bt, int32_t iterations, int32_t* active) {
  ABI_BEGIN
  if (!bt || iterations < 0) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  int a = plan_active(*bt->plan);
  for (int k = 0; k < iterations && a > 0; ++k) {
    plan_step(*bt->plan);
    a = plan_active(*bt->plan);
  }
  check_counters(*bt->plan, bt->plan->stream);
  if (active) *active = a;
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_batch_result(nnms_batch* bt, int32_t slot, double* x_dev, nnms_solve_info* info) {
  ABI_BEGIN
  if (!bt || slot < 0 || slot >= bt->plan->nd) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  nnms_system* s = bt->plan->sys[slot];
  if (x_dev) {
    // after the caller's stream has finished its earlier work on x, and
    // before its later work
    join_in(bt->user, bt->plan->stream);
    HIP_CHECK(hipMemcpyAsync(x_dev, s->x, s->h->host.lev[0].nv * sizeof(double), hipMemcpyDeviceToDevice,
                             bt->plan->stream));
    join_in(bt->plan->stream, bt->user);
  }
  nnms_solve_info in = read_info(s, bt->plan->stream);
  if (info) *info = in;
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_batch_destroy(nnms_batch* bt) {
  if (bt && bt->plan) (void)hipStreamSynchronize(bt->plan->stream);
  delete bt;
  return NNMS_OK;
}

extern "C" nnms_status nnms_system_ilu_values(const nnms_system* s, int32_t level, double* val) {
  ABI_BEGIN
  if (!s || !val || level < 0 || level + 1 >= s->h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  const HostLevel& hl = s->h->host.lev[level];
  if (hl.subsolver != NNMS_SUBSOLVER_ILU) throw Error(NNMS_ERR_INVALID_ARG, "the level has no ILU subdomain solver");
  const size_t n = hl.ilu_col.size();
  if (s->prec == NNMS_FP64) {
    HIP_CHECK(hipMemcpy(val, s->lev[level].ilu_val, n * sizeof(double), hipMemcpyDeviceToHost));
  } else {
    std::vector<float> f(n);
    HIP_CHECK(hipMemcpy(f.data(), s->lev[level].ilu_val, n * sizeof(float), hipMemcpyDeviceToHost));
    for (size_t e = 0; e < n; ++e) val[e] = f[e];
  }
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_time_kernel(nnms_system* s, int32_t kind, int32_t level, int32_t reps, double* ms) {
  ABI_BEGIN
  if (!s || !ms || reps < 1 || level < 0 || level >= s->h->host.L || kind < 0 || kind > 6)
    throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  const int L = s->h->host.L;
  if ((kind == 1 || kind == 2 || kind == 3) && level == L - 1)
    throw Error(NNMS_ERR_INVALID_ARG, "the coarsest level has only the direct solve");
  const bool ilu_level = level < L - 1 && s->h->host.lev[level].subsolver == NNMS_SUBSOLVER_ILU;
  if ((kind == 4 || kind == 5) && ilu_level)
    throw Error(NNMS_ERR_INVALID_ARG, "the copy and read references stream dense factors");
  Plan& P = apply_plan(s);
  hipStream_t st = P.stream;
  const bool f64 = s->prec == NNMS_FP64;
  const bool fac64 = f64 || level == L - 1;
  const int64_t copy_bytes = (s->h->host.lev[level].fac_elems * (fac64 ? 8 : 4)) & ~int64_t(15);
  std::unique_ptr<Arena> copy_dst;
  const int read_grid = ras_grid_default() * 2;
  if (kind == 4) {
    copy_dst = std::make_unique<Arena>(s->h->has_alloc ? &s->h->alloc : nullptr);
    copy_dst->raw(size_t(copy_bytes));
  } else if (kind == 5) {
    copy_dst = std::make_unique<Arena>(s->h->has_alloc ? &s->h->alloc : nullptr);
    copy_dst->raw(size_t(read_grid) * 4 * sizeof(int));
  }
  // kind 6 refactors the level in place: the same values give the same factors
  std::unique_ptr<Arena> fac_mem;
  FactorJob job;
  IluJob ijob;
  int* ferr = nullptr;
  if (kind == 6) {
    fac_mem = std::make_unique<Arena>(s->h->has_alloc ? &s->h->alloc : nullptr);
    if (ilu_level)
      ijob = ilu_job(*s, level, *fac_mem, st);
    else
      job = factor_job(*s, level, *fac_mem, st);
    ferr = fac_mem->alloc<int>(1, st);
  }
  auto launch = [&]() {
    if (kind == 6) {
      if (ilu_level)
        HIP_CHECK(enqueue_ilu(ijob, ferr, st));
      else
        HIP_CHECK(enqueue_factor(job, ferr, st));
    } else if (kind == 4) {
      HIP_CHECK(launch_copy16(s->lev[level].fac, copy_dst->bufs[0].first, copy_bytes, st));
    } else if (kind == 5) {
      HIP_CHECK(launch_read16(s->lev[level].fac, copy_bytes, (int*)copy_dst->bufs[0].first, read_grid, st));
    } else if (kind == 0) {
      if (level == L - 1) {
        if (f64)
          HIP_CHECK((launch_ras_groups<double, double>(P.coarse, false, st)));
        else
          HIP_CHECK((launch_ras_groups<double, float>(P.coarse, false, st)));
      } else if (f64) {
        HIP_CHECK(launch_smoother_level<double>(P.lev[level], true, st));
      } else {
        HIP_CHECK(launch_smoother_level<float>(P.lev[level], true, st));
      }
    } else if (kind == 1) {
      if (f64)
        HIP_CHECK(launch_spmv_groups<double>(P.lev[level].res, st));
      else
        HIP_CHECK(launch_spmv_groups<float>(P.lev[level].res, st));
    } else if (kind == 2) {
      if (f64)
        HIP_CHECK(launch_prolong_level<double>(P.lev[level], st));
      else
        HIP_CHECK(launch_prolong_level<float>(P.lev[level], st));
    } else {
      if (f64)
        HIP_CHECK(launch_spmv_groups<double>(P.lev[level].rst, st));
      else
        HIP_CHECK(launch_spmv_groups<float>(P.lev[level].rst, st));
    }
  };
  launch();  // warm-up
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  HIP_CHECK(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) launch();
  HIP_CHECK(hipEventRecord(e1, st));
  HIP_CHECK(hipEventSynchronize(e1));
  float t = 0;
  HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  check_counters(P, st);
  *ms = double(t) / reps;
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_system_factor(const nnms_system* s, int32_t level, int32_t part, double* lu, double* invl,
                                          int32_t* Nout) {
  ABI_BEGIN
  if (!s || level < 0 || level >= s->h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad level");
  const HostLevel& hl = s->h->host.lev[level];
  if (part < 0 || part >= hl.nparts) throw Error(NNMS_ERR_INVALID_ARG, "bad part");
  if (level < s->h->host.L - 1 && hl.subsolver == NNMS_SUBSOLVER_ILU)
    throw Error(NNMS_ERR_INVALID_ARG, "the level has ILU factors, not dense ones");
  const int N = hl.nblk[part];
  if (Nout) *Nout = N;
  const bool f64 = (level == s->h->host.L - 1) || s->prec == NNMS_FP64;
  const size_t fsz = f64 ? 8 : 4;
  const size_t ne = (size_t(N) * N + N) * TILE_ELEMS;
  std::vector<char> raw(ne * fsz);
  HIP_CHECK(hipMemcpy(raw.data(), (const char*)s->lev[level].fac + size_t(hl.fac_off[part]) * fsz, raw.size(),
                      hipMemcpyDeviceToHost));
  auto get = [&](size_t tile, int r, int c) -> double {
    if (f64) {
      const double* t = (const double*)raw.data() + tile * TILE_ELEMS;
      return t[((c / 2) * 64 + r) * 2 + (c % 2)];
    }
    const float* t = (const float*)raw.data() + tile * TILE_ELEMS;
    return t[((c / 4) * 64 + r) * 4 + (c % 4)];
  };
  const size_t np = size_t(N) * 64;
  if (lu)
    for (int ti = 0; ti < N; ++ti)
      for (int tj = 0; tj < N; ++tj)
        for (int r = 0; r < 64; ++r)
          for (int c = 0; c < 64; ++c) lu[(size_t(ti) * 64 + r) * np + size_t(tj) * 64 + c] = get(size_t(ti) * N + tj, r, c);
  if (invl)
    for (int ti = 0; ti < N; ++ti)
      for (int r = 0; r < 64; ++r)
        for (int c = 0; c < 64; ++c) invl[(size_t(ti) * 64 + r) * 64 + c] = get(size_t(N) * N + ti, r, c);
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_system_inverse_panels(const nnms_system* s, int32_t level, int32_t part, double* x,
                                                  int32_t* N_out, int32_t* No_out) {
  ABI_BEGIN
  if (!s || level < 0 || level >= s->h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad level");
  const HostLevel& hl = s->h->host.lev[level];
  if (part < 0 || part >= hl.nparts) throw Error(NNMS_ERR_INVALID_ARG, "bad part");
  if (!hl.xinv) throw Error(NNMS_ERR_INVALID_ARG, "the level does not apply inverse panels");
  const int N = hl.nblk[part], No = (hl.nown[part] + TILE - 1) / TILE;
  if (N_out) *N_out = N;
  if (No_out) *No_out = No;
  if (!x) return NNMS_OK;
  const bool f64 = (level == s->h->host.L - 1) || s->prec == NNMS_FP64;
  const size_t fsz = f64 ? 8 : 4;
  // the packed symmetric form, unpacked: X_v tiles, then X_oo's lower
  // triangle by columns (its upper triangle by transposition)
  const int n = int(hl.s_ptr[part + 1] - hl.s_ptr[part]), no = hl.nown[part], nv = n - no;
  const int Nv = (nv + TILE - 1) / TILE;
  std::vector<char> raw(size_t(hl.xs_off[part + 1] - hl.xs_off[part]) * fsz);
  HIP_CHECK(hipMemcpy(raw.data(), (const char*)s->lev[level].xinv + size_t(hl.xs_off[part]) * fsz, raw.size(),
                      hipMemcpyDeviceToHost));
  auto get = [&](size_t tile, int r, int c) -> double {
    return f64 ? ((const double*)raw.data())[tile * TILE_ELEMS + ((c / 2) * 64 + r) * 2 + (c % 2)]
               : ((const float*)raw.data())[tile * TILE_ELEMS + ((c / 4) * 64 + r) * 4 + (c % 4)];
  };
  auto low = [&](int a, int b) { return size_t(Nv) * No + size_t(b) * No - size_t(b) * (b - 1) / 2 + (a - b); };
  const size_t cols = size_t(No) * 64;
  for (int lr = 0; lr < N * 64; ++lr)
    for (int col = 0; col < No * 64; ++col) {
      double v = 0.0;
      const int b = col / 64, c = col % 64;
      if (lr < nv) {
        v = get(size_t(b) * Nv + lr / 64, lr % 64, c);
      } else if (lr < n && col < no) {
        const int oi = lr - nv, a = oi / 64, r = oi % 64;
        v = a >= b ? get(low(a, b), r, c) : get(low(b, a), c, r);
      }
      x[size_t(lr) * cols + col] = v;
    }
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_system_factor_pairs(const nnms_system* s, int32_t level, int32_t part, double* xl,
                                                double* xu, int32_t* npairs) {
  ABI_BEGIN
  if (!s || level < 0 || level >= s->h->host.L) throw Error(NNMS_ERR_INVALID_ARG, "bad level");
  const HostLevel& hl = s->h->host.lev[level];
  if (part < 0 || part >= hl.nparts) throw Error(NNMS_ERR_INVALID_ARG, "bad part");
  if (level < s->h->host.L - 1 && hl.subsolver == NNMS_SUBSOLVER_ILU)
    throw Error(NNMS_ERR_INVALID_ARG, "the level has ILU factors, not dense ones");
  const int N = hl.nblk[part], NP = N / 2;
  if (npairs) *npairs = NP;
  if (!xl && !xu) return NNMS_OK;
  const bool f64 = (level == s->h->host.L - 1) || s->prec == NNMS_FP64;
  const size_t fsz = f64 ? 8 : 4;
  const size_t first = (size_t(N) * N + N) * TILE_ELEMS, ne = size_t(2 * NP) * TILE_ELEMS;
  std::vector<char> raw(std::max<size_t>(ne * fsz, 1));
  if (ne)
    HIP_CHECK(hipMemcpy(raw.data(), (const char*)s->lev[level].fac + (size_t(hl.fac_off[part]) + first) * fsz,
                        ne * fsz, hipMemcpyDeviceToHost));
  auto get = [&](size_t tile, int r, int c) -> double {
    if (f64) return ((const double*)raw.data())[tile * TILE_ELEMS + ((c / 2) * 64 + r) * 2 + (c % 2)];
    return ((const float*)raw.data())[tile * TILE_ELEMS + ((c / 4) * 64 + r) * 4 + (c % 4)];
  };
  for (int p = 0; p < NP; ++p)
    for (int r = 0; r < 64; ++r)
      for (int c = 0; c < 64; ++c) {
        if (xl) xl[(size_t(p) * 64 + r) * 64 + c] = get(size_t(p), r, c);
        if (xu) xu[(size_t(p) * 64 + r) * 64 + c] = get(size_t(NP + p), r, c);
      }
  return NNMS_OK;
  ABI_END
}

// ---------------------------------------------------------------------------
// launch-shape tuning
// ---------------------------------------------------------------------------
static bool lanes_ok(int g) { return is_sell(g) || g == 4 || g == 8 || g == 16 || g == 32 || g == 64; }

extern "C" nnms_status nnms_hierarchy_get_tuning(const nnms_hierarchy* h, nnms_tuning* out) {
  ABI_BEGIN
  if (!h || !out) throw Error(NNMS_ERR_INVALID_ARG, "null argument");
  *out = h->tune;
  return NNMS_OK;
  ABI_END
}

extern "C" nnms_status nnms_hierarchy_set_tuning(nnms_hierarchy* h, const nnms_tuning* t) {
  ABI_BEGIN
  if (!h || !t) throw Error(NNMS_ERR_INVALID_ARG, "null argument");
  for (int l = 0; l < NNMS_MAX_LEVELS; ++l) {
    // the column-sorted slices only for a P^T that has them (entries of
    // levels without a P^T are not used)
    const bool csort_ok = t->pt_lanes[l] == SPMV_CSORT && (l + 1 >= h->host.L || h->dev[l].ptc_key);
    if (!lanes_ok(t->spmv_lanes[l]) || !(lanes_ok(t->pt_lanes[l]) || csort_ok) || t->ras_groups[l] < 0 ||
        t->ras_groups[l] > 65536 || !(t->ras_blocks[l] == 1 || t->ras_blocks[l] == 2 || t->ras_blocks[l] == 4))
      throw Error(NNMS_ERR_INVALID_ARG, "bad tuning entry");
  }
  if (!lanes_ok(t->krylov_lanes)) throw Error(NNMS_ERR_INVALID_ARG, "bad tuning entry");
  h->tune = *t;
  h->tune.tuned = 1;
  return NNMS_OK;
  ABI_END
}

template <typename Fn>
static double time_ms(hipStream_t st, int reps, Fn&& fn) {
  fn();
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  HIP_CHECK(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) fn();
  HIP_CHECK(hipEventRecord(e1, st));
  HIP_CHECK(hipEventSynchronize(e1));
  float t = 0;
  HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return double(t) / reps;
}

extern "C" nnms_status nnms_autotune(nnms_system* s, int32_t reps, nnms_tuning* out) {
  ABI_BEGIN
  if (!s || reps < 1) throw Error(NNMS_ERR_INVALID_ARG, "bad arguments");
  nnms_hierarchy* h = s->h;
  const int L = h->host.L;
  const bool f64 = s->prec == NNMS_FP64;
  nnms_tuning t = h->tune;
  Plan& P = apply_plan(s);
  hipStream_t st = P.stream;
  Arena tmp(h->has_alloc ? &h->alloc : nullptr);
  const int lanes[] = {4, 8, 16, 32, 64};
  // fastest lanes per CSR row; with the sliced ELL arrays given, 0 and 1
  // (that layout, one wave per slice or four) are candidates too, and with
  // the column-sorted slices given, SPMV_CSORT
  auto spmv_best = [&](const int32_t* rp, const int32_t* col, const void* val, const void* x, const void* r, void* y,
                       int64_t n, bool dbl, const int32_t* soff = nullptr, const int32_t* scol = nullptr,
                       const void* sval = nullptr, const int32_t* ckey = nullptr, const int32_t* cbase = nullptr,
                       const void* cval = nullptr, int ccap = 0) {
    int best = 16;
    double bt = 1e30;
    std::vector<int> cand(std::begin(lanes), std::end(lanes));
    if (soff) cand.push_back(0), cand.push_back(1);
    if (ckey && ccap > 0) cand.push_back(SPMV_CSORT);
    for (int g : cand) {
      SpmvDesc d{};
      if (g == SPMV_CSORT)
        d.rp = rp, d.col = ckey, d.val = cval, d.base = cbase, d.cap = ccap;
      else if (is_sell(g))
        d.rp = soff, d.col = scol, d.val = sval;
      else
        d.rp = rp, d.col = col, d.val = val;
      d.x = x, d.r = r, d.y = y, d.n = int(n), d.blk0 = 0, d.when = WHEN_RUNNING;
      std::vector<SpmvDesc> v{d};
      SpmvDesc* dd = tmp.upload(v, st);
      const int nb = spmv_blocks(n, g);
      double ms = time_ms(st, reps, [&]() {
        if (g == SPMV_CSORT) {
          if (dbl)
            HIP_CHECK(launch_csort<double>(dd, 1, nb, ccap, st));
          else
            HIP_CHECK(launch_csort<float>(dd, 1, nb, ccap, st));
        } else if (is_sell(g)) {
          if (dbl)
            HIP_CHECK(launch_sell<double>(dd, 1, nb, g, st));
          else
            HIP_CHECK(launch_sell<float>(dd, 1, nb, g, st));
        } else if (dbl) {
          HIP_CHECK(launch_spmv<double>(dd, 1, nb, g, st));
        } else {
          HIP_CHECK(launch_spmv<float>(dd, 1, nb, g, st));
        }
      });
      if (ms < bt) bt = ms, best = g;
    }
    return best;
  };
  int cus = ras_grid_default() / 4;
  std::vector<int32_t*> tcounters;
  // best (blocks per work item, grid) of the smoother on level l
  auto ras_best = [&](int l, bool coarse, int32_t& groups_out, int32_t& blocks_out) {
    double bt = 1e30;
    for (int K : {1, 2, 4}) {
      RasLaunch rr, rt;
      build_ras_pair(tmp, tcounters, {s}, l, coarse, s->prec, false, K, st, rr, rt);
      HIP_CHECK(hipStreamSynchronize(st));
      const RasLaunch& rl = coarse ? rr : rt;
      for (int per = 1; per <= 6; ++per) {
        const int grid = per * cus;
        double ms = time_ms(st, reps, [&]() {
          if (coarse) {
            if (f64)
              HIP_CHECK((launch_ras<double, double>(rl, grid, st)));
            else
              HIP_CHECK((launch_ras<double, float>(rl, grid, st)));
          } else if (f64) {
            HIP_CHECK((launch_ras<double, double>(rl, grid, st)));
          } else {
            HIP_CHECK((launch_ras<float, float>(rl, grid, st)));
          }
        });
        if (ms < bt) bt = ms, groups_out = grid, blocks_out = K;
        if (grid >= rl.ntasks) break;  // a larger grid cannot help
      }
    }
  };
  for (int l = 0; l < L - 1; ++l) {
    const DevLevel& dl = h->dev[l];
    SysLevel& sl = s->lev[l];
    const int64_t n = h->host.lev[l].nv, nc = h->host.lev[l + 1].nv;
    const void* val = f64 ? (const void*)sl.val64 : (const void*)sl.val32;
    const void* ell = f64 ? (const void*)sl.ell64 : (const void*)sl.ell32;
    t.spmv_lanes[l] = spmv_best(dl.rp, dl.col, val, sl.z, sl.r, sl.t, n, f64, dl.sell_off, dl.sell_col, ell);
    const void* ptw = f64 ? (const void*)dl.pt_w64 : (const void*)dl.pt_w32;
    const void* ptsw = f64 ? (const void*)dl.pts_w64 : (const void*)dl.pts_w32;
    const void* ptcw = f64 ? (const void*)dl.ptc_w64 : (const void*)dl.ptc_w32;
    t.pt_lanes[l] = spmv_best(dl.pt_rp, dl.pt_col, ptw, sl.t, nullptr, s->lev[l + 1].r, nc, f64, dl.pts_off,
                              dl.pts_col, ptsw, dl.ptc_key, dl.ptc_base, ptcw, dl.ptc_cap);
    // the dense smoother's launch shape (ILU levels have no dense factors)
    // (ILU levels have no dense factors; inverse panels have no shape to choose)
    if (h->host.lev[l].subsolver != NNMS_SUBSOLVER_ILU && !h->host.lev[l].xinv)
      ras_best(l, false, t.ras_groups[l], t.ras_blocks[l]);
  }
  if (!h->host.lev[L - 1].xinv) ras_best(L - 1, true, t.ras_groups[L - 1], t.ras_blocks[L - 1]);
  for (int32_t* c : tcounters) {
    int32_t v[4];
    HIP_CHECK(hipMemcpy(v, c, sizeof v, hipMemcpyDeviceToHost));
    if (v[2]) throw Error(NNMS_ERR_DEVICE, "triangular-solve wait limit exceeded while tuning");
  }
  {
    const DevLevel& d0 = h->dev[0];
    t.krylov_lanes = spmv_best(d0.rp, d0.col, s->lev[0].val64, s->x, nullptr, s->w, h->host.lev[0].nv, true,
                               d0.sell_off, d0.sell_col, s->lev[0].ell64);
  }
  check_counters(P, st);
  t.tuned = 1;
  h->tune = t;
  s->solo.reset();
  s->apply.reset();
  if (out) *out = t;
  return NNMS_OK;
  ABI_END
}
