// ec_api.hip - host runtime behind the C ABI of include/ec.h.
//
// Context: device, allocator hooks, HBM admission ledger, twiddle tables and the
// cached windows of the discrete Green kernel.  State: one replica's resident
// eigenstrain (fixed point), FP64 stress, half spectrum, footprint lists and
// energies.  The defect description is double-buffered so a failed solve leaves
// the previous one intact.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <climits>
#include <cstddef>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ec_internal.h"

using namespace ec;

namespace {

thread_local std::string g_err;

ec_status fail(ec_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(EC_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

}  // namespace

// A window of the discrete Green kernel, shared by the states of one problem.
// States hold it by shared_ptr: when a wider window replaces it in the
// context's cache, the old one stays alive (and its device memory allocated)
// until the last state using it lets go; its destructor waits for the device
// before freeing.  It must never be destroyed while the context's mutex is
// held (the free takes that mutex for the ledger).
struct WinCache {
  ec_ctx* ctx = nullptr;
  int n = 0;
  double C11 = 0, C12 = 0, C44 = 0;
  std::array<double, 9> frame{};  // all zeros: cube axes
  int bc = 0;
  int D = 0;
  double* K = nullptr;
  size_t bytes = 0;
  ~WinCache();
};

// Host worker threads for per-defect preparation of large defect lists.
// run(n, fn) calls fn(c) for every chunk c in [0, n) on the workers and the
// calling thread and returns when all chunks are done; a worker that wakes
// after the job has closed does nothing.  Solves of a running simulation come
// a millisecond or two apart, so after a job the workers poll for the next
// one for SPIN_MS (yielding the core between polls) before they sleep: a
// sleeping worker takes tens of microseconds to wake, longer than its share
// of a 2000-defect list.
class WorkPool {
  static constexpr int SPIN_MS = 5;

 public:
  explicit WorkPool(int nworkers) {
    for (int i = 0; i < nworkers; ++i) th_.emplace_back([this] { loop(); });
  }
  ~WorkPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      astop_.store(true, std::memory_order_release);
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  void run(int nchunks, const std::function<void(int)>& fn) {
    if (th_.empty() || nchunks <= 1) {
      for (int c = 0; c < nchunks; ++c) fn(c);
      return;
    }
    // states of one context may be driven from several host threads: one job
    // at a time
    std::lock_guard<std::mutex> one(run_mu_);
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn;
      nchunks_ = nchunks;
      next_.store(0);
      open_ = true;
      ++gen_;
      agen_.store(gen_, std::memory_order_release);
    }
    cv_.notify_all();
    work();
    std::unique_lock<std::mutex> lk(mu_);
    open_ = false;
    done_.wait(lk, [&] { return inside_ == 0; });
    fn_ = nullptr;
  }

 private:
  void work() {
    for (int c; (c = next_.fetch_add(1)) < nchunks_;) (*fn_)(c);
  }
  void loop() {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> lk(mu_, std::defer_lock);
    for (;;) {
      const auto until = std::chrono::steady_clock::now() + std::chrono::milliseconds(SPIN_MS);
      while (agen_.load(std::memory_order_acquire) == seen && !astop_.load(std::memory_order_acquire) &&
             std::chrono::steady_clock::now() < until)
        std::this_thread::yield();
      lk.lock();
      cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
      if (stop_) return;
      seen = gen_;
      if (open_) {
        ++inside_;
        lk.unlock();
        work();
        lk.lock();
        if (--inside_ == 0) done_.notify_all();
      }
      lk.unlock();
    }
  }
  std::vector<std::thread> th_;
  std::mutex run_mu_, mu_;
  std::condition_variable cv_, done_;
  const std::function<void(int)>* fn_ = nullptr;
  int nchunks_ = 0, inside_ = 0;
  std::atomic<int> next_{0};
  uint64_t gen_ = 0;
  bool open_ = false, stop_ = false;
  std::atomic<uint64_t> agen_{0};  // gen_, readable without the lock
  std::atomic<bool> astop_{false};
};

// ------------------------------------------------ fixed device scratch area
//
// Scratch of ec_interaction_energies_noalloc: the self-term work list, the
// per-defect item offsets, the per-item partial sums and the per-defect run
// sums of the energies (k_self_plan / k_self / k_self_runs / k_self_finish),
// for up to NA_MAX_DEFECTS defects and
// NA_MAX_ITEMS work items.  Every GPU the library runs on holds one copy until
// the process ends; every call on a GPU shares it (calls that overlap on one
// GPU race).  Nothing in it needs to start at zero: the plan writes every
// offset and item it uses, every item writes its partial, and every defect on
// the run path writes its run sum (the others' entries are not read).  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device (noalloc_scratch()); the array's name in host code is a
// host-side stand-in, not a device address.
namespace {
constexpr int64_t NA_MAX_DEFECTS = 16384;
constexpr int64_t NA_MAX_ITEMS = 262144;
constexpr size_t NA_WORK_OFF = 0;
constexpr size_t NA_PART_OFF = NA_WORK_OFF + NA_MAX_ITEMS * sizeof(SelfWork);
constexpr size_t NA_WBEG_OFF = NA_PART_OFF + NA_MAX_ITEMS * sizeof(double);
constexpr size_t NA_RUN_OFF = NA_WBEG_OFF + (NA_MAX_DEFECTS + 8) * sizeof(int64_t);
constexpr size_t NA_BYTES = NA_RUN_OFF + NA_MAX_DEFECTS * sizeof(double);
}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {
constexpr int NA_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NA_MAX_DEVICES] = {};

// Device address of the scratch area on `device` (which must be current),
// looked up once per device.
hipError_t noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= NA_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}
}  // namespace

// Buffers (and, once captured, the executable graph) of batched hops of one
// shape, batch size and stream: the pinned job table the host fills, its device
// copy, the tile counters, a zero mean-stress change and the frame maps.  The
// graph reads the pinned table at a fixed address, so a new batch waits for the
// previous launch from the same entry before rewriting it.
struct BatchEntry {
  HopJob* pin = nullptr;
  HopJob* dev = nullptr;
  uint32_t* ctr = nullptr;
  double* zero6 = nullptr;
  double* frm = nullptr;
  hipGraphExec_t exec = nullptr;
  bool graph_failed = false;
  hipEvent_t done = nullptr;
  bool pending = false;
};
struct BatchKey {
  int n, prec, k;
  double C11, C12, C44;
  std::array<double, 9> frame;
  void* stream;
  bool operator<(const BatchKey& o) const {
    return std::tie(n, prec, k, C11, C12, C44, frame, stream) <
           std::tie(o.n, o.prec, o.k, o.C11, o.C12, o.C44, o.frame, o.stream);
  }
};

struct ec_ctx {
  int device = 0;
  void* scratch = nullptr;  // this device's copy of the fixed scratch area
  std::map<BatchKey, BatchEntry> batches;
  size_t budget = 0, used = 0;
  ec_alloc_fn af = nullptr;
  ec_free_fn ff = nullptr;
  void* user = nullptr;
  std::mutex mu;
  std::map<int, double2*> tw;
  std::vector<std::shared_ptr<WinCache>> wins;
  std::unique_ptr<WorkPool> pool;
};

namespace {

struct DefBuf {
  DevDefect* tab = nullptr;
  int32_t* cnt = nullptr;  // footprint counts, written by the rasteriser
  size_t cap = 0;
  int32_t* ids = nullptr;  // footprint slots; defect i owns [slot_i, slot_i + box volume)
  int2* lnk = nullptr;     // per membership entry: {defect, next entry of the same voxel}
  int64_t ids_cap = 0;
};

struct ProfRec {
  int fam;
  hipEvent_t a, b;
  double bytes;
};

// Pinned host staging for asynchronous uploads: reused across calls, the
// previous upload from the same buffer is waited for before it is overwritten.
struct Pinned {
  char* p = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};

}  // namespace

struct ec_state {
  ec_ctx* ctx = nullptr;
  ec_problem prob{};
  int n = 0;
  int64_t n3 = 0;
  bool fp64 = true;
  SpecGeom g{};
  Cubic C{};
  double h3c = 0;
  size_t spec_bytes = 0, held = 0;
  void* spec = nullptr;
  int32_t* own = nullptr;  // per-voxel head of the membership list
  double* sig = nullptr;   // resident FP64 stress, voxel-major [n^3][6]
  double* add6 = nullptr;  // [0..6) additive stress of the full solve, [6..12) zeros, [12..18) update delta
  double2* tw = nullptr;
  // defect list
  int ndef = 0;
  bool solved = false;
  // The stress of the last solve is stored only at the voxels its defects
  // cover (all that the energy reductions read); the rest is formed from the
  // resident spectrum (the y inverse pass's output) when something first needs
  // the whole field (ensure_sigma).  A solve stores only the covered voxels
  // when nothing read the whole field since the solve before it (a caller
  // that reads it after every solve, an OkMC loop or a serving replica
  // between hops, gets it stored at once instead of formed twice).
  bool sig_lazy = false;
  bool whole_read = false;  // the whole field was needed since the last solve
  std::vector<DevDefect> hdefs;
  std::vector<int32_t> hcnt;  // host copy of the counts, valid when hcnt_ok
  bool hcnt_ok = false;
  std::vector<int64_t> hcap;  // slot capacity per defect
  int64_t ids_used = 0;       // slot space in use
  DefBuf db[2];
  int cur = 0;
  double* B = nullptr;
  double* E = nullptr;
  double* S6 = nullptr;
  double* runsum = nullptr;  // self-term run sums (scratch of the self terms)
  size_t pd_cap = 0;
  bool B_valid = false;
  // self terms of a fresh solve run on a side stream beside the Fourier
  // passes: it starts after the rasterisation (ev_fill) and every later use
  // of the self terms or of the defect buffers waits for ev_self
  hipStream_t side = nullptr;
  hipEvent_t ev_fill = nullptr, ev_self = nullptr;
  bool self_pending = false;
  // eigenstrain direction classes and their scalar windows; the classes of a
  // new defect list are assigned when first needed (classes_ok false until then)
  bool classes_ok = true;
  std::vector<std::array<double, 6>> classes;
  // run classes (class, run direction) and their self-term tables (double
  // prefix sums of the class windows along the run direction)
  std::vector<std::array<int, 4>> runcls;
  int4* runinfo = nullptr;  // MAXRUN entries {class, tx, ty, tz}
  double* gff = nullptr;
  size_t gff_bytes = 0;
  int gff_D = -1, gff_nrun = -1;
  int max_runs = 0;  // largest run bound over the list (host, with the run classes)
  ClassTag* tags = nullptr;
  size_t tags_cap = 0;
  double* dirs = nullptr;
  double* gcls = nullptr;
  size_t gcls_bytes = 0;
  int gcls_D = -1, gcls_ncls = -1;
  std::shared_ptr<const WinCache> win;
  std::array<double, 9> frame{};  // the problem's frame, all zeros for cube axes
  std::array<double, FRAME_LEN> frmh{};  // host copy of its maps
  // dislocation lines: stress planes per axis ([3][n^2][6]) added to every
  // solve's stress, the axes present, and the scratch of their computation
  double* bg = nullptr;
  size_t bg_cap = 0;
  int bg_mask = 0;
  double2* bgspec = nullptr;
  size_t bgspec_cap = 0;
  DevLine* dlines = nullptr;
  size_t dlines_cap = 0;
  // dislocation paths in any direction: their stress ([n^3][6] FP64), added to
  // the resident stress of every solve while bg3_on
  double* bg3 = nullptr;
  size_t bg3_cap = 0;
  bool bg3_on = false;
  double* frm = nullptr;          // its device form (FRAME_LEN doubles), null for cube axes
  // self-term work list (built on the device)
  SelfWork* work = nullptr;
  size_t work_cap = 0;
  double* partial = nullptr;
  size_t partial_cap = 0;
  int64_t* wbeg = nullptr;
  size_t wbeg_cap = 0;
  // update scratch
  int32_t* upd_ids = nullptr;
  int64_t upd_cap = 0;
  double* updE = nullptr;     // 12 doubles: the old and the new eigenstrain of a moved defect
  uint32_t* tilectr = nullptr;  // NTILECTR tile counters of the persistent passes
  // jump probes: energy changes of the last ec_jump_energies call (jn per
  // defect) and their scratch
  int jn = 0;
  bool jdE_ok = false;
  int32_t* jjumps = nullptr;
  size_t jjumps_cap = 0;
  double *jdE = nullptr, *jt1 = nullptr, *jpartial = nullptr, *jsel = nullptr, *jnu = nullptr;
  size_t jdE_cap = 0, jt1_cap = 0, jpartial_cap = 0, jsel_cap = 0, jnu_cap = 0;
  SelfWork* jwork = nullptr;
  size_t jwork_cap = 0;
  // cross parts h^3 c X(lambda) + B_i of the jumps jx_jumps, valid while the
  // list changes by whole-voxel translations only
  double* jxc = nullptr;
  size_t jxc_cap = 0;
  bool jx_ok = false;
  std::vector<int32_t> jx_jumps;
  int64_t* jwbeg = nullptr;
  size_t jwbeg_cap = 0;
  int32_t* jchoice = nullptr;
  size_t jchoice_cap = 0;
  double* dip = nullptr;  // dipole-tensor energies
  size_t dip_cap = 0;
  // stored defect types (Sec. 3.3): the eigenstrain and stress half spectra of
  // each prototype at its reference centre X0, and the phase tables, partial
  // sums and energies of ec_type_energies
  struct TypeSpec {
    void* eps = nullptr;
    void* sig = nullptr;
    double X0[3] = {0, 0, 0};
  };
  std::vector<TypeSpec> types;
  double* tbuf = nullptr;
  size_t tbuf_cap = 0;
  // pinned staging: defect table, per-update records, moved footprint
  Pinned pin_tab, pin_upd, pin_ids, pin_tags, pin_jump, pin_choice, pin_out;
  // profiling
  bool prof = false;
  int32_t prof_mask = (1 << EC_NPROF) - 1;  // families whose launches are timed
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> evpool;
};

namespace {

// ------------------------------------------------------------------ memory / ledger

void* raw_alloc(ec_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 64;
  if (c->af) return c->af(bytes, nullptr, c->user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void raw_free(ec_ctx* c, void* p) {
  if (!p) return;
  if (c->ff)
    c->ff(p, nullptr, c->user);
  else
    (void)hipFree(p);
}

bool admit(ec_ctx* c, size_t bytes) {
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->used + bytes > c->budget) return false;
  c->used += bytes;
  return true;
}

void release(ec_ctx* c, size_t bytes) {
  std::lock_guard<std::mutex> lk(c->mu);
  c->used = bytes > c->used ? 0 : c->used - bytes;
}

// Allocation charged to the ledger; *out is left untouched on failure.
ec_status ledger_alloc(ec_ctx* c, size_t bytes, void** out) {
  if (!admit(c, bytes)) return fail(EC_ERR_ADMIT, "HBM budget exceeded (%zu bytes requested)", bytes);
  void* p = raw_alloc(c, bytes);
  if (!p) {
    release(c, bytes);
    return fail(EC_ERR_DEVICE, "device allocation of %zu bytes failed", bytes);
  }
  *out = p;
  return EC_OK;
}

void ledger_free(ec_ctx* c, void* p, size_t bytes) {
  if (!p) return;
  raw_free(c, p);
  release(c, bytes);
}

// A temporary device buffer charged to the ledger, freed when it goes out of
// scope (callers synchronise before that when kernels may still use it).
struct Tmp {
  ec_ctx* c;
  void* p = nullptr;
  size_t b = 0;
  ~Tmp() { ledger_free(c, p, b); }
};

}  // namespace

WinCache::~WinCache() {
  if (!K) return;
  (void)hipDeviceSynchronize();  // kernels of any stream may still read the window
  ledger_free(ctx, K, bytes);
}

namespace {

template <class T>
ec_status st_grow(ec_state* st, T** p, size_t* cap_elems, size_t need, bool keep = false, hipStream_t s = nullptr) {
  if (need <= *cap_elems && *p) return EC_OK;
  size_t ncap = std::max<size_t>(need, *cap_elems + *cap_elems / 2);
  ncap = std::max<size_t>(ncap, 16);
  void* q = nullptr;
  ec_status r = ledger_alloc(st->ctx, ncap * sizeof(T), &q);
  if (r != EC_OK) return r;
  if (keep && *p && *cap_elems) {
    if (hipMemcpyAsync(q, *p, *cap_elems * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess) {
      ledger_free(st->ctx, q, ncap * sizeof(T));
      return fail(EC_ERR_DEVICE, "device copy failed while growing a buffer");
    }
    (void)hipStreamSynchronize(s);
  }
  if (*p) ledger_free(st->ctx, *p, *cap_elems * sizeof(T));
  st->held += ncap * sizeof(T);
  st->held -= std::min(st->held, *cap_elems * sizeof(T));
  *p = (T*)q;
  *cap_elems = ncap;
  return EC_OK;
}

// ------------------------------------------------------------------ pinned staging

ec_status pin_begin(Pinned& b, size_t bytes, char** host) {
  if (b.pending) {
    HIPCHK(hipEventSynchronize(b.ev));
    b.pending = false;
  }
  if (!b.ev) HIPCHK(hipEventCreateWithFlags(&b.ev, hipEventDisableTiming));
  if (bytes > b.cap) {
    if (b.p) HIPCHK(hipHostFree(b.p));
    b.p = nullptr;
    b.cap = 0;
    const size_t cap = std::max<size_t>(bytes, 4096);
    HIPCHK(hipHostMalloc((void**)&b.p, cap, hipHostMallocDefault));
    b.cap = cap;
  }
  *host = b.p;
  return EC_OK;
}

ec_status pin_end(Pinned& b, hipStream_t s) {
  HIPCHK(hipEventRecord(b.ev, s));
  b.pending = true;
  return EC_OK;
}

void pin_free(Pinned& b) {
  if (b.pending) (void)hipEventSynchronize(b.ev);
  if (b.p) (void)hipHostFree(b.p);
  if (b.ev) (void)hipEventDestroy(b.ev);
  b = Pinned{};
}

// ------------------------------------------------------------------ profiling

hipEvent_t take_event(ec_state* st) {
  if (!st->evpool.empty()) {
    hipEvent_t e = st->evpool.back();
    st->evpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

template <class F>
hipError_t run(ec_state* st, hipStream_t s, int fam, double bytes, F&& f) {
  if (!st->prof || !((st->prof_mask >> fam) & 1)) return f();
  hipEvent_t a = take_event(st), b = take_event(st);
  (void)hipEventRecord(a, s);
  hipError_t e = f();
  (void)hipEventRecord(b, s);
  st->recs.push_back({fam, a, b, bytes});
  return e;
}

#define LAUNCH(st, s, fam, bytes, call)                                                     \
  do {                                                                                      \
    hipError_t e_ = run(st, s, fam, (double)(bytes), [&]() { return (call); });             \
    if (e_ != hipSuccess) return fail(EC_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------ twiddles

double2* ctx_twiddles(ec_ctx* c, int n) {
  {
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->tw.find(n);
    if (it != c->tw.end()) return it->second;
  }
  // built and allocated without the lock: an allocator the caller supplies may
  // run code that re-enters the library (a garbage collector destroying
  // another state, say), which takes the lock
  std::vector<double2> h(n);
  const long double pi = acosl(-1.0L);
  for (int e = 0; e < n; ++e) {
    const long double a = 2.0L * pi * (long double)e / (long double)n;
    h[e] = make_double2((double)cosl(a), (double)(-sinl(a)));
  }
  void* p = raw_alloc(c, n * sizeof(double2));
  if (!p) return nullptr;
  if (hipMemcpy(p, h.data(), n * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess) {
    raw_free(c, p);
    return nullptr;
  }
  void* drop = nullptr;
  double2* out = nullptr;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    auto ins = c->tw.emplace(n, (double2*)p);
    if (!ins.second) drop = p;  // another thread made the table meanwhile
    out = ins.first->second;
  }
  raw_free(c, drop);
  return out;
}

// ------------------------------------------------------------------ quantisation
//
// The same integer description the oracle derives independently: centre
// c_q = rint(c s) mod 1024 n with s = (1024 n)/L, R2_q = rint((R s)^2),
// thickness e_q = rint(e s) (1024 for e = 0), habit normal as the smallest
// integer lattice vector (components up to 8).

#pragma clang fp contract(off)

bool lattice_normal(const double v[3], int m[3]) {
  double amax = 0.0;
  for (int k = 0; k < 3; ++k) amax = std::max(amax, std::fabs(v[k]));
  if (!std::isfinite(amax) || amax == 0.0) return false;
  double a[3];
  for (int k = 0; k < 3; ++k) a[k] = v[k] / amax;
  for (int mult = 1; mult <= 8; ++mult) {
    bool ok = true;
    double r[3];
    for (int k = 0; k < 3; ++k) {
      const double w = a[k] * (double)mult;
      r[k] = std::nearbyint(w);
      if (!(std::fabs(w - r[k]) < 1e-9)) ok = false;
    }
    if (ok) {
      int g = 0;
      for (int k = 0; k < 3; ++k) {
        m[k] = (int)r[k];
        int x = std::abs(m[k]);
        int y = g;
        while (y) {
          int t = x % y;
          x = y;
          y = t;
        }
        g = x;
      }
      for (int k = 0; k < 3; ++k) m[k] /= g;
      return true;
    }
  }
  return false;
}

int64_t box_volume(const DevDefect& d) { return (int64_t)d.w[0] * d.w[1] * d.w[2]; }

int64_t floordiv(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

int64_t isqrt64(int64_t v) {
  int64_t r = (int64_t)std::sqrt((double)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// Whether a problem's frame rotates the crystal (all zeros and the identity do not).
bool frame_rotates(const double* fr) {
  bool any = false, id = true;
  for (int k = 0; k < 9; ++k) {
    any |= fr[k] != 0.0;
    id &= fr[k] == (k % 4 == 0 ? 1.0 : 0.0);
  }
  return any && !id;
}

// Tensor components (xx yy zz yz xz xy) in the cube frame, T_c = A^T T A, for a
// frame A whose rows are the cell axes in cube coordinates.
void to_cube(const double* A, const double* t, double* out) {
  const double T[3][3] = {{t[0], t[5], t[4]}, {t[5], t[1], t[3]}, {t[4], t[3], t[2]}};
  double U[3][3];
  for (int i = 0; i < 3; ++i)
    for (int q = 0; q < 3; ++q) U[i][q] = T[i][0] * A[q] + T[i][1] * A[3 + q] + T[i][2] * A[6 + q];
  auto tc = [&](int p, int q) { return A[p] * U[0][q] + A[3 + p] * U[1][q] + A[6 + p] * U[2][q]; };
  out[0] = tc(0, 0);
  out[1] = tc(1, 1);
  out[2] = tc(2, 2);
  out[3] = tc(1, 2);
  out[4] = tc(0, 2);
  out[5] = tc(0, 1);
}

// Run direction of a loop for the self terms: the shortest lattice vector t in
// the habit plane (m . t = 0) with components in [-2, 2] (first nonzero one
// positive, ties in a fixed order); none found leaves t = 0 (no run path).
void run_direction_search(const int32_t m[3], int32_t t[3]) {
  t[0] = t[1] = t[2] = 0;
  for (int len2 = 1; len2 <= 12; ++len2)
    for (int a = -2; a <= 2; ++a)
      for (int b = -2; b <= 2; ++b)
        for (int c = -2; c <= 2; ++c) {
          if (a * a + b * b + c * c != len2) continue;
          const int first = a != 0 ? a : (b != 0 ? b : c);
          if (first < 0 || m[0] * a + m[1] * b + m[2] * c != 0) continue;
          t[0] = a;
          t[1] = b;
          t[2] = c;
          return;
        }
}

// The search above, remembered per thread for the last few normals (a defect
// list uses a handful of habit planes).
void run_direction(const int32_t m[3], int32_t t[3]) {
  struct Entry {
    int32_t m[3], t[3];
  };
  thread_local Entry memo[8];
  thread_local int used = 0, next = 0;
  for (int i = 0; i < used; ++i)
    if (memo[i].m[0] == m[0] && memo[i].m[1] == m[1] && memo[i].m[2] == m[2]) {
      std::copy(memo[i].t, memo[i].t + 3, t);
      return;
    }
  run_direction_search(m, t);
  Entry& e = memo[next];
  std::copy(m, m + 3, e.m);
  std::copy(t, t + 3, e.t);
  next = (next + 1) % 8;
  used = std::max(used, next == 0 ? 8 : next);
}

bool quantise(const ec_problem& P, const ec_defect& rec, DevDefect& d, std::string& err) {
  std::memset(&d, 0, sizeof d);
  d.rcls = -1;
  const int n = P.n;
  const double L = P.L;
  const double s = (1024.0 * n) / L;
  const int64_t Lq = (int64_t)QSUB * n;
  const double R = rec.radius;
  if (!(R > 0.0) || !std::isfinite(R)) return err = "radius must be positive and finite", false;
  for (int k = 0; k < 3; ++k) {
    const double v = rec.c[k] * s;
    if (!std::isfinite(v) || std::fabs(v) > 4.0e18) return err = "centre not finite", false;
    int64_t q = (int64_t)std::nearbyint(v) % Lq;
    if (q < 0) q += Lq;
    d.cq[k] = (int32_t)q;
  }
  const double Rs = R * s;
  const double R2 = Rs * Rs;
  d.R2q = (int64_t)std::nearbyint(R2);
  d.kind = rec.kind;
  d.cls = -1;
  double E[3][3] = {{0}};
  int64_t ext = isqrt64(d.R2q) + 1;
  if (rec.kind == EC_LOOP) {
    const double bb = rec.b[0] * rec.b[0] + rec.b[1] * rec.b[1] + rec.b[2] * rec.b[2];
    if (!(bb > 0.0) || !std::isfinite(bb)) return err = "zero or non-finite Burgers vector", false;
    const double e = rec.thickness;
    if (e < 0.0 || !std::isfinite(e)) return err = "negative thickness", false;
    double e_nm;
    if (e == 0.0) {
      d.eq = QSUB;
      e_nm = L / n;
    } else {
      d.eq = (int32_t)std::nearbyint(e * s);
      e_nm = e;
      if (d.eq <= 0) return err = "thickness below the quantisation step", false;
    }
    if (R + 0.5 * e_nm >= 0.5 * L) return err = "loop extent reaches half the cell", false;
    if (!lattice_normal(rec.normal, d.m)) return err = "habit normal is not a small-integer lattice direction", false;
    d.mm = d.m[0] * d.m[0] + d.m[1] * d.m[1] + d.m[2] * d.m[2];
    run_direction(d.m, d.rt);
    const double nrm = std::sqrt((double)d.mm);
    double nh[3];
    for (int k = 0; k < 3; ++k) nh[k] = (double)d.m[k] / nrm;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) E[a][b] = (rec.b[a] * nh[b] + nh[a] * rec.b[b]) / (2.0 * e_nm);
    ext += (d.eq + 1) / 2;
  } else if (rec.kind == EC_SPHERE) {
    if (R >= 0.5 * L) return err = "sphere extent reaches half the cell", false;
    d.rt[0] = 1;  // runs along x
    if (!std::isfinite(rec.eig_v)) return err = "eigenstrain not finite", false;
    for (int a = 0; a < 3; ++a) E[a][a] = rec.eig_v;
  } else {
    return err = "unknown defect kind", false;
  }
  d.E[0] = E[0][0];
  d.E[1] = E[1][1];
  d.E[2] = E[2][2];
  d.E[3] = E[1][2];
  d.E[4] = E[0][2];
  d.E[5] = E[0][1];
  // the rasterised eigenstrain (fixed point) is kept in the cube frame of a
  // rotated crystal, where the Green step applies the cubic operator; E stays
  // in cell coordinates for the energies
  double Ef[6];
  if (frame_rotates(P.frame))
    to_cube(P.frame, d.E, Ef);
  else
    std::copy(d.E, d.E + 6, Ef);
  for (int a = 0; a < 6; ++a) {
    if (!(std::fabs(d.E[a]) < 64.0) || !(std::fabs(Ef[a]) < 64.0))
      return err = "eigenstrain component too large", false;
    d.efix[a] = (int64_t)std::llrint(Ef[a] * FIX_SCALE);
  }
  set_efd(d);
  for (int k = 0; k < 3; ++k) {
    const int64_t lo = floordiv((int64_t)d.cq[k] - ext - 512 + (QSUB - 1), QSUB);
    const int64_t hi = floordiv((int64_t)d.cq[k] + ext - 512, QSUB);
    const int64_t w = std::min<int64_t>(hi - lo + 1, n);
    d.w[k] = (int32_t)w;
    d.lo[k] = (int32_t)(((lo % n) + n) % n);
    d.d0[k] = (int32_t)(QSUB * lo + QSUB / 2 - d.cq[k]);
  }
  return true;
}

#pragma clang fp contract(on)

// Direction class of an eigenstrain: E = s e with e's largest-magnitude entry = 1.
void direction(const DevDefect& d, std::array<double, 6>& e, double& s) {
  int am = 0;
  for (int a = 1; a < 6; ++a)
    if (std::fabs(d.E[a]) > std::fabs(d.E[am])) am = a;
  s = d.E[am];
  for (int a = 0; a < 6; ++a) e[a] = s != 0.0 ? d.E[a] / s : 0.0;
}

constexpr int MAXCLS = 32;
constexpr int MAXRUN = 32;  // run classes (class, run direction) with self-term tables

// Bound on the number of runs of a footprint along its run direction: the
// lattice lines along t that meet its box.  Each such line has a first point p
// in the box with p - t outside, so p lies within |t_k| layers of a face
// normal to an axis k with t_k != 0: at most sum_k |t_k| prod_{j != k} w_j.
int64_t run_bound(const DevDefect& d) {
  int64_t lines = 0;
  for (int k = 0; k < 3; ++k)
    lines += (int64_t)std::abs(d.rt[k]) * d.w[(k + 1) % 3] * d.w[(k + 2) % 3];
  return lines;
}

// Run class of a defect whose class is set: the pair (class, run direction),
// added to the state's list on first appearance (-1: no class, no direction,
// a run bound above SELF_RUN_MAX, or the list is full).
void assign_run_class(ec_state* st, DevDefect& d) {
  d.rcls = -1;
  if (d.cls < 0 || (d.rt[0] == 0 && d.rt[1] == 0 && d.rt[2] == 0) || run_bound(d) > SELF_RUN_MAX) return;
  const std::array<int, 4> key{d.cls, d.rt[0], d.rt[1], d.rt[2]};
  for (size_t r = 0; r < st->runcls.size(); ++r)
    if (st->runcls[r] == key) {
      d.rcls = (int)r;
      return;
    }
  if ((int)st->runcls.size() < MAXRUN) {
    st->runcls.push_back(key);
    d.rcls = (int)st->runcls.size() - 1;
  }
}

void assign_class(ec_state* st, DevDefect& d) {
  std::array<double, 6> e;
  double s;
  direction(d, e, s);
  d.s = s;
  d.cls = -1;
  d.rcls = -1;
  if (s == 0.0) return;
  const size_t nrun_before = st->runcls.size();
  for (size_t c = 0; c < st->classes.size(); ++c)
    if (std::memcmp(st->classes[c].data(), e.data(), sizeof(double) * 6) == 0) {
      d.cls = (int)c;
      break;
    }
  if (d.cls < 0 && (int)st->classes.size() < MAXCLS) {
    st->classes.push_back(e);
    d.cls = (int)st->classes.size() - 1;
  }
  assign_run_class(st, d);
  if (d.rcls >= 0) st->max_runs = std::max<int64_t>(st->max_runs, run_bound(d));
  if (st->runcls.size() != nrun_before) st->gff_nrun = -1;
}

// Classes of a whole list, the same as assign_class on each defect in list
// order: the directions are computed on the workers, then looked up in list
// order (so indices follow first appearance) through a small open-addressing
// table keyed by the direction's bit pattern.
void assign_classes(ec_state* st, std::vector<DevDefect>& defs) {
  const size_t nd = defs.size();
  std::vector<std::array<double, 6>> dir(nd);
  std::vector<double> sc(nd);
  constexpr size_t CH = 256;
  st->ctx->pool->run((int)((nd + CH - 1) / CH), [&](int c) {
    for (size_t i = c * CH; i < std::min(nd, (c + 1) * CH); ++i) direction(defs[i], dir[i], sc[i]);
  });
  constexpr int HS = 2 * MAXCLS;  // at most MAXCLS keys
  static_assert((HS & (HS - 1)) == 0, "power-of-two table");
  int slot[HS];
  std::fill(slot, slot + HS, -1);
  auto home = [](const std::array<double, 6>& e) {
    uint64_t h = 1469598103934665603ull;
    for (double v : e) {
      uint64_t b;
      std::memcpy(&b, &v, 8);
      h = (h ^ b) * 1099511628211ull;
    }
    return (int)(h >> 58) & (HS - 1);
  };
  for (size_t i = 0; i < nd; ++i) {
    DevDefect& d = defs[i];
    d.s = sc[i];
    d.cls = -1;
    if (sc[i] == 0.0) continue;
    for (int k = home(dir[i]);; k = (k + 1) & (HS - 1)) {
      const int c = slot[k];
      if (c < 0) {
        if ((int)st->classes.size() < MAXCLS) {
          st->classes.push_back(dir[i]);
          d.cls = slot[k] = (int)st->classes.size() - 1;
        }
        break;
      }
      if (std::memcmp(st->classes[c].data(), dir[i].data(), sizeof(double) * 6) == 0) {
        d.cls = c;
        break;
      }
    }
  }
  for (size_t i = 0; i < nd; ++i) assign_run_class(st, defs[i]);
  int64_t mr = 0;
  for (size_t i = 0; i < nd; ++i)
    if (defs[i].rcls >= 0) mr = std::max(mr, run_bound(defs[i]));
  st->max_runs = (int)mr;
}

// ------------------------------------------------------------------ solve pipeline

double spec_valid_bytes(const ec_state* st, bool fp64) {
  return 6.0 * st->n * st->n * (st->n / 2 + 1) * (fp64 ? 16.0 : 8.0);
}

// ctr: the state's tile counters, or nullptr (fixed tile order; for solves
// that may run beside the state's own passes)
ec_status self_terms_beside(ec_state* st);
ec_status join_self(ec_state* st, hipStream_t s);

// `between` (may be empty) runs on the host after the forward x and y passes
// are enqueued and before the z pass is.
ec_status pipeline(ec_state* st, hipStream_t s, bool fp64, const int32_t* own, const int2* lnk, const DevDefect* defs,
                   int ndef, void* spec, double* sig, const double* add6, uint32_t* ctr,
                   const std::function<ec_status()>& between = {}, const double* bg = nullptr, int bg_mask = 0,
                   const double* bg3 = nullptr, bool covered_only = false) {
  const Prune full{0, st->n, 0, st->n};
  const double sb = spec_valid_bytes(st, fp64), fb = 48.0 * (double)st->n3;
  SpecGeom g{st->n, 0};
  g.P = spec_pitch(st->n, fp64);
  LAUNCH(st, s, PF_XF, 4.0 * (double)st->n3 + sb,
         launch_x_forward(fp64, own, lnk, defs, ndef, nullptr, spec, g, st->tw, ctr, s));
  LAUNCH(st, s, PF_Y, 2 * sb, launch_pencil(fp64, false, 1, spec, g, full, st->tw, ctr ? ctr : nullptr, s));
  if (between) {
    const ec_status r = between();
    if (r != EC_OK) return r;
  }
  LAUNCH(st, s, PF_Z, 2 * sb, launch_z_green(fp64, spec, g, st->C, full, st->tw, ctr ? ctr + 8 : nullptr, s));
  LAUNCH(st, s, PF_Y, 2 * sb, launch_pencil(fp64, true, 1, spec, g, full, st->tw, ctr ? ctr + 16 : nullptr, s));
  // covered_only: the spectrum and the owner map are read, and the stress is
  // stored at the covered voxels only (their bytes not counted here)
  LAUNCH(st, s, PF_XI, covered_only ? sb + 4.0 * (double)st->n3 : sb + (bg3 ? 2 : 1) * fb,
         launch_x_inverse(fp64, false, spec, sig, g, add6, st->tw, s, bg, bg_mask, bg3, own, !covered_only));
  return EC_OK;
}

// The whole stress field of the last solve, where it was stored only at the
// covered voxels: the x inverse pass again over the resident spectrum, with the
// mean term and the dislocation stresses the solve added.  Called by every
// entry point that reads the stress at other voxels or overwrites the spectrum.
ec_status ensure_sigma(ec_state* st, hipStream_t s) {
  st->whole_read = true;
  if (!st->sig_lazy) return EC_OK;
  const double sb = spec_valid_bytes(st, st->fp64), fb = 48.0 * (double)st->n3;
  const double* bg3 = st->bg3_on ? st->bg3 : nullptr;
  LAUNCH(st, s, PF_XI, sb + (bg3 ? 2 : 1) * fb,
         launch_x_inverse(st->fp64, false, st->spec, st->sig, st->g, st->add6, st->tw, s, st->bg, st->bg_mask, bg3,
                          st->own, true));
  st->sig_lazy = false;
  return EC_OK;
}

// out = -C:m for the state's crystal (the cubic stiffness applied in the cube
// frame when the crystal is rotated).
void neg_C_dot(const ec_state* st, const double* m, double* out) {
  double mc[6], t[6];
  if (st->frm)
    rot6(st->frmh.data(), m, mc);
  else
    std::copy(m, m + 6, mc);
  const Cubic& C = st->C;
  t[0] = -(C.C11 * mc[0] + C.C12 * (mc[1] + mc[2]));
  t[1] = -(C.C11 * mc[1] + C.C12 * (mc[0] + mc[2]));
  t[2] = -(C.C11 * mc[2] + C.C12 * (mc[0] + mc[1]));
  for (int a = 3; a < 6; ++a) t[a] = -2.0 * C.C44 * mc[a];
  if (st->frm)
    rot6(st->frmh.data() + 36, t, out);
  else
    std::copy(t, t + 6, out);
}

// Window of the discrete kernel G for this problem: six FP64 impulse solves.
// The context caches one window per problem (n, C, mean condition, frame); a
// wider one replaces it in the cache, and states still holding the narrower
// one keep it alive until they move on (see WinCache).
ec_status ensure_window(ec_state* st, int Dneed, hipStream_t s) {
  ec_ctx* c = st->ctx;
  Dneed = std::max(1, std::min(Dneed, st->n / 2));
  auto same_problem = [&](const WinCache& w) {
    return w.n == st->n && w.C11 == st->C.C11 && w.C12 == st->C.C12 && w.C44 == st->C.C44 && w.bc == st->prob.bc &&
           w.frame == st->frame;
  };
  {
    std::shared_ptr<const WinCache> found;
    {
      std::lock_guard<std::mutex> lk(c->mu);
      for (auto& w : c->wins)
        if (same_problem(*w) && w->D >= Dneed) {
          found = w;
          break;
        }
    }
    if (found) {
      if (found != st->win) st->gcls_D = -1;
      st->win = std::move(found);  // a window released here is freed outside the lock
      return EC_OK;
    }
  }
  const int D = Dneed;
  const int W = 2 * D + 1;
  const size_t Kbytes = (size_t)W * W * W * KWIN * sizeof(double);
  const int n = st->n;
  const int P64 = ((n / 2 + 1 + 7) / 8) * 8;
  const size_t sp64 = (size_t)6 * n * n * P64 * sizeof(double2);
  const size_t fbytes = (size_t)6 * st->n3 * 8;
  void *K = nullptr, *own = nullptr, *sp = nullptr, *sg = nullptr, *ad = nullptr, *imp = nullptr;
  const size_t ownbytes = (size_t)st->n3 * 4;
  ec_status r;
  if ((r = ledger_alloc(c, Kbytes, &K)) != EC_OK) return r;
  auto cleanup = [&]() {
    ledger_free(c, own, ownbytes);
    ledger_free(c, imp, 6 * sizeof(DevDefect) + 64);
    ledger_free(c, sp, sp64);
    ledger_free(c, sg, fbytes);
    ledger_free(c, ad, 6 * 64);
  };
  if ((r = ledger_alloc(c, ownbytes, &own)) != EC_OK || (r = ledger_alloc(c, sp64, &sp)) != EC_OK ||
      (r = ledger_alloc(c, fbytes, &sg)) != EC_OK || (r = ledger_alloc(c, 6 * 64, &ad)) != EC_OK ||
      (r = ledger_alloc(c, 6 * sizeof(DevDefect) + 64, &imp)) != EC_OK) {
    cleanup();
    ledger_free(c, K, Kbytes);
    return r;
  }
  const bool prof = st->prof;
  st->prof = false;
  auto body = [&]() -> ec_status {
    // additive mean stress per impulse: -C:<eps*> for mean strain zero, else 0
    double add[6][8] = {};
    if (st->prob.bc == EC_MEAN_STRAIN_ZERO)
      for (int b = 0; b < 6; ++b) {
        double m[6] = {0, 0, 0, 0, 0, 0};
        m[b] = 1.0 / (double)st->n3;
        neg_C_dot(st, m, add[b]);
      }
    // six one-voxel "defects" with unit eigenstrain component b at voxel 0
    DevDefect unit[6];
    std::memset(unit, 0, sizeof unit);
    for (int b = 0; b < 6; ++b) {
      double e[6] = {0, 0, 0, 0, 0, 0}, ec[6];
      e[b] = 1.0;
      if (st->frm)
        to_cube(st->frame.data(), e, ec);  // the unit component in the cube frame
      else
        std::copy(e, e + 6, ec);
      for (int a = 0; a < 6; ++a) unit[b].efix[a] = (int64_t)std::llrint(ec[a] * FIX_SCALE);
      set_efd(unit[b]);
    }
    DevDefect* dunit = (DevDefect*)imp;
    int2* dlnk = (int2*)((char*)imp + 6 * sizeof(DevDefect));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(ad, add, sizeof add, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dunit, unit, sizeof unit, hipMemcpyHostToDevice));
    HIPCHK(launch_fill_i32((int32_t*)own, st->n3, -1, s));
    HIPCHK(hipMemsetAsync(K, 0, Kbytes, s));
    for (int b = 0; b < 6; ++b) {
      HIPCHK(launch_fill_i32((int32_t*)own, 1, b, s));  // voxel 0 owned by unit defect b
      ec_status q =
          pipeline(st, s, true, (const int32_t*)own, dlnk, dunit, 6, sp, (double*)sg, (const double*)ad + 8 * b, nullptr);
      if (q != EC_OK) return q;
      HIPCHK(launch_window_crop((const double*)sg, n, D, b, (double*)K, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return EC_OK;
  };
  r = body();
  st->prof = prof;
  cleanup();
  if (r != EC_OK) {
    ledger_free(c, K, Kbytes);
    return r;
  }
  auto w = std::make_shared<WinCache>();
  w->ctx = c;
  w->n = st->n;
  w->C11 = st->C.C11;
  w->C12 = st->C.C12;
  w->C44 = st->C.C44;
  w->bc = st->prob.bc;
  w->frame = st->frame;
  w->D = D;
  w->K = (double*)K;
  w->bytes = Kbytes;
  std::vector<std::shared_ptr<WinCache>> dropped;  // released after the lock
  {
    std::lock_guard<std::mutex> lk(c->mu);
    for (auto it = c->wins.begin(); it != c->wins.end();) {
      if (same_problem(**it) && (*it)->D <= D) {
        dropped.push_back(std::move(*it));
        it = c->wins.erase(it);
      } else {
        ++it;
      }
    }
    c->wins.push_back(w);
  }
  st->win = w;
  st->gcls_D = -1;
  return EC_OK;
}

int window_need(const ec_state* st) {
  int D = 1;
  for (const auto& d : st->hdefs)
    for (int k = 0; k < 3; ++k) D = std::max(D, d.w[k] - 1);
  return std::min(D, st->n / 2);
}

// Direction classes of the current defect list, assigned on the host (ids in
// order of first appearance) and written into the device table.
ec_status ensure_classes(ec_state* st, hipStream_t s) {
  if (st->classes_ok) return EC_OK;
  const size_t nd = st->hdefs.size();
  ec_status r;
  if (nd > 0 && (r = st_grow(st, &st->tags, &st->tags_cap, nd)) != EC_OK) return r;
  const std::vector<std::array<double, 6>> old = st->classes;
  const std::vector<std::array<int, 4>> oldrun = st->runcls;
  st->classes.clear();
  st->runcls.clear();
  assign_classes(st, st->hdefs);
  if (old != st->classes) st->gcls_ncls = -1;
  if (oldrun != st->runcls) st->gff_nrun = -1;
  if (nd > 0) {
    char* hp = nullptr;
    if ((r = pin_begin(st->pin_tags, nd * sizeof(ClassTag), &hp)) != EC_OK) return r;
    ClassTag* t = (ClassTag*)hp;
    for (size_t i = 0; i < nd; ++i) t[i] = ClassTag{st->hdefs[i].s, st->hdefs[i].cls, st->hdefs[i].rcls};
    HIPCHK(hipMemcpyAsync(st->tags, hp, nd * sizeof(ClassTag), hipMemcpyHostToDevice, s));
    if ((r = pin_end(st->pin_tags, s)) != EC_OK) return r;
    LAUNCH(st, s, PF_OTHER, 0, launch_set_class(st->db[st->cur].tab, (int)nd, st->tags, s));
  }
  st->classes_ok = true;
  return EC_OK;
}

// Kernel window covering every footprint's pair offsets plus `reach` voxels
// (the largest jump of a jump probe; 0 for the self terms), and the class
// windows on it.  Classes must be current.
ec_status ensure_windows(ec_state* st, int reach, hipStream_t s) {
  ec_status r = ensure_window(st, window_need(st) + reach, s);
  if (r != EC_OK) return r;
  const WinCache* w = st->win.get();
  const int D = w->D;
  const int W = 2 * D + 1;
  const size_t W3 = (size_t)W * W * W;
  const int ncls = (int)st->classes.size();
  if (st->gcls_D != D || st->gcls_ncls != ncls) {
    const size_t need_b = std::max<size_t>(1, (size_t)ncls) * W3 * sizeof(double);
    if (need_b > st->gcls_bytes) {
      void* q = nullptr;
      if ((r = ledger_alloc(st->ctx, need_b, &q)) != EC_OK) return r;
      if (st->gcls) HIPCHK(hipDeviceSynchronize());  // self-term kernels may still read the old windows
      ledger_free(st->ctx, st->gcls, st->gcls_bytes);
      st->held += need_b;
      st->held -= std::min(st->held, st->gcls_bytes);
      st->gcls = (double*)q;
      st->gcls_bytes = need_b;
    }
    std::vector<double> dirs(6 * std::max(ncls, 1), 0.0);
    for (int c = 0; c < ncls; ++c)
      for (int a = 0; a < 6; ++a) dirs[6 * c + a] = st->classes[c][a];
    HIPCHK(hipMemcpyAsync(st->dirs, dirs.data(), dirs.size() * sizeof(double), hipMemcpyHostToDevice, s));
    LAUNCH(st, s, PF_OTHER, W3 * ncls * 8.0 * 22, launch_class_windows(w->K, D, st->dirs, ncls, st->gcls, s));
    HIPCHK(hipStreamSynchronize(s));  // dirs staging buffer is pageable
    st->gcls_D = D;
    st->gcls_ncls = ncls;
    st->gff_D = -1;  // the run tables come from the class windows
  }
  // the run tables on the state's own window need (<= D), so that they do not
  // depend on the width the shared window has for other states
  const int nrun = (int)st->runcls.size();
  const int Drun = std::min(D, window_need(st));
  if (st->gff_D != Drun || st->gff_nrun != nrun) {
    const size_t Wr = 2 * (size_t)Drun + 1;
    const size_t need_b = std::max<size_t>(1, (size_t)nrun) * Wr * Wr * Wr * sizeof(double);
    if (need_b > st->gff_bytes) {
      void* q = nullptr;
      if ((r = ledger_alloc(st->ctx, need_b, &q)) != EC_OK) return r;
      if (st->gff) HIPCHK(hipDeviceSynchronize());  // self-term kernels may still read the old tables
      ledger_free(st->ctx, st->gff, st->gff_bytes);
      st->held += need_b;
      st->held -= std::min(st->held, st->gff_bytes);
      st->gff = (double*)q;
      st->gff_bytes = need_b;
    }
    std::vector<int4> info(std::max(nrun, 1));
    for (int k = 0; k < nrun; ++k)
      info[k] = make_int4(st->runcls[k][0], st->runcls[k][1], st->runcls[k][2], st->runcls[k][3]);
    HIPCHK(hipMemcpyAsync(st->runinfo, info.data(), info.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    LAUNCH(st, s, PF_OTHER, Wr * Wr * Wr * nrun * 16.0,
           launch_run_tables(st->gcls, D, Drun, st->runinfo, nrun, st->gff, s));
    HIPCHK(hipStreamSynchronize(s));  // info staging buffer is pageable
    st->gff_D = Drun;
    st->gff_nrun = nrun;
  }
  return EC_OK;
}

RunTables run_tables(const ec_state* st) {
  RunTables t;
  t.ff = st->gff;
  t.info = st->runinfo;
  t.nrun = st->gff_nrun > 0 && st->gff_D > 0 ? st->gff_nrun : 0;
  t.D = std::max(st->gff_D, 0);
  t.max_runs = st->max_runs;
  return t;
}

// Self-term work-list capacity of the pair path: at most 64 items per defect
// off the run path, fewer for small boxes (the device plan, from the footprint
// counts, never needs more); 0 when every defect takes the run path.  The run
// tables must be current (after ensure_windows).
int64_t self_work_cap(const ec_state* st) {
  const int nrun = st->gff_D > 0 ? st->gff_nrun : 0, Dr = st->gff_D;
  int64_t cap = 0;
  for (const auto& d : st->hdefs) {
    if (d.rcls >= 0 && d.rcls < nrun && d.w[0] <= Dr + 1 && d.w[1] <= Dr + 1 && d.w[2] <= Dr + 1) continue;
    const double m = (double)box_volume(d);
    const double k = std::ceil(m * (m + 1) / 2 / 32768.0);
    cap += (int64_t)std::min(64.0, std::max(1.0, k));
  }
  return cap;
}

ec_status compute_self_terms(ec_state* st, hipStream_t s) {
  ec_status r = ensure_classes(st, s);
  if (r != EC_OK) return r;
  if ((r = ensure_windows(st, 0, s)) != EC_OK) return r;
  const WinCache* w = st->win.get();
  const int D = w->D;
  const int64_t cap = self_work_cap(st);
  if ((r = st_grow(st, &st->work, &st->work_cap, (size_t)std::max<int64_t>(cap, 1))) != EC_OK) return r;
  if ((r = st_grow(st, &st->partial, &st->partial_cap, (size_t)std::max<int64_t>(cap, 1))) != EC_OK) return r;
  if ((r = st_grow(st, &st->wbeg, &st->wbeg_cap, (size_t)st->ndef + 1)) != EC_OK) return r;
  const DefBuf& b = st->db[st->cur];
  LAUNCH(st, s, PF_SELF, 0,
         launch_self_terms(b.tab, st->ndef, b.cnt, b.ids, st->n, w->K, st->gcls, D, run_tables(st), st->work, cap,
                           st->wbeg, st->partial, st->runsum, st->h3c, st->B, s));
  st->B_valid = true;
  return EC_OK;
}

// Make stream s wait for self terms still running on the side stream.
ec_status join_self(ec_state* st, hipStream_t s) {
  if (!st->self_pending) return EC_OK;
  HIPCHK(hipStreamWaitEvent(s, st->ev_self, 0));
  st->self_pending = false;
  return EC_OK;
}

// Self terms of the list just rasterised on stream s, computed on the side
// stream after ev_fill while s runs the Fourier passes.
ec_status self_terms_beside(ec_state* st) {
  if (!st->side) {
    HIPCHK(hipStreamCreateWithFlags(&st->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&st->ev_self, hipEventDisableTiming));
  }
  HIPCHK(hipStreamWaitEvent(st->side, st->ev_fill, 0));
  ec_status r = compute_self_terms(st, st->side);
  if (r != EC_OK) return r;
  HIPCHK(hipEventRecord(st->ev_self, st->side));
  st->self_pending = true;
  return EC_OK;
}

ec_status copy_out(void* dst, const void* src, size_t bytes, bool on_device, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  if (!on_device) HIPCHK(hipStreamSynchronize(s));
  return EC_OK;
}

// A per-defect output: to the host through the state's pinned bounce buffer (a
// direct copy into pageable memory is staged by the runtime), synchronously.
// Small results returned to a waiting host caller: copied into pinned memory
// behind an event that the calling thread polls, since a thread blocked in
// the driver's stream synchronisation resumes tens of microseconds after the
// copy has landed.
ec_status copy_small(ec_state* st, void* dst, const void* src, size_t bytes, bool on_device, hipStream_t s) {
  if (on_device || bytes == 0) return copy_out(dst, src, bytes, on_device, s);
  char* hp = nullptr;
  ec_status r = pin_begin(st->pin_out, bytes, &hp);
  if (r != EC_OK) return r;
  HIPCHK(hipMemcpyAsync(hp, src, bytes, hipMemcpyDeviceToHost, s));
  HIPCHK(hipEventRecord(st->pin_out.ev, s));
  hipError_t q;
  while ((q = hipEventQuery(st->pin_out.ev)) == hipErrorNotReady) {
  }
  HIPCHK(q);
  std::memcpy(dst, hp, bytes);
  return EC_OK;
}

ec_status write_field(ec_state* st, int which, void* out, bool on_device, hipStream_t s) {
  {
    const ec_status r0 = ensure_sigma(st, s);
    if (r0 != EC_OK) return r0;
  }
  const bool f32 = !st->fp64;
  const size_t bytes = (size_t)6 * st->n3 * (f32 ? 4 : 8);
  if (on_device) {
    const DefBuf& b = st->db[st->cur];
    LAUNCH(st, s, PF_OTHER, 96.0 * st->n3,
           launch_sig_to_out(st->sig, st->own, b.lnk, b.tab, st->ndef, st->n3, st->C, which, f32, out, s));
    return EC_OK;
  }
  void* tmp = nullptr;
  ec_status r = ledger_alloc(st->ctx, bytes, &tmp);
  if (r != EC_OK) return r;
  const DefBuf& b = st->db[st->cur];
  hipError_t e = launch_sig_to_out(st->sig, st->own, b.lnk, b.tab, st->ndef, st->n3, st->C, which, f32, tmp, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  ledger_free(st->ctx, tmp, bytes);
  if (e != hipSuccess) return fail(EC_ERR_DEVICE, "field output: %s", hipGetErrorString(e));
  return EC_OK;
}

ec_status ensure_per_defect(ec_state* st, size_t ndef) {
  if (ndef <= st->pd_cap && st->B) return EC_OK;
  size_t cap = std::max<size_t>(ndef, 16);
  void *b = nullptr, *e = nullptr, *s6 = nullptr, *rs = nullptr;
  ec_status r;
  if ((r = ledger_alloc(st->ctx, cap * 8, &b)) != EC_OK) return r;
  if ((r = ledger_alloc(st->ctx, cap * 8, &e)) != EC_OK) {
    ledger_free(st->ctx, b, cap * 8);
    return r;
  }
  if ((r = ledger_alloc(st->ctx, cap * 48, &s6)) != EC_OK) {
    ledger_free(st->ctx, b, cap * 8);
    ledger_free(st->ctx, e, cap * 8);
    return r;
  }
  if ((r = ledger_alloc(st->ctx, cap * 8, &rs)) != EC_OK) {
    ledger_free(st->ctx, b, cap * 8);
    ledger_free(st->ctx, e, cap * 8);
    ledger_free(st->ctx, s6, cap * 48);
    return r;
  }
  // the current list's values move along: a call that fails after growing
  // these leaves the state's self terms and energies as they were
  if (st->B && st->pd_cap > 0) {
    const size_t k = st->pd_cap;
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(b, st->B, k * 8, hipMemcpyDeviceToDevice) != hipSuccess ||
        hipMemcpy(e, st->E, k * 8, hipMemcpyDeviceToDevice) != hipSuccess ||
        hipMemcpy(s6, st->S6, k * 48, hipMemcpyDeviceToDevice) != hipSuccess ||
        hipMemcpy(rs, st->runsum, k * 8, hipMemcpyDeviceToDevice) != hipSuccess) {
      ledger_free(st->ctx, b, cap * 8);
      ledger_free(st->ctx, e, cap * 8);
      ledger_free(st->ctx, s6, cap * 48);
      ledger_free(st->ctx, rs, cap * 8);
      return fail(EC_ERR_DEVICE, "device copy failed while growing the per-defect buffers");
    }
  }
  ledger_free(st->ctx, st->B, st->pd_cap * 8);
  ledger_free(st->ctx, st->E, st->pd_cap * 8);
  ledger_free(st->ctx, st->S6, st->pd_cap * 48);
  ledger_free(st->ctx, st->runsum, st->pd_cap * 8);
  st->held += cap * 72;
  st->held -= std::min(st->held, st->pd_cap * 72);
  st->B = (double*)b;
  st->E = (double*)e;
  st->S6 = (double*)s6;
  st->runsum = (double*)rs;
  st->pd_cap = cap;
  return EC_OK;
}

ec_status ensure_defbuf(ec_state* st, DefBuf& b, size_t ndef) {
  if (ndef + 1 <= b.cap && b.tab) return EC_OK;
  size_t cap = std::max<size_t>(ndef + 1, 16);
  void *t = nullptr, *c = nullptr;
  ec_status r;
  if ((r = ledger_alloc(st->ctx, cap * sizeof(DevDefect), &t)) != EC_OK) return r;
  if ((r = ledger_alloc(st->ctx, cap * 4, &c)) != EC_OK) {
    ledger_free(st->ctx, t, cap * sizeof(DevDefect));
    return r;
  }
  ledger_free(st->ctx, b.tab, b.cap * sizeof(DevDefect));
  ledger_free(st->ctx, b.cnt, b.cap * 4);
  st->held += cap * (sizeof(DevDefect) + 4);
  st->held -= std::min(st->held, b.cap * (sizeof(DevDefect) + 4));
  b.tab = (DevDefect*)t;
  b.cnt = (int32_t*)c;
  b.cap = cap;
  return EC_OK;
}

ec_status fetch_counts(ec_state* st) {
  if (st->hcnt_ok) return EC_OK;
  st->hcnt.assign(st->ndef, 0);
  HIPCHK(hipDeviceSynchronize());
  if (st->ndef > 0)
    HIPCHK(hipMemcpy(st->hcnt.data(), st->db[st->cur].cnt, st->ndef * 4, hipMemcpyDeviceToHost));
  st->hcnt_ok = true;
  return EC_OK;
}

// Smallest cyclic interval of [0, n) covering [lo1, lo1+w1) and [lo2, lo2+w2).
void cyclic_cover(int lo1, int w1, int lo2, int w2, int n, int& lo, int& len) {
  std::vector<char> mark(n, 0);
  for (int i = 0; i < w1; ++i) mark[(lo1 + i) % n] = 1;
  for (int i = 0; i < w2; ++i) mark[(lo2 + i) % n] = 1;
  int best = 0, best_end = 0;
  for (int start = 0; start < n; ++start) {
    if (mark[start] || !mark[(start + n - 1) % n]) continue;  // zero run must start after a mark
    int l = 0;
    while (l < n && !mark[(start + l) % n]) ++l;
    if (l > best) {
      best = l;
      best_end = (start + l) % n;
    }
  }
  if (best == 0) {
    lo = 0;
    len = n;
    return;
  }
  lo = best_end;
  len = n - best;
}

// Device form of a crystal frame (rows of A: the cell axes in cube
// coordinates): the maps of the six tensor components cell -> cube
// (T_c = A^T T A) and cube -> cell (T = A T_c A^T), then A itself.
static_assert(sizeof(ec_problem) == 120 && offsetof(ec_problem, frame) == 48, "ec_problem layout of include/ec.h");
static_assert(sizeof(ec_line) == 56 && offsetof(ec_line, axis) == 24 && offsetof(ec_line, b) == 32,
              "ec_line layout of include/ec.h");

void frame_maps(const double* A, double* out) {
  static const int P[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};
  auto a = [&](int i, int p) { return A[3 * i + p]; };
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) {
      const int p = P[r][0], q = P[r][1], i = P[c][0], j = P[c][1];
      out[6 * r + c] = a(i, p) * a(j, q) + (i != j ? a(j, p) * a(i, q) : 0.0);
      const int ii = P[r][0], jj = P[r][1], pp = P[c][0], qq = P[c][1];
      out[36 + 6 * r + c] = a(ii, pp) * a(jj, qq) + (pp != qq ? a(ii, qq) * a(jj, pp) : 0.0);
    }
  for (int k = 0; k < 9; ++k) out[72 + k] = A[k];
}

// Commits the quantised list h (ndef entries in the pinned staging buffer of
// the device table, pin_begin already called on it) and solves: footprint
// slots from the box volumes, the old eigenstrain out and the new one in, the
// Fourier passes, the self terms beside them.  keep_self: h is the current list
// with whole-voxel translations only (same order, shapes and classes, the
// classes already in h), so the self terms, classes and windows stay valid.
// With h null, fill_dev writes the new table on the device instead: the list
// is the current one with whole-voxel translations (keep_self must hold), so
// the slots stay, and the caller brings the host copy of the list up to date.
ec_status solve_table(ec_state* st, DevDefect* h, int32_t ndef, hipStream_t s, bool keep_self = false,
                      const std::function<ec_status(DevDefect*)>& fill_dev = {}) {
  ec_status r;
  const char* hp = (const char*)h;
  int64_t total = 0;
  if (h) {
    for (int i = 0; i < ndef; ++i) {
      h[i].slot = total;
      total += box_volume(h[i]);
    }
  } else {
    total = st->ids_used;
  }
  // buffers of the new list (the spare set)
  DefBuf& nb = st->db[1 - st->cur];
  size_t idcap = (size_t)nb.ids_cap, lkcap = (size_t)nb.ids_cap;
  const size_t need = (size_t)std::max<int64_t>(total, 1);
  if ((r = ensure_defbuf(st, nb, ndef)) != EC_OK || (r = ensure_per_defect(st, ndef)) != EC_OK ||
      (r = st_grow(st, &nb.ids, &idcap, need)) != EC_OK || (r = st_grow(st, &nb.lnk, &lkcap, need)) != EC_OK)
    return r;
  nb.ids_cap = (int64_t)std::min(idcap, lkcap);
  if (ndef > 0 && h) {
    HIPCHK(hipMemcpyAsync(nb.tab, hp, ndef * sizeof(DevDefect), hipMemcpyHostToDevice, s));
    if ((r = pin_end(st->pin_tab, s)) != EC_OK) return r;
  } else if (ndef > 0 && (r = fill_dev(nb.tab)) != EC_OK) {
    return r;
  }
  // commit: remove the old eigenstrain, add the new one
  if ((r = join_self(st, s)) != EC_OK) return r;
  const DefBuf& ob = st->db[st->cur];
  if (st->ndef > 0)
    LAUNCH(st, s, PF_RASTER, 0, launch_unraster(ob.tab, st->ndef, ob.cnt, ob.ids, st->own, s));
  LAUNCH(st, s, PF_RASTER, 0, launch_raster_fill(nb.tab, ndef, st->n, nb.ids, nb.lnk, nb.cnt, st->own, s));
  if (!st->ev_fill) HIPCHK(hipEventCreateWithFlags(&st->ev_fill, hipEventDisableTiming));
  HIPCHK(hipEventRecord(st->ev_fill, s));
  st->cur = 1 - st->cur;
  st->hcnt_ok = false;
  st->ndef = ndef;
  st->ids_used = total;
  if (!keep_self) {
    st->B_valid = false;
    st->classes_ok = false;
    st->jx_ok = false;
  }
  st->jdE_ok = false;
  LAUNCH(st, s, PF_OTHER, 0,
         launch_mean_stress(nb.tab, nb.cnt, ndef, st->n3, st->C, st->prob.bc, st->add6, s));
  // Fourier solve.  The self terms run on the side stream beside the forward x and y passes
  // (after the rasterisation), and the z pass waits for them: its workgroups
  // each take most of a CU's LDS, so self-term blocks still resident would
  // hold some of them back and stretch the pass.
  auto beside = [&]() -> ec_status {
    // host copies of the list while the device works (the staging buffer is
    // only read by the pending upload); the self-term set-up reads them
    if (h) {
      st->hdefs.assign(h, h + ndef);
      st->hcap.resize(ndef);
      for (int i = 0; i < ndef; ++i) st->hcap[i] = box_volume(h[i]);
    }
    if (ndef == 0 || keep_self) return EC_OK;
    // self terms that cannot be set up now (an allocation of their windows or
    // work lists failed) are left to the next energies call, which reports
    // the failure if it recurs; the solve itself has all it needs
    if (self_terms_beside(st) != EC_OK) {
      st->B_valid = false;
      return EC_OK;
    }
    return join_self(st, s);
  };
  // the stress of dislocation lines, if any, is added by the x inverse pass
  const bool covered = !st->whole_read;
  r = pipeline(st, s, st->fp64, st->own, nb.lnk, nb.tab, ndef, st->spec, st->sig, st->add6, st->tilectr, beside, st->bg,
               st->bg_mask, st->bg3_on ? st->bg3 : nullptr, covered);
  if (r != EC_OK) return r;
  st->solved = true;
  st->sig_lazy = covered;
  st->whole_read = false;
  return EC_OK;
}

// Biased frequencies and the frequency-line choice from the jump energies of
// the current list; with u, the Poisson gate of the time step dt first (-1: no
// event).  Arguments already validated.
ec_status run_select(ec_state* st, const double* Em, double nu0, double kT, const double* xi, const double* u,
                     double dt, hipStream_t s, double* nu_out, int32_t* choice_out, bool on_device,
                     bool choice_kept = false) {
  const int nd = st->ndef, nj = st->jn;
  const size_t nu = (size_t)nd * nj;
  ec_status r;
  if ((r = st_grow(st, &st->jsel, &st->jsel_cap, 3 * (size_t)nd)) != EC_OK) return r;
  if (nu_out && (r = st_grow(st, &st->jnu, &st->jnu_cap, nu)) != EC_OK) return r;
  const bool want_choice = choice_out || choice_kept;
  if (want_choice && (r = st_grow(st, &st->jchoice, &st->jchoice_cap, (size_t)nd)) != EC_OK) return r;
  char* hp = nullptr;
  if ((r = pin_begin(st->pin_jump, 3 * (size_t)nd * 8, &hp)) != EC_OK) return r;
  std::memcpy(hp, Em, (size_t)nd * 8);
  if (xi) std::memcpy(hp + (size_t)nd * 8, xi, (size_t)nd * 8);
  if (u) std::memcpy(hp + 2 * (size_t)nd * 8, u, (size_t)nd * 8);
  HIPCHK(hipMemcpyAsync(st->jsel, hp, 3 * (size_t)nd * 8, hipMemcpyHostToDevice, s));
  if ((r = pin_end(st->pin_jump, s)) != EC_OK) return r;
  LAUNCH(st, s, PF_OTHER, 0,
         launch_jump_select(st->jdE, nd, nj, st->jsel, nu0, kT, xi ? st->jsel + nd : nullptr,
                            u ? st->jsel + 2 * nd : nullptr, dt, nu_out ? st->jnu : nullptr,
                            want_choice ? st->jchoice : nullptr, s));
  if (nu_out && (r = copy_small(st, nu_out, st->jnu, nu * 8, on_device, s)) != EC_OK) return r;
  if (choice_out) return copy_small(st, choice_out, st->jchoice, (size_t)nd * 4, on_device, s);
  return EC_OK;
}

// Footprint of a quantised defect on the host, ascending voxel ids: the same
// box enumeration and membership test as the rasteriser.
void footprint_ids(const DevDefect& d, int n, std::vector<int32_t>& ids) {
  ids.clear();
  for (int iz = 0; iz < d.w[2]; ++iz)
    for (int iy = 0; iy < d.w[1]; ++iy) {
      const int y = box_axis(d.lo[1], d.w[1], n, iy), z = box_axis(d.lo[2], d.w[2], n, iz);
      for (int ix = 0; ix < d.w[0]; ++ix) {
        const int x = box_axis(d.lo[0], d.w[0], n, ix);
        if (member(d, n, x, y, z)) ids.push_back((z * n + y) * n + x);
      }
    }
}

// Moves defect idx to the quantised record nd (validated): by linearity only
// the eigenstrain difference is solved and the resident stress accumulated;
// a whole-voxel move of the same shape translates the footprint.
ec_status update_q(ec_state* st, int32_t idx, DevDefect nd, hipStream_t s) {
  {
    ec_status rc = join_self(st, s);
    if (rc == EC_OK) rc = ensure_classes(st, s);
    if (rc == EC_OK) rc = ensure_sigma(st, s);  // the update adds to the whole field
    if (rc != EC_OK) return rc;
  }
  st->jdE_ok = false;
  const DevDefect od = st->hdefs[idx];
  const int n = st->n;
  // whole-voxel move of the same shape: the footprint translates and B_i is unchanged
  bool hop = od.kind == nd.kind && od.R2q == nd.R2q && od.eq == nd.eq && od.mm == nd.mm;
  for (int k = 0; k < 3 && hop; ++k) hop = od.m[k] == nd.m[k] && ((nd.cq[k] - od.cq[k]) % QSUB) == 0;
  for (int a = 0; a < 6 && hop; ++a) hop = od.efix[a] == nd.efix[a];
  if (!hop) st->jx_ok = false;  // a translation keeps the probe's cross parts
  int sh[3] = {0, 0, 0};
  if (hop)
    for (int k = 0; k < 3; ++k) {
      int d = ((nd.cq[k] - od.cq[k]) / QSUB) % n;
      if (d < 0) d += n;
      if (d >= n / 2) d -= n;
      sh[k] = d;
    }
  const size_t ncls_before = st->classes.size(), nrun_before = st->runcls.size();
  if (hop) {
    nd.cls = od.cls;
    nd.s = od.s;
    nd.rcls = od.rcls;
  } else {
    assign_class(st, nd);
  }
  DefBuf& b = st->db[st->cur];
  std::vector<int32_t> new_ids;
  int cnt_new = -1;  // hop: same count as the old footprint (read on the device)
  int64_t cap_new = st->hcap[idx];
  nd.slot = od.slot;
  ec_status r;
  if (!hop) {
    footprint_ids(nd, n, new_ids);
    cnt_new = (int)new_ids.size();
    size_t ucap = (size_t)st->upd_cap;
    if ((r = st_grow(st, &st->upd_ids, &ucap, std::max<size_t>(cnt_new, 1))) != EC_OK) {
      st->classes.resize(ncls_before);
      st->runcls.resize(nrun_before);
      return r;
    }
    st->upd_cap = (int64_t)ucap;
    if (cnt_new > st->hcap[idx]) {  // does not fit the old slot: take a new one at the end
      nd.slot = st->ids_used;
      cap_new = box_volume(nd);
      size_t icap = (size_t)b.ids_cap, lcap = (size_t)b.ids_cap;
      const size_t need = (size_t)(st->ids_used + cap_new);
      if ((r = st_grow(st, &b.ids, &icap, need, true, s)) != EC_OK ||
          (r = st_grow(st, &b.lnk, &lcap, need, true, s)) != EC_OK) {
        st->classes.resize(ncls_before);
        st->runcls.resize(nrun_before);
        return r;
      }
      b.ids_cap = (int64_t)std::min(icap, lcap);
    }
  }
  // rows of the eigenstrain change
  int ylo, ylen, zlo, zlen;
  cyclic_cover(od.lo[1], od.w[1], nd.lo[1], nd.w[1], n, ylo, ylen);
  cyclic_cover(od.lo[2], od.w[2], nd.lo[2], nd.w[2], n, zlo, zlen);
  double dadd[6] = {0, 0, 0, 0, 0, 0};
  if (!hop && st->prob.bc == EC_MEAN_STRAIN_ZERO) {
    // mean strain zero: the mean stress moves with the eigenstrain volume
    if ((r = fetch_counts(st)) != EC_OK) return r;
    double m[6];
    for (int a = 0; a < 6; ++a)
      m[a] = ((double)cnt_new * nd.E[a] - (double)st->hcnt[idx] * od.E[a]) / (double)st->n3;
    neg_C_dot(st, m, dadd);
  }
  // --- commit
  // [old E 48][new E 48][dadd 48][count 8][record]: the eigenstrain change is
  // -E_old on the old footprint and +E_new on the new one; both as the
  // rasterised field holds them (the fixed-point components, in the cube
  // frame of a rotated crystal, where the sparse transform works)
  char* up = nullptr;
  if ((r = pin_begin(st->pin_upd, 152 + sizeof(DevDefect), &up)) != EC_OK) return r;
  {
    double eo[6], en[6];
    for (int a = 0; a < 6; ++a) {
      eo[a] = (double)od.efix[a] * FIX_INV;
      en[a] = (double)nd.efix[a] * FIX_INV;
    }
    std::memcpy(up, eo, 48);
    std::memcpy(up + 48, en, 48);
  }
  std::memcpy(up + 96, dadd, 48);
  std::memcpy(up + 144, &cnt_new, 4);
  std::memcpy(up + 152, &nd, sizeof nd);
  if (!hop && cnt_new > 0) {
    char* ip = nullptr;
    if ((r = pin_begin(st->pin_ids, (size_t)cnt_new * 4, &ip)) != EC_OK) return r;
    std::memcpy(ip, new_ids.data(), (size_t)cnt_new * 4);
    HIPCHK(hipMemcpyAsync(st->upd_ids, ip, (size_t)cnt_new * 4, hipMemcpyHostToDevice, s));
    if ((r = pin_end(st->pin_ids, s)) != EC_OK) return r;
  }
  HIPCHK(hipMemcpyAsync(st->updE, up, 96, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(st->add6 + 12, up + 96, 48, hipMemcpyHostToDevice, s));
  const int32_t* oids = b.ids + od.slot;
  const int32_t* ocnt = b.cnt + idx;
  const int32_t* nids = hop ? nullptr : st->upd_ids;
  {
    const bool fp64 = st->fp64;
    const double sb = spec_valid_bytes(st, fp64), fb = 48.0 * (double)st->n3;
    const double frac_z = (double)zlen / n;
    LAUNCH(st, s, PF_XF, frac_z * ylen / n * sb,
           launch_x_forward_sparse(fp64, oids, ocnt, nids, cnt_new, sh[0], sh[1], sh[2], st->updE, st->spec, st->g,
                                   ylo, ylen, zlo, zlen, st->tw, st->tilectr, s));
    const Prune py{ylo, ylen, zlo, zlen};
    LAUNCH(st, s, PF_Y, 2 * frac_z * sb, launch_pencil(fp64, false, 1, st->spec, st->g, py, st->tw, st->tilectr, s));
    const Prune pz{zlo, zlen, 0, n};
    const Prune full{0, n, 0, n};
    LAUNCH(st, s, PF_Z, (1 + frac_z) * sb,
           launch_z_green(fp64, st->spec, st->g, st->C, pz, st->tw, st->tilectr + 8, s));
    LAUNCH(st, s, PF_Y, 2 * sb, launch_pencil(fp64, true, 1, st->spec, st->g, full, st->tw, st->tilectr + 16, s));
    LAUNCH(st, s, PF_XI, sb + 2 * fb,
           launch_x_inverse(fp64, true, st->spec, st->sig, st->g, st->add6 + 12, st->tw, s));
  }
  // membership lists and footprint ids of the moved defect (after the sparse
  // forward pass, which still reads the old footprint)
  LAUNCH(st, s, PF_RASTER, 0,
         launch_move_lists(idx, st->ndef, ocnt, od.slot, nids, cnt_new, nd.slot, sh[0], sh[1], sh[2], n, b.ids, b.lnk,
                           st->own, s));
  if (!hop) {
    HIPCHK(hipMemcpyAsync(b.cnt + idx, up + 144, 4, hipMemcpyHostToDevice, s));
    if (nd.slot != od.slot) {
      st->ids_used += cap_new;
      st->hcap[idx] = cap_new;
    }
    if (st->hcnt_ok) st->hcnt[idx] = cnt_new;
    st->B_valid = false;
    if (st->classes.size() != ncls_before) st->gcls_ncls = -1;
  }
  HIPCHK(hipMemcpyAsync(b.tab + idx, up + 152, sizeof nd, hipMemcpyHostToDevice, s));
  if ((r = pin_end(st->pin_upd, s)) != EC_OK) return r;
  st->hdefs[idx] = nd;
  return EC_OK;
}

// The hop job of moving defect idx of st to the quantised record nd, if that
// move is a whole-voxel translation of the same shape and eigenstrain (false
// otherwise).  The record takes the defect's class, run class and slot.
bool hop_job(ec_state* st, int32_t idx, DevDefect& nd, HopJob& job) {
  const DevDefect& od = st->hdefs[idx];
  const int n = st->n;
  bool hop = od.kind == nd.kind && od.R2q == nd.R2q && od.eq == nd.eq && od.mm == nd.mm;
  for (int k = 0; k < 3 && hop; ++k) hop = od.m[k] == nd.m[k] && ((nd.cq[k] - od.cq[k]) % QSUB) == 0;
  for (int a = 0; a < 6 && hop; ++a) hop = od.efix[a] == nd.efix[a];
  if (!hop) return false;
  int sh[3];
  for (int k = 0; k < 3; ++k) {
    int d = ((nd.cq[k] - od.cq[k]) / QSUB) % n;
    if (d < 0) d += n;
    if (d >= n / 2) d -= n;
    sh[k] = d;
  }
  nd.cls = od.cls;
  nd.s = od.s;
  nd.rcls = od.rcls;
  nd.slot = od.slot;
  std::memset(&job, 0, sizeof job);
  const DefBuf& b = st->db[st->cur];
  job.spec = st->spec;
  job.sig = st->sig;
  job.own = st->own;
  job.ids = b.ids;
  job.lnk = b.lnk;
  job.cnt = b.cnt;
  job.tab = b.tab;
  job.B = st->B;
  job.S6 = st->S6;
  job.E = st->E;
  job.slot = od.slot;
  job.idx = idx;
  job.ndef = st->ndef;
  job.sx = sh[0];
  job.sy = sh[1];
  job.sz = sh[2];
  cyclic_cover(od.lo[1], od.w[1], nd.lo[1], nd.w[1], n, job.ylo, job.ylen);
  cyclic_cover(od.lo[2], od.w[2], nd.lo[2], nd.w[2], n, job.zlo, job.zlen);
  job.xitems = job.zlen * ((job.ylen + x_rows(n) - 1) / x_rows(n));
  job.h3c = st->h3c;
  for (int a = 0; a < 6; ++a) job.E12[a] = job.E12[6 + a] = od.efd[a];
  job.rec = nd;
  return true;
}

ec_status batch_entry(ec_ctx* c, const BatchKey& key, const ec_state* st0, BatchEntry** out) {
  {
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->batches.find(key);
    if (it != c->batches.end()) {
      *out = &it->second;
      return EC_OK;
    }
  }
  BatchEntry e;
  auto undo = [&]() {
    if (e.pin) (void)hipHostFree(e.pin);
    if (e.done) (void)hipEventDestroy(e.done);
    raw_free(c, e.dev);
    raw_free(c, e.ctr);
    raw_free(c, e.zero6);
    raw_free(c, e.frm);
  };
  if (hipHostMalloc((void**)&e.pin, MAXBATCH * sizeof(HopJob), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&e.done, hipEventDisableTiming) != hipSuccess) {
    undo();
    return fail(EC_ERR_DEVICE, "batch staging allocation failed");
  }
  e.dev = (HopJob*)raw_alloc(c, MAXBATCH * sizeof(HopJob));
  e.ctr = (uint32_t*)raw_alloc(c, NTILECTR * sizeof(uint32_t));
  e.zero6 = (double*)raw_alloc(c, 64);
  if (st0->frm) e.frm = (double*)raw_alloc(c, FRAME_LEN * sizeof(double));
  if (!e.dev || !e.ctr || !e.zero6 || (st0->frm && !e.frm)) {
    undo();
    return fail(EC_ERR_DEVICE, "batch buffer allocation failed");
  }
  hipError_t r = hipMemset(e.zero6, 0, 64);
  if (r == hipSuccess && e.frm)
    r = hipMemcpy(e.frm, st0->frmh.data(), FRAME_LEN * sizeof(double), hipMemcpyHostToDevice);
  if (r != hipSuccess) {
    undo();
    return fail(EC_ERR_DEVICE, "batch buffer set-up: %s", hipGetErrorString(r));
  }
  bool dup = false;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    auto ins = c->batches.emplace(key, e);
    dup = !ins.second;  // another thread made the same entry meanwhile
    *out = &ins.first->second;
  }
  if (dup) undo();  // outside the lock (the caller's free may re-enter the library)
  return EC_OK;
}

// The launches of one batch: the job table to the device, the Fourier passes,
// the lists and records, the energies.
ec_status batch_launches(const ec_state* st0, BatchEntry& e, int k, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(e.dev, e.pin, (size_t)k * sizeof(HopJob), hipMemcpyHostToDevice, s));
  Cubic C = st0->C;
  C.frm = e.frm;
  HIPCHK(launch_hop_batch_fft(st0->fp64, e.dev, k, st0->g, C, st0->tw, e.ctr, e.zero6, s));
  HIPCHK(launch_hop_batch_lists(e.dev, k, st0->n, s));
  HIPCHK(launch_hop_batch_energies(e.dev, k, s));
  return EC_OK;
}

}  // namespace

// =============================================================================== ABI

extern "C" {

const char* ec_last_error(void) { return g_err.c_str(); }

ec_status ec_ctx_create(int device, size_t budget, ec_alloc_fn af, ec_free_fn ff, void* user, ec_ctx** out) {
  if (!out) return fail(EC_ERR_ARG, "out is NULL");
  if ((af == nullptr) != (ff == nullptr)) return fail(EC_ERR_ARG, "give both allocator hooks or neither");
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(EC_ERR_ARG, "device %d not present (%d devices)", device, ndev);
  HIPCHK(hipSetDevice(device));
  size_t fr = 0, tot = 0;
  HIPCHK(hipMemGetInfo(&fr, &tot));
  void* scr = nullptr;
  HIPCHK(noalloc_scratch(device, &scr));
  ec_ctx* c = new ec_ctx;
  c->device = device;
  c->scratch = scr;
  c->budget = budget ? budget : fr;
  c->af = af;
  c->ff = ff;
  c->user = user;
  const unsigned hw = std::thread::hardware_concurrency();
  c->pool.reset(new WorkPool(hw > 2 ? (int)std::min(8u, hw - 1) : 0));
  *out = c;
  return EC_OK;
}

void ec_ctx_destroy(ec_ctx* c) {
  if (!c) return;
  for (auto& kv : c->tw) raw_free(c, kv.second);
  c->wins.clear();  // windows no state holds any more are freed here
  for (auto& kv : c->batches) {
    BatchEntry& b = kv.second;
    if (b.pending) (void)hipEventSynchronize(b.done);
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.done) (void)hipEventDestroy(b.done);
    if (b.pin) (void)hipHostFree(b.pin);
    raw_free(c, b.dev);
    raw_free(c, b.ctr);
    raw_free(c, b.zero6);
    raw_free(c, b.frm);
  }
  delete c;
}

ec_status ec_ctx_graphs(const ec_ctx* c, int32_t* count) {
  if (!c || !count) return fail(EC_ERR_ARG, "NULL argument");
  ec_ctx* m = const_cast<ec_ctx*>(c);
  std::lock_guard<std::mutex> lk(m->mu);
  int32_t k = 0;
  for (const auto& kv : c->batches) k += kv.second.exec != nullptr;
  *count = k;
  return EC_OK;
}

ec_status ec_ctx_ledger(const ec_ctx* c, size_t* used, size_t* budget) {
  if (!c) return fail(EC_ERR_ARG, "ctx is NULL");
  ec_ctx* m = const_cast<ec_ctx*>(c);
  std::lock_guard<std::mutex> lk(m->mu);
  if (used) *used = c->used;
  if (budget) *budget = c->budget;
  return EC_OK;
}

ec_status ec_state_create(ec_ctx* c, const ec_problem* p, ec_state** out) {
  if (!c || !p || !out) return fail(EC_ERR_ARG, "NULL argument");
  if (!fft_supported(p->n)) return fail(EC_ERR_SIZE, "grid size n = %d is not supported", p->n);
  if (!(p->L > 0.0) || !std::isfinite(p->L)) return fail(EC_ERR_ARG, "cell side must be positive");
  if (p->prec != EC_FP64 && p->prec != EC_FP32) return fail(EC_ERR_ARG, "unknown precision");
  if (p->bc != EC_MEAN_STRESS_ZERO && p->bc != EC_MEAN_STRAIN_ZERO) return fail(EC_ERR_ARG, "unknown mean condition");
  if (p->nyq != EC_NYQ_PAPER) return fail(EC_ERR_ARG, "unknown Nyquist rule");
  if (!(p->C11 - p->C12 > 0.0) || !(p->C11 + 2.0 * p->C12 > 0.0) || !(p->C44 > 0.0))
    return fail(EC_ERR_ARG, "stiffness is not positive definite");
  std::array<double, FRAME_LEN> fr{};
  bool rotated = false;
  for (int k = 0; k < 9; ++k) {
    if (!std::isfinite(p->frame[k])) return fail(EC_ERR_ARG, "frame is not finite");
    rotated |= p->frame[k] != (k % 4 == 0 ? 1.0 : 0.0);
  }
  bool zero = true;
  for (int k = 0; k < 9; ++k) zero &= p->frame[k] == 0.0;
  if (zero) rotated = false;
  if (rotated) {
    const double* A = p->frame;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double d = A[3 * i] * A[3 * j] + A[3 * i + 1] * A[3 * j + 1] + A[3 * i + 2] * A[3 * j + 2];
        if (std::fabs(d - (i == j ? 1.0 : 0.0)) > 1e-9) return fail(EC_ERR_ARG, "frame rows are not orthonormal");
      }
    const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                       A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(det > 0.0)) return fail(EC_ERR_ARG, "frame is not a rotation (determinant %g)", det);
    frame_maps(A, fr.data());
  }
  ec_state* st = new ec_state;
  if (rotated) {
    std::copy(p->frame, p->frame + 9, st->frame.begin());
    st->frmh = fr;
  }
  st->ctx = c;
  st->prob = *p;
  st->n = p->n;
  st->n3 = (int64_t)p->n * p->n * p->n;
  st->fp64 = p->prec == EC_FP64;
  st->g.n = p->n;
  st->g.P = spec_pitch(p->n, st->fp64);
  st->C = Cubic{p->C11, p->C12, p->C44, nullptr};
  const double h = p->L / p->n;
  st->h3c = h * h * h * GPA_NM3_EV;
  st->spec_bytes = (size_t)6 * p->n * p->n * st->g.P * (st->fp64 ? 16 : 8);
  const size_t fb = (size_t)6 * st->n3 * 8;
  st->tw = ctx_twiddles(c, p->n);
  if (!st->tw) {
    delete st;
    return fail(EC_ERR_DEVICE, "twiddle table allocation failed");
  }
  void *sp = nullptr, *own = nullptr, *sg = nullptr, *ad = nullptr, *dirs = nullptr, *ue = nullptr, *ri = nullptr;
  void* tc = nullptr;
  void* fm = nullptr;
  const size_t ob = (size_t)st->n3 * 4;
  ec_status r;
  auto undo = [&]() {
    ledger_free(c, sp, st->spec_bytes);
    ledger_free(c, own, ob);
    ledger_free(c, sg, fb);
    ledger_free(c, ad, 256);
    ledger_free(c, dirs, MAXCLS * 48);
    ledger_free(c, ue, 128);
    ledger_free(c, ri, MAXRUN * sizeof(int4));
    ledger_free(c, tc, 128);
    ledger_free(c, fm, FRAME_LEN * 8);
  };
  if ((r = ledger_alloc(c, st->spec_bytes, &sp)) != EC_OK || (r = ledger_alloc(c, ob, &own)) != EC_OK ||
      (r = ledger_alloc(c, fb, &sg)) != EC_OK || (r = ledger_alloc(c, 256, &ad)) != EC_OK ||
      (r = ledger_alloc(c, MAXCLS * 48, &dirs)) != EC_OK || (r = ledger_alloc(c, 128, &ue)) != EC_OK ||
      (r = ledger_alloc(c, 128, &tc)) != EC_OK || (r = ledger_alloc(c, MAXRUN * sizeof(int4), &ri)) != EC_OK ||
      (rotated && (r = ledger_alloc(c, FRAME_LEN * 8, &fm)) != EC_OK)) {
    undo();
    delete st;
    return r;
  }
  st->spec = sp;
  st->own = (int32_t*)own;
  st->sig = (double*)sg;
  st->add6 = (double*)ad;
  st->dirs = (double*)dirs;
  st->updE = (double*)ue;
  st->runinfo = (int4*)ri;
  st->tilectr = (uint32_t*)tc;
  st->frm = (double*)fm;
  st->C.frm = st->frm;
  st->held = st->spec_bytes + fb + ob + 256 + MAXCLS * 48 + 128 + 128 + MAXRUN * sizeof(int4) +
             (rotated ? FRAME_LEN * 8 : 0);
  hipError_t e = launch_fill_i32(st->own, st->n3, -1, nullptr);
  if (e == hipSuccess) e = hipMemset(st->sig, 0, fb);
  if (e == hipSuccess) e = hipMemset(st->add6, 0, 256);
  if (e == hipSuccess && rotated) e = hipMemcpy(st->frm, fr.data(), FRAME_LEN * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    undo();
    delete st;
    return fail(EC_ERR_DEVICE, "state initialisation: %s", hipGetErrorString(e));
  }
  *out = st;
  return EC_OK;
}

void ec_state_destroy(ec_state* st) {
  if (!st) return;
  ec_ctx* c = st->ctx;
  (void)hipDeviceSynchronize();
  const size_t fb = (size_t)6 * st->n3 * 8;
  ledger_free(c, st->spec, st->spec_bytes);
  ledger_free(c, st->own, (size_t)st->n3 * 4);
  ledger_free(c, st->sig, fb);
  ledger_free(c, st->add6, 256);
  ledger_free(c, st->dirs, MAXCLS * 48);
  ledger_free(c, st->updE, 128);
  ledger_free(c, st->tilectr, 128);
  for (auto& b : st->db) {
    ledger_free(c, b.tab, b.cap * sizeof(DevDefect));
    ledger_free(c, b.cnt, b.cap * 4);
    ledger_free(c, b.ids, b.ids_cap * 4);
    ledger_free(c, b.lnk, b.ids_cap * 8);
  }
  ledger_free(c, st->B, st->pd_cap * 8);
  ledger_free(c, st->E, st->pd_cap * 8);
  ledger_free(c, st->S6, st->pd_cap * 48);
  ledger_free(c, st->runsum, st->pd_cap * 8);
  ledger_free(c, st->gcls, st->gcls_bytes);
  ledger_free(c, st->gff, st->gff_bytes);
  ledger_free(c, st->runinfo, MAXRUN * sizeof(int4));
  ledger_free(c, st->upd_ids, st->upd_cap * 4);
  ledger_free(c, st->work, st->work_cap * sizeof(SelfWork));
  ledger_free(c, st->partial, st->partial_cap * 8);
  ledger_free(c, st->wbeg, st->wbeg_cap * 8);
  ledger_free(c, st->jjumps, st->jjumps_cap * 4);
  ledger_free(c, st->jdE, st->jdE_cap * 8);
  ledger_free(c, st->jt1, st->jt1_cap * 8);
  ledger_free(c, st->frm, st->frm ? FRAME_LEN * 8 : 0);
  ledger_free(c, st->jxc, st->jxc_cap * 8);
  ledger_free(c, st->bg, st->bg_cap * 8);
  ledger_free(c, st->bgspec, st->bgspec_cap * 16);
  ledger_free(c, st->dlines, st->dlines_cap * sizeof(DevLine));
  ledger_free(c, st->bg3, st->bg3_cap * 8);
  ledger_free(c, st->jpartial, st->jpartial_cap * 8);
  ledger_free(c, st->jsel, st->jsel_cap * 8);
  ledger_free(c, st->jnu, st->jnu_cap * 8);
  ledger_free(c, st->jwork, st->jwork_cap * sizeof(SelfWork));
  for (const auto& t : st->types) {
    ledger_free(c, t.eps, st->spec_bytes);
    ledger_free(c, t.sig, st->spec_bytes);
  }
  ledger_free(c, st->tbuf, st->tbuf_cap * 8);
  ledger_free(c, st->jwbeg, st->jwbeg_cap * 8);
  ledger_free(c, st->jchoice, st->jchoice_cap * 4);
  ledger_free(c, st->dip, st->dip_cap * 8);
  pin_free(st->pin_jump);
  pin_free(st->pin_choice);
  pin_free(st->pin_out);
  pin_free(st->pin_tab);
  pin_free(st->pin_upd);
  pin_free(st->pin_ids);
  pin_free(st->pin_tags);
  ledger_free(c, st->tags, st->tags_cap * sizeof(ClassTag));
  if (st->ev_fill) (void)hipEventDestroy(st->ev_fill);
  if (st->ev_self) (void)hipEventDestroy(st->ev_self);
  if (st->side) (void)hipStreamDestroy(st->side);
  for (auto& r : st->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : st->evpool) (void)hipEventDestroy(e);
  delete st;
}

ec_status ec_state_bytes(const ec_state* st, size_t* bytes) {
  if (!st || !bytes) return fail(EC_ERR_ARG, "NULL argument");
  *bytes = st->held;
  return EC_OK;
}

ec_status ec_solve_fields(ec_state* st, const ec_defect* defs, int32_t ndef, void* stream, void* eps_out,
                          void* sig_out, int32_t on_device) {
  if (!st) return fail(EC_ERR_ARG, "state is NULL");
  if (ndef < 0 || (ndef > 0 && !defs)) return fail(EC_ERR_ARG, "bad defect array");
  hipStream_t s = (hipStream_t)stream;
  // validate and quantise everything before touching the state, straight into
  // the pinned staging buffer of the device table
  ec_status r;
  char* hp = nullptr;
  if ((r = pin_begin(st->pin_tab, std::max<size_t>(ndef, 1) * sizeof(DevDefect), &hp)) != EC_OK) return r;
  DevDefect* h = (DevDefect*)hp;
  {
    // chunks of 64 defects on the context's workers; the first invalid
    // defect in list order is reported
    const int nch = (ndef + 63) / 64;
    std::vector<int> bad(nch, INT_MAX);
    std::vector<std::string> why(nch);
    st->ctx->pool->run(nch, [&](int c) {
      std::string e;
      for (int i = c * 64; i < std::min(ndef, (c + 1) * 64); ++i)
        if (!quantise(st->prob, defs[i], h[i], e)) {
          bad[c] = i;
          why[c] = e;
          return;
        }
    });
    for (int c = 0; c < nch; ++c)
      if (bad[c] != INT_MAX) return fail(EC_ERR_ARG, "defect %d: %s", bad[c], why[c].c_str());
  }
  if ((r = solve_table(st, h, ndef, s)) != EC_OK) return r;
  if (eps_out && (r = write_field(st, 1, eps_out, on_device != 0, s)) != EC_OK) return r;
  if (sig_out && (r = write_field(st, 0, sig_out, on_device != 0, s)) != EC_OK) return r;
  return EC_OK;
}

ec_status ec_interaction_energies(ec_state* st, void* stream, double* E_out, int32_t on_device) {
  if (!st) return fail(EC_ERR_ARG, "state is NULL");
  if (!st->solved) return fail(EC_ERR_STATE, "no solve on this state yet");
  hipStream_t s = (hipStream_t)stream;
  ec_status r;
  if (!st->B_valid && (r = compute_self_terms(st, s)) != EC_OK) return r;
  if ((r = join_self(st, s)) != EC_OK) return r;
  const DefBuf& b = st->db[st->cur];
  LAUNCH(st, s, PF_REDUCE, 0,
         launch_reduce(b.tab, st->ndef, b.cnt, b.ids, st->sig, st->B, st->h3c, st->S6, st->E, s));
  if (E_out && st->ndef > 0) return copy_small(st, E_out, st->E, (size_t)st->ndef * 8, on_device != 0, s);
  return EC_OK;
}

ec_status ec_interaction_energies_noalloc(ec_state* st, void* stream, double* E_dev) {
  if (!st || !E_dev) return fail(EC_ERR_ARG, "NULL argument");
  if (!st->solved) return fail(EC_ERR_STATE, "no solve on this state yet");
  if (st->ndef > NA_MAX_DEFECTS)
    return fail(EC_ERR_SIZE, "%d defects: the no-allocation energies take at most %lld", st->ndef,
                (long long)NA_MAX_DEFECTS);
  if (!st->ctx->scratch) return fail(EC_ERR_DEVICE, "no scratch area on this device");
  hipStream_t s = (hipStream_t)stream;
  ec_status r;
  if ((r = join_self(st, s)) != EC_OK) return r;
  const DefBuf& b = st->db[st->cur];
  if (!st->B_valid && st->ndef > 0) {
    // the self terms again (a footprint changed shape): the kernel and class
    // windows must already cover the list, since building them allocates
    const WinCache* w = st->win.get();
    if (!st->classes_ok || !w || window_need(st) > w->D || st->gcls_D != w->D ||
        st->gcls_ncls != (int)st->classes.size() || st->gff_nrun != (int)st->runcls.size())
      return fail(EC_ERR_STATE,
                  "the self terms need new kernel or class windows (a footprint outgrew the window or a new "
                  "eigenstrain direction appeared): call ec_interaction_energies once");
    // run tables on a new window need are rebuilt in place when they fit the
    // state's buffer (their run classes are already on the device)
    const int Drun = std::min(w->D, window_need(st));
    if (st->gff_D != Drun) {
      const size_t Wr = 2 * (size_t)Drun + 1;
      if (std::max<size_t>(1, st->runcls.size()) * Wr * Wr * Wr * sizeof(double) > st->gff_bytes)
        return fail(EC_ERR_STATE,
                    "the self-term run tables must grow (a footprint grew): call ec_interaction_energies once");
      LAUNCH(st, s, PF_OTHER, 0,
             launch_run_tables(st->gcls, w->D, Drun, st->runinfo, (int)st->runcls.size(), st->gff, s));
      st->gff_D = Drun;
    }
    const int64_t cap = self_work_cap(st);
    if (cap > NA_MAX_ITEMS)
      return fail(EC_ERR_SIZE, "the self terms need %lld work items: the no-allocation energies take at most %lld",
                  (long long)cap, (long long)NA_MAX_ITEMS);
    char* base = (char*)st->ctx->scratch;
    LAUNCH(st, s, PF_SELF, 0,
           launch_self_terms(b.tab, st->ndef, b.cnt, b.ids, st->n, w->K, st->gcls, w->D, run_tables(st),
                             (SelfWork*)(base + NA_WORK_OFF), cap, (int64_t*)(base + NA_WBEG_OFF),
                             (double*)(base + NA_PART_OFF), (double*)(base + NA_RUN_OFF), st->h3c, st->B, s));
    st->B_valid = true;
  }
  LAUNCH(st, s, PF_REDUCE, 0,
         launch_reduce(b.tab, st->ndef, b.cnt, b.ids, st->sig, st->B, st->h3c, st->S6, st->E, s));
  if (st->ndef > 0)
    HIPCHK(hipMemcpyAsync(E_dev, st->E, (size_t)st->ndef * 8, hipMemcpyDeviceToDevice, s));
  return EC_OK;
}

ec_status ec_update_defect(ec_state* st, int32_t idx, const ec_defect* moved, void* stream, double* E_out,
                           int32_t on_device) {
  if (!st || !moved) return fail(EC_ERR_ARG, "NULL argument");
  if (!st->solved) return fail(EC_ERR_STATE, "no solve on this state yet");
  if (idx < 0 || idx >= st->ndef) return fail(EC_ERR_ARG, "defect index %d out of range", idx);
  hipStream_t s = (hipStream_t)stream;
  DevDefect nd;
  std::string err;
  if (!quantise(st->prob, *moved, nd, err)) return fail(EC_ERR_ARG, "moved defect: %s", err.c_str());
  ec_status r0 = update_q(st, idx, nd, s);
  if (r0 != EC_OK) return r0;
  if (E_out) return ec_interaction_energies(st, stream, E_out, on_device);
  return EC_OK;
}

ec_status ec_update_batch(ec_state* const* states, const int32_t* idx, const ec_defect* moved, int32_t k,
                          void* stream, double* const* E_dev, int32_t use_graph) {
  if (!states || !idx || !moved) return fail(EC_ERR_ARG, "NULL argument");
  if (k < 1 || k > MAXBATCH) return fail(EC_ERR_ARG, "batch size %d outside [1, %d]", k, MAXBATCH);
  hipStream_t s = (hipStream_t)stream;
  const ec_state* st0 = states[0];
  if (!st0) return fail(EC_ERR_ARG, "NULL state");
  // validate every hop before touching any state
  HopJob jobs[MAXBATCH];
  DevDefect recs[MAXBATCH];
  for (int j = 0; j < k; ++j) {
    ec_state* st = states[j];
    if (!st) return fail(EC_ERR_ARG, "NULL state %d", j);
    for (int i = 0; i < j; ++i)
      if (states[i] == st) return fail(EC_ERR_ARG, "state %d appears twice in the batch", j);
    if (st->ctx != st0->ctx || st->n != st0->n || st->fp64 != st0->fp64 || st->C.C11 != st0->C.C11 ||
        st->C.C12 != st0->C.C12 || st->C.C44 != st0->C.C44 || st->frame != st0->frame)
      return fail(EC_ERR_ARG, "state %d does not have the shape of state 0", j);
    if (!st->solved) return fail(EC_ERR_STATE, "state %d has no solve yet", j);
    if (idx[j] < 0 || idx[j] >= st->ndef) return fail(EC_ERR_ARG, "defect index %d of state %d out of range", idx[j], j);
    std::string err;
    if (!quantise(st->prob, moved[j], recs[j], err)) return fail(EC_ERR_ARG, "moved defect %d: %s", j, err.c_str());
    if (!hop_job(st, idx[j], recs[j], jobs[j]))
      return fail(EC_ERR_ARG, "move %d is not a whole-voxel hop of the same defect (use ec_update_defect)", j);
    jobs[j].Eout = E_dev ? E_dev[j] : nullptr;
  }
  // self terms of every state current and joined on this stream
  ec_status r;
  for (int j = 0; j < k; ++j) {
    ec_state* st = states[j];
    if ((r = join_self(st, s)) != EC_OK) return r;
    if (!st->B_valid && (r = compute_self_terms(st, s)) != EC_OK) return r;
    if ((r = ensure_sigma(st, s)) != EC_OK) return r;  // the hops add to the whole field
  }
  BatchKey key{st0->n, st0->fp64 ? 0 : 1, k, st0->C.C11, st0->C.C12, st0->C.C44, st0->frame, stream};
  BatchEntry* e = nullptr;
  if ((r = batch_entry(st0->ctx, key, st0, &e)) != EC_OK) return r;
  if (e->pending) HIPCHK(hipEventSynchronize(e->done));  // the previous batch read the table
  e->pending = false;
  std::memcpy(e->pin, jobs, (size_t)k * sizeof(HopJob));
  if (!s) use_graph = 0;  // the null stream cannot be captured: direct launches
  if (use_graph && !e->exec && !e->graph_failed) {
    // capture the launch sequence once; it reads the pinned table at replay
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const ec_status rc = batch_launches(st0, *e, k, s);
    const hipError_t ec2 = hipStreamEndCapture(s, &g);
    if (rc != EC_OK || ec2 != hipSuccess || hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      e->exec = nullptr;
      e->graph_failed = true;  // direct launches from now on
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
  }
  if (use_graph && e->exec) {
    HIPCHK(hipGraphLaunch(e->exec, s));
  } else if ((r = batch_launches(st0, *e, k, s)) != EC_OK) {
    return r;
  }
  HIPCHK(hipEventRecord(e->done, s));
  e->pending = true;
  for (int j = 0; j < k; ++j) {
    ec_state* st = states[j];
    st->hdefs[idx[j]] = recs[j];
    st->jdE_ok = false;
  }
  return EC_OK;
}

ec_status ec_state_footprints(ec_state* st, int32_t* counts, int32_t* ids, int64_t cap, int64_t* total) {
  if (!st) return fail(EC_ERR_ARG, "state is NULL");
  ec_status r = fetch_counts(st);
  if (r != EC_OK) return r;
  int64_t tot = 0;
  for (int i = 0; i < st->ndef; ++i) tot += st->hcnt[i];
  if (total) *total = tot;
  if (counts)
    for (int i = 0; i < st->ndef; ++i) counts[i] = st->hcnt[i];
  if (!ids) return EC_OK;
  if (cap < tot) return fail(EC_ERR_ARG, "ids buffer too small (%lld < %lld)", (long long)cap, (long long)tot);
  const DefBuf& b = st->db[st->cur];
  std::vector<int32_t> all((size_t)std::max<int64_t>(st->ids_used, 1));
  if (st->ids_used > 0) HIPCHK(hipMemcpy(all.data(), b.ids, st->ids_used * 4, hipMemcpyDeviceToHost));
  int64_t o = 0;
  for (int i = 0; i < st->ndef; ++i) {
    std::memcpy(ids + o, all.data() + st->hdefs[i].slot, st->hcnt[i] * 4);
    o += st->hcnt[i];
  }
  return EC_OK;
}

ec_status ec_state_field(ec_state* st, int32_t which, double* out) {
  if (!st || !out) return fail(EC_ERR_ARG, "NULL argument");
  // the state's earlier work may still run on another stream (which the null
  // stream need not wait for): it ends before the whole stress is formed
  HIPCHK(hipDeviceSynchronize());
  {
    const ec_status r0 = ensure_sigma(st, nullptr);
    if (r0 != EC_OK) return r0;
  }
  HIPCHK(hipDeviceSynchronize());
  const size_t cnt = (size_t)6 * st->n3;
  if (which >= 0 && which <= 2) {
    // component-major copy of the voxel-major stress, or the strain or
    // eigenstrain derived from it, through a device temporary
    void* tmp = nullptr;
    ec_status r = ledger_alloc(st->ctx, cnt * 8, &tmp);
    if (r != EC_OK) return r;
    const DefBuf& b = st->db[st->cur];
    hipError_t e = launch_sig_to_out(st->sig, st->own, b.lnk, b.tab, st->ndef, st->n3, st->C, which, false, tmp, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, tmp, cnt * 8, hipMemcpyDeviceToHost);
    ledger_free(st->ctx, tmp, cnt * 8);
    if (e != hipSuccess) return fail(EC_ERR_DEVICE, "field output %d: %s", which, hipGetErrorString(e));
  } else {
    return fail(EC_ERR_ARG, "unknown field %d", which);
  }
  return EC_OK;
}

ec_status ec_state_self_terms(ec_state* st, double* out) {
  if (!st || !out) return fail(EC_ERR_ARG, "NULL argument");
  if (!st->solved) return fail(EC_ERR_STATE, "no solve on this state yet");
  ec_status r;
  HIPCHK(hipDeviceSynchronize());  // earlier work of the state on other streams
  if (!st->B_valid && (r = compute_self_terms(st, nullptr)) != EC_OK) return r;
  HIPCHK(hipDeviceSynchronize());
  if (st->ndef > 0) HIPCHK(hipMemcpy(out, st->B, st->ndef * 8, hipMemcpyDeviceToHost));
  return EC_OK;
}

ec_status ec_profile_enable(ec_state* st, int32_t on) {
  if (!st) return fail(EC_ERR_ARG, "state is NULL");
  st->prof = on != 0;
  return EC_OK;
}

ec_status ec_profile_select(ec_state* st, int32_t family_mask) {
  if (!st) return fail(EC_ERR_ARG, "state is NULL");
  if (family_mask & ~((1 << EC_NPROF) - 1)) return fail(EC_ERR_ARG, "family mask 0x%x names no family", family_mask);
  st->prof_mask = family_mask;
  return EC_OK;
}

ec_status ec_profile_read(ec_state* st, int64_t* launches, double* ms, double* bytes) {
  if (!st) return fail(EC_ERR_ARG, "state is NULL");
  HIPCHK(hipDeviceSynchronize());
  double tms[EC_NPROF] = {0}, tb[EC_NPROF] = {0};
  int64_t cnt[EC_NPROF] = {0};
  for (auto& r : st->recs) {
    float m = 0.f;
    HIPCHK(hipEventElapsedTime(&m, r.a, r.b));
    tms[r.fam] += m;
    tb[r.fam] += r.bytes;
    cnt[r.fam] += 1;
    st->evpool.push_back(r.a);
    st->evpool.push_back(r.b);
  }
  st->recs.clear();
  for (int f = 0; f < EC_NPROF; ++f) {
    if (launches) launches[f] = cnt[f];
    if (ms) ms[f] = tms[f];
    if (bytes) bytes[f] = cnt[f] ? tb[f] / cnt[f] : 0.0;
  }
  return EC_OK;
}

// ---------------------------------------------------------------- jump probes

constexpr int JUMP_MAX = 8;  // largest jump component, in voxels
constexpr int OKMC_FEW = 1;  // acting defects up to which a step moves them one by one

ec_status ec_jump_energies(ec_state* st, const int32_t* jumps, int32_t njump, void* stream, double* dE_out,
                           int32_t on_device) {
  if (!st) return fail(EC_ERR_ARG, "state is NULL");
  if (!st->solved) return fail(EC_ERR_STATE, "no solve on this state yet");
  if (njump < 1 || njump > 64) return fail(EC_ERR_ARG, "njump %d outside [1, 64]", njump);
  const int nd = st->ndef;
  const size_t nu = (size_t)nd * njump;
  if (nd > 0 && !jumps) return fail(EC_ERR_ARG, "jumps is NULL");
  int reach = 0;
  for (size_t k = 0; k < 3 * nu; ++k) {
    const int v = std::abs(jumps[k]);
    if (v > JUMP_MAX || 2 * v >= st->n)
      return fail(EC_ERR_ARG, "jump %zu of defect %zu: component %d beyond %d voxels or half the cell", (k / 3) % njump,
                  k / 3 / njump, jumps[k], JUMP_MAX);
    reach = std::max(reach, v);
  }
  hipStream_t s = (hipStream_t)stream;
  st->jdE_ok = false;
  if (nd == 0) {
    st->jn = njump;
    st->jdE_ok = true;
    return EC_OK;
  }
  ec_status r;
  if ((r = join_self(st, s)) != EC_OK) return r;
  if ((r = ensure_sigma(st, s)) != EC_OK) return r;  // the jumped footprints leave the covered voxels
  if ((r = ensure_classes(st, s)) != EC_OK) return r;
  if ((r = ensure_windows(st, reach, s)) != EC_OK) return r;
  if (!st->B_valid && (r = compute_self_terms(st, s)) != EC_OK) return r;
  // work items: per (defect, jump) all ordered pairs of the footprint
  int64_t cap = 0;
  for (const auto& d : st->hdefs) {
    const double m = (double)box_volume(d);
    cap += (int64_t)njump * (int64_t)std::min(64.0, std::max(1.0, std::ceil(m * m / 32768.0)));
  }
  if (st->jxc_cap < nu) st->jx_ok = false;
  if ((r = st_grow(st, &st->jjumps, &st->jjumps_cap, 3 * nu)) != EC_OK ||
      (r = st_grow(st, &st->jxc, &st->jxc_cap, nu)) != EC_OK ||
      (r = st_grow(st, &st->jdE, &st->jdE_cap, nu, st->jdE_ok, s)) != EC_OK ||  // the last energies stay if this fails
      (r = st_grow(st, &st->jt1, &st->jt1_cap, nu)) != EC_OK ||
      (r = st_grow(st, &st->jwbeg, &st->jwbeg_cap, nu + 1)) != EC_OK ||
      (r = st_grow(st, &st->jwork, &st->jwork_cap, (size_t)cap)) != EC_OK ||
      (r = st_grow(st, &st->jpartial, &st->jpartial_cap, (size_t)cap)) != EC_OK)
    return r;
  char* hp = nullptr;
  if ((r = pin_begin(st->pin_jump, 3 * nu * 4, &hp)) != EC_OK) return r;
  std::memcpy(hp, jumps, 3 * nu * 4);
  HIPCHK(hipMemcpyAsync(st->jjumps, hp, 3 * nu * 4, hipMemcpyHostToDevice, s));
  if ((r = pin_end(st->pin_jump, s)) != EC_OK) return r;
  const DefBuf& b = st->db[st->cur];
  const bool xc_valid = st->jx_ok && st->jx_jumps.size() == 3 * nu &&
                        std::memcmp(st->jx_jumps.data(), jumps, 3 * nu * 4) == 0;
  // S(0): the footprint sums of the energies reduction (which also refreshes E)
  LAUNCH(st, s, PF_REDUCE, 0,
         launch_reduce(b.tab, nd, b.cnt, b.ids, st->sig, st->B, st->h3c, st->S6, st->E, s));
  LAUNCH(st, s, PF_SELF, 0,
         launch_jump_energies(b.tab, nd, b.cnt, b.ids, st->sig, st->n, st->jjumps, njump, st->S6, st->win->K,
                              st->gcls, st->win->D, st->jwork, (int64_t)st->jwork_cap, st->jwbeg, st->jpartial,
                              st->jt1, st->B, st->h3c, st->jxc, xc_valid, st->jdE, s));
  st->jn = njump;
  st->jdE_ok = true;
  if (!xc_valid) {
    st->jx_jumps.assign(jumps, jumps + 3 * nu);
    st->jx_ok = true;
  }
  if (dE_out) return copy_small(st, dE_out, st->jdE, nu * 8, on_device != 0, s);
  return EC_OK;
}

ec_status ec_jump_select(ec_state* st, const double* Em, double nu0, double kT, const double* xi, void* stream,
                         double* nu_out, int32_t* choice_out, int32_t on_device) {
  if (!st) return fail(EC_ERR_ARG, "state is NULL");
  if (!st->jdE_ok) return fail(EC_ERR_STATE, "no jump energies for the current defect list");
  if (!(nu0 > 0.0) || !std::isfinite(nu0) || !(kT > 0.0) || !std::isfinite(kT))
    return fail(EC_ERR_ARG, "nu0 and kT must be positive and finite");
  const int nd = st->ndef, nj = st->jn;
  if (nd == 0) return EC_OK;
  if (!Em) return fail(EC_ERR_ARG, "Em is NULL");
  if (choice_out && !xi) return fail(EC_ERR_ARG, "xi is NULL");
  for (int i = 0; i < nd; ++i) {
    if (!std::isfinite(Em[i])) return fail(EC_ERR_ARG, "Em of defect %d not finite", i);
    if (xi && !(xi[i] > 0.0 && xi[i] <= 1.0)) return fail(EC_ERR_ARG, "xi of defect %d outside (0, 1]", i);
  }
  return run_select(st, Em, nu0, kT, xi, nullptr, 0.0, (hipStream_t)stream, nu_out, choice_out, on_device != 0);
}

ec_status ec_okmc_step(ec_state* st, const int32_t* jumps, int32_t njump, const double* Em, double nu0, double kT,
                       double dt, const double* u, const double* xi, void* stream, int32_t* choice_out,
                       double* E_out) {
  if (!st) return fail(EC_ERR_ARG, "state is NULL");
  if (!st->solved) return fail(EC_ERR_STATE, "no solve on this state yet");
  if (!(nu0 > 0.0) || !std::isfinite(nu0) || !(kT > 0.0) || !std::isfinite(kT))
    return fail(EC_ERR_ARG, "nu0 and kT must be positive and finite");
  if (!std::isfinite(dt)) return fail(EC_ERR_ARG, "dt is not finite");
  const int nd = st->ndef;
  if (nd > 0 && (!Em || !u || !xi)) return fail(EC_ERR_ARG, "Em, u or xi is NULL");
  double numax = 0.0;
  for (int i = 0; i < nd; ++i) {
    if (!std::isfinite(Em[i])) return fail(EC_ERR_ARG, "Em of defect %d not finite", i);
    if (!(u[i] > 0.0 && u[i] <= 1.0)) return fail(EC_ERR_ARG, "u of defect %d outside (0, 1]", i);
    if (!(xi[i] > 0.0 && xi[i] <= 1.0)) return fail(EC_ERR_ARG, "xi of defect %d outside (0, 1]", i);
    numax = std::max(numax, nu0 * std::exp(-Em[i] / kT));
  }
  // the paper's fixed step: one event on average for the fastest defect
  if (dt <= 0.0 && nd > 0) {
    if (!(numax > 0.0) || !std::isfinite(numax)) return fail(EC_ERR_ARG, "no finite positive frequency for dt");
    dt = 1.0 / numax;
  }
  hipStream_t s = (hipStream_t)stream;
  ec_status r;
  if ((r = ec_jump_energies(st, jumps, njump, stream, nullptr, 0)) != EC_OK) return r;
  if (nd == 0) return EC_OK;
  std::vector<int32_t> ch(nd);
  const int n = st->n;
  const int32_t Lq = QSUB * n;
  // the gate needs only the nominal frequencies, so the host knows how many
  // defects act; a few are moved one by one with the incremental update (each
  // a fraction of a re-solve), all choices still taken against the field at
  // the start of the step
  int acting = 0;
  for (int i = 0; i < nd; ++i) acting += u[i] > std::exp(-nu0 * std::exp(-Em[i] / kT) * dt);
  if (acting <= OKMC_FEW) {
    if ((r = run_select(st, Em, nu0, kT, xi, u, dt, s, nullptr, ch.data(), false)) != EC_OK) return r;
    for (int i = 0; i < nd; ++i) {
      if (ch[i] < 0) continue;
      DevDefect q = st->hdefs[i];
      const int32_t* lam = jumps + ((size_t)i * njump + ch[i]) * 3;
      for (int k = 0; k < 3; ++k) {
        q.cq[k] = (int32_t)((((int64_t)q.cq[k] + (int64_t)lam[k] * QSUB) % Lq + Lq) % Lq);
        q.lo[k] = ((q.lo[k] + lam[k]) % n + n) % n;
      }
      if ((r = update_q(st, i, q, s)) != EC_OK) return r;
    }
    if (choice_out) std::memcpy(choice_out, ch.data(), (size_t)nd * 4);
    if (E_out) return ec_interaction_energies(st, stream, E_out, 0);
    return EC_OK;
  }
  if (st->B_valid && st->classes_ok) {
    // the probe left the self terms and classes current, and a translation by
    // whole voxels keeps every footprint's shape: the choices stay on the
    // device, the moved table is written there, and the host waits only at
    // the end (for its copy of the choices)
    if ((r = run_select(st, Em, nu0, kT, xi, u, dt, s, nullptr, nullptr, false, true)) != EC_OK) return r;
    char* hc = nullptr;
    if ((r = pin_begin(st->pin_choice, (size_t)nd * 4, &hc)) != EC_OK) return r;
    HIPCHK(hipMemcpyAsync(hc, st->jchoice, (size_t)nd * 4, hipMemcpyDeviceToHost, s));
    if ((r = pin_end(st->pin_choice, s)) != EC_OK) return r;
    const DevDefect* src = st->db[st->cur].tab;
    r = solve_table(st, nullptr, nd, s, true, [&](DevDefect* dst) -> ec_status {
      LAUNCH(st, s, PF_OTHER, 0, launch_apply_jumps(src, dst, nd, st->jchoice, st->jjumps, njump, n, s));
      return EC_OK;
    });
    if (r != EC_OK) return r;
    HIPCHK(hipEventSynchronize(st->pin_choice.ev));
    st->pin_choice.pending = false;
    std::memcpy(ch.data(), hc, (size_t)nd * 4);
    for (int i = 0; i < nd; ++i) {
      if (ch[i] < 0) continue;
      const int32_t* lam = jumps + ((size_t)i * njump + ch[i]) * 3;
      DevDefect& d = st->hdefs[i];
      for (int k = 0; k < 3; ++k) {
        d.cq[k] = (int32_t)((((int64_t)d.cq[k] + (int64_t)lam[k] * QSUB) % Lq + Lq) % Lq);
        d.lo[k] = ((d.lo[k] + lam[k]) % n + n) % n;
      }
    }
    if (choice_out) std::memcpy(choice_out, ch.data(), (size_t)nd * 4);
    if (E_out) return ec_interaction_energies(st, stream, E_out, 0);
    return EC_OK;
  }
  if ((r = run_select(st, Em, nu0, kT, xi, u, dt, s, nullptr, ch.data(), false)) != EC_OK) return r;
  // the chosen jumps: whole-voxel translations of the quantised centres (box,
  // offsets and eigenstrain are unchanged), then the field of the new positions
  char* hp = nullptr;
  if ((r = pin_begin(st->pin_tab, (size_t)nd * sizeof(DevDefect), &hp)) != EC_OK) return r;
  DevDefect* h = (DevDefect*)hp;
  for (int i = 0; i < nd; ++i) {
    h[i] = st->hdefs[i];
    if (ch[i] < 0) continue;
    const int32_t* lam = jumps + ((size_t)i * njump + ch[i]) * 3;
    for (int k = 0; k < 3; ++k) {
      h[i].cq[k] = (int32_t)((((int64_t)h[i].cq[k] + (int64_t)lam[k] * QSUB) % Lq + Lq) % Lq);
      h[i].lo[k] = ((h[i].lo[k] + lam[k]) % n + n) % n;
    }
  }
  if ((r = solve_table(st, h, nd, s)) != EC_OK) return r;
  if (choice_out) std::memcpy(choice_out, ch.data(), (size_t)nd * 4);
  if (E_out) return ec_interaction_energies(st, stream, E_out, 0);
  return EC_OK;
}

// ---------------------------------------------------------------- dipole energies

ec_status ec_set_dislocations(ec_state* st, const ec_line* lines, int32_t nlines, void* stream) {
  if (!st) return fail(EC_ERR_ARG, "state is NULL");
  if (nlines < 0 || nlines > 64) return fail(EC_ERR_ARG, "nlines %d outside [0, 64]", nlines);
  if (nlines > 0 && !lines) return fail(EC_ERR_ARG, "lines is NULL");
  const int n = st->n;
  const double h = st->prob.L / n;
  std::vector<DevLine> by[3];
  for (int i = 0; i < nlines; ++i) {
    const ec_line& l = lines[i];
    bool fin = true;
    for (int k = 0; k < 3; ++k) fin &= std::isfinite(l.p[k]) && std::isfinite(l.b[k]);
    if (!fin) return fail(EC_ERR_ARG, "line %d: non-finite value", i);
    if (l.axis < 0 || l.axis > 2) return fail(EC_ERR_ARG, "line %d: axis %d not in {0, 1, 2}", i, l.axis);
    if (l.sense != 1 && l.sense != -1) return fail(EC_ERR_ARG, "line %d: sense %d not +-1", i, l.sense);
    if (!(l.b[0] * l.b[0] + l.b[1] * l.b[1] + l.b[2] * l.b[2] > 0.0))
      return fail(EC_ERR_ARG, "line %d: zero Burgers vector", i);
    const int a1 = l.axis == 0 ? 1 : 0, a2 = l.axis == 2 ? 1 : 2;
    DevLine d{};
    d.u1 = l.p[a1] / h - 0.5;
    d.u2 = l.p[a2] / h - 0.5;
    if (!(std::fabs(d.u1) < 1e9 && std::fabs(d.u2) < 1e9)) return fail(EC_ERR_ARG, "line %d: position too far", i);
    for (int k = 0; k < 3; ++k) {
      d.b[k] = l.b[k];
      d.t[k] = k == l.axis ? (double)l.sense : 0.0;
    }
    by[l.axis].push_back(d);
  }
  hipStream_t s = (hipStream_t)stream;
  ec_status r;
  // the whole field with the old lines' stress, before it is exchanged
  if ((r = ensure_sigma(st, s)) != EC_OK) return r;
  const size_t nn = (size_t)n * n;
  if ((r = st_grow(st, &st->bg, &st->bg_cap, 3 * nn * 6, true, s)) != EC_OK ||
      (r = st_grow(st, &st->bgspec, &st->bgspec_cap, 12 * nn)) != EC_OK ||
      (r = st_grow(st, &st->dlines, &st->dlines_cap, 64)) != EC_OK)
    return r;
  if ((r = join_self(st, s)) != EC_OK) return r;
  // take the old lines' stress out of the resident field, put the new one in
  if (st->solved && st->bg_mask)
    LAUNCH(st, s, PF_OTHER, 0, launch_bg_add(st->sig, st->bg, st->bg_mask, n, -1.0, s));
  int mask = 0;
  for (int a = 0; a < 3; ++a) {
    if (by[a].empty()) continue;
    HIPCHK(hipMemcpyAsync(st->dlines, by[a].data(), by[a].size() * sizeof(DevLine), hipMemcpyHostToDevice, s));
    LAUNCH(st, s, PF_OTHER, 0,
           launch_disl_plane(st->dlines, (int)by[a].size(), a, n, st->prob.L, st->C, st->bgspec,
                             st->bgspec + 6 * nn, st->bg + (size_t)a * nn * 6, s));
    HIPCHK(hipStreamSynchronize(s));  // the line table is pageable host memory reused per axis
    mask |= 1 << a;
  }
  st->bg_mask = mask;
  if (st->solved && mask) LAUNCH(st, s, PF_OTHER, 0, launch_bg_add(st->sig, st->bg, mask, n, 1.0, s));
  st->jdE_ok = false;
  return EC_OK;
}

ec_status ec_set_dislocation_paths(ec_state* st, const ec_path* paths, int32_t npaths, const double* verts,
                                   int32_t nverts, void* stream) {
  if (!st) return fail(EC_ERR_ARG, "state is NULL");
  if (npaths < 0 || npaths > 256) return fail(EC_ERR_ARG, "npaths %d outside [0, 256]", npaths);
  if (npaths > 0 && (!paths || !verts || nverts <= 0)) return fail(EC_ERR_ARG, "NULL argument");
  const int n = st->n;
  const double L = st->prob.L, h = L / n, h3 = h * h * h;
  std::vector<DevPiece> pieces;
  double Ubar[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // mean plastic distortion of the loops
  const size_t max_pieces = (size_t)1 << 20;
  for (int k = 0; k < npaths; ++k) {
    const ec_path& P = paths[k];
    if (P.count < 1 || P.first < 0 || (int64_t)P.first + P.count > nverts)
      return fail(EC_ERR_ARG, "path %d: vertices [%d, %d) outside the %d given", k, P.first, P.first + P.count, nverts);
    bool fin = true, loop = true;
    double bb = 0.0;
    for (int a = 0; a < 3; ++a) {
      fin &= std::isfinite(P.b[a]) && std::isfinite(P.shift[a]);
      bb += P.b[a] * P.b[a];
      const double m = P.shift[a] / L;
      if (!(std::fabs(m - std::nearbyint(m)) < 1e-9) || std::fabs(m) > 64.0)
        return fail(EC_ERR_ARG, "path %d: shift is not a lattice vector of the cell", k);
      loop &= P.shift[a] == 0.0 || std::nearbyint(m) == 0.0;
    }
    if (!fin) return fail(EC_ERR_ARG, "path %d: non-finite value", k);
    if (!(bb > 0.0)) return fail(EC_ERR_ARG, "path %d: zero Burgers vector", k);
    if (loop && P.count < 3) return fail(EC_ERR_ARG, "path %d: a loop needs at least three vertices", k);
    const double* v = verts + 3 * (size_t)P.first;
    for (int j = 0; j < 3 * P.count; ++j)
      if (!std::isfinite(v[j]) || std::fabs(v[j]) > 1e6 * L) return fail(EC_ERR_ARG, "path %d: vertex out of range", k);
    double A[3] = {0, 0, 0};
    for (int j = 0; j < P.count; ++j) {
      double a[3], d[3];
      for (int c = 0; c < 3; ++c) {
        a[c] = v[3 * j + c];
        const double e = j + 1 < P.count ? v[3 * (j + 1) + c] : v[c] + (loop ? 0.0 : P.shift[c]);
        d[c] = e - a[c];
      }
      if (loop) {  // vector area 1/2 sum v_j x v_{j+1}
        const double* w = j + 1 < P.count ? v + 3 * (j + 1) : v;
        A[0] += 0.5 * (a[1] * w[2] - a[2] * w[1]);
        A[1] += 0.5 * (a[2] * w[0] - a[0] * w[2]);
        A[2] += 0.5 * (a[0] * w[1] - a[1] * w[0]);
      }
      const double len = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const int m = std::max(1, (int)std::ceil(len / h - 1e-12));
      if (pieces.size() + (size_t)m > max_pieces) return fail(EC_ERR_ARG, "paths cut into more than 2^20 pieces");
      for (int q = 0; q < m; ++q) {
        DevPiece pc{};
        for (int c = 0; c < 3; ++c) {
          const double mid = a[c] + (q + 0.5) * d[c] / m;
          const double u = mid / h - 0.5;
          const double f = std::floor(u);
          pc.fr[c] = u - f;
          pc.f[c] = (int32_t)(((int64_t)f % n + n) % n);
        }
        for (int i = 0; i < 3; ++i)
          for (int l = 0; l < 3; ++l) pc.M[3 * i + l] = P.b[i] * (d[l] / m) / h3;
        pieces.push_back(pc);
      }
    }
    for (int i = 0; i < 3; ++i)
      for (int l = 0; l < 3; ++l) Ubar[3 * i + l] -= P.b[i] * A[l] / (L * L * L);
  }
  hipStream_t s = (hipStream_t)stream;
  ec_status r;
  // the whole field with the old loops' stress, before the spectrum is reused
  // for the new ones and their stress exchanged
  if ((r = ensure_sigma(st, s)) != EC_OK) return r;
  if (pieces.empty()) {  // remove the paths
    if (st->bg3_on) {
      if ((r = join_self(st, s)) != EC_OK) return r;
      if (st->solved) LAUNCH(st, s, PF_OTHER, 0, launch_bg3_add(st->sig, st->bg3, st->n3, -1.0, s));
      st->bg3_on = false;
      st->jdE_ok = false;
    }
    return EC_OK;
  }
  const size_t need = (size_t)st->n3 * 6;
  size_t cap = st->bg3_cap;
  if ((r = st_grow(st, &st->bg3, &cap, need, st->bg3_on, s)) != EC_OK) return r;
  st->bg3_cap = cap;
  Tmp tp{st->ctx}, tm{st->ctx};
  if ((r = ledger_alloc(st->ctx, tp.b = pieces.size() * sizeof(DevPiece), &tp.p)) != EC_OK) return r;
  if ((r = ledger_alloc(st->ctx, tm.b = 64, &tm.p)) != EC_OK) return r;
  // mean stress of the compatible part (zero-mean-strain condition only)
  double mean6[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (st->prob.bc == EC_MEAN_STRAIN_ZERO) {
    const double e6[6] = {Ubar[0], Ubar[4], Ubar[8], 0.5 * (Ubar[5] + Ubar[7]), 0.5 * (Ubar[2] + Ubar[6]),
                          0.5 * (Ubar[1] + Ubar[3])};
    neg_C_dot(st, e6, mean6);
  }
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpy(tp.p, pieces.data(), tp.b, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(tm.p, mean6, 64, hipMemcpyHostToDevice));
  if ((r = join_self(st, s)) != EC_OK) return r;
  // take the old paths' stress out of the resident field, put the new one in
  if (st->solved && st->bg3_on) LAUNCH(st, s, PF_OTHER, 0, launch_bg3_add(st->sig, st->bg3, st->n3, -1.0, s));
  st->bg3_on = false;
  const bool fp64 = st->fp64;
  const Prune full{0, n, 0, n};
  LAUNCH(st, s, PF_OTHER, 0,
         launch_path_spectrum(fp64, (const DevPiece*)tp.p, (int)pieces.size(), st->g, L, st->C, st->tw, st->spec, s));
  LAUNCH(st, s, PF_Z, 0, launch_pencil(fp64, true, 2, st->spec, st->g, full, st->tw, nullptr, s));
  LAUNCH(st, s, PF_Y, 0, launch_pencil(fp64, true, 1, st->spec, st->g, full, st->tw, nullptr, s));
  LAUNCH(st, s, PF_XI, 0, launch_x_inverse(fp64, false, st->spec, st->bg3, st->g, (const double*)tm.p, st->tw, s));
  st->bg3_on = true;
  if (st->solved) LAUNCH(st, s, PF_OTHER, 0, launch_bg3_add(st->sig, st->bg3, st->n3, 1.0, s));
  st->jdE_ok = false;
  HIPCHK(hipStreamSynchronize(s));  // the piece table is freed on return
  return EC_OK;
}

ec_status ec_dipole_energies(ec_state* st, void* stream, double* E_out, int32_t on_device) {
  if (!st) return fail(EC_ERR_ARG, "state is NULL");
  if (!st->solved) return fail(EC_ERR_STATE, "no solve on this state yet");
  const int nd = st->ndef;
  if (nd == 0) return EC_OK;
  hipStream_t s = (hipStream_t)stream;
  ec_status r;
  if ((r = join_self(st, s)) != EC_OK) return r;
  if ((r = ensure_sigma(st, s)) != EC_OK) return r;  // the stress at the centres
  if ((r = ensure_classes(st, s)) != EC_OK) return r;
  if ((r = ensure_windows(st, 0, s)) != EC_OK) return r;
  if ((r = st_grow(st, &st->dip, &st->dip_cap, (size_t)nd)) != EC_OK) return r;
  const DefBuf& b = st->db[st->cur];
  LAUNCH(st, s, PF_REDUCE, 0,
         launch_dipole(b.tab, nd, b.cnt, b.ids, st->sig, st->n, st->win->K, st->gcls, st->win->D, st->h3c, st->dip,
                       s));
  if (E_out) return copy_small(st, E_out, st->dip, (size_t)nd * 8, on_device != 0, s);
  return EC_OK;
}

// ---------------------------------------------------------------- debug passes

}  // extern "C"

namespace {

// Host arrays are [6][n][n][n/2+1] complex (re, im); the device spectrum is
// component-interleaved with row pitch P (spec_at).
ec_status upload_spec(ec_state* st, const double* host, void* dev) {
  const int n = st->n, nh = n / 2 + 1, P = st->g.P;
  const size_t total = (size_t)6 * n * n * P;
  std::vector<double> d(2 * total, 0.0);
  for (int c = 0; c < 6; ++c)
    for (int z = 0; z < n; ++z)
      for (int y = 0; y < n; ++y)
        for (int k = 0; k < nh; ++k) {
          const size_t h = (((size_t)c * n + z) * n + y) * nh + k;
          const size_t o = spec_at(z, y, k, c, n, P);
          d[2 * o] = host[2 * h];
          d[2 * o + 1] = host[2 * h + 1];
        }
  if (st->fp64) {
    HIPCHK(hipMemcpy(dev, d.data(), total * 16, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(2 * total);
    for (size_t i = 0; i < f.size(); ++i) f[i] = (float)d[i];
    HIPCHK(hipMemcpy(dev, f.data(), total * 8, hipMemcpyHostToDevice));
  }
  return EC_OK;
}

ec_status download_spec(ec_state* st, const void* dev, double* host) {
  const int n = st->n, nh = n / 2 + 1, P = st->g.P;
  const size_t total = (size_t)6 * n * n * P;
  std::vector<double> d(2 * total);
  if (st->fp64) {
    HIPCHK(hipMemcpy(d.data(), dev, total * 16, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> f(2 * total);
    HIPCHK(hipMemcpy(f.data(), dev, total * 8, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < f.size(); ++i) d[i] = (double)f[i];
  }
  for (int c = 0; c < 6; ++c)
    for (int z = 0; z < n; ++z)
      for (int y = 0; y < n; ++y)
        for (int k = 0; k < nh; ++k) {
          const size_t h = (((size_t)c * n + z) * n + y) * nh + k;
          const size_t o = spec_at(z, y, k, c, n, P);
          host[2 * h] = d[2 * o];
          host[2 * h + 1] = d[2 * o + 1];
        }
  return EC_OK;
}

}  // namespace

extern "C" {

ec_status ec_type_store(ec_state* st, const ec_defect* proto, void* stream, int32_t* type) {
  if (!st || !proto || !type) return fail(EC_ERR_ARG, "NULL argument");
  if (st->types.size() >= 64) return fail(EC_ERR_ARG, "at most 64 stored types per state");
  hipStream_t s = (hipStream_t)stream;
  DevDefect d;
  std::string err;
  if (!quantise(st->prob, *proto, d, err)) return fail(EC_ERR_ARG, "prototype: %s", err.c_str());
  std::vector<int32_t> ids;
  footprint_ids(d, st->n, ids);
  const int m = (int)ids.size();
  ec_ctx* c = st->ctx;
  Tmp ti{c}, te{c};
  ec_status r;
  // [ids][zero count]; E: no old eigenstrain, the prototype's (cell frame) as the new one
  if ((r = ledger_alloc(c, ti.b = (size_t)m * 4 + 64, &ti.p)) != EC_OK) return r;
  if ((r = ledger_alloc(c, te.b = 96, &te.p)) != EC_OK) return r;
  ec_state::TypeSpec t;
  if ((r = ledger_alloc(c, st->spec_bytes, &t.eps)) != EC_OK) return r;
  if ((r = ledger_alloc(c, st->spec_bytes, &t.sig)) != EC_OK) {
    ledger_free(c, t.eps, st->spec_bytes);
    return r;
  }
  auto undo = [&](ec_status rc) {
    (void)hipStreamSynchronize(s);
    ledger_free(c, t.eps, st->spec_bytes);
    ledger_free(c, t.sig, st->spec_bytes);
    return rc;
  };
  for (int k = 0; k < 3; ++k) t.X0[k] = proto->c[k];
  double E12[12] = {0, 0, 0, 0, 0, 0};
  std::copy(d.E, d.E + 6, E12 + 6);
  const int32_t zero = 0;
  int32_t* dids = (int32_t*)ti.p;
  int32_t* dzero = (int32_t*)((char*)ti.p + (size_t)m * 4);
  if (hipMemcpy(dzero, &zero, 4, hipMemcpyHostToDevice) != hipSuccess ||
      (m > 0 && hipMemcpy(dids, ids.data(), (size_t)m * 4, hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(te.p, E12, 96, hipMemcpyHostToDevice) != hipSuccess)
    return undo(fail(EC_ERR_DEVICE, "upload of the prototype failed"));
  const bool fp64 = st->fp64;
  const int n = st->n;
  const Prune rows{d.lo[1], d.w[1], d.lo[2], d.w[2]}, full{0, n, 0, n};
  // eps*_hat_0: the rasterised prototype's rows, then the y pass over its
  // planes and the z pass over the cleared spectrum
  hipError_t e = launch_fill_i32((int32_t*)t.eps, (int64_t)(st->spec_bytes / 4), 0, s);
  if (e == hipSuccess)
    e = launch_x_forward_sparse(fp64, dids, dzero, dids, m, 0, 0, 0, (const double*)te.p, t.eps, st->g, d.lo[1],
                                d.w[1], d.lo[2], d.w[2], st->tw, nullptr, s);
  if (e == hipSuccess) e = launch_pencil(fp64, false, 1, t.eps, st->g, rows, st->tw, nullptr, s);
  if (e == hipSuccess) e = launch_pencil(fp64, false, 2, t.eps, st->g, full, st->tw, nullptr, s);
  // sigma_hat_0 = S(xi):eps*_hat_0, the mean stress at xi = 0
  if (e == hipSuccess) e = hipMemcpyAsync(t.sig, t.eps, st->spec_bytes, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = launch_green(fp64, t.sig, st->g, st->C, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && st->prob.bc == EC_MEAN_STRAIN_ZERO) {
    double m6[6], s6[6];
    for (int a = 0; a < 6; ++a) m6[a] = (double)m * d.E[a];
    neg_C_dot(st, m6, s6);  // N <sigma> = -C : (m E)
    if (fp64) {
      double2 v[6];
      for (int a = 0; a < 6; ++a) v[a] = make_double2(s6[a], 0.0);
      e = hipMemcpy(t.sig, v, sizeof v, hipMemcpyHostToDevice);
    } else {
      float2 v[6];
      for (int a = 0; a < 6; ++a) v[a] = make_float2((float)s6[a], 0.0f);
      e = hipMemcpy(t.sig, v, sizeof v, hipMemcpyHostToDevice);
    }
  }
  if (e != hipSuccess) return undo(fail(EC_ERR_DEVICE, "HIP error %s", hipGetErrorString(e)));
  st->types.push_back(t);
  st->held += 2 * st->spec_bytes;
  *type = (int32_t)st->types.size() - 1;
  return EC_OK;
}

ec_status ec_type_energies(ec_state* st, int32_t type, const double* X, int32_t k, const double* X_excl,
                           void* stream, double* E_out) {
  if (!st) return fail(EC_ERR_ARG, "NULL argument");
  if (k < 0) return fail(EC_ERR_ARG, "negative position count");
  if (k > 0 && (!X || !E_out)) return fail(EC_ERR_ARG, "NULL argument");
  if (!st->solved) return fail(EC_ERR_STATE, "no solve on this state yet");
  if (type < 0 || type >= (int32_t)st->types.size()) return fail(EC_ERR_ARG, "type %d is not stored", type);
  for (int64_t i = 0; i < 3 * (int64_t)k; ++i)
    if (!std::isfinite(X[i])) return fail(EC_ERR_ARG, "position %lld is not finite", (long long)(i / 3));
  if (X_excl)
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(X_excl[a])) return fail(EC_ERR_ARG, "excluded position is not finite");
  if (k == 0) return EC_OK;
  hipStream_t s = (hipStream_t)stream;
  {
    const ec_status r0 = ensure_sigma(st, s);  // the whole resident field is transformed
    if (r0 != EC_OK) return r0;
  }
  const int n = st->n;
  const double L = st->prob.L;
  const int grid = type_energy_grid(n);
  const size_t ntab = (size_t)(TYPE_NP + 1) * 3 * n, nnyq = (size_t)(TYPE_NP + 1) * 3;
  const size_t need = 2 * (ntab + nnyq) + (size_t)grid * TYPE_NP + (size_t)k;
  ec_status r;
  size_t cap = st->tbuf_cap;
  if ((r = st_grow(st, &st->tbuf, &cap, need)) != EC_OK) return r;
  st->tbuf_cap = cap;
  double2* dtab = (double2*)st->tbuf;
  double2* dnyq = dtab + ntab;
  double* partial = (double*)(dnyq + nnyq);
  double* dE = partial + (size_t)grid * TYPE_NP;
  const ec_state::TypeSpec& T = st->types[type];
  const bool fp64 = st->fp64;
  const Prune full{0, n, 0, n};
  // sigma_hat of the resident stress in the work spectrum
  hipError_t e = launch_x_forward_vm(fp64, st->sig, st->spec, st->g, st->tw, s);
  if (e == hipSuccess) e = launch_pencil(fp64, false, 1, st->spec, st->g, full, st->tw, nullptr, s);
  if (e == hipSuccess) e = launch_pencil(fp64, false, 2, st->spec, st->g, full, st->tw, nullptr, s);
  if (e != hipSuccess) return fail(EC_ERR_DEVICE, "HIP error %s", hipGetErrorString(e));
  // phase factors exp(-2 pi i l d / L) per axis and label l (the centred label
  // of each bin, -n/2 at an even n's Nyquist bin; +n/2 in the second table)
  std::vector<double2> htab(ntab), hnyq(nnyq);
  auto factor = [&](int l, double u) {
    double t = (double)l * u;
    t -= std::floor(t);
    return make_double2(std::cos(2.0 * M_PI * t), -std::sin(2.0 * M_PI * t));
  };
  auto fill = [&](int p, const double* Xp) {
    for (int a = 0; a < 3; ++a) {
      const double u = (Xp[a] - T.X0[a]) / L;
      double2* row = htab.data() + ((size_t)p * 3 + a) * n;
      for (int q = 0; q < n; ++q) row[q] = factor(q <= (n - 1) / 2 ? q : q - n, u);
      hnyq[(size_t)p * 3 + a] = factor(n / 2, u);
    }
  };
  const double scale = -st->h3c / (double)st->n3;
  for (int p0 = 0; p0 < k; p0 += TYPE_NP) {
    const int np = std::min(TYPE_NP, k - p0);
    if (p0 > 0 && (e = hipStreamSynchronize(s)) != hipSuccess) break;  // the host tables are refilled
    for (int p = 0; p < np; ++p) fill(p, X + 3 * (size_t)(p0 + p));
    if (X_excl) fill(np, X_excl);
    const size_t rows = (size_t)(np + (X_excl ? 1 : 0));
    if ((e = hipMemcpyAsync(dtab, htab.data(), rows * 3 * n * sizeof(double2), hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(dnyq, hnyq.data(), rows * 3 * sizeof(double2), hipMemcpyHostToDevice, s)) !=
            hipSuccess)
      break;
    // the excluded mover's factors sit in entry np of the tables
    if ((e = launch_type_energies(fp64, st->spec, T.eps, T.sig, st->g, dtab, dnyq, np, X_excl != nullptr, partial,
                                  scale, dE + p0, s)) != hipSuccess)
      break;
  }
  if (e == hipSuccess) e = hipMemcpyAsync(E_out, dE, (size_t)k * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(EC_ERR_DEVICE, "HIP error %s", hipGetErrorString(e));
  return EC_OK;
}

ec_status ec_debug_forward(ec_state* st, const double* field, double* out) {
  if (!st || !field || !out) return fail(EC_ERR_ARG, "NULL argument");
  const size_t cnt = (size_t)6 * st->n3;
  Tmp fd{st->ctx}, sp{st->ctx};
  ec_status r;
  if ((r = ledger_alloc(st->ctx, fd.b = cnt * 8, &fd.p)) != EC_OK) return r;
  if ((r = ledger_alloc(st->ctx, sp.b = st->spec_bytes, &sp.p)) != EC_OK) return r;
  HIPCHK(hipMemcpy(fd.p, field, cnt * 8, hipMemcpyHostToDevice));
  const Prune full{0, st->n, 0, st->n};
  HIPCHK(launch_x_forward(st->fp64, nullptr, nullptr, nullptr, 0, (const double*)fd.p, sp.p, st->g, st->tw, nullptr,
                          nullptr));
  HIPCHK(launch_pencil(st->fp64, false, 1, sp.p, st->g, full, st->tw, nullptr, nullptr));
  HIPCHK(launch_pencil(st->fp64, false, 2, sp.p, st->g, full, st->tw, nullptr, nullptr));
  HIPCHK(hipDeviceSynchronize());
  return download_spec(st, sp.p, out);
}

ec_status ec_debug_green(ec_state* st, const double* in, double* out) {
  if (!st || !in || !out) return fail(EC_ERR_ARG, "NULL argument");
  Tmp sp{st->ctx};
  ec_status r;
  if ((r = ledger_alloc(st->ctx, sp.b = st->spec_bytes, &sp.p)) != EC_OK) return r;
  if ((r = upload_spec(st, in, sp.p)) != EC_OK) return r;
  HIPCHK(launch_green(st->fp64, sp.p, st->g, st->C, nullptr));
  HIPCHK(hipDeviceSynchronize());
  return download_spec(st, sp.p, out);
}

ec_status ec_debug_inverse(ec_state* st, const double* in, double* out) {
  if (!st || !in || !out) return fail(EC_ERR_ARG, "NULL argument");
  const size_t cnt = (size_t)6 * st->n3;
  Tmp sp{st->ctx}, sg{st->ctx}, ad{st->ctx}, cm{st->ctx};
  ec_status r;
  if ((r = ledger_alloc(st->ctx, sp.b = st->spec_bytes, &sp.p)) != EC_OK) return r;
  if ((r = ledger_alloc(st->ctx, sg.b = cnt * 8, &sg.p)) != EC_OK) return r;
  if ((r = ledger_alloc(st->ctx, cm.b = cnt * 8, &cm.p)) != EC_OK) return r;
  if ((r = ledger_alloc(st->ctx, ad.b = 64, &ad.p)) != EC_OK) return r;
  if ((r = upload_spec(st, in, sp.p)) != EC_OK) return r;
  HIPCHK(hipMemset(ad.p, 0, 64));
  const Prune full{0, st->n, 0, st->n};
  HIPCHK(launch_pencil(st->fp64, true, 2, sp.p, st->g, full, st->tw, nullptr, nullptr));
  HIPCHK(launch_pencil(st->fp64, true, 1, sp.p, st->g, full, st->tw, nullptr, nullptr));
  HIPCHK(launch_x_inverse(st->fp64, false, sp.p, (double*)sg.p, st->g, (const double*)ad.p, st->tw, nullptr));
  // voxel-major result -> the component-major [6][n^3] of the entry point
  HIPCHK(launch_sig_to_out((const double*)sg.p, nullptr, nullptr, nullptr, 0, st->n3, st->C, 0, false, cm.p, nullptr));
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(out, cm.p, cnt * 8, hipMemcpyDeviceToHost));
  return EC_OK;
}

}  // extern "C"
