// Fit server: continuous batching of pseudo-experiment fits (the toy studies
// of Sec. 4) on one GPU.
//
// Each fit minimises the NLL of its own data sample over the coefficients
// and x, y with BFGS; the lineshapes are fixed, so the normalisation comes
// from one shared MC Gram matrix and an evaluation streams the fit's data
// only. A streamed server lets the fits float the masses and widths too: it
// keeps the MC sample's tier-0 cache and every tick evaluates all active fits'
// MC sums in one launch that reads each range of MC events once for all of
// them. The scheduler (scheduler.h) runs ticks on a worker thread: it admits
// queued fits while a slot and the HBM budget allow (here: building each
// fit's cache: with fixed lineshapes its basis, otherwise its tier-0
// record), asks every active fit for the point its minimiser wants
// evaluated, evaluates all of them in one device call (the constants read in
// place from mapped host memory, one persistent launch over a (fit, event
// range) work table, the per-fit totals reduced into mapped host memory, a
// flag set behind them),
// forms each fit's NLL and gradient from its totals on the host, and feeds
// the results back. Finished fits free their slot and
// memory at once, so later arrivals join the running batch. A fit's result
// does not depend on the fits it shares launches with.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>
#include <new>
#include <vector>

#include "../../include/mixamp.h"
#include "bfgs.h"
#include "internal.h"
#include "scheduler.h"

using namespace mxa;

namespace {

#define SRV_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return set_error(e_ == hipErrorOutOfMemory ? MXA_ENOMEM : MXA_EDEVICE, "%s: %s", #expr, \
                       hipGetErrorString(e_));                                               \
  } while (0)

int64_t round256(int64_t b) { return (b + 255) / 256 * 256; }
int64_t word_of(int precision) { return precision == MXA_FP64 ? sizeof(double) : sizeof(float); }
// Device bytes a fit of n events holds: its cache of `cols` columns in the
// server's precision (the tier-0 record on a streamed server, the basis with
// fixed lineshapes) and the decay times.
int64_t footprint(int64_t n, int precision, int cols) {
  const int64_t ld = (n + 63) / 64 * 64;
  return ld * (cols * word_of(precision) + static_cast<int64_t>(sizeof(double)));
}
// Device bytes a fit holds while it is admitted only: its events and times
// as copied from the host (none when they are on the device already), a
// validation counter and, with fixed lineshapes, the tier-0 record its basis
// is computed from.
int64_t events_bytes(int64_t n, bool host) { return host ? round256(n * 16 * 8) + round256(n * 8) : 0; }
int64_t staging_bytes(int64_t n, int precision, bool basis, bool host) {
  const int64_t ld = (n + 63) / 64 * 64;
  return events_bytes(n, host) + 256 + (basis ? round256(NCOL * ld * word_of(precision)) : 0);
}

// Admission threads: each copies a fit's events to the device and builds its
// cache on a stream of its own, so that admissions overlap one another (the
// copy from pageable host memory, not the link, limits one admission).
constexpr int N_ADMIT = 4;

// The device memory of the admitted fits: one allocation of the HBM budget,
// made when the server is created and carved first-fit into 256-byte
// aligned blocks (a fit's cache and decay times, followed while it is
// admitted by its staging); freed ranges merge with their free neighbours.
// Host bookkeeping only; every call runs under the scheduler's lock.
class Arena {
 public:
  hipError_t init(int64_t bytes) {
    size_ = bytes / 256 * 256;
    const hipError_t e = hipMalloc(&base_, size_);
    if (e == hipSuccess) free_[0] = size_;
    return e;
  }
  void destroy() {
    if (base_) (void)hipFree(base_);
    base_ = nullptr;
  }
  char* base() const { return base_; }
  // first free range that holds n bytes; false if none does
  bool alloc(int64_t n, int64_t* off) {
    n = round256(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const int64_t rest = it->second - n;
      free_.erase(it);
      if (rest > 0) free_[*off + n] = rest;
      used_[*off] = n;
      return true;
    }
    return false;
  }
  // shrink the block at off to its first n bytes
  void shrink(int64_t off, int64_t n) {
    auto it = used_.find(off);
    if (it == used_.end()) return;
    n = round256(n);
    if (n >= it->second) return;
    put_back(off + n, it->second - n);
    it->second = n;
  }
  void release(int64_t off) {
    auto it = used_.find(off);
    if (it == used_.end()) return;
    const int64_t n = it->second;
    used_.erase(it);
    put_back(off, n);
  }

 private:
  void put_back(int64_t off, int64_t n) {
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }
  char* base_ = nullptr;
  int64_t size_ = 0;
  std::map<int64_t, int64_t> free_, used_;  // offset -> bytes
};

struct GpuDev;

}  // namespace

struct mxa_server {
  mxa_model_desc model;
  int device = 0;
  int precision = MXA_FP32AMP;
  int ma = 0, mb = 0, n_theta = 0;
  int cache_cols = NCOL;        // columns of a fit's cache: NCOL, or its basis's
  double shape[6];
  EvalParams shape_params;      // fixed lineshapes: constants the bases are computed at
  int64_t n_mc = 0;
  int64_t budget = 0;
  Arena arena;  // the admitted fits' device memory (the HBM budget)
  int max_slots = 0, max_rows = 0;
  hipStream_t stream = nullptr;        // the worker's ticks
  hipStream_t admit_streams[N_ADMIT] = {};  // each admission thread's copies and cache builds
  double h_gram[128] = {};             // shared MC Gram of the reduced chain amplitudes
  // streamed server (floating lineshapes): shared MC tier-0 cache and rows
  bool streamed = false;
  void* d_mc = nullptr;
  int64_t mc_ld = 0, epb_mc = 0;
  int32_t nb_mc = 0, mc_grid = 0;
  int32_t* d_active = nullptr;
  int32_t* d_nactive = nullptr;
  double* d_mc_rows = nullptr;
  // batch tables
  int n_groups = 1;                // groups of slots evaluated alternately
  FitItem* d_items = nullptr;      // [n_groups][max_items]
  int32_t* d_nitems = nullptr;     // [n_groups]
  FitView* d_views = nullptr;
  // per group, [max_slots]: mapped coherent host memory, written by the host
  // before a launch and read in place by the kernels (no upload per tick)
  EvalParams* h_params[2] = {};
  EvalParams* d_params[2] = {};    // their device addresses
  double* d_rows = nullptr;
  double* h_tot = nullptr;         // [max_slots][2][64] totals, mapped pinned
  double* d_tot = nullptr;         // its device address
  unsigned* h_done = nullptr;      // per group: set by the device behind the totals, mapped pinned
  unsigned* d_done = nullptr;
  std::vector<char> outside;       // per slot: its point is outside the model's domain
  std::vector<double> results;     // [max_slots][RES_WORDS], formed on the host
  int max_items = 0;
  hipGraph_t graph[2] = {};
  hipGraphExec_t exec[2] = {};
  std::atomic<bool> use_graph{false};
  Scheduler sched;
  GpuDev* dev = nullptr;
};

namespace {

// A fit's device state, in one arena block: dev[0] the FP64 or dev[1] the
// FP32 tier-0 cache, dev[2] the decay times, and during admission the staging
// after them.
int64_t block_of(mxa_server* s, const Fit* f) {
  const void* p = f->dev[0] ? f->dev[0] : f->dev[1];
  return p ? static_cast<const char*>(p) - s->arena.base() : -1;
}

// Set aside the fit's block (scheduler lock held).
bool reserve(mxa_server* s, Fit* f) {
  int64_t off = 0;
  if (!s->arena.alloc(f->footprint + f->staging, &off)) return false;
  f->ld = (f->n + 63) / 64 * 64;
  char* b = s->arena.base() + off;
  const int64_t cache = s->cache_cols * f->ld * word_of(s->precision);
  f->dev[s->precision == MXA_FP64 ? 0 : 1] = b;
  f->dev[2] = b + cache;
  return true;
}

void free_fit_device(mxa_server* s, Fit* f) {
  const int64_t off = block_of(s, f);
  if (off >= 0) s->arena.release(off);
  for (void*& p : f->dev) p = nullptr;
}

// Build the fit's cache in its block (called by the admission thread,
// without the scheduler's lock, on its own stream while the worker's ticks go
// on): its tier-0 record, and with fixed lineshapes the basis from it. No
// device allocation: the staging is the block's tail.
int32_t admit(mxa_server* s, Fit* f, int lane) {
  hipStream_t as = s->admit_streams[lane];
  const bool host = f->d_p4 == nullptr;
  char* tail = static_cast<char*>(f->dev[2]) + f->ld * sizeof(double);
  const double* sp = host ? reinterpret_cast<double*>(tail) : f->d_p4;
  const double* st = host ? reinterpret_cast<double*>(tail + round256(f->n * 16 * 8)) : f->d_t;
  char* after = tail + events_bytes(f->n, host);
  unsigned* bad = reinterpret_cast<unsigned*>(after);
  void* rec = s->streamed ? (f->dev[0] ? f->dev[0] : f->dev[1]) : after + 256;
  const bool f64 = s->precision == MXA_FP64;
  unsigned hbad = 0;
  hipError_t e = hipSuccess;
  if (host) {
    e = hipMemcpyAsync(const_cast<double*>(sp), f->p4.data(), f->n * 16 * sizeof(double), hipMemcpyHostToDevice,
                       as);
    if (e == hipSuccess)
      e = hipMemcpyAsync(const_cast<double*>(st), f->t.data(), f->n * sizeof(double), hipMemcpyHostToDevice, as);
  }
  if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(unsigned), as);
  Tier0Const k;
  k.m_D = s->model.m_D;
  k.m_K = s->model.m_K;
  k.m_pi = s->model.m_pi;
  k.r = s->model.r;
  k.tol_p = 1e-6;
  k.tol_m2 = 1e-6;
  k.allow_neg_t = s->model.sigma_t > 0.0 ? 1 : 0;  // measured times under a resolution
  if (e == hipSuccess)
    e = launch_tier0(k, sp, st, f->n, f->ld, f64 ? static_cast<double*>(rec) : nullptr,
                     f64 ? nullptr : static_cast<float*>(rec), static_cast<double*>(f->dev[2]), bad,
                     as);
  if (e == hipSuccess && !s->streamed)
    e = launch_basis(f64 ? 0 : 1, s->ma, s->mb, rec, f->ld, f->n, s->shape_params, f64 ? f->dev[0] : f->dev[1],
                     f->ld, as);
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(unsigned), hipMemcpyDeviceToHost, as);
  if (e == hipSuccess) e = hipStreamSynchronize(as);
  if (e != hipSuccess) return set_error(MXA_EDEVICE, "admission: %s", hipGetErrorString(e));
  if (hbad) return set_error(MXA_EINVAL, "%u data events fail validation", hbad);
  std::vector<double>().swap(f->p4);
  std::vector<double>().swap(f->t);
  return MXA_OK;
}

// Rewrite the work tables (one per group of slots) and views for the current
// set of active fits.
int32_t upload_tables(mxa_server* s, const std::vector<Fit*>& slots) {
  std::vector<FitItem> items[2];
  std::vector<FitView> views(s->max_slots);
  int row = 0;
  for (int sl = 0; sl < s->max_slots; ++sl) {
    FitView& v = views[sl];
    memset(&v, 0, sizeof v);
    Fit* f = slots[sl];
    if (!f) continue;
    v.cache = s->precision == MXA_FP64 ? f->dev[0] : f->dev[1];
    v.t = static_cast<const double*>(f->dev[2]);
    v.ld = f->ld;
    v.n = f->n;
    v.row0 = row;
    v.active = 1;
    // chunks by the fit's own size only, so that its rows (and result) do not
    // depend on the other fits
    const int64_t chunk = fit_chunk(f->n);
    for (int64_t lo = 0; lo < f->n; lo += chunk) {
      FitItem it;
      it.slot = sl;
      it.row = row++;
      it.lo = lo;
      it.hi = std::min<int64_t>(lo + chunk, f->n);
      items[sl % s->n_groups].push_back(it);
    }
    v.nrows = row - v.row0;
  }
  if (s->streamed) {
    std::vector<int32_t> act;
    for (int sl = 0; sl < s->max_slots; ++sl)
      if (slots[sl]) act.push_back(sl);
    const int32_t na = static_cast<int32_t>(act.size());
    if (na > 0)
      SRV_TRY(hipMemcpyAsync(s->d_active, act.data(), na * sizeof(int32_t), hipMemcpyHostToDevice, s->stream));
    SRV_TRY(hipMemcpyAsync(s->d_nactive, &na, sizeof na, hipMemcpyHostToDevice, s->stream));
  }
  int32_t ni[2] = {};
  for (int g = 0; g < s->n_groups; ++g) {
    if (static_cast<int>(items[g].size()) > s->max_items)
      return set_error(MXA_EINVAL, "work table overflow (%zu items)", items[g].size());
    ni[g] = static_cast<int32_t>(items[g].size());
    if (ni[g] > 0)
      SRV_TRY(hipMemcpyAsync(s->d_items + static_cast<int64_t>(g) * s->max_items, items[g].data(),
                             ni[g] * sizeof(FitItem), hipMemcpyHostToDevice, s->stream));
  }
  SRV_TRY(hipMemcpyAsync(s->d_nitems, ni, s->n_groups * sizeof(int32_t), hipMemcpyHostToDevice, s->stream));
  SRV_TRY(hipMemcpyAsync(s->d_views, views.data(), views.size() * sizeof(FitView), hipMemcpyHostToDevice,
                         s->stream));
  SRV_TRY(hipStreamSynchronize(s->stream));
  return MXA_OK;
}

BatchArgs batch_args(mxa_server* s, int g) {
  BatchArgs a;
  a.items = s->d_items + static_cast<int64_t>(g) * s->max_items;
  a.n_items = s->d_nitems + g;
  a.views = s->d_views;
  a.params = s->d_params[g];
  a.rows = s->d_rows;
  a.max_rows = s->max_rows;
  a.max_slots = s->max_slots;
  a.n_mc = s->n_mc;
  a.mc_cache = s->streamed ? s->d_mc : nullptr;
  a.mc_ld = s->mc_ld;
  a.epb_mc = s->epb_mc;
  a.nb_mc = s->nb_mc;
  a.mc_grid = s->mc_grid;
  a.active = s->d_active;
  a.n_active = s->d_nactive;
  a.mc_rows = s->d_mc_rows;
  a.tot = s->d_tot;
  a.done = s->d_done + g;
  a.group = g;
  a.ngroups = s->n_groups;
  a.bkg = s->model.g_bkg > 0.0 ? 1 : 0;
  a.res = s->model.sigma_t > 0.0 ? 1 : 0;
  return a;
}

// One group's device work: the batched passes (which read the fits'
// parameters in place from mapped host memory: against an upload per tick,
// Poisson p50 2.78 -> 2.55 ms, one fit at a time 3.35 -> 3.01 ms), the
// reduction into host memory, the group's flag.
int32_t enqueue_tick(mxa_server* s, int g) {
  SRV_TRY(launch_batch(s->precision, s->ma, s->mb, batch_args(s, g), s->stream));
  return MXA_OK;
}

// Waiting for a tick: the host watches the flag for up to TICK_SPIN_NS, then
// synchronises the stream (which also reports a launch error).
constexpr int64_t TICK_SPIN_NS = 2000000;
bool wait_flag(const unsigned* flag) {
  const auto t0 = std::chrono::steady_clock::now();
  while (true) {
    for (int i = 0; i < 256; ++i)
      if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == 1u) return true;
    if (std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count() >
        TICK_SPIN_NS)
      return false;
  }
}

// Direct launches by default: on one MI355X they took 8-9 us of host time per
// tick against 21-22 us for replaying the same work as a graph (then a
// parameter copy and three kernels), and the fixed-lineshape tick of one fit
// ran 40 against 45 us.
int32_t launch_tick(mxa_server* s, int g) {
  __atomic_store_n(s->h_done + g, 0u, __ATOMIC_RELEASE);  // the device sets it once the totals are out
  if (s->use_graph) {
    if (!s->exec[g]) {
      SRV_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
      const int32_t rc = enqueue_tick(s, g);
      hipGraph_t gr = nullptr;
      const hipError_t e = hipStreamEndCapture(s->stream, &gr);
      if (rc) return rc;
      SRV_TRY(e);
      s->graph[g] = gr;
      SRV_TRY(hipGraphInstantiate(&s->exec[g], s->graph[g], nullptr, nullptr, 0));
    }
    SRV_TRY(hipGraphLaunch(s->exec[g], s->stream));
    return MXA_OK;
  }
  return enqueue_tick(s, g);
}

int32_t wait_tick(mxa_server* s, int g) {
  if (!wait_flag(s->h_done + g)) SRV_TRY(hipStreamSynchronize(s->stream));
  return MXA_OK;
}

// The scheduler's device policy (see scheduler.h).
struct GpuDev {
  mxa_server* s;
  void thread_init() { (void)hipSetDevice(s->device); }
  bool reserve(Fit& f) { return ::reserve(s, &f); }
  int32_t admit(Fit& f, int lane) { return ::admit(s, &f, lane); }
  void drop_staging(Fit& f) {
    const int64_t off = block_of(s, &f);
    if (off >= 0) s->arena.shrink(off, f.footprint);
  }
  void release(Fit& f) { free_fit_device(s, &f); }
  int32_t tables(const std::vector<Fit*>& slots) { return upload_tables(s, slots); }
  int groups() const { return s->n_groups; }
  // Group g's active fits at their next points: their constants (a point
  // outside the model's domain, |y| >= 1, ..., is evaluated with neutral
  // constants and reported to the minimiser as +inf; with a background
  // component each fit's 1 / Nhat comes from the shared Gram matrix here,
  // before the data pass), then the group's device call, without waiting.
  int32_t launch(const std::vector<Fit*>& slots, int g) {
    const bool bkg = s->model.g_bkg > 0.0;
    for (size_t sl = g; sl < slots.size(); sl += s->n_groups) {
      Fit* f = slots[sl];
      if (!f) continue;
      EvalParams& P = s->h_params[g][sl];
      s->outside[sl] = 0;
      if (make_params(s->model, f->bfgs.point(), P) != MXA_OK) {
        s->outside[sl] = 1;
        make_params(s->model, f->theta0.data(), P);
      }
      if (bkg) P.mix.inv_nhat = static_cast<double>(s->n_mc) / gram_sum_t(s->ma, s->mb, P, s->h_gram);
    }
    return launch_tick(s, g);
  }
  // Wait for group g: the device has reduced every fit's sums into host
  // memory, and each fit's NLL and gradient are formed here.
  int32_t collect(const std::vector<Fit*>& slots, int g, std::vector<double>& nll,
                  std::vector<const double*>& grad) {
    const int32_t rc = wait_tick(s, g);
    if (rc) return rc;
    for (size_t sl = g; sl < slots.size(); sl += s->n_groups) {
      Fit* f = slots[sl];
      if (!f) continue;
      double D[64], M[64];
      const double* T = s->h_tot + static_cast<int64_t>(sl) * 128;
      memcpy(D, T, sizeof D);
      if (s->streamed) memcpy(M, T + 64, sizeof M);
      EvalArgs e = {};
      e.n_d = f->n;
      e.n_m = s->n_mc;
      e.result = s->results.data() + static_cast<int64_t>(sl) * RES_WORDS;
      finalize_host(s->ma, s->mb, true, e, s->h_params[g][sl], D, M, s->streamed ? nullptr : s->h_gram);
      nll[sl] = s->outside[sl] ? INFINITY : e.result[0];
      grad[sl] = e.result + 8;
    }
    return MXA_OK;
  }
  const char* error() { return mxa_last_error(); }
};

// Streamed server: the MC sample's tier-0 cache in the server's precision,
// and its split into nb_mc ranges (a multiple of 8, as the MC walk needs).
int32_t build_mc_cache(mxa_server* s, const double* mc_p4) {
  const int64_t n = s->n_mc;
  s->mc_ld = (n + 63) / 64 * 64;
  const int64_t bm = std::min<int64_t>(1024, (n + 4 * BLOCK - 1) / (4 * BLOCK));
  s->nb_mc = static_cast<int32_t>((bm + 7) / 8 * 8);
  s->epb_mc = (n + s->nb_mc - 1) / s->nb_mc;
  s->mc_grid = batch_mc_grid(s->precision, s->ma, s->mb, s->device);
  if (s->mc_grid < 8) return set_error(MXA_EDEVICE, "occupancy query of the MC walk failed");
  const size_t word = s->precision == MXA_FP64 ? sizeof(double) : sizeof(float);
  SRV_TRY(hipMalloc(&s->d_mc, NCOL * s->mc_ld * word));
  SRV_TRY(hipMalloc(&s->d_active, s->max_slots * sizeof(int32_t)));
  SRV_TRY(hipMalloc(&s->d_nactive, sizeof(int32_t)));
  SRV_TRY(hipMemsetAsync(s->d_nactive, 0, sizeof(int32_t), s->stream));
  SRV_TRY(hipMalloc(&s->d_mc_rows, static_cast<size_t>(43) * s->max_slots * s->nb_mc * 2 * sizeof(double)));
  double* sp = nullptr;
  unsigned* bad = nullptr;
  unsigned hbad = 0;
  hipError_t e = hipMalloc(&sp, n * 16 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&bad, sizeof(unsigned));
  if (e == hipSuccess) e = hipMemcpyAsync(sp, mc_p4, n * 16 * sizeof(double), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(unsigned), s->stream);
  Tier0Const k;
  k.m_D = s->model.m_D;
  k.m_K = s->model.m_K;
  k.m_pi = s->model.m_pi;
  k.r = s->model.r;
  k.tol_p = 1e-6;
  k.tol_m2 = 1e-6;
  double* c64 = s->precision == MXA_FP64 ? static_cast<double*>(s->d_mc) : nullptr;
  float* c32 = s->precision == MXA_FP64 ? nullptr : static_cast<float*>(s->d_mc);
  if (e == hipSuccess) e = launch_tier0(k, sp, nullptr, n, s->mc_ld, c64, c32, nullptr, bad, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(unsigned), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (sp) (void)hipFree(sp);
  if (bad) (void)hipFree(bad);
  if (e != hipSuccess)
    return set_error(e == hipErrorOutOfMemory ? MXA_ENOMEM : MXA_EDEVICE, "MC tier-0 cache: %s",
                     hipGetErrorString(e));
  if (hbad) return set_error(MXA_EINVAL, "%u MC events fail validation", hbad);
  return MXA_OK;
}

// Shared set-up of both server kinds: shape null makes a streamed server.
int32_t create_server(const mxa_model_desc* model, int32_t device, int32_t precision,
                      const double* shape, const double* mc_p4, int64_t n_mc,
                      int64_t hbm_budget_bytes, int32_t max_slots, mxa_server** out) {
  if (!out) return set_error(MXA_EINVAL, "out is NULL");
  *out = nullptr;
  int32_t rc = check_model_desc(model);
  if (rc) return rc;
  if (model->cpv) return set_error(MXA_EINVAL, "the fit server does not take models with CP violation");
  if (!shape && (model->g_bkg > 0.0 || model->sigma_t > 0.0))
    return set_error(MXA_EINVAL, "the streamed server does not take models with a background component or "
                     "a decay-time resolution");
  if (precision != MXA_FP64 && precision != MXA_FP32AMP) return set_error(MXA_EINVAL, "bad precision");
  if (!mc_p4 || n_mc <= 0) return set_error(MXA_EINVAL, "an MC sample is required");
  if (!shape && n_mc > INT32_MAX - 1024) return set_error(MXA_EINVAL, "n_mc must be below 2^31 - 1024");
  if (max_slots < 1 || max_slots > 256) return set_error(MXA_EINVAL, "max_slots must be in 1..256");
  if (hbm_budget_bytes <= 0) return set_error(MXA_EINVAL, "HBM budget must be positive");
  mxa_server* s = new (std::nothrow) mxa_server();
  if (!s) return set_error(MXA_ENOMEM, "host allocation failed");
  s->dev = new (std::nothrow) GpuDev{s};
  if (!s->dev) {
    delete s;
    return set_error(MXA_ENOMEM, "host allocation failed");
  }
  s->model = *model;
  s->device = device;
  s->precision = precision;
  s->n_theta = theta_count(*model);
  s->streamed = shape == nullptr;
  if (shape)
    memcpy(s->shape, shape, sizeof s->shape);
  else
    for (double& v : s->shape) v = NAN;
  s->n_mc = n_mc;
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  for (int j = 0; j < model->n_a; ++j) s->ma |= 1 << (model->comp_a[j] - 1);
  for (int j = 0; j < model->n_ab; ++j) s->mb |= 1 << (model->comp_ab[j] - 1);
  s->sched.init(max_slots, hbm_budget_bytes, s->n_theta);
  double g[128] = {};
  if (!s->streamed) {
    // the shared MC Gram at the fixed masses and widths, built by a context
    mxa_ctx* ctx = nullptr;
    rc = mxa_create(model, device, nullptr, &ctx);
    std::vector<double> th(s->n_theta, 0.0);
    for (int i = 0; i < 2 * (model->n_a + model->n_ab); i += 2) th[i] = 1.0;
    th[2 * (model->n_a + model->n_ab) + 1] = 0.0;
    memcpy(th.data() + shape_offset(*model), shape, 6 * sizeof(double));
    if (!rc) rc = mxa_load_events(ctx, MXA_MC, mc_p4, nullptr, n_mc);
    if (!rc) rc = mxa_set_params(ctx, th.data(), s->n_theta);
    if (!rc) rc = mxa_gram(ctx, precision, g);
    if (ctx) mxa_destroy(ctx);
    if (rc) {
      mxa_server_destroy(s);
      return rc;
    }
    // mxa_gram returns the Gram of the chain amplitudes B_k = kappa_k beta_k; the
    // kernels use the reduced one
    EvalParams& P = s->shape_params;
    rc = make_params(*model, th.data(), P);
    if (rc) {
      mxa_server_destroy(s);
      return rc;
    }
    s->cache_cols = basis_columns(s->ma, s->mb);
    for (int k = 0; k < 8; ++k)
      for (int l = 0; l < 8; ++l)
        for (int q = 0; q < 2; ++q) {
          const double kk = P.fin.kappa[k] * P.fin.kappa[l];
          g[(k * 8 + l) * 2 + q] = kk != 0.0 ? g[(k * 8 + l) * 2 + q] / kk : 0.0;
        }
  }
  const int32_t NSmax = 43 + 2;  // the general model's sums, + 2 with a background component
  s->max_items = static_cast<int>(max_slots * MAX_FIT_ITEMS + 64);
  s->max_rows = s->max_items;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  for (hipStream_t& as : s->admit_streams)
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&as, hipStreamNonBlocking);
  if (e == hipSuccess) e = s->arena.init(hbm_budget_bytes);
  // One group of slots: every active fit in each device call. Two groups
  // evaluated alternately (each group's results fed back while the device
  // evaluates the other) were measured on the serving benchmark and not
  // kept: all fits at once 1,840 -> 1,894 fits/s, but Poisson p50 2.8 ->
  // 3.2 ms and the 256 MB budget run 1,340 -> 1,187 fits/s, each group's
  // call carrying the fixed costs of a tick. (A streamed server's single MC
  // walk serves all its fits, so it keeps one group in any case.)
  s->n_groups = 1;
  if (e == hipSuccess) e = hipMalloc(&s->d_items, s->n_groups * s->max_items * sizeof(FitItem));
  if (e == hipSuccess) e = hipMalloc(&s->d_nitems, 2 * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&s->d_views, max_slots * sizeof(FitView));
  for (int g = 0; g < 2; ++g) {
    if (e == hipSuccess)
      e = hipHostMalloc(&s->h_params[g], max_slots * sizeof(EvalParams), hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&s->d_params[g]), s->h_params[g], 0);
  }
  if (e == hipSuccess) e = hipMalloc(&s->d_rows, static_cast<size_t>(NSmax) * s->max_rows * 2 * sizeof(double));
  if (e == hipSuccess)
    e = hipHostMalloc(&s->h_tot, static_cast<size_t>(max_slots) * 128 * sizeof(double),
                      hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&s->d_tot), s->h_tot, 0);
  if (e == hipSuccess) e = hipHostMalloc(&s->h_done, 256, hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&s->d_done), s->h_done, 0);
  if (e != hipSuccess) {
    mxa_server_destroy(s);
    return set_error(e == hipErrorOutOfMemory ? MXA_ENOMEM : MXA_EDEVICE, "server setup: %s",
                     hipGetErrorString(e));
  }
  for (EvalParams* hp : s->h_params) memset(hp, 0, max_slots * sizeof(EvalParams));
  s->outside.assign(max_slots, 0);
  memcpy(s->h_gram, g, sizeof g);
  s->results.assign(static_cast<size_t>(max_slots) * RES_WORDS, 0.0);
  if (s->streamed) {
    rc = build_mc_cache(s, mc_p4);
    if (rc) {
      mxa_server_destroy(s);
      return rc;
    }
  }
  s->sched.start(s->dev, N_ADMIT);
  *out = s;
  return MXA_OK;
}

}  // namespace

extern "C" {

int32_t mxa_server_create(const mxa_model_desc* model, int32_t device, int32_t precision,
                          const double* shape, const double* mc_p4, int64_t n_mc,
                          int64_t hbm_budget_bytes, int32_t max_slots, mxa_server** out) {
  if (!shape) return set_error(MXA_EINVAL, "shape is required (mxa_server_create_streamed floats it)");
  return create_server(model, device, precision, shape, mc_p4, n_mc, hbm_budget_bytes, max_slots, out);
}

int32_t mxa_server_create_streamed(const mxa_model_desc* model, int32_t device, int32_t precision,
                                   const double* mc_p4, int64_t n_mc, int64_t hbm_budget_bytes,
                                   int32_t max_slots, mxa_server** out) {
  return create_server(model, device, precision, nullptr, mc_p4, n_mc, hbm_budget_bytes, max_slots, out);
}

int32_t mxa_server_set_graph(mxa_server* s, int32_t on) {
  if (!s) return set_error(MXA_EINVAL, "server is NULL");
  s->use_graph = on != 0;
  return MXA_OK;
}

int32_t mxa_fit_submit(mxa_server* s, const mxa_fit_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return set_error(MXA_EINVAL, "NULL argument");
  if (req->n <= 0 || !req->p4 || !req->t || !req->theta0 || !req->scale)
    return set_error(MXA_EINVAL, "request needs events, times, theta0 and scale");
  if (req->n > MAX_FIT_EVENTS) return set_error(MXA_EINVAL, "a fit holds at most %d events", MAX_FIT_EVENTS);
  if (req->gradient != MXA_GRAD_ADJOINT)
    return set_error(MXA_EINVAL, "the fit server evaluates the adjoint gradient only");
  const bool host = req->events_on_device == 0;
  if (!host) {
    // device memory of the server's device
    for (const double* q : {req->p4, req->t}) {
      hipPointerAttribute_t at;
      if (hipPointerGetAttributes(&at, q) != hipSuccess || at.type != hipMemoryTypeDevice ||
          at.device != s->device) {
        (void)hipGetLastError();
        return set_error(MXA_EINVAL, "events_on_device: p4 and t must be device memory of device %d", s->device);
      }
    }
  }
  const int64_t need =
      footprint(req->n, s->precision, s->cache_cols) + staging_bytes(req->n, s->precision, !s->streamed, host);
  if (need > s->budget / 256 * 256)
    return set_error(MXA_ENOMEM, "fit needs %lld bytes while it is admitted, budget is %lld",
                     static_cast<long long>(need), static_cast<long long>(s->budget));
  Fit* f = new (std::nothrow) Fit();
  if (!f) return set_error(MXA_ENOMEM, "host allocation failed");
  f->n = req->n;
  if (host) {
    f->p4.assign(req->p4, req->p4 + req->n * 16);
    f->t.assign(req->t, req->t + req->n);
  } else {
    f->d_p4 = req->p4;
    f->d_t = req->t;
  }
  f->theta0.assign(req->theta0, req->theta0 + s->n_theta);
  // with fixed lineshapes the masses and widths are the server's
  const int sh0 = shape_offset(s->model);
  if (!s->streamed) memcpy(f->theta0.data() + sh0, s->shape, 6 * sizeof(double));
  std::vector<int> idx;
  std::vector<double> sc;
  for (int i = 0; i < s->n_theta; ++i)
    if (req->scale[i] > 0.0 && (s->streamed || i < sh0 || i >= sh0 + 6)) {
      idx.push_back(i);
      sc.push_back(req->scale[i]);
    }
  if (idx.empty()) {
    delete f;
    return set_error(MXA_EINVAL, "no free parameter (all scales are 0)");
  }
  EvalParams P;
  if (make_params(s->model, f->theta0.data(), P) != MXA_OK) {
    delete f;
    return MXA_EDOMAIN;
  }
  f->bfgs.init(f->theta0.data(), s->n_theta, idx.data(), sc.data(), static_cast<int>(idx.size()),
               req->max_evals > 0 ? req->max_evals : 150, req->gtol > 0 ? req->gtol : 1e-3, req->ftol,
               req->edm_tol > 0 ? req->edm_tol : 0.0, req->errors != 0);
  f->footprint = footprint(req->n, s->precision, s->cache_cols);
  f->staging = staging_bytes(req->n, s->precision, !s->streamed, host);
  char msg[320];
  const int32_t rc = s->sched.submit(f, ticket, msg, sizeof msg);
  return rc ? set_error(rc, "%s", msg) : MXA_OK;
}

int32_t mxa_fit_poll(mxa_server* s, uint64_t ticket, mxa_fit_result* out) {
  if (!s || !out) return set_error(MXA_EINVAL, "NULL argument");
  char msg[320];
  const int32_t rc = s->sched.result(ticket, out, false, msg, sizeof msg);
  return rc && rc != MXA_EAGAIN ? set_error(rc, "%s", msg) : rc;
}

int32_t mxa_fit_wait(mxa_server* s, uint64_t ticket, mxa_fit_result* out) {
  if (!s || !out) return set_error(MXA_EINVAL, "NULL argument");
  char msg[320];
  const int32_t rc = s->sched.result(ticket, out, true, msg, sizeof msg);
  return rc ? set_error(rc, "%s", msg) : MXA_OK;
}

int32_t mxa_fit_cancel(mxa_server* s, uint64_t ticket) {
  if (!s) return set_error(MXA_EINVAL, "server is NULL");
  char msg[320];
  const int32_t rc = s->sched.cancel(ticket, msg, sizeof msg);
  return rc ? set_error(rc, "%s", msg) : MXA_OK;
}

int32_t mxa_fit_release(mxa_server* s, uint64_t ticket) {
  if (!s) return set_error(MXA_EINVAL, "server is NULL");
  char msg[320];
  const int32_t rc = s->sched.release(ticket, msg, sizeof msg);
  return rc ? set_error(rc, "%s", msg) : MXA_OK;
}

int32_t mxa_server_stats(mxa_server* s, int64_t* out) {
  if (!s || !out) return set_error(MXA_EINVAL, "NULL argument");
  s->sched.stats(out);
  return MXA_OK;
}

int32_t mxa_server_destroy(mxa_server* s) {
  if (!s) return MXA_OK;
  if (s->dev) {
    s->sched.shutdown(*s->dev);  // joins the worker, then frees every fit
    (void)hipSetDevice(s->device);
  }
  delete s->dev;
  for (hipGraphExec_t x : s->exec)
    if (x) (void)hipGraphExecDestroy(x);
  for (hipGraph_t gr : s->graph)
    if (gr) (void)hipGraphDestroy(gr);
  if (s->d_mc) (void)hipFree(s->d_mc);
  if (s->d_active) (void)hipFree(s->d_active);
  if (s->d_nactive) (void)hipFree(s->d_nactive);
  if (s->d_mc_rows) (void)hipFree(s->d_mc_rows);
  if (s->d_items) (void)hipFree(s->d_items);
  if (s->d_nitems) (void)hipFree(s->d_nitems);
  if (s->d_views) (void)hipFree(s->d_views);
  for (EvalParams* hp : s->h_params)
    if (hp) (void)hipHostFree(hp);
  if (s->d_rows) (void)hipFree(s->d_rows);
  if (s->h_tot) (void)hipHostFree(s->h_tot);
  if (s->h_done) (void)hipHostFree(s->h_done);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  for (hipStream_t as : s->admit_streams)
    if (as) (void)hipStreamDestroy(as);
  s->arena.destroy();
  delete s;
  return MXA_OK;
}

}  // extern "C"
