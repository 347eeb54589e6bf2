// C ABI of librgf: argument checks, per-(device, stream) workspaces,
// chunking of the energy batch to the free device memory, kernel timing.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "engine.h"

namespace rgf {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

// ---------------------------------------------------------------- profiler
// Kernel timing by class: while on, every `every`-th launch of a class in the
// mask (counted per class) gets a HIP event pair on its own stream; the
// algorithmic flops of every launch of every class are counted, timed or not.
// Records are reaped without blocking (completed events only) while launches
// go on; rgf_profile_read* wait for the rest.
struct Profiler {
  std::mutex mu;
  bool on = false;
  int every = 1;
  uint32_t mask = 1u << PC_SWEEP;
  struct Rec {
    hipEvent_t a, b;
    double flops;
    int cls;
  };
  std::deque<Rec> recs;
  std::vector<hipEvent_t> pool;
  struct Cls {
    int64_t seen = 0;       // launches seen while on (sampling counter)
    int64_t launches = 0;   // timed launches reaped
    double ms = 0.0, flops = 0.0;
    int64_t launches_all = 0;
    double flops_all = 0.0;
  } cls[PC_COUNT];
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    RGF_HIP(hipEventCreate(&e));
    return e;
  }
  void reap(const Rec& r) {
    float t = 0.f;
    RGF_HIP(hipEventElapsedTime(&t, r.a, r.b));
    Cls& c = cls[r.cls];
    c.ms += t;
    c.flops += r.flops;
    ++c.launches;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  // completed records only, oldest first (never waits)
  void reap_ready() {
    while (!recs.empty()) {
      const hipError_t q = hipEventQuery(recs.front().b);
      if (q == hipErrorNotReady) break;
      RGF_HIP(q);
      reap(recs.front());
      recs.pop_front();
    }
  }
  void drain() {
    for (auto& r : recs) {
      RGF_HIP(hipEventSynchronize(r.b));
      reap(r);
    }
    recs.clear();
  }
};
static Profiler g_prof;
static thread_local hipEvent_t t_pending_begin = nullptr;
static thread_local int t_prof_site = PC_OTHER;
static thread_local bool t_prof_lead = false;
static thread_local double t_prof_flops = 0.0;  // flops counted by this thread's launches
Profiler& profiler() { return g_prof; }
bool profiling() { return g_prof.on; }
ProfSite::ProfSite(int cls) : prev(t_prof_site) { t_prof_site = cls; }
ProfSite::~ProfSite() { t_prof_site = prev; }
ProfLead::ProfLead() : prev(t_prof_lead) { t_prof_lead = true; }
ProfLead::~ProfLead() { t_prof_lead = prev; }
int profile_class(int role, int rows) {
  if (role == 1) return PC_SWEEP;
  if (t_prof_lead) return PC_LEAD;
  if (rows == LU_NB) return PC_ROW64;
  return t_prof_site;
}
int profile_panel_class() { return t_prof_lead ? PC_LEAD : PC_PANEL; }
double profile_thread_flops() { return t_prof_flops; }
void profile_uncount_flops(int cls, double flops) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (g_prof.on) g_prof.cls[cls].flops_all -= flops;
}
void profile_launch_begin(hipStream_t st, int cls) {
  t_pending_begin = nullptr;
  if (!g_prof.on) return;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (!g_prof.on || !(g_prof.mask & (1u << cls))) return;
  if (g_prof.cls[cls].seen++ % g_prof.every != 0) return;  // not sampled
  t_pending_begin = g_prof.get();
  RGF_HIP(hipEventRecord(t_pending_begin, st));
}
void profile_launch_end(hipStream_t st, int cls, double flops) {
  if (!g_prof.on) return;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.cls[cls].flops_all += flops;
  ++g_prof.cls[cls].launches_all;
  t_prof_flops += flops;
  if (!t_pending_begin) return;
  hipEvent_t e = g_prof.get();
  RGF_HIP(hipEventRecord(e, st));
  g_prof.recs.push_back({t_pending_begin, e, flops, cls});
  t_pending_begin = nullptr;
  if (g_prof.recs.size() > 1024) g_prof.reap_ready();
  if (g_prof.recs.size() > 65536) g_prof.drain();  // bound the event pool
}

// ------------------------------------------------------------- tuning table
// Per (precision, padded block size class Mp/64): block-product tile and energy
// lanes; 0 = the built-in default.  Written by rgf_set_tuning / rgf_autotune,
// read by every later call.  A choice depends only on (M, precision), never on
// the batch, so results do not depend on which energies share a call.
static std::atomic<int> g_tune_tile[2][MAX_M / 64 + 1];
static std::atomic<int> g_tune_lanes[2][MAX_M / 64 + 1];
static std::atomic<int> g_tile_default[2] = {0, 0};  // 0: the built-in choice per size
static int pidx(int prec) { return prec == PREC_F64 ? 0 : 1; }
// Built-in tile: 128, except FP64 at Mp = 256, where 64 x 64 tiles measured faster on the
// production sweep (18.3 vs 19.2 ms for 392 energies of three layers, both with two lanes).
static int builtin_tile(int prec, int Mp) { return (prec == PREC_F64 && Mp == 256) ? 64 : 128; }
int tile_for(int prec, int Mp) {
  int t = g_tune_tile[pidx(prec)][std::min(Mp / 64, MAX_M / 64)].load();
  if (!t) t = g_tile_default[pidx(prec)].load();
  return t ? t : builtin_tile(prec, Mp);
}
static int g_mixed_parts = RGF_MIXED_ALL;
int mixed_parts() { return g_mixed_parts; }
static std::atomic<int> g_sr_maxit{SR_MAXIT};
int sr_maxit() { return g_sr_maxit.load(); }

// -------------------------------------------------------------- workspaces
struct Workspace {
  char* base = nullptr;
  size_t bytes = 0;
  int32_t* host_active = nullptr;
};
static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

static void drop_graphs_on(const void* base);

// One call at a time enqueues into the workspace of a (device, stream): two
// host threads calling on the same stream would otherwise share one arena
// (and a reallocation by one could free memory the other has enqueued work
// into).  The lock is held while a call enqueues its work, not until it runs;
// the stream orders the executions.
static std::mutex g_call_mu;
static std::map<std::pair<int, hipStream_t>, std::mutex> g_call_locks;
static std::mutex& stream_call_mutex(int dev, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_call_mu);
  return g_call_locks[{dev, st}];
}

static Workspace& workspace(int dev, hipStream_t st, size_t need) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  Workspace& w = g_ws[{dev, st}];
  if (!w.host_active) RGF_HIP(hipHostMalloc((void**)&w.host_active, sizeof(int32_t), hipHostMallocDefault));
  if (w.bytes < need) {
    if (w.base) {
      RGF_HIP(hipStreamSynchronize(st));
      drop_graphs_on(w.base);
      RGF_HIP(hipFree(w.base));
      w.base = nullptr;
      w.bytes = 0;
    }
    hipError_t e = hipMalloc((void**)&w.base, need);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      w.base = nullptr;
      throw Error{RGF_ENOMEM, "workspace allocation of " + std::to_string(need) + " bytes failed"};
    }
    w.bytes = need;
  }
  return w;
}

// Largest energy chunk whose workspace fits the memory budget (a `share` of it
// when several workers allocate side by side).
static int chunk_for(int Mp, int64_t nE, double share = 1.0) {
  size_t fr = 0, tot = 0;
  RGF_HIP(hipMemGetInfo(&fr, &tot));
  double frac = 0.80;
  if (const char* s = std::getenv("RGF_MEM_FRACTION")) frac = std::atof(s);
  const size_t budget = (size_t)(frac * share * (double)fr);
  const size_t per = Layout::make(Mp, 1).bytes;
  int64_t b = std::max<int64_t>(1, (int64_t)(budget / std::max<size_t>(per, 1)));
  if (const char* s = std::getenv("RGF_MAX_CHUNK")) b = std::min<int64_t>(b, std::max(1, std::atoi(s)));
  b = std::min<int64_t>(b, nE);
  b = std::min<int64_t>(b, 65535);
  return (int)b;
}

// ------------------------------------------------------------------- lanes
// Internal streams (default priority) over which one call splits its energies.
struct Lane {
  hipStream_t st = nullptr;
  hipEvent_t fork = nullptr, done = nullptr;
};
static std::mutex g_lane_mu;
static std::map<int, std::vector<Lane>> g_lanes, g_workers;

static std::mutex& lane_mutex(int dev) {
  static std::mutex mus[64];
  return mus[dev & 63];
}

static std::vector<Lane>& lane_streams(int dev, int n, bool workers = false) {
  std::lock_guard<std::mutex> lk(g_lane_mu);
  std::vector<Lane>& v = (workers ? g_workers : g_lanes)[dev];
  while ((int)v.size() < n) {
    Lane l;
    RGF_HIP(hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking));
    RGF_HIP(hipEventCreateWithFlags(&l.fork, hipEventDisableTiming));
    RGF_HIP(hipEventCreateWithFlags(&l.done, hipEventDisableTiming));
    v.push_back(l);
  }
  return v;
}

// Lanes per call: from the tuning table, else two from padded block size 256
// up (there the panel kernels, one workgroup per energy, leave half the chip
// idle), else one.  RGF_LANES overrides (1..4).
int lanes_for(int Mp, int prec) {
  int n = g_tune_lanes[pidx(prec)][std::min(Mp / 64, MAX_M / 64)].load();
  if (!n) n = Mp >= 256 ? 2 : 1;
  if (const char* s = std::getenv("RGF_LANES")) n = std::atoi(s);
  return std::max(1, std::min(n, 4));
}

// ----------------------------------------------------------- validation
static void check_lead(const rgf_lead& l, int M, const char* name) {
  RGF_CHECK(l.H00 && l.H01 && l.S00 && l.S01, RGF_EINVAL, std::string(name) + ": null block pointer");
  RGF_CHECK(l.M == M, RGF_EINVAL, std::string(name) + ": lead block size differs from the device's");
}

static void check_common(const double* E, int64_t nE, double eta, int precision, const void* out) {
  RGF_CHECK(nE >= 0, RGF_EINVAL, "nE < 0");
  RGF_CHECK(nE == 0 || (E && out), RGF_EINVAL, "null energy or output pointer");
  RGF_CHECK(std::isfinite(eta) && eta >= 0.0, RGF_EINVAL, "eta must be finite and >= 0");
  RGF_CHECK(precision == RGF_FP64 || precision == RGF_MIXED, RGF_EINVAL, "unknown precision");
}

static bool same_lead(const rgf_lead& a, const rgf_lead& b) {
  return a.H00 == b.H00 && a.H01 == b.H01 && a.S00 == b.S00 && a.S01 == b.S01;
}

void check_device(const rgf_device& d) {
  RGF_CHECK(d.N >= 1, RGF_EINVAL, "N < 1");
  RGF_CHECK(d.M >= 1 && d.M <= MAX_M, RGF_EINVAL, "M must be in [1, 2048]");
  RGF_CHECK(d.Hd && d.Sd, RGF_EINVAL, "null device block pointer");
  RGF_CHECK(d.N == 1 || (d.Hu && d.Su), RGF_EINVAL, "null coupling block pointer");
  check_lead(d.left, d.M, "left lead");
  check_lead(d.right, d.M, "right lead");
}

// ------------------------------------------------------------ input checks
static int g_checks = 0;
bool input_checks() { return g_checks != 0; }

// Hermiticity of every H_ii, S_ii (and of the electrodes' H00, S00 when `leads`), and a
// positive real diagonal of every overlap block.  Synchronous; throws RGF_EINVAL naming
// the first block that fails.  Returns max |X - X^+| / max(1, max |X|) over the blocks.
double check_inputs(const rgf_device& d, double tol, bool leads, hipStream_t st) {
  struct Arr {
    const rgf_z* p;
    int nblk;
    bool overlap;
    const char* name;
  };
  std::vector<Arr> arrs = {{d.Hd, d.N, false, "H_ii"}, {d.Sd, d.N, true, "S_ii"}};
  if (leads) {
    arrs.push_back({d.left.H00, 1, false, "left electrode H00"});
    arrs.push_back({d.left.S00, 1, true, "left electrode S00"});
    arrs.push_back({d.right.H00, 1, false, "right electrode H00"});
    arrs.push_back({d.right.S00, 1, true, "right electrode S00"});
  }
  int total = 0;
  for (const Arr& a : arrs) total += a.nblk;
  double* dev_out = nullptr;
  RGF_HIP(hipMalloc((void**)&dev_out, sizeof(double) * 4 * total));
  std::vector<double> out(4 * (size_t)total);
  int off = 0;
  for (const Arr& a : arrs) {
    launch_herm_check(reinterpret_cast<const z64*>(a.p), d.M, a.nblk, dev_out + 4 * off, st);
    off += a.nblk;
  }
  RGF_HIP(hipMemcpyAsync(out.data(), dev_out, sizeof(double) * 4 * total, hipMemcpyDeviceToHost, st));
  RGF_HIP(hipStreamSynchronize(st));
  RGF_HIP(hipFree(dev_out));
  double worst = 0.0;
  off = 0;
  for (const Arr& a : arrs) {
    for (int b = 0; b < a.nblk; ++b, ++off) {
      const double* o = out.data() + 4 * off;
      const double scale = std::max(1.0, o[1]), dev = o[0] / scale;
      worst = std::max(worst, dev);
      const std::string where = std::string(a.name) + (a.nblk > 1 ? " of layer " + std::to_string(b) : "");
      RGF_CHECK(std::isfinite(o[0]) && std::isfinite(o[1]), RGF_EINVAL, "non-finite entries in " + where);
      RGF_CHECK(dev <= tol, RGF_EINVAL, "not Hermitian: " + where + " (max |X - X^+| / max(1, max |X|) = " +
                                            std::to_string(dev) + ")");
      RGF_CHECK(!a.overlap || (o[2] > 0.0 && o[3] <= tol * scale), RGF_EINVAL,
                "overlap diagonal not real and positive: " + where);
    }
  }
  return worst;
}

bool uses_small_path(int M, int precision) {
  int small_max = SMALL_MAX_M;
  if (const char* s = std::getenv("RGF_SMALL_MAX_M")) small_max = std::min(SMALL_MAX_M, std::atoi(s));
  return M <= small_max && precision == RGF_FP64;
}

SmallArgs small_args(const rgf_device& d, const double* E, int64_t nE, double eta, double* T, int32_t* info) {
  SmallArgs a;
  a.N = d.N;
  a.M = d.M;
  a.Hd = reinterpret_cast<const z64*>(d.Hd);
  a.Hu = reinterpret_cast<const z64*>(d.Hu);
  a.Sd = reinterpret_cast<const z64*>(d.Sd);
  a.Su = reinterpret_cast<const z64*>(d.Su);
  a.LH00 = reinterpret_cast<const z64*>(d.left.H00);
  a.LH01 = reinterpret_cast<const z64*>(d.left.H01);
  a.LS00 = reinterpret_cast<const z64*>(d.left.S00);
  a.LS01 = reinterpret_cast<const z64*>(d.left.S01);
  a.RH00 = reinterpret_cast<const z64*>(d.right.H00);
  a.RH01 = reinterpret_cast<const z64*>(d.right.H01);
  a.RS00 = reinterpret_cast<const z64*>(d.right.S00);
  a.RS01 = reinterpret_cast<const z64*>(d.right.S01);
  a.same_leads = same_lead(d.left, d.right) ? 1 : 0;
  a.E = E;
  a.nE = nE;
  a.eta = eta;
  a.T = T;
  a.info = info;
  a.sr_tol = SR_TOL;
  a.sr_maxit = sr_maxit();
  a.u_l = 0.0;
  a.u_r = 0.0;
  return a;
}

// ------------------------------------------------------ captured sweeps
// With graphs on, the sweep of one energy chunk (every layer's LU panels,
// solves and block products, the final inverse and the trace) is captured
// once per (device, shape, precision, tile, workspace, stream) into a HIP
// graph and replayed on later calls.  The energies are staged into the
// workspace first and the sweep writes T and info into the workspace, so the
// captured arguments stay valid for any energies and output buffers.  The
// sweep records no memset, only kernels.  Decimation stays eager: its
// iteration count depends on the data.
// Everything the captured kernels read as an argument is part of the key: the
// block addresses, the shape, the product configuration, eta (formed into
// every operator block) and whether the two electrodes share one decimation
// (which done-flags the trace reads).
struct GraphKey {
  const void *Hd, *Hu, *Sd, *Su, *lH01, *lS01, *rH01, *rS01;
  int N, M, B, prec, parts, tile, same;
  uint64_t eta_bits;
  const void* base;
  hipStream_t st;
  bool operator<(const GraphKey& o) const {
    return std::memcmp(this, &o, sizeof(GraphKey)) < 0;
  }
};
struct GraphEntry {
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  uint64_t used = 0;
};
static std::mutex g_graph_mu;
static std::map<GraphKey, GraphEntry> g_graphs;
static uint64_t g_graph_clock = 0;
static std::atomic<int> g_graphs_on{-1};  // -1: from RGF_GRAPHS (default off)
static constexpr size_t MAX_GRAPHS = 32;

static bool graphs_enabled() {
  int v = g_graphs_on.load();
  if (v < 0) {
    const char* s = std::getenv("RGF_GRAPHS");
    v = (s && std::atoi(s) != 0) ? 1 : 0;
  }
  return v != 0 && !profiling();
}

static void drop_graph(GraphEntry& e) {
  if (e.ex) (void)hipGraphExecDestroy(e.ex);
  if (e.g) (void)hipGraphDestroy(e.g);
  e.ex = nullptr;
  e.g = nullptr;
}

// Graphs that point into a workspace about to be freed.
static void drop_graphs_on(const void* base) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto it = g_graphs.begin(); it != g_graphs.end();) {
    if (it->first.base == base) {
      drop_graph(it->second);
      it = g_graphs.erase(it);
    } else {
      ++it;
    }
  }
}

// Replay (capturing on first use) the sweep of `eng` on stream `ls`.
static void sweep_graph(Engine& eng, const rgf_device& d, bool same, double eta, int B, int prec, char* base,
                        const Layout& lay, hipStream_t ls) {
  GraphKey k;
  std::memset(&k, 0, sizeof(k));
  k.Hd = d.Hd;
  k.Hu = d.Hu;
  k.Sd = d.Sd;
  k.Su = d.Su;
  k.lH01 = d.left.H01;
  k.lS01 = d.left.S01;
  k.rH01 = d.right.H01;
  k.rS01 = d.right.S01;
  k.N = d.N;
  k.M = d.M;
  k.B = B;
  k.prec = prec;
  k.parts = mixed_parts();
  k.tile = tile_for(prec, lay.Mp);
  k.same = same ? 1 : 0;
  std::memcpy(&k.eta_bits, &eta, sizeof(double));
  k.base = base;
  k.st = ls;
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto it = g_graphs.find(k);
  if (it == g_graphs.end()) {
    if (g_graphs.size() >= MAX_GRAPHS) {  // evict the least recently used
      auto lru = g_graphs.begin();
      for (auto j = g_graphs.begin(); j != g_graphs.end(); ++j)
        if (j->second.used < lru->second.used) lru = j;
      RGF_HIP(hipStreamSynchronize(lru->first.st));
      drop_graph(lru->second);
      g_graphs.erase(lru);
    }
    GraphEntry e;
    RGF_HIP(hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal));
    try {
      eng.sweep_and_trace(d, reinterpret_cast<double*>(base + lay.tout), reinterpret_cast<int32_t*>(base + lay.iout),
                          same);
    } catch (...) {
      hipGraph_t broken = nullptr;
      (void)hipStreamEndCapture(ls, &broken);
      if (broken) (void)hipGraphDestroy(broken);
      throw;
    }
    RGF_HIP(hipStreamEndCapture(ls, &e.g));
    RGF_HIP(hipGraphInstantiate(&e.ex, e.g, nullptr, nullptr, 0));
    it = g_graphs.emplace(k, e).first;
  }
  it->second.used = ++g_graph_clock;
  RGF_HIP(hipGraphLaunch(it->second.ex, ls));
}

// One energy chunk [e0, e0 + B) of one device through the whole path on stream
// ls, in the arena `base` laid out as `lay` (lay.batch == B).
static void run_chunk(const rgf_device& d, const double* E, int64_t e0, int B, double eta, int precision,
                      double* T, int32_t* info, char* base, const Layout& lay, int32_t* host_active, bool graphs,
                      hipStream_t ls, double u_l, double u_r, const Grouping& grp, bool lookahead = true) {
  // one decimation serves both sides only for the same electrode at the same shift
  const bool same = same_lead(d.left, d.right) && u_l == u_r;
  const bool biased = u_l != 0.0 || u_r != 0.0;
  const int prec = precision == RGF_MIXED ? PREC_F32 : PREC_F64;
  const double* Ec = E + e0;
  if (graphs) {  // stage the energies at a stable address
    double* Ew = reinterpret_cast<double*>(base + lay.energies);
    RGF_HIP(hipMemcpyAsync(Ew, Ec, sizeof(double) * B, hipMemcpyDeviceToDevice, ls));
    Ec = Ew;
  }
  Engine eng(base, lay, ls, prec, d.M, Ec, eta, host_active);
  eng.set_lookahead(lookahead);
  if (grp.per > 0) eng.set_group(grp.per, e0, grp.stride);
  if (biased) {  // a rigidly shifted electrode is the unshifted one at E - u
    double* El = reinterpret_cast<double*>(base + lay.elead);
    double* Er = reinterpret_cast<double*>(base + lay.erlead);
    launch_shift(El, Ec, B, u_l, ls);
    launch_shift(Er, Ec, B, u_r, ls);
    eng.set_lead_energies(El, Er);
  }
  eng.decimate(d.left, eng.done_l(), true);
  eng.self_energy(d.left, true, eng.sigL());
  if (!same) eng.decimate(d.right, eng.done_r(), false);
  eng.self_energy(d.right, false, eng.sigR());
  eng.broadenings();
  if (graphs) {
    sweep_graph(eng, d, same, eta, B, prec, base, lay, ls);
    RGF_HIP(hipMemcpyAsync(T + e0, base + lay.tout, sizeof(double) * B, hipMemcpyDeviceToDevice, ls));
    if (info)
      RGF_HIP(hipMemcpyAsync(info + e0, base + lay.iout, sizeof(int32_t) * B, hipMemcpyDeviceToDevice, ls));
  } else {
    eng.sweep_and_trace(d, T + e0, info ? info + e0 : nullptr, same);
  }
}

// Energies [lo, hi) of one device on one stream, in chunks of at most `chunk`.
static void run_range(const rgf_device& d, const double* E, int64_t lo, int64_t hi, double eta, int precision,
                      double* T, int32_t* info, int chunk, hipStream_t ls, double u_l, double u_r,
                      const Grouping& grp) {
  const int Mp = (int)round_up(d.M, 64);
  const bool graphs = graphs_enabled() && grp.per == 0;  // a captured sweep keys on one device
  int dev = 0;
  RGF_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> call(stream_call_mutex(dev, ls));
  for (int64_t e0 = lo; e0 < hi;) {
    const int B = (int)std::min<int64_t>(chunk, hi - e0);
    const Layout lay = Layout::make(Mp, B);
    Workspace& w = workspace(dev, ls, lay.bytes);
    run_chunk(d, E, e0, B, eta, precision, T, info, w.base, lay, w.host_active, graphs, ls, u_l, u_r, grp);
    e0 += B;
  }
}

// ------------------------------------------------ allocation-free variant
// The arena of rgf_transmission_noalloc: a file-scope device array (each GPU
// holds its own copy from module load until the process ends).  Host code
// never passes the array's name to a kernel: the host-side name is a shadow,
// not a device address.  The device address is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[RGF_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[64] = {};
static int32_t g_scratch_active[64];  // the decimation's still-active count, read back by the host

static char* scratch_arena(int dev) {
  RGF_CHECK(dev >= 0 && dev < 64, RGF_EDEVICE, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    RGF_CHECK(e == hipSuccess && p, RGF_EDEVICE,
              std::string("scratch array address lookup failed: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  return g_scratch_ptr[dev];
}

// Largest energy chunk whose layout fits the scratch array (0: not even one energy).
static int noalloc_chunk(int Mp, int64_t nE) {
  const size_t per = Layout::make(Mp, 1).bytes;
  int64_t b = std::min<int64_t>(nE, (int64_t)(RGF_NOALLOC_SCRATCH_BYTES / per));
  while (b > 0 && Layout::make(Mp, (int)b).bytes > RGF_NOALLOC_SCRATCH_BYTES) --b;
  return (int)b;
}

static void transmission_noalloc_impl(const rgf_device& d, const double* E, int64_t nE, double eta, int precision,
                                      double* T, int32_t* info, hipStream_t st) {
  if (uses_small_path(d.M, precision)) {  // every block in LDS: no scratch memory at all
    launch_small(small_args(d, E, nE, eta, T, info), st);
    return;
  }
  const int Mp = (int)round_up(d.M, 64);
  const int chunk = noalloc_chunk(Mp, nE);
  RGF_CHECK(chunk >= 1, RGF_ETOOBIG,
            "rgf_transmission_noalloc: one energy at M = " + std::to_string(d.M) + " needs " +
                std::to_string(Layout::make(Mp, 1).bytes) + " bytes, more than the " +
                std::to_string((size_t)RGF_NOALLOC_SCRATCH_BYTES) + "-byte scratch array");
  int dev = 0;
  RGF_HIP(hipGetDevice(&dev));
  char* base = scratch_arena(dev);
  std::lock_guard<std::mutex> call(stream_call_mutex(dev, st));
  for (int64_t e0 = 0; e0 < nE;) {
    const int B = (int)std::min<int64_t>(chunk, nE - e0);
    // no look-ahead in the blocked LU: its side stream would be created on first use
    run_chunk(d, E, e0, B, eta, precision, T, info, base, Layout::make(Mp, B), &g_scratch_active[dev], false, st,
              0.0, 0.0, Grouping(), false);
    e0 += B;
  }
}

void run_device(const rgf_device& d, const double* E, int64_t nE, double eta, int precision, double* T,
                int32_t* info, hipStream_t st, double mem_share, double u_l, double u_r, const Grouping& grp) {
  if (nE <= 0) return;
  if (uses_small_path(d.M, precision)) {
    RGF_CHECK(grp.per == 0, RGF_EINVAL, "grouped batches need the batched path");
    SmallArgs a = small_args(d, E, nE, eta, T, info);
    a.u_l = u_l;
    a.u_r = u_r;
    launch_small(a, st);
    return;
  }
  const int Mp = (int)round_up(d.M, 64);
  run_range(d, E, 0, nE, eta, precision, T, info, chunk_for(Mp, nE, mem_share), st, u_l, u_r, grp);
}

// One device, energies [0, nE): small-block fused kernel or the batched path,
// the latter split over the energy lanes.
void transmission_impl(const rgf_device& d, const double* E, int64_t nE, double eta, int precision, double* T,
                       int32_t* info, hipStream_t st, double u_l, double u_r, const Grouping& grp) {
  const int Mp = (int)round_up(d.M, 64);
  const int prec = precision == RGF_MIXED ? PREC_F32 : PREC_F64;
  const bool small = uses_small_path(d.M, precision);
  const int nl = small ? 1 : (int)std::max<int64_t>(1, std::min<int64_t>(lanes_for(Mp, prec), nE));
  // Captured sweeps always run on library streams (a capture cannot run on the
  // caller's stream when that is the legacy default stream), so one lane then
  // also goes through the lane path.
  if (small || (nl == 1 && !graphs_enabled())) {
    run_device(d, E, nE, eta, precision, T, info, st, 1.0, u_l, u_r, grp);
    return;
  }
  int dev = 0;
  RGF_HIP(hipGetDevice(&dev));
  const int chunk = chunk_for(Mp, nE);
  // Several lanes: each takes a contiguous share of the energies on its own
  // stream, driven by its own host thread, so one lane's latency-bound steps
  // (pivot panels, decimation convergence checks) overlap the other lanes'
  // matrix-core products.  Every per-energy step is independent of the
  // other energies, so the results equal those of a single lane bitwise.
  std::vector<Lane>& lanes = lane_streams(dev, nl);
  std::lock_guard<std::mutex> lk(lane_mutex(dev));  // one multi-lane call at a time per device
  RGF_HIP(hipEventRecord(lanes[0].fork, st));
  std::vector<std::thread> th;
  std::vector<Error> errs(nl, Error{RGF_OK, ""});
  const int lane_chunk = std::max(1, chunk / nl);
  for (int i = 0; i < nl; ++i) {
    const int64_t lo = nE * i / nl, hi = nE * (i + 1) / nl;
    th.emplace_back([&, i, lo, hi] {
      try {
        RGF_HIP(hipSetDevice(dev));
        RGF_HIP(hipStreamWaitEvent(lanes[i].st, lanes[0].fork, 0));
        run_range(d, E, lo, hi, eta, precision, T, info, lane_chunk, lanes[i].st, u_l, u_r, grp);
        RGF_HIP(hipEventRecord(lanes[i].done, lanes[i].st));
      } catch (const Error& e) {
        errs[i] = e;
      } catch (const std::exception& e) {
        errs[i] = Error{RGF_EDEVICE, e.what()};
      }
    });
  }
  for (auto& t : th) t.join();
  for (int i = 0; i < nl; ++i) {
    if (errs[i].code != RGF_OK) throw errs[i];
    RGF_HIP(hipStreamWaitEvent(st, lanes[i].done, 0));
  }
}

// ------------------------------------------------------- many devices
// Job list of the persistent small-block launch, per (device, stream): the
// buffer is reused once the previous launch from it has finished.
struct JobBuf {
  void* p = nullptr;     // device copy
  void* host = nullptr;  // pinned staging of the same size
  size_t bytes = 0;
  hipEvent_t done = nullptr;
};
static std::mutex g_job_mu;
static std::map<std::pair<int, hipStream_t>, JobBuf> g_jobs;

static std::mutex& batch_mutex(int dev) {
  static std::mutex mus[64];
  return mus[dev & 63];
}

void transmission_batch_impl(const rgf_device* devs, int ndev, const double* const* E, const int64_t* nE,
                             double eta, int precision, double* const* T, int32_t* const* info, hipStream_t st) {
  int dev = 0;
  RGF_HIP(hipGetDevice(&dev));
  std::vector<int> big;
  std::vector<SmallJob> jobs;
  int64_t total = 0;
  for (int d = 0; d < ndev; ++d) {
    if (nE[d] == 0) continue;
    if (uses_small_path(devs[d].M, precision)) {
      SmallJob j;
      j.a = small_args(devs[d], E[d], nE[d], eta, T[d], info ? info[d] : nullptr);
      j.item0 = total;
      total += nE[d];
      jobs.push_back(j);
    } else {
      big.push_back(d);
    }
  }
  // ---- small blocks: one persistent launch over every (device, energy) item ----
  if (!jobs.empty()) {
    const size_t need = sizeof(SmallJob) * jobs.size() + sizeof(unsigned long long);
    std::lock_guard<std::mutex> lk(g_job_mu);
    JobBuf& jb = g_jobs[{dev, st}];
    if (!jb.done) RGF_HIP(hipEventCreateWithFlags(&jb.done, hipEventDisableTiming));
    RGF_HIP(hipEventSynchronize(jb.done));  // the previous copy and launch from these buffers are done
    if (jb.bytes < need) {
      if (jb.p) RGF_HIP(hipFree(jb.p));
      if (jb.host) RGF_HIP(hipHostFree(jb.host));
      jb.p = jb.host = nullptr;
      jb.bytes = 0;
      RGF_HIP(hipMalloc(&jb.p, need));
      RGF_HIP(hipHostMalloc(&jb.host, need, hipHostMallocDefault));
      jb.bytes = need;
    }
    char* host = static_cast<char*>(jb.host);
    std::memcpy(host, jobs.data(), sizeof(SmallJob) * jobs.size());
    std::memset(host + sizeof(SmallJob) * jobs.size(), 0, sizeof(unsigned long long));  // the work counter
    RGF_HIP(hipMemcpyAsync(jb.p, host, need, hipMemcpyHostToDevice, st));
    auto* dj = static_cast<SmallJob*>(jb.p);
    auto* counter = reinterpret_cast<unsigned long long*>(static_cast<char*>(jb.p) + sizeof(SmallJob) * jobs.size());
    const int grid = (int)std::min<int64_t>(total, 512);  // two 64 KiB-LDS workgroups per CU
    launch_small_queue(dj, (int)jobs.size(), total, counter, grid, st);
    RGF_HIP(hipEventRecord(jb.done, st));
  }
  if (big.empty()) return;
  // ---- larger blocks: the costliest device first, on worker streams ----
  std::sort(big.begin(), big.end(), [&](int a, int b) {
    const double ca = (double)devs[a].N * nE[a] * std::pow((double)round_up(devs[a].M, 64), 3.0);
    const double cb = (double)devs[b].N * nE[b] * std::pow((double)round_up(devs[b].M, 64), 3.0);
    return ca > cb || (ca == cb && a < b);
  });
  if (big.size() == 1) {
    const int d = big[0];
    transmission_impl(devs[d], E[d], nE[d], eta, precision, T[d], info ? info[d] : nullptr, st);
    return;
  }
  const int nw = 2;
  std::vector<Lane>& ws = lane_streams(dev, nw, true);
  std::lock_guard<std::mutex> lk(batch_mutex(dev));  // one multi-device call at a time per device
  RGF_HIP(hipEventRecord(ws[0].fork, st));
  std::atomic<int> next{0};
  std::vector<Error> errs(nw, Error{RGF_OK, ""});
  std::vector<std::thread> th;
  for (int w = 0; w < nw; ++w) {
    th.emplace_back([&, w] {
      try {
        RGF_HIP(hipSetDevice(dev));
        RGF_HIP(hipStreamWaitEvent(ws[w].st, ws[0].fork, 0));
        for (int i = next++; i < (int)big.size(); i = next++) {
          const int d = big[i];
          run_device(devs[d], E[d], nE[d], eta, precision, T[d], info ? info[d] : nullptr, ws[w].st, 1.0 / nw);
        }
        RGF_HIP(hipEventRecord(ws[w].done, ws[w].st));
      } catch (const Error& e) {
        errs[w] = e;
      } catch (const std::exception& e) {
        errs[w] = Error{RGF_EDEVICE, e.what()};
      }
    });
  }
  for (auto& t : th) t.join();
  for (int w = 0; w < nw; ++w) {
    if (errs[w].code != RGF_OK) throw errs[w];
    RGF_HIP(hipStreamWaitEvent(st, ws[w].done, 0));
  }
}

// LDOS: the chunk keeps N padded blocks per energy besides the usual
// workspace, so it is sized from the whole per-energy footprint.
static int64_t ldos_chunk(int Mp, int N, int64_t nE, double share) {
  size_t fr = 0, tot = 0;
  RGF_HIP(hipMemGetInfo(&fr, &tot));
  double frac = 0.80;
  if (const char* s = std::getenv("RGF_MEM_FRACTION")) frac = std::atof(s);
  const size_t per =
      Layout::make(Mp, 1).bytes + sizeof(z64) * (size_t)N * Mp * Mp + 2 * sizeof(double) + 512;
  // each lane's three shared overlap blocks
  const size_t fixed = (size_t)((double)(sizeof(z64) * 3 * (size_t)Mp * Mp) / share);
  fr = fr > fixed ? fr - fixed : 0;
  int64_t chunk = std::max<int64_t>(1, (int64_t)(frac * share * (double)fr / (double)per));
  if (const char* s = std::getenv("RGF_MAX_CHUNK")) chunk = std::min<int64_t>(chunk, std::max(1, std::atoi(s)));
  return std::min<int64_t>(std::min<int64_t>(chunk, nE), 65535);
}

// Energies [lo, hi) of the LDOS on one stream, in chunks of at most `chunk`.
static void ldos_range(const rgf_device& d, const double* E, int64_t lo, int64_t hi, double eta, double* dos,
                       double* ados_l, double* ados_r, int32_t* info, hipStream_t st, int64_t chunk) {
  const int M = d.M, N = d.N;
  const int Mp = (int)round_up(M, 64);
  const int64_t MM = (int64_t)Mp * Mp;
  const bool same = same_lead(d.left, d.right);
  int dev = 0;
  RGF_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> call(stream_call_mutex(dev, st));
  const int64_t out_per = (int64_t)N * M;
  for (int64_t e0 = lo; e0 < hi;) {
    const int B = (int)std::min<int64_t>(chunk, hi - e0);
    const Layout lay = Layout::make(Mp, B);
    const size_t store_off = round_up((int64_t)lay.bytes, 256);
    const size_t twos_off = store_off + round_up((int64_t)(sizeof(z64) * (size_t)B * N * MM), 256);
    const size_t sblk_off = twos_off + round_up((int64_t)(sizeof(double) * B), 256);
    Workspace& w = workspace(dev, st, sblk_off + sizeof(z64) * 3 * MM);
    Engine eng(w.base, lay, st, PREC_F64, M, E + e0, eta, w.host_active);
    eng.decimate(d.left, eng.done_l(), true);
    eng.self_energy(d.left, true, eng.sigL());
    if (!same) eng.decimate(d.right, eng.done_r(), false);
    eng.self_energy(d.right, false, eng.sigR());
    eng.broadenings();
    eng.local_dos(d, reinterpret_cast<z64*>(w.base + store_off), reinterpret_cast<double*>(w.base + twos_off),
                  reinterpret_cast<z64*>(w.base + sblk_off),
                  dos ? dos + e0 * out_per : nullptr, ados_l ? ados_l + e0 * out_per : nullptr,
                  ados_r ? ados_r + e0 * out_per : nullptr, info ? info + e0 : nullptr, same);
    e0 += B;
  }
}

// The LDOS energies split over the energy lanes like the transmission (each
// lane a contiguous share on its own stream and host thread); every energy is
// independent, so the results equal those of one lane bitwise.
void ldos_impl(const rgf_device& d, const double* E, int64_t nE, double eta, double* dos, double* ados_l,
               double* ados_r, int32_t* info, hipStream_t st) {
  const int Mp = (int)round_up(d.M, 64);
  const int nl = (int)std::max<int64_t>(1, std::min<int64_t>(lanes_for(Mp, PREC_F64), nE));
  if (nl == 1) {
    ldos_range(d, E, 0, nE, eta, dos, ados_l, ados_r, info, st, ldos_chunk(Mp, d.N, nE, 1.0));
    return;
  }
  int dev = 0;
  RGF_HIP(hipGetDevice(&dev));
  const int64_t chunk = ldos_chunk(Mp, d.N, (nE + nl - 1) / nl, 1.0 / nl);
  std::vector<Lane>& lanes = lane_streams(dev, nl);
  std::lock_guard<std::mutex> lk(lane_mutex(dev));
  RGF_HIP(hipEventRecord(lanes[0].fork, st));
  std::vector<std::thread> th;
  std::vector<Error> errs(nl, Error{RGF_OK, ""});
  for (int i = 0; i < nl; ++i) {
    const int64_t lo = nE * i / nl, hi = nE * (i + 1) / nl;
    th.emplace_back([&, i, lo, hi] {
      try {
        RGF_HIP(hipSetDevice(dev));
        RGF_HIP(hipStreamWaitEvent(lanes[i].st, lanes[0].fork, 0));
        ldos_range(d, E, lo, hi, eta, dos, ados_l, ados_r, info, lanes[i].st, chunk);
        RGF_HIP(hipEventRecord(lanes[i].done, lanes[i].st));
      } catch (const Error& e) {
        errs[i] = e;
      } catch (const std::exception& e) {
        errs[i] = Error{RGF_EDEVICE, e.what()};
      }
    });
  }
  for (auto& t : th) t.join();
  for (int i = 0; i < nl; ++i) {
    if (errs[i].code != RGF_OK) throw errs[i];
    RGF_HIP(hipStreamWaitEvent(st, lanes[i].done, 0));
  }
}

void self_energy_impl(const rgf_lead& lead, int side, const double* E, int64_t nE, double eta, int precision,
                      rgf_z* sigma, int32_t* info, hipStream_t st) {
  (void)precision;  // decimation and self-energies always run in FP64
  const int M = lead.M;
  const int Mp = (int)round_up(M, 64);
  int dev = 0;
  RGF_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> call(stream_call_mutex(dev, st));
  for (int64_t e0 = 0; e0 < nE;) {
    const int B = chunk_for(Mp, nE - e0);
    const Layout lay = Layout::make(Mp, B);
    Workspace& w = workspace(dev, st, lay.bytes);
    Engine eng(w.base, lay, st, PREC_F64, M, E + e0, eta, w.host_active);
    eng.decimate(lead, eng.done_l());
    z64* out = side == RGF_LEFT ? eng.sigL() : eng.sigR();
    eng.self_energy(lead, side == RGF_LEFT, out);
    eng.export_sigma(out, sigma + e0 * (int64_t)M * M);
    if (info) eng.lead_info(side == RGF_LEFT ? RGF_INFO_SR_LEFT : RGF_INFO_SR_RIGHT, eng.done_l(), info + e0);
    e0 += B;
  }
}

}  // namespace rgf

using namespace rgf;

template <class F>
static int guarded(F&& f) {
  try {
    f();
    return RGF_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return RGF_EDEVICE;
  }
}

extern "C" {

const char* rgf_last_error(void) { return g_last_error.c_str(); }
const char* rgf_version(void) { return "librgf 0.1 (gfx950)"; }

int rgf_transmission(const rgf_device* dev, const double* E, int64_t nE, double eta, int precision, double* T,
                     int32_t* info, void* stream) {
  return guarded([&] {
    RGF_CHECK(dev, RGF_EINVAL, "null device");
    check_device(*dev);
    check_common(E, nE, eta, precision, T);
    if (g_checks) check_inputs(*dev, INPUT_CHECK_TOL, true, (hipStream_t)stream);
    if (nE == 0) return;
    transmission_impl(*dev, E, nE, eta, precision, T, info, (hipStream_t)stream);
  });
}

int rgf_transmission_noalloc(const rgf_device* dev, const double* E, int64_t nE, double eta, int precision,
                             double* T, int32_t* info, void* stream) {
  return guarded([&] {
    RGF_CHECK(dev, RGF_EINVAL, "null device");
    check_device(*dev);
    check_common(E, nE, eta, precision, T);
    if (nE == 0) return;
    transmission_noalloc_impl(*dev, E, nE, eta, precision, T, info, (hipStream_t)stream);
  });
}

int rgf_transmission_bias(const rgf_device* dev, const double* E, int64_t nE, double eta, double u_left,
                          double u_right, int precision, double* T, int32_t* info, void* stream) {
  return guarded([&] {
    RGF_CHECK(dev, RGF_EINVAL, "null device");
    check_device(*dev);
    check_common(E, nE, eta, precision, T);
    RGF_CHECK(std::isfinite(u_left) && std::isfinite(u_right), RGF_EINVAL, "electrode shifts must be finite");
    if (g_checks) check_inputs(*dev, INPUT_CHECK_TOL, true, (hipStream_t)stream);
    if (nE == 0) return;
    transmission_impl(*dev, E, nE, eta, precision, T, info, (hipStream_t)stream, u_left, u_right);
  });
}

int rgf_ldos(const rgf_device* dev, const double* E, int64_t nE, double eta, double* dos, double* ados_left,
             double* ados_right, int32_t* info, void* stream) {
  return guarded([&] {
    RGF_CHECK(dev, RGF_EINVAL, "null device");
    check_device(*dev);
    RGF_CHECK(dos || ados_left || ados_right, RGF_EINVAL, "no output requested");
    check_common(E, nE, eta, RGF_FP64, dos ? dos : (ados_left ? ados_left : ados_right));
    if (g_checks) check_inputs(*dev, INPUT_CHECK_TOL, true, (hipStream_t)stream);
    if (nE == 0) return;
    ldos_impl(*dev, E, nE, eta, dos, ados_left, ados_right, info, (hipStream_t)stream);
  });
}

int rgf_landauer_current(const double* E, const double* T, int64_t nE, double mu_left, double mu_right, double kT,
                         double* I, void* stream) {
  return guarded([&] {
    RGF_CHECK(nE >= 0, RGF_EINVAL, "nE < 0");
    RGF_CHECK(I && (nE == 0 || (E && T)), RGF_EINVAL, "null energy, transmission or output pointer");
    RGF_CHECK(std::isfinite(mu_left) && std::isfinite(mu_right), RGF_EINVAL, "chemical potentials must be finite");
    RGF_CHECK(std::isfinite(kT) && kT >= 0.0, RGF_EINVAL, "kT must be finite and >= 0");
    launch_landauer(E, T, nE, mu_left, mu_right, kT, I, (hipStream_t)stream);
  });
}

int rgf_transmission_batch(const rgf_device* devs, int32_t ndev, const double* const* E, const int64_t* nE,
                           double eta, int precision, double* const* T, int32_t* const* info, void* stream) {
  return guarded([&] {
    RGF_CHECK(ndev >= 0, RGF_EINVAL, "ndev < 0");
    if (ndev == 0) return;
    RGF_CHECK(devs && E && nE && T, RGF_EINVAL, "null device, energy, count or output array");
    for (int d = 0; d < ndev; ++d) {
      check_device(devs[d]);
      check_common(E[d], nE[d], eta, precision, T[d]);
      if (g_checks) check_inputs(devs[d], INPUT_CHECK_TOL, true, (hipStream_t)stream);
    }
    transmission_batch_impl(devs, ndev, E, nE, eta, precision, T, info, (hipStream_t)stream);
  });
}

int lead_self_energy(const rgf_lead* lead, int side, const double* E, int64_t nE, double eta, int precision,
                     rgf_z* sigma, int32_t* info, void* stream) {
  return guarded([&] {
    RGF_CHECK(lead, RGF_EINVAL, "null lead");
    RGF_CHECK(lead->M >= 1 && lead->M <= MAX_M, RGF_EINVAL, "M must be in [1, 2048]");
    check_lead(*lead, lead->M, "lead");
    RGF_CHECK(side == RGF_LEFT || side == RGF_RIGHT, RGF_EINVAL, "side must be RGF_LEFT or RGF_RIGHT");
    check_common(E, nE, eta, precision, sigma);
    if (nE == 0) return;
    self_energy_impl(*lead, side, E, nE, eta, precision, sigma, info, (hipStream_t)stream);
  });
}

int rgf_release_workspaces(void) {
  return guarded([&] {
    int dev = 0;
    RGF_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto it = g_ws.begin(); it != g_ws.end();) {
      if (it->first.first == dev) {
        RGF_HIP(hipDeviceSynchronize());
        if (it->second.base) drop_graphs_on(it->second.base);
        if (it->second.base) RGF_HIP(hipFree(it->second.base));
        if (it->second.host_active) RGF_HIP(hipHostFree(it->second.host_active));
        it = g_ws.erase(it);
      } else {
        ++it;
      }
    }
    std::lock_guard<std::mutex> lj(g_job_mu);
    for (auto it = g_jobs.begin(); it != g_jobs.end();) {
      if (it->first.first == dev) {
        if (it->second.done) RGF_HIP(hipEventSynchronize(it->second.done));
        if (it->second.p) RGF_HIP(hipFree(it->second.p));
        if (it->second.host) RGF_HIP(hipHostFree(it->second.host));
        if (it->second.done) RGF_HIP(hipEventDestroy(it->second.done));
        it = g_jobs.erase(it);
      } else {
        ++it;
      }
    }
    RGF_HIP(hipDeviceSynchronize());
    release_kmesh_arenas(dev);
    release_kpm_arenas(dev);
  });
}

int rgf_profile(int every) { return rgf_profile_classes(every, 1u << RGF_PROF_SWEEP); }

int rgf_profile_classes(int every, uint32_t classes) {
  return guarded([&] {
    RGF_CHECK(every >= 0, RGF_EINVAL, "rgf_profile: negative sampling period");
    RGF_CHECK((classes & ~((1u << PC_COUNT) - 1)) == 0, RGF_EINVAL, "rgf_profile_classes: unknown class bits");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = every != 0;
    g_prof.every = every > 0 ? every : 1;
    g_prof.mask = classes;
    for (auto& c : g_prof.cls) c.seen = 0;
  });
}

int rgf_profile_read_class(int cls, int64_t* launches, double* total_ms, double* flops, int64_t* launches_all,
                           double* flops_all) {
  return guarded([&] {
    RGF_CHECK(cls >= 0 && cls < PC_COUNT, RGF_EINVAL, "rgf_profile_read_class: unknown class");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.drain();
    Profiler::Cls& c = g_prof.cls[cls];
    if (launches) *launches = c.launches;
    if (total_ms) *total_ms = c.ms;
    if (flops) *flops = c.flops;
    if (launches_all) *launches_all = c.launches_all;
    if (flops_all) *flops_all = c.flops_all;
    c = Profiler::Cls();
  });
}

int rgf_profile_read(int64_t* launches, double* total_ms, double* flops) {
  return rgf_profile_read_class(RGF_PROF_SWEEP, launches, total_ms, flops, nullptr, nullptr);
}

int rgf_set_mixed_parts(int parts) {
  return guarded([&] {
    RGF_CHECK((parts & ~RGF_MIXED_ALL) == 0, RGF_EINVAL, "unknown RGF_MIXED_* bits");
    g_mixed_parts = parts;
  });
}

int rgf_get_mixed_parts(void) { return g_mixed_parts; }

int rgf_set_sr_maxit(int32_t maxit) {
  return guarded([&] {
    RGF_CHECK(maxit >= 0 && maxit <= SR_MAXIT, RGF_EINVAL, "decimation cap must be in [0, 100]");
    g_sr_maxit = maxit ? maxit : SR_MAXIT;
  });
}

int rgf_get_sr_maxit(void) { return g_sr_maxit.load(); }

int rgf_get_tile(int precision, int32_t* tile) {
  return guarded([&] {
    RGF_CHECK(tile, RGF_EINVAL, "null tile pointer");
    RGF_CHECK(precision == RGF_FP64 || precision == RGF_MIXED, RGF_EINVAL, "unknown precision");
    const int t = g_tile_default[precision == RGF_FP64 ? 0 : 1].load();
    *tile = t ? t : 128;
  });
}

int rgf_set_tile(int precision, int32_t tile) {
  return guarded([&] {
    RGF_CHECK(precision == RGF_FP64 || precision == RGF_MIXED, RGF_EINVAL, "unknown precision");
    RGF_CHECK(tile == 64 || tile == 128, RGF_EINVAL, "tile must be 64 or 128");
    const int p = precision == RGF_FP64 ? 0 : 1;
    g_tile_default[p] = tile;
    for (auto& t : g_tune_tile[p]) t = 0;  // a global tile replaces any per-size choice
  });
}

int rgf_set_graphs(int enable) {
  return guarded([&] { g_graphs_on = enable ? 1 : 0; });
}

int rgf_get_graphs(void) { return graphs_enabled() ? 1 : 0; }

int rgf_set_checks(int enable) {
  return guarded([&] { g_checks = enable ? 1 : 0; });
}

int rgf_get_checks(void) { return g_checks; }

int rgf_check_device(const rgf_device* dev, double tol, double* max_dev, void* stream) {
  return guarded([&] {
    RGF_CHECK(dev, RGF_EINVAL, "null device");
    check_device(*dev);
    RGF_CHECK(std::isfinite(tol) && tol >= 0.0, RGF_EINVAL, "tol must be finite and >= 0");
    const double w = check_inputs(*dev, tol, true, (hipStream_t)stream);
    if (max_dev) *max_dev = w;
  });
}

int rgf_get_tuning(int32_t M, int precision, int32_t* tile, int32_t* lanes) {
  return guarded([&] {
    RGF_CHECK(M >= 1 && M <= MAX_M, RGF_EINVAL, "M must be in [1, 2048]");
    RGF_CHECK(precision == RGF_FP64 || precision == RGF_MIXED, RGF_EINVAL, "unknown precision");
    const int prec = precision == RGF_FP64 ? PREC_F64 : PREC_F32;
    const int Mp = (int)round_up(M, 64);
    if (tile) *tile = tile_for(prec, Mp);
    if (lanes) *lanes = lanes_for(Mp, prec);
  });
}

int rgf_set_tuning(int32_t M, int precision, int32_t tile, int32_t lanes) {
  return guarded([&] {
    RGF_CHECK(M >= 1 && M <= MAX_M, RGF_EINVAL, "M must be in [1, 2048]");
    RGF_CHECK(precision == RGF_FP64 || precision == RGF_MIXED, RGF_EINVAL, "unknown precision");
    RGF_CHECK(tile == 0 || tile == 64 || tile == 128, RGF_EINVAL, "tile must be 0, 64 or 128");
    RGF_CHECK(lanes >= 0 && lanes <= 4, RGF_EINVAL, "lanes must be in [0, 4]");
    const int p = precision == RGF_FP64 ? 0 : 1;
    const int k = (int)round_up(M, 64) / 64;
    g_tune_tile[p][k] = tile;
    g_tune_lanes[p][k] = lanes;
  });
}

}  // extern "C"
