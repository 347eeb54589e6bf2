// C ABI of librgf: argument checks, per-(device, stream) workspaces,
// chunking of the energy batch to the free device memory, kernel timing.
#include <algorithm>
#include <cmath>
#include <cstdlib>
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
struct Profiler {
  std::mutex mu;
  bool on = false;
  struct Rec {
    hipEvent_t a, b;
    double flops;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  int64_t launches = 0;
  double ms = 0.0, flops = 0.0;
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
  void drain() {
    for (auto& r : recs) {
      RGF_HIP(hipEventSynchronize(r.b));
      float t = 0.f;
      RGF_HIP(hipEventElapsedTime(&t, r.a, r.b));
      ms += t;
      flops += r.flops;
      ++launches;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
  }
};
static Profiler g_prof;
static thread_local hipEvent_t t_pending_begin = nullptr;
Profiler& profiler() { return g_prof; }
bool profiling() { return g_prof.on; }
void profile_launch_begin(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  t_pending_begin = g_prof.get();
  RGF_HIP(hipEventRecord(t_pending_begin, st));
}
void profile_launch_end(hipStream_t st, double flops) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  hipEvent_t e = g_prof.get();
  RGF_HIP(hipEventRecord(e, st));
  g_prof.recs.push_back({t_pending_begin, e, flops});
  if (g_prof.recs.size() > 4096) g_prof.drain();
}

// ------------------------------------------------------------- tile config
static int g_tile[2] = {128, 128};
int tile_for(int prec) { return g_tile[prec == PREC_F64 ? 0 : 1]; }
static int g_mixed_parts = RGF_MIXED_ALL;
int mixed_parts() { return g_mixed_parts; }

// -------------------------------------------------------------- workspaces
struct Workspace {
  char* base = nullptr;
  size_t bytes = 0;
  int32_t* host_active = nullptr;
};
static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

static Workspace& workspace(int dev, hipStream_t st, size_t need) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  Workspace& w = g_ws[{dev, st}];
  if (!w.host_active) RGF_HIP(hipHostMalloc((void**)&w.host_active, sizeof(int32_t), hipHostMallocDefault));
  if (w.bytes < need) {
    if (w.base) {
      RGF_HIP(hipStreamSynchronize(st));
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

// Largest energy chunk whose workspace fits the memory budget.
static int chunk_for(int Mp, int64_t nE) {
  size_t fr = 0, tot = 0;
  RGF_HIP(hipMemGetInfo(&fr, &tot));
  double frac = 0.80;
  if (const char* s = std::getenv("RGF_MEM_FRACTION")) frac = std::atof(s);
  const size_t budget = (size_t)(frac * (double)fr);
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
static std::map<int, std::vector<Lane>> g_lanes;

static std::vector<Lane>& lane_streams(int dev, int n) {
  std::lock_guard<std::mutex> lk(g_lane_mu);
  std::vector<Lane>& v = g_lanes[dev];
  while ((int)v.size() < n) {
    Lane l;
    RGF_HIP(hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking));
    RGF_HIP(hipEventCreateWithFlags(&l.fork, hipEventDisableTiming));
    RGF_HIP(hipEventCreateWithFlags(&l.done, hipEventDisableTiming));
    v.push_back(l);
  }
  return v;
}

// Lanes per call: two from padded block size 256 up (there the panel kernels,
// one workgroup per energy, leave half the chip idle), else one.  RGF_LANES
// overrides (1..4).
static int lanes_for(int Mp) {
  int n = Mp >= 256 ? 2 : 1;
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

constexpr int MAX_M = 2048;

// One device, energies [0, nE): small-block fused kernel or the batched path.
void transmission_impl(const rgf_device& d, const double* E, int64_t nE, double eta, int precision, double* T,
                       int32_t* info, hipStream_t st) {
  const int M = d.M;
  const bool same = same_lead(d.left, d.right);
  int small_max = SMALL_MAX_M;
  if (const char* s = std::getenv("RGF_SMALL_MAX_M")) small_max = std::min(SMALL_MAX_M, std::atoi(s));
  if (M <= small_max && precision == RGF_FP64) {
    SmallArgs a;
    a.N = d.N;
    a.M = M;
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
    a.same_leads = same ? 1 : 0;
    a.E = E;
    a.nE = nE;
    a.eta = eta;
    a.T = T;
    a.info = info;
    a.sr_tol = SR_TOL;
    a.sr_maxit = SR_MAXIT;
    launch_small(a, st);
    return;
  }
  const int Mp = (int)round_up(M, 64);
  int dev = 0;
  RGF_HIP(hipGetDevice(&dev));
  const int prec = precision == RGF_MIXED ? PREC_F32 : PREC_F64;
  // energies [lo, hi) of one lane, in chunks of at most `chunk`, on stream `ls`
  auto run_range = [&](int64_t lo, int64_t hi, int chunk, hipStream_t ls) {
    for (int64_t e0 = lo; e0 < hi;) {
      const int B = (int)std::min<int64_t>(chunk, hi - e0);
      const Layout lay = Layout::make(Mp, B);
      Workspace& w = workspace(dev, ls, lay.bytes);
      Engine eng(w.base, lay, ls, prec, M, E + e0, eta, w.host_active);
      eng.decimate(d.left, eng.done_l());
      eng.self_energy(d.left, true, eng.sigL());
      if (!same) eng.decimate(d.right, eng.done_r());
      eng.self_energy(d.right, false, eng.sigR());
      eng.broadenings();
      eng.sweep_and_trace(d, T + e0, info ? info + e0 : nullptr, same);
      e0 += B;
    }
  };
  const int chunk = chunk_for(Mp, nE);
  const int nl = (int)std::min<int64_t>(lanes_for(Mp), nE);
  if (nl <= 1) {
    run_range(0, nE, chunk, st);
    return;
  }
  // Several lanes: each takes a contiguous share of the energies on its own
  // stream, driven by its own host thread, so one lane's latency-bound steps
  // (pivot panels, decimation convergence checks) overlap the other lanes'
  // matrix-core products.  Every per-energy step is independent of the
  // other energies, so the results equal those of a single lane bitwise.
  std::vector<Lane>& lanes = lane_streams(dev, nl);
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
        run_range(lo, hi, lane_chunk, lanes[i].st);
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
    RGF_CHECK(dev->N >= 1, RGF_EINVAL, "N < 1");
    RGF_CHECK(dev->M >= 1 && dev->M <= MAX_M, RGF_EINVAL, "M must be in [1, 2048]");
    RGF_CHECK(dev->Hd && dev->Sd, RGF_EINVAL, "null device block pointer");
    RGF_CHECK(dev->N == 1 || (dev->Hu && dev->Su), RGF_EINVAL, "null coupling block pointer");
    check_lead(dev->left, dev->M, "left lead");
    check_lead(dev->right, dev->M, "right lead");
    check_common(E, nE, eta, precision, T);
    if (nE == 0) return;
    transmission_impl(*dev, E, nE, eta, precision, T, info, (hipStream_t)stream);
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
        if (it->second.base) RGF_HIP(hipFree(it->second.base));
        if (it->second.host_active) RGF_HIP(hipHostFree(it->second.host_active));
        it = g_ws.erase(it);
      } else {
        ++it;
      }
    }
  });
}

int rgf_profile(int enable) {
  return guarded([&] {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = enable != 0;
  });
}

int rgf_profile_read(int64_t* launches, double* total_ms, double* flops) {
  return guarded([&] {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.drain();
    if (launches) *launches = g_prof.launches;
    if (total_ms) *total_ms = g_prof.ms;
    if (flops) *flops = g_prof.flops;
    g_prof.launches = 0;
    g_prof.ms = 0.0;
    g_prof.flops = 0.0;
  });
}

int rgf_set_mixed_parts(int parts) {
  return guarded([&] {
    RGF_CHECK((parts & ~RGF_MIXED_ALL) == 0, RGF_EINVAL, "unknown RGF_MIXED_* bits");
    g_mixed_parts = parts;
  });
}

int rgf_get_mixed_parts(void) { return g_mixed_parts; }

int rgf_get_tile(int precision, int32_t* tile) {
  return guarded([&] {
    RGF_CHECK(tile, RGF_EINVAL, "null tile pointer");
    RGF_CHECK(precision == RGF_FP64 || precision == RGF_MIXED, RGF_EINVAL, "unknown precision");
    *tile = g_tile[precision == RGF_FP64 ? 0 : 1];
  });
}

int rgf_set_tile(int precision, int32_t tile) {
  return guarded([&] {
    RGF_CHECK(precision == RGF_FP64 || precision == RGF_MIXED, RGF_EINVAL, "unknown precision");
    RGF_CHECK(tile == 64 || tile == 128, RGF_EINVAL, "tile must be 64 or 128");
    g_tile[precision == RGF_FP64 ? 0 : 1] = tile;
  });
}

}  // extern "C"
