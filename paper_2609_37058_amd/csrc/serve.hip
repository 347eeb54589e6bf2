// Serving: a request loop with continuous batching and a device-resident
// cache of lead self-energies.
//
// transport_submit copies a request's host inputs into library-owned host
// staging and queues it.  max_slots worker threads each own one HIP stream
// (default priority); a free worker takes the request at the head of the
// queue as soon as the memory it needs (device blocks, energies, results
// and the engine workspace for its energy chunk) fits in what is left of
// the HBM budget, so requests that arrive while others run are admitted as
// slots and memory free up, and their kernels overlap on the device.
//
// Lead cache: Sigma_L and Sigma_R (padded Mp x Mp, FP64) per
// (lead key, side, eta, E) in slabs of device memory under
// lead_cache_bytes, evicted least-recently-used.  A request splits its
// energies into those with both self-energies cached (decimation skipped,
// Sigma copied in) and the rest (full path; their Sigma inserted after).
// An entry written on one stream carries an event that readers on other
// streams wait on; entries in use by a request are pinned.
//
// Results for an energy do not depend on the mix: every per-energy step is
// independent of the other energies in the chunk, and a cached Sigma is the
// bitwise value the same FP64 path computed.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.h"

namespace rgf {
namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct CacheKey {
  uint64_t lead, eta_bits, e_bits;
  int side;
  bool operator==(const CacheKey& o) const {
    return lead == o.lead && eta_bits == o.eta_bits && e_bits == o.e_bits && side == o.side;
  }
};
struct CacheKeyHash {
  size_t operator()(const CacheKey& k) const {
    uint64_t h = k.lead * 0x9E3779B97F4A7C15ull ^ (k.e_bits + 0x632BE59BD9B4E019ull + (k.eta_bits << 7));
    return (size_t)(h ^ (h >> 29) ^ (uint64_t)k.side);
  }
};

struct Entry {
  CacheKey key;
  int mp;
  z64* ptr;
  hipEvent_t ready;
  int pins = 0;
  std::list<Entry*>::iterator lru;
};

// Slab pool of Mp x Mp slots per padded block size.
class LeadCache {
 public:
  explicit LeadCache(uint64_t budget) : budget_(budget) {}
  ~LeadCache() {
    for (auto& kv : map_) {
      (void)hipEventDestroy(kv.second->ready);
      delete kv.second;
    }
    for (auto& s : slabs_) (void)hipFree(s.base);
  }
  std::mutex mu;
  uint64_t hits = 0, misses = 0;

  // Lookup + pin (caller holds mu).
  Entry* find(const CacheKey& k) {
    auto it = map_.find(k);
    if (it == map_.end()) return nullptr;
    Entry* e = it->second;
    lru_.splice(lru_.begin(), lru_, e->lru);
    return e;
  }
  // New entry (caller holds mu); nullptr when the budget is exhausted by pinned entries.
  Entry* insert(const CacheKey& k, int mp) {
    if (budget_ == 0) return nullptr;
    z64* p = take_slot(mp);
    if (!p) return nullptr;
    Entry* e = new Entry;
    e->key = k;
    e->mp = mp;
    e->ptr = p;
    if (hipEventCreateWithFlags(&e->ready, hipEventDisableTiming) != hipSuccess) {
      give_slot(mp, p);
      delete e;
      return nullptr;
    }
    lru_.push_front(e);
    e->lru = lru_.begin();
    map_[k] = e;
    return e;
  }
  uint64_t bytes() const { return slab_bytes_; }

 private:
  static constexpr int SLOTS_PER_SLAB = 16;
  struct Slab {
    char* base;
    int mp;
  };
  z64* take_slot(int mp) {
    auto& fl = free_[mp];
    if (fl.empty()) {
      const size_t slot = (size_t)mp * mp * sizeof(z64);
      const size_t sz = slot * SLOTS_PER_SLAB;
      if (slab_bytes_ + sz <= budget_) {
        char* base = nullptr;
        if (hipMalloc((void**)&base, sz) == hipSuccess) {
          slabs_.push_back({base, mp});
          slab_bytes_ += sz;
          for (int i = SLOTS_PER_SLAB - 1; i >= 0; --i) fl.push_back(reinterpret_cast<z64*>(base + i * slot));
        } else {
          (void)hipGetLastError();
        }
      }
    }
    if (fl.empty()) evict(mp);
    if (fl.empty()) return nullptr;
    z64* p = fl.back();
    fl.pop_back();
    return p;
  }
  void give_slot(int mp, z64* p) { free_[mp].push_back(p); }
  void evict(int mp) {
    for (auto it = lru_.rbegin(); it != lru_.rend(); ++it) {
      Entry* e = *it;
      if (e->pins == 0 && e->mp == mp) {
        (void)hipEventSynchronize(e->ready);
        (void)hipEventDestroy(e->ready);
        give_slot(mp, e->ptr);
        map_.erase(e->key);
        lru_.erase(std::next(it).base());
        delete e;
        return;
      }
    }
  }
  uint64_t budget_;
  uint64_t slab_bytes_ = 0;
  std::vector<Slab> slabs_;
  std::map<int, std::vector<z64*>> free_;
  std::list<Entry*> lru_;
  std::unordered_map<CacheKey, Entry*, CacheKeyHash> map_;
};

struct Request {
  uint64_t ticket = 0;
  int N = 0, M = 0;
  int64_t nE = 0;
  double eta = 0.0;
  int prec = RGF_FP64;
  uint64_t keyL = 0, keyR = 0;
  bool same_leads = false;
  std::vector<rgf_z> blocks;  // Hd, Sd [N], Hu, Su [N-1], left 4, right 4 (right absent if same)
  std::vector<double> E;
  std::vector<double> T;
  std::vector<int32_t> info;
  int chunk = 1;
  size_t reserve = 0;
  double t_submit = 0.0, t_done = 0.0;
  int state = 0;  // 0 queued, 1 running, 2 done, 3 failed
  int err = RGF_OK;
  std::string msg;
};

size_t block_count(int N, bool same) { return (size_t)2 * N + 2 * (size_t)std::max(N - 1, 0) + (same ? 4 : 8); }

class Server {
 public:
  Server(const rgf_server_opts& o) : cache_(o.lead_cache_bytes) {
    RGF_HIP(hipGetDevice(&dev_));
    size_t fr = 0, tot = 0;
    RGF_HIP(hipMemGetInfo(&fr, &tot));
    budget_ = o.hbm_budget_bytes ? o.hbm_budget_bytes : (uint64_t)(0.6 * (double)fr);
    const int slots = o.max_slots > 0 ? o.max_slots : 4;
    for (int i = 0; i < slots; ++i) workers_.emplace_back([this] { work(); });
  }
  ~Server() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_work_.notify_all();
    for (auto& t : workers_) t.join();
  }

  uint64_t submit(std::unique_ptr<Request> r) {
    std::lock_guard<std::mutex> lk(mu_);
    r->ticket = ++next_;
    r->t_submit = now_s();
    Request* p = r.get();
    all_[p->ticket] = std::move(r);
    queue_.push_back(p);
    cv_work_.notify_all();
    return p->ticket;
  }
  int poll(uint64_t ticket, double* T, int32_t* info, double* lat) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = all_.find(ticket);
    if (it == all_.end()) throw Error{RGF_ENOTICKET, "unknown or collected ticket"};
    Request* r = it->second.get();
    if (r->state < 2) return RGF_EAGAIN;
    if (r->state == 3) {
      Error e{r->err, r->msg};
      all_.erase(it);
      throw e;
    }
    if (T) std::memcpy(T, r->T.data(), sizeof(double) * r->nE);
    if (info) std::memcpy(info, r->info.data(), sizeof(int32_t) * r->nE);
    if (lat) *lat = r->t_done - r->t_submit;
    all_.erase(it);
    return RGF_OK;
  }
  uint64_t budget() const { return budget_; }
  void stats(rgf_server_stats* s) {
    std::lock_guard<std::mutex> lk(mu_);
    s->finished = finished_;
    s->peak_inflight_bytes = peak_;
    std::lock_guard<std::mutex> lc(cache_.mu);
    s->cache_hits = cache_.hits;
    s->cache_misses = cache_.misses;
    s->cache_bytes = cache_.bytes();
  }

 private:
  void work();
  void process(Request* r, hipStream_t st, int32_t* host_active);

  int dev_ = 0;
  uint64_t budget_ = 0;
  std::mutex mu_;
  std::condition_variable cv_work_;
  std::deque<Request*> queue_;
  std::map<uint64_t, std::unique_ptr<Request>> all_;
  uint64_t next_ = 0, inflight_ = 0, peak_ = 0, finished_ = 0;
  bool stop_ = false;
  std::vector<std::thread> workers_;
  LeadCache cache_;
};

void Server::work() {
  (void)hipSetDevice(dev_);
  hipStream_t st = nullptr;
  int32_t* host_active = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
      hipHostMalloc((void**)&host_active, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
    return;
  }
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_work_.wait(lk, [&] {
        return (stop_ && queue_.empty()) || (!queue_.empty() && inflight_ + queue_.front()->reserve <= budget_);
      });
      if (queue_.empty()) break;
      r = queue_.front();
      queue_.pop_front();
      inflight_ += r->reserve;
      peak_ = std::max(peak_, inflight_);
      r->state = 1;
    }
    int state = 2, err = RGF_OK;
    std::string msg;
    try {
      process(r, st, host_active);
    } catch (const Error& e) {
      state = 3;
      err = e.code;
      msg = e.msg;
      (void)hipStreamSynchronize(st);
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      r->t_done = now_s();
      r->err = err;
      r->msg = msg;
      r->state = state;
      inflight_ -= r->reserve;
      ++finished_;
    }
    cv_work_.notify_all();
  }
  (void)hipStreamDestroy(st);
  (void)hipHostFree(host_active);
}

struct DevBuf {
  void* p = nullptr;
  explicit DevBuf(size_t n) {
    if (n && hipMalloc(&p, n) != hipSuccess) {
      (void)hipGetLastError();
      throw Error{RGF_ENOMEM, "serving: device allocation failed"};
    }
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

void Server::process(Request* r, hipStream_t st, int32_t* host_active) {
  const int N = r->N, M = r->M;
  const int Mp = (int)round_up(M, 64);
  const size_t MMu = (size_t)M * M;
  const size_t nb = block_count(N, r->same_leads);
  DevBuf blocks(nb * MMu * sizeof(rgf_z));
  RGF_HIP(hipMemcpyAsync(blocks.p, r->blocks.data(), nb * MMu * sizeof(rgf_z), hipMemcpyHostToDevice, st));
  rgf_z* b0 = static_cast<rgf_z*>(blocks.p);
  rgf_device d;
  d.N = N;
  d.M = M;
  d.Hd = b0;
  d.Sd = b0 + N * MMu;
  d.Hu = b0 + 2 * N * MMu;
  d.Su = b0 + (2 * N + std::max(N - 1, 0)) * MMu;
  rgf_z* lp = b0 + (2 * N + 2 * std::max(N - 1, 0)) * MMu;
  d.left = rgf_lead{M, lp, lp + MMu, lp + 2 * MMu, lp + 3 * MMu};
  d.right = r->same_leads ? d.left : rgf_lead{M, lp + 4 * MMu, lp + 5 * MMu, lp + 6 * MMu, lp + 7 * MMu};

  const int B = r->chunk;
  const Layout lay = Layout::make(Mp, B);
  DevBuf ws(lay.bytes);
  DevBuf dE(sizeof(double) * B);
  DevBuf dT(sizeof(double) * B);
  DevBuf dI(sizeof(int32_t) * B);
  std::vector<double> hE(B);
  std::vector<double> hT(B);
  std::vector<int32_t> hI(B);

  // split the energies into cache hits (both sides cached) and misses
  const uint64_t eta_bits = [&] {
    uint64_t v;
    std::memcpy(&v, &r->eta, 8);
    return v;
  }();
  std::vector<int64_t> hit_idx, miss_idx;
  std::vector<Entry*> pinned;
  std::vector<std::pair<Entry*, Entry*>> hit_entries;
  {
    std::lock_guard<std::mutex> lk(cache_.mu);
    for (int64_t k = 0; k < r->nE; ++k) {
      uint64_t eb;
      std::memcpy(&eb, &r->E[k], 8);
      Entry* el = cache_.find({r->keyL, eta_bits, eb, RGF_LEFT});
      Entry* er = cache_.find({r->keyR, eta_bits, eb, RGF_RIGHT});
      if (el && er && el->mp == Mp && er->mp == Mp) {
        el->pins++;
        er->pins++;
        pinned.push_back(el);
        pinned.push_back(er);
        hit_idx.push_back(k);
        hit_entries.push_back({el, er});
        cache_.hits++;
      } else {
        miss_idx.push_back(k);
        cache_.misses++;
      }
    }
  }
  auto unpin = [&] {
    std::lock_guard<std::mutex> lk(cache_.mu);
    for (Entry* e : pinned) e->pins--;
    pinned.clear();
  };
  try {
    auto run = [&](const std::vector<int64_t>& idx, bool cached) {
      for (size_t c0 = 0; c0 < idx.size(); c0 += B) {
        const int nb_ = (int)std::min<size_t>(B, idx.size() - c0);
        for (int j = 0; j < nb_; ++j) hE[j] = r->E[idx[c0 + j]];
        RGF_HIP(hipMemcpyAsync(dE.p, hE.data(), sizeof(double) * nb_, hipMemcpyHostToDevice, st));
        Layout l2 = Layout::make(Mp, nb_);
        Engine eng(static_cast<char*>(ws.p), l2, st, r->prec == RGF_MIXED ? PREC_F32 : PREC_F64, M,
                   static_cast<double*>(dE.p), r->eta, host_active);
        if (cached) {
          for (int j = 0; j < nb_; ++j) {
            auto pr = hit_entries[c0 + j];
            RGF_HIP(hipStreamWaitEvent(st, pr.first->ready, 0));
            RGF_HIP(hipStreamWaitEvent(st, pr.second->ready, 0));
            RGF_HIP(hipMemcpyAsync(eng.sigma_slot(j, true), pr.first->ptr, sizeof(z64) * eng.block_elems(),
                                   hipMemcpyDeviceToDevice, st));
            RGF_HIP(hipMemcpyAsync(eng.sigma_slot(j, false), pr.second->ptr, sizeof(z64) * eng.block_elems(),
                                   hipMemcpyDeviceToDevice, st));
          }
          RGF_HIP(hipMemsetAsync(eng.done_l(), 0xFF, sizeof(int32_t) * 2 * nb_, st));  // decimation not run
        } else {
          eng.decimate(d.left, eng.done_l());
          eng.self_energy(d.left, true, eng.sigL());
          if (!r->same_leads) eng.decimate(d.right, eng.done_r());
          eng.self_energy(d.right, false, eng.sigR());
        }
        eng.broadenings();
        eng.sweep_and_trace(d, static_cast<double*>(dT.p), static_cast<int32_t*>(dI.p), r->same_leads);
        if (!cached) {
          // insert the new self-energies (only fully converged ones)
          RGF_HIP(hipMemcpyAsync(hI.data(), dI.p, sizeof(int32_t) * nb_, hipMemcpyDeviceToHost, st));
          RGF_HIP(hipStreamSynchronize(st));
          std::lock_guard<std::mutex> lk(cache_.mu);
          for (int j = 0; j < nb_; ++j) {
            if (hI[j] != 0) continue;
            uint64_t eb;
            std::memcpy(&eb, &hE[j], 8);
            for (int side = 0; side < 2; ++side) {
              const CacheKey key{side == 0 ? r->keyL : r->keyR, eta_bits, eb, side};
              if (cache_.find(key)) continue;
              Entry* e = cache_.insert(key, Mp);
              if (!e) continue;
              RGF_HIP(hipMemcpyAsync(e->ptr, eng.sigma_slot(j, side == 0), sizeof(z64) * eng.block_elems(),
                                     hipMemcpyDeviceToDevice, st));
              RGF_HIP(hipEventRecord(e->ready, st));
            }
          }
        }
        RGF_HIP(hipMemcpyAsync(hT.data(), dT.p, sizeof(double) * nb_, hipMemcpyDeviceToHost, st));
        RGF_HIP(hipMemcpyAsync(hI.data(), dI.p, sizeof(int32_t) * nb_, hipMemcpyDeviceToHost, st));
        RGF_HIP(hipStreamSynchronize(st));
        for (int j = 0; j < nb_; ++j) {
          r->T[idx[c0 + j]] = hT[j];
          r->info[idx[c0 + j]] = hI[j];
        }
      }
    };
    run(miss_idx, false);
    run(hit_idx, true);
  } catch (...) {
    unpin();
    throw;
  }
  unpin();
}

// Bytes one request needs on the device at once, for an energy chunk of B.
size_t request_bytes(int N, int M, bool same, int B) {
  const size_t Mp = (size_t)round_up(M, 64);
  return block_count(N, same) * (size_t)M * M * sizeof(rgf_z) + Layout::make((int)Mp, B).bytes + 24 * (size_t)B;
}

}  // namespace
}  // namespace rgf

using namespace rgf;

template <class F>
static int sguard(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return RGF_EDEVICE;
  }
}

extern "C" {

int transport_open(const rgf_server_opts* opts, void** server) {
  return sguard([&] {
    RGF_CHECK(server, RGF_EINVAL, "null server pointer");
    rgf_server_opts o{0, 0, 0};
    if (opts) o = *opts;
    RGF_CHECK(o.max_slots >= 0 && o.max_slots <= 64, RGF_EINVAL, "max_slots must be in [0, 64]");
    *server = new Server(o);
    return RGF_OK;
  });
}

int transport_submit(void* server, const rgf_device* dev, uint64_t lead_key_L, uint64_t lead_key_R, const double* E,
                     int64_t nE, double eta, int precision, uint64_t* ticket) {
  return sguard([&] {
    RGF_CHECK(server && dev && ticket, RGF_EINVAL, "null argument");
    RGF_CHECK(dev->N >= 1 && dev->M >= 1 && dev->M <= 2048, RGF_EINVAL, "N >= 1 and 1 <= M <= 2048 required");
    RGF_CHECK(nE >= 1 && E, RGF_EINVAL, "at least one energy required");
    RGF_CHECK(std::isfinite(eta) && eta >= 0.0, RGF_EINVAL, "eta must be finite and >= 0");
    RGF_CHECK(precision == RGF_FP64 || precision == RGF_MIXED, RGF_EINVAL, "unknown precision");
    RGF_CHECK(dev->Hd && dev->Sd && (dev->N == 1 || (dev->Hu && dev->Su)), RGF_EINVAL, "null device block");
    for (const rgf_lead* l : {&dev->left, &dev->right}) {
      RGF_CHECK(l->M == dev->M && l->H00 && l->H01 && l->S00 && l->S01, RGF_EINVAL, "bad lead");
    }
    Server* s = static_cast<Server*>(server);
    auto r = std::make_unique<Request>();
    r->N = dev->N;
    r->M = dev->M;
    r->nE = nE;
    r->eta = eta;
    r->prec = precision;
    r->keyL = lead_key_L;
    r->keyR = lead_key_R;
    r->same_leads = lead_key_L == lead_key_R;
    const size_t MMu = (size_t)dev->M * dev->M;
    const int N = dev->N;
    r->blocks.resize(block_count(N, r->same_leads) * MMu);
    rgf_z* p = r->blocks.data();
    auto put = [&](const rgf_z* src, size_t n) {
      std::memcpy(p, src, n * MMu * sizeof(rgf_z));
      p += n * MMu;
    };
    put(dev->Hd, N);
    put(dev->Sd, N);
    if (N > 1) {
      put(dev->Hu, N - 1);
      put(dev->Su, N - 1);
    }
    put(dev->left.H00, 1);
    put(dev->left.H01, 1);
    put(dev->left.S00, 1);
    put(dev->left.S01, 1);
    if (!r->same_leads) {
      put(dev->right.H00, 1);
      put(dev->right.H01, 1);
      put(dev->right.S00, 1);
      put(dev->right.S01, 1);
    }
    r->E.assign(E, E + nE);
    r->T.assign(nE, 0.0);
    r->info.assign(nE, 0);
    // largest energy chunk whose footprint leaves room for at least one more request
    int B = (int)std::min<int64_t>(nE, 1024);
    while (B > 1 && request_bytes(N, dev->M, r->same_leads, B) > s->budget() / 2) B = (B + 1) / 2;
    const size_t need = request_bytes(N, dev->M, r->same_leads, B);
    RGF_CHECK(need <= s->budget(), RGF_ETOOBIG, "request needs " + std::to_string(need) +
                                                    " bytes, more than the whole HBM budget");
    r->chunk = B;
    r->reserve = need;
    *ticket = s->submit(std::move(r));
    return RGF_OK;
  });
}

int transport_poll(void* server, uint64_t ticket, double* T, int32_t* info, double* latency_s) {
  return sguard([&] {
    RGF_CHECK(server, RGF_EINVAL, "null server");
    return static_cast<Server*>(server)->poll(ticket, T, info, latency_s);
  });
}

int transport_close(void* server) {
  return sguard([&] {
    delete static_cast<Server*>(server);
    return RGF_OK;
  });
}

int transport_stats(void* server, rgf_server_stats* stats) {
  return sguard([&] {
    RGF_CHECK(server && stats, RGF_EINVAL, "null argument");
    static_cast<Server*>(server)->stats(stats);
    return RGF_OK;
  });
}

}  // extern "C"
