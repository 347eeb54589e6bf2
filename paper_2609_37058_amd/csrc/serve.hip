// Serving: a request loop with continuous batching and a device-resident
// cache of lead self-energies.
//
// transport_submit copies a request's host inputs into library-owned host
// staging and queues it.  A request is ADMITTED when its device blocks fit in
// what the HBM budget leaves after the requests in flight (the workers'
// arenas are reserved up front): the queue is scanned in arrival order and
// every request that fits is admitted, so a large request at the head does
// not block smaller ones behind it -- but once the head has been passed over
// AGING_MAX times, nothing more is admitted ahead of it until it fits (no
// starvation).  An admitted request is split into WORK ITEMS of at most B
// energies (B sized so one item's engine workspace fits a worker's arena and
// its work stays bounded), separately for energies whose two self-energies
// are cached and for the rest.  max_slots worker threads, each with its own
// HIP stream (default priority) and arena, take items round-robin over the
// admitted requests: items of one request run on several workers at once,
// and a long request never holds a worker for longer than one item, so
// requests that arrive later start as soon as a worker frees up and their
// kernels overlap on the device with the others'.
//
// A request's blocks are copied to the device (stream-ordered allocation) by
// the worker that takes its first item; the others wait on that copy's
// event.  The last item to finish frees them.
//
// Lead cache: Sigma_L and Sigma_R (padded Mp x Mp, FP64) per
// (lead key, side, eta, E) in slabs of device memory under
// lead_cache_bytes, evicted least-recently-used.  An entry written on one
// stream carries an event that readers on other streams wait on; entries in
// use by a request are pinned.
//
// Results for an energy do not depend on the mix: every per-energy step is
// independent of the other energies of a work item, and a cached Sigma is the
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

struct Request;

// A work item: energies idx (positions in the request) of one request, with both
// self-energies cached (`cached`, the pinned entries in `hits`) or computed.
struct Item {
  Request* r = nullptr;
  std::vector<int64_t> idx;
  bool cached = false;
  std::vector<std::pair<Entry*, Entry*>> hits;
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
  size_t reserve = 0;  // device bytes while in flight (its blocks)
  double t_submit = 0.0, t_done = 0.0;
  int state = 0;       // 0 queued, 1 admitted, 2 done, 3 failed
  int err = RGF_OK;
  std::string msg;
  // scheduling (under the server lock)
  int bypassed = 0;            // times a later request was admitted ahead of this one
  std::deque<Item> todo;       // items not started
  int left = 0;                // items not finished
  int stage = 0;               // 0 not staged, 1 being staged, 2 staged
  std::vector<Entry*> pinned;  // cache entries pinned for the cached items
  // device copy of the blocks (valid once stage == 2; readers wait on `staged`)
  rgf_z* dblocks = nullptr;
  hipEvent_t staged = nullptr;
  rgf_device dev{};
};

size_t block_count(int N, bool same) { return (size_t)2 * N + 2 * (size_t)std::max(N - 1, 0) + (same ? 4 : 8); }

class Server {
 public:
  static constexpr int AGING_MAX = 4;  // later requests admitted ahead of the head at most this often

  Server(const rgf_server_opts& o) : cache_(o.lead_cache_bytes) {
    RGF_HIP(hipGetDevice(&dev_));
    size_t fr = 0, tot = 0;
    RGF_HIP(hipMemGetInfo(&fr, &tot));
    budget_ = o.hbm_budget_bytes ? o.hbm_budget_bytes : (uint64_t)(0.6 * (double)fr);
    slots_ = o.max_slots > 0 ? o.max_slots : 4;
    // every worker's arena is reserved up front: half of the budget over the slots (at most 16 GiB
    // each, which holds 64 energies at M = 1024)
    ws_bytes_ = std::min<uint64_t>(budget_ / (2 * (uint64_t)slots_), (uint64_t)16 << 30);
    inflight_ = ws_bytes_ * slots_;
    peak_ = inflight_;
    for (int i = 0; i < slots_; ++i) workers_.emplace_back([this] { work(); });
  }
  ~Server() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_work_.notify_all();
    for (auto& t : workers_) t.join();
  }

  uint64_t budget() const { return budget_; }
  uint64_t ws_bytes() const { return ws_bytes_; }
  // room for the blocks of requests in flight
  uint64_t block_budget() const { return budget_ > ws_bytes_ * slots_ ? budget_ - ws_bytes_ * slots_ : 0; }

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
  void stats(rgf_server_stats* s) {
    std::lock_guard<std::mutex> lk(mu_);
    s->finished = finished_;
    s->peak_inflight_bytes = peak_;
    s->admitted_ahead = ahead_;
    std::lock_guard<std::mutex> lc(cache_.mu);
    s->cache_hits = cache_.hits;
    s->cache_misses = cache_.misses;
    s->cache_bytes = cache_.bytes();
  }

 private:
  void work();
  void admit_locked();
  Item* pick_locked(Request** owner);
  void stage_blocks(Request* r, hipStream_t st);
  void run_item(Item& it, char* ws, hipStream_t st, int32_t* host_active, std::vector<double>& hT,
                std::vector<int32_t>& hI);
  void finish_item_locked(Request* r, bool failed, const Error& e, hipStream_t st);

  int dev_ = 0, slots_ = 4;
  uint64_t budget_ = 0, ws_bytes_ = 0;
  std::mutex mu_;
  std::condition_variable cv_work_;
  std::deque<Request*> queue_;   // submitted, not admitted (arrival order)
  std::vector<Request*> active_;  // admitted with items not yet started
  size_t rr_ = 0;                 // round-robin cursor over active_
  std::map<uint64_t, std::unique_ptr<Request>> all_;
  uint64_t next_ = 0, inflight_ = 0, peak_ = 0, finished_ = 0, ahead_ = 0;
  int running_ = 0;  // items being run
  bool stop_ = false;
  std::vector<std::thread> workers_;
  LeadCache cache_;
};

// Admit queued requests in arrival order while their blocks fit; the head may be passed over
// at most AGING_MAX times.  Each admitted request gets its work items (cache lookup and pins).
void Server::admit_locked() {
  const uint64_t room = block_budget();
  const uint64_t used = inflight_ - ws_bytes_ * slots_;
  uint64_t free_b = room > used ? room - used : 0;
  for (auto it = queue_.begin(); it != queue_.end();) {
    Request* r = *it;
    const bool head = it == queue_.begin();
    if (r->reserve > free_b) {
      if (head && r->bypassed >= AGING_MAX) return;  // the head waits for room
      ++it;
      continue;
    }
    if (!head) {  // admitted ahead of the waiting head: at most AGING_MAX times per head
      Request* h = queue_.front();
      if (h->bypassed >= AGING_MAX) return;
      h->bypassed++;
      ++ahead_;
    }
    free_b -= r->reserve;
    inflight_ += r->reserve;
    peak_ = std::max(peak_, inflight_);
    r->state = 1;
    // work items: cached energies (both sides, this block size) and the rest, B at a time
    const int Mp = (int)round_up(r->M, 64);
    uint64_t eta_bits;
    std::memcpy(&eta_bits, &r->eta, 8);
    std::vector<int64_t> miss;
    std::vector<std::pair<int64_t, std::pair<Entry*, Entry*>>> hit;
    {
      std::lock_guard<std::mutex> lc(cache_.mu);
      for (int64_t k = 0; k < r->nE; ++k) {
        uint64_t eb;
        std::memcpy(&eb, &r->E[k], 8);
        Entry* el = cache_.find({r->keyL, eta_bits, eb, RGF_LEFT});
        Entry* er = cache_.find({r->keyR, eta_bits, eb, RGF_RIGHT});
        if (el && er && el->mp == Mp && er->mp == Mp) {
          el->pins++;
          er->pins++;
          r->pinned.push_back(el);
          r->pinned.push_back(er);
          hit.push_back({k, {el, er}});
          cache_.hits++;
        } else {
          miss.push_back(k);
          cache_.misses++;
        }
      }
    }
    for (size_t c = 0; c < miss.size(); c += r->chunk) {
      Item w;
      w.r = r;
      w.idx.assign(miss.begin() + c, miss.begin() + std::min(miss.size(), c + r->chunk));
      r->todo.push_back(std::move(w));
    }
    for (size_t c = 0; c < hit.size(); c += r->chunk) {
      Item w;
      w.r = r;
      w.cached = true;
      for (size_t j = c; j < std::min(hit.size(), c + r->chunk); ++j) {
        w.idx.push_back(hit[j].first);
        w.hits.push_back(hit[j].second);
      }
      r->todo.push_back(std::move(w));
    }
    r->left = (int)r->todo.size();
    active_.push_back(r);
    it = queue_.erase(it);
  }
}

// The next item, round-robin over the admitted requests; a request being staged by another
// worker is skipped until its copy is enqueued.  Returns nullptr when nothing can start.
Item* Server::pick_locked(Request** owner) {
  const size_t n = active_.size();
  for (size_t k = 0; k < n; ++k) {
    const size_t i = (rr_ + k) % n;
    Request* r = active_[i];
    if (r->todo.empty() || r->stage == 1) continue;
    rr_ = (i + 1) % std::max<size_t>(1, n);
    *owner = r;
    return &r->todo.front();
  }
  return nullptr;
}

void Server::stage_blocks(Request* r, hipStream_t st) {
  const size_t MMu = (size_t)r->M * r->M;
  const size_t bytes = block_count(r->N, r->same_leads) * MMu * sizeof(rgf_z);
  void* p = nullptr;
  if (hipMallocAsync(&p, bytes, st) != hipSuccess) {
    (void)hipGetLastError();
    throw Error{RGF_ENOMEM, "serving: device allocation of the request's blocks failed"};
  }
  r->dblocks = static_cast<rgf_z*>(p);
  RGF_HIP(hipMemcpyAsync(p, r->blocks.data(), bytes, hipMemcpyHostToDevice, st));
  RGF_HIP(hipEventCreateWithFlags(&r->staged, hipEventDisableTiming));
  RGF_HIP(hipEventRecord(r->staged, st));
  const int N = r->N, M = r->M;
  rgf_z* b0 = r->dblocks;
  rgf_device& d = r->dev;
  d.N = N;
  d.M = M;
  d.Hd = b0;
  d.Sd = b0 + N * MMu;
  d.Hu = b0 + 2 * N * MMu;
  d.Su = b0 + (2 * N + std::max(N - 1, 0)) * MMu;
  rgf_z* lp = b0 + (2 * N + 2 * std::max(N - 1, 0)) * MMu;
  d.left = rgf_lead{M, lp, lp + MMu, lp + 2 * MMu, lp + 3 * MMu};
  d.right = r->same_leads ? d.left : rgf_lead{M, lp + 4 * MMu, lp + 5 * MMu, lp + 6 * MMu, lp + 7 * MMu};
}

// One work item on this worker's stream and arena (the chunk's Layout plus its staged
// energies and outputs); results land in the request's host arrays.
void Server::run_item(Item& it, char* ws, hipStream_t st, int32_t* host_active, std::vector<double>& hT,
                      std::vector<int32_t>& hI) {
  Request* r = it.r;
  const int M = r->M, Mp = (int)round_up(M, 64);
  const int nb = (int)it.idx.size();
  const Layout lay = Layout::make(Mp, nb);
  double* dE = reinterpret_cast<double*>(ws + lay.energies);
  double* dT = reinterpret_cast<double*>(ws + lay.tout);
  int32_t* dI = reinterpret_cast<int32_t*>(ws + lay.iout);
  hT.resize(nb);
  hI.resize(nb);
  std::vector<double> hE(nb);
  for (int j = 0; j < nb; ++j) hE[j] = r->E[it.idx[j]];
  RGF_HIP(hipStreamWaitEvent(st, r->staged, 0));
  RGF_HIP(hipMemcpyAsync(dE, hE.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
  Engine eng(ws, lay, st, r->prec == RGF_MIXED ? PREC_F32 : PREC_F64, M, dE, r->eta, host_active);
  const rgf_device& d = r->dev;
  if (it.cached) {
    for (int j = 0; j < nb; ++j) {
      const auto& pr = it.hits[j];
      RGF_HIP(hipStreamWaitEvent(st, pr.first->ready, 0));
      RGF_HIP(hipStreamWaitEvent(st, pr.second->ready, 0));
      RGF_HIP(hipMemcpyAsync(eng.sigma_slot(j, true), pr.first->ptr, sizeof(z64) * eng.block_elems(),
                             hipMemcpyDeviceToDevice, st));
      RGF_HIP(hipMemcpyAsync(eng.sigma_slot(j, false), pr.second->ptr, sizeof(z64) * eng.block_elems(),
                             hipMemcpyDeviceToDevice, st));
    }
    RGF_HIP(hipMemsetAsync(eng.done_l(), 0xFF, sizeof(int32_t) * 2 * nb, st));  // decimation not run
  } else {
    eng.decimate(d.left, eng.done_l());
    eng.self_energy(d.left, true, eng.sigL());
    if (!r->same_leads) eng.decimate(d.right, eng.done_r());
    eng.self_energy(d.right, false, eng.sigR());
  }
  eng.broadenings();
  eng.sweep_and_trace(d, dT, dI, r->same_leads);
  RGF_HIP(hipMemcpyAsync(hT.data(), dT, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
  RGF_HIP(hipMemcpyAsync(hI.data(), dI, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, st));
  RGF_HIP(hipStreamSynchronize(st));
  if (!it.cached) {  // insert the new self-energies (fully converged energies only)
    uint64_t eta_bits;
    std::memcpy(&eta_bits, &r->eta, 8);
    std::lock_guard<std::mutex> lk(cache_.mu);
    for (int j = 0; j < nb; ++j) {
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
    // the copies out of the arena precede, on this stream, the next item that reuses it
  }
}

// Book-keeping after an item (the worker has synchronised its stream): the last item of a
// request frees its blocks, unpins its cache entries and completes it.
void Server::finish_item_locked(Request* r, bool failed, const Error& e, hipStream_t st) {
  --running_;
  if (failed && r->state != 3) {
    r->state = 3;
    r->err = e.code;
    r->msg = e.msg;
    r->left -= (int)r->todo.size();  // items not started are dropped
    r->todo.clear();
  }
  if (--r->left > 0) return;
  if (r->dblocks) (void)hipFreeAsync(r->dblocks, st);
  r->dblocks = nullptr;
  if (r->staged) (void)hipEventDestroy(r->staged);
  r->staged = nullptr;
  {
    std::lock_guard<std::mutex> lc(cache_.mu);
    for (Entry* en : r->pinned) en->pins--;
    r->pinned.clear();
  }
  active_.erase(std::remove(active_.begin(), active_.end(), r), active_.end());
  inflight_ -= r->reserve;
  r->t_done = now_s();
  if (r->state != 3) r->state = 2;
  r->blocks.clear();
  r->blocks.shrink_to_fit();
  ++finished_;
}

void Server::work() {
  (void)hipSetDevice(dev_);
  hipStream_t st = nullptr;
  int32_t* host_active = nullptr;
  char* ws = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
      hipHostMalloc((void**)&host_active, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
    return;
  }
  std::vector<double> hT;
  std::vector<int32_t> hI;
  for (;;) {
    Item it;
    Request* r = nullptr;
    bool do_stage = false;
    {
      std::unique_lock<std::mutex> lk(mu_);
      Item* p = nullptr;
      cv_work_.wait(lk, [&] {
        admit_locked();
        p = pick_locked(&r);
        return p != nullptr || (stop_ && queue_.empty() && active_.empty());
      });
      if (!p) break;
      it = std::move(*p);
      r->todo.pop_front();
      do_stage = r->stage == 0;
      if (do_stage) r->stage = 1;
      ++running_;
    }
    bool failed = false;
    Error err{RGF_OK, ""};
    try {
      if (!ws) {
        if (hipMalloc((void**)&ws, ws_bytes_) != hipSuccess) {
          (void)hipGetLastError();
          ws = nullptr;
          throw Error{RGF_ENOMEM, "serving: worker arena allocation failed"};
        }
      }
      if (do_stage) {
        stage_blocks(r, st);
        std::lock_guard<std::mutex> lk(mu_);
        r->stage = 2;
        cv_work_.notify_all();  // its other items may start now
      }
      run_item(it, ws, st, host_active, hT, hI);
      std::lock_guard<std::mutex> lk(mu_);
      for (size_t j = 0; j < it.idx.size(); ++j) {
        r->T[it.idx[j]] = hT[j];
        r->info[it.idx[j]] = hI[j];
      }
    } catch (const Error& e) {
      failed = true;
      err = e;
      (void)hipStreamSynchronize(st);
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (failed && do_stage && r->stage == 1) r->stage = 2;  // let the remaining items drop out
      finish_item_locked(r, failed, err, st);
    }
    cv_work_.notify_all();
  }
  (void)hipStreamSynchronize(st);
  if (ws) (void)hipFree(ws);
  (void)hipStreamDestroy(st);
  (void)hipHostFree(host_active);
}

// Work-item size: the largest B (at most 128) whose engine workspace fits a worker's arena.
int item_energies(int M, int64_t nE, uint64_t ws_bytes) {
  const int Mp = (int)round_up(M, 64);
  int B = (int)std::min<int64_t>(nE, 128);
  while (B > 0 && Layout::make(Mp, B).bytes > ws_bytes) B = B > 8 ? B * 3 / 4 : B - 1;
  return B;
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
    // work items of B energies fit a worker's arena; the blocks must fit what the arenas leave
    const int B = item_energies(dev->M, nE, s->ws_bytes());
    const size_t need = block_count(N, r->same_leads) * MMu * sizeof(rgf_z);
    RGF_CHECK(B >= 1, RGF_ETOOBIG, "one energy's workspace at M = " + std::to_string(dev->M) +
                                       " exceeds a worker's share of the HBM budget");
    RGF_CHECK(need <= s->block_budget(), RGF_ETOOBIG,
              "request needs " + std::to_string(need) + " bytes of blocks, more than the HBM budget leaves");
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
