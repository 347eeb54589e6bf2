// Tile and lane autotuner: picks, for one (block size class, precision), the
// block-product tile (64 or 128) and the number of energy lanes (1 or 2) by
// timing the production sweep -- the layer recursion with its LU panels,
// triangular solves and block products, and the final inverse and trace --
// on a synthetic device of three random layers at that block size.  The
// winner goes into the tuning table that every later call consults; a choice
// depends only on (M, precision), so results stay independent of the batch.
#include <memory>
#include <thread>
#include <vector>

#include "engine.h"

namespace rgf {
namespace {

// device buffers released on scope exit
struct DevBuf {
  void* p = nullptr;
  explicit DevBuf(size_t bytes) { RGF_HIP(hipMalloc(&p, bytes)); }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

struct Streams {
  hipStream_t s[2] = {nullptr, nullptr};
  Streams() {
    for (auto& x : s) RGF_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
  }
  ~Streams() {
    for (auto& x : s)
      if (x) (void)hipStreamDestroy(x);
  }
};

// Three random layers at block size M (S = I + small, couplings damped), one
// lead equal to the first layer; energies uniform in [-1, 1).
struct Synthetic {
  static constexpr int N = 3;
  int M;
  DevBuf Hd, Hu, Sd, Su, E;
  rgf_device dev{};
  Synthetic(int M_, int batch, hipStream_t st)
      : M(M_),
        Hd(sizeof(z64) * N * M_ * M_),
        Hu(sizeof(z64) * (N - 1) * M_ * M_),
        Sd(sizeof(z64) * N * M_ * M_),
        Su(sizeof(z64) * (N - 1) * M_ * M_),
        E(sizeof(z64) * ((batch + 1) / 2)) {
    const int64_t MM = (int64_t)M * M;
    launch_random(Hd.as<z64>(), N * MM, M, M, 1.0, 0.0, 11, st);
    launch_random(Hu.as<z64>(), (N - 1) * MM, M, M, 0.5, 0.0, 12, st);
    launch_random(Sd.as<z64>(), N * MM, M, M, 0.05, 1.0, 13, st);
    launch_random(Su.as<z64>(), (N - 1) * MM, M, M, 0.02, 0.0, 14, st);
    launch_random(E.as<z64>(), (batch + 1) / 2, 1, 1, 1.0, 0.0, 15, st);  // read as `batch` doubles
    dev.N = N;
    dev.M = M;
    dev.Hd = Hd.as<rgf_z>();
    dev.Hu = Hu.as<rgf_z>();
    dev.Sd = Sd.as<rgf_z>();
    dev.Su = Su.as<rgf_z>();
    const rgf_lead l{M, dev.Hd, dev.Hu, dev.Sd, dev.Su};
    dev.left = l;
    dev.right = l;
  }
  const double* energies() const { return E.as<double>(); }
};

// One sweep of the energies [E, E + lay.batch) on `st`, self-energies set to zero.
void sweep_once(const Synthetic& syn, char* arena, const Layout& lay, int prec, const double* E, double* T,
                int32_t* host_active, hipStream_t st) {
  Engine eng(arena, lay, st, prec, syn.M, E, 1e-6, host_active);
  const int64_t U = (int64_t)lay.batch * lay.Mp * lay.Mp;
  RGF_HIP(hipMemsetAsync(eng.sigL(), 0, sizeof(z64) * U, st));
  RGF_HIP(hipMemsetAsync(eng.sigR(), 0, sizeof(z64) * U, st));
  eng.broadenings();
  eng.sweep_and_trace(syn.dev, T, nullptr, true);
}

}  // namespace
}  // namespace rgf

using namespace rgf;

extern "C" int rgf_autotune(int32_t M, int precision, int32_t batch, int32_t* tile_out, int32_t* lanes_out,
                            double* ms_out) {
  int32_t old_tile = 0, old_lanes = 0;
  bool touched = false;
  try {
    RGF_CHECK(M >= 1 && M <= MAX_M, RGF_EINVAL, "M must be in [1, 2048]");
    RGF_CHECK(precision == RGF_FP64 || precision == RGF_MIXED, RGF_EINVAL, "unknown precision");
    RGF_CHECK(batch >= 0, RGF_EINVAL, "batch < 0");
    const int prec = precision == RGF_MIXED ? PREC_F32 : PREC_F64;
    const int Mp = (int)round_up(M, 64);
    if (batch == 0) batch = 64;
    // the three workspaces (one batch, two halves) take at most 40% of free memory
    size_t fr = 0, tot = 0;
    RGF_HIP(hipMemGetInfo(&fr, &tot));
    const size_t per = Layout::make(Mp, 1).bytes;
    batch = (int)std::max<int64_t>(1, std::min<int64_t>(batch, (int64_t)(0.4 * (double)fr / (2.0 * per))));
    RGF_CHECK(rgf_get_tuning(M, precision, &old_tile, &old_lanes) == RGF_OK, RGF_EDEVICE, "tuning table");
    int dev = 0;
    RGF_HIP(hipGetDevice(&dev));

    Streams st;
    Synthetic syn(M, batch, st.s[0]);
    const int half = std::max(1, batch / 2);
    const Layout lay1 = Layout::make(Mp, batch), lay2 = Layout::make(Mp, half);
    DevBuf w1(lay1.bytes), w2a(lay2.bytes), w2b(lay2.bytes), T(sizeof(double) * batch);
    int32_t* host_active = nullptr;
    RGF_HIP(hipHostMalloc((void**)&host_active, 2 * sizeof(int32_t), hipHostMallocDefault));
    std::unique_ptr<int32_t, void (*)(int32_t*)> ha(host_active, [](int32_t* p) { (void)hipHostFree(p); });
    RGF_HIP(hipStreamSynchronize(st.s[0]));

    const int tiles[2] = {64, 128};
    double best = 1e300;
    int best_tile = 128, best_lanes = 1;
    hipEvent_t e0, e1;
    RGF_HIP(hipEventCreate(&e0));
    RGF_HIP(hipEventCreate(&e1));
    int k = 0;
    for (int ti = 0; ti < 2; ++ti) {
      for (int lanes = 1; lanes <= 2; ++lanes, ++k) {
        double ms = -1.0;
        if (lanes == 1 || batch >= 2) {
          touched = true;
          RGF_CHECK(rgf_set_tuning(M, precision, tiles[ti], lanes) == RGF_OK, RGF_EDEVICE, "tuning table");
          auto run = [&] {
            if (lanes == 1) {
              sweep_once(syn, w1.as<char>(), lay1, prec, syn.energies(), T.as<double>(), host_active, st.s[0]);
            } else {
              Error err{RGF_OK, ""};
              std::thread other([&] {
                try {
                  RGF_HIP(hipSetDevice(dev));
                  sweep_once(syn, w2b.as<char>(), lay2, prec, syn.energies() + half, T.as<double>() + half,
                             host_active + 1, st.s[1]);
                } catch (const Error& e) {
                  err = e;
                }
              });
              sweep_once(syn, w2a.as<char>(), lay2, prec, syn.energies(), T.as<double>(), host_active, st.s[0]);
              other.join();
              if (err.code != RGF_OK) throw err;
            }
            RGF_HIP(hipDeviceSynchronize());
          };
          run();  // warm-up: code objects and caches
          const int reps = 2;
          RGF_HIP(hipEventRecord(e0, st.s[0]));
          for (int r = 0; r < reps; ++r) run();
          RGF_HIP(hipEventRecord(e1, st.s[0]));
          RGF_HIP(hipEventSynchronize(e1));
          float t = 0.f;
          RGF_HIP(hipEventElapsedTime(&t, e0, e1));
          ms = t / reps;
          if (ms < best) {
            best = ms;
            best_tile = tiles[ti];
            best_lanes = lanes;
          }
        }
        if (ms_out) ms_out[k] = ms;
      }
    }
    RGF_HIP(hipEventDestroy(e0));
    RGF_HIP(hipEventDestroy(e1));
    RGF_CHECK(rgf_set_tuning(M, precision, best_tile, best_lanes) == RGF_OK, RGF_EDEVICE, "tuning table");
    if (tile_out) *tile_out = best_tile;
    if (lanes_out) *lanes_out = best_lanes;
    return RGF_OK;
  } catch (const Error& e) {
    if (touched) (void)rgf_set_tuning(M, precision, 0, 0);  // back to the defaults
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    if (touched) (void)rgf_set_tuning(M, precision, 0, 0);
    set_error(e.what());
    return RGF_EDEVICE;
  }
}
