// Transverse k-point sampling: the devices of the paper are periodic across
// the transport direction and their transmission is sampled on transverse
// k-point meshes (the per-stage cost is per energy and per transverse
// k-point).  Every block is given for a set of transverse lattice images R;
// at the fractional wavevector k each block is X(k) = sum_R X(R)
// exp(2 pi i k.R) (one HBM-bound Bloch-sum kernel per block array).  The
// assembled devices of a group of k-points sit at one stride in memory and
// all have the shape (N, M), so their energies run as one grouped batch of
// the batched path (k-points x energies fill the chip even at a few
// energies); blocks small enough for the fused small-block kernel go through
// the multi-device batch instead.  T(E) = sum_k w_k T_k(E) is accumulated in
// mesh order.
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "engine.h"

namespace rgf {

void transmission_batch_impl(const rgf_device* devs, int ndev, const double* const* E, const int64_t* nE,
                             double eta, int precision, double* const* T, int32_t* const* info, hipStream_t st);

namespace {

// Assembled k-devices, per (device, stream); reused once the previous call's work is done.
struct KArena {
  char* p = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
};
std::mutex g_kmu;
std::map<std::pair<int, hipStream_t>, KArena> g_karena;

bool same_ptrs(const rgf_lead& a, const rgf_lead& b) {
  return a.H00 == b.H00 && a.H01 == b.H01 && a.S00 == b.S00 && a.S01 == b.S01;
}

}  // namespace

void release_kmesh_arenas(int dev) {
  std::lock_guard<std::mutex> lk(g_kmu);
  for (auto it = g_karena.begin(); it != g_karena.end();) {
    if (it->first.first == dev) {
      if (it->second.done) RGF_HIP(hipEventDestroy(it->second.done));
      if (it->second.p) RGF_HIP(hipFree(it->second.p));
      it = g_karena.erase(it);
    } else {
      ++it;
    }
  }
}

}  // namespace rgf

using namespace rgf;

extern "C" int rgf_transmission_kmesh(const rgf_device* images, int32_t nR, const int32_t* R, const double* kpts,
                                      const double* weights, int32_t nk, const double* E, int64_t nE, double eta,
                                      int precision, double* T, double* Tk, int32_t* info, void* stream) {
  try {
    RGF_CHECK(images && R && kpts && weights, RGF_EINVAL, "null image, lattice, k-point or weight array");
    RGF_CHECK(nR >= 1 && nR <= MAX_IMAGES, RGF_EINVAL, "nR must be in [1, 32]");
    RGF_CHECK(nk >= 1, RGF_EINVAL, "nk < 1");
    RGF_CHECK(nE >= 0, RGF_EINVAL, "nE < 0");
    RGF_CHECK(nE == 0 || (E && T), RGF_EINVAL, "null energy or output pointer");
    RGF_CHECK(std::isfinite(eta) && eta >= 0.0, RGF_EINVAL, "eta must be finite and >= 0");
    RGF_CHECK(precision == RGF_FP64 || precision == RGF_MIXED, RGF_EINVAL, "unknown precision");
    const int N = images[0].N, M = images[0].M;
    RGF_CHECK(N >= 1 && M >= 1 && M <= MAX_M, RGF_EINVAL, "N < 1 or M outside [1, 2048]");
    bool shared_leads = true;
    for (int r = 0; r < nR; ++r) {
      RGF_CHECK(images[r].N == N && images[r].M == M, RGF_EINVAL, "images differ in N or M");
      shared_leads = shared_leads && same_ptrs(images[r].left, images[r].right);
    }
    bool any_lead = false;
    for (int r = 0; r < nR; ++r) any_lead = any_lead || images[r].left.H00 || images[r].left.S00;
    RGF_CHECK(any_lead, RGF_EINVAL, "no image has electrode blocks");
    if (nE == 0) return RGF_OK;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    RGF_HIP(hipGetDevice(&dev));

    // ---- sizes: one assembled device per k-point of a group ----
    const int64_t MM = (int64_t)M * M;
    const int64_t nd = (int64_t)N * MM, nu = (int64_t)std::max(N - 1, 0) * MM;
    const int64_t per_k = 2 * nd + 2 * nu + (shared_leads ? 4 : 8) * MM;  // complex elements
    size_t fr = 0, tot = 0;
    RGF_HIP(hipMemGetInfo(&fr, &tot));
    const size_t per_k_bytes = sizeof(z64) * per_k + (2 * sizeof(double) + sizeof(int32_t)) * nE + 1024;
    int G = (int)std::max<int64_t>(1, std::min<int64_t>(nk, (int64_t)(0.2 * (double)fr / (double)per_k_bytes)));
    G = std::min(G, 64);
    const size_t need = (size_t)G * per_k_bytes + (Tk ? 0 : sizeof(double) * nE * nk) + 4096;

    std::lock_guard<std::mutex> lk(g_kmu);
    KArena& ka = g_karena[{dev, st}];
    if (!ka.done) RGF_HIP(hipEventCreateWithFlags(&ka.done, hipEventDisableTiming));
    RGF_HIP(hipEventSynchronize(ka.done));
    if (ka.bytes < need) {
      if (ka.p) RGF_HIP(hipFree(ka.p));
      ka.p = nullptr;
      ka.bytes = 0;
      RGF_HIP(hipMalloc((void**)&ka.p, need));
      ka.bytes = need;
    }
    char* cursor = ka.p;
    auto take = [&](size_t n) {
      char* q = cursor;
      cursor += (n + 255) / 256 * 256;
      return q;
    };
    std::vector<z64*> slots(G);
    for (int g = 0; g < G; ++g) slots[g] = reinterpret_cast<z64*>(take(sizeof(z64) * per_k));
    const int64_t stride = round_up((int64_t)sizeof(z64) * per_k, 256) / (int64_t)sizeof(z64);
    double* Tk_rows = Tk ? Tk : reinterpret_cast<double*>(take(sizeof(double) * nE * nk));
    const bool grouped = !uses_small_path(M, precision) && nE <= (1 << 30);
    double* Eall = nullptr;  // the energies once per k-point of a group
    if (grouped) {
      Eall = reinterpret_cast<double*>(take(sizeof(double) * nE * G));
      for (int g = 0; g < G; ++g)
        RGF_HIP(hipMemcpyAsync(Eall + (int64_t)g * nE, E, sizeof(double) * nE, hipMemcpyDeviceToDevice, st));
    }

    for (int k0 = 0; k0 < nk; k0 += G) {
      const int gn = std::min(G, nk - k0);
      std::vector<rgf_device> kdev(gn);
      std::vector<const double*> Es(gn, E);
      std::vector<int64_t> counts(gn, nE);
      std::vector<double*> Ts(gn);
      std::vector<int32_t*> Is(gn);
      for (int g = 0; g < gn; ++g) {
        const int k = k0 + g;
        BlochArgs b;
        b.nR = nR;
        for (int r = 0; r < nR; ++r) {
          const double ph = 6.283185307179586476925 * (kpts[2 * k] * R[2 * r] + kpts[2 * k + 1] * R[2 * r + 1]);
          b.w[r] = zmake(std::cos(ph), std::sin(ph));
        }
        z64* base = slots[g];
        auto assemble = [&](z64* dst, int64_t n, auto get) {
          for (int r = 0; r < nR; ++r) b.src[r] = reinterpret_cast<const z64*>(get(images[r]));
          b.dst = dst;
          b.n = n;
          launch_bloch(b, st);
          return reinterpret_cast<rgf_z*>(dst);
        };
        rgf_device& d = kdev[g];
        d.N = N;
        d.M = M;
        z64* q = base;
        d.Hd = assemble(q, nd, [](const rgf_device& x) { return x.Hd; });
        q += nd;
        d.Sd = assemble(q, nd, [](const rgf_device& x) { return x.Sd; });
        q += nd;
        d.Hu = N > 1 ? assemble(q, nu, [](const rgf_device& x) { return x.Hu; }) : nullptr;
        q += nu;
        d.Su = N > 1 ? assemble(q, nu, [](const rgf_device& x) { return x.Su; }) : nullptr;
        q += nu;
        auto lead = [&](bool left) {
          rgf_lead l;
          l.M = M;
          l.H00 = assemble(q, MM, [left](const rgf_device& x) { return (left ? x.left : x.right).H00; });
          q += MM;
          l.H01 = assemble(q, MM, [left](const rgf_device& x) { return (left ? x.left : x.right).H01; });
          q += MM;
          l.S00 = assemble(q, MM, [left](const rgf_device& x) { return (left ? x.left : x.right).S00; });
          q += MM;
          l.S01 = assemble(q, MM, [left](const rgf_device& x) { return (left ? x.left : x.right).S01; });
          q += MM;
          return l;
        };
        d.left = lead(true);
        d.right = shared_leads ? d.left : lead(false);
        Ts[g] = Tk_rows + (int64_t)k * nE;
        Is[g] = info ? info + (int64_t)k * nE : nullptr;
      }
      if (grouped) {
        Grouping grp;
        grp.per = (int)nE;
        grp.stride = stride;
        transmission_impl(kdev[0], Eall, (int64_t)gn * nE, eta, precision, Ts[0], info ? Is[0] : nullptr, st,
                          0.0, 0.0, grp);
      } else {
        transmission_batch_impl(kdev.data(), gn, Es.data(), counts.data(), eta, precision, Ts.data(),
                                info ? Is.data() : nullptr, st);
      }
      for (int g = 0; g < gn; ++g) launch_kaccum(T, Tk_rows + (int64_t)(k0 + g) * nE, weights[k0 + g], nE, k0 + g == 0, st);
    }
    RGF_HIP(hipEventRecord(ka.done, st));
    return RGF_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return RGF_EDEVICE;
  }
}
