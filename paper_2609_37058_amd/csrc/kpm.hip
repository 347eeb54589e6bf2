// Nonorthogonal kernel polynomial method for the Fermi level of the central
// region (paper: Introduction and Results -- Chebyshev moments of
// S^-1 (H - b S) / a from random vectors, S applied through linear solves,
// the Fermi level from the electron-number constraint, at O(N_mom N_rand N)).
//
// Moments: with R random vectors r (columns), A~ = S^-1 (H - b S) / a,
//   v_0 = r, v_1 = A~ r, v_{n+1} = 2 A~ v_n - v_{n-1},  mu_n = Re sum r^+ v_n / R.
// One Chebyshev step on the GPU, with V [N][Mp][Rp] (layer-major, the R
// columns padded to Rp):
//   W = c (H - b S) V / a        three batched products over the layers (the
//                                diagonal, upper and lower blocks of b S - H,
//                                written once per call, one block per batch entry)
//   W <- S^-1 W                  block-Thomas solve with the factors of S:
//                                forward  Z_i = W_i - Lf_i Z_{i-1},
//                                then     X = Dinv Z (one batched product),
//                                back     X_i = X_i - Uf_i X_{i+1},
//                                each sweep step split over chunks of its
//                                inner dimension (partial products in one
//                                launch, then a fixed-order sum),
//                                with D_0 = S_00, D_i = S_ii - S_{i,i-1} Uf_{i-1},
//                                Dinv_i = D_i^-1, Uf_i = D_i^-1 S_{i,i+1},
//                                Lf_i = S_{i,i-1} D_{i-1}^-1 (factored once per call)
//   v_{n+1} = X - v_{n-1}        (c = 2; c = 1 and no subtraction for v_1), fused
//                                with the per-block partial sums of r^+ v_{n+1}
// The sweeps of the solve are sequential over the layers (one product of an
// M x M factor with an M x R panel each), the rest is batched over layers.
// Every sum runs in a fixed order, so the moments do not depend on the launch.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "engine.h"

namespace rgf {

namespace {

constexpr double KPM_EPS = 0.01;  // a = (e_max - e_min) / (2 - eps)
constexpr int DOT_BLOCKS = 1024;
constexpr int KPM_TILE = 64;      // skinny M x R products: 64 x 64 output tiles

__global__ void kpm_fill_kernel(double* p, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// dst[l][m][c] = src[(l M + m) R + c] (zero padding to Mp x Rp)
__global__ void kpm_pad_kernel(const z64* src, z64* dst, int N, int M, int R, int Mp, int Rp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)N * Mp * Rp;
  if (i >= total) return;
  const int c = (int)(i % Rp);
  const int m = (int)((i / Rp) % Mp);
  const int l = (int)(i / ((int64_t)Rp * Mp));
  dst[i] = (m < M && c < R) ? src[((int64_t)l * M + m) * R + c] : zmake(0.0, 0.0);
}

// x <- x - prev (prev may be null), partial[block] = sum of conj(r) x over the block's elements
__global__ void __launch_bounds__(256) kpm_next_kernel(z64* x, const z64* prev, const z64* r, int64_t n,
                                                       double* partial) {
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    z64 v = x[i];
    if (prev) {
      const z64 p = prev[i];
      v = zmake(v.x - p.x, v.y - p.y);
      x[i] = v;
    }
    const z64 q = r[i];
    acc += q.x * v.x + q.y * v.y;  // Re(conj(r) v)
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) kpm_moment_kernel(const double* partial, int nblk, double inv_r, double* mu) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *mu = red[0] * inv_r;
}

// C[i] -= sum_c partial[c][i], c = 0..nc-1 in order (the split-K partial products of a sweep step)
__global__ void kpm_ksum_kernel(z64* C, const z64* partial, int nc, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < nc; ++c) {
    const z64 p = partial[(int64_t)c * n + i];
    re += p.x;
    im += p.y;
  }
  const z64 v = C[i];
  C[i] = zmake(v.x - re, v.y - im);
}

__device__ inline double jackson_g(int n, int N) {
  const double q = 3.14159265358979323846 / (N + 1);
  return ((N - n + 1) * cos(q * n) + sin(q * n) * cos(q) / sin(q)) / (N + 1);
}

// N(x) = g_0 mu_0 (pi - th) / pi - (2/pi) sum_{n>=1} g_n mu_n sin(n th) / n, th = acos x;
// one workgroup, fixed-order reduction; every thread returns the total
__device__ double states_below(const double* mu, int nm, double x, double* red) {
  const double pi = 3.14159265358979323846;
  const double th = acos(fmin(1.0, fmax(-1.0, x)));
  double acc = 0.0;
  for (int n = 1 + threadIdx.x; n < nm; n += blockDim.x) acc += jackson_g(n, nm) * mu[n] * sin(n * th) / n;
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double total = jackson_g(0, nm) * mu[0] * (pi - th) / pi - (2.0 / pi) * red[0];
  __syncthreads();
  return total;
}

__global__ void __launch_bounds__(256) kpm_fermi_kernel(const double* mu, int nm, double a, double b,
                                                        double n_states, double* ef) {
  __shared__ double red[256];
  double lo = -1.0, hi = 1.0;
  for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (states_below(mu, nm, mid, red) < n_states)
      lo = mid;
    else
      hi = mid;
  }
  if (threadIdx.x == 0) *ef = a * 0.5 * (lo + hi) + b;
}

// rho(E) = [g_0 mu_0 + 2 sum g_n mu_n T_n(x)] / (pi sqrt(1 - x^2) a); one thread per energy
__global__ void kpm_dos_kernel(const double* mu, int nm, double a, double b, const double* E, int64_t nE,
                               double* out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nE) return;
  const double x = (E[k] - b) / a;
  const double th = acos(fmin(1.0, fmax(-1.0, x)));
  double s = jackson_g(0, nm) * mu[0];
  for (int n = 1; n < nm; ++n) s += 2.0 * jackson_g(n, nm) * mu[n] * cos(n * th);
  out[k] = s / (3.14159265358979323846 * sqrt(fmax(1.0 - x * x, 1e-300)) * a);
}

// the Chebyshev step's products, timed per launch when profiling is on
void timed_gemm(const GemmArgs& g, hipStream_t st) { launch_gemm(g, PREC_F64, KPM_TILE, st, 1); }

// Chunks of the inner dimension for a sweep step: enough (Mp/64 x Rp/64 x nc)
// workgroups to fill the chip, nc dividing Mp / 16.
int ksplit(int Mp, int Rp) {
  const int tiles = (Mp / 64) * (Rp / 64);
  int nc = std::min(Mp / 16, std::max(1, 256 / tiles));
  while ((Mp / 16) % nc) --nc;
  return nc;
}

// One step of a solve sweep, C = C - A B (A: Mp x Mp, B, C: Mp x Rp panels), as
// nc partial products over chunks of the inner dimension (one batched launch,
// so a single sequential step still spreads over the chip) and a fixed-order sum.
void sweep_step(const z64* A, const z64* Bp, z64* Cp, z64* partial, int Mp, int Rp, hipStream_t st) {
  const int nc = ksplit(Mp, Rp);
  const int kc = Mp / nc;
  GemmArgs g = gemm_args(Mp, Rp, kc, nc);
  g.A = mat(const_cast<z64*>(A), kc, Mp);
  g.B = mat(const_cast<z64*>(Bp), (int64_t)kc * Rp, Rp);
  g.C = mat(partial, (int64_t)Mp * Rp, Rp);
  timed_gemm(g, st);
  const int64_t n = (int64_t)Mp * Rp;
  hipLaunchKernelGGL(kpm_ksum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Cp, partial, nc, n);
  RGF_HIP(hipGetLastError());
}

struct KpmArena {
  char* p = nullptr;
  size_t bytes = 0;
};
std::mutex g_kpm_mu;
std::map<std::pair<int, hipStream_t>, KpmArena> g_kpm;

}  // namespace

void release_kpm_arenas(int dev) {
  std::lock_guard<std::mutex> lk(g_kpm_mu);
  for (auto it = g_kpm.begin(); it != g_kpm.end();) {
    if (it->first.first == dev) {
      if (it->second.p) RGF_HIP(hipFree(it->second.p));
      it = g_kpm.erase(it);
    } else {
      ++it;
    }
  }
}

// Moments of one central region (blocks of `d`; its electrodes are not used).
void kpm_moments_impl(const rgf_device& d, double e_min, double e_max, int n_mom, const rgf_z* vectors, int R,
                      double* mu, hipStream_t st) {
  const int N = d.N, M = d.M;
  const int Mp = (int)round_up(M, 64), Rp = (int)round_up(R, 64);
  const int64_t MM = (int64_t)Mp * Mp, M2 = (int64_t)M * M;
  const int64_t VB = (int64_t)Mp * Rp;  // one layer of a vector panel
  const int64_t VN = (int64_t)N * VB;
  const double a = (e_max - e_min) / (2.0 - KPM_EPS), b = 0.5 * (e_max + e_min);
  // the factorisation of S runs one block at a time: 64 x 64 tiles give its products
  // four times the workgroups of the batched default
  const int tile = KPM_TILE;

  // ---- memory: factors, vector panels, lu buffers, constants ----
  size_t off = 0;
  auto take = [&](size_t n) {
    size_t o = off;
    off += (n + 255) / 256 * 256;
    return o;
  };
  const size_t o_dinv = take(sizeof(z64) * N * MM), o_uf = take(sizeof(z64) * N * MM),
               o_lf = take(sizeof(z64) * N * MM), o_t = take(sizeof(z64) * MM);
  // b S - H blocks (diagonal, upper, lower), formed once: every Chebyshev step reads them
  const size_t o_ad = take(sizeof(z64) * N * MM), o_au = take(sizeof(z64) * N * MM),
               o_al = take(sizeof(z64) * N * MM);
  size_t o_v[5];
  for (int i = 0; i < 5; ++i) o_v[i] = take(sizeof(z64) * VN);
  const size_t o_linv = take(sizeof(z64) * 64 * Mp), o_uinv = take(sizeof(z64) * 64 * Mp);
  const size_t o_perm = take(4 * Mp), o_cand = take(4 * Mp), o_flags = take(Mp), o_sing = take(4);
  const size_t o_bv = take(sizeof(double) * N), o_two = take(sizeof(double) * N);
  const size_t o_part = take(sizeof(double) * DOT_BLOCKS);
  const size_t o_ksplit = take(sizeof(z64) * (size_t)ksplit(Mp, Rp) * Mp * Rp);
  int dev = 0;
  RGF_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_kpm_mu);
  KpmArena& ar = g_kpm[{dev, st}];
  if (ar.bytes < off) {
    if (ar.p) {
      RGF_HIP(hipStreamSynchronize(st));
      RGF_HIP(hipFree(ar.p));
    }
    ar.p = nullptr;
    ar.bytes = 0;
    hipError_t e = hipMalloc((void**)&ar.p, off);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error{RGF_ENOMEM, "KPM workspace of " + std::to_string(off) + " bytes does not fit"};
    }
    ar.bytes = off;
  }
  char* base = ar.p;
  z64* Dinv = reinterpret_cast<z64*>(base + o_dinv);
  z64* Uf = reinterpret_cast<z64*>(base + o_uf);
  z64* Lf = reinterpret_cast<z64*>(base + o_lf);
  z64* T = reinterpret_cast<z64*>(base + o_t);
  z64* Ad = reinterpret_cast<z64*>(base + o_ad);
  z64* Au = reinterpret_cast<z64*>(base + o_au);
  z64* Al = reinterpret_cast<z64*>(base + o_al);
  z64* V[5];
  for (int i = 0; i < 5; ++i) V[i] = reinterpret_cast<z64*>(base + o_v[i]);
  LuBufs lu;
  lu.linv = reinterpret_cast<z64*>(base + o_linv);
  lu.uinv = reinterpret_cast<z64*>(base + o_uinv);
  lu.perm = reinterpret_cast<int32_t*>(base + o_perm);
  lu.cand = reinterpret_cast<int32_t*>(base + o_cand);
  lu.flags = reinterpret_cast<uint8_t*>(base + o_flags);
  lu.sing = reinterpret_cast<int32_t*>(base + o_sing);
  double* bvals = reinterpret_cast<double*>(base + o_bv);
  double* twos = reinterpret_cast<double*>(base + o_two);
  double* partial = reinterpret_cast<double*>(base + o_part);
  z64* kpart = reinterpret_cast<z64*>(base + o_ksplit);
  hipLaunchKernelGGL(kpm_fill_kernel, dim3((N + 255) / 256), dim3(256), 0, st, bvals, N, b);
  hipLaunchKernelGGL(kpm_fill_kernel, dim3((N + 255) / 256), dim3(256), 0, st, twos, N, 2.0);
  RGF_HIP(hipMemsetAsync(lu.sing, 0, sizeof(int32_t), st));

  // overlap-only operands, formed as 2 S - S (exact); `pad`: identity on the padded diagonal
  auto sblk = [&](const rgf_z* s, bool conj, bool pad) { return form(s, s, M, conj, pad, twos, 0.0); };
  auto mat1 = [&](z64* p, int64_t ld) { return mat(p, MM, ld); };

  // ---- block-Thomas factors of S ----
  for (int i = 0; i < N; ++i) {
    if (i == 0) {
      FillArgs f = fill_args(mat1(T, Mp), Mp, Mp, FILL_FORM);
      f.f = sblk(d.Sd, false, true);
      launch_fill(f, 1, st);
    } else {  // D_i = S_ii - S_{i,i-1} Uf_{i-1}
      GemmArgs g = gemm_args(Mp, Mp, Mp, 1);
      g.a_kind = SRC_FORM;
      g.Af = sblk(d.Su + (i - 1) * M2, true, false);
      g.B = mat1(Uf + (i - 1) * MM, Mp);
      g.c_kind = SRC_FORM;
      g.Cf = sblk(d.Sd + i * M2, false, true);
      g.C = mat1(T, Mp);
      g.alpha = -1.0;
      launch_gemm(g, PREC_F64, tile, st);
    }
    lu_factor(lu, T, MM, Mp, 1, nullptr, i + 1, PREC_F64, tile, st);
    FillArgs f = fill_args(mat1(Dinv + i * MM, Mp), Mp, Mp, FILL_IDENTITY);
    f.ridx = lu.perm;
    f.ridx_bs = Mp;
    launch_fill(f, 1, st);
    lu_solve(lu, T, MM, Mp, Dinv + i * MM, MM, Mp, 1, nullptr, PREC_F64, tile, st);
    if (i + 1 < N) {
      f = fill_args(mat1(Uf + i * MM, Mp), Mp, Mp, FILL_FORM);
      f.f = sblk(d.Su + i * M2, false, false);
      f.ridx = lu.perm;
      f.ridx_bs = Mp;
      launch_fill(f, 1, st);
      lu_solve(lu, T, MM, Mp, Uf + i * MM, MM, Mp, 1, nullptr, PREC_F64, tile, st);
      GemmArgs g = gemm_args(Mp, Mp, Mp, 1);  // Lf_{i+1} = S_{i+1,i} Dinv_i
      g.a_kind = SRC_FORM;
      g.Af = sblk(d.Su + i * M2, true, false);
      g.B = mat1(Dinv + i * MM, Mp);
      g.C = mat1(Lf + (i + 1) * MM, Mp);
      launch_gemm(g, PREC_F64, tile, st);
    }
  }
  int32_t sing = 0;
  RGF_HIP(hipMemcpyAsync(&sing, lu.sing, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  RGF_HIP(hipStreamSynchronize(st));
  RGF_CHECK(sing == 0, RGF_EINVAL,
            "overlap matrix singular (zero pivot in layer " + std::to_string(((sing - 1) & 0xFFFFFF)) + ")");

  // ---- Chebyshev recursion ----
  z64* r = V[0];
  z64* W = V[1];
  z64* ring[3] = {V[2], V[3], V[4]};
  {
    const int64_t total = VN;
    hipLaunchKernelGGL(kpm_pad_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<const z64*>(vectors), r, N, M, R, Mp, Rp);
    RGF_HIP(hipGetLastError());
  }
  const double inv_r = 1.0 / R;
  auto moment = [&](z64* x, const z64* prev, double* out) {
    hipLaunchKernelGGL(kpm_next_kernel, dim3(DOT_BLOCKS), dim3(256), 0, st, x, prev, r, VN, partial);
    hipLaunchKernelGGL(kpm_moment_kernel, dim3(1), dim3(256), 0, st, partial, DOT_BLOCKS, inv_r, out);
    RGF_HIP(hipGetLastError());
  };
  moment(r, nullptr, mu);
  const z64* vprev = nullptr;
  const z64* vcur = r;
  auto panel = [&](const z64* p, int64_t layer) { return mat(const_cast<z64*>(p) + layer * VB, VB, Rp); };
  auto grouped = [&](FormRef f) {
    f.gper = 1;
    f.gb0 = 0;
    f.gstride = M2;
    return f;
  };
  {  // the operator's blocks, one per batch entry (= layer)
    FillArgs f = fill_args(mat(Ad, MM, Mp), Mp, Mp, FILL_FORM);
    f.f = grouped(form(d.Hd, d.Sd, M, false, false, bvals, 0.0));
    launch_fill(f, N, st);
    if (N > 1) {
      f = fill_args(mat(Au, MM, Mp), Mp, Mp, FILL_FORM);
      f.f = grouped(form(d.Hu, d.Su, M, false, false, bvals, 0.0));
      launch_fill(f, N - 1, st);
      launch_form_ct(grouped(form(d.Hu, d.Su, M, true, false, bvals, 0.0)), mat(Al, MM, Mp), Mp, N - 1, st);
    }
  }
  for (int n = 0; n + 1 < n_mom; ++n) {
    z64* X = ring[n % 3];
    const double alpha = (n == 0 ? -1.0 : -2.0) / a;  // c (H - b S) / a = -(c / a) (b S - H)
    // W = c (H - b S) V / a: diagonal, upper and lower blocks
    GemmArgs g = gemm_args(Mp, Rp, Mp, N);
    g.A = mat(Ad, MM, Mp);
    g.B = panel(vcur, 0);
    g.C = panel(W, 0);
    g.alpha = alpha;
    timed_gemm(g, st);
    if (N > 1) {
      g = gemm_args(Mp, Rp, Mp, N - 1);
      g.A = mat(Au, MM, Mp);
      g.B = panel(vcur, 1);
      g.c_kind = SRC_MAT;
      g.Cin = panel(W, 0);
      g.C = panel(W, 0);
      g.alpha = alpha;
      timed_gemm(g, st);
      g.A = mat(Al, MM, Mp);
      g.B = panel(vcur, 0);
      g.Cin = panel(W, 1);
      g.C = panel(W, 1);
      timed_gemm(g, st);
    }
    // forward sweep Z_i = W_i - Lf_i Z_{i-1}
    for (int i = 1; i < N; ++i) sweep_step(Lf + i * MM, W + (i - 1) * VB, W + i * VB, kpart, Mp, Rp, st);
    // X = Dinv Z, then the back sweep X_i = X_i - Uf_i X_{i+1}
    g = gemm_args(Mp, Rp, Mp, N);
    g.A = mat(Dinv, MM, Mp);
    g.B = panel(W, 0);
    g.C = panel(X, 0);
    timed_gemm(g, st);
    for (int i = N - 2; i >= 0; --i) sweep_step(Uf + i * MM, X + (i + 1) * VB, X + i * VB, kpart, Mp, Rp, st);
    moment(X, vprev, mu + n + 1);
    vprev = vcur;
    vcur = X;
  }
}

}  // namespace rgf

using namespace rgf;

extern "C" {

int rgf_kpm_moments(const rgf_device* dev, double e_min, double e_max, int32_t n_mom, const rgf_z* vectors,
                    int32_t R, double* mu, void* stream) {
  try {
    RGF_CHECK(dev && vectors && mu, RGF_EINVAL, "null device, vector or output pointer");
    RGF_CHECK(dev->N >= 1 && dev->M >= 1 && dev->M <= MAX_M, RGF_EINVAL, "N < 1 or M outside [1, 2048]");
    RGF_CHECK(dev->Hd && dev->Sd && (dev->N == 1 || (dev->Hu && dev->Su)), RGF_EINVAL, "null block pointer");
    RGF_CHECK(n_mom >= 1 && R >= 1, RGF_EINVAL, "n_mom and R must be >= 1");
    RGF_CHECK(std::isfinite(e_min) && std::isfinite(e_max) && e_max > e_min, RGF_EINVAL,
              "spectral bounds must be finite with e_max > e_min");
    if (input_checks()) check_inputs(*dev, INPUT_CHECK_TOL, false, (hipStream_t)stream);  // no electrodes here
    kpm_moments_impl(*dev, e_min, e_max, n_mom, vectors, R, mu, (hipStream_t)stream);
    return RGF_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return RGF_EDEVICE;
  }
}

int rgf_kpm_fermi(const double* mu, int32_t n_mom, double e_min, double e_max, double n_states, double* e_fermi,
                  void* stream) {
  try {
    RGF_CHECK(mu && e_fermi, RGF_EINVAL, "null moment or output pointer");
    RGF_CHECK(n_mom >= 1, RGF_EINVAL, "n_mom < 1");
    RGF_CHECK(std::isfinite(e_min) && std::isfinite(e_max) && e_max > e_min, RGF_EINVAL,
              "spectral bounds must be finite with e_max > e_min");
    RGF_CHECK(std::isfinite(n_states), RGF_EINVAL, "n_states must be finite");
    const double a = (e_max - e_min) / (2.0 - KPM_EPS), b = 0.5 * (e_max + e_min);
    hipLaunchKernelGGL(kpm_fermi_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, mu, n_mom, a, b, n_states,
                       e_fermi);
    RGF_HIP(hipGetLastError());
    return RGF_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}

int rgf_kpm_dos(const double* mu, int32_t n_mom, double e_min, double e_max, const double* E, int64_t nE,
                double* dos, void* stream) {
  try {
    RGF_CHECK(n_mom >= 1 && nE >= 0, RGF_EINVAL, "n_mom < 1 or nE < 0");
    RGF_CHECK(nE == 0 || (mu && E && dos), RGF_EINVAL, "null moment, energy or output pointer");
    RGF_CHECK(std::isfinite(e_min) && std::isfinite(e_max) && e_max > e_min, RGF_EINVAL,
              "spectral bounds must be finite with e_max > e_min");
    if (nE == 0) return RGF_OK;
    const double a = (e_max - e_min) / (2.0 - KPM_EPS), b = 0.5 * (e_max + e_min);
    hipLaunchKernelGGL(kpm_dos_kernel, dim3((unsigned)((nE + 255) / 256)), dim3(256), 0, (hipStream_t)stream, mu,
                       n_mom, a, b, E, nE, dos);
    RGF_HIP(hipGetLastError());
    return RGF_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}

}  // extern "C"
