// Memory-bound helpers of the transmission path: block fills (operator
// formation z S - H, identities, copies with row gathers), the elementwise
// half of a decimation step, Gamma = i (Sigma - Sigma^+), Frobenius scales
// and the Caroli trace.  Reductions use a fixed order (per-thread strided
// sums, then a fixed LDS tree), so results do not depend on the batch a
// request runs in.
#include "common.h"
#include "kernels.h"

namespace rgf {
namespace {

constexpr int ET = 256;

// One wavefront per destination row (FILL_ROWS rows per workgroup), so row indices, row
// gathers and block offsets are resolved once per row and the columns stream through; the
// batch index varies fastest over the grid, so the workgroups of different energies that read
// the same source rows of a shared block run together and find them in L2.
constexpr int FILL_ROWS = ET / 64;

__global__ __launch_bounds__(ET) void fill_kernel(FillArgs a, int batch, int groups) {
  const int b = blockIdx.x % batch, grp = blockIdx.x / batch;
  if (a.ctl.skip && a.ctl.skip[b]) return;
  if (a.flags)
    for (int e = grp * ET + threadIdx.x; e < a.flags_n; e += groups * ET) a.flags[(int64_t)b * a.flags_bs + e] = 0;
  const int r = grp * FILL_ROWS + threadIdx.x / 64, lane = threadIdx.x % 64;
  if (r >= a.rows) return;
  const int rs = a.ridx ? a.ridx[(int64_t)b * a.ridx_bs + r] : r;
  z64* dst = a.dst.p + mat_off(a.dst, b, r, 0);
  const double sc = a.scale;
  if (a.kind == FILL_MAT) {
    const z64* src = a.src.p + mat_off(a.src, b, r, 0);
#pragma unroll 4
    for (int c = lane; c < a.cols; c += 64) {
      const z64 s = src[c];
      dst[c] = zmake(sc * s.x, sc * s.y);
    }
  } else if (a.kind == FILL_FORM && !a.f.conj_t && !a.f.sub.p) {  // z S - H read along rows
    const FormRef& f = a.f;
    const z64 z = zmake(f.E[b], f.eta);
    const bool in = rs < f.M;
    const int64_t o = form_group_off(f, b) + (int64_t)(in ? rs : 0) * f.M;
    const z64 *S = f.S + o, *H = f.H + o;
    const int cm = in ? min(a.cols, f.M) : 0;
#pragma unroll 4
    for (int c = lane; c < cm; c += 64) {
      const z64 v = zform(z, S[c], H[c]);
      dst[c] = zmake(sc * v.x, sc * v.y);
    }
    for (int c = cm + lane; c < a.cols; c += 64) dst[c] = zmake((f.pad_identity && rs == c) ? sc : 0.0, 0.0);
  } else {
    for (int c = lane; c < a.cols; c += 64) {
      z64 v;
      switch (a.kind) {
        case FILL_IDENTITY: v = zmake(rs == c ? sc : 0.0, 0.0); break;
        case FILL_FORM: {
          const z64 s = form_elem(a.f, b, rs, c);
          v = zmake(sc * s.x, sc * s.y);
          break;
        }
        default: v = zmake(0.0, 0.0);
      }
      dst[c] = v;
    }
  }
}

// Stored adjoint operand: dst[b] = z_b S^+ - H^+ over the padded Mp x Mp block,
// with the zero (or identity) padding of a formed operand.  One workgroup
// stages a 32 x 32 tile of S and H through LDS (reading rows, writing the
// transposed rows, both coalesced) and writes it for `per` consecutive
// batch entries, reloading only when the group's blocks change.
constexpr int FT = 32;

__global__ __launch_bounds__(ET) void form_ct_kernel(FormRef f, MatRef dst, int batch, int per) {
  __shared__ z64 ss[FT][FT + 1], sh[FT][FT + 1];
  const int r0 = blockIdx.x * FT, c0 = blockIdx.y * FT;
  const int tx = threadIdx.x % FT, ty = threadIdx.x / FT;
  const int b0 = blockIdx.z * per, b1 = min(batch, b0 + per);
  int64_t loaded = -1;
  for (int b = b0; b < b1; ++b) {
    const int64_t g = form_group_off(f, b);
    if (g != loaded) {  // uniform over the workgroup
      __syncthreads();
      for (int j = 0; j < FT; j += ET / FT) {
        const int sr = c0 + ty + j, sc = r0 + tx;  // source (sr, sc) is output (sc, sr)
        const bool ok = sr < f.M && sc < f.M;
        ss[ty + j][tx] = ok ? f.S[g + (int64_t)sr * f.M + sc] : zmake(0.0, 0.0);
        sh[ty + j][tx] = ok ? f.H[g + (int64_t)sr * f.M + sc] : zmake(0.0, 0.0);
      }
      __syncthreads();
      loaded = g;
    }
    const z64 z = zmake(f.E[b], f.eta);
    for (int j = 0; j < FT; j += ET / FT) {
      const int r = r0 + ty + j, c = c0 + tx;
      const z64 v = (r < f.M && c < f.M) ? zform(z, zconj(ss[tx][ty + j]), zconj(sh[tx][ty + j]))
                                         : zmake((f.pad_identity && r == c) ? 1.0 : 0.0, 0.0);
      dst.p[mat_off(dst, b, r, c)] = v;
    }
  }
}

// Input check of `nblk` consecutive M x M blocks (block b at X + b M^2): out[4 b ..] =
// max |X - X^+| (component-wise sum), max |X| (the same measure), min Re X_ii, max |Im X_ii|.
// One workgroup per block; max and min do not depend on the reduction order.
__global__ __launch_bounds__(ET) void herm_check_kernel(const z64* X, int M, double* out) {
  __shared__ double red[4][ET];
  const z64* B = X + (int64_t)blockIdx.x * M * M;
  double asym = 0.0, amax = 0.0, dmin = 1.0e300, dim = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)M * M; e += ET) {
    const int r = (int)(e / M), c = (int)(e % M);
    const z64 x = B[e], y = B[(int64_t)c * M + r];
    asym = fmax(asym, fabs(x.x - y.x) + fabs(x.y + y.y));
    amax = fmax(amax, fabs(x.x) + fabs(x.y));
    if (r == c) {
      dmin = fmin(dmin, x.x);
      dim = fmax(dim, fabs(x.y));
    }
  }
  red[0][threadIdx.x] = asym;
  red[1][threadIdx.x] = amax;
  red[2][threadIdx.x] = dmin;
  red[3][threadIdx.x] = dim;
  __syncthreads();
  for (int w = ET / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + w]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
      red[2][threadIdx.x] = fmin(red[2][threadIdx.x], red[2][threadIdx.x + w]);
      red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) out[4 * (int64_t)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(ET) void axpy_kernel(MatRef dst, MatRef src, double s, int rows, int cols,
                                                   BatchCtl ctl) {
  const int b = blockIdx.y;
  if (ctl.skip && ctl.skip[b]) return;
  const int64_t e = (int64_t)blockIdx.x * ET + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int r = (int)(e / cols), c = (int)(e % cols);
  z64 x = src.p[mat_off(src, b, r, c)];
  z64* d = dst.p + mat_off(dst, b, r, c);
  *d = zmake(d->x + s * x.x, d->y + s * x.y);
}

__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = ET / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Elementwise half of a decimation step (products already in C):
//   eps_R -= aXb, eps_L -= bXa, eps -= aXb + bXa, alpha = -aXa, beta = -bXb
// and the partial sums ||alpha||^2, ||beta||^2 of this block.
constexpr int SR_EPT = 16;
__global__ __launch_bounds__(ET) void sr_update_kernel(SrUpdateArgs a) {
  const int b = blockIdx.y;
  if (a.ctl.skip && a.ctl.skip[b]) return;
  __shared__ double sh[ET];
  const int Mp = a.Mp;
  const int64_t n = (int64_t)Mp * Mp;
  double sa = 0.0, sb = 0.0;
  for (int q = 0; q < SR_EPT; ++q) {
    const int64_t e = ((int64_t)blockIdx.x * SR_EPT + q) * ET + threadIdx.x;
    if (e >= n) break;
    const int r = (int)(e / Mp), c = (int)(e % Mp);
    const z64 aXa = a.C.p[mat_off(a.C, b, r, c)];
    const z64 aXb = a.C.p[mat_off(a.C, b, r, Mp + c)];
    const z64 bXa = a.C.p[mat_off(a.C, b, Mp + r, c)];
    const z64 bXb = a.C.p[mat_off(a.C, b, Mp + r, Mp + c)];
    z64* pe = a.eps.p + mat_off(a.eps, b, r, c);
    z64* pl = a.epsL.p + mat_off(a.epsL, b, r, c);
    z64* pr = a.epsR.p + mat_off(a.epsR, b, r, c);
    const z64 ne = zsub(zsub(*pe, aXb), bXa);
    *pe = ne;
    *pl = zsub(*pl, bXa);
    *pr = zsub(*pr, aXb);
    const z64 al = zneg(aXa), be = zneg(bXb);
    a.AB.p[mat_off(a.AB, b, r, c)] = al;
    a.AB.p[mat_off(a.AB, b, Mp + r, c)] = be;
    sa += al.x * al.x + al.y * al.y;
    sb += be.x * be.x + be.y * be.y;
  }
  sa = block_sum(sa, sh);
  sb = block_sum(sb, sh);
  if (threadIdx.x == 0) {
    a.partial[((int64_t)b * a.nblk + blockIdx.x) * 2 + 0] = sa;
    a.partial[((int64_t)b * a.nblk + blockIdx.x) * 2 + 1] = sb;
  }
}

__global__ void sr_check_kernel(const double* partial, int nblk, const double* scale, double tol, int it,
                                int32_t* done, int32_t* iters, int32_t* active_count, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  if (done[b]) return;
  double sa = 0.0, sb = 0.0;
  for (int k = 0; k < nblk; ++k) {
    sa += partial[((int64_t)b * nblk + k) * 2 + 0];
    sb += partial[((int64_t)b * nblk + k) * 2 + 1];
  }
  iters[b] = it;
  if (sqrt(sa) + sqrt(sb) <= tol * scale[b]) {
    done[b] = 1;
  } else {
    atomicAdd(active_count, 1);
  }
}

__global__ __launch_bounds__(ET) void frob_scale_kernel(MatRef X, int rows, int cols, double* scale) {
  const int b = blockIdx.x;
  __shared__ double sh[ET];
  double s = 0.0;
  const int64_t n = (int64_t)rows * cols;
  for (int64_t e = threadIdx.x; e < n; e += ET) {
    const z64 v = X.p[mat_off(X, b, (int)(e / cols), (int)(e % cols))];
    s += v.x * v.x + v.y * v.y;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) scale[b] = fmax(1.0, sqrt(s));
}

__global__ __launch_bounds__(ET) void broadening_kernel(MatRef sig, MatRef gam, int Mp) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * ET + threadIdx.x;
  if (e >= (int64_t)Mp * Mp) return;
  const int r = (int)(e / Mp), c = (int)(e % Mp);
  const z64 x = sig.p[mat_off(sig, b, r, c)];
  const z64 y = zconj(sig.p[mat_off(sig, b, c, r)]);
  gam.p[mat_off(gam, b, r, c)] = zmake(-(x.y - y.y), x.x - y.x);
}

__global__ __launch_bounds__(ET) void trace_kernel(TraceArgs a) {
  const int b = blockIdx.x;
  __shared__ double sh[ET];
  const int Mp = a.Mp;
  double s = 0.0;
  const int64_t n = (int64_t)Mp * Mp;
  for (int64_t e = threadIdx.x; e < n; e += ET) {
    const int r = (int)(e / Mp), c = (int)(e % Mp);
    const z64 x = a.Z1.p[mat_off(a.Z1, b, r, c)];
    const z64 y = a.Z2.p[mat_off(a.Z2, b, r, c)];
    s += x.x * y.x + x.y * y.y;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    int32_t info = 0;
    if (a.sr_done_l && !a.sr_done_l[b]) info |= RGF_INFO_SR_LEFT;
    if (a.sr_done_r && !a.sr_done_r[b]) info |= RGF_INFO_SR_RIGHT;
    const int32_t sc = a.sing ? a.sing[b] : 0;
    if (sc != 0) info |= RGF_INFO_SINGULAR | ((sc - 1) & 0xFFFFFF) << 8;
    if (sc == 0 && !isfinite(s)) info |= RGF_INFO_NONFINITE;
    if (info & (RGF_INFO_SINGULAR | RGF_INFO_NONFINITE)) s = __builtin_nan("");
    a.T[b] = s;
    if (a.info) a.info[b] = info;
  }
}

__global__ __launch_bounds__(ET) void unpad_kernel(MatRef src, z64* dst, int M) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * ET + threadIdx.x;
  if (e >= (int64_t)M * M) return;
  const int r = (int)(e / M), c = (int)(e % M);
  dst[(int64_t)b * M * M + e] = src.p[mat_off(src, b, r, c)];
}

__global__ void sr_info_kernel(const int32_t* done, int32_t bit, const int32_t* sing, int32_t* info,
                               int batch, int accumulate) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  int32_t v = accumulate ? info[b] : 0;
  if (!done[b]) v |= bit;
  if (sing && sing[b] != 0) v |= RGF_INFO_SINGULAR | ((sing[b] - 1) & 0xFFFFFF) << 8;
  info[b] = v;
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + ET - 1) / ET); }

// Counter-based pseudo-random fill (SplitMix64 of seed + index): entries
// scale * (u + i v) with u, v uniform in [-1, 1), plus `diag` on the diagonal
// of each rows x ld block.  Synthetic inputs for tuning only.
__global__ void random_kernel(z64* p, int64_t n, int64_t ld, int64_t rows, double scale, double diag,
                              uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  auto mix = [](uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
  };
  const uint64_t h1 = mix(seed + 2 * (uint64_t)i), h2 = mix(seed + 2 * (uint64_t)i + 1);
  const double u = (double)(h1 >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  const double v = (double)(h2 >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  const int64_t r = (i / ld) % rows, c = i % ld;
  p[i] = zmake(scale * u + (r == c ? diag : 0.0), scale * v);
}



__global__ void shift_kernel(double* dst, const double* src, int64_t n, double u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i] - u;
}

// Fermi-Dirac occupation; kT = 0: the step, 1/2 exactly at E = mu
__device__ inline double fermi(double E, double mu, double kT) {
  if (kT == 0.0) return E < mu ? 1.0 : (E > mu ? 0.0 : 0.5);
  const double x = (E - mu) / kT;
  const double e = exp(-fabs(x));  // <= 1: no overflow on either side
  return x > 0.0 ? e / (1.0 + e) : 1.0 / (1.0 + e);
}

constexpr int LT = 256;
// Landauer integral in one workgroup: thread t sums the trapezoids of the
// contiguous interval range [t*chunk, (t+1)*chunk) in order, then a fixed
// binary tree in LDS; the result does not depend on the launch.
__global__ __launch_bounds__(LT) void landauer_kernel(const double* E, const double* T, int64_t n, double mu_l,
                                                      double mu_r, double kT, double g0, double* I) {
  __shared__ double part[LT];
  const int t = threadIdx.x;
  const int64_t nint = n - 1;  // intervals
  const int64_t chunk = (nint + LT - 1) / LT;
  double s = 0.0;
  const int64_t a = t * chunk, bnd = (a + chunk < nint) ? a + chunk : nint;
  for (int64_t k = a; k < bnd; ++k) {
    const double g0k = (fermi(E[k], mu_l, kT) - fermi(E[k], mu_r, kT)) * T[k];
    const double g1k = (fermi(E[k + 1], mu_l, kT) - fermi(E[k + 1], mu_r, kT)) * T[k + 1];
    s += (E[k + 1] - E[k]) * (g0k + g1k) * 0.5;
  }
  part[t] = s;
  __syncthreads();
  for (int w = LT / 2; w > 0; w >>= 1) {
    if (t < w) part[t] += part[t + w];
    __syncthreads();
  }
  if (t == 0) I[0] = g0 * part[0];
}

// X(k) block elements from the real-space images (HBM-bound: nR reads, one write per element)
__global__ void bloch_kernel(BlochArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  z64 acc = zmake(0.0, 0.0);
  for (int r = 0; r < a.nR; ++r)
    if (a.src[r]) acc = zfma(a.w[r], a.src[r][i], acc);
  a.dst[i] = acc;
}

__global__ void kaccum_kernel(double* T, const double* Tk, double w, int64_t n, int first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) T[i] = (first ? 0.0 : T[i]) + w * Tk[i];
}

}  // namespace

void launch_bloch(const BlochArgs& a, hipStream_t st) {
  if (a.n <= 0) return;
  hipLaunchKernelGGL(bloch_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  RGF_HIP(hipGetLastError());
}

void launch_kaccum(double* T, const double* Tk, double w, int64_t n, int first, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(kaccum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, T, Tk, w, n, first);
  RGF_HIP(hipGetLastError());
}

void launch_shift(double* dst, const double* src, int64_t n, double u, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(shift_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, src, n, u);
  RGF_HIP(hipGetLastError());
}

void launch_landauer(const double* E, const double* T, int64_t n, double mu_l, double mu_r, double kT, double* I,
                     hipStream_t st) {
  // 2 e^2 / h with the exact SI constants (C, J s): the spin-degenerate conductance quantum
  const double e = 1.602176634e-19, h = 6.62607015e-34;
  hipLaunchKernelGGL(landauer_kernel, dim3(1), dim3(LT), 0, st, E, T, n, mu_l, mu_r, kT, 2.0 * e * e / h, I);
  RGF_HIP(hipGetLastError());
}

void launch_random(z64* p, int64_t n, int64_t ld, int64_t rows, double scale, double diag, uint64_t seed,
                   hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(random_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, ld, rows, scale,
                     diag, seed);
  RGF_HIP(hipGetLastError());
}

void launch_fill(const FillArgs& a, int batch, hipStream_t st) {
  if (batch <= 0) return;
  const int64_t groups = std::max<int64_t>((a.rows + FILL_ROWS - 1) / FILL_ROWS,
                                           a.flags ? ((int64_t)a.flags_n + ET - 1) / ET : 0);
  if (groups <= 0) return;
  if (groups * batch > INT32_MAX)
    throw Error{RGF_EINVAL, "fill: grid of " + std::to_string(groups * batch) + " workgroups"};
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)(groups * batch)), dim3(ET), 0, st, a, batch, (int)groups);
  RGF_HIP(hipGetLastError());
}

void launch_herm_check(const z64* X, int M, int nblk, double* out, hipStream_t st) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(herm_check_kernel, dim3((unsigned)nblk), dim3(ET), 0, st, X, M, out);
  RGF_HIP(hipGetLastError());
}

void launch_form_ct(const FormRef& f, MatRef dst, int Mp, int batch, hipStream_t st) {
  if (batch <= 0) return;
  RGF_CHECK(Mp % FT == 0 && f.M <= Mp && !f.sub.p && !dst.rowidx, RGF_EINVAL, "form_ct: bad operand");
  const int per = 8;
  const dim3 grid((unsigned)(Mp / FT), (unsigned)(Mp / FT), (unsigned)((batch + per - 1) / per));
  hipLaunchKernelGGL(form_ct_kernel, grid, dim3(ET), 0, st, f, dst, batch, per);
  RGF_HIP(hipGetLastError());
}

void launch_axpy(MatRef dst, MatRef src, double s, int rows, int cols, int batch, BatchCtl ctl,
                 hipStream_t st) {
  if (batch <= 0) return;
  hipLaunchKernelGGL(axpy_kernel, dim3(nblocks((int64_t)rows * cols), batch), dim3(ET), 0, st, dst, src, s,
                     rows, cols, ctl);
  RGF_HIP(hipGetLastError());
}

void launch_sr_update(const SrUpdateArgs& a, int batch, hipStream_t st) {
  hipLaunchKernelGGL(sr_update_kernel, dim3(a.nblk, batch), dim3(ET), 0, st, a);
  RGF_HIP(hipGetLastError());
}

void launch_sr_check(const double* partial, int nblk, const double* scale, double tol, int it,
                     int32_t* done, int32_t* iters, int32_t* active_count, int batch, hipStream_t st) {
  hipLaunchKernelGGL(sr_check_kernel, dim3((batch + 127) / 128), dim3(128), 0, st, partial, nblk, scale, tol,
                     it, done, iters, active_count, batch);
  RGF_HIP(hipGetLastError());
}

void launch_frob_scale(MatRef X, int rows, int cols, double* scale, int batch, hipStream_t st) {
  hipLaunchKernelGGL(frob_scale_kernel, dim3(batch), dim3(ET), 0, st, X, rows, cols, scale);
  RGF_HIP(hipGetLastError());
}

void launch_broadening(MatRef sigma, MatRef gamma, int Mp, int batch, hipStream_t st) {
  hipLaunchKernelGGL(broadening_kernel, dim3(nblocks((int64_t)Mp * Mp), batch), dim3(ET), 0, st, sigma,
                     gamma, Mp);
  RGF_HIP(hipGetLastError());
}

void launch_trace(const TraceArgs& a, int batch, hipStream_t st) {
  hipLaunchKernelGGL(trace_kernel, dim3(batch), dim3(ET), 0, st, a);
  RGF_HIP(hipGetLastError());
}

void launch_unpad(MatRef src, z64* dst, int M, int batch, hipStream_t st) {
  hipLaunchKernelGGL(unpad_kernel, dim3(nblocks((int64_t)M * M), batch), dim3(ET), 0, st, src, dst, M);
  RGF_HIP(hipGetLastError());
}

void launch_sr_info(const int32_t* done, int32_t bit, const int32_t* sing, int32_t* info, int batch,
                    int accumulate, hipStream_t st) {
  hipLaunchKernelGGL(sr_info_kernel, dim3((batch + 127) / 128), dim3(128), 0, st, done, bit, sing, info,
                     batch, accumulate);
  RGF_HIP(hipGetLastError());
}

}  // namespace rgf
