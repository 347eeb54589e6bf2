// Fused transmission kernel for small blocks (M <= 16): one wavefront per
// energy runs the whole path -- decimation of both leads, self-energies,
// the recursive sweep over all layers and the Caroli trace -- with every
// block held in LDS.  At these sizes the path is latency-bound, so the aim
// is one launch and no HBM round trips between steps.
//
// Arithmetic (FP64 throughout):
//   decimation   eps [Xa Xb] = [alpha beta];  eps_R -= alpha Xb,
//                eps_L -= beta Xa, eps -= alpha Xb + beta Xa,
//                alpha <- -alpha Xa, beta <- -beta Xb
//                (Lopez Sancho, Lopez Sancho, Rubio 1985)
//   self-energy  Sigma_L = L_L (eps_L^-1 U_L),  Sigma_R = U_R (eps_R^-1 L_R)
//   sweep        B_0 = A_00 - Sigma_L;  X = B_l^-1 U_l;
//                W = X (l = 0) or W <- -W X;  B_{l+1} = A - L_{l+1} X
//                (- Sigma_R on the last layer);  G_1N = -W B_{N-1}^-1
//   trace        T = Re sum_jk (Gamma_L G)_jk conj((G Gamma_R)_jk)
//                = Re Tr[Gamma_L G Gamma_R G^+]
// Each solve is Gauss-Jordan elimination with partial pivoting (largest
// |Re|+|Im|, lowest row on ties) on the augmented block [B | RHS].
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace rgf {
namespace {

constexpr int SM_MAX = 16;
constexpr int SM_T = 64;
constexpr int SM_MM = SM_MAX * SM_MAX;

__device__ inline void bar() { __syncthreads(); }

// C = alpha * A*B (+ c0s * C0).  C may alias C0 (same index), never A or B.
__device__ void mm(int M, const z64* A, int lda, const z64* B, int ldb, z64* C, int ldc,
                   double alpha, const z64* C0, int ldc0, double c0s) {
  for (int e = threadIdx.x; e < M * M; e += SM_T) {
    int r = e / M, c = e - r * M;
    z64 acc = zmake(0.0, 0.0);
    for (int k = 0; k < M; ++k) acc = zfma(A[r * lda + k], B[k * ldb + c], acc);
    z64 v = zmake(alpha * acc.x, alpha * acc.y);
    if (C0) v = zmake(v.x + c0s * C0[r * ldc0 + c].x, v.y + c0s * C0[r * ldc0 + c].y);
    C[r * ldc + c] = v;
  }
  bar();
}

__device__ void copy(int M, const z64* A, int lda, z64* C, int ldc, double s) {
  for (int e = threadIdx.x; e < M * M; e += SM_T) {
    int r = e / M, c = e - r * M;
    z64 v = A[r * lda + c];
    C[r * ldc + c] = zmake(s * v.x, s * v.y);
  }
  bar();
}

// dst = z S - H  (conj_t: z S^+ - H^+), M x M from global blocks of size M
__device__ void load_form(int M, const z64* H, const z64* S, z64 z, bool conj_t, z64* dst, int ld) {
  for (int e = threadIdx.x; e < M * M; e += SM_T) {
    int r = e / M, c = e - r * M;
    z64 v;
    if (conj_t) v = zform(z, zconj(S[c * M + r]), zconj(H[c * M + r]));
    else v = zform(z, S[r * M + c], H[r * M + c]);
    dst[r * ld + c] = v;
  }
  bar();
}

// Gauss-Jordan with partial pivoting on Wk = [B | R] (M x (M + nr), ld M + nr):
// afterwards Wk[:, M:] = B^-1 R.  Returns true if an exactly zero pivot was met.
__device__ bool gje(int M, int nr, z64* Wk) {
  const int ld = M + nr;
  const int lane = threadIdx.x;
  bool singular = false;
  for (int j = 0; j < M; ++j) {
    double v = -1.0;
    int idx = 0x7fffffff;
    if (lane >= j && lane < M) {
      v = zabs1(Wk[lane * ld + j]);
      // a NaN entry ranks above every number (as the batched panel's integer key does), so
      // the butterfly below leaves one winner in every lane and only an exact zero column
      // counts as a singular pivot; the NaN then reaches T, which reports it as non-finite
      if (v != v) v = __builtin_inf();
      idx = lane;
    }
    for (int off = 32; off > 0; off >>= 1) {
      double ov = __shfl_xor(v, off);
      int oi = __shfl_xor(idx, off);
      if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
      }
    }
    const int p = idx;
    if (!(v > 0.0)) singular = true;
    if (p != j && p < M) {
      for (int c = j + lane; c < ld; c += SM_T) {
        z64 t = Wk[j * ld + c];
        Wk[j * ld + c] = Wk[p * ld + c];
        Wk[p * ld + c] = t;
      }
    }
    bar();
    const z64 inv = zinv(Wk[j * ld + j]);
    bar();
    for (int c = j + 1 + lane; c < ld; c += SM_T) Wk[j * ld + c] = zmul(Wk[j * ld + c], inv);
    bar();
    const int w = ld - (j + 1);
    for (int e = lane; e < M * w; e += SM_T) {
      int r = e / w, c = j + 1 + (e - r * w);
      if (r != j) Wk[r * ld + c] = zfms(Wk[r * ld + j], Wk[j * ld + c], Wk[r * ld + c]);
    }
    bar();
  }
  return singular;
}

__device__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ double frob2(int M, const z64* A) {
  double s = 0.0;
  for (int e = threadIdx.x; e < M * M; e += SM_T) s += A[e].x * A[e].x + A[e].y * A[e].y;
  return wave_sum(s);
}

struct Bufs {
  z64 *eps, *epsL, *epsR, *al, *be, *t1, *t2, *t3, *t4, *Wk, *sigL, *sigR, *gamL, *gamR;
};

// Decimation of one lead; leaves eps_L, eps_R (surface inverses' operands) in b.
__device__ int sancho_rubio(int M, const z64* H00, const z64* H01, const z64* S00, const z64* S01,
                            z64 z, double tol, int maxit, Bufs& b, bool* converged, bool* singular) {
  load_form(M, H00, S00, z, false, b.eps, M);
  copy(M, b.eps, M, b.epsL, M, 1.0);
  copy(M, b.eps, M, b.epsR, M, 1.0);
  load_form(M, H01, S01, z, false, b.al, M);
  load_form(M, H01, S01, z, true, b.be, M);
  const double scale = fmax(1.0, sqrt(frob2(M, b.eps)));
  *converged = false;
  const int ld = 3 * M;
  int it = 0;
  while (it < maxit) {
    ++it;
    copy(M, b.eps, M, b.Wk, ld, 1.0);
    copy(M, b.al, M, b.Wk + M, ld, 1.0);
    copy(M, b.be, M, b.Wk + 2 * M, ld, 1.0);
    if (gje(M, 2 * M, b.Wk)) *singular = true;
    const z64* Xa = b.Wk + M;
    const z64* Xb = b.Wk + 2 * M;
    mm(M, b.al, M, Xb, ld, b.t1, M, 1.0, nullptr, 0, 0.0);  // alpha Xb
    mm(M, b.be, M, Xa, ld, b.t2, M, 1.0, nullptr, 0, 0.0);  // beta Xa
    mm(M, b.al, M, Xa, ld, b.t3, M, 1.0, nullptr, 0, 0.0);  // alpha Xa
    mm(M, b.be, M, Xb, ld, b.t4, M, 1.0, nullptr, 0, 0.0);  // beta Xb
    for (int e = threadIdx.x; e < M * M; e += SM_T) {
      b.epsR[e] = zsub(b.epsR[e], b.t1[e]);
      b.epsL[e] = zsub(b.epsL[e], b.t2[e]);
      b.eps[e] = zsub(zsub(b.eps[e], b.t1[e]), b.t2[e]);
      b.al[e] = zneg(b.t3[e]);
      b.be[e] = zneg(b.t4[e]);
    }
    bar();
    const double na = sqrt(frob2(M, b.al));
    const double nb = sqrt(frob2(M, b.be));
    if (na + nb <= tol * scale) {
      *converged = true;
      break;
    }
  }
  return it;
}

// sigma = X (eps^-1 Y): X, Y formed from the lead coupling (conj flags select U or L)
__device__ void self_energy(int M, const z64* H01, const z64* S01, z64 z, const z64* epsS,
                            bool left, Bufs& b, z64* sigma, bool* singular) {
  // left:  Sigma = L (eps_L^-1 U);  right: Sigma = U (eps_R^-1 L)
  const int ld = 2 * M;
  copy(M, epsS, M, b.Wk, ld, 1.0);
  load_form(M, H01, S01, z, left ? false : true, b.Wk + M, ld);
  if (gje(M, M, b.Wk)) *singular = true;
  load_form(M, H01, S01, z, left ? true : false, b.t1, M);
  mm(M, b.t1, M, b.Wk + M, ld, sigma, M, 1.0, nullptr, 0, 0.0);
}

__device__ void broadening(int M, const z64* sig, z64* gam) {
  for (int e = threadIdx.x; e < M * M; e += SM_T) {
    int r = e / M, c = e - r * M;
    z64 a = sig[r * M + c], bT = zconj(sig[c * M + r]);
    // i (a - b) = (-(a.y - b.y), a.x - b.x)
    gam[e] = zmake(-(a.y - bT.y), a.x - bT.x);
  }
  bar();
}

}  // namespace

// The whole path for energy k of one device (one wavefront, blocks in `sm`).
__device__ void small_solve(const SmallArgs& a, int k, z64* sm) {
  const int M = a.M;
  Bufs b;
  b.eps = sm;
  b.epsL = sm + 1 * SM_MM;
  b.epsR = sm + 2 * SM_MM;
  b.al = sm + 3 * SM_MM;
  b.be = sm + 4 * SM_MM;
  b.t1 = sm + 5 * SM_MM;
  b.t2 = sm + 6 * SM_MM;
  b.t3 = sm + 7 * SM_MM;
  b.t4 = sm + 8 * SM_MM;
  b.sigL = sm + 9 * SM_MM;
  b.sigR = sm + 10 * SM_MM;
  b.gamL = sm + 11 * SM_MM;
  b.gamR = sm + 12 * SM_MM;
  b.Wk = sm + 13 * SM_MM;

  const z64 z = zmake(a.E[k], a.eta);
  int32_t info = 0;
  bool sing_lead = false, conv_l = false, conv_r = false;

  // a rigidly shifted electrode (H -> H + u S) is the unshifted one at z - u
  const z64 zl = zmake(z.x - a.u_l, z.y), zr = zmake(z.x - a.u_r, z.y);
  sancho_rubio(M, a.LH00, a.LH01, a.LS00, a.LS01, zl, a.sr_tol, a.sr_maxit, b, &conv_l, &sing_lead);
  self_energy(M, a.LH01, a.LS01, zl, b.epsL, true, b, b.sigL, &sing_lead);
  if (a.same_leads && a.u_l == a.u_r) {
    conv_r = conv_l;
  } else {
    sancho_rubio(M, a.RH00, a.RH01, a.RS00, a.RS01, zr, a.sr_tol, a.sr_maxit, b, &conv_r, &sing_lead);
  }
  self_energy(M, a.RH01, a.RS01, zr, b.epsR, false, b, b.sigR, &sing_lead);
  broadening(M, b.sigL, b.gamL);
  broadening(M, b.sigR, b.gamR);
  if (!conv_l) info |= RGF_INFO_SR_LEFT;
  if (!conv_r) info |= RGF_INFO_SR_RIGHT;
  int sing_layer = sing_lead ? 0xFFFFFF : -1;

  // ---- sweep ----
  const int N = a.N;
  const int64_t MM = (int64_t)M * M;
  z64* B = b.eps;
  z64* W = b.epsL;
  z64* A = b.al;
  z64* L = b.be;
  const int ld2 = 2 * M;
  load_form(M, a.Hd, a.Sd, z, false, B, M);
  for (int e = threadIdx.x; e < M * M; e += SM_T) {
    z64 v = zsub(B[e], b.sigL[e]);
    if (N == 1) v = zsub(v, b.sigR[e]);
    B[e] = v;
  }
  bar();
  for (int l = 0; l + 1 < N; ++l) {
    copy(M, B, M, b.Wk, ld2, 1.0);
    load_form(M, a.Hu + l * MM, a.Su + l * MM, z, false, b.Wk + M, ld2);
    if (gje(M, M, b.Wk) && sing_layer < 0) sing_layer = l;
    const z64* X = b.Wk + M;
    if (l == 0) {
      copy(M, X, ld2, W, M, 1.0);
    } else {
      mm(M, W, M, X, ld2, b.t1, M, 1.0, nullptr, 0, 0.0);
      copy(M, b.t1, M, W, M, -1.0);
    }
    load_form(M, a.Hd + (l + 1) * MM, a.Sd + (l + 1) * MM, z, false, A, M);
    load_form(M, a.Hu + l * MM, a.Su + l * MM, z, true, L, M);
    // B = A - L X (- Sigma_R on the last layer)
    mm(M, L, M, X, ld2, B, M, -1.0, A, M, 1.0);
    if (l + 2 == N) {
      for (int e = threadIdx.x; e < M * M; e += SM_T) B[e] = zsub(B[e], b.sigR[e]);
      bar();
    }
  }
  // G_1N = -W B^-1 (or B^-1 when N = 1)
  copy(M, B, M, b.Wk, ld2, 1.0);
  for (int e = threadIdx.x; e < M * M; e += SM_T) {
    int r = e / M, c = e - r * M;
    b.Wk[r * ld2 + M + c] = zmake(r == c ? 1.0 : 0.0, 0.0);
  }
  bar();
  if (gje(M, M, b.Wk) && sing_layer < 0) sing_layer = N;
  z64* P = b.t2;
  if (N == 1) copy(M, b.Wk + M, ld2, P, M, 1.0);
  else mm(M, W, M, b.Wk + M, ld2, P, M, -1.0, nullptr, 0, 0.0);
  mm(M, b.gamL, M, P, M, b.t3, M, 1.0, nullptr, 0, 0.0);
  mm(M, P, M, b.gamR, M, b.t4, M, 1.0, nullptr, 0, 0.0);
  double s = 0.0;
  for (int e = threadIdx.x; e < M * M; e += SM_T) s += b.t3[e].x * b.t4[e].x + b.t3[e].y * b.t4[e].y;
  s = wave_sum(s);
  if (sing_layer >= 0) info |= RGF_INFO_SINGULAR | (int32_t)((sing_layer & 0xFFFFFF) << 8);
  if (!(sing_layer >= 0) && !isfinite(s)) info |= RGF_INFO_NONFINITE;
  if ((info & (RGF_INFO_SINGULAR | RGF_INFO_NONFINITE)) != 0) s = __builtin_nan("");
  if (threadIdx.x == 0) {
    a.T[k] = s;
    if (a.info) a.info[k] = info;
  }
}


constexpr int SM_LDS = 13 * SM_MM + SM_MAX * 3 * SM_MAX;

__global__ __launch_bounds__(SM_T) void rgf_small_kernel(SmallArgs a) {
  const int k = blockIdx.x;
  if (k >= a.nE) return;
  __shared__ z64 sm[SM_LDS];
  small_solve(a, k, sm);
}

// Persistent form over many devices: every workgroup takes (device, energy)
// items from a global counter until the list is exhausted, so devices of
// uneven block size, length and energy count share one launch and the
// workgroups stay busy until the last item.
__global__ __launch_bounds__(SM_T) void rgf_small_queue_kernel(const SmallJob* jobs, int njobs, int64_t total,
                                                                unsigned long long* counter) {
  __shared__ z64 sm[SM_LDS];
  __shared__ long long sh_item;
  for (;;) {
    if (threadIdx.x == 0) sh_item = (long long)atomicAdd(counter, 1ull);
    bar();
    const long long item = sh_item;
    bar();  // every lane has the item before lane 0 takes the next one
    if (item >= total) return;
    int lo = 0, hi = njobs - 1;  // the last job whose first item is <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (jobs[mid].item0 <= item) lo = mid;
      else hi = mid - 1;
    }
    small_solve(jobs[lo].a, (int)(item - jobs[lo].item0), sm);
    bar();
  }
}

void launch_small(const SmallArgs& a, hipStream_t st) {
  if (a.nE <= 0) return;
  hipLaunchKernelGGL(rgf_small_kernel, dim3((unsigned)a.nE), dim3(SM_T), 0, st, a);
  RGF_HIP(hipGetLastError());
}

void launch_small_queue(const SmallJob* jobs, int njobs, int64_t total, unsigned long long* counter, int grid,
                        hipStream_t st) {
  if (total <= 0 || njobs <= 0) return;
  hipLaunchKernelGGL(rgf_small_queue_kernel, dim3((unsigned)std::max(1, grid)), dim3(SM_T), 0, st, jobs, njobs,
                     total, counter);
  RGF_HIP(hipGetLastError());
}

}  // namespace rgf
