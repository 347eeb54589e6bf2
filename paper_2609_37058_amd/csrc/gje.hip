// Blocked Gauss-Jordan elimination with partial pivoting, batched: the
// panel step.
//
// The solve X = B^-1 R is carried out on the augmented block T = [B | R]
// (Mp rows) in panels of 64 columns.  Rows never move: a per-batch flag
// marks rows that already pivoted, and perm[c] records the physical row
// that pivots column c, so after the last panel X[c, :] = T[perm[c], Mp:].
//
// For the panel K = [k0, k0+64) this kernel
//   1. chooses the 64 pivot rows among the rows not yet pivoted by LU with
//      partial pivoting of the panel restricted to those rows: per column
//      the largest |Re|+|Im| wins (lowest row index on ties), found by a
//      wavefront butterfly and a cross-wavefront pass in LDS.  This gives
//      A_KK = T[piv, K] = L11 U11 and, for every other candidate row r, its
//      multipliers l_r (T[r, K] = l_r U11);
//   2. forms, in FP64, the elimination multipliers of every row,
//        candidate row r        m_r = l_r L11^-1
//        earlier pivot row r    m_r = T[r, K] A_KK^-1
//        pivot row piv_j        m_r = e_j - (A_KK^-1)_j
//      (L11^-1 and A_KK^-1 by Gauss-Jordan in LDS, in the chosen pivot
//      order, where L11 has unit diagonal and |entries| <= 1);
//   3. copies the pivot rows right of the panel, P = T[piv, rest].
// One block product on the matrix cores then finishes the panel:
//   T[:, rest] -= m P,
// which eliminates the panel columns from every other row and leaves the
// normalised pivot rows (A_KK^-1 P)_j in place.  Candidate rows use l_r L11^-1
// rather than T[r, K] A_KK^-1 (equal in exact arithmetic): the latter would
// multiply their rounding errors by the condition number of A_KK.
//
// Step 1 holds an 8-column sub-panel of each row in registers (thread per
// row, or two rows per thread when Mp = 2048), applies the rank-8 update of
// the remaining panel columns from LDS-resident pivot rows, and keeps the
// partially eliminated panel in a per-batch scratch block.
#include "common.h"
#include "kernels.h"

namespace rgf {
namespace {

constexpr int NB = GJE_NB;
constexpr int MAXMP = 2048;
constexpr int MC = 8;  // multiplier columns per register chunk

// In-place Gauss-Jordan inverse of an NB x NB block in LDS, no pivoting.
__device__ void lds_invert(z64* A, z64* colj, int tid, int nt) {
  for (int j = 0; j < NB; ++j) {
    const z64 inv = zinv(A[j * NB + j]);
    __syncthreads();
    if (tid < NB) {
      const int c = tid;
      A[j * NB + c] = (c == j) ? inv : zmul(A[j * NB + c], inv);
      colj[c] = (c == j) ? zmake(0.0, 0.0) : A[c * NB + j];
    }
    __syncthreads();
    for (int e = tid; e < NB * NB; e += nt) {
      const int i = e / NB, c = e % NB;
      if (i != j) {
        const z64 base = (c == j) ? zmake(0.0, 0.0) : A[e];
        A[e] = zfms(colj[i], A[j * NB + c], base);
      }
    }
    __syncthreads();
  }
}

template <int RPT, int SW>
__global__ __launch_bounds__(1024) void gje_panel_kernel(PanelArgs a) {
  constexpr int NSUB = NB / SW;
  const int b = blockIdx.x;
  if (a.ctl.skip && a.ctl.skip[b]) return;
  const int nt = blockDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
  const int Mp = a.Mp, k0 = a.k0;

  __shared__ z64 U[NB * NB];    // pivot rows' U entries; later A_KK^-1
  __shared__ z64 Lf[NB * NB];   // L11, then L11^-1
  __shared__ z64 Ls[SW * SW];
  __shared__ z64 colj[NB];
  __shared__ uint8_t fl[MAXMP];  // 0 candidate, 1 earlier pivot, 2 pivot of this panel
  __shared__ int piv[NB];
  __shared__ double rv[16];
  __shared__ int ri[16];
  __shared__ int sh_p, sh_sing;

  uint8_t* gflags = a.flags + (int64_t)b * a.flags_bs;
  for (int r = tid; r < Mp; r += nt) fl[r] = gflags[r] ? 1 : 0;
  if (tid == 0) sh_sing = 0;
  __syncthreads();

  z64* Tb = a.T.p + (int64_t)b * a.T.bstride;
  const int64_t ld = a.T.ld;
  z64* scr = a.scratch + (int64_t)b * a.scratch_bs;  // partially eliminated panel, ld NB
  z64* mult = a.mult + (int64_t)b * a.mult_bs;        // multipliers, ld NB

  bool cand[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = tid + i * nt;
    cand[i] = (r < Mp) && (fl[r] == 0);
  }

  z64 v[RPT][SW];
  for (int s = 0; s < NSUB; ++s) {
    const int cb = SW * s;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = tid + i * nt;
#pragma unroll
      for (int j = 0; j < SW; ++j) {
        z64 x = zmake(0.0, 0.0);
        if (cand[i]) x = (s == 0) ? Tb[(int64_t)r * ld + k0 + cb + j] : scr[(int64_t)r * NB + cb + j];
        v[i][j] = x;
      }
    }
#pragma unroll
    for (int j = 0; j < SW; ++j) {
      double best = -1.0;
      int bi = 0x7fffffff;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        if (cand[i]) {
          const double x = zabs1(v[i][j]);
          if (x > best) {
            best = x;
            bi = tid + i * nt;
          }
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == 0) {
        rv[wave] = best;
        ri[wave] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        double bb = rv[0];
        int bx = ri[0];
        for (int w = 1; w < nwaves; ++w) {
          if (rv[w] > bb || (rv[w] == bb && ri[w] < bx)) {
            bb = rv[w];
            bx = ri[w];
          }
        }
        if (!(bb > 0.0)) sh_sing = 1;
        if (bx >= Mp) bx = 0;  // no candidate left: cannot happen for a square system
        sh_p = bx;
        piv[cb + j] = bx;
      }
      __syncthreads();
      const int p = sh_p;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        if (tid + i * nt == p) {
#pragma unroll
          for (int t = j; t < SW; ++t) U[(cb + j) * NB + cb + t] = v[i][t];
#pragma unroll
          for (int m = 0; m < j; ++m) {
            Ls[j * SW + m] = v[i][m];
            mult[(int64_t)p * NB + cb + m] = v[i][m];
          }
          cand[i] = false;
          fl[p] = 2;
        }
      }
      __syncthreads();
      const z64 inv = zinv(U[(cb + j) * NB + cb + j]);
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        if (cand[i]) {
          const z64 l = zmul(v[i][j], inv);
          v[i][j] = l;
#pragma unroll
          for (int t = j + 1; t < SW; ++t) v[i][t] = zfms(l, U[(cb + j) * NB + cb + t], v[i][t]);
        }
      }
    }
    // multipliers of the rows still candidates for this sub-panel's columns
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      if (cand[i]) {
        const int r = tid + i * nt;
#pragma unroll
        for (int m = 0; m < SW; ++m) mult[(int64_t)r * NB + cb + m] = v[i][m];
      }
    }
    if (s + 1 < NSUB) {
      const int c_begin = cb + SW;
      const int nrem = NB - c_begin;
      // pivot rows of this sub-panel: their U entries at the remaining panel columns
      if (tid < nrem) {
        const int c = c_begin + tid;
        for (int j = 0; j < SW; ++j) {
          const int p = piv[cb + j];
          z64 x = (s == 0) ? Tb[(int64_t)p * ld + k0 + c] : scr[(int64_t)p * NB + c];
          for (int m = 0; m < j; ++m) x = zfms(Ls[j * SW + m], U[(cb + m) * NB + c], x);
          U[(cb + j) * NB + c] = x;
        }
      }
      __syncthreads();
      // remaining candidate rows: rank-SW update of the rest of the panel
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        if (cand[i]) {
          const int r = tid + i * nt;
          for (int c = c_begin; c < NB; ++c) {
            z64 x = (s == 0) ? Tb[(int64_t)r * ld + k0 + c] : scr[(int64_t)r * NB + c];
#pragma unroll
            for (int m = 0; m < SW; ++m) x = zfms(v[i][m], U[(cb + m) * NB + c], x);
            scr[(int64_t)r * NB + c] = x;
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- A_KK^-1 (from the original panel values) and L11^-1 ----
  for (int e = tid; e < NB * NB; e += nt) {
    const int j = e / NB, c = e % NB;
    U[e] = Tb[(int64_t)piv[j] * ld + k0 + c];
    Lf[e] = (c < j) ? mult[(int64_t)piv[j] * NB + c] : zmake(c == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  lds_invert(U, colj, tid, nt);
  lds_invert(Lf, colj, tid, nt);

  // ---- multipliers of every row ----
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = tid + i * nt;
    if (r >= Mp) continue;
    const int kind = fl[r];  // 0 candidate, 1 earlier pivot, 2 pivot of this panel
    z64* mrow = mult + (int64_t)r * NB;
    const z64* in = (kind == 1) ? Tb + (int64_t)r * ld + k0 : mrow;
    const z64* Mx = (kind == 0) ? Lf : U;
    for (int c0 = 0; c0 < NB; c0 += MC) {
      z64 acc[MC];
#pragma unroll
      for (int c = 0; c < MC; ++c) acc[c] = zmake(0.0, 0.0);
      if (kind != 2) {
        // candidates: L11^-1 is lower triangular, so only m >= c0 contributes
        const int m0 = (kind == 0) ? c0 : 0;
        for (int m = m0; m < NB; ++m) {
          const z64 x = in[m];
#pragma unroll
          for (int c = 0; c < MC; ++c) acc[c] = zfma(x, Mx[m * NB + c0 + c], acc[c]);
        }
      }
      if (kind == 2) {
        int j = 0;
        for (int q = 0; q < NB; ++q)
          if (piv[q] == r) j = q;
#pragma unroll
        for (int c = 0; c < MC; ++c) {
          const z64 w = U[j * NB + c0 + c];
          acc[c] = zmake((c0 + c == j ? 1.0 : 0.0) - w.x, -w.y);
        }
      }
      // chunks go left to right and chunk c0 reads columns >= c0 only, so a
      // candidate's l_r can be overwritten in place
#pragma unroll
      for (int c = 0; c < MC; ++c) mrow[c0 + c] = acc[c];
    }
  }
  __syncthreads();

  // ---- pivot rows right of the panel, and bookkeeping ----
  const int rest = a.W - k0 - NB;
  z64* P = a.prow + (int64_t)b * a.prow_bs;  // 64 x rest, ld = a.W
  for (int64_t e = tid; e < (int64_t)NB * rest; e += nt) {
    const int j = (int)(e / rest), c = (int)(e % rest);
    P[(int64_t)j * a.W + c] = Tb[(int64_t)piv[j] * ld + k0 + NB + c];
  }
  if (tid < NB) a.perm[(int64_t)b * a.perm_bs + k0 + tid] = piv[tid];
  for (int r = tid; r < Mp; r += nt) gflags[r] = fl[r] ? 1 : 0;
  if (tid == 0 && sh_sing && a.sing && a.sing[b] == 0) a.sing[b] = a.sing_code;
}

}  // namespace

void launch_gje_panel(const PanelArgs& a, int batch, hipStream_t st) {
  RGF_CHECK(a.Mp % 64 == 0 && a.Mp <= MAXMP, RGF_EINVAL, "panel: Mp must be a multiple of 64, <= 2048");
  if (a.Mp <= 1024) {
    hipLaunchKernelGGL((gje_panel_kernel<1, 8>), dim3(batch), dim3(a.Mp), 0, st, a);
  } else {
    hipLaunchKernelGGL((gje_panel_kernel<2, 8>), dim3(batch), dim3(1024), 0, st, a);
  }
  RGF_HIP(hipGetLastError());
}

}  // namespace rgf
