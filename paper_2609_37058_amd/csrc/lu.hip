// Batched blocked LU with partial pivoting: the panel step.
//
// B (Mp x Mp per batch) is factored in place in panels of 64 columns.
// Rows never move: a per-batch flag marks rows that already pivoted and
// perm[j] records the physical row that pivots column j.  In pivot order
// the factors are
//   L[j][m] = B[perm[j]][m]   (m < j, unit diagonal implied)
//   U[j][c] = B[perm[j]][c]   (c >= j, outside the diagonal 64 x 64 blocks)
// and the inverses of the diagonal blocks of L and U are kept per panel.
//
// For the panel K = [k0, k0+64) this kernel
//   1. factors the panel restricted to the rows not yet pivoted: per column
//      the largest |Re|+|Im| wins (lowest row index on ties), found by a
//      wavefront butterfly and a cross-wavefront pass in LDS; each
//      candidate row r is eliminated in registers (8-column sub-panels,
//      thread per row) and its multipliers l_r are written over its panel
//      entries; the rest of the panel is updated in place (rank 8 from
//      LDS-resident pivot rows);
//   2. inverts the diagonal blocks L11 (unit lower, |l| <= 1) and U11 in LDS
//      by Gauss-Jordan (no pivoting is needed for triangular blocks);
//   3. writes perm, the flags and the ascending list of rows still
//      candidates, which the trailing update of the matrix cores uses:
//        B[piv, rest]  = L11^-1 B[piv, rest]          (U12, in place)
//        B[cand, rest] -= B[cand, K] B[piv, rest]     (l_r U12)
#include "common.h"
#include "kernels.h"

namespace rgf {
namespace {

constexpr int NB = LU_NB;
constexpr int MAXMP = 2048;

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
__global__ __launch_bounds__(1024) void lu_panel_kernel(LuPanelArgs a) {
  constexpr int NSUB = NB / SW;
  const int b = blockIdx.x;
  if (a.ctl.skip && a.ctl.skip[b]) return;
  const int nt = blockDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
  const int Mp = a.Mp, k0 = a.k0;

  __shared__ z64 U[NB * NB];   // U11 rows, then U11^-1
  __shared__ z64 Lf[NB * NB];  // L11, then L11^-1
  __shared__ z64 Ls[SW * SW];
  __shared__ z64 colj[NB];
  __shared__ uint8_t fl[MAXMP];  // 0 candidate, 1 earlier pivot, 2 pivot of this panel
  __shared__ int piv[NB];
  __shared__ double rv[16];
  __shared__ int ri[16];
  __shared__ int wcount[16];
  __shared__ int sh_p, sh_sing, sh_base;

  uint8_t* gflags = a.flags + (int64_t)b * a.flags_bs;
  for (int r = tid; r < Mp; r += nt) fl[r] = gflags[r] ? 1 : 0;
  if (tid == 0) sh_sing = 0;
  __syncthreads();

  z64* Tb = a.T.p + (int64_t)b * a.T.bstride;
  const int64_t ld = a.T.ld;

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
      for (int j = 0; j < SW; ++j) v[i][j] = cand[i] ? Tb[(int64_t)r * ld + k0 + cb + j] : zmake(0.0, 0.0);
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
            Tb[(int64_t)p * ld + k0 + cb + m] = v[i][m];
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
    // multipliers over the sub-panel's entries
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      if (cand[i]) {
        const int r = tid + i * nt;
#pragma unroll
        for (int m = 0; m < SW; ++m) Tb[(int64_t)r * ld + k0 + cb + m] = v[i][m];
      }
    }
    if (s + 1 < NSUB) {
      const int c_begin = cb + SW;
      const int nrem = NB - c_begin;
      // pivot rows of this sub-panel: their U entries at the remaining panel columns
      if (tid < nrem) {
        const int c = c_begin + tid;
        for (int j = 0; j < SW; ++j) {
          z64 x = Tb[(int64_t)piv[cb + j] * ld + k0 + c];
          for (int m = 0; m < j; ++m) x = zfms(Ls[j * SW + m], U[(cb + m) * NB + c], x);
          U[(cb + j) * NB + c] = x;
        }
      }
      __syncthreads();
      // remaining candidate rows: rank-SW update of the rest of the panel, in place
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        if (cand[i]) {
          z64* row = Tb + (int64_t)(tid + i * nt) * ld + k0;
          for (int c = c_begin; c < NB; c += 8) {
            z64 x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = row[c + q];
#pragma unroll
            for (int m = 0; m < SW; ++m)
#pragma unroll
              for (int q = 0; q < 8; ++q) x[q] = zfms(v[i][m], U[(cb + m) * NB + c + q], x[q]);
#pragma unroll
            for (int q = 0; q < 8; ++q) row[c + q] = x[q];
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- diagonal blocks: L11 (unit lower) and U11, inverted in LDS ----
  for (int e = tid; e < NB * NB; e += nt) {
    const int j = e / NB, m = e % NB;
    Lf[e] = (m < j) ? Tb[(int64_t)piv[j] * ld + k0 + m] : zmake(m == j ? 1.0 : 0.0, 0.0);
    if (m < j) U[e] = zmake(0.0, 0.0);
  }
  __syncthreads();
  lds_invert(Lf, colj, tid, nt);
  lds_invert(U, colj, tid, nt);
  z64* li = a.linv + (int64_t)b * a.inv_bs + (int64_t)(k0 / NB) * NB * NB;
  z64* ui = a.uinv + (int64_t)b * a.inv_bs + (int64_t)(k0 / NB) * NB * NB;
  for (int e = tid; e < NB * NB; e += nt) {
    li[e] = Lf[e];
    ui[e] = U[e];
  }
  if (tid < NB) a.perm[(int64_t)b * a.perm_bs + k0 + tid] = piv[tid];
  for (int r = tid; r < Mp; r += nt) gflags[r] = fl[r] ? 1 : 0;
  if (tid == 0 && sh_sing && a.sing && a.sing[b] == 0) a.sing[b] = a.sing_code;

  // ---- ascending list of the rows still candidates ----
  int32_t* clist = a.cand + (int64_t)b * a.cand_bs;
  if (tid == 0) sh_base = 0;
  __syncthreads();
  for (int i = 0; i < RPT; ++i) {
    const int r = tid + i * nt;
    const bool c = (r < Mp) && fl[r] == 0;
    const unsigned long long m = __ballot(c);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[wave] = __popcll(m);
    __syncthreads();
    int off = sh_base;
    for (int w = 0; w < wave; ++w) off += wcount[w];
    if (c) clist[off + before] = r;
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int w = 0; w < nwaves; ++w) t += wcount[w];
      sh_base += t;
    }
    __syncthreads();
  }
}

}  // namespace

void launch_lu_panel(const LuPanelArgs& a, int batch, hipStream_t st) {
  RGF_CHECK(a.Mp % 64 == 0 && a.Mp <= MAXMP, RGF_EINVAL, "lu panel: Mp must be a multiple of 64, <= 2048");
  if (a.Mp <= 1024) {
    hipLaunchKernelGGL((lu_panel_kernel<1, 8>), dim3(batch), dim3(a.Mp), 0, st, a);
  } else {
    hipLaunchKernelGGL((lu_panel_kernel<2, 8>), dim3(batch), dim3(1024), 0, st, a);
  }
  RGF_HIP(hipGetLastError());
}

}  // namespace rgf
