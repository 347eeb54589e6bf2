// Batched blocked LU with partial pivoting: the panel step.
//
// B (Mp x Mp per batch) is factored in place in panels of 64 columns.
// Rows never move: a per-batch flag marks rows that already pivoted and
// perm[j] records the physical row that pivots column j.  In pivot order
// the factors are
//   L[j][m] = B[perm[j]][m]   (m < j, unit diagonal implied)
//   U[j][c] = B[perm[j]][c]   (c >= j)
// and the inverses of the diagonal 64 x 64 blocks of L and U are kept per
// panel for the block products that follow.
//
// For the panel K = [k0, k0+64) one workgroup per batch entry (up to 512
// threads; RPT = Mp / threads rows per thread) works in sub-panels of SW
// columns.  Rows still candidates are updated left-looking: a thread brings
// its row's SW sub-panel entries up to date from its own earlier multipliers
// and the U rows of the earlier pivots (in LDS), so no candidate row is
// written back until its multipliers are final.  Pivot rows are updated
// right-looking: once a sub-panel's SW pivots are known, their U rows at all
// remaining panel columns are formed at once (a product with the earlier U
// rows, then a forward substitution with their SW x SW unit-lower block).
//   Per column, each wavefront finds its largest |Re|+|Im| among its
//   candidate rows with DPP row steps and readlane (lowest row index on
//   ties); the owner of that row publishes the row's sub-panel entries in an
//   LDS slot; after ONE barrier every wavefront reduces the per-wavefront
//   winners itself, reads the pivot row from the winner's slot and eliminates
//   in registers.  The two slot sets alternate between columns.
// The diagonal blocks L11 and U11 are then inverted by substitution with 8
// lanes per column (one 8-lane DPP sum per row), and perm, the flags and the
// ascending list of rows still candidates are written.  The matrix cores then
// form U12 = L11^-1 B[piv, rest] in place and the candidates' trailing update
// (for pairs of panels, one update with both panels' multipliers; the driver
// in lu_solve.hip).  Only the multipliers of candidate rows and the U12 rows
// outside the panel are read back from B; the diagonal 64 x 64 block is
// represented by the two inverses.
#include "common.h"
#include "kernels.h"

namespace rgf {
namespace {

constexpr int NB = LU_NB;
constexpr int MAXMP = 2048;
constexpr int MAXW = 8;  // wavefronts per workgroup (512 threads)

// ---- cross-lane steps on DPP row patterns (VALU latency, no LDS permute) ----
// Within each row of 16 lanes: xor 1 and xor 2 (quad permutes), then the
// half-row and row mirrors.  Applied in this order to a commutative
// operation they leave every lane of the row with the same result.
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140;

template <int CTRL>
__device__ inline int dpp32(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ inline uint64_t dpp64(uint64_t x) {
  const int lo = dpp32<CTRL>((int)(uint32_t)x), hi = dpp32<CTRL>((int)(uint32_t)(x >> 32));
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
template <int CTRL>
__device__ inline double dppd(double x) {
  return __longlong_as_double((long long)dpp64<CTRL>((uint64_t)__double_as_longlong(x)));
}
template <int CTRL>
__device__ inline z64 dppz(z64 v) { return zmake(dppd<CTRL>(v.x), dppd<CTRL>(v.y)); }

__device__ inline uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }
__device__ inline uint64_t readlane64(uint64_t x, int l) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
// maximum over the 8 lanes of each half-row group, left in all of them
__device__ inline uint64_t max8(uint64_t k) {
  k = umax64(k, dpp64<DPP_XOR1>(k));
  k = umax64(k, dpp64<DPP_XOR2>(k));
  return umax64(k, dpp64<DPP_HALF_MIRROR>(k));
}
__device__ inline int min8(int r) {
  r = min(r, dpp32<DPP_XOR1>(r));
  r = min(r, dpp32<DPP_XOR2>(r));
  return min(r, dpp32<DPP_HALF_MIRROR>(r));
}
// maximum over the whole wavefront (uniform result)
__device__ inline uint64_t wave_max64(uint64_t k) {
  k = max8(k);
  k = umax64(k, dpp64<DPP_MIRROR>(k));
  return umax64(umax64(readlane64(k, 0), readlane64(k, 16)), umax64(readlane64(k, 32), readlane64(k, 48)));
}
// Pivot key: |Re|+|Im| >= 0 orders like its IEEE bit pattern; +1 keeps 0 for "no candidate".
__device__ inline uint64_t pivot_key(z64 v) { return (uint64_t)__double_as_longlong(zabs1(v)) + 1ull; }

// sum over each group of 8 lanes (half rows), identical in all of them
__device__ inline z64 sum8(z64 s) {
  s = zadd(s, dppz<DPP_XOR1>(s));
  s = zadd(s, dppz<DPP_XOR2>(s));
  return zadd(s, dppz<DPP_HALF_MIRROR>(s));
}

// X = L^-1 (unit lower) or X = U^-1 (upper), NB x NB row-major in LDS, into the
// row-major global block `out`.  Column c is solved by 8 lanes (lane q holds
// x[m] for m = q (mod 8)); a row costs one 8-lane sum, and the next row's
// entries are read from LDS while the current one is reduced.
template <bool LOWER>
__device__ void tri_invert(const z64* A, const z64* dinv, z64* out, int tid, int nt) {
  constexpr int H = NB / 8;
  const int q = tid & 7;
  for (int c = tid >> 3; c < NB; c += nt >> 3) {
    z64 x[H];
#pragma unroll
    for (int h = 0; h < H; ++h) x[h] = zmake(0.0, 0.0);
#pragma unroll
    for (int h = 0; h < H; ++h)
      if (q + 8 * h == c) x[h] = LOWER ? zmake(1.0, 0.0) : dinv[c];
    const int i0 = LOWER ? c + 1 : c - 1, step = LOWER ? 1 : -1;
    const int n = LOWER ? NB - 1 - c : c;  // rows left to solve
    z64 a[H];
    if (n > 0) {
#pragma unroll
      for (int h = 0; h < H; ++h) a[h] = A[i0 * NB + q + 8 * h];
    }
    for (int k = 0, i = i0; k < n; ++k, i += step) {
      z64 s = zmake(0.0, 0.0);
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int m = q + 8 * h;
        const bool in = LOWER ? (m >= c && m < i) : (m > i && m <= c);
        if (in) s = zfma(a[h], x[h], s);
      }
      if (k + 1 < n) {
#pragma unroll
        for (int h = 0; h < H; ++h) a[h] = A[(i + step) * NB + q + 8 * h];
      }
      s = sum8(s);
      const z64 xi = LOWER ? zneg(s) : zneg(zmul(s, dinv[i]));
#pragma unroll
      for (int h = 0; h < H; ++h)
        if (q + 8 * h == i) x[h] = xi;
    }
#pragma unroll
    for (int h = 0; h < H; ++h) out[(q + 8 * h) * NB + c] = x[h];
  }
}

template <int RPT, int SW>
__global__ __launch_bounds__(512) void lu_panel_kernel(LuPanelArgs a) {
  constexpr int NSUB = NB / SW;
  const int b = blockIdx.x;
  if (a.ctl.skip && a.ctl.skip[b]) return;
  const int nt = blockDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
  const int Mp = a.Mp, k0 = a.k0;

  __shared__ z64 U[NB * NB];   // U11 rows in pivot order (row j = pivot of column k0 + j), all panel columns
  __shared__ z64 Lw[NB * NB];  // L11 rows in pivot order (strictly lower part)
  __shared__ z64 slot[2][MAXW][SW];
  __shared__ uint64_t skey[2][MAXW];
  __shared__ int sidx[2][MAXW];
  __shared__ z64 dinv[NB];
  __shared__ uint8_t fl[MAXMP];  // 0 candidate, 1 earlier pivot, 2 pivot of this panel
  __shared__ int piv[NB];
  __shared__ int wcount[MAXW];
  __shared__ int sh_sing, sh_base;

  uint8_t* gflags = a.flags + (int64_t)b * a.flags_bs;
  for (int r = tid; r < Mp; r += nt) fl[r] = gflags[r] ? 1 : 0;
  if (tid == 0) sh_sing = 0;
  __syncthreads();
  z64* Tb = a.T.p + (int64_t)b * a.T.bstride;
  const int64_t ld = a.T.ld;

  bool cand[RPT];
  z64 v[RPT * SW];  // the thread's rows' sub-panel entries, row-major
#pragma clang loop unroll(full)
  for (int i = 0; i < RPT; ++i) {
    const int r = tid + i * nt;
    cand[i] = (r < Mp) && (fl[r] == 0);
  }

  for (int s = 0; s < NSUB; ++s) {
    const int cb = SW * s;
    // ---- candidates: sub-panel entries brought up to date (left-looking) ----
#pragma clang loop unroll(full)
    for (int i = 0; i < RPT; ++i) {
      if (cand[i]) {
        const z64* row = Tb + (int64_t)(tid + i * nt) * ld + k0;
#pragma clang loop unroll(full)
        for (int t = 0; t < SW; ++t) v[i * SW + (t)] = row[cb + t];
        if constexpr (RPT == 1) {
          // one row per thread leaves registers to fetch the next 8 multipliers
          // while the current 8 are applied
          z64 ln[8];
          if (cb > 0) {
#pragma clang loop unroll(full)
            for (int m = 0; m < 8; ++m) ln[m] = row[m];
          }
          for (int m0 = 0; m0 < cb; m0 += 8) {
            z64 l[8];
#pragma clang loop unroll(full)
            for (int m = 0; m < 8; ++m) l[m] = ln[m];
            if (m0 + 8 < cb) {
#pragma clang loop unroll(full)
              for (int m = 0; m < 8; ++m) ln[m] = row[m0 + 8 + m];
            }
#pragma clang loop unroll(full)
            for (int m = 0; m < 8; ++m)
#pragma clang loop unroll(full)
              for (int t = 0; t < SW; ++t) v[t] = zfms(l[m], U[(m0 + m) * NB + cb + t], v[t]);
          }
        } else {
          for (int m0 = 0; m0 < cb; m0 += 8) {
            z64 l[8];
#pragma clang loop unroll(full)
            for (int m = 0; m < 8; ++m) l[m] = row[m0 + m];
#pragma clang loop unroll(full)
            for (int m = 0; m < 8; ++m)
#pragma clang loop unroll(full)
              for (int t = 0; t < SW; ++t) v[i * SW + (t)] = zfms(l[m], U[(m0 + m) * NB + cb + t], v[i * SW + (t)]);
          }
        }
      }
    }
#pragma clang loop unroll(full)
    for (int j = 0; j < SW; ++j) {
      const int buf = j & 1;
      // ---- wavefront argmax of |Re|+|Im| over the candidate rows (lowest row on ties) ----
      uint64_t key = 0;
      int bi_local = 0;  // which of the thread's rows holds its best key (lowest on ties)
#pragma clang loop unroll(full)
      for (int i = 0; i < RPT; ++i) {
        const uint64_t k = cand[i] ? pivot_key(v[i * SW + (j)]) : 0ull;
        if (k > key) {
          key = k;
          bi_local = i;
        }
      }
      const uint64_t wmax = wave_max64(key);
      // rows tid + i*nt: every row of share i lies below every row of share i+1,
      // and within a share lower lanes hold lower rows
      int bi = 0x7fffffff;
#pragma clang loop unroll(full)
      for (int i = RPT - 1; i >= 0; --i) {
        const unsigned long long m = __ballot(key == wmax && wmax != 0 && bi_local == i);
        if (m) bi = (wave << 6) + (int)__builtin_ctzll(m) + i * nt;
      }
      // the owner of the wavefront's winner publishes its sub-panel row
#pragma clang loop unroll(full)
      for (int i = 0; i < RPT; ++i) {
        if (cand[i] && tid + i * nt == bi) {
#pragma clang loop unroll(full)
          for (int t = 0; t < SW; ++t) slot[buf][wave][t] = v[i * SW + (t)];
        }
      }
      if (lane == 0) {
        skey[buf][wave] = wmax;
        sidx[buf][wave] = bi;
      }
      __syncthreads();
      // ---- every wavefront reduces the per-wavefront winners itself ----
      const uint64_t wk = lane < nwaves ? skey[buf][lane] : 0ull;
      const int wr = lane < nwaves ? sidx[buf][lane] : 0x7fffffff;
      const uint64_t gk = readlane64(max8(wk), 0);
      const int gi = __builtin_amdgcn_readfirstlane(min8((wk == gk && lane < 8) ? wr : 0x7fffffff));
      // wavefront that owns the winning row: the lowest lane holding it (lane w = wavefront w)
      const unsigned long long wmask = __ballot(lane < nwaves && wr == gi);
      const int gw = wmask ? (int)__builtin_ctzll(wmask) : 0;
      const int p = (gi < Mp) ? gi : 0;  // a square system always has a candidate left
      const z64* u = slot[buf][gw];  // the pivot row's sub-panel entries (LDS broadcast reads)
      if (tid == 0) {
        piv[cb + j] = p;
        // key 1 is an exact zero (|Re|+|Im| = +0); a NaN pivot has the largest key and is not
        // a zero pivot: it reaches T, which reports it as non-finite
        if (gk <= 1ull) sh_sing = 1;
      }
      // ---- the pivot row leaves the candidates; its entries are U (t >= j) and L (t < j) ----
#pragma clang loop unroll(full)
      for (int i = 0; i < RPT; ++i) {
        if (cand[i] && tid + i * nt == p) {
          cand[i] = false;
          fl[p] = 2;
#pragma clang loop unroll(full)
          for (int t = 0; t < SW; ++t) {
            if (t >= j) U[(cb + j) * NB + cb + t] = v[i * SW + (t)];
            else Lw[(cb + j) * NB + cb + t] = v[i * SW + (t)];
          }
        }
      }
      // ---- elimination in registers ----
      const z64 inv = zinv(u[j]);
#pragma clang loop unroll(full)
      for (int i = 0; i < RPT; ++i) {
        if (cand[i]) {
          const z64 l = zmul(v[i * SW + (j)], inv);
          v[i * SW + (j)] = l;
#pragma clang loop unroll(full)
          for (int t = j + 1; t < SW; ++t) v[i * SW + (t)] = zfms(l, u[t], v[i * SW + (t)]);
        }
      }
    }
    // multipliers of this sub-panel
#pragma clang loop unroll(full)
    for (int i = 0; i < RPT; ++i) {
      if (cand[i]) {
        const int64_t ro = (int64_t)(tid + i * nt) * ld + k0 + cb;
#pragma clang loop unroll(full)
        for (int m = 0; m < SW; ++m) Tb[ro + m] = v[i * SW + (m)];
      }
    }
    __syncthreads();  // piv[] of this sub-panel, Lw/U entries of its pivots
    // ---- this sub-panel's pivot rows: L entries of earlier sub-panels, then U rows ----
    for (int e = tid; e < SW * cb; e += nt) {
      const int j = e / cb, m = e % cb;
      Lw[(cb + j) * NB + m] = Tb[(int64_t)piv[cb + j] * ld + k0 + m];
    }
    __syncthreads();
    const int c_begin = cb + SW;
    const int nrem = NB - c_begin;
    if (nrem > 0) {
      // U[cb+j][c] = B[p_j][c] - sum_{m<cb} L[cb+j][m] U[m][c] for c >= c_begin
      for (int e = tid; e < SW * nrem; e += nt) {
        const int j = e / nrem, c = c_begin + e % nrem;
        z64 x = Tb[(int64_t)piv[cb + j] * ld + k0 + c];
        for (int m = 0; m < cb; ++m) x = zfms(Lw[(cb + j) * NB + m], U[m * NB + c], x);
        U[(cb + j) * NB + c] = x;
      }
      __syncthreads();
      // ... then the forward substitution with the sub-panel's unit-lower block
      if (tid < nrem) {
        const int c = c_begin + tid;
        z64 x[SW];
#pragma clang loop unroll(full)
        for (int j = 0; j < SW; ++j) x[j] = U[(cb + j) * NB + c];
#pragma clang loop unroll(full)
        for (int j = 1; j < SW; ++j) {
#pragma clang loop unroll(full)
          for (int m = 0; m < j; ++m) x[j] = zfms(Lw[(cb + j) * NB + cb + m], x[m], x[j]);
          U[(cb + j) * NB + c] = x[j];
        }
      }
      __syncthreads();
    }
  }

  // ---- diagonal blocks: unit diagonal of L11, zero lower part of U11 ----
  for (int e = tid; e < NB * NB; e += nt) {
    const int j = e / NB, m = e % NB;
    if (m >= j) Lw[e] = zmake(m == j ? 1.0 : 0.0, 0.0);
    else U[e] = zmake(0.0, 0.0);
  }
  if (tid < NB) dinv[tid] = zinv(U[tid * NB + tid]);
  __syncthreads();
  z64* li = a.linv + (int64_t)b * a.inv_bs + (int64_t)(k0 / NB) * NB * NB;
  z64* ui = a.uinv + (int64_t)b * a.inv_bs + (int64_t)(k0 / NB) * NB * NB;
  tri_invert<true>(Lw, dinv, li, tid, nt);
  if (a.u_plain) {
    for (int e = tid; e < NB * NB; e += nt) ui[e] = U[e];
  } else {
    tri_invert<false>(U, dinv, ui, tid, nt);
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
  // whole wavefronts only: the butterflies and the per-wavefront slots assume full waves
  auto threads = [&](int rpt) { return (unsigned)round_up((a.Mp + rpt - 1) / rpt, 64); };
  const bool prof = profiling();
  const int cls = prof ? profile_panel_class() : 0;
  if (prof) profile_launch_begin(st, cls);
  if (a.Mp <= 512) {
    hipLaunchKernelGGL((lu_panel_kernel<1, 16>), dim3(batch), dim3(threads(1)), 0, st, a);
  } else if (a.Mp <= 1024) {
    hipLaunchKernelGGL((lu_panel_kernel<2, 16>), dim3(batch), dim3(threads(2)), 0, st, a);
  } else {
    hipLaunchKernelGGL((lu_panel_kernel<4, 8>), dim3(batch), dim3(threads(4)), 0, st, a);
  }
  RGF_HIP(hipGetLastError());
  if (prof) profile_launch_end(st, cls, 0.0);
}

}  // namespace rgf
