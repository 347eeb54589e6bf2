// Fused factor-and-solve for small blocks: X = B^-1 Y for every batch entry
// in ONE launch, one workgroup per entry, by blocked Gauss-Jordan
// elimination with partial pivoting on the augmented [B | Y].
//
// For Mp <= 256 the batched LU (a latency-bound panel launch per 64 columns,
// 64-row products, trailing updates and two block triangular solves, about
// 20 launches per layer at Mp = 256) leaves most of the chip idle between
// short launches.  Here each workgroup owns one entry's B (Mp x Mp) and Y
// (Mp x nrhs) in global memory (L2 / MALL resident at these sizes) and walks
// the panels itself; several workgroups share a CU, so one entry's pivot
// search overlaps another's matrix-core updates.
//
// Per panel of NB = 16 columns [k0, k0 + NB):
//   1. pivots: the panel's columns of every row not yet pivoted are copied
//      into registers (one row per thread) and factored there, left to
//      right: per column the largest |Re| + |Im| among the candidates wins
//      (lowest row on ties), candidates are eliminated against it.  B in
//      global memory is not modified by this step.
//   2. D^-1: the NB pivot rows' eliminated entries are the L and U factors of
//      the panel's diagonal block D (pivot order); D^-1 = U^-1 L^-1 by
//      substitution, 8 lanes per column (the first 8 NB threads).
//   3. R = D^-1 A[pivots, rest] over the remaining columns of B and all
//      columns of Y, written in place into the pivot rows (matrix cores).
//   4. every other row i: A[i, rest] -= A[i, panel] R (matrix cores, K = NB),
//      rows above the panel included -- Gauss-Jordan, so after the last panel
//      the pivot rows of Y hold X.
// Rows never move: perm[j] is the row of Y that holds row j of X, and the
// consumers read X through that row map.  Exactly zero pivots record the
// entry's singular code (the arithmetic then runs into inf / NaN, which the
// trace reports); a NaN pivot has the largest key and is not a zero pivot.
//
// Cost: sum over panels of 8 NB (Mp + NB) (Mp - k0 - NB + nrhs) real flops on
// the matrix cores (about 12 Mp^3 for nrhs = Mp against 10.7 Mp^3 for LU and
// two triangular solves), plus NB columns of vector-unit pivoting per panel.
// At 126 VGPRs three workgroups share a CU.
#include "common.h"
#include "kernels.h"

namespace rgf {
namespace {

constexpr int NB = 16;   // panel width (32 would need twice the registers of the row copy and spill)
constexpr int NT = 256;  // threads: 4 wavefronts
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline v4d mfma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Pivot key: |Re| + |Im| >= 0 orders like its IEEE bit pattern; +1 keeps 0 for "no candidate".
__device__ inline uint64_t pkey(z64 v) { return (uint64_t)__double_as_longlong(zabs1(v)) + 1ull; }

__device__ inline uint64_t shfl_xor_u64(uint64_t x, int m) {
  const int lo = __shfl_xor((int)(uint32_t)x, m), hi = __shfl_xor((int)(uint32_t)(x >> 32), m);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// sum over each group of 8 lanes, identical in all of them
__device__ inline z64 sum8(z64 s) {
#pragma unroll
  for (int m = 1; m < 8; m <<= 1) s = zadd(s, zmake(__shfl_xor(s.x, m), __shfl_xor(s.y, m)));
  return s;
}

// The 16-column tile t of the remaining columns: B's columns [k0 + NB, MP) first, then Y's.
struct ColTile {
  z64* base;  // element (row, 0) of the tile is base[row * ld]
  int64_t ld;
};
template <int MP>
__device__ inline ColTile col_tile(z64* T, z64* Y, int nrhs, int k0, int t) {
  const int nb = (MP - k0 - NB) / 16;
  if (t < nb) return {T + k0 + NB + 16 * t, MP};
  return {Y + 16 * (t - nb), nrhs};
}

template <int MP>
__global__ __launch_bounds__(NT) void gj_kernel(GjArgs a) {
  static_assert(MP % NB == 0 && MP % 64 == 0 && MP <= NT, "one row per thread in the pivot phase");
  const int b = blockIdx.x;
  if (a.skip && a.skip[b]) return;
  z64* T = a.T + (int64_t)b * a.tbs;
  z64* Y = a.Y + (int64_t)b * a.ybs;
  const int nrhs = a.nrhs;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  __shared__ z64 slot[2][4][NB];      // each wavefront's candidate winner's panel row (two sets)
  __shared__ uint64_t wkey[2][4];
  __shared__ int wrow[2][4];
  __shared__ z64 LU[NB][NB + 1];      // pivot rows after elimination: L (c < j), U (c >= j)
  __shared__ z64 Dinv[NB][NB + 1];    // (L U)^-1
  __shared__ int prows[NB];           // row of pivot j of this panel
  __shared__ unsigned char curpiv[MP];
  __shared__ int s_sing;
  if (tid == 0) s_sing = 0;

  const int r = tid;  // this thread's row in the pivot phase
  const bool have = r < MP;
  bool used = false;  // the row pivoted in an earlier panel
  for (int k0 = 0; k0 < MP; k0 += NB) {
    // ---------------- 1. pivots of the panel, in registers ----------------
    z64 v[NB];
    bool cand = have && !used;
    if (have) {
      curpiv[r] = 0;
      const z64* src = T + (int64_t)r * MP + k0;
#pragma unroll
      for (int c = 0; c < NB; ++c) v[c] = src[c];
    } else {
#pragma unroll
      for (int c = 0; c < NB; ++c) v[c] = zmake(0.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int buf = j & 1;
      uint64_t wk = cand ? pkey(v[j]) : 0ull;
      int wr = cand ? r : 0x7fffffff;
#pragma unroll
      for (int m = 32; m > 0; m >>= 1) {
        const uint64_t ok = shfl_xor_u64(wk, m);
        const int orow = __shfl_xor(wr, m);
        if (ok > wk || (ok == wk && orow < wr)) {
          wk = ok;
          wr = orow;
        }
      }
      // the owner of the wavefront's winner publishes its panel row
      if (cand && r == wr) {
#pragma unroll
        for (int c = 0; c < NB; ++c) slot[buf][wave][c] = v[c];
      }
      if (lane == 0) {
        wkey[buf][wave] = wk;
        wrow[buf][wave] = wr;
      }
      __syncthreads();
      uint64_t gk = wkey[buf][0];
      int gr = wrow[buf][0], gw = 0;
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        const uint64_t k = wkey[buf][w];
        const int rw = wrow[buf][w];
        if (k > gk || (k == gk && rw < gr)) {
          gk = k;
          gr = rw;
          gw = w;
        }
      }
      if (tid == 0 && gk <= 1ull) s_sing = 1;  // key 1: an exact zero (a square system has a candidate)
      if (cand && r == gr) {
        cand = false;
        used = true;
        curpiv[r] = 1;
        prows[j] = r;
#pragma unroll
        for (int c = 0; c < NB; ++c) LU[j][c] = v[c];
      } else if (cand) {
        const z64* pv = slot[buf][gw];
        const z64 m = zmul(v[j], zinv(pv[j]));
        v[j] = m;
        // the pivot row is read from LDS four entries at a time (the fence keeps the compiler
        // from hoisting all of them, which would double the registers of the row copy)
#pragma unroll
        for (int c = j + 1; c < NB; ++c) {
          v[c] = zfms(m, pv[c], v[c]);
          if ((c & 3) == 3) __asm__ volatile("" ::: "memory");
        }
      }
    }
    __syncthreads();  // LU, prows, curpiv complete

    // ---------------- 2. D^-1 = U^-1 L^-1, 8 lanes per column ----------------
    if (tid < 8 * NB) {  // whole 8-lane groups, one per column
      const int c = tid >> 3, q = tid & 7;
      constexpr int H = NB / 8;
      z64 x[H], y[H];
#pragma unroll
      for (int h = 0; h < H; ++h) {
        x[h] = zmake(q + 8 * h == c ? 1.0 : 0.0, 0.0);
        y[h] = zmake(0.0, 0.0);
      }
      for (int i = c + 1; i < NB; ++i) {  // unit lower: x_i = -sum_{k < i} L[i][k] x_k
        z64 s = zmake(0.0, 0.0);
#pragma unroll
        for (int h = 0; h < H; ++h)
          if (q + 8 * h < i) s = zfma(LU[i][q + 8 * h], x[h], s);
        s = sum8(s);
        if ((i & 7) == q) {
#pragma unroll
          for (int h = 0; h < H; ++h)  // compile-time register index
            if (h == (i >> 3)) x[h] = zneg(s);
        }
      }
      for (int i = NB - 1; i >= 0; --i) {  // upper: y_i = (x_i - sum_{k > i} U[i][k] y_k) / U[i][i]
        z64 s = zmake(0.0, 0.0);
#pragma unroll
        for (int h = 0; h < H; ++h)
          if (q + 8 * h > i) s = zfma(LU[i][q + 8 * h], y[h], s);
        s = sum8(s);
        if ((i & 7) == q) {
          const z64 d = zinv(LU[i][i]);
#pragma unroll
          for (int h = 0; h < H; ++h)
            if (h == (i >> 3)) y[h] = zmul(zsub(x[h], s), d);
        }
      }
#pragma unroll
      for (int h = 0; h < H; ++h) Dinv[q + 8 * h][c] = y[h];
    }
    if (tid < NB) a.perm[(int64_t)b * a.perm_bs + k0 + tid] = prows[tid];
    __syncthreads();

    const int ntiles = (MP - k0 - NB) / 16 + nrhs / 16;
    const int kr = lane >> 4, lc = lane & 15;
    // ---------------- 3. R = D^-1 A[pivots, rest], in place ----------------
    for (int t = wave; t < ntiles; t += 4) {
      const ColTile ct = col_tile<MP>(T, Y, nrhs, k0, t);
      z64 bf[NB / 4];
#pragma unroll
      for (int s = 0; s < NB / 4; ++s) bf[s] = ct.base[(int64_t)prows[4 * s + kr] * ct.ld + lc];
#pragma unroll
      for (int h = 0; h < NB / 16; ++h) {
        v4d cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < NB / 4; ++s) {
          const z64 af = Dinv[16 * h + lc][4 * s + kr];
          cr = mfma64(af.x, bf[s].x, cr);
          cr = mfma64(-af.y, bf[s].y, cr);
          ci = mfma64(af.x, bf[s].y, ci);
          ci = mfma64(af.y, bf[s].x, ci);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) ct.base[(int64_t)prows[16 * h + kr + 4 * e] * ct.ld + lc] = zmake(cr[e], ci[e]);
      }
    }
    __syncthreads();  // R complete

    // ---------------- 4. A[i, rest] -= A[i, panel] R for every other row ----------------
    for (int strip = wave; strip < MP / 16; strip += 4) {
      const int i0 = strip * 16;
      const int ar = i0 + lc;
      const bool skip_row = curpiv[ar] != 0;
      z64 af[NB / 4];
#pragma unroll
      for (int s = 0; s < NB / 4; ++s)
        af[s] = skip_row ? zmake(0.0, 0.0) : T[(int64_t)ar * MP + k0 + 4 * s + kr];
      bool keep[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) keep[e] = curpiv[i0 + kr + 4 * e] == 0;
      for (int t = 0; t < ntiles; ++t) {
        const ColTile ct = col_tile<MP>(T, Y, nrhs, k0, t);
        z64 bf[NB / 4];
#pragma unroll
        for (int s = 0; s < NB / 4; ++s) bf[s] = ct.base[(int64_t)prows[4 * s + kr] * ct.ld + lc];
        v4d cr, ci;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const z64 c = ct.base[(int64_t)(i0 + kr + 4 * e) * ct.ld + lc];
          cr[e] = c.x;
          ci[e] = c.y;
        }
#pragma unroll
        for (int s = 0; s < NB / 4; ++s) {
          cr = mfma64(-af[s].x, bf[s].x, cr);
          cr = mfma64(af[s].y, bf[s].y, cr);
          ci = mfma64(-af[s].x, bf[s].y, ci);
          ci = mfma64(-af[s].y, bf[s].x, ci);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (keep[e]) ct.base[(int64_t)(i0 + kr + 4 * e) * ct.ld + lc] = zmake(cr[e], ci[e]);
      }
    }
    __syncthreads();  // the next panel reads the updated columns
  }
  if (tid == 0 && s_sing && a.sing && a.sing[b] == 0) a.sing[b] = a.sing_code;
}

}  // namespace

double launch_gj(const GjArgs& a, int batch, hipStream_t st) {
  if (batch <= 0) return 0.0;
  RGF_CHECK(a.Mp % 64 == 0 && a.Mp >= 64 && a.Mp <= GJ_MAX_MP, RGF_EINVAL, "gj: Mp must be 64..256, a multiple of 64");
  RGF_CHECK(a.nrhs > 0 && a.nrhs % 16 == 0, RGF_EINVAL, "gj: nrhs must be a positive multiple of 16");
  double flops = 0.0;
  for (int k0 = 0; k0 < a.Mp; k0 += NB)
    flops += 8.0 * NB * (a.Mp + NB) * (double)(a.Mp - k0 - NB + a.nrhs);
  flops *= batch;
  const bool prof = profiling();
  if (prof) profile_launch_begin(st, PC_FUSED);
  switch (a.Mp) {
    case 64: hipLaunchKernelGGL(gj_kernel<64>, dim3(batch), dim3(NT), 0, st, a); break;
    case 128: hipLaunchKernelGGL(gj_kernel<128>, dim3(batch), dim3(NT), 0, st, a); break;
    case 192: hipLaunchKernelGGL(gj_kernel<192>, dim3(batch), dim3(NT), 0, st, a); break;
    default: hipLaunchKernelGGL(gj_kernel<256>, dim3(batch), dim3(NT), 0, st, a); break;
  }
  RGF_HIP(hipGetLastError());
  if (prof) profile_launch_end(st, PC_FUSED, flops);
  return flops;
}

}  // namespace rgf
