// Batched complex block products on the CDNA4 matrix cores.
//
// C[b] = Cin[b] + alpha * opA[b] * opB[b] with complex operands, computed by
// the 4M method: four real products per complex multiply-add on split
// real/imaginary fragments,
//   Re C += Re A Re B - Im A Im B,   Im C += Re A Im B + Im A Re B,
// so a complex multiply-add costs 8 real flops (the LAWN 41 convention).
//
// Layout: operands stay interleaved complex (re, im) in HBM; one 16-byte
// load brings both parts of an element, and the LDS tiles keep them
// interleaved so one LDS read feeds the real and the imaginary MFMA.  The
// FP64 path uses v_mfma_f64_16x16x4 (16x16 output block, K = 4 per
// instruction; its output rows are interleaved by 4 across registers); the FP32 path converts operands to float when they are
// staged into LDS and uses v_mfma_f32_16x16x4 with FP32 accumulation.
// Operator blocks z S - H (and z S^+ - H^+) are formed while staging, so
// the energy-dependent operands are never written to HBM.
//
// Work split: 256 threads = 4 wavefronts in a 2x2 grid, each owning a
// (TILE/2) x (TILE/2) output block; K advances 16 complex columns per LDS
// stage with the next stage's global loads issued before the current
// stage's MFMAs.  Tiles are handed out so that each of the 8 XCDs works on
// a contiguous range of (batch, row-tile, col-tile) ids: the operands of
// one batch entry stay in one XCD's L2.
#include "common.h"
#include "kernels.h"

namespace rgf {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int BK = 16;
constexpr int GT = 256;

template <typename R>
struct CT;
template <>
struct CT<double> {
  typedef double2 c;
  typedef v4d acc;
  __device__ static c cvt(z64 v) { return v; }
  __device__ static acc mfma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output register v of lane l holds row l/16 + 4v (rows interleaved by 4)
  __device__ static int out_row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct CT<float> {
  typedef float2 c;
  typedef v4f acc;
  __device__ static c cvt(z64 v) { return make_float2((float)v.x, (float)v.y); }
  __device__ static acc mfma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output register v of lane l holds row 4 (l/16) + v
  __device__ static int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Element (r, k) of opA for batch b.
__device__ inline z64 load_a_mat(const GemmArgs& g, int b, int r, int k) {
  return g.A.p[mat_off(g.A, b, r, k)];
}

template <typename R, int TILE, int ROLE>
__global__ __launch_bounds__(GT) void zgemm_kernel(GemmArgs g, int tiles_m, int tiles_n) {
  typedef typename CT<R>::c cR;
  typedef typename CT<R>::acc accT;
  constexpr int PAD = 1;
  constexpr int LDT = TILE + PAD;
  constexpr int WT = TILE / 2;  // wave tile
  constexpr int F = WT / 16;    // 16x16 blocks per wave dimension
  constexpr int EPT = TILE * BK / GT;  // staged elements per thread per operand

  __shared__ cR As[BK * LDT];
  __shared__ cR Bs[BK * LDT];

  // ---- tile id, XCD-aware ----
  const int64_t total = (int64_t)tiles_m * tiles_n * g.batch;
  int64_t L = blockIdx.x;
  const int64_t per = total / 8;
  if (L < per * 8) L = (L % 8) * per + L / 8;
  const int tn = (int)(L % tiles_n);
  const int tm = (int)((L / tiles_n) % tiles_m);
  const int b = (int)(L / ((int64_t)tiles_n * tiles_m));
  if (g.ctl.skip && g.ctl.skip[b]) return;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int row0 = tm * TILE, col0 = tn * TILE;

  accT accr[F][F], acci[F][F];
#pragma unroll
  for (int i = 0; i < F; ++i)
#pragma unroll
    for (int j = 0; j < F; ++j) {
      accr[i][j] = accT{0, 0, 0, 0};
      acci[i][j] = accT{0, 0, 0, 0};
    }

  z64 ra[EPT], rb[EPT];
  const z64 zz = (g.a_kind == SRC_FORM) ? zmake(g.Af.E[b], g.Af.eta) : zmake(0.0, 0.0);

  // staging maps: "row-major" (4 threads x 4 elements per 16-wide row) and
  // "k-major" (16 threads x 4 elements along a TILE-wide row)
  auto load_a = [&](int k0) {
    if (g.a_kind == SRC_FORM && g.Af.conj_t) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int idx = tid + e * GT;
        const int k = idx / TILE, r = idx % TILE;
        const int gr = row0 + r, gk = k0 + k;
        z64 v = zmake(0.0, 0.0);
        if (gr < g.Af.M && gk < g.Af.M) {
          z64 s = g.Af.S[(int64_t)gk * g.Af.M + gr];
          z64 h = g.Af.H[(int64_t)gk * g.Af.M + gr];
          v = zform(zz, zconj(s), zconj(h));
        }
        ra[e] = v;
      }
    } else {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int idx = tid + e * GT;
        const int r = idx / BK, k = idx % BK;
        const int gr = row0 + r, gk = k0 + k;
        z64 v;
        if (g.a_kind == SRC_FORM) {
          v = zmake(0.0, 0.0);
          if (gr < g.Af.M && gk < g.Af.M)
            v = zform(zz, g.Af.S[(int64_t)gr * g.Af.M + gk], g.Af.H[(int64_t)gr * g.Af.M + gk]);
        } else {
          v = load_a_mat(g, b, gr, gk);
        }
        ra[e] = v;
      }
    }
  };
  auto store_a = [&]() {
    if (g.a_kind == SRC_FORM && g.Af.conj_t) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int idx = tid + e * GT;
        As[(idx / TILE) * LDT + idx % TILE] = CT<R>::cvt(ra[e]);
      }
    } else {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int idx = tid + e * GT;
        As[(idx % BK) * LDT + idx / BK] = CT<R>::cvt(ra[e]);
      }
    }
  };
  auto load_b = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int idx = tid + e * GT;
      const int k = idx / TILE, c = idx % TILE;
      rb[e] = g.B.p[mat_off(g.B, b, k0 + k, col0 + c)];
    }
  };
  auto store_b = [&]() {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int idx = tid + e * GT;
      Bs[(idx / TILE) * LDT + idx % TILE] = CT<R>::cvt(rb[e]);
    }
  };

  load_a(0);
  load_b(0);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    __syncthreads();
    store_a();
    store_b();
    __syncthreads();
    if (k0 + BK < g.K) {
      load_a(k0 + BK);
      load_b(k0 + BK);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      cR af[F], bf[F];
#pragma unroll
      for (int i = 0; i < F; ++i) af[i] = As[kr * LDT + wm * WT + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < F; ++j) bf[j] = Bs[kr * LDT + wn * WT + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < F; ++i)
#pragma unroll
        for (int j = 0; j < F; ++j) {
          accr[i][j] = CT<R>::mfma(af[i].x, bf[j].x, accr[i][j]);
          accr[i][j] = CT<R>::mfma(-af[i].y, bf[j].y, accr[i][j]);
          acci[i][j] = CT<R>::mfma(af[i].x, bf[j].y, acci[i][j]);
          acci[i][j] = CT<R>::mfma(af[i].y, bf[j].x, acci[i][j]);
        }
    }
  }

  // ---- epilogue: C = Cin + alpha * acc ----
  const z64 zc = (g.c_kind == SRC_FORM) ? zmake(g.Cf.E[b], g.Cf.eta) : zmake(0.0, 0.0);
#pragma unroll
  for (int i = 0; i < F; ++i)
#pragma unroll
    for (int j = 0; j < F; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + wm * WT + i * 16 + CT<R>::out_row(lane, v);
        const int c = col0 + wn * WT + j * 16 + (lane & 15);
        z64 out = zmake(g.alpha * (double)accr[i][j][v], g.alpha * (double)acci[i][j][v]);
        if (g.c_kind == SRC_MAT) {
          out = zadd(out, g.Cin.p[mat_off(g.Cin, b, r, c)]);
        } else if (g.c_kind == SRC_FORM) {
          z64 f = zmake(0.0, 0.0);
          if (r < g.Cf.M && c < g.Cf.M)
            f = zform(zc, g.Cf.S[(int64_t)r * g.Cf.M + c], g.Cf.H[(int64_t)r * g.Cf.M + c]);
          else if (g.Cf.pad_identity && r == c)
            f = zmake(1.0, 0.0);
          if (g.Cf.sub.p) {
            z64 s = g.Cf.sub.p[mat_off(g.Cf.sub, b, r, c)];
            f = zmake(f.x + g.Cf.sub_sign * s.x, f.y + g.Cf.sub_sign * s.y);
          }
          out = zadd(out, f);
        }
        g.C.p[mat_off(g.C, b, r, c)] = out;
      }
}

template <typename R, int TILE>
void launch_t(const GemmArgs& g, hipStream_t st, int role) {
  const int tm = g.rows / TILE, tn = g.cols / TILE;
  const int64_t total = (int64_t)tm * tn * g.batch;
  if (role == 1)
    hipLaunchKernelGGL((zgemm_kernel<R, TILE, 1>), dim3((unsigned)total), dim3(GT), 0, st, g, tm, tn);
  else
    hipLaunchKernelGGL((zgemm_kernel<R, TILE, 0>), dim3((unsigned)total), dim3(GT), 0, st, g, tm, tn);
}

}  // namespace

double launch_gemm(const GemmArgs& g, int prec, int tile, hipStream_t st, int role) {
  if (g.rows <= 0 || g.cols <= 0 || g.batch <= 0) return 0.0;
  RGF_CHECK(g.K % BK == 0, RGF_EINVAL, "gemm: K not a multiple of 16");
  if (tile == 128 && (g.rows % 128 || g.cols % 128)) tile = 64;
  RGF_CHECK(g.rows % tile == 0 && g.cols % tile == 0, RGF_EINVAL, "gemm: shape not tiled");
  if (prec == PREC_F64) {
    if (tile == 128) launch_t<double, 128>(g, st, role);
    else launch_t<double, 64>(g, st, role);
  } else {
    if (tile == 128) launch_t<float, 128>(g, st, role);
    else launch_t<float, 64>(g, st, role);
  }
  RGF_HIP(hipGetLastError());
  return 8.0 * g.rows * (double)g.cols * g.K * g.batch;
}

}  // namespace rgf
