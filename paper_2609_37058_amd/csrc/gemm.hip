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
// instruction; its output rows are interleaved by 4 across registers);
// the FP32 path converts operands to float when they are staged into LDS
// and uses v_mfma_f32_16x16x4 with FP32 accumulation.  Operator blocks
// z S - H (and z S^+ - H^+) are formed while staging, so the
// energy-dependent operands are never written to HBM.
//
// Work split: a BM x BN output tile per workgroup of WGM x WGN wavefronts,
// each wavefront owning a (BM/WGM) x (BN/WGN) block of 16x16 MFMA tiles.
// K advances BK complex columns per LDS stage, with two LDS stages: the
// next stage's global loads are issued before the current stage's MFMAs and
// written to the other LDS stage after them, so one barrier per stage
// suffices and HBM/L2 latency hides behind the (64-cycle) FP64 MFMAs.
// Products with a short inner dimension (the LU's trailing updates and
// 64-row blocks, K <= 128) spend as long reading and writing C as in their
// MFMAs.  With the 128 x 128 tile (8 wavefronts, BK = 16, 132 KB of LDS in
// FP64) one workgroup fills a CU and those phases cannot overlap, so such
// products take 128 x 64 (or 64 x 128) tiles of 4 wavefronts with BK = 8:
// 50 KB of LDS and two workgroups per CU, whose C traffic and MFMAs
// interleave.  Every output element still sums its K terms in the same order,
// so the choice of tile does not change a result.
// Shapes are multiples of 64; a 128-wide tile that overhangs the matrix
// leaves its outer wavefront blocks idle.  Tiles are handed out so that
// each of the 8 XCDs works on a contiguous range of (batch, row-tile,
// col-tile) ids: the operands of one batch entry stay in one XCD's L2.
#include <atomic>
#include <cstdlib>

#include "common.h"
#include "kernels.h"

namespace rgf {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// inner-dimension granularity every launch must respect (the largest stage depth)
constexpr int K_ALIGN = 16;

template <typename R>
struct CT;
template <>
struct CT<double> {
  typedef double2 c;
  typedef v4d acc;
  static constexpr bool exact = true;  // accumulates in FP64
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
  static constexpr bool exact = false;
  __device__ static c cvt(z64 v) { return make_float2((float)v.x, (float)v.y); }
  __device__ static acc mfma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output register v of lane l holds row 4 (l/16) + v
  __device__ static int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Row offsets (in elements, from the batch entry's base) of the 4 output rows r0 + out_row(lane, v)
// of a lane in one 16-row MFMA block row.  With a row gather the 4 index loads are issued
// together, so a block row waits for memory once instead of once per element.
template <typename R>
__device__ inline void frag_rows(const MatRef& m, int b, int r0, int lane, int (&ro)[4]) {
  if (m.rowidx) {
    const int32_t* ri = m.rowidx + (int64_t)b * m.ridx_bstride;
#pragma unroll
    for (int v = 0; v < 4; ++v) ro[v] = ri[r0 + CT<R>::out_row(lane, v)];
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) ro[v] = r0 + CT<R>::out_row(lane, v);
  }
}

// One element (r, c) of the Cin operand of batch entry b (FP32 epilogue; see c_quad).
__device__ inline z64 c_value(const GemmArgs& g, int b, int r, int c, z64 zc, int64_t coff) {
  if (g.c_kind == SRC_MAT) return g.Cin.p[mat_off(g.Cin, b, r, c)];
  z64 f = zmake(0.0, 0.0);
  if (r < g.Cf.M && c < g.Cf.M) {
    const int64_t o = coff + (int64_t)r * g.Cf.M + c;
    f = zform(zc, g.Cf.S[o], g.Cf.H[o]);
  }
  else if (g.Cf.pad_identity && r == c)
    f = zmake(1.0, 0.0);
  if (g.Cf.sub.p) {
    const z64 s = g.Cf.sub.p[mat_off(g.Cf.sub, b, r, c)];
    f = zmake(f.x + g.Cf.sub_sign * s.x, f.y + g.Cf.sub_sign * s.y);
  }
  return f;
}

// Gathered rows of the C operand's stored source for one block row: Cin for a matrix operand,
// the subtracted Sigma for a formed one (whose z S - H part is read at the logical rows).
template <typename R>
__device__ inline void c_src_rows(const GemmArgs& g, int b, int r0, int lane, int (&ro)[4]) {
  if (g.c_kind == SRC_MAT) frag_rows<R>(g.Cin, b, r0, lane, ro);
  else if (g.Cf.sub.p) frag_rows<R>(g.Cf.sub, b, r0, lane, ro);
}

// The Cin operand (a matrix, or a formed block z S - H with identity padding and an optional
// -+ Sigma, whose blocks start coff elements after Cf's: a grouped batch) at the lane's 4
// elements of one 16 x 16 block: rows r0 + out_row(lane, v), column c (FP64).  The quad's
// loads are all issued before a scheduling barrier and used after it; otherwise the scheduler,
// seeing the main loop's register pressure, issues each load just before its use and waits for
// it, one memory latency per element.  Out-of-range formed elements read element 0 of the
// blocks (when there are any) and discard it.  (The FP32 kernels, held to 128 VGPRs, have no
// room for grouped loads and read Cin one element at a time in their epilogue.)
template <typename R>
__device__ inline void c_quad(const GemmArgs& g, int b, int r0, int c, int lane, int64_t coff, const int (&ro)[4],
                              z64 (&cv)[4]) {
  if (g.c_kind == SRC_MAT) {
    const z64* base = g.Cin.p + (int64_t)b * g.Cin.bstride;
#pragma unroll
    for (int v = 0; v < 4; ++v) cv[v] = base[(int64_t)ro[v] * g.Cin.ld + c];
    __builtin_amdgcn_sched_barrier(0);
    return;
  }
  const int M = g.Cf.M;
  const z64* S = g.Cf.S + coff;
  const z64* H = g.Cf.H + coff;
  const z64* sb = g.Cf.sub.p ? g.Cf.sub.p + (int64_t)b * g.Cf.sub.bstride : nullptr;
  z64 sv[4], hv[4], sg[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = r0 + CT<R>::out_row(lane, v);
    const int64_t o = (r < M && c < M) ? (int64_t)r * M + c : 0;
    // an operand without blocks (M = 0: the identity, S = H = null) reads nothing
    sv[v] = M > 0 ? S[o] : zmake(0.0, 0.0);
    hv[v] = M > 0 ? H[o] : zmake(0.0, 0.0);
    if (sb) sg[v] = sb[(int64_t)ro[v] * g.Cf.sub.ld + c];
  }
  __builtin_amdgcn_sched_barrier(0);
  const z64 zc = zmake(g.Cf.E[b], g.Cf.eta);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = r0 + CT<R>::out_row(lane, v);
    z64 f = (r < M && c < M) ? zform(zc, sv[v], hv[v]) : zmake((g.Cf.pad_identity && r == c) ? 1.0 : 0.0, 0.0);
    if (sb) f = zmake(f.x + g.Cf.sub_sign * sg[v].x, f.y + g.Cf.sub_sign * sg[v].y);
    cv[v] = f;
  }
}

// How the A operand is staged: a per-batch matrix, a formed block z S - H,
// or the adjoint form z S^+ - H^+ (read transposed, so staged k-major).
enum { AK_MAT = 0, AK_FORM = 1, AK_FORM_CT = 2 };

// FP64: two wavefronts per SIMD (an 8-wavefront workgroup per CU, or two of 4 wavefronts).
// FP32 with a stored A operand: four, so that two 8-wavefront workgroups share a CU (at most
// 128 VGPRs); the formed-operand FP32 variants need more registers and stay at two.
template <typename R, int BM, int BN, int WGM, int WGN, int BK, int AK, int ROLE>
__global__ __launch_bounds__(64 * WGM * WGN, (!CT<R>::exact && AK == AK_MAT) ? 4 : 2) void zgemm_kernel(
    GemmArgs g, int tiles_m, int tiles_n) {
  typedef typename CT<R>::c cR;
  typedef typename CT<R>::acc accT;
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int EA = BM * BK / NT;  // staged A elements per thread
  constexpr int EB = BK * BN / NT;  // staged B elements per thread
  constexpr int LDA = BM + 1, LDB = BN + 1;
  constexpr bool FORM = AK != AK_MAT;
  static_assert(EA >= 1 && EB >= 1 && BK % EA == 0 && BN % EB == 0 && BM % EA == 0, "tile split");
  static_assert(64 % EA == 0 && 64 % EB == 0 && WTM % 16 == 0 && WTN % 16 == 0, "64-row groups");

  // two LDS stages: the next stage is stored while the current one feeds the MFMAs
  __shared__ cR As[2][BK * LDA];
  __shared__ cR Bs[2][BK * LDB];

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
  const int wm = wave / WGN, wn = wave % WGN;
  const int row0 = tm * BM, col0 = tn * BN;
  // rows and columns are multiples of 64, so a partial tile drops whole wavefront blocks
  const bool w_active = (row0 + wm * WTM < g.rows) && (col0 + wn * WTN < g.cols);

  accT accr[FM][FN], acci[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      accr[i][j] = accT{0, 0, 0, 0};
      acci[i][j] = accT{0, 0, 0, 0};
    }

  // ---- A staging: row-major map (BK/EA threads per row); k-major for the adjoint form ----
  const int a_r = (AK == AK_FORM_CT) ? (tid % (BM / EA)) * EA : tid / (BK / EA);
  const int a_k = (AK == AK_FORM_CT) ? tid / (BM / EA) : (tid % (BK / EA)) * EA;
  // the thread's A rows lie in one 64-row group: valid or not as a whole
  const bool a_ok = row0 + a_r < g.rows;
  const z64* a_ptr = nullptr;  // MAT: element (a_r, a_k) at k0 = 0
  const z64 *a_s = nullptr, *a_h = nullptr;
  int a_M = 0;
  z64 zz = zmake(0.0, 0.0);
  if constexpr (FORM) {
    a_M = g.Af.M;
    a_s = g.Af.S + form_group_off(g.Af, b);
    a_h = g.Af.H + form_group_off(g.Af, b);
    zz = zmake(g.Af.E[b], g.Af.eta);
  } else {
    a_ptr = g.A.p + mat_off(g.A, b, a_ok ? row0 + a_r : 0, a_k);
  }
  const bool a_pad = FORM && g.Af.pad_identity;
  // ---- B staging: k-major map ----
  const int b_k = tid / (BN / EB);
  const int b_c = (tid % (BN / EB)) * EB;
  const bool b_ok = col0 + b_c < g.cols;
  const z64* b_base = g.B.p + b * g.B.bstride + (b_ok ? col0 + b_c : 0);
  const int32_t* b_ridx = g.B.rowidx ? g.B.rowidx + (int64_t)b * g.B.ridx_bstride : nullptr;

  // Staging registers.  Formed operands keep the raw S and H entries here and
  // form z S - H when the stage is written to LDS, so no load waits on another.
  z64 ra[EA], rh[FORM ? EA : 1], rb[EB];
  int b_row = b_ridx ? b_ridx[b_k] : 0;  // gathered row of B for the stage being loaded

#define RGF_GEMM_LOAD(k0)                                                          \
  do {                                                                             \
    if constexpr (AK == AK_MAT) {                                                  \
      _Pragma("unroll") for (int e = 0; e < EA; ++e) ra[e] = a_ptr[(k0) + e];      \
    } else if constexpr (AK == AK_FORM_CT) {                                       \
      const int gk = (k0) + a_k;                                                   \
      _Pragma("unroll") for (int e = 0; e < EA; ++e) {                             \
        const int gr = row0 + a_r + e;                                             \
        const int64_t o = (gr < a_M && gk < a_M) ? (int64_t)gk * a_M + gr : 0;     \
        ra[e] = a_s[o];                                                            \
        rh[e] = a_h[o];                                                            \
      }                                                                            \
    } else {                                                                       \
      const int gr = row0 + a_r;                                                   \
      _Pragma("unroll") for (int e = 0; e < EA; ++e) {                             \
        const int gk = (k0) + a_k + e;                                             \
        const int64_t o = (gr < a_M && gk < a_M) ? (int64_t)gr * a_M + gk : 0;     \
        ra[e] = a_s[o];                                                            \
        rh[e] = a_h[o];                                                            \
      }                                                                            \
    }                                                                              \
    const int64_t brow_ = b_ridx ? (int64_t)b_row : (int64_t)((k0) + b_k);         \
    const z64* bp_ = b_base + brow_ * g.B.ld;                                      \
    _Pragma("unroll") for (int e = 0; e < EB; ++e) rb[e] = bp_[e];                 \
    /* gathered B rows: the next stage's row index is fetched one stage ahead, */  \
    /* so no load of a stage waits on an index load */                             \
    if (b_ridx && (k0) + BK < g.K) b_row = b_ridx[(k0) + BK + b_k];                \
  } while (0)

#define RGF_GEMM_STORE(buf, k0)                                                              \
  do {                                                                                       \
    cR* as_ = As[buf];                                                                       \
    cR* bs_ = Bs[buf];                                                                       \
    _Pragma("unroll") for (int e = 0; e < EA; ++e) {                                         \
      const int r_ = row0 + a_r + ((AK == AK_FORM_CT) ? e : 0);                              \
      const int k_ = (k0) + a_k + ((AK == AK_FORM_CT) ? 0 : e);                              \
      z64 v_ = ra[e];                                                                        \
      if constexpr (AK == AK_FORM_CT) {                                                      \
        v_ = (r_ < a_M && k_ < a_M) ? zform(zz, zconj(ra[e]), zconj(rh[e]))                  \
                                    : zmake((a_pad && r_ == k_) ? 1.0 : 0.0, 0.0);           \
      } else if constexpr (AK == AK_FORM) {                                                  \
        v_ = (r_ < a_M && k_ < a_M) ? zform(zz, ra[e], rh[e])                                \
                                    : zmake((a_pad && r_ == k_) ? 1.0 : 0.0, 0.0);           \
      }                                                                                      \
      if (!a_ok) v_ = zmake(0.0, 0.0);                                                       \
      if constexpr (AK == AK_FORM_CT) as_[a_k * LDA + a_r + e] = CT<R>::cvt(v_);             \
      else as_[(a_k + e) * LDA + a_r] = CT<R>::cvt(v_);                                      \
    }                                                                                        \
    _Pragma("unroll") for (int e = 0; e < EB; ++e)                                           \
        bs_[b_k * LDB + b_c + e] = CT<R>::cvt(b_ok ? rb[e] : zmake(0.0, 0.0));               \
  } while (0)

  // FP64 with alpha = +-1: the accumulators start at Cin / alpha, so the epilogue does not
  // wait for Cin loads.  (Issuing the first stage's operand loads before them would overlap the
  // two, but with both live the 128 x 128 kernels spill.)
  const bool c_pre = CT<R>::exact && g.c_kind != SRC_NONE && (g.alpha == 1.0 || g.alpha == -1.0);
  const int64_t c_off = form_group_off(g.Cf, b);
  const int r_w = row0 + wm * WTM, c_w = col0 + wn * WTN + (lane & 15);
  if (c_pre && w_active) {
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      int ro[4];
      c_src_rows<R>(g, b, r_w + 16 * i, lane, ro);
      if (g.c_kind == SRC_MAT) {  // a whole block row's loads in flight at once
        const z64* base = g.Cin.p + (int64_t)b * g.Cin.bstride;
        z64 cv[FN][4];
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) cv[j][v] = base[(int64_t)ro[v] * g.Cin.ld + c_w + 16 * j];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            accr[i][j][v] = (R)(g.alpha * cv[j][v].x);
            acci[i][j][v] = (R)(g.alpha * cv[j][v].y);
          }
      } else {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          z64 cv[4];
          c_quad<R>(g, b, r_w + 16 * i, c_w + 16 * j, lane, c_off, ro, cv);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            accr[i][j][v] = (R)(g.alpha * cv[v].x);
            acci[i][j][v] = (R)(g.alpha * cv[v].y);
          }
        }
      }
    }
  }

  const int nst = g.K / BK;
  RGF_GEMM_LOAD(0);
  RGF_GEMM_STORE(0, 0);
  __syncthreads();
  for (int s = 0; s < nst; ++s) {
    const int cur = s & 1;
    const bool more = s + 1 < nst;
    if (more) RGF_GEMM_LOAD((s + 1) * BK);
    if (w_active) {
      const cR* as = As[cur];
      const cR* bs = Bs[cur];
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const int kr = kk + (lane >> 4);
        cR af[FM], bf[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) af[i] = as[kr * LDA + wm * WTM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < FN; ++j) bf[j] = bs[kr * LDB + wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            accr[i][j] = CT<R>::mfma(af[i].x, bf[j].x, accr[i][j]);
            accr[i][j] = CT<R>::mfma(-af[i].y, bf[j].y, accr[i][j]);
            acci[i][j] = CT<R>::mfma(af[i].x, bf[j].y, acci[i][j]);
            acci[i][j] = CT<R>::mfma(af[i].y, bf[j].x, acci[i][j]);
          }
      }
    }
    // the other stage was last read before the previous barrier: safe to overwrite
    if (more) RGF_GEMM_STORE(cur ^ 1, (s + 1) * BK);
    __syncthreads();
  }
#undef RGF_GEMM_LOAD
#undef RGF_GEMM_STORE
  if (!w_active) return;

  // ---- epilogue: C = Cin + alpha * acc ----
  z64* cbase = g.C.p + (int64_t)b * g.C.bstride;
  if constexpr (CT<R>::exact) {
    // the output rows' gathered indices first (one wait for the whole tile), then a 16-row
    // block row at a time
    int ro[FM][4];
#pragma unroll
    for (int i = 0; i < FM; ++i) frag_rows<R>(g.C, b, r_w + 16 * i, lane, ro[i]);
    __builtin_amdgcn_sched_barrier(0);
    const bool c_post = !c_pre && g.c_kind != SRC_NONE;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      int rs[4];
      if (c_post) c_src_rows<R>(g, b, r_w + 16 * i, lane, rs);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        z64 cv[4];
        if (c_post) c_quad<R>(g, b, r_w + 16 * i, c_w + 16 * j, lane, c_off, rs, cv);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          z64 out = zmake(g.alpha * accr[i][j][v], g.alpha * acci[i][j][v]);
          if (c_post) out = zadd(out, cv[v]);
          cbase[(int64_t)ro[i][v] * g.C.ld + c_w + 16 * j] = out;
        }
      }
    }
  } else if (g.c_kind != SRC_FORM) {
    // FP32 with a stored Cin or none (the LU updates, U12 blocks and solves of the mixed form):
    // the output rows' indices per block row and one 16 x 16 block's Cin loads at a time, within
    // the 128-VGPR budget
    const bool has_c = g.c_kind == SRC_MAT;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      int rs[4], ro[4];
      if (has_c) frag_rows<R>(g.Cin, b, r_w + 16 * i, lane, rs);
      frag_rows<R>(g.C, b, r_w + 16 * i, lane, ro);
      const z64* cin = has_c ? g.Cin.p + (int64_t)b * g.Cin.bstride : nullptr;
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        z64 cv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (has_c) cv[v] = cin[(int64_t)rs[v] * g.Cin.ld + c_w + 16 * j];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          z64 out = zmake(g.alpha * (double)accr[i][j][v], g.alpha * (double)acci[i][j][v]);
          if (has_c) out = zadd(out, cv[v]);
          cbase[(int64_t)ro[v] * g.C.ld + c_w + 16 * j] = out;
        }
      }
    }
  } else {
    const z64 zc = (g.c_kind == SRC_FORM) ? zmake(g.Cf.E[b], g.Cf.eta) : zmake(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = r_w + i * 16 + CT<R>::out_row(lane, v);
          const int c = c_w + j * 16;
          z64 out = zmake(g.alpha * (double)accr[i][j][v], g.alpha * (double)acci[i][j][v]);
          if (g.c_kind != SRC_NONE) out = zadd(out, c_value(g, b, r, c, zc, c_off));
          g.C.p[mat_off(g.C, b, r, c)] = out;
        }
  }
}

template <typename R, int BM, int BN, int WGM, int WGN, int BK, int AK>
void launch_kind(const GemmArgs& g, dim3 grid, hipStream_t st, int role, int tm, int tn) {
  constexpr int NT = 64 * WGM * WGN;
  if (role == 1)
    hipLaunchKernelGGL((zgemm_kernel<R, BM, BN, WGM, WGN, BK, AK, 1>), grid, dim3(NT), 0, st, g, tm, tn);
  else
    hipLaunchKernelGGL((zgemm_kernel<R, BM, BN, WGM, WGN, BK, AK, 0>), grid, dim3(NT), 0, st, g, tm, tn);
}

template <typename R, int BM, int BN, int WGM, int WGN, int BK = 16>
void launch_cfg(const GemmArgs& g, hipStream_t st, int role) {
  const int tm = (g.rows + BM - 1) / BM, tn = (g.cols + BN - 1) / BN;
  // a product written in place over its B operand must keep each column block in one workgroup
  const bool in_place = g.C.p == g.B.p && g.C.rowidx == g.B.rowidx && g.C.bstride == g.B.bstride;
  RGF_CHECK(!(in_place && tm > 1), RGF_EINVAL, "gemm: in-place product spans several row tiles");
  const dim3 grid((unsigned)((int64_t)tm * tn * g.batch));
  if (g.a_kind != SRC_FORM)
    launch_kind<R, BM, BN, WGM, WGN, BK, AK_MAT>(g, grid, st, role, tm, tn);
  else if (g.Af.conj_t)
    launch_kind<R, BM, BN, WGM, WGN, BK, AK_FORM_CT>(g, grid, st, role, tm, tn);
  else
    launch_kind<R, BM, BN, WGM, WGN, BK, AK_FORM>(g, grid, st, role, tm, tn);
}

// Tile choice depends only on the shape and the requested tile size, never on
// the batch, so a result does not depend on which other energies share a launch.
template <typename R>
void launch_prec(const GemmArgs& g, int tile, hipStream_t st, int role) {
  if (tile >= 128 && g.K <= small_k_max()) {
    if (g.rows >= 128) launch_cfg<R, 128, 64, 2, 2, 8>(g, st, role);
    else launch_cfg<R, 64, 128, 1, 4, 8>(g, st, role);
  } else if (tile >= 128 && g.rows >= 128) {
    launch_cfg<R, 128, 128, 2, 4>(g, st, role);
  } else if (tile >= 128) {
    launch_cfg<R, 64, 128, 2, 4>(g, st, role);
  } else {
    launch_cfg<R, 64, 64, 2, 2>(g, st, role);
  }
}

}  // namespace

static std::atomic<int> g_small_k_max{-1};
int small_k_max() {
  int k = g_small_k_max.load(std::memory_order_relaxed);
  if (k < 0) {
    k = 128;
    if (const char* s = std::getenv("RGF_SMALLK_MAXK")) k = std::max(0, std::atoi(s));
    int expect = -1;
    if (!g_small_k_max.compare_exchange_strong(expect, k)) k = expect;
  }
  return k;
}
int set_small_k_max(int k) {
  const int prev = small_k_max();
  g_small_k_max.store(std::max(0, k));
  return prev;
}

double launch_gemm(const GemmArgs& g, int prec, int tile, hipStream_t st, int role) {
  if (g.rows <= 0 || g.cols <= 0 || g.batch <= 0) return 0.0;
  RGF_CHECK(g.K % K_ALIGN == 0, RGF_EINVAL, "gemm: K not a multiple of 16");
  RGF_CHECK(g.rows % 64 == 0 && g.cols % 64 == 0, RGF_EINVAL, "gemm: shape not tiled");
  const double flops = 8.0 * g.rows * (double)g.cols * g.K * g.batch;
  const bool prof = profiling();
  const int cls = prof ? profile_class(role, g.rows) : 0;
  if (prof) profile_launch_begin(st, cls);
  if (prec == PREC_F64) launch_prec<double>(g, tile, st, role);
  else launch_prec<float>(g, tile, st, role);
  RGF_HIP(hipGetLastError());
  if (prof) profile_launch_end(st, cls, flops);
  return flops;
}

}  // namespace rgf
