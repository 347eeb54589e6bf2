// Driver of the batched blocked LU with partial pivoting and of the two
// block triangular solves that follow it.
//
// Factorisation in pairs of 64-column panels a, b (one panel kernel each):
//   B[piv_a, b]    = La^-1 B[piv_a, b];  B[cand_a, b] -= B[cand_a, a] B[piv_a, b]
//   panel b, then for the columns r right of the pair
//   B[piv_a, r]    = La^-1 B[piv_a, r];  B[piv_b, r] -= B[piv_b, a] B[piv_a, r]
//   B[piv_b, r]    = Lb^-1 B[piv_b, r]
//   B[cand_b, r]  -= B[cand_b, a b] B[piv_ab, r]    trailing update, K = 128
// over the candidate rows only (their ascending list comes from the panel
// kernel), so the trailing work shrinks as the factorisation proceeds.
// Solves, left-looking by 128-row blocks, so each block of the result is
// written once with the whole inner dimension in one product:
//   forward  Y_k = L_kk^-1 (Y_k - L[k, <k] Y_<k)
//   backward Y_k = U_kk^-1 (Y_k - U[k, >k] Y_>k)
// with L[k, :] = B[perm[k-block], :] (multipliers) and U likewise; the
// 128 x 128 diagonal triangle is applied as two 64-row inverse blocks and one
// 64-row coupling product.
#include <map>
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace rgf {


// The side stream of a look-ahead factorisation on stream `st` (created once per device and
// stream, default priority), with its fork and join events; null while st captures a graph.
struct SideStream {
  hipStream_t st = nullptr;
  hipEvent_t fork = nullptr, far = nullptr;
};
static SideStream* side_stream(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  RGF_HIP(hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone) return nullptr;
  int dev = 0;
  RGF_HIP(hipGetDevice(&dev));
  static std::mutex mu;
  static std::map<std::pair<int, hipStream_t>, SideStream> sides;
  std::lock_guard<std::mutex> lk(mu);
  SideStream& s = sides[{dev, st}];
  if (!s.st) {
    RGF_HIP(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
    RGF_HIP(hipEventCreateWithFlags(&s.fork, hipEventDisableTiming));
    RGF_HIP(hipEventCreateWithFlags(&s.far, hipEventDisableTiming));
  }
  return &s;
}

void lu_factor(const LuBufs& g, z64* T, int64_t bs, int Mp, int batch, const int32_t* skip, int32_t code,
               int prec, int tile, hipStream_t st) {
  ProfSite site(PC_LU_UPDATE);
  const int64_t inv_bs = (int64_t)64 * Mp;
  {  // every row starts as a pivot candidate
    FillArgs f = fill_args(nomat(), 0, 0, FILL_ZERO);
    f.scale = 0.0;
    f.flags = g.flags;
    f.flags_bs = Mp;
    f.flags_n = Mp;
    f.ctl.skip = skip;
    launch_fill(f, batch, st);
  }
  // the panel kernel writes the list of rows still candidates into `cand`
  auto panel = [&](int k0, int32_t* cand) {
    LuPanelArgs pa;
    pa.T = mat(T, bs, Mp);
    pa.Mp = Mp;
    pa.k0 = k0;
    pa.linv = g.linv;
    pa.uinv = g.uinv;
    pa.inv_bs = inv_bs;
    pa.perm = g.perm;
    pa.perm_bs = Mp;
    pa.flags = g.flags;
    pa.flags_bs = Mp;
    pa.cand = cand;
    pa.cand_bs = Mp;
    pa.sing = g.sing;
    pa.sing_code = code;
    pa.ctl.skip = skip;
    pa.u_plain = g.exact_u ? 1 : 0;
    launch_lu_panel(pa, batch, st);
  };
  // B[piv(k0), c0 : c0 + ncols] = L11(k0)^-1 B[piv(k0), ...], in place (one row tile)
  auto u12 = [&](int k0, int c0, int ncols, hipStream_t s) {
    GemmArgs u = gemm_args(LU_NB, ncols, LU_NB, batch, skip);
    u.A = mat(g.linv + (int64_t)(k0 / LU_NB) * 64 * 64, inv_bs, 64);
    u.B = mat(T + c0, bs, Mp, g.perm + k0, Mp);
    u.C = u.B;
    launch_gemm(u, prec, tile, s, 0);
  };
  // B[rows, c0 : c0 + ncols] -= B[rows, k0 : k0 + K] B[piv(k0 .. k0 + K), c0 : ...]
  auto update = [&](const int32_t* rows, int nrows, int k0, int K, int c0, int ncols, hipStream_t s) {
    GemmArgs t = gemm_args(nrows, ncols, K, batch, skip);
    t.A = mat(T + k0, bs, Mp, rows, Mp);
    t.B = mat(T + c0, bs, Mp, g.perm + k0, Mp);
    t.c_kind = SRC_MAT;
    t.Cin = mat(T + c0, bs, Mp, rows, Mp);
    t.C = t.Cin;
    t.alpha = -1.0;
    launch_gemm(t, prec, tile, s, 0);
  };
  // Panels in pairs (k0, k0 + 64): the second panel's columns are updated by the first
  // alone, then the columns right of the pair by both at once (inner dimension 128),
  // which halves the trailing updates and their C traffic.
  //   Look-ahead: of the columns right of a pair, the next pair's 128 ("near") are updated on
  // st and the rest ("far") on the side stream, so the next pair's panels -- one latency-bound
  // workgroup per energy -- run beside the large far update instead of after it.  The far
  // update reads only this pair's multipliers, pivots and candidate list and writes only far
  // columns; the next pair touches only its near columns until it waits for the far update
  // (its own right-hand columns are this pair's far ones).  The candidate lists of consecutive
  // pairs alternate between cand and cand2, since the far update still reads this pair's list
  // while the next pair's panels write theirs.
  SideStream* side = g.cand2 ? side_stream(st) : nullptr;
  bool far_pending = false;
  auto join = [&]() {
    if (far_pending) RGF_HIP(hipStreamWaitEvent(st, side->far, 0));
    far_pending = false;
  };
  auto rest_ops = [&](int k0, int32_t* cand, int rest, int c, int ncols, hipStream_t s) {
    const int kb = k0 + LU_NB;
    u12(k0, c, ncols, s);
    update(g.perm + kb, LU_NB, k0, LU_NB, c, ncols, s);  // the second panel's pivot rows
    u12(kb, c, ncols, s);
    update(cand, rest, k0, 2 * LU_NB, c, ncols, s);      // candidates of the second panel
  };
  int k0 = 0, pair = 0;
  for (; k0 + 2 * LU_NB <= Mp; k0 += 2 * LU_NB, ++pair) {
    const int kb = k0 + LU_NB, c0 = k0 + 2 * LU_NB;
    const int rest = Mp - c0;
    int32_t* cand = (side && (pair & 1)) ? g.cand2 : g.cand;
    panel(k0, cand);
    u12(k0, kb, LU_NB, st);
    update(cand, Mp - kb, k0, LU_NB, kb, LU_NB, st);  // candidates of the first panel
    panel(kb, cand);
    if (rest <= 0) continue;
    join();  // this pair's right-hand columns were the previous pair's far ones
    const int near = side ? std::min(rest, 2 * LU_NB) : rest;
    rest_ops(k0, cand, rest, c0, near, st);
    if (rest > near) {
      RGF_HIP(hipEventRecord(side->fork, st));
      RGF_HIP(hipStreamWaitEvent(side->st, side->fork, 0));
      rest_ops(k0, cand, rest, c0 + near, rest - near, side->st);
      RGF_HIP(hipEventRecord(side->far, side->st));
      far_pending = true;
    }
  }
  join();
  if (k0 < Mp) panel(k0, (side && (pair & 1)) ? g.cand2 : g.cand);  // an odd panel count ends on a single panel
}

// Y_rows = Y_rows - A_rows Y_src  (rows x nrhs, inner dimension K)
static void update(GemmArgs base, z64* Yrows, int rows, const MatRef& A, z64* Ysrc, int K, int64_t ybs, int nrhs,
                   int prec, int tile, hipStream_t st) {
  if (K <= 0) return;
  GemmArgs o = base;
  o.rows = rows;
  o.cols = nrhs;
  o.K = K;
  o.A = A;
  o.B = mat(Ysrc, ybs, nrhs);
  o.c_kind = SRC_MAT;
  o.Cin = mat(Yrows, ybs, nrhs);
  o.C = o.Cin;
  o.alpha = -1.0;
  launch_gemm(o, prec, tile, st, 0);
}

// Y_rows <- U^-1 Y_rows in place for one 64 x 64 upper-triangular block U (row-major, batch
// stride u_bs) by back substitution: one right-hand-side column per thread.  U is staged in
// LDS (read as a broadcast), the thread's 64 unknowns in an LDS column of their own; each dot
// product runs as four partial sums, so the chain of dependent multiply-adds is a quarter long.
__global__ __launch_bounds__(64) void usolve_kernel(const z64* U, int64_t u_bs, z64* Y, int64_t ybs, int nrhs,
                                                    const int32_t* skip) {
  __shared__ z64 u[LU_NB * LU_NB];
  __shared__ z64 x[LU_NB * 64];
  const int b = blockIdx.y;
  if (skip && skip[b]) return;  // uniform over the workgroup
  const int t = threadIdx.x;
  const z64* Ub = U + (int64_t)b * u_bs;
  for (int e = t; e < LU_NB * LU_NB; e += 64) u[e] = Ub[e];
  const int c = blockIdx.x * 64 + t;
  const bool act = c < nrhs;
  z64* y = Y + (int64_t)b * ybs + (act ? c : 0);
  for (int i = 0; i < LU_NB; ++i) x[i * 64 + t] = act ? y[(int64_t)i * nrhs] : zmake(0.0, 0.0);
  __syncthreads();  // u complete; each thread touches only its own column of x
  for (int i = LU_NB - 1; i >= 0; --i) {
    z64 s0 = x[i * 64 + t], s1 = zmake(0.0, 0.0), s2 = s1, s3 = s1;
    const z64* ui = u + i * LU_NB;
    int j = i + 1;
    for (; j + 3 < LU_NB; j += 4) {
      s0 = zfms(ui[j], x[j * 64 + t], s0);
      s1 = zfms(ui[j + 1], x[(j + 1) * 64 + t], s1);
      s2 = zfms(ui[j + 2], x[(j + 2) * 64 + t], s2);
      s3 = zfms(ui[j + 3], x[(j + 3) * 64 + t], s3);
    }
    for (; j < LU_NB; ++j) s0 = zfms(ui[j], x[j * 64 + t], s0);
    x[i * 64 + t] = zmul(zadd(zadd(s0, s1), zadd(s2, s3)), zinv(ui[i]));
  }
  if (act)
    for (int i = 0; i < LU_NB; ++i) y[(int64_t)i * nrhs] = x[i * 64 + t];
}

static void usolve(z64* Yrows, const z64* U, int64_t u_bs, int64_t ybs, int nrhs, int batch, const int32_t* skip,
                   hipStream_t st) {
  hipLaunchKernelGGL(usolve_kernel, dim3((unsigned)((nrhs + 63) / 64), (unsigned)batch), dim3(64), 0, st, U, u_bs,
                     Yrows, ybs, nrhs, skip);
  RGF_HIP(hipGetLastError());
}

// Y_rows = D Y_rows in place (64 rows: one row tile, so each workgroup owns its columns)
static void diag(GemmArgs base, z64* Yrows, const z64* D, int64_t inv_bs, int64_t ybs, int nrhs, int prec, int tile,
                 hipStream_t st) {
  GemmArgs d = base;
  d.rows = LU_NB;
  d.cols = nrhs;
  d.K = LU_NB;
  d.A = mat(const_cast<z64*>(D), inv_bs, 64);
  d.B = mat(Yrows, ybs, nrhs);
  d.C = d.B;
  launch_gemm(d, prec, tile, st, 0);
}

void lu_solve(const LuBufs& g, z64* T, int64_t bs, int Mp, z64* Y, int64_t ybs, int nrhs, int batch,
              const int32_t* skip, int prec, int tile, hipStream_t st) {
  ProfSite site(PC_SOLVE);
  // Blocks of two panels (128 rows): one product over the whole inner dimension on
  // 128-row tiles, then the 2 x 2 block triangle with 64-row products.
  const int64_t inv_bs = (int64_t)64 * Mp;
  const int np = Mp / LU_NB;
  const GemmArgs base = gemm_args(LU_NB, nrhs, LU_NB, batch, skip);
  auto Yr = [&](int panel) { return Y + (int64_t)panel * LU_NB * nrhs; };
  auto Lrows = [&](int panel, int col0) { return mat(T + col0, bs, Mp, g.perm + panel * LU_NB, Mp); };
  auto Linv = [&](int panel) { return g.linv + (int64_t)panel * 64 * 64; };
  auto Uinv = [&](int panel) { return g.uinv + (int64_t)panel * 64 * 64; };
  // forward: L Z = Y
  for (int p = 0; p < np; p += 2) {
    const int two = (p + 1 < np) ? 2 : 1;
    const int r0 = p * LU_NB;
    update(base, Yr(p), two * LU_NB, Lrows(p, 0), Y, r0, ybs, nrhs, prec, tile, st);
    diag(base, Yr(p), Linv(p), inv_bs, ybs, nrhs, prec, tile, st);
    if (two == 2) {
      update(base, Yr(p + 1), LU_NB, Lrows(p + 1, r0), Yr(p), LU_NB, ybs, nrhs, prec, tile, st);
      diag(base, Yr(p + 1), Linv(p + 1), inv_bs, ybs, nrhs, prec, tile, st);
    }
  }
  // backward: U X = Z
  int p = np - 1;
  while (p >= 0) {
    const int two = (p >= 1) ? 2 : 1;
    const int q = p - two + 1;  // first panel of this block
    const int rend = (p + 1) * LU_NB;
    update(base, Yr(q), two * LU_NB, Lrows(q, rend), Yr(p + 1), Mp - rend, ybs, nrhs, prec, tile, st);
    if (g.exact_u) usolve(Yr(p), Uinv(p), inv_bs, ybs, nrhs, batch, skip, st);
    else diag(base, Yr(p), Uinv(p), inv_bs, ybs, nrhs, prec, tile, st);
    if (two == 2) {
      update(base, Yr(q), LU_NB, Lrows(q, p * LU_NB), Yr(p), LU_NB, ybs, nrhs, prec, tile, st);
      if (g.exact_u) usolve(Yr(q), Uinv(q), inv_bs, ybs, nrhs, batch, skip, st);
      else diag(base, Yr(q), Uinv(q), inv_bs, ybs, nrhs, prec, tile, st);
    }
    p -= two;
  }
}

}  // namespace rgf
