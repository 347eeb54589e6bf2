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
#include "common.h"
#include "kernels.h"

namespace rgf {


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
  auto panel = [&](int k0) {
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
    pa.cand = g.cand;
    pa.cand_bs = Mp;
    pa.sing = g.sing;
    pa.sing_code = code;
    pa.ctl.skip = skip;
    launch_lu_panel(pa, batch, st);
  };
  // B[piv(k0), c0 : c0 + ncols] = L11(k0)^-1 B[piv(k0), ...], in place (one row tile)
  auto u12 = [&](int k0, int c0, int ncols) {
    GemmArgs u = gemm_args(LU_NB, ncols, LU_NB, batch, skip);
    u.A = mat(g.linv + (int64_t)(k0 / LU_NB) * 64 * 64, inv_bs, 64);
    u.B = mat(T + c0, bs, Mp, g.perm + k0, Mp);
    u.C = u.B;
    launch_gemm(u, prec, tile, st, 0);
  };
  // B[rows, c0 : c0 + ncols] -= B[rows, k0 : k0 + K] B[piv(k0 .. k0 + K), c0 : ...]
  auto update = [&](const int32_t* rows, int nrows, int k0, int K, int c0, int ncols) {
    GemmArgs t = gemm_args(nrows, ncols, K, batch, skip);
    t.A = mat(T + k0, bs, Mp, rows, Mp);
    t.B = mat(T + c0, bs, Mp, g.perm + k0, Mp);
    t.c_kind = SRC_MAT;
    t.Cin = mat(T + c0, bs, Mp, rows, Mp);
    t.C = t.Cin;
    t.alpha = -1.0;
    launch_gemm(t, prec, tile, st, 0);
  };
  // Panels in pairs (k0, k0 + 64): the second panel's columns are updated by the first
  // alone, then the columns right of the pair by both at once (inner dimension 128),
  // which halves the trailing updates and their C traffic.
  int k0 = 0;
  for (; k0 + 2 * LU_NB <= Mp; k0 += 2 * LU_NB) {
    const int kb = k0 + LU_NB, c0 = k0 + 2 * LU_NB;
    const int rest = Mp - c0;
    panel(k0);
    u12(k0, kb, LU_NB);
    update(g.cand, Mp - kb, k0, LU_NB, kb, LU_NB);  // candidates of the first panel
    panel(kb);
    if (rest <= 0) continue;
    u12(k0, c0, rest);
    update(g.perm + kb, LU_NB, k0, LU_NB, c0, rest);  // the second panel's pivot rows
    u12(kb, c0, rest);
    update(g.cand, rest, k0, 2 * LU_NB, c0, rest);    // candidates of the second panel
  }
  if (k0 < Mp) panel(k0);  // an odd panel count ends on a single panel
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
    diag(base, Yr(p), Uinv(p), inv_bs, ybs, nrhs, prec, tile, st);
    if (two == 2) {
      update(base, Yr(q), LU_NB, Lrows(q, p * LU_NB), Yr(p), LU_NB, ybs, nrhs, prec, tile, st);
      diag(base, Yr(q), Uinv(q), inv_bs, ybs, nrhs, prec, tile, st);
    }
    p -= two;
  }
}

}  // namespace rgf
