// Driver of the batched blocked Gauss-Jordan solve: per 64-column panel one
// pivot/multiplier kernel (which also copies the pivot rows P) and one block
// product on the matrix cores,
//   T[:, rest] = T[:, rest] - m P    (Mp x rest, K = 64)
// where rest = the columns right of the panel (the remaining columns of B and
// every RHS column).
#include "common.h"
#include "kernels.h"

namespace rgf {

void gje_solve(const GjeBufs& g, z64* T, int W, int64_t bs, int Mp, int batch, const int32_t* skip,
               int32_t code, int prec, int tile, hipStream_t st) {
  const int64_t Pbs = (int64_t)64 * 3 * Mp;
  RGF_CHECK(W - Mp <= 2 * Mp && W > Mp, RGF_EINVAL, "gje: between 1 and 2 Mp right-hand sides");
  for (int k0 = 0; k0 < Mp; k0 += GJE_NB) {
    PanelArgs pa;
    pa.T = mat(T, bs, W);
    pa.Mp = Mp;
    pa.W = W;
    pa.k0 = k0;
    pa.scratch = g.scr;
    pa.scratch_bs = (int64_t)Mp * 64;
    pa.mult = g.mult;
    pa.mult_bs = (int64_t)Mp * 64;
    pa.prow = g.P;
    pa.prow_bs = Pbs;
    pa.perm = g.perm;
    pa.perm_bs = Mp;
    pa.flags = g.flags;
    pa.flags_bs = Mp;
    pa.sing = g.sing;
    pa.sing_code = code;
    pa.ctl.skip = skip;
    launch_gje_panel(pa, batch, st);
    const int rest = W - k0 - GJE_NB;
    if (rest <= 0) continue;
    GemmArgs u;
    u.rows = Mp;
    u.cols = rest;
    u.K = GJE_NB;
    u.batch = batch;
    u.a_kind = SRC_MAT;
    u.A = mat(g.mult, (int64_t)Mp * 64, 64);
    u.Af = form(nullptr, nullptr, 0, false, false, nullptr, 0.0);
    u.B = mat(g.P, Pbs, W);
    u.c_kind = SRC_MAT;
    u.Cin = mat(T + k0 + GJE_NB, bs, W);
    u.Cf = u.Af;
    u.C = u.Cin;
    u.alpha = -1.0;
    u.ctl.skip = skip;
    launch_gemm(u, prec, tile, st, 0);
  }
}

}  // namespace rgf
