// Host-side driver of the batched transmission path for one chunk of
// energies (all launches stream-ordered on one HIP stream).
//
// Per energy the path is (z = E + i eta, A = z S - H, blocks padded to Mp):
//   decimation   eps [Xa Xb] = [alpha beta] (LU of eps, two block triangular
//                solves), then the four products [alpha; beta] [Xa Xb] in one
//                matrix-core launch and the elementwise update; repeated until
//                ||alpha||_F + ||beta||_F <= 1e-14 max(1, ||D||_F)
//   self-energy  Sigma_L = L_L (eps_L^-1 U_L), Sigma_R = U_R (eps_R^-1 L_R)
//   sweep        B_0 = A_00 - Sigma_L; for l = 0..N-2:
//                  X = B_l^-1 U_l                (LU of B_l, solves)
//                  W = X (l = 0), else W <- -W X
//                  B_{l+1} = A_{l+1} - L_{l+1} X (- Sigma_R on the last layer)
//                G_1N = -W B_{N-1}^-1
//   trace        T = Re sum (Gamma_L G_1N) .* conj(G_1N Gamma_R)
// Mixed precision (prec = FP32): the block products of the sweep, of the LU
// trailing updates and of the triangular solves run on the FP32 matrix cores
// with FP32 accumulation; pivot search, the diagonal-block inverses,
// decimation, self-energies and the trace stay in FP64, and the one explicit
// block inverse of the sweep, g = B_{N-1}^-1, gets one FP64 Newton-Schulz
// correction g <- g + g (I - B g) before G_1N = -W g.
// This is the first-row-propagator recursion of the recursive Green's
// function method written with solves instead of explicit inverses: per
// point-layer it costs an LU (8/3 M^3 real flops), two triangular solves
// with M right-hand sides (8 M^3) and two block products (16 M^3), against
// 40 M^3 when every g_i is inverted and multiplied out.  No per-layer state
// is kept beyond B, X and W, so memory per energy does not grow with N.
#include <algorithm>
#include <cstdlib>

#include "engine.h"

namespace rgf {

namespace {
constexpr int NBLK_EPT = 256 * 16;  // elements per sr_update block
}

Layout Layout::make(int Mp, int batch) {
  Layout l;
  l.Mp = Mp;
  l.batch = batch;
  const int64_t MM = (int64_t)Mp * Mp;
  l.nblk_sr = (int)((MM + NBLK_EPT - 1) / NBLK_EPT);
  size_t off = 0;
  auto take = [&](size_t n) {
    size_t o = off;
    off += (n + 255) / 256 * 256;
    return o;
  };
  const size_t Z = sizeof(z64);
  l.sig = take(4 * batch * MM * Z);
  l.un = take(12 * batch * MM * Z);
  l.linv = take((size_t)batch * 64 * Mp * Z);
  l.uinv = take((size_t)batch * 64 * Mp * Z);
  l.perm = take((size_t)batch * Mp * 4);
  l.cand = take((size_t)batch * Mp * 4);
  l.cand2 = take((size_t)batch * Mp * 4);
  l.flags = take((size_t)batch * Mp);
  l.ints = take((size_t)(4 * batch + 64) * 4);
  l.dbl = take((size_t)(batch + batch * l.nblk_sr * 2) * 8);
  l.energies = take((size_t)batch * 8);
  l.tout = take((size_t)batch * 8);
  l.iout = take((size_t)batch * 4);
  l.elead = take((size_t)batch * 8);
  l.erlead = take((size_t)batch * 8);
  l.bytes = off;
  return l;
}

// The sweep's solves at padded block sizes up to 192 take the fused factor-and-solve: measured
// against the batched LU and triangular solves (X = B^-1 U, 64 / 256 / 784 energies) it is
// 2.5-4.3x faster at Mp = 64, 1.4-2.0x at 128 and 1.04-1.26x at 192, but 0.72-0.80x at 256,
// where its K = 16 updates make it HBM-bound.  RGF_FUSED=0 in the environment selects the
// batched LU everywhere.
constexpr int FUSED_MAX_MP = 192;
// Look-ahead in the blocked LU (lu_factor) is opt-in: RGF_LOOKAHEAD=1 in the environment.
// Measured at Mp = 1024, 64 energies: the factorisation alone 9.67 -> 8.64 ms and a one-lane
// sweep +4.9%, but the default two-lane C4 run 1353 -> 1251 point-layers/s (there one lane's
// panels already overlap the other's products).
static bool lookahead_default() {
  const char* s = std::getenv("RGF_LOOKAHEAD");
  return s && std::atoi(s) == 1;
}
static bool fused_for(int Mp) {
  if (Mp > FUSED_MAX_MP) return false;
  const char* s = std::getenv("RGF_FUSED");
  return !(s && std::atoi(s) == 0);
}

Engine::Engine(char* arena, const Layout& lay, hipStream_t st, int prec, int M, const double* E, double eta,
               int32_t* host_active)
    : st_(st), prec_(prec), M_(M), Mp_(lay.Mp), B_(lay.batch), fused_(fused_for(lay.Mp)), E_(E), EL_(E), ER_(E),
      eta_(eta), host_active_(host_active) {
  MM_ = (int64_t)Mp_ * Mp_;
  nblk_sr_ = lay.nblk_sr;
  const int64_t U = (int64_t)B_ * MM_;
  z64* sig = reinterpret_cast<z64*>(arena + lay.sig);
  sigL_ = sig;
  sigR_ = sig + U;
  gamL_ = sig + 2 * U;
  gamR_ = sig + 3 * U;
  z64* un = reinterpret_cast<z64*>(arena + lay.un);
  // decimation view of the union region
  eps_ = un;
  epsL_ = un + U;
  epsR_ = un + 2 * U;
  AB_ = un + 3 * U;    // per batch 2 MM
  C_ = un + 5 * U;     // per batch 4 MM
  Tsr_ = un + 9 * U;   // per batch MM
  Ysr_ = un + 10 * U;  // per batch 2 MM
  // sweep view of the same region (used after both self-energies exist)
  T_ = un;
  Y_ = un + U;
  Wa_ = un + 2 * U;
  Wb_ = un + 3 * U;
  P_ = un + 4 * U;
  Z1_ = un + 5 * U;
  Z2_ = un + 6 * U;
  lu_.linv = reinterpret_cast<z64*>(arena + lay.linv);
  lu_.uinv = reinterpret_cast<z64*>(arena + lay.uinv);
  lu_.perm = reinterpret_cast<int32_t*>(arena + lay.perm);
  lu_.cand = reinterpret_cast<int32_t*>(arena + lay.cand);
  cand2_ = reinterpret_cast<int32_t*>(arena + lay.cand2);
  lu_.cand2 = lookahead_default() ? cand2_ : nullptr;
  lu_.flags = reinterpret_cast<uint8_t*>(arena + lay.flags);
  int32_t* ints = reinterpret_cast<int32_t*>(arena + lay.ints);
  done_l_ = ints;
  done_r_ = ints + B_;
  iters_ = ints + 2 * B_;
  sing_ = ints + 3 * B_;
  active_ = ints + 4 * B_;
  lu_.sing = sing_;
  double* dbl = reinterpret_cast<double*>(arena + lay.dbl);
  scale_ = dbl;
  partial_ = dbl + B_;
  RGF_HIP(hipMemsetAsync(sing_, 0, sizeof(int32_t) * B_, st_));
  RGF_HIP(hipMemsetAsync(done_l_, 0, sizeof(int32_t) * 2 * B_, st_));
}

MatRef Engine::mref(z64* p, int64_t ld, int64_t bstride, const int32_t* ridx) const {
  return mat(p, bstride, ld, ridx, ridx ? Mp_ : 0);
}

MatRef Engine::factor_solve(z64* T, z64* Y, int64_t yld, int64_t ybs, int nrhs, std::vector<FillArgs> rhs,
                            const int32_t* skip, int32_t code, int lp, int tp, int tile, bool fusable,
                            bool exact_u) {
  if (fused_ && fusable) {
    for (FillArgs& f : rhs) launch_fill(f, B_, st_);
    GjArgs a;
    a.T = T;
    a.tbs = MM_;
    a.Y = Y;
    a.ybs = ybs;
    a.nrhs = nrhs;
    a.Mp = Mp_;
    a.perm = lu_.perm;
    a.perm_bs = Mp_;
    a.sing = sing_;
    a.sing_code = code;
    a.skip = skip;
    launch_gj(a, B_, st_);
    return mref(Y, yld, ybs, lu_.perm);
  }
  LuBufs lu = lu_;
  lu.exact_u = exact_u;
  lu_factor(lu, T, MM_, Mp_, B_, skip, code, lp, tile, st_);
  for (FillArgs& f : rhs) {  // the right-hand sides in pivot order
    if (f.kind == FILL_MAT) {
      f.src.rowidx = lu_.perm;
      f.src.ridx_bstride = Mp_;
    } else {
      f.ridx = lu_.perm;
      f.ridx_bs = Mp_;
    }
    launch_fill(f, B_, st_);
  }
  lu_solve(lu, T, MM_, Mp_, Y, ybs, nrhs, B_, skip, tp, tile, st_);
  return mref(Y, yld, ybs);
}

double Engine::gemm(GemmArgs g, int prec, bool timed) {
  return launch_gemm(g, prec, tile_for(prec, Mp_), st_, timed ? 1 : 0);
}

void Engine::decimate(const rgf_lead& lead, int32_t* done, bool left) {
  ProfLead lead_scope;
  const int Mp = Mp_;
  const double* El = left ? EL_ : ER_;
  const int tile = tile_for(PREC_F64, Mp_);
  RGF_HIP(hipMemsetAsync(done, 0, sizeof(int32_t) * B_, st_));
  RGF_HIP(hipMemsetAsync(iters_, 0, sizeof(int32_t) * B_, st_));
  // eps = eps_L = eps_R = D (identity padding), alpha = U, beta = L
  FillArgs f = fill_args(mref(eps_, Mp, MM_), Mp, Mp, FILL_FORM);
  f.f = gform(form(lead.H00, lead.S00, M_, false, true, El, eta_));
  launch_fill(f, B_, st_);
  f = fill_args(mref(epsL_, Mp, MM_), Mp, Mp, FILL_MAT);
  f.src = mref(eps_, Mp, MM_);
  launch_fill(f, B_, st_);
  f.dst = mref(epsR_, Mp, MM_);
  launch_fill(f, B_, st_);
  f = fill_args(mref(AB_, Mp, 2 * MM_), Mp, Mp, FILL_FORM);
  f.f = gform(form(lead.H01, lead.S01, M_, false, false, El, eta_));
  launch_fill(f, B_, st_);
  f.dst = mref(AB_ + MM_, Mp, 2 * MM_);
  f.f.conj_t = 1;
  launch_fill(f, B_, st_);
  launch_frob_scale(mref(eps_, Mp, MM_), M_, M_, scale_, B_, st_);

  const int maxit = sr_maxit();
  const bool prof = profiling();
  const double flops0 = prof ? profile_thread_flops() : 0.0;
  int run = 0;  // iterations launched
  for (int it = 1; it <= maxit; ++it) {
    run = it;
    // [Xa Xb] = eps^-1 [alpha beta]
    FillArgs c = fill_args(mref(Tsr_, Mp, MM_), Mp, Mp, FILL_MAT);
    c.src = mref(eps_, Mp, MM_);
    c.ctl.skip = done;
    launch_fill(c, B_, st_);
    FillArgs ra = fill_args(mref(Ysr_, 2 * Mp, 2 * MM_), Mp, Mp, FILL_MAT);
    ra.src = mref(AB_, Mp, 2 * MM_);
    ra.ctl.skip = done;
    FillArgs rb = ra;
    rb.dst = mref(Ysr_ + Mp, 2 * Mp, 2 * MM_);
    rb.src = mref(AB_ + MM_, Mp, 2 * MM_);
    // near band extrema eps is ill-conditioned: the solves substitute with U's diagonal blocks
    const MatRef Xab = factor_solve(Tsr_, Ysr_, 2 * Mp, 2 * MM_, 2 * Mp, {ra, rb}, done, SING_LEAD, PREC_F64,
                                    PREC_F64, tile, false, true);
    // the four products [alpha; beta] [Xa Xb]
    GemmArgs g = gemm_args(2 * Mp, 2 * Mp, Mp, B_);
    g.A = mref(AB_, Mp, 2 * MM_);
    g.B = Xab;
    g.C = mref(C_, 2 * Mp, 4 * MM_);
    g.ctl.skip = done;
    gemm(g, PREC_F64, false);
    SrUpdateArgs u;
    u.Mp = Mp;
    u.C = mref(C_, 2 * Mp, 4 * MM_);
    u.eps = mref(eps_, Mp, MM_);
    u.epsL = mref(epsL_, Mp, MM_);
    u.epsR = mref(epsR_, Mp, MM_);
    u.AB = mref(AB_, Mp, 2 * MM_);
    u.partial = partial_;
    u.nblk = nblk_sr_;
    u.ctl.skip = done;
    launch_sr_update(u, B_, st_);
    RGF_HIP(hipMemsetAsync(active_, 0, sizeof(int32_t), st_));
    launch_sr_check(partial_, nblk_sr_, scale_, SR_TOL, it, done, iters_, active_, B_, st_);
    if ((it >= 12 && it % 4 == 0) || it == maxit) {
      RGF_HIP(hipMemcpyAsync(host_active_, active_, sizeof(int32_t), hipMemcpyDeviceToHost, st_));
      RGF_HIP(hipStreamSynchronize(st_));
      if (*host_active_ == 0) break;
    }
  }
  if (prof && run > 0) {
    // Every launch of the loop counted all B energies, but an energy stops at its convergence
    // check (the products of later iterations skip it): energy b ran iterations 1 .. iters[b].
    std::vector<int32_t> its(B_);
    RGF_HIP(hipMemcpyAsync(its.data(), iters_, sizeof(int32_t) * B_, hipMemcpyDeviceToHost, st_));
    RGF_HIP(hipStreamSynchronize(st_));
    double ran = 0.0;
    for (int32_t n : its) ran += std::min<int32_t>(std::max<int32_t>(n, 0), run);
    const double counted = profile_thread_flops() - flops0;
    profile_uncount_flops(PC_LEAD, counted * (1.0 - ran / ((double)run * B_)));
  }
}

void Engine::self_energy(const rgf_lead& lead, bool left, z64* out) {
  ProfLead lead_scope;
  const int Mp = Mp_;
  const int tile = tile_for(PREC_F64, Mp_);
  FillArgs f = fill_args(mref(Tsr_, Mp, MM_), Mp, Mp, FILL_MAT);
  f.src = mref(left ? epsL_ : epsR_, Mp, MM_);
  launch_fill(f, B_, st_);
  // RHS: U of the lead (left side) or L (right side)
  f = fill_args(mref(Ysr_, Mp, 2 * MM_), Mp, Mp, FILL_FORM);
  const double* El = left ? EL_ : ER_;
  f.f = gform(form(lead.H01, lead.S01, M_, /*conj_t=*/!left, false, El, eta_));
  const MatRef X =
      factor_solve(Tsr_, Ysr_, Mp, 2 * MM_, Mp, {f}, nullptr, SING_LEAD, PREC_F64, PREC_F64, tile, false, true);
  GemmArgs g = gemm_args(Mp, Mp, Mp, B_);
  g.a_kind = SRC_FORM;
  g.Af = gform(form(lead.H01, lead.S01, M_, /*conj_t=*/left, false, El, eta_));
  g.B = X;
  g.C = mref(out, Mp, MM_);
  gemm(g, PREC_F64, false);
}

void Engine::broadenings() {
  launch_broadening(mref(sigL_, Mp_, MM_), mref(gamL_, Mp_, MM_), Mp_, B_, st_);
  launch_broadening(mref(sigR_, Mp_, MM_), mref(gamR_, Mp_, MM_), Mp_, B_, st_);
}

void Engine::sweep_and_trace(const rgf_device& d, double* T, int32_t* info, bool same_leads) {
  const int Mp = Mp_;
  const int64_t M2 = (int64_t)M_ * M_;
  const int N = d.N;
  // mixed precision: which block products run on the FP32 matrix cores
  // (bit 0: sweep products, bit 1: LU trailing updates, bit 2: triangular solves)
  const int mask = prec_ != PREC_F64 ? mixed_parts() : 0;
  const int sp = (mask & 1) ? PREC_F32 : PREC_F64;
  const int lp = (mask & 2) ? PREC_F32 : PREC_F64;
  const int tp = (mask & 4) ? PREC_F32 : PREC_F64;
  const int tile = tile_for(sp, Mp_);
  MatRef X = mref(Y_, Mp, MM_);

  // B_0 = A_00 - Sigma_L (- Sigma_R when N = 1)
  FillArgs f = fill_args(mref(T_, Mp, MM_), Mp, Mp, FILL_FORM);
  f.f = gform(form(d.Hd, d.Sd, M_, false, true, E_, eta_));
  f.f.sub = mref(sigL_, Mp, MM_);
  f.f.sub_sign = -1.0;
  launch_fill(f, B_, st_);
  if (N == 1) {
    BatchCtl none;
    none.skip = nullptr;
    launch_axpy(mref(T_, Mp, MM_), mref(sigR_, Mp, MM_), -1.0, Mp, Mp, B_, none, st_);
  }
  z64* Wcur = Wa_;
  z64* Wnxt = Wb_;
  for (int l = 0; l + 1 < N; ++l) {
    // X = B_l^-1 U_l
    f = fill_args(mref(Y_, Mp, MM_), Mp, Mp, FILL_FORM);
    f.f = gform(form(d.Hu + l * M2, d.Su + l * M2, M_, false, false, E_, eta_));
    X = factor_solve(T_, Y_, Mp, MM_, Mp, {f}, nullptr, l + 1, lp, tp, tile, true);
    if (l == 0) {
      FillArgs c = fill_args(mref(Wcur, Mp, MM_), Mp, Mp, FILL_MAT);
      c.src = X;
      launch_fill(c, B_, st_);
    } else {
      GemmArgs g = gemm_args(Mp, Mp, Mp, B_);
      g.A = mref(Wcur, Mp, MM_);
      g.B = X;
      g.C = mref(Wnxt, Mp, MM_);
      g.alpha = -1.0;
      gemm(g, sp, true);
      std::swap(Wcur, Wnxt);
    }
    // B_{l+1} = A_{l+1} - L_{l+1} X (- Sigma_R on the last layer).  L_{l+1} = z S_u^+ - H_u^+
    // is stored per energy first (Z1 is free until the end of the sweep): formed inside the
    // product, its two shared-block loads per element cost more than the extra pass.
    launch_form_ct(gform(form(d.Hu + l * M2, d.Su + l * M2, M_, true, false, E_, eta_)), mref(Z1_, Mp, MM_), Mp,
                   B_, st_);
    GemmArgs g = gemm_args(Mp, Mp, Mp, B_);
    g.A = mref(Z1_, Mp, MM_);
    g.B = X;
    g.c_kind = SRC_FORM;
    g.Cf = gform(form(d.Hd + (l + 1) * M2, d.Sd + (l + 1) * M2, M_, false, true, E_, eta_));
    if (l + 2 == N) {
      g.Cf.sub = mref(sigR_, Mp, MM_);
      g.Cf.sub_sign = -1.0;
    }
    g.C = mref(T_, Mp, MM_);
    g.alpha = -1.0;
    gemm(g, sp, true);
  }
  // G_1N = -W B^-1  (B^-1 when N = 1)
  const bool refine = (lp | tp) != PREC_F64;
  if (refine) {  // keep B_{N-1} for the FP64 correction of its inverse
    FillArgs c = fill_args(mref(Z2_, Mp, MM_), Mp, Mp, FILL_MAT);
    c.src = mref(T_, Mp, MM_);
    launch_fill(c, B_, st_);
  }
  f = fill_args(mref(Y_, Mp, MM_), Mp, Mp, FILL_IDENTITY);
  X = factor_solve(T_, Y_, Mp, MM_, Mp, {f}, nullptr, N + 1, lp, tp, tile, true);
  MatRef ginv = X;
  if (refine) {
    // one Newton-Schulz step in FP64: g <- g + g (I - B g)
    GemmArgs r = gemm_args(Mp, Mp, Mp, B_);
    r.A = mref(Z2_, Mp, MM_);
    r.B = X;
    r.c_kind = SRC_FORM;
    r.Cf = form(nullptr, nullptr, 0, false, true, E_, eta_);  // identity
    r.C = mref(Z1_, Mp, MM_);
    r.alpha = -1.0;
    gemm(r, PREC_F64, false);
    GemmArgs c = gemm_args(Mp, Mp, Mp, B_);
    c.A = X;
    c.B = mref(Z1_, Mp, MM_);
    c.c_kind = SRC_MAT;
    c.Cin = X;
    c.C = mref(Z2_, Mp, MM_);
    gemm(c, PREC_F64, false);
    ginv = mref(Z2_, Mp, MM_);
  }
  if (N == 1) {
    FillArgs c = fill_args(mref(P_, Mp, MM_), Mp, Mp, FILL_MAT);
    c.src = ginv;
    launch_fill(c, B_, st_);
  } else {
    GemmArgs g = gemm_args(Mp, Mp, Mp, B_);
    g.A = mref(Wcur, Mp, MM_);
    g.B = ginv;
    g.C = mref(P_, Mp, MM_);
    g.alpha = -1.0;
    gemm(g, PREC_F64, false);
  }
  GemmArgs g = gemm_args(Mp, Mp, Mp, B_);
  g.A = mref(gamL_, Mp, MM_);
  g.B = mref(P_, Mp, MM_);
  g.C = mref(Z1_, Mp, MM_);
  gemm(g, PREC_F64, false);
  g.A = mref(P_, Mp, MM_);
  g.B = mref(gamR_, Mp, MM_);
  g.C = mref(Z2_, Mp, MM_);
  gemm(g, PREC_F64, false);
  TraceArgs t;
  t.Z1 = mref(Z1_, Mp, MM_);
  t.Z2 = mref(Z2_, Mp, MM_);
  t.Mp = Mp;
  t.T = T;
  t.info = info;
  t.sr_done_l = done_l_;
  t.sr_done_r = same_leads ? done_l_ : done_r_;
  t.sing = sing_;
  launch_trace(t, B_, st_);
}

void Engine::export_sigma(z64* sigma_ws, rgf_z* out) {
  launch_unpad(mref(sigma_ws, Mp_, MM_), reinterpret_cast<z64*>(out), M_, B_, st_);
}

void Engine::lead_info(int side_bit, int32_t* done, int32_t* info) {
  launch_sr_info(done, side_bit, sing_, info, B_, 0, st_);
}

}  // namespace rgf
