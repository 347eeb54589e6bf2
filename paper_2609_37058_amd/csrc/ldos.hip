// Orbital-resolved local density of states of the device (the spatially
// resolved LDOS the paper reports at zero and finite bias, Discussion).
//
// Per energy, with G = (z S - H - Sigma_L (+) Sigma_R)^-1 on the device:
//   rho_mu   = (1 / 2 pi) Re [A S]_mu,mu,   A   = i (G - G^+)
//   rho^X_mu = (1 / 2 pi) Re [A_X S]_mu,mu, A_X = G Gamma_X G^+
// (the Mulliken projection inside the device).  Only the blocks of G within
// one layer of the diagonal enter [A S]_pp, and only the block column of the
// injecting electrode's contact layer enters [A_X S]_pp.
//
// Two passes per direction over the layers in "pass order" (left to right
// for the left electrode, right to left for the right one), p = 0..N-1,
// C_p = A_{p,p+1}, D_{p+1} = A_{p+1,p}, s = the starting electrode, e = the
// other one:
//   pass A, p = N-1 .. 0: the end-connected inverse of the layers p..N-1,
//     gE_{N-1} = (A_{N-1} - Sigma_e)^-1,
//     gE_p = (A_p - C_p X_{p+1})^-1 with X_{p+1} = gE_{p+1} D_{p+1}
//     (- Sigma_s on p = 0); every gE_p is kept in HBM (N Mp^2 per energy),
//     LU-factored and inverted by solves against P I, X by a solve against
//     P D.  gE_0 = G_00.
//   pass B, p = 1 .. N-1 (partition of the device between p-1 and p):
//     G_{p,p-1} = -gE_p D_p G_{p-1,p-1},   G_{p-1,p} = -G_{p-1,p-1} C_{p-1} gE_p,
//     G_pp      = gE_p - G_{p,p-1} C_{p-1} gE_p,
//     G_{p,0}   = -gE_p D_p G_{p-1,0}       (the block column of the contact)
// and the O(M^2) projections
//   [A S]_pp[mu]   = -Im sum_q ( rowsum(G_pq .* conj S_pq)[mu] + colsum(G_qp .* conj S_qp)[mu] ),
//   [A_s S]_pp[mu] = Re rowsum(X_p .* conj W_p)[mu],
//   X_p = G_{p,0} Gamma_s,  W_p = sum_q S_pq G_{q,0}   (q = p-1, p, p+1).
// The energy-dependent couplings C_p, D_p are written per energy before their
// products (a formed operand costs the product two block loads per element);
// the overlap-only operands S_pq are written once per layer as padded blocks
// shared by all energies, formed as z S - H with H = S and z = 2 (exact in
// binary floating point).
#include <utility>

#include "engine.h"

namespace rgf {

namespace {

constexpr double INV_2PI = 0.15915494309189533577;  // 1 / (2 pi)

struct ProjArgs {
  MatRef G;      // per batch, rows x cols of the padded block
  const z64* S;  // shared M x M block (row-major); conj_s: the operand is its adjoint
  int conj_s;
  int M;
  double* out;   // [batch][N][M]
  int64_t out_bs;
  int layer;     // output layer
};

__device__ inline z64 s_elem(const ProjArgs& a, int r, int c) {
  return a.conj_s ? zconj(a.S[(int64_t)c * a.M + r]) : a.S[(int64_t)r * a.M + c];
}

// out[layer][r] += -(1/2pi) Im sum_c G[r][c] conj(S[r][c]); one wavefront per row
__global__ void __launch_bounds__(256) proj_rows_kernel(ProjArgs a) {
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= a.M) return;
  double acc = 0.0;
  for (int c = lane; c < a.M; c += 64) {
    const z64 g = a.G.p[mat_off(a.G, b, r, c)];
    const z64 s = s_elem(a, r, c);
    acc += g.y * s.x - g.x * s.y;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) a.out[b * a.out_bs + (int64_t)a.layer * a.M + r] -= INV_2PI * acc;
}

// out[layer][c] += -(1/2pi) Im sum_r G[r][c] conj(S[r][c]); a workgroup takes 16 columns,
// its 16 row groups stride the rows and their partial sums are added in row-group order
constexpr int PC_COLS = 16, PC_GROUPS = 16;
__global__ void __launch_bounds__(PC_COLS * PC_GROUPS) proj_cols_kernel(ProjArgs a) {
  __shared__ double part[PC_GROUPS][PC_COLS];
  const int b = blockIdx.y;
  const int tx = threadIdx.x % PC_COLS, ty = threadIdx.x / PC_COLS;
  const int c = blockIdx.x * PC_COLS + tx;
  double acc = 0.0;
  if (c < a.M) {
    for (int r = ty; r < a.M; r += PC_GROUPS) {
      const z64 g = a.G.p[mat_off(a.G, b, r, c)];
      const z64 s = s_elem(a, r, c);
      acc += g.y * s.x - g.x * s.y;
    }
  }
  part[ty][tx] = acc;
  __syncthreads();
  if (ty == 0 && c < a.M) {
    double t = 0.0;
    for (int k = 0; k < PC_GROUPS; ++k) t += part[k][tx];
    a.out[b * a.out_bs + (int64_t)a.layer * a.M + c] -= INV_2PI * t;
  }
}

struct InjArgs {
  MatRef X, W;
  int M;
  double* out;
  int64_t out_bs;
  int layer;
};

// out[layer][r] = (1/2pi) Re sum_c X[r][c] conj(W[r][c]); one wavefront per row
__global__ void __launch_bounds__(256) injected_kernel(InjArgs a) {
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= a.M) return;
  double acc = 0.0;
  for (int c = lane; c < a.M; c += 64) {
    const z64 x = a.X.p[mat_off(a.X, b, r, c)];
    const z64 w = a.W.p[mat_off(a.W, b, r, c)];
    acc += x.x * w.x + x.y * w.y;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) a.out[b * a.out_bs + (int64_t)a.layer * a.M + r] = INV_2PI * acc;
}

__global__ void fill_value_kernel(double* p, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_proj(const ProjArgs& a, bool rows, int batch, hipStream_t st) {
  if (rows)
    hipLaunchKernelGGL(proj_rows_kernel, dim3((a.M + 3) / 4, batch), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(proj_cols_kernel, dim3((a.M + PC_COLS - 1) / PC_COLS, batch), dim3(PC_COLS * PC_GROUPS), 0,
                       st, a);
  RGF_HIP(hipGetLastError());
}

}  // namespace

MatRef Engine::store_form(const FormRef& f, z64* dst, int batch) {
  if (f.conj_t) {
    launch_form_ct(f, mref(dst, Mp_, MM_), Mp_, batch, st_);
  } else {
    FillArgs a = fill_args(mref(dst, Mp_, MM_), Mp_, Mp_, FILL_FORM);
    a.f = f;
    launch_fill(a, batch, st_);
  }
  return mref(dst, Mp_, MM_);
}

void Engine::local_dos(const rgf_device& d, z64* store, double* twos, z64* sblk, double* dos, double* ados_l,
                       double* ados_r, int32_t* info, bool same_leads) {
  hipLaunchKernelGGL(fill_value_kernel, dim3((B_ + 255) / 256), dim3(256), 0, st_, twos, B_, 2.0);
  RGF_HIP(hipGetLastError());
  if (dos) RGF_HIP(hipMemsetAsync(dos, 0, sizeof(double) * (size_t)B_ * d.N * M_, st_));
  if (dos || ados_l) ldos_pass(d, store, twos, sblk, true, dos, ados_l);
  if (ados_r) ldos_pass(d, store, twos, sblk, false, nullptr, ados_r);
  if (info) {
    launch_sr_info(done_l_, RGF_INFO_SR_LEFT, sing_, info, B_, 0, st_);
    launch_sr_info(same_leads ? done_l_ : done_r_, RGF_INFO_SR_RIGHT, sing_, info, B_, 1, st_);
  }
}

void Engine::ldos_pass(const rgf_device& d, z64* store, const double* twos, z64* sblk, bool fwd, double* dos,
                       double* inj) {
  const int Mp = Mp_, N = d.N, M = M_;
  const int64_t M2 = (int64_t)M * M;
  const int64_t SB = (int64_t)N * MM_;  // batch stride of the kept inverses
  const int64_t U = (int64_t)B_ * MM_;
  const int64_t out_bs = (int64_t)N * M;
  const int tile = tile_for(PREC_F64, Mp);
  auto layer = [&](int p) { return fwd ? p : N - 1 - p; };
  auto cpl = [&](int p) { return fwd ? p : N - 2 - p; };  // coupling block between pass layers p and p+1
  // A_{p,p+1} and A_{p+1,p} in pass order, formed at the chunk's energies
  auto Aup = [&](int p) {
    const int k = cpl(p);
    return gform(form(d.Hu + k * M2, d.Su + k * M2, M, !fwd, false, E_, eta_));
  };
  auto Adn = [&](int p) {
    const int k = cpl(p);
    return gform(form(d.Hu + k * M2, d.Su + k * M2, M, fwd, false, E_, eta_));
  };
  auto Adiag = [&](int p) {
    const int l = layer(p);
    return gform(form(d.Hd + l * M2, d.Sd + l * M2, M, false, true, E_, eta_));
  };
  // overlap blocks alone: 2 S - S
  auto Sform = [&](const rgf_z* s, bool conj) { return form(s, s, M, conj, false, twos, 0.0); };
  z64* sig_s = fwd ? sigL_ : sigR_;
  z64* sig_e = fwd ? sigR_ : sigL_;
  z64* gam_s = fwd ? gamL_ : gamR_;
  z64* un = eps_;
  auto kept = [&](int p) { return mref(store + (int64_t)p * MM_, Mp, SB); };
  auto work = [&](int i) { return un + (int64_t)i * U; };

  // ---- pass A: end-connected inverses gE_p, kept for every layer ----
  z64* Bm = work(0);
  z64* Xm = work(1);
  for (int p = N - 1; p >= 0; --p) {
    if (p == N - 1) {
      FillArgs f = fill_args(mref(Bm, Mp, MM_), Mp, Mp, FILL_FORM);
      f.f = Adiag(p);
      f.f.sub = mref(sig_e, Mp, MM_);
      f.f.sub_sign = -1.0;
      launch_fill(f, B_, st_);
      if (N == 1) {
        BatchCtl none;
        none.skip = nullptr;
        launch_axpy(mref(Bm, Mp, MM_), mref(sig_s, Mp, MM_), -1.0, Mp, Mp, B_, none, st_);
      }
    } else {
      GemmArgs g = gemm_args(Mp, Mp, Mp, B_);
      g.A = store_form(Aup(p), work(2), B_);
      g.B = mref(Xm, Mp, MM_);
      g.c_kind = SRC_FORM;
      g.Cf = Adiag(p);
      if (p == 0) {
        g.Cf.sub = mref(sig_s, Mp, MM_);
        g.Cf.sub_sign = -1.0;
      }
      g.C = mref(Bm, Mp, MM_);
      g.alpha = -1.0;
      gemm(g, PREC_F64, true);
    }
    lu_factor(lu_, Bm, MM_, Mp, B_, nullptr, layer(p) + 1, PREC_F64, tile, st_);
    FillArgs f = fill_args(kept(p), Mp, Mp, FILL_IDENTITY);
    f.ridx = lu_.perm;
    f.ridx_bs = Mp;
    launch_fill(f, B_, st_);
    lu_solve(lu_, Bm, MM_, Mp, store + (int64_t)p * MM_, SB, Mp, B_, nullptr, PREC_F64, tile, st_);
    if (p > 0) {  // X_p = gE_p D_p for the next layer down
      f = fill_args(mref(Xm, Mp, MM_), Mp, Mp, FILL_FORM);
      f.f = Adn(p - 1);
      f.ridx = lu_.perm;
      f.ridx_bs = Mp;
      launch_fill(f, B_, st_);
      lu_solve(lu_, Bm, MM_, Mp, Xm, MM_, Mp, B_, nullptr, PREC_F64, tile, st_);
    }
  }

  // ---- pass B ----
  z64* Gd[2] = {work(0), work(1)};
  z64* ring[3] = {work(2), work(3), work(4)};
  z64* Yb = work(5);
  z64* Gl = work(6);
  z64* Vb = work(7);
  z64* Gu = work(8);
  z64* Xb = work(9);
  z64* Wb = work(10);
  z64* Cst = work(11);  // the current coupling, stored per energy
  auto col = [&](int q) { return q == 0 ? kept(0) : mref(ring[q % 3], Mp, MM_); };
  auto proj = [&](MatRef G, const rgf_z* s, bool conj, int row_layer, int col_layer) {
    ProjArgs a;
    a.G = G;
    a.S = reinterpret_cast<const z64*>(s);
    a.conj_s = conj ? 1 : 0;
    a.M = M;
    a.out = dos;
    a.out_bs = out_bs;
    a.layer = row_layer;
    launch_proj(a, true, B_, st_);
    a.layer = col_layer;
    launch_proj(a, false, B_, st_);
  };
  // S_{p,p+1} and S_{p+1,p} in pass order (raw block and whether it enters as its adjoint)
  auto s_up = [&](int p) { return std::make_pair(d.Su + cpl(p) * M2, !fwd); };
  auto s_dn = [&](int p) { return std::make_pair(d.Su + cpl(p) * M2, fwd); };
  // an overlap block as a padded Mp x Mp operand shared by every energy (slot 0..2 of sblk)
  auto shared_s = [&](int slot, const rgf_z* s, bool conj) {
    z64* dst = sblk + (int64_t)slot * MM_;
    store_form(Sform(s, conj), dst, 1);
    return mat(dst, 0, Mp);  // batch stride 0: every energy reads the one block
  };
  auto injected = [&](int q) {  // rho^s of pass layer q, from G_{q-1,0}, G_{q,0}, G_{q+1,0}
    GemmArgs g = gemm_args(Mp, Mp, Mp, B_);
    g.A = col(q);
    g.B = mref(gam_s, Mp, MM_);
    g.C = mref(Xb, Mp, MM_);
    gemm(g, PREC_F64, true);
    bool first = true;
    auto add = [&](MatRef s, MatRef c) {
      GemmArgs w = gemm_args(Mp, Mp, Mp, B_);
      w.A = s;
      w.B = c;
      if (!first) {
        w.c_kind = SRC_MAT;
        w.Cin = mref(Wb, Mp, MM_);
      }
      w.C = mref(Wb, Mp, MM_);
      gemm(w, PREC_F64, true);
      first = false;
    };
    if (q >= 1) {
      auto s = s_dn(q - 1);
      add(shared_s(0, s.first, s.second), col(q - 1));
    }
    add(shared_s(1, d.Sd + layer(q) * M2, false), col(q));
    if (q + 1 <= N - 1) {
      auto s = s_up(q);
      add(shared_s(2, s.first, s.second), col(q + 1));
    }
    InjArgs a;
    a.X = mref(Xb, Mp, MM_);
    a.W = mref(Wb, Mp, MM_);
    a.M = M;
    a.out = inj;
    a.out_bs = out_bs;
    a.layer = layer(q);
    hipLaunchKernelGGL(injected_kernel, dim3((M + 3) / 4, B_), dim3(256), 0, st_, a);
    RGF_HIP(hipGetLastError());
  };

  MatRef gprev = kept(0);  // G_00
  int cur = 0;
  if (dos) proj(kept(0), d.Sd + layer(0) * M2, false, layer(0), layer(0));
  for (int p = 1; p < N; ++p) {
    const MatRef gE = kept(p);
    const MatRef Dp = store_form(Adn(p - 1), Cst, B_);
    if (dos) {  // G_{p,p-1} = -gE_p (D_p G_{p-1,p-1})
      GemmArgs g = gemm_args(Mp, Mp, Mp, B_);
      g.A = Dp;
      g.B = gprev;
      g.C = mref(Yb, Mp, MM_);
      gemm(g, PREC_F64, true);
      g = gemm_args(Mp, Mp, Mp, B_);
      g.A = gE;
      g.B = mref(Yb, Mp, MM_);
      g.C = mref(Gl, Mp, MM_);
      g.alpha = -1.0;
      gemm(g, PREC_F64, true);
    }
    {  // G_{p,0} = -gE_p (D_p G_{p-1,0})
      GemmArgs g = gemm_args(Mp, Mp, Mp, B_);
      g.A = Dp;
      g.B = col(p - 1);
      g.C = mref(Yb, Mp, MM_);
      gemm(g, PREC_F64, true);
      g = gemm_args(Mp, Mp, Mp, B_);
      g.A = gE;
      g.B = mref(Yb, Mp, MM_);
      g.C = mref(ring[p % 3], Mp, MM_);
      g.alpha = -1.0;
      gemm(g, PREC_F64, true);
    }
    if (dos) {
      // V = C_{p-1} gE_p; G_{p-1,p} = -G_{p-1,p-1} V; G_pp = gE_p - G_{p,p-1} V
      GemmArgs g = gemm_args(Mp, Mp, Mp, B_);
      g.A = store_form(Aup(p - 1), Cst, B_);  // D_p's products are queued before this overwrite
      g.B = gE;
      g.C = mref(Vb, Mp, MM_);
      gemm(g, PREC_F64, true);
      g = gemm_args(Mp, Mp, Mp, B_);
      g.A = gprev;
      g.B = mref(Vb, Mp, MM_);
      g.C = mref(Gu, Mp, MM_);
      g.alpha = -1.0;
      gemm(g, PREC_F64, true);
      g = gemm_args(Mp, Mp, Mp, B_);
      g.A = mref(Gl, Mp, MM_);
      g.B = mref(Vb, Mp, MM_);
      g.c_kind = SRC_MAT;
      g.Cin = gE;
      g.C = mref(Gd[cur], Mp, MM_);
      g.alpha = -1.0;
      gemm(g, PREC_F64, true);
      const auto dn = s_dn(p - 1), up = s_up(p - 1);
      proj(mref(Gl, Mp, MM_), dn.first, dn.second, layer(p), layer(p - 1));
      proj(mref(Gu, Mp, MM_), up.first, up.second, layer(p - 1), layer(p));
      proj(mref(Gd[cur], Mp, MM_), d.Sd + layer(p) * M2, false, layer(p), layer(p));
      gprev = mref(Gd[cur], Mp, MM_);
      cur ^= 1;
    }
    if (inj) injected(p - 1);
  }
  if (inj) injected(N - 1);
}

}  // namespace rgf
