// Test-only entry points (librgf_ktest.so): single kernels of librgf driven
// on caller buffers, so the tests can check each against numpy.  Not part
// of the product ABI.
#include <cstring>
#include <vector>

#include "../common.h"
#include "../kernels.h"

using namespace rgf;

template <class F>
static int kt_guard(F&& f) {
  try {
    f();
    return 0;
  } catch (const Error& e) {
    fprintf(stderr, "ktest: %s\n", e.msg.c_str());
    return e.code;
  }
}

// Whether the harness's LU runs look ahead (a second candidate list, see lu_factor).
static int g_kt_lookahead = 1;
static int g_kt_exact_u = 0;

extern "C" {

// Turn the look-ahead of the harness's LU on (1) or off (0); returns the previous setting.
int rgf_ktest_set_lookahead(int on) {
  const int prev = g_kt_lookahead;
  g_kt_lookahead = on ? 1 : 0;
  return prev;
}

// Solve with U's diagonal blocks by substitution (1) or with their explicit inverses (0, the
// default) in the harness's LU; returns the previous setting.
int rgf_ktest_set_exact_u(int on) {
  const int prev = g_kt_exact_u;
  g_kt_exact_u = on ? 1 : 0;
  return prev;
}

// C[b] = alpha * A[b] B[b] (+ C[b] when accumulate), dense row-major, device pointers.
int rgf_ktest_gemm(int prec, int tile, int rows, int cols, int K, int batch, const void* A, const void* B,
                   void* C, double alpha, int accumulate) {
  return kt_guard([&] {
    GemmArgs g;
    g.rows = rows;
    g.cols = cols;
    g.K = K;
    g.batch = batch;
    g.a_kind = SRC_MAT;
    g.A = mat((z64*)A, (int64_t)rows * K, K);
    g.Af = form(nullptr, nullptr, 0, false, false, nullptr, 0.0);
    g.B = mat((z64*)B, (int64_t)K * cols, cols);
    g.c_kind = accumulate ? SRC_MAT : SRC_NONE;
    g.Cin = mat((z64*)C, (int64_t)rows * cols, cols);
    g.Cf = g.Af;
    g.C = g.Cin;
    g.alpha = alpha;
    g.ctl.skip = nullptr;
    launch_gemm(g, prec, tile, nullptr, 0);
    RGF_HIP(hipDeviceSynchronize());
  });
}

// X[b] = B[b]^-1 RHS[b] by the batched LU and the two triangular solves; B (Mp x Mp) is destroyed,
// RHS (Mp x nrhs, host order) is read; X (Mp x nrhs) receives the solution.
int rgf_ktest_lu(int prec, int Mp, int nrhs, int batch, void* B, const void* RHS, void* X, int32_t* perm_out,
                 int32_t* sing_out) {
  return kt_guard([&] {
    LuBufs g;
    RGF_HIP(hipMalloc((void**)&g.linv, sizeof(z64) * batch * 64 * Mp));
    RGF_HIP(hipMalloc((void**)&g.uinv, sizeof(z64) * batch * 64 * Mp));
    RGF_HIP(hipMalloc((void**)&g.perm, sizeof(int32_t) * batch * Mp));
    RGF_HIP(hipMalloc((void**)&g.cand, sizeof(int32_t) * batch * Mp));
    if (g_kt_lookahead) RGF_HIP(hipMalloc((void**)&g.cand2, sizeof(int32_t) * batch * Mp));
    RGF_HIP(hipMalloc((void**)&g.flags, batch * Mp));
    RGF_HIP(hipMalloc((void**)&g.sing, sizeof(int32_t) * batch));
    RGF_HIP(hipMemset(g.sing, 0, sizeof(int32_t) * batch));
    g.exact_u = g_kt_exact_u != 0;
    const int64_t bs = (int64_t)Mp * Mp, ybs = (int64_t)Mp * nrhs;
    lu_factor(g, (z64*)B, bs, Mp, batch, nullptr, 1, prec, 128, nullptr);
    FillArgs f;
    f.dst = mat((z64*)X, ybs, nrhs);
    f.rows = Mp;
    f.cols = nrhs;
    f.kind = FILL_MAT;
    f.scale = 1.0;
    f.src = mat((z64*)RHS, ybs, nrhs, g.perm, Mp);
    f.f = form(nullptr, nullptr, 0, false, false, nullptr, 0.0);
    f.flags = nullptr;
    f.flags_bs = 0;
    f.flags_n = 0;
    f.ridx = nullptr;
    f.ridx_bs = 0;
    f.ctl.skip = nullptr;
    launch_fill(f, batch, nullptr);
    lu_solve(g, (z64*)B, bs, Mp, (z64*)X, ybs, nrhs, batch, nullptr, prec, 128, nullptr);
    RGF_HIP(hipDeviceSynchronize());
    if (perm_out) RGF_HIP(hipMemcpy(perm_out, g.perm, sizeof(int32_t) * batch * Mp, hipMemcpyDeviceToHost));
    if (sing_out) RGF_HIP(hipMemcpy(sing_out, g.sing, sizeof(int32_t) * batch, hipMemcpyDeviceToHost));
    RGF_HIP(hipFree(g.linv));
    RGF_HIP(hipFree(g.uinv));
    RGF_HIP(hipFree(g.perm));
    RGF_HIP(hipFree(g.cand));
    if (g.cand2) RGF_HIP(hipFree(g.cand2));
    RGF_HIP(hipFree(g.flags));
    RGF_HIP(hipFree(g.sing));
  });
}

// X[b] = B[b]^-1 Y[b] by the fused factor-and-solve kernel (one workgroup per entry): B (Mp x Mp)
// is destroyed, Y (Mp x nrhs) is overwritten in pivot-row order; X (Mp x nrhs) receives the
// solution gathered through the pivot rows.  skip (host, may be null): entries left alone.
int rgf_ktest_gj(int Mp, int nrhs, int batch, void* B, void* Y, void* X, const int32_t* skip_host,
                 int32_t* perm_out, int32_t* sing_out) {
  return kt_guard([&] {
    int32_t *perm = nullptr, *sing = nullptr, *skip = nullptr;
    RGF_HIP(hipMalloc((void**)&perm, sizeof(int32_t) * batch * Mp));
    RGF_HIP(hipMalloc((void**)&sing, sizeof(int32_t) * batch));
    RGF_HIP(hipMemset(sing, 0, sizeof(int32_t) * batch));
    RGF_HIP(hipMemset(perm, 0, sizeof(int32_t) * batch * Mp));
    if (skip_host) {
      RGF_HIP(hipMalloc((void**)&skip, sizeof(int32_t) * batch));
      RGF_HIP(hipMemcpy(skip, skip_host, sizeof(int32_t) * batch, hipMemcpyHostToDevice));
    }
    const int64_t bs = (int64_t)Mp * Mp, ybs = (int64_t)Mp * nrhs;
    GjArgs a;
    a.T = (z64*)B;
    a.tbs = bs;
    a.Y = (z64*)Y;
    a.ybs = ybs;
    a.nrhs = nrhs;
    a.Mp = Mp;
    a.perm = perm;
    a.perm_bs = Mp;
    a.sing = sing;
    a.sing_code = 7;
    a.skip = skip;
    launch_gj(a, batch, nullptr);
    FillArgs f;
    f.dst = mat((z64*)X, ybs, nrhs);
    f.rows = Mp;
    f.cols = nrhs;
    f.kind = FILL_MAT;
    f.scale = 1.0;
    f.src = mat((z64*)Y, ybs, nrhs, perm, Mp);
    f.f = form(nullptr, nullptr, 0, false, false, nullptr, 0.0);
    f.flags = nullptr;
    f.flags_bs = 0;
    f.flags_n = 0;
    f.ridx = nullptr;
    f.ridx_bs = 0;
    f.ctl.skip = skip;
    launch_fill(f, batch, nullptr);
    RGF_HIP(hipDeviceSynchronize());
    if (perm_out) RGF_HIP(hipMemcpy(perm_out, perm, sizeof(int32_t) * batch * Mp, hipMemcpyDeviceToHost));
    if (sing_out) RGF_HIP(hipMemcpy(sing_out, sing, sizeof(int32_t) * batch, hipMemcpyDeviceToHost));
    RGF_HIP(hipFree(perm));
    RGF_HIP(hipFree(sing));
    if (skip) RGF_HIP(hipFree(skip));
  });
}

// Pseudo-random complex entries in [-1, 1) plus `diag` on the diagonal (timing inputs).
__global__ void kt_fill_random(z64* p, int64_t n, int64_t ld, int64_t rows_per_batch, double diag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull;
  h ^= h >> 31;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 29;
  const double a = (double)(h >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
  const double b = (double)((h * 0x94D049BB133111EBull) >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
  const int64_t r = (i / ld) % rows_per_batch, c = i % ld;
  p[i] = zmake(a + (r == c ? diag : 0.0), b);
}

static void kt_random(z64* p, int64_t n, int64_t ld, int64_t rows, double diag) {
  hipLaunchKernelGGL(kt_fill_random, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, nullptr, p, n, ld, rows, diag);
  RGF_HIP(hipGetLastError());
}

// Average duration (ms, HIP events) of `reps` launches of one batched block product
// C = C - A B on device buffers it allocates; inplace: C aliases B (rows must fit one tile).
int rgf_ktest_gemm_time(int prec, int tile, int rows, int cols, int K, int batch, int inplace, int reps,
                        double* ms) {
  return kt_guard([&] {
    z64 *A, *B, *Cm;
    const int64_t na = (int64_t)batch * rows * K, nb = (int64_t)batch * K * cols, nc = (int64_t)batch * rows * cols;
    RGF_HIP(hipMalloc((void**)&A, sizeof(z64) * na));
    RGF_HIP(hipMalloc((void**)&B, sizeof(z64) * nb));
    RGF_HIP(hipMalloc((void**)&Cm, sizeof(z64) * nc));
    kt_random(A, na, K, rows, 0.0);
    kt_random(B, nb, cols, K, 0.0);
    kt_random(Cm, nc, cols, rows, 0.0);
    GemmArgs g;
    g.rows = rows;
    g.cols = cols;
    g.K = K;
    g.batch = batch;
    g.a_kind = SRC_MAT;
    g.A = mat(A, (int64_t)rows * K, K);
    g.Af = form(nullptr, nullptr, 0, false, false, nullptr, 0.0);
    g.B = mat(B, (int64_t)K * cols, cols);
    g.c_kind = inplace ? SRC_NONE : SRC_MAT;
    g.Cin = inplace ? g.B : mat(Cm, (int64_t)rows * cols, cols);
    g.Cf = g.Af;
    g.C = g.Cin;
    g.alpha = -1.0;
    g.ctl.skip = nullptr;
    hipEvent_t e0, e1;
    RGF_HIP(hipEventCreate(&e0));
    RGF_HIP(hipEventCreate(&e1));
    launch_gemm(g, prec, tile, nullptr, 0);
    RGF_HIP(hipEventRecord(e0, nullptr));
    for (int r = 0; r < reps; ++r) launch_gemm(g, prec, tile, nullptr, 0);
    RGF_HIP(hipEventRecord(e1, nullptr));
    RGF_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    RGF_HIP(hipEventElapsedTime(&t, e0, e1));
    *ms = t / reps;
    RGF_HIP(hipEventDestroy(e0));
    RGF_HIP(hipEventDestroy(e1));
    RGF_HIP(hipFree(A));
    RGF_HIP(hipFree(B));
    RGF_HIP(hipFree(Cm));
  });
}

// Average durations (ms) of the batched LU factorisation and of the two triangular
// solves with nrhs right-hand sides, on a random diagonally weighted matrix.
int rgf_ktest_lu_time(int prec, int Mp, int nrhs, int batch, int reps, double* ms_factor, double* ms_solve) {
  return kt_guard([&] {
    LuBufs g;
    z64 *B0, *B, *Y;
    const int64_t bs = (int64_t)Mp * Mp, ybs = (int64_t)Mp * nrhs;
    RGF_HIP(hipMalloc((void**)&g.linv, sizeof(z64) * batch * 64 * Mp));
    RGF_HIP(hipMalloc((void**)&g.uinv, sizeof(z64) * batch * 64 * Mp));
    RGF_HIP(hipMalloc((void**)&g.perm, sizeof(int32_t) * batch * Mp));
    RGF_HIP(hipMalloc((void**)&g.cand, sizeof(int32_t) * batch * Mp));
    if (g_kt_lookahead) RGF_HIP(hipMalloc((void**)&g.cand2, sizeof(int32_t) * batch * Mp));
    RGF_HIP(hipMalloc((void**)&g.flags, batch * Mp));
    RGF_HIP(hipMalloc((void**)&g.sing, sizeof(int32_t) * batch));
    RGF_HIP(hipMalloc((void**)&B0, sizeof(z64) * batch * bs));
    RGF_HIP(hipMalloc((void**)&B, sizeof(z64) * batch * bs));
    RGF_HIP(hipMalloc((void**)&Y, sizeof(z64) * batch * ybs));
    RGF_HIP(hipMemset(g.sing, 0, sizeof(int32_t) * batch));
    kt_random(B0, batch * bs, Mp, Mp, 4.0);
    kt_random(Y, batch * ybs, nrhs, Mp, 0.0);
    hipEvent_t e[3];
    for (auto& x : e) RGF_HIP(hipEventCreate(&x));
    double tf = 0.0, ts = 0.0;
    for (int r = 0; r <= reps; ++r) {
      RGF_HIP(hipMemcpy(B, B0, sizeof(z64) * batch * bs, hipMemcpyDeviceToDevice));
      RGF_HIP(hipEventRecord(e[0], nullptr));
      lu_factor(g, B, bs, Mp, batch, nullptr, 1, prec, 128, nullptr);
      RGF_HIP(hipEventRecord(e[1], nullptr));
      lu_solve(g, B, bs, Mp, Y, ybs, nrhs, batch, nullptr, prec, 128, nullptr);
      RGF_HIP(hipEventRecord(e[2], nullptr));
      RGF_HIP(hipEventSynchronize(e[2]));
      float a = 0.f, b = 0.f;
      RGF_HIP(hipEventElapsedTime(&a, e[0], e[1]));
      RGF_HIP(hipEventElapsedTime(&b, e[1], e[2]));
      if (r > 0) {
        tf += a;
        ts += b;
      }
    }
    *ms_factor = tf / reps;
    *ms_solve = ts / reps;
    for (auto& x : e) RGF_HIP(hipEventDestroy(x));
    for (void* q : {(void*)g.linv, (void*)g.uinv, (void*)g.perm, (void*)g.cand, (void*)g.flags, (void*)g.sing,
                    (void*)B0, (void*)B, (void*)Y})
      RGF_HIP(hipFree(q));
    if (g.cand2) RGF_HIP(hipFree(g.cand2));
  });
}

// Average duration (ms, HIP events) of one fused factor-and-solve launch on random diagonally
// weighted B (Mp x Mp) and Y (Mp x nrhs), `batch` entries.
int rgf_ktest_gj_time(int Mp, int nrhs, int batch, int reps, double* ms) {
  return kt_guard([&] {
    z64 *B0, *B, *Y0, *Y;
    int32_t *perm, *sing;
    const int64_t bs = (int64_t)Mp * Mp, ybs = (int64_t)Mp * nrhs;
    RGF_HIP(hipMalloc((void**)&B0, sizeof(z64) * batch * bs));
    RGF_HIP(hipMalloc((void**)&B, sizeof(z64) * batch * bs));
    RGF_HIP(hipMalloc((void**)&Y0, sizeof(z64) * batch * ybs));
    RGF_HIP(hipMalloc((void**)&Y, sizeof(z64) * batch * ybs));
    RGF_HIP(hipMalloc((void**)&perm, sizeof(int32_t) * batch * Mp));
    RGF_HIP(hipMalloc((void**)&sing, sizeof(int32_t) * batch));
    RGF_HIP(hipMemset(sing, 0, sizeof(int32_t) * batch));
    kt_random(B0, batch * bs, Mp, Mp, 4.0);
    kt_random(Y0, batch * ybs, nrhs, Mp, 0.0);
    GjArgs a;
    a.T = B;
    a.tbs = bs;
    a.Y = Y;
    a.ybs = ybs;
    a.nrhs = nrhs;
    a.Mp = Mp;
    a.perm = perm;
    a.perm_bs = Mp;
    a.sing = sing;
    a.sing_code = 1;
    a.skip = nullptr;
    hipEvent_t e[2];
    for (auto& x : e) RGF_HIP(hipEventCreate(&x));
    double t = 0.0;
    for (int r = 0; r <= reps; ++r) {
      RGF_HIP(hipMemcpy(B, B0, sizeof(z64) * batch * bs, hipMemcpyDeviceToDevice));
      RGF_HIP(hipMemcpy(Y, Y0, sizeof(z64) * batch * ybs, hipMemcpyDeviceToDevice));
      RGF_HIP(hipEventRecord(e[0], nullptr));
      launch_gj(a, batch, nullptr);
      RGF_HIP(hipEventRecord(e[1], nullptr));
      RGF_HIP(hipEventSynchronize(e[1]));
      float x = 0.f;
      RGF_HIP(hipEventElapsedTime(&x, e[0], e[1]));
      if (r > 0) t += x;
    }
    *ms = t / reps;
    for (auto& x : e) RGF_HIP(hipEventDestroy(x));
    for (void* q : {(void*)B0, (void*)B, (void*)Y0, (void*)Y, (void*)perm, (void*)sing}) RGF_HIP(hipFree(q));
  });
}

// Average duration (ms) of one sweep-layer block product on Mp x Mp blocks, `batch` energies,
// with the operand forms the sweep uses.  variant 0: W' = -W X (both operands stored);
// 1: B' = A_ii - L X with L = z S^+ - H^+ and A_ii = z S - H formed from shared blocks;
// 2: as 1 with L stored; 3: as 1 with L formed untransposed (z S - H); 4: -L X, L formed
// transposed, no C operand; 5: L stored by the adjoint-formation kernel, then as 2 (both timed).
int rgf_ktest_sweep_time(int prec, int variant, int Mp, int batch, int reps, double* ms) {
  return kt_guard([&] {
    RGF_CHECK(variant >= 0 && variant <= 5 && Mp % 64 == 0 && batch > 0, RGF_EINVAL, "ktest: bad sweep case");
    const int64_t bs = (int64_t)Mp * Mp, n = bs * batch;
    z64 *S, *H, *A, *X, *Cm;
    double* E;
    RGF_HIP(hipMalloc((void**)&S, sizeof(z64) * bs));
    RGF_HIP(hipMalloc((void**)&H, sizeof(z64) * bs));
    RGF_HIP(hipMalloc((void**)&A, sizeof(z64) * n));
    RGF_HIP(hipMalloc((void**)&X, sizeof(z64) * n));
    RGF_HIP(hipMalloc((void**)&Cm, sizeof(z64) * n));
    RGF_HIP(hipMalloc((void**)&E, sizeof(double) * batch));
    kt_random(S, bs, Mp, Mp, 4.0);
    kt_random(H, bs, Mp, Mp, 0.0);
    kt_random(A, n, Mp, Mp, 0.0);
    kt_random(X, n, Mp, Mp, 0.0);
    std::vector<double> eh(batch);
    for (int b = 0; b < batch; ++b) eh[b] = -1.0 + 2.0 * b / batch;
    RGF_HIP(hipMemcpy(E, eh.data(), sizeof(double) * batch, hipMemcpyHostToDevice));
    GemmArgs g = gemm_args(Mp, Mp, Mp, batch);
    g.B = mat(X, bs, Mp);
    g.C = mat(Cm, bs, Mp);
    g.alpha = -1.0;
    const FormRef lf = form(reinterpret_cast<const rgf_z*>(H), reinterpret_cast<const rgf_z*>(S), Mp, true,
                            false, E, 1e-6);
    if (variant == 0 || variant == 2 || variant == 5) {
      g.A = mat(A, bs, Mp);
    } else {
      g.a_kind = SRC_FORM;
      g.Af = form(reinterpret_cast<const rgf_z*>(H), reinterpret_cast<const rgf_z*>(S), Mp, variant != 3,
                  false, E, 1e-6);
    }
    if (variant >= 1 && variant != 4) {
      g.c_kind = SRC_FORM;
      g.Cf = form(reinterpret_cast<const rgf_z*>(H), reinterpret_cast<const rgf_z*>(S), Mp, false, true, E, 1e-6);
    }
    hipEvent_t e0, e1;
    RGF_HIP(hipEventCreate(&e0));
    RGF_HIP(hipEventCreate(&e1));
    if (variant == 5) launch_form_ct(lf, mat(A, bs, Mp), Mp, batch, nullptr);
    launch_gemm(g, prec, 128, nullptr, 1);
    RGF_HIP(hipEventRecord(e0, nullptr));
    for (int r = 0; r < reps; ++r) {
      if (variant == 5) launch_form_ct(lf, mat(A, bs, Mp), Mp, batch, nullptr);
      launch_gemm(g, prec, 128, nullptr, 1);
    }
    RGF_HIP(hipEventRecord(e1, nullptr));
    RGF_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    RGF_HIP(hipEventElapsedTime(&t, e0, e1));
    *ms = t / reps;
    RGF_HIP(hipEventDestroy(e0));
    RGF_HIP(hipEventDestroy(e1));
    for (void* q : {(void*)S, (void*)H, (void*)A, (void*)X, (void*)Cm, (void*)E}) RGF_HIP(hipFree(q));
  });
}

// The stored adjoint operand two ways: out_ct by the tiled formation kernel, out_fill by the
// element-wise fill (the formed operand's definition), both [batch][Mp][Mp].  H, S: `groups`
// consecutive M x M blocks; batch entry b reads group b / per (per = ceil(batch / groups)).
int rgf_ktest_form_ct(int M, int Mp, int batch, int groups, int pad, const void* H, const void* S, const double* E,
                      double eta, void* out_ct, void* out_fill) {
  return kt_guard([&] {
    RGF_CHECK(M >= 1 && Mp >= M && Mp % 64 == 0 && batch >= 1 && groups >= 1 && groups <= batch, RGF_EINVAL,
              "ktest: bad form case");
    FormRef f = form(reinterpret_cast<const rgf_z*>(H), reinterpret_cast<const rgf_z*>(S), M, true, pad != 0, E, eta);
    f.gper = (batch + groups - 1) / groups;
    f.gb0 = 0;
    f.gstride = (int64_t)M * M;
    const int64_t bs = (int64_t)Mp * Mp;
    launch_form_ct(f, mat((z64*)out_ct, bs, Mp), Mp, batch, nullptr);
    FillArgs a = fill_args(mat((z64*)out_fill, bs, Mp), Mp, Mp, FILL_FORM);
    a.f = f;
    launch_fill(a, batch, nullptr);
    RGF_HIP(hipDeviceSynchronize());
  });
}

// Largest inner dimension that takes the short-K product tiles (0: never); returns the previous.
int rgf_ktest_set_small_k(int k) { return set_small_k_max(k); }

}  // extern "C"
