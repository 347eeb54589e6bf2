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

extern "C" {

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
    RGF_HIP(hipMalloc((void**)&g.flags, batch * Mp));
    RGF_HIP(hipMalloc((void**)&g.sing, sizeof(int32_t) * batch));
    RGF_HIP(hipMemset(g.sing, 0, sizeof(int32_t) * batch));
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
    RGF_HIP(hipFree(g.flags));
    RGF_HIP(hipFree(g.sing));
  });
}

}  // extern "C"
