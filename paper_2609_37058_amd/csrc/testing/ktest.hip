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

// X[b] = B[b]^-1 RHS[b] by the batched Gauss-Jordan solve; T[b] = [B | RHS] (Mp x W) is destroyed.
// perm/sing outputs are copied to the caller (perm: Mp ints per batch; sing: 1 int per batch).
int rgf_ktest_gje(int prec, int Mp, int W, int batch, void* T, void* X, int32_t* perm_out, int32_t* sing_out) {
  return kt_guard([&] {
    GjeBufs g;
    RGF_HIP(hipMalloc((void**)&g.P, sizeof(z64) * batch * 64 * 3 * Mp));
    RGF_HIP(hipMalloc((void**)&g.scr, sizeof(z64) * batch * Mp * 64));
    RGF_HIP(hipMalloc((void**)&g.mult, sizeof(z64) * batch * Mp * 64));
    RGF_HIP(hipMalloc((void**)&g.perm, sizeof(int32_t) * batch * Mp));
    RGF_HIP(hipMalloc((void**)&g.flags, batch * Mp));
    RGF_HIP(hipMalloc((void**)&g.sing, sizeof(int32_t) * batch));
    RGF_HIP(hipMemset(g.flags, 0, batch * Mp));
    RGF_HIP(hipMemset(g.sing, 0, sizeof(int32_t) * batch));
    gje_solve(g, (z64*)T, W, (int64_t)Mp * W, Mp, batch, nullptr, 1, prec, 64, nullptr);
    RGF_HIP(hipDeviceSynchronize());
    const int nr = W - Mp;
    std::vector<int32_t> perm((size_t)batch * Mp);
    RGF_HIP(hipMemcpy(perm.data(), g.perm, sizeof(int32_t) * batch * Mp, hipMemcpyDeviceToHost));
    for (int b = 0; b < batch; ++b)
      for (int c = 0; c < Mp; ++c)
        RGF_HIP(hipMemcpy((z64*)X + ((int64_t)b * Mp + c) * nr,
                          (z64*)T + (int64_t)b * Mp * W + (int64_t)perm[(size_t)b * Mp + c] * W + Mp,
                          sizeof(z64) * nr, hipMemcpyDeviceToDevice));
    if (perm_out) memcpy(perm_out, perm.data(), sizeof(int32_t) * batch * Mp);
    if (sing_out) RGF_HIP(hipMemcpy(sing_out, g.sing, sizeof(int32_t) * batch, hipMemcpyDeviceToHost));
    RGF_HIP(hipFree(g.P));
    RGF_HIP(hipFree(g.scr));
    RGF_HIP(hipFree(g.mult));
    RGF_HIP(hipFree(g.perm));
    RGF_HIP(hipFree(g.flags));
    RGF_HIP(hipFree(g.sing));
  });
}

}  // extern "C"
