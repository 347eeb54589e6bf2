// Shared device/host definitions of librgf (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <string>

#include "../../include/rgf.h"

namespace rgf {

typedef double2 z64;
typedef float2 z32;

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
__host__ __device__ inline z64 zmake(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline z64 zadd(z64 a, z64 b) { return zmake(a.x + b.x, a.y + b.y); }
__host__ __device__ inline z64 zsub(z64 a, z64 b) { return zmake(a.x - b.x, a.y - b.y); }
__host__ __device__ inline z64 zmul(z64 a, z64 b) { return zmake(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__host__ __device__ inline z64 zconj(z64 a) { return zmake(a.x, -a.y); }
__host__ __device__ inline z64 zneg(z64 a) { return zmake(-a.x, -a.y); }
// c + a*b
__host__ __device__ inline z64 zfma(z64 a, z64 b, z64 c) {
  return zmake(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
// c - a*b
__host__ __device__ inline z64 zfms(z64 a, z64 b, z64 c) {
  return zmake(fma(-a.x, b.x, fma(a.y, b.y, c.x)), fma(-a.x, b.y, fma(-a.y, b.x, c.y)));
}
__host__ __device__ inline double zabs1(z64 a) { return fabs(a.x) + fabs(a.y); }
// 1/b with scaling (Smith's method) so that |b| near the range limits does not overflow
__host__ __device__ inline z64 zinv(z64 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return zmake(1.0 / d, -r / d);
  } else {
    double r = b.x / b.y, d = b.x * r + b.y;
    return zmake(r / d, -1.0 / d);
  }
}
// z*S - H (the operator entry for energy z)
__host__ __device__ inline z64 zform(z64 z, z64 s, z64 h) {
  return zmake(z.x * s.x - z.y * s.y - h.x, z.x * s.y + z.y * s.x - h.y);
}

// ---------------------------------------------------------------------------
// Operand descriptors of the batched block kernels
// ---------------------------------------------------------------------------

// A per-batch dense matrix: element (r, c) of batch b lives at
//   p[b*bstride + row(r)*ld + c],  row(r) = rowidx ? rowidx[b*ridx_bstride + r] : r.
struct MatRef {
  z64* p;
  int64_t bstride;
  int64_t ld;
  const int32_t* rowidx;
  int64_t ridx_bstride;
};

// An operator block formed on the fly: z_b*S - H from blocks shared by all
// batches (logical size M; rows/cols >= M read as zero, or as the identity
// on the diagonal when pad_identity is set).  conj_t forms (z_b*S - H)
// with S, H replaced by their adjoints: z_b*S^+ - H^+.
// z_b = E[b] + i*eta.  When sub is set, sub_sign*sub[b] is added.
// Grouped batches (gper > 0): batch entry b reads the blocks of group
// (gb0 + b) / gper, which sit gstride elements after those of the group
// before (several devices of one shape, e.g. the k-points of a mesh, in one
// batch).
struct FormRef {
  const z64* H;
  const z64* S;
  int32_t M;
  int32_t conj_t;
  int32_t pad_identity;
  int32_t gper;
  int64_t gb0;
  int64_t gstride;
  const double* E;
  double eta;
  MatRef sub;        // optional per-batch matrix added with sub_sign (p == nullptr: none)
  double sub_sign;
};

// element offset of batch entry b's blocks in a grouped batch
__host__ __device__ inline int64_t form_group_off(const FormRef& f, int b) {
  return f.gper > 0 ? ((f.gb0 + b) / f.gper) * f.gstride : 0;
}

// Per-batch skip flags: a batch entry with skip[b] != 0 is left untouched.
struct BatchCtl {
  const int32_t* skip;
};

__device__ inline z64 form_elem(const FormRef& f, int b, int r, int c) {
  z64 v = zmake(0.0, 0.0);
  if (r < f.M && c < f.M) {
    z64 z = zmake(f.E[b], f.eta);
    const int64_t g = form_group_off(f, b);
    if (f.conj_t) {
      z64 s = f.S[g + (int64_t)c * f.M + r];
      z64 h = f.H[g + (int64_t)c * f.M + r];
      v = zform(z, zconj(s), zconj(h));
    } else {
      v = zform(z, f.S[g + (int64_t)r * f.M + c], f.H[g + (int64_t)r * f.M + c]);
    }
  } else if (f.pad_identity && r == c) {
    v = zmake(1.0, 0.0);
  }
  if (f.sub.p) {
    z64 s = f.sub.p[b * f.sub.bstride + (int64_t)r * f.sub.ld + c];
    v = zmake(v.x + f.sub_sign * s.x, v.y + f.sub_sign * s.y);
  }
  return v;
}

__device__ inline int64_t mat_off(const MatRef& m, int b, int r, int c) {
  int64_t row = m.rowidx ? (int64_t)m.rowidx[b * m.ridx_bstride + r] : (int64_t)r;
  return b * m.bstride + row * m.ld + c;
}

inline MatRef mat(z64* p, int64_t bstride, int64_t ld, const int32_t* ridx = nullptr, int64_t rbs = 0) {
  MatRef m;
  m.p = p;
  m.bstride = bstride;
  m.ld = ld;
  m.rowidx = ridx;
  m.ridx_bstride = rbs;
  return m;
}
inline MatRef nomat() { return mat(nullptr, 0, 0); }

inline FormRef form(const rgf_z* H, const rgf_z* S, int M, bool conj_t, bool pad_identity,
                    const double* E, double eta) {
  FormRef f;
  f.H = reinterpret_cast<const z64*>(H);
  f.S = reinterpret_cast<const z64*>(S);
  f.M = M;
  f.conj_t = conj_t ? 1 : 0;
  f.pad_identity = pad_identity ? 1 : 0;
  f.gper = 0;
  f.gb0 = 0;
  f.gstride = 0;
  f.E = E;
  f.eta = eta;
  f.sub = nomat();
  f.sub_sign = 0.0;
  return f;
}

// ---------------------------------------------------------------------------
// Host-side error plumbing
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
struct Error {
  int code;
  std::string msg;
};

#define RGF_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::rgf::Error{RGF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define RGF_CHECK(cond, code, msg)                      \
  do {                                                  \
    if (!(cond)) throw ::rgf::Error{(code), (msg)};     \
  } while (0)

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace rgf
