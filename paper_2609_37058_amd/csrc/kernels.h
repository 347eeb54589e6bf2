// Kernel argument blocks and launchers of librgf (host + device declarations).
#pragma once

#include "common.h"

namespace rgf {

// ---------------------------------------------------------------- small path
struct SmallArgs {
  int N, M;
  const z64 *Hd, *Hu, *Sd, *Su;
  const z64 *LH00, *LH01, *LS00, *LS01;
  const z64 *RH00, *RH01, *RS00, *RS01;
  int same_leads;
  const double* E;
  int64_t nE;
  double eta;
  double* T;
  int32_t* info;
  double sr_tol;
  int sr_maxit;
  double u_l, u_r;  // rigid shifts of the electrodes: each lead runs at z - u
};
constexpr int SMALL_MAX_M = 16;
void launch_small(const SmallArgs& a, hipStream_t st);
// one device's energies [item0, item0 + a.nE) of a persistent multi-device launch
struct SmallJob {
  SmallArgs a;
  int64_t item0;
};
// persistent launch of `grid` workgroups over `total` items of the jobs (device
// memory, item0 ascending); *counter must be 0 on entry
void launch_small_queue(const SmallJob* jobs, int njobs, int64_t total, unsigned long long* counter, int grid,
                        hipStream_t st);

// ---------------------------------------------------------- block products
// C[b] = Cin[b] + alpha * opA[b] * opB[b], complex, for rows x cols outputs
// with inner dimension K (all multiples of the tile).  opA is a per-batch
// matrix or a formed operator block; opB is a per-batch matrix (optionally
// row-gathered); Cin is none, a per-batch matrix or a formed block.
enum { SRC_NONE = 0, SRC_MAT = 1, SRC_FORM = 2 };
enum { PREC_F64 = 0, PREC_F32 = 1 };

struct GemmArgs {
  int rows, cols, K, batch;
  int a_kind;
  MatRef A;
  FormRef Af;
  MatRef B;
  int c_kind;
  MatRef Cin;
  FormRef Cf;
  MatRef C;
  double alpha;
  BatchCtl ctl;
};

// A product of rows x cols outputs with inner dimension K over `batch` entries,
// every operand unset (A, B, Cin and C are filled in by the caller), alpha = 1.
inline GemmArgs gemm_args(int rows, int cols, int K, int batch, const int32_t* skip = nullptr) {
  GemmArgs g;
  g.rows = rows;
  g.cols = cols;
  g.K = K;
  g.batch = batch;
  g.a_kind = SRC_MAT;
  g.A = nomat();
  g.Af = form(nullptr, nullptr, 0, false, false, nullptr, 0.0);
  g.B = nomat();
  g.c_kind = SRC_NONE;
  g.Cin = nomat();
  g.Cf = g.Af;
  g.C = nomat();
  g.alpha = 1.0;
  g.ctl.skip = skip;
  return g;
}

// ------------------------------------------------------- kernel timing
// Classes of launches for the kernel-time breakdown (rgf_profile_classes);
// the values are the RGF_PROF_* bits of the C ABI.
enum {
  PC_SWEEP = RGF_PROF_SWEEP,
  PC_LU_UPDATE = RGF_PROF_LU_UPDATE,
  PC_SOLVE = RGF_PROF_SOLVE,
  PC_ROW64 = RGF_PROF_ROW64,
  PC_PANEL = RGF_PROF_PANEL,
  PC_LEAD = RGF_PROF_LEAD,
  PC_OTHER = RGF_PROF_OTHER,
  PC_FUSED = RGF_PROF_FUSED,
  PC_COUNT = RGF_PROF_COUNT
};
bool profiling();
// event pair around one launch on `st` when its class is sampled; end() also
// counts the launch's algorithmic flops (timed or not) while profiling is on
void profile_launch_begin(hipStream_t st, int cls);
void profile_launch_end(hipStream_t st, int cls, double flops);
// the class of a block product of `rows` output rows with kernel role `role`, and of an LU panel,
// given the calling thread's site and phase
int profile_class(int role, int rows);
int profile_panel_class();
// Flops counted so far by the calling thread's launches (a running total while profiling), and
// the removal of counted flops from a class: a launch counts every energy of its batch, so work
// that energies skip in-kernel (a converged decimation) is taken back out afterwards.
double profile_thread_flops();
void profile_uncount_flops(int cls, double flops);
// Scope guards (thread-local): products launched inside belong to `cls` (unless they are
// role-1 or 64-row products), or, inside a lead scope, to the decimation and self-energies.
struct ProfSite {
  explicit ProfSite(int cls);
  ~ProfSite();
  int prev;
};
struct ProfLead {
  ProfLead();
  ~ProfLead();
  bool prev;
};

// tile = 64 or 128 (square output tiles); role 1 marks the sweep's main block
// products (a separate kernel symbol, so profiles can single them out).
// Returns the algorithmic flops launched.
double launch_gemm(const GemmArgs& g, int prec, int tile, hipStream_t st, int role = 0);
// Largest inner dimension that takes the short-K product tiles (0: never).  Defaults to 128,
// or RGF_SMALLK_MAXK from the environment; the setter returns the previous value.
int small_k_max();
int set_small_k_max(int k);

// ------------------------------------------- LU with partial pivoting
constexpr int LU_NB = 64;
struct LuPanelArgs {
  MatRef T;  // Mp x Mp per batch, factored in place; ld >= Mp
  int Mp;
  int k0;
  z64* linv;  // per batch: Mp/64 blocks of 64 x 64 (inverse diagonal blocks of L)
  z64* uinv;  // per batch: Mp/64 blocks of 64 x 64 (inverse diagonal blocks of U)
  int64_t inv_bs;
  int32_t* perm;
  int64_t perm_bs;  // Mp per batch
  uint8_t* flags;
  int64_t flags_bs;  // Mp per batch
  int32_t* cand;
  int64_t cand_bs;  // Mp per batch: rows still candidates after the panel, ascending
  int32_t* sing;    // per batch: first singular event code (0 = none)
  int32_t sing_code;
  BatchCtl ctl;
  int u_plain = 0;  // 1: uinv receives the diagonal blocks of U themselves, not their inverses
};
void launch_lu_panel(const LuPanelArgs& a, int batch, hipStream_t st);

// Buffers of a batched LU (per batch: linv, uinv 64 x Mp each, perm, cand Mp, flags Mp, sing 1).
// cand2 (Mp per batch, optional) is a second candidate list: with it the factorisation looks
// ahead (see lu_factor), alternating the two lists between pairs of panels.
struct LuBufs {
  z64* linv;
  z64* uinv;
  int32_t* perm;
  int32_t* cand;
  uint8_t* flags;
  int32_t* sing;
  int32_t* cand2 = nullptr;
  // Exact diagonal blocks of U: the factorisation keeps U's 64 x 64 diagonal blocks (in uinv's
  // storage) and the solve substitutes with them instead of applying their explicit inverses,
  // which lose digits when U is ill-conditioned (the lead decimation near band extrema).
  bool exact_u = false;
};
// Factor T (Mp x Mp per batch, batch stride bs) in place.  Block products
// (trailing updates) run in `prec`; pivoting and diagonal blocks in FP64.
// With g.cand2 set (and st not capturing a graph), the columns more than one
// pair of panels ahead are updated on a side stream while st factors the next
// pair; st has waited for all of it when the call returns.
void lu_factor(const LuBufs& g, z64* T, int64_t bs, int Mp, int batch, const int32_t* skip, int32_t code,
               int prec, int tile, hipStream_t st);
// Y <- U^-1 L^-1 Y in place (Y = P RHS already gathered; Mp x nrhs per batch, ld nrhs).
void lu_solve(const LuBufs& g, z64* T, int64_t bs, int Mp, z64* Y, int64_t ybs, int nrhs, int batch,
              const int32_t* skip, int prec, int tile, hipStream_t st);

// Fused factor-and-solve for padded block sizes up to GJ_MAX_MP: X = B^-1 Y per batch entry
// in one launch (one workgroup per entry; blocked Gauss-Jordan with partial pivoting, rows in
// place).  B is destroyed; Y is overwritten so that row perm[j] of Y holds row j of X.
constexpr int GJ_MAX_MP = 256;
struct GjArgs {
  z64* T;            // B, Mp x Mp (ld Mp) per entry
  int64_t tbs;       // batch stride of T
  z64* Y;            // right-hand sides, Mp x nrhs (ld nrhs) per entry
  int64_t ybs;       // batch stride of Y
  int nrhs;          // multiple of 16
  int Mp;            // 64, 128, 192 or 256
  int32_t* perm;     // out: Mp per entry
  int64_t perm_bs;
  int32_t* sing;     // per entry: first singular event code (0 = none)
  int32_t sing_code;
  const int32_t* skip;  // entries to leave alone (null: none)
};
// returns the matrix-core flops launched
double launch_gj(const GjArgs& a, int batch, hipStream_t st);

// ---------------------------------------------------------- elementwise
enum { FILL_ZERO = 0, FILL_IDENTITY = 1, FILL_MAT = 2, FILL_FORM = 3 };
struct FillArgs {
  MatRef dst;  // rows x cols block
  int rows, cols;
  int kind;
  double scale;  // multiplies the source (identity: the diagonal value)
  MatRef src;
  FormRef f;
  uint8_t* flags;  // optional: zeroed (Mp per batch) -- reset of pivot flags
  int64_t flags_bs;
  int flags_n;
  const int32_t* ridx;  // optional row gather of FORM / IDENTITY sources: source row = ridx[r]
  int64_t ridx_bs;
  BatchCtl ctl;
};
void launch_fill(const FillArgs& a, int batch, hipStream_t st);
// dst[b] (Mp x Mp) = the formed operand f with f.conj_t taken as set: z_b S^+ - H^+,
// padded like a formed operand; f.sub must be unset.
void launch_form_ct(const FormRef& f, MatRef dst, int Mp, int batch, hipStream_t st);
// out[4 b .. 4 b + 3] for each of nblk consecutive M x M blocks of X: max |X - X^+|, max |X|
// (component-wise |re| + |im| measures), min Re of the diagonal, max |Im| of the diagonal
void launch_herm_check(const z64* X, int M, int nblk, double* out, hipStream_t st);
// A fill of `kind` into dst (rows x cols) with no source, no row gather and scale 1.
inline FillArgs fill_args(MatRef dst, int rows, int cols, int kind) {
  FillArgs f;
  f.dst = dst;
  f.rows = rows;
  f.cols = cols;
  f.kind = kind;
  f.scale = 1.0;
  f.src = nomat();
  f.f = form(nullptr, nullptr, 0, false, false, nullptr, 0.0);
  f.flags = nullptr;
  f.flags_bs = 0;
  f.flags_n = 0;
  f.ridx = nullptr;
  f.ridx_bs = 0;
  f.ctl.skip = nullptr;
  return f;
}
// synthetic inputs: p[i] = scale (u + i v) (+ diag on block diagonals), u, v uniform in [-1, 1)
void launch_random(z64* p, int64_t n, int64_t ld, int64_t rows, double scale, double diag, uint64_t seed,
                   hipStream_t st);

// Bloch sum over transverse images: dst[i] = sum_r w[r] src[r][i] (null src[r]: a zero block)
constexpr int MAX_IMAGES = 32;
struct BlochArgs {
  const z64* src[MAX_IMAGES];
  z64 w[MAX_IMAGES];
  int nR;
  z64* dst;
  int64_t n;
};
void launch_bloch(const BlochArgs& a, hipStream_t st);
// T[e] = (first ? 0 : T[e]) + w * Tk[e]: the k-point average, accumulated in mesh order
void launch_kaccum(double* T, const double* Tk, double w, int64_t n, int first, hipStream_t st);

// dst[k] = src[k] - u, k < n (energies of a rigidly shifted electrode)
void launch_shift(double* dst, const double* src, int64_t n, double u, hipStream_t st);
// I[0] = G0 * trapezoid over the ascending E of (f(E, mu_L) - f(E, mu_R)) T, one workgroup,
// fixed summation order
void launch_landauer(const double* E, const double* T, int64_t n, double mu_l, double mu_r, double kT, double* I,
                     hipStream_t st);

// dst[b] += s * src[b] (rows x cols)
void launch_axpy(MatRef dst, MatRef src, double s, int rows, int cols, int batch, BatchCtl ctl,
                 hipStream_t st);

struct SrUpdateArgs {
  int Mp;
  MatRef C;      // 2Mp x 2Mp products [aXa aXb; bXa bXb]
  MatRef eps, epsL, epsR;
  MatRef AB;     // 2Mp x Mp: alpha over beta
  double* partial;  // per batch: gridDim.x blocks x 2 sums of squares
  int nblk;
  BatchCtl ctl;
};
void launch_sr_update(const SrUpdateArgs& a, int batch, hipStream_t st);
// per batch: sqrt-sums of partials vs tol*scale -> done/iters; counts still-active batches
void launch_sr_check(const double* partial, int nblk, const double* scale, double tol, int it,
                     int32_t* done, int32_t* iters, int32_t* active_count, int batch, hipStream_t st);
// per batch: scale[b] = max(1, ||X[b]||_F) over rows x cols
void launch_frob_scale(MatRef X, int rows, int cols, double* scale, int batch, hipStream_t st);
// gamma[b] = i (sigma[b] - sigma[b]^+), Mp x Mp
void launch_broadening(MatRef sigma, MatRef gamma, int Mp, int batch, hipStream_t st);
// T[b] = Re sum Z1 .* conj(Z2); info composition; NaN on singular/nonfinite
struct TraceArgs {
  MatRef Z1, Z2;
  int Mp;
  double* T;
  int32_t* info;
  const int32_t* sr_done_l;  // decimation converged flags (1 = converged) of left/right
  const int32_t* sr_done_r;
  const int32_t* sing;       // per batch singular code (0 = none)
};
void launch_trace(const TraceArgs& a, int batch, hipStream_t st);
// copy sigma (Mp-padded workspace) into a dense [batch][M][M] user buffer, and info bits
void launch_unpad(MatRef src, z64* dst, int M, int batch, hipStream_t st);
void launch_sr_info(const int32_t* done, int32_t bit, const int32_t* sing, int32_t* info, int batch,
                    int accumulate, hipStream_t st);

}  // namespace rgf
