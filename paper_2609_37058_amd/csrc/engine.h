// Host-side driver of the batched transmission path (one chunk of energies).
#pragma once

#include <vector>

#include "common.h"
#include "kernels.h"

namespace rgf {

constexpr double SR_TOL = 1e-14;
constexpr int SR_MAXIT = 100;  // decimation cap (2^100 layers, far beyond 1/eta)
// the cap in effect: SR_MAXIT unless lowered by rgf_set_sr_maxit
int sr_maxit();
constexpr int32_t SING_LEAD = 0x1000000;  // stored code; decodes to layer field 0xFFFFFF

struct Profiler;
Profiler& profiler();

constexpr int MAX_M = 2048;  // largest block size the library accepts

// tuning table: block-product tile and energy lanes for (precision, padded size)
int tile_for(int prec, int Mp);
int lanes_for(int Mp, int prec);
int mixed_parts();  // RGF_MIXED_* bits in effect for the mixed path

// Device memory for `batch` energies at padded block size Mp.
struct Layout {
  int Mp = 0, batch = 0;
  int nblk_sr = 0;
  size_t bytes = 0;
  // offsets (bytes) into the arena
  size_t sig, un, linv, uinv, perm, cand, cand2, flags, ints, dbl;
  size_t energies, tout, iout;  // staged energies and sweep outputs (stable addresses for graphs)
  size_t elead, erlead;         // energies of the left / right electrode when biased (E - u)
  static Layout make(int Mp, int batch);
};

class Engine {
 public:
  Engine(char* arena, const Layout& lay, hipStream_t st, int prec, int M, const double* E, double eta,
         int32_t* host_active);

  // The lead steps run at the chunk's energies, or at energies given per side:
  // an electrode rigidly shifted by u (H -> H + u S) is the unshifted one at E - u.
  void set_lead_energies(const double* EL, const double* ER) {
    EL_ = EL;
    ER_ = ER;
  }
  // A grouped batch: entry b uses the device and electrode blocks of group
  // (b0 + b) / per, `stride` elements after those of the group before; the
  // blocks passed to the calls below are those of group 0.
  // Look-ahead in the blocked LU (a side stream per stream, created on first use; on with
  // RGF_LOOKAHEAD=1).  Callers that must not create streams turn it off.
  void set_lookahead(bool on) {
    if (!on) lu_.cand2 = nullptr;
  }
  void set_group(int per, int64_t b0, int64_t stride) {
    gper_ = per;
    gb0_ = b0;
    gstride_ = stride;
  }
  // decimation of `lead` for all energies of the chunk (those of side `left`);
  // leaves eps_L, eps_R
  void decimate(const rgf_lead& lead, int32_t* done, bool left = true);
  // sigma = L (eps_L^-1 U) for the left side, U (eps_R^-1 L) for the right side
  void self_energy(const rgf_lead& lead, bool left, z64* out);
  // Gamma_L, Gamma_R from Sigma_L, Sigma_R
  void broadenings();
  // recursive sweep over the device, then the Caroli trace into T/info
  void sweep_and_trace(const rgf_device& d, double* T, int32_t* info, bool same_leads);
  // orbital-resolved LDOS and the electrode-injected parts, each [batch][N][M]
  // (any may be null), after the self-energies and broadenings; `store` holds
  // N Mp^2 per energy (batch stride N Mp^2), `twos` one double per energy,
  // `sblk` three Mp^2 blocks shared by all energies (overlap operands)
  void local_dos(const rgf_device& d, z64* store, double* twos, z64* sblk, double* dos, double* ados_l,
                 double* ados_r, int32_t* info, bool same_leads);
  // lead-only output: copy sigma into the caller's dense [batch][M][M]
  void export_sigma(z64* sigma_ws, rgf_z* out);
  void lead_info(int side_bit, int32_t* done, int32_t* info);

  z64* sigL() { return sigL_; }
  z64* sigR() { return sigR_; }
  // Sigma of batch entry b (Mp x Mp, padded), e.g. to fill it from a cache or copy it out
  z64* sigma_slot(int b, bool left) { return (left ? sigL_ : sigR_) + (int64_t)b * MM_; }
  int64_t block_elems() const { return MM_; }
  int32_t* done_l() { return done_l_; }
  int32_t* done_r() { return done_r_; }

 private:
  MatRef mref(z64* p, int64_t ld, int64_t bstride, const int32_t* ridx = nullptr) const;
  // X = T^-1 Y for every batch entry (T destroyed).  The right-hand sides are written into Y by
  // the fills `rhs` (their destination and shape set, no row gather).  Returns Y as the block
  // products should read X: through the pivot rows (fused path) or as it stands (LU path).
  // `fusable`: the fused Gauss-Jordan kernel may serve this solve (the sweep's); the decimation
  // iterates on blocks whose conditioning degrades, where LU with substitution keeps more digits.
  MatRef factor_solve(z64* T, z64* Y, int64_t yld, int64_t ybs, int nrhs, std::vector<FillArgs> rhs,
                      const int32_t* skip, int32_t code, int lp, int tp, int tile, bool fusable,
                      bool exact_u = false);
  double gemm(GemmArgs g, int prec, bool timed);
  void ldos_pass(const rgf_device& d, z64* store, const double* twos, z64* sblk, bool forward, double* dos,
                 double* inj);
  // dst (Mp x Mp per batch entry, batch stride Mp^2) = the formed operand f for `batch` entries
  MatRef store_form(const FormRef& f, z64* dst, int batch);
  FormRef gform(FormRef f) const {
    f.gper = gper_;
    f.gb0 = gb0_;
    f.gstride = gstride_;
    return f;
  }

  hipStream_t st_;
  int prec_, M_, Mp_, B_;
  bool fused_;  // padded blocks up to 192: one fused factor-and-solve launch per sweep solve
  const double* E_;
  const double *EL_, *ER_;  // lead energies per side (E_ unless shifted)
  double eta_;
  int gper_ = 0;
  int64_t gb0_ = 0, gstride_ = 0;
  int64_t MM_;
  int nblk_sr_;
  z64 *sigL_, *sigR_, *gamL_, *gamR_;
  z64 *eps_, *epsL_, *epsR_, *AB_, *C_, *Tsr_, *Ysr_;
  z64 *T_, *Y_, *Wa_, *Wb_, *P_, *Z1_, *Z2_;
  LuBufs lu_;
  int32_t* cand2_ = nullptr;
  int32_t *done_l_, *done_r_, *iters_, *sing_, *active_;
  double *scale_, *partial_;
  int32_t* host_active_;
};

// Several devices of one shape in one batch: group g's blocks (device and
// electrodes) sit g * stride elements after those of the device passed, and
// its `per` energies are entries [g * per, (g + 1) * per) of the batch.
struct Grouping {
  int per = 0;  // 0: one device
  int64_t stride = 0;
};

// ---- one device through the path (api.hip) ----
void check_device(const rgf_device& d);
// Debug input checks (rgf_set_checks): Hermitian H_ii, S_ii (and the electrodes' H00, S00 when
// `leads`), overlap diagonals real and positive; synchronous, throws RGF_EINVAL naming the first
// failing block, returns max |X - X^+| / max(1, max |X|).
constexpr double INPUT_CHECK_TOL = 1e-10;
bool input_checks();
double check_inputs(const rgf_device& d, double tol, bool leads, hipStream_t st);
bool uses_small_path(int M, int precision);
SmallArgs small_args(const rgf_device& d, const double* E, int64_t nE, double eta, double* T, int32_t* info);
// the whole path for one device on one stream (no lanes); mem_share scales the
// workspace budget when several devices run side by side
// u_l, u_r: rigid shifts of the left / right electrode (finite bias; 0 at zero bias)
void run_device(const rgf_device& d, const double* E, int64_t nE, double eta, int precision, double* T,
                int32_t* info, hipStream_t st, double mem_share, double u_l = 0.0, double u_r = 0.0,
                const Grouping& grp = Grouping());
void transmission_impl(const rgf_device& d, const double* E, int64_t nE, double eta, int precision, double* T,
                       int32_t* info, hipStream_t st, double u_l = 0.0, double u_r = 0.0,
                       const Grouping& grp = Grouping());
// free the k-mesh and KPM arenas held for device `dev` (the caller has synchronized it)
void release_kmesh_arenas(int dev);
void release_kpm_arenas(int dev);

// orbital-resolved LDOS ([nE][N][M] each, any may be null), FP64, on one stream
void ldos_impl(const rgf_device& d, const double* E, int64_t nE, double eta, double* dos, double* ados_l,
               double* ados_r, int32_t* info, hipStream_t st);

}  // namespace rgf
