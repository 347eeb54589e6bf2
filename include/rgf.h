/*
 * rgf.h -- C ABI of librgf: energy-resolved transmission through a
 * block-tridiagonal nonorthogonal device, on AMD Instinct MI355X (gfx950).
 *
 * The operation (paper: Introduction and the Results paragraph on the cost
 * of each stage; Fig. 1(b)): a device of N principal layers of M orbitals
 * with a static Hamiltonian H and overlap S, coupled to two semi-infinite
 * electrodes whose self-energies are computed from the bulk electrode, is
 * solved by the recursive Green's function method at O(N M^3) per energy.
 * With z = E + i*eta the library computes, per energy,
 *
 *   lead surface GFs g_L, g_R        Sancho-Rubio decimation of the lead
 *   Sigma_L = L_L g_L U_L            U = z S01 - H01, L = z S01^+ - H01^+
 *   Sigma_R = U_R g_R L_R            (of the left / right lead)
 *   Gamma   = i (Sigma - Sigma^+)
 *   G_1N    first-row block of (z S - H - Sigma_L (+) 0 (+) Sigma_R)^-1
 *   T(E)    = Re Tr[Gamma_L G_1N Gamma_R G_1N^+]      (Caroli formula)
 *
 * Data layout
 *   - Complex scalars are rgf_z = {double re, im}: the memory layout of
 *     std::complex<double>, numpy complex128 and torch.complex128.
 *   - A block is M x M, row-major, dense.  Per-layer blocks are stacked
 *     layer-major: Hd[i] (i = 0..N-1) is H_ii at Hd + i*M*M.
 *   - Hu[i] (i = 0..N-2) is H_{i,i+1}: rows in layer i, columns in layer i+1;
 *     H_{i+1,i} = Hu[i]^+.  Su likewise.
 *   - A lead is one principal layer: H00, S00 (on-site) and H01, S01
 *     (coupling of lead layer n to n+1 in the +z direction, for BOTH leads;
 *     the left lead's H01 points towards the device, the right lead's away
 *     from it).  Device layer 0 couples to the left lead's surface layer via
 *     the left lead's (H01, S01); device layer N-1 couples to the right
 *     lead's surface layer via the right lead's (H01, S01).
 *   - eta (eV, > 0) multiplies S everywhere: A = (E + i eta) S - H, in the
 *     leads and in the device.  z is never conjugated in the lower blocks.
 *
 * Return codes are RGF_OK or a negative RGF_E*; the message of the last
 * failure on the calling thread is available from rgf_last_error().
 * Per-energy numerical status goes to info[k] (LAPACK style), 0 = ok:
 *   RGF_INFO_SR_LEFT / RGF_INFO_SR_RIGHT  decimation hit the iteration cap
 *                                         (the last iterate is used)
 *   RGF_INFO_SINGULAR   an exactly zero pivot; bits 8.. hold the layer index
 *                       (layer N means the final inverse, -1 i.e. 0xFFFFFF a
 *                       lead); T[k] is NaN
 *   RGF_INFO_NONFINITE  T[k] is not finite (T[k] = NaN)
 *
 * Ownership: the caller owns every buffer it passes.  The library owns its
 * device workspaces (grown on demand, per device and stream, released by
 * rgf_release_workspaces or at process exit), its staging copies and the
 * serving lead cache.
 */
#ifndef RGF_H
#define RGF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } rgf_z;

typedef struct {
  int32_t M;
  const rgf_z *H00, *H01, *S00, *S01;
} rgf_lead;

typedef struct {
  int32_t N, M;
  const rgf_z *Hd, *Hu, *Sd, *Su; /* Hd, Sd: [N][M][M]; Hu, Su: [N-1][M][M] */
  rgf_lead left, right;
} rgf_device;

enum { RGF_FP64 = 0, RGF_MIXED = 1 };
enum { RGF_LEFT = 0, RGF_RIGHT = 1 };
enum {
  RGF_OK = 0,
  RGF_EINVAL = -1,   /* null pointer, N < 1, M < 1, nE < 0, eta < 0 or NaN, lead.M != M,
                        bad precision or side */
  RGF_ENOMEM = -2,   /* a device workspace could not be allocated */
  RGF_EDEVICE = -3,  /* a HIP runtime error (launch failure, no device) */
  RGF_EAGAIN = -4,   /* serving: the ticket is not finished yet */
  RGF_ETOOBIG = -5,  /* serving: the request exceeds the whole HBM budget */
  RGF_ENOTICKET = -6 /* serving: unknown or already collected ticket */
};
enum {
  RGF_INFO_SR_LEFT = 1,
  RGF_INFO_SR_RIGHT = 2,
  RGF_INFO_SINGULAR = 4,
  RGF_INFO_NONFINITE = 8
};

/*
 * rgf_transmission -- T(E_k), k = 0..nE-1, of one device (the whole path:
 * decimation for both leads, self-energies, the recursive sweep over the N
 * layers and the Caroli trace).
 *
 * All pointers are DEVICE pointers on the current HIP device (e.g. torch
 * tensor data_ptr()): the blocks in *dev, E[nE], T[nE] (output) and
 * info[nE] (output, may be NULL).  *dev itself is a host struct.
 * stream: a hipStream_t, NULL for the default stream.  The call is
 * stream-ordered: it validates, enqueues and returns; the caller
 * synchronises the stream before reading T.  Inputs must stay valid until
 * the stream reaches the end of the enqueued work.
 * precision: RGF_FP64 (all arithmetic in FP64) or RGF_MIXED (the block
 * products selected by rgf_set_mixed_parts -- by default those of the sweep,
 * of the LU trailing updates and of the triangular solves -- on the FP32
 * matrix cores with FP32 accumulation; decimation, self-energies, pivot
 * search, the diagonal-block inverses and the trace in FP64, and the final
 * block inverse of the sweep refined by one FP64 Newton-Schulz step).  The
 * FP32 rounding is amplified by the conditioning of the layer blocks, so the
 * mixed result can differ from the FP64 one by far more than FP32 rounding
 * when eta is small (measured up to 5e-3 absolute in T at eta = 1e-6 on
 * 60-200 layer devices of M = 256-512).
 * Two calls on different streams of one device may run concurrently; two
 * calls on the same stream are serialised by the stream.
 * Equal left and right lead pointers share one decimation loop.
 */
int rgf_transmission(const rgf_device* dev, const double* E, int64_t nE, double eta,
                     int precision, double* T, int32_t* info, void* stream);

/*
 * rgf_transmission_noalloc -- rgf_transmission for callers that cannot
 * allocate device memory: code in tight serving loops, harnesses that forbid
 * hipMalloc, or callers that set up all memory in advance.  It computes the
 * same T(E) with the same kernels (bitwise the values rgf_transmission
 * returns: every per-energy step is independent of how energies are
 * chunked), but it calls no hipMalloc, hipFree or other allocating routine:
 * its workspace is a file-scope device array of RGF_NOALLOC_SCRATCH_BYTES
 * (128 MiB) that each GPU the library runs on holds from module load until
 * the process ends.  The energies run in chunks that fit that array, on the
 * caller's stream only (one lane, no captured graphs, no debug input checks).
 * Blocks with M <= 16 (FP64) take the small-block kernel, which needs no
 * scratch memory at all.  RGF_ETOOBIG when one energy's workspace does not fit
 * the array (M above 704).  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (on different streams or from different
 * threads) race, so serialise them.  The array keeps the last call's
 * contents; every flag and counter the path reads is cleared by the call
 * before use.  The call synchronises its stream during decimation (as
 * rgf_transmission does), so it cannot be captured into a graph.  Pointers,
 * precision, info and the other errors as rgf_transmission.
 */
#define RGF_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int rgf_transmission_noalloc(const rgf_device* dev, const double* E, int64_t nE, double eta, int precision,
                             double* T, int32_t* info, void* stream);

/*
 * rgf_transmission_batch -- the batching form: many devices of uneven block
 * size, length and energy count in one call.  devs[ndev] (host array of host
 * structs); E[d], T[d] and info[d] are host arrays of DEVICE pointers to
 * nE[d] energies, results and statuses of device d (info, or any info[d], may
 * be NULL).  Devices that take the small-block path (M <= 16, RGF_FP64) share
 * ONE persistent launch whose workgroups draw (device, energy) items from a
 * work counter until the list is exhausted; the others run costliest first on
 * two internal streams driven by their own host threads.  Every T[d][k] equals
 * what rgf_transmission returns for device d alone (bitwise: no step depends on
 * the other devices or energies).  Same pointer, stream and precision
 * conventions as rgf_transmission; the call returns once the work is
 * enqueued.  RGF_EINVAL for ndev < 0, a null array or any invalid device.
 */
int rgf_transmission_batch(const rgf_device* devs, int32_t ndev, const double* const* E, const int64_t* nE,
                           double eta, int precision, double* const* T, int32_t* const* info, void* stream);

/*
 * rgf_transmission_bias -- T(E, V_b) at finite bias with the zero-bias
 * Hamiltonian (paper: Method, the paragraph after eq. (1): H0 is supplied to
 * the NEGF solver at finite bias, without self-consistent iterations).  The
 * device blocks are used as given; the left / right electrode is rigidly
 * shifted by u_left / u_right (eV): H00 -> H00 + u S00, H01 -> H01 + u S01,
 * S unchanged, so its self-energy is the zero-bias one at E - u.  For a
 * symmetric bias V_b: u_left = +V_b/2, u_right = -V_b/2.  u_left = u_right = 0
 * is rgf_transmission.  Same pointers, stream, precision and info conventions
 * as rgf_transmission; RGF_EINVAL also for non-finite shifts.
 */
int rgf_transmission_bias(const rgf_device* dev, const double* E, int64_t nE, double eta, double u_left,
                          double u_right, int precision, double* T, int32_t* info, void* stream);

/*
 * rgf_landauer_current -- the current of eq. (1) (paper: Method),
 *   I = (2e/h) * integral dE [f(E, mu_left) - f(E, mu_right)] T(E),
 * on the caller's grid: E[nE] (eV, ascending) and T[nE] are DEVICE pointers,
 * f is the Fermi-Dirac occupation at temperature kT (eV; kT = 0: the step,
 * 1/2 at E = mu), the integral is the trapezoid rule, and with energies in eV
 * the prefactor is G0 = 2e^2/h (spin-degenerate conductance quantum, exact SI
 * constants), so I[0] (DEVICE pointer) receives amperes.  One workgroup sums
 * in a fixed order, so the result does not depend on the launch.  nE < 2
 * gives 0.  RGF_EINVAL for nE < 0, null pointers, non-finite mu or kT < 0.
 * Stream-ordered.
 */
int rgf_landauer_current(const double* E, const double* T, int64_t nE, double mu_left, double mu_right,
                         double kT, double* I, void* stream);

/*
 * rgf_transmission_kmesh -- transmission averaged over transverse k-points
 * (paper: Method, the transverse k-point meshes of the transport runs;
 * Results, the cost per energy and per transverse k-point).  images[nR]
 * (host array, 1 <= nR <= 32) holds the real-space blocks of the transverse
 * lattice images R[r] = (R[2r], R[2r+1]) (host int32): image r's Hd, Hu, Sd,
 * Su and electrode blocks are DEVICE pointers as in rgf_transmission, all
 * images of the same N and M; a null block pointer is a zero block.  At the
 * fractional wavevector k = (kpts[2j], kpts[2j+1]) (host) every block is
 *   X(k) = sum_r X(R_r) exp(2 pi i (k_1 R_r1 + k_2 R_r2)),
 * the k-resolved transmission T_k(E) is computed from the X(k) device, and
 *   T[e] = sum_j weights[j] T_kj(E[e])            (weights: host, as given).
 * The caller keeps X(-R) = X(R)^+ for on-site blocks (Hermitian X(k)).
 * Outputs (DEVICE pointers): T[nE]; Tk[nk][nE] (may be NULL); info[nk][nE]
 * (may be NULL).  Electrodes whose blocks are pointer-equal in every image
 * share one decimation.  The assembled devices of up to 64 k-points at a
 * time (within 20% of free memory) run as one batch of k-points x energies
 * (blocks with M <= 16: one multi-device rgf_transmission_batch).
 * Stream-ordered; RGF_EINVAL for nR outside [1, 32], nk < 1, images of
 * different N or M, or no image with electrode blocks.
 */
int rgf_transmission_kmesh(const rgf_device* images, int32_t nR, const int32_t* R, const double* kpts,
                           const double* weights, int32_t nk, const double* E, int64_t nE, double eta,
                           int precision, double* T, double* Tk, int32_t* info, void* stream);

/*
 * rgf_ldos -- orbital-resolved local density of states of the device (paper:
 * Discussion, the spatially resolved LDOS at zero and finite bias; textbook
 * NEGF definitions with the Mulliken projection inside the device).  With
 * G = (z S - H - Sigma_L (+) Sigma_R)^-1, z = E + i eta, on the device:
 *   dos[e][l][mu]        = (1/2pi) Re [A S]_mu,mu,   A = i (G - G^+)
 *   ados_left[e][l][mu]  = (1/2pi) Re [A_L S]_mu,mu, A_L = G Gamma_L G^+
 *   ados_right[e][l][mu] = (1/2pi) Re [A_R S]_mu,mu, A_R = G Gamma_R G^+
 * for layer l and orbital mu (S the device overlap; device-electrode overlap
 * terms are not part of the projection).  dos = ados_left + ados_right +
 * (eta/pi) Re diag(G S G^+ S).  Arrays are [nE][N][M] doubles, DEVICE
 * pointers, row-major; any of the three may be NULL (not all).  info[nE]
 * (DEVICE, may be NULL) as in rgf_transmission.  FP64 only.  The library keeps
 * N padded M x M blocks per energy in its workspace (N Mp^2 x 16 bytes, Mp =
 * M rounded up to 64) and three padded overlap blocks per energy lane, so
 * energies run in chunks that fit 80% of free HBM.
 * Stream-ordered; RGF_EINVAL as rgf_transmission and when no output is given.
 */
int rgf_ldos(const rgf_device* dev, const double* E, int64_t nE, double eta, double* dos, double* ados_left,
             double* ados_right, int32_t* info, void* stream);

/*
 * rgf_kpm_moments -- Chebyshev moments of the nonorthogonal kernel polynomial
 * method (paper: Introduction and Results -- the rescaled operator
 * S^-1 (H - b S) / a of the central region, S applied through linear solves,
 * random vectors, cost O(N_mom N_rand N); textbook KPM: Weisse et al., Rev.
 * Mod. Phys. 78, 275 (2006)).  The central region is the device blocks of dev
 * (Hd, Hu, Sd, Su as in rgf_transmission; the electrode blocks are not read).
 * With a = (e_max - e_min) / (2 - 0.01), b = (e_max + e_min) / 2 and the
 * R random vectors r_j = columns of vectors[(l M + m) R + j] (DEVICE,
 * complex, the caller draws them, e.g. random phases):
 *   mu[n] = Re sum_j r_j^+ T_n(A~) r_j / R,  A~ = S^-1 (H - b S) / a,
 * for n < n_mom (DEVICE array of doubles).  [e_min, e_max] must enclose the
 * spectrum of (H, S).  S is factored once per call (block Thomas, FP64;
 * RGF_EINVAL if a pivot is exactly zero).  The library keeps 3 N Mp^2 complex
 * factors, the 3 N Mp^2 complex blocks of b S - H and 5 N Mp Rp complex
 * vector panels (Mp, Rp = M, R rounded up to 64) in a workspace per stream
 * (RGF_ENOMEM when it does not fit).  Stream-ordered (blocks for the S check);
 * RGF_EINVAL for null pointers, N < 1, M outside [1, 2048], n_mom < 1, R < 1
 * or bad bounds.
 */
int rgf_kpm_moments(const rgf_device* dev, double e_min, double e_max, int32_t n_mom, const rgf_z* vectors,
                    int32_t R, double* mu, void* stream);

/*
 * rgf_kpm_fermi -- the Fermi level from KPM moments by the electron-number
 * constraint (paper: Introduction): with the Jackson kernel g_n,
 *   N(x) = g_0 mu_0 (pi - acos x) / pi - (2/pi) sum_{n>=1} g_n mu_n sin(n acos x) / n
 * counts the states below x = (e - b) / a; e_fermi[0] (DEVICE) receives
 * a x_F + b with N(x_F) = n_states (occupied states, spin not counted), by
 * bisection on [-1, 1] in one workgroup.  mu: DEVICE [n_mom].  Same a, b as
 * rgf_kpm_moments.  Stream-ordered.
 */
int rgf_kpm_fermi(const double* mu, int32_t n_mom, double e_min, double e_max, double n_states, double* e_fermi,
                  void* stream);

/*
 * rgf_kpm_dos -- the kernel-smoothed density of states per unit energy,
 *   rho(E) = [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n T_n(x)] / (pi a sqrt(1 - x^2)),
 * x = (E - b) / a, at E[nE] into dos[nE] (DEVICE pointers).  Stream-ordered.
 */
int rgf_kpm_dos(const double* mu, int32_t n_mom, double e_min, double e_max, const double* E, int64_t nE,
                double* dos, void* stream);

/*
 * lead_self_energy -- Sigma of one lead for side RGF_LEFT (L g_L U) or
 * RGF_RIGHT (U g_R L), written to sigma[nE][M][M] (device pointer, row-major,
 * device-side block).  The paper takes the electrode self-energies from the
 * bulk electrode's Hamiltonian (Introduction; Abstract); here the lead's
 * surface Green's function comes from Sancho-Rubio decimation of its
 * principal layer and Sigma = L g U (left) or U g L (right) with
 * U = z S01 - H01, L = z S01^+ - H01^+.  Same pointer, stream and info
 * conventions as rgf_transmission; info bits 1/2 flag decimation that hit the
 * iteration cap.
 */
int lead_self_energy(const rgf_lead* lead, int side, const double* E, int64_t nE, double eta,
                     int precision, rgf_z* sigma, int32_t* info, void* stream);

/*
 * Serving: a request loop with continuous batching.  transport_submit copies
 * the HOST inputs (device blocks, energies) into library staging before it
 * returns, so the caller may free them at once.  Admission: the queue is
 * scanned in arrival order and every request whose device blocks fit in what
 * the HBM budget leaves is admitted, so a request that does not fit does not
 * block smaller ones behind it; once the oldest waiting request has been
 * passed over 4 times, nothing more is admitted ahead of it until it fits.
 * An admitted request runs as work items of up to 128 energies (fewer when
 * the engine workspace of that many does not fit a worker's arena);
 * max_slots worker threads, each with its own stream and arena, take items
 * round-robin over the admitted requests, so requests in flight overlap on
 * the device and a long request never holds a worker for more than one item.
 * Lead self-energies (always FP64) are cached on the device per (lead key,
 * side, E bit pattern, eta) under lead_cache_bytes; equal keys MUST mean
 * identical lead blocks.  transport_poll copies T and info to HOST buffers
 * [nE] and the submit-to-completion latency in seconds; it returns
 * RGF_EAGAIN while the request is not finished, and RGF_ENOTICKET once
 * collected.  submit and poll may be called from several threads.
 * transport_submit returns RGF_ETOOBIG when one energy's workspace exceeds a
 * worker's arena or the request's blocks exceed the room the arenas leave.
 * transport_close drains the requests in flight and frees every device
 * buffer of the server.
 */
typedef struct {
  uint64_t hbm_budget_bytes; /* device memory of the server (0: 60% of free): half of it, at most
                                16 GiB per slot, is the workers' arenas, the rest holds the blocks
                                of the requests in flight */
  uint64_t lead_cache_bytes; /* device memory for cached lead self-energies */
  int32_t max_slots;         /* requests in flight at once (0: 4) */
} rgf_server_opts;

int transport_open(const rgf_server_opts* opts, void** server);
int transport_submit(void* server, const rgf_device* dev, uint64_t lead_key_L, uint64_t lead_key_R,
                     const double* E, int64_t nE, double eta, int precision, uint64_t* ticket);
int transport_poll(void* server, uint64_t ticket, double* T, int32_t* info, double* latency_s);
int transport_close(void* server);

/* Serving counters: requests finished, lead-cache hits and misses (energies), peak device bytes in
   flight (arenas included), lead-cache bytes, and requests admitted ahead of an older waiting one. */
typedef struct {
  uint64_t finished, cache_hits, cache_misses, peak_inflight_bytes, cache_bytes, admitted_ahead;
} rgf_server_stats;
int transport_stats(void* server, rgf_server_stats* stats);

/* Diagnostics.  rgf_last_error: message of the last failure on this thread
 * (static storage, valid until the next call on the thread). */
const char* rgf_last_error(void);
const char* rgf_version(void);

/*
 * Input checks (debug).  The operator z S - H assumes the Hamiltonian and overlap
 * matrices of a local-orbital basis (paper: Method -- the DFT Hamiltonian and overlap
 * matrices), Hermitian with S positive definite; the library does not check this by
 * itself.  rgf_check_device checks on the device, synchronously on `stream`, that every
 * H_ii, S_ii and both electrodes' H00, S00 are Hermitian to
 * max |X - X^+| <= tol max(1, max |X|) (|x| = |Re x| + |Im x|), that the diagonal of every
 * overlap block is real to the same tolerance and positive, and that the entries are
 * finite; the coupling blocks have no such constraint, and positive diagonals are
 * necessary for S > 0, not sufficient.  Returns RGF_OK with *max_dev (may be NULL) = the
 * largest relative deviation, or RGF_EINVAL with rgf_last_error naming the first failing
 * block.  rgf_set_checks(1) runs the same check with tol = 1e-10 at the start of every
 * rgf_transmission, rgf_transmission_bias, rgf_transmission_batch, rgf_ldos and (device
 * blocks only) rgf_kpm_moments call, which then fails with its error; it synchronizes the
 * stream, so it is off by default.
 */
int rgf_check_device(const rgf_device* dev, double tol, double* max_dev, void* stream);
int rgf_set_checks(int enable);
int rgf_get_checks(void);

/* Release every cached device workspace of the current device (sweep workspaces, batch job
   buffers, k-mesh and KPM arenas); synchronizes the device first. */
int rgf_release_workspaces(void);

/*
 * Kernel timing.  rgf_profile(n), n >= 1, makes later calls record a HIP event
 * pair around every n-th launch of the dominant block-product kernel (counted
 * over all streams from this call on) on the stream it is launched on;
 * rgf_profile(0) stops recording.  rgf_profile_read returns the number of
 * recorded launches, their summed duration in milliseconds and their summed
 * algorithmic flops (8 real flops per complex multiply-add), then resets the
 * counters.  Recording costs two event records per sampled launch, so sample
 * (n > 1) where the launches are short and many, and leave it off outside
 * measurement.  RGF_EINVAL for n < 0.
 */
int rgf_profile(int every);
int rgf_profile_read(int64_t* launches, double* total_ms, double* flops);

/*
 * Kernel timing by class (a breakdown of where a call's kernel time goes).
 * rgf_profile_classes(n, mask) records, like rgf_profile, a HIP event pair
 * around every n-th launch (counted per class) of each class whose bit
 * (1 << RGF_PROF_*) is set in mask; rgf_profile_classes(0, 0) stops.  While
 * either form of profiling is on, the algorithmic flops (8 real flops per
 * complex multiply-add) and the count of EVERY block-product launch of every
 * class are added up too, timed or not.  rgf_profile_read_class returns, for
 * one class, the timed launches, their summed duration (ms) and flops, and
 * the count and flops of all its launches, then resets that class.  The
 * classes:
 *   RGF_PROF_SWEEP      the sweep's two block products (W <- -W X and
 *                       B' = A - L X; in the LDOS and KPM forms their main
 *                       block products)
 *   RGF_PROF_LU_UPDATE  trailing updates of the block LU with more than 64 rows
 *   RGF_PROF_SOLVE      block triangular-solve updates with more than 64 rows
 *   RGF_PROF_ROW64      64-row products (U12 blocks, diagonal-block inverses
 *                       applied in the solves, the second pivot group's update)
 *   RGF_PROF_PANEL      LU panel kernels (pivot search and in-panel elimination
 *                       on the vector units; 0 flops counted)
 *   RGF_PROF_LEAD       every product and panel of the decimation and
 *                       self-energies
 *   RGF_PROF_OTHER      the remaining products (final block inverse, its
 *                       refinement, G_1N and the trace products)
 *   RGF_PROF_FUSED      the sweep's fused factor-and-solve launches at padded
 *                       block sizes up to 192 (one workgroup per energy)
 * RGF_EINVAL for n < 0, unknown mask bits or an unknown class.
 */
enum {
  RGF_PROF_SWEEP = 0,
  RGF_PROF_LU_UPDATE = 1,
  RGF_PROF_SOLVE = 2,
  RGF_PROF_ROW64 = 3,
  RGF_PROF_PANEL = 4,
  RGF_PROF_LEAD = 5,
  RGF_PROF_OTHER = 6,
  RGF_PROF_FUSED = 7,
  RGF_PROF_COUNT = 8
};
int rgf_profile_classes(int every, uint32_t classes);
int rgf_profile_read_class(int cls, int64_t* launches, double* total_ms, double* flops, int64_t* launches_all,
                           double* flops_all);

/* Tile configuration of the FP64 and mixed block products: 128 (128x128 output
 * tiles, 64-row tiles for 64-row products) or 64 (64x64 tiles).  rgf_set_tile
 * sets one tile for every size (replacing the built-in per-size choice and any
 * rgf_set_tuning tile); rgf_get_tile reports it (128 while none was set).
 * Applies to later calls in the process. */
int rgf_get_tile(int precision, int32_t* tile);
int rgf_set_tile(int precision, int32_t tile);

/*
 * Tuning table (the batching form's per-size configuration).  For each padded
 * block size class Mp = ceil(M/64)*64 and precision, the library keeps the
 * block-product tile (64 or 128) and the number of energy lanes (internal
 * streams, each driven by its own host thread, over which one call splits its
 * energies).  0 means the built-in default (tile: the rgf_set_tile value if one
 * was set, else 128 except 64 for FP64 at Mp = 256, the measured faster choice
 * there; lanes: 2 from Mp = 256, else 1).  A setting depends only on (M, precision),
 * never on the batch, so a result does not depend on which energies share a
 * call.  rgf_get_tuning reports the values in effect (defaults resolved);
 * rgf_set_tuning returns RGF_EINVAL for M outside [1, 2048], a tile other than
 * 0/64/128 or lanes outside [0, 4].  Settings apply to later calls in the process.
 */
int rgf_get_tuning(int32_t M, int precision, int32_t* tile, int32_t* lanes);
int rgf_set_tuning(int32_t M, int precision, int32_t tile, int32_t lanes);

/*
 * Captured sweeps.  rgf_set_graphs(1) makes later calls (rgf_transmission and
 * rgf_transmission_batch) capture the sweep of each energy chunk -- the layer
 * recursion's LU panels, triangular solves and block products, the final
 * inverse and the trace -- into a HIP graph the first time a (device blocks,
 * N, M, chunk size, precision, tile, workspace, stream) combination is seen,
 * and replay the instantiated graph on later calls of that shape; the
 * energies are staged into the workspace and the outputs copied out, so a
 * replay serves any energies and output buffers.  Decimation stays eager.
 * At most 32 graphs are kept (least recently used dropped); freeing or
 * growing a workspace drops the graphs that point into it.  Off by default
 * (or as RGF_GRAPHS=1 in the environment sets it); ignored while rgf_profile
 * is on.  The device blocks must stay at the same addresses for a replay to
 * be valid: keep graphs off when a device's block memory is freed and reused.
 */
int rgf_set_graphs(int enable);
int rgf_get_graphs(void);

/*
 * rgf_autotune -- measure the four (tile, lanes) choices {64, 128} x {1, 2}
 * for block size M and `precision` by timing the production sweep (layer
 * recursion, final inverse, trace) on a synthetic three-layer device of
 * `batch` energies (0: 64; reduced to fit 40% of free device memory), store
 * the fastest in the tuning table and return it in *tile and *lanes (either
 * may be NULL).  ms[4] (may be NULL) receives the mean time of one sweep for
 * (64,1), (64,2), (128,1), (128,2), -1 for a choice not timed (lanes 2 with one
 * energy).  Synchronous: it allocates and frees its own device buffers and
 * synchronises the device, so run it while no other call is in flight.  On an
 * error the entry for (M, precision) is reset to the defaults.
 */
int rgf_autotune(int32_t M, int precision, int32_t batch, int32_t* tile, int32_t* lanes, double* ms);

/* Which block products of the sweep run on the FP32 matrix cores when
 * precision == RGF_MIXED (later calls in the process; default RGF_MIXED_ALL).
 * Pivot search, the diagonal-block inverses, decimation, self-energies and the
 * trace are FP64 in every case. */
enum {
  RGF_MIXED_SWEEP = 1, /* W <- -W X and B' = A - L X */
  RGF_MIXED_LU = 2,    /* trailing updates of the block LU */
  RGF_MIXED_SOLVE = 4, /* block triangular solves */
  RGF_MIXED_ALL = 7
};
int rgf_set_mixed_parts(int parts);
int rgf_get_mixed_parts(void);

/*
 * Decimation cap.  The Sancho-Rubio loop stops when ||alpha||_F + ||beta||_F
 * <= 1e-14 max(1, ||D||_F) or after the cap, 100 steps by default (2^100
 * layers, far beyond the 1/eta decay length); an energy that reaches the cap
 * keeps its last iterate and reports RGF_INFO_SR_LEFT / RGF_INFO_SR_RIGHT.
 * rgf_set_sr_maxit(n) lowers the cap to n in [1, 100] for later calls in the
 * process (0 restores 100), e.g. to check the status reporting or to bound
 * the time of a scan; RGF_EINVAL outside [0, 100].
 */
int rgf_set_sr_maxit(int32_t maxit);
int rgf_get_sr_maxit(void);

#ifdef __cplusplus
}
#endif

#endif /* RGF_H */
