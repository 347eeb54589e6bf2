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
 * block inverse of the sweep refined by one FP64 Newton-Schulz step).
 * Two calls on different streams of one device may run concurrently; two
 * calls on the same stream are serialised by the stream.
 * Equal left and right lead pointers share one decimation loop.
 */
int rgf_transmission(const rgf_device* dev, const double* E, int64_t nE, double eta,
                     int precision, double* T, int32_t* info, void* stream);

/*
 * lead_self_energy -- Sigma of one lead for side RGF_LEFT (L g_L U) or
 * RGF_RIGHT (U g_R L), written to sigma[nE][M][M] (device pointer, row-major,
 * device-side block).  Same pointer, stream and info conventions as
 * rgf_transmission; info bits 1/2 flag decimation that hit the iteration cap.
 */
int lead_self_energy(const rgf_lead* lead, int side, const double* E, int64_t nE, double eta,
                     int precision, rgf_z* sigma, int32_t* info, void* stream);

/*
 * Serving: a request loop with continuous batching.  transport_submit copies
 * the HOST inputs (device blocks, energies) into library staging before it
 * returns, so the caller may free them at once; the request is admitted to
 * the GPU when the HBM budget and a slot allow; requests in flight overlap on
 * the device.  Lead self-energies (always FP64) are cached on the device per
 * (lead key, side, E bit pattern, eta) under lead_cache_bytes;
 * equal keys MUST mean identical lead blocks.  transport_poll copies T and
 * info to HOST buffers [nE] and the submit-to-completion latency in seconds;
 * it returns RGF_EAGAIN while the request is not finished, and RGF_ENOTICKET
 * once collected.  submit and poll may be called from several threads.
 * transport_close drains the requests in flight and frees every device
 * buffer of the server.
 */
typedef struct {
  uint64_t hbm_budget_bytes; /* device memory for requests in flight (0: 60% of free) */
  uint64_t lead_cache_bytes; /* device memory for cached lead self-energies */
  int32_t max_slots;         /* requests in flight at once (0: 4) */
} rgf_server_opts;

int transport_open(const rgf_server_opts* opts, void** server);
int transport_submit(void* server, const rgf_device* dev, uint64_t lead_key_L, uint64_t lead_key_R,
                     const double* E, int64_t nE, double eta, int precision, uint64_t* ticket);
int transport_poll(void* server, uint64_t ticket, double* T, int32_t* info, double* latency_s);
int transport_close(void* server);

/* Serving counters: requests finished, lead-cache hits and misses, peak bytes in flight. */
typedef struct {
  uint64_t finished, cache_hits, cache_misses, peak_inflight_bytes, cache_bytes;
} rgf_server_stats;
int transport_stats(void* server, rgf_server_stats* stats);

/* Diagnostics.  rgf_last_error: message of the last failure on this thread
 * (static storage, valid until the next call on the thread). */
const char* rgf_last_error(void);
const char* rgf_version(void);

/* Release every cached device workspace of the current device. */
int rgf_release_workspaces(void);

/*
 * Kernel timing.  rgf_profile(1) makes later calls record a HIP event pair
 * around every launch of the dominant block-product kernel on the stream it
 * is launched on; rgf_profile_read returns the number of such launches, their
 * summed duration in milliseconds and their summed algorithmic flops (8 real
 * flops per complex multiply-add), then resets the counters.  Recording adds
 * a little overhead, so leave it off outside measurement.
 */
int rgf_profile(int enable);
int rgf_profile_read(int64_t* launches, double* total_ms, double* flops);

/* Tile configuration of the FP64 and mixed block products: 128 (128x128 output
 * tiles, 64-row tiles for 64-row products) or 64 (64x64 tiles).  Applies to later
 * calls in the process. */
int rgf_get_tile(int precision, int32_t* tile);
int rgf_set_tile(int precision, int32_t tile);

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

#ifdef __cplusplus
}
#endif

#endif /* RGF_H */
