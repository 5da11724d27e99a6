/*
 * mondpm.h -- C ABI of the MI355X particle-mesh step for AQUAL MOND.
 *
 * One PM step of Visser, Eijt & de Nijs, "Fast particle-mesh code for
 * Milgromian dynamics" (A&A 2023): Gaussian mass deposition (Eq. smooth),
 * the FFT-based fixed-point solve of the AQUAL equation (Sect. 2.1 and the
 * appendix "Flow scheme of the PM code"), kernel-smoothed forces (Eq. gi)
 * and leapfrog (Eq. motion).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Device pointers are HIP device memory owned by the caller; the library
 *    never frees them.  Host pointers are marked "host".
 *  - Every call is enqueued on the stream given to pm_create and returns
 *    without waiting, except where "synchronises" is stated.  A context is
 *    not thread safe; use one context per stream.
 *  - Lengths are in the caller's units; the pixel width is s = box / n.
 *    Positions are measured from the centre of the FFT box (appendix
 *    "Fourier transforms"): grid index j on an axis is the point
 *    (j - n_pad/2) s.  Grids are [z][y][x] with x fastest.
 *  - Particle arrays: pos and vel are float [N][3] (x, y, z), mass is
 *    float [N].  N may be 0 (the call then does nothing but clears outputs).
 *  - Errors: argument errors return PM_E_INVAL at once and enqueue nothing;
 *    HIP runtime failures return PM_E_DEVICE.  Conditions found on the
 *    device (a kernel ball leaving the physical region, a non-finite
 *    residual, no convergence) are reported in the info structures filled
 *    by the calls that take one; those calls synchronise the stream.
 *    Nothing aborts and nothing throws across this interface.
 */
#ifndef MONDPM_H
#define MONDPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Interpolation function mu (Eq. PDE).  STANDARD: mu(x) = x / sqrt(1+x^2)
 * (Eq. mu) with its inverse nu printed in Sect. 2.1.  DEEP: mu(x) = x,
 * nu(y) = 1/sqrt(y) (Sect. 4).  NEWTON: mu = nu = 1, the high-acceleration
 * limit, in which the solve reduces to a Poisson solve. */
typedef enum { PM_MU_STANDARD = 0, PM_MU_DEEP = 1, PM_MU_NEWTON = 2 } pm_mu;

typedef enum {
  PM_OK = 0,
  PM_E_INVAL = -1,      /* bad argument; nothing was enqueued               */
  PM_E_DEVICE = -2,     /* a HIP runtime call failed                         */
  PM_E_NOMEM = -3,      /* device allocation failed in pm_create             */
  PM_E_BOUNDS = -4,     /* warning: a particle's ball left the physical n^3
                           region; it was computed with indices wrapped
                           modulo n_pad                                      */
  PM_E_NOTCONV = -5,    /* warning: tol > 0 and the residual did not reach it
                           within iters iterations                           */
  PM_E_NONFINITE = -6   /* a residual was NaN or Inf                         */
} pm_status;

/* Flags (pm_params.flags). */
#define PM_F_ANALYTIC_NORM 0x1u /* literal Gaussian prefactor 1/((2pi)^1.5 sigma^3)
                                   of Eq. smooth instead of dividing by the
                                   FP64 sum of the weights over the ball      */
#define PM_F_RESIDUAL      0x2u /* compute r_k every iteration in fixed-K mode
                                   (always on when tol > 0)                   */
#define PM_F_WARM_START    0x4u /* start each solve on the context from the last
                                   F of the previous one (the paper's remark
                                   that the previous step's H is a good start,
                                   Sect. 2.1): F0 = P_L g_N + P_T F_prev, i.e.
                                   H0 = divergence-free part of F_prev - g_N.
                                   The first solve starts from zero; keeps one
                                   more 3-component real field.  Needs
                                   iters >= 2: F is updated only between two
                                   evaluations of nu.                         */

#define PM_F_DFT_BF16X3    0x8u /* the y passes of every 3D transform run their
                                   radix-16 stage as dense 16-point DFT matrix
                                   products on the matrix cores with BF16x3
                                   split operands (about 16 bits kept, FP32
                                   accumulation) instead of FP32 butterflies;
                                   a precision and speed option measured
                                   against the FP32 path.  n_pad 64..512.      */

/* Statement of the problem (Sect. 2, Sect. 3 and the table of symbols). */
typedef struct {
  int32_t  n;        /* physical cells per axis, power of two, 8..512          */
  int32_t  n_pad;    /* FFT box cells per axis, power of two, n..1024;
                        2n leaves the empty margin Sect. 3 asks for           */
  double   box;      /* side of the physical grid; s = box / n               */
  double   G;        /* Newton's constant                                    */
  double   a0;       /* Milgrom's acceleration scale (> 0)                    */
  int32_t  mu;       /* pm_mu                                                */
  double   sigma;    /* Gaussian kernel std in cells (paper: 1), 0.5..2.5    */
  double   cutoff;   /* ball radius in units of sigma, strict |d| < cutoff*sigma
                        (paper: 4, giving 251 cells at sigma = 1)            */
  int32_t  iters;    /* K: evaluations of nu per solve (paper: 4), 1..64     */
  double   tol;      /* 0: exactly K iterations.  > 0: stop at iteration k
                        once r_{k-1} <= tol (K is the maximum); decided on
                        the device: all K iterations are enqueued and those
                        after the stop return at once, so the host never
                        waits and the solve can be captured in a graph   */
  uint32_t flags;    /* PM_F_*                                               */
} pm_params;

/* Residual history of one solve.  r_k = ||H_k - H_{k-1}||_2 / ||g_N||_2 over
 * the whole n_pad^3 box, accumulated in FP64 (the paper estimates the error
 * from the change of H, Sect. 2.1). */
typedef struct {
  int32_t iterations;      /* evaluations of nu performed                     */
  int32_t status;          /* PM_OK, PM_E_NOTCONV or PM_E_NONFINITE           */
  int32_t n_residuals;     /* entries of residual[] that are valid            */
  int32_t bounds_flag;     /* 1 if a deposited ball left the physical region  */
  double  residual[64];    /* r_1 .. r_{n_residuals}                          */
  double  gN_norm;         /* ||g_N||_2 over the box                          */
} pm_solve_info;

typedef struct pm_ctx pm_ctx;

/* Bytes of device memory a context needs for these parameters (the spectra,
 * the Newton potential's spectrum, two real grids, sort buffers for
 * max_particles particles, the tables and, with PM_F_RESIDUAL, tol > 0 or
 * PM_F_WARM_START, the previous iterate of F); 0 for invalid parameters or
 * max_particles outside [0, 2^30]. */
size_t pm_workspace_bytes(const pm_params* p, int64_t max_particles);

/* Validates p (host) and sets up a context on the current HIP device: the
 * workspace is cut into the context's buffers and the tables (twiddles,
 * wavevectors, ball offsets) are written into it.  workspace: device memory
 * of at least pm_workspace_bytes(p, max_particles) bytes, 256-byte aligned,
 * owned by the caller, which keeps it alive and unused by anything else
 * until pm_destroy (the library never frees it); NULL makes the library
 * allocate and own the workspace (PM_E_NOMEM if that fails).  A too small or
 * misaligned workspace is PM_E_INVAL.  stream is a hipStream_t (NULL = the
 * default stream).  Synchronises.  max_particles in [0, 2^30] bounds the N of
 * every later call. */
pm_status pm_create(const pm_params* p, int64_t max_particles, void* workspace, size_t workspace_bytes,
                    void* stream, pm_ctx** out);
pm_status pm_destroy(pm_ctx* ctx);

/* Mass density of Eq. smooth on the FFT box.  rho: device float [n_pad^3],
 * overwritten.  Each particle adds m_i w_id / s^3 to the cells c_i + d of its
 * ball (central pixel c_i = floor(x_i/s + 1/2) per axis), with w the Gaussian
 * weights normalised by their FP64 sum over the ball (or the literal prefactor
 * with PM_F_ANALYTIC_NORM).  For the balls of radius 4 sigma with sigma = 1
 * or 1.5 cells, every cell is an exact fixed-point sum per 8^3 tile of
 * particles, rounded to FP32 once per tile and added in a fixed order, so
 * rho is the same bits for any order of the particles (as long as the tiles'
 * pieces of at most 1024 particles fit the context's 2 GB of staging; pieces
 * beyond it, and other balls, add their cells with FP32 atomics, whose last
 * bits vary from run to run).  N <= max_particles. */
pm_status pm_deposit(pm_ctx* ctx, const float* pos, const float* mass, int64_t N, float* rho);

/* MOND potential phi from rho by the fixed-point iteration of Sect. 2.1:
 * Newton field g_N from rho (-4 pi G A rho_hat, finite-difference gradient),
 * H = the divergence-free part of H0 (or 0), then K times: F = g_N + H, g_M = nu(|F|/a0) F, curl-free
 * projection in Fourier space, and (except after the K-th) F' = mu(|g_M|/a0)
 * g_M, H = divergence-free part of F' - g_N.  phi comes from the last
 * projection.  rho: device float [n_pad^3] (read); H0: device float
 * [3][n_pad^3] or NULL; phi: device float [n_pad^3] (written).  rho and phi
 * may be the same buffer.  info (host) may be NULL; when given, the call
 * synchronises and fills it (iterations done, residuals, status).  With iters = 1, no H0 and no
 * warm start the result is quasi-linear MOND (the equivalent system for
 * QuMOND in Sect. 2): g_M = curl-free part of nu(|g_N|/a0) g_N. */
pm_status aqual_solve(pm_ctx* ctx, const float* rho, const float* H0, float* phi,
                      pm_solve_info* info);

/* pm_deposit for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no context, no workspace, and no allocation of any kind.  The density of
 * pm_deposit on a context with parameters p up to FP32 rounding (its cell
 * sums use atomic adds, whose last bits vary from run to run; rho: device
 * float [n_pad^3], overwritten; pos, mass as there), enqueued on stream (a hipStream_t, NULL
 * = the default stream) without waiting.  Its scratch (the ball table and the
 * sort buffers, about 18 MB) is one fixed array per GPU that the library
 * holds until the process ends; every call on a GPU uses it, so calls that
 * overlap on one GPU (other streams or threads) race and must be serialised
 * by the caller.  Limits: N <= 2^20 and n_pad <= 512, otherwise PM_E_INVAL
 * with nothing enqueued. */
pm_status pm_deposit_noalloc(const pm_params* p, const float* pos, const float* mass, int64_t N, float* rho,
                             void* stream);

/* Kernel-smoothed acceleration of Eq. gi: g_i = -sum_d w_id (D phi)(c_i + d)
 * with D the central-difference gradient and the same weights as pm_deposit.
 * phi: device float [n_pad^3]; acc: device float [N][3] (written). */
pm_status smooth_accel(pm_ctx* ctx, const float* phi, const float* pos, int64_t N, float* acc);

/* Gather plus leapfrog (Eq. motion): v <- v + g_i dt_kick, then
 * r <- r + v dt_drift, in place.  With v half a step behind r, the initial
 * half step is interp_push(dt_kick = -dt/2, dt_drift = 0). */
pm_status interp_push(pm_ctx* ctx, const float* phi, float* pos, float* vel, int64_t N,
                      double dt_kick, double dt_drift);

/* One PM step: deposit at r, solve, kick by dt, drift by dt (pos, vel in
 * place; the flow scheme's alternation with one fixed phase).  info may be
 * NULL (then nothing synchronises, in either mode). */
pm_status pm_step(pm_ctx* ctx, float* pos, float* vel, const float* mass, int64_t N,
                  double dt, pm_solve_info* info);

/* One pm_step (info = NULL) recorded as a HIP graph and replayed: the whole
 * step of the flow scheme's main loop, every kernel of deposit, solve and
 * push, with one launch call per step.  pm_step_capture records the step on
 * the context's stream with these buffers and this dt, without running it,
 * and keeps the graph in the context (replacing an earlier one; pm_destroy
 * frees it).  pm_step_replay launches it count times on the stream; each
 * replay is one pm_step on the captured buffers, which the caller keeps alive
 * and in place; with tol > 0 each replay stops its solve where the residual
 * test does, on the device.  PM_E_INVAL if the context was created on the
 * null stream, has event timing on, or has
 * PM_F_WARM_START before its first solve (capture after one pm_step so the
 * recorded solve starts warm); on a capture error no graph is kept. */
pm_status pm_step_capture(pm_ctx* ctx, float* pos, float* vel, const float* mass, int64_t N,
                          double dt);
pm_status pm_step_replay(pm_ctx* ctx, int32_t count);

/* FP64 diagnostics (constants of motion of Sect. 4.1): out (host) receives
 * 10 doubles: P (3), L (3), E_kin, total mass, and, if phi is not NULL,
 * sum_i m_i phi_i with phi smoothed by the particle kernel (else 0), and the
 * number of particles whose ball leaves the physical region.  Synchronises. */
pm_status pm_diagnostics(pm_ctx* ctx, const float* pos, const float* vel, const float* mass,
                         int64_t N, const float* phi, double* out);

/* 3D real transforms of the FFT box used inside aqual_solve, exposed for
 * testing.  Spectrum layout: kx = 0..n_pad/2 valid, in groups of 16:
 * complex (float2) [pitch / 16][n_pad][n_pad][16] indexed
 * [kx / 16][kz][ky][kx % 16], pitch = pm_spectrum_pitch(n_pad) =
 * 16 * ceil((n_pad/2 + 1) / 16) kx slots (n_pad^2 * pitch complex values).
 * Unnormalised in both directions: c2r(r2c(f)) = n_pad^3 f.  in and out
 * must not overlap. */
int32_t   pm_spectrum_pitch(int32_t n_pad);
pm_status pm_fft_r2c(pm_ctx* ctx, const float* in, void* spectrum_out);
pm_status pm_fft_c2r(pm_ctx* ctx, const void* spectrum_in, float* out);

/* Per-kernel timing with HIP events on the context's stream.  Timer ids:
 * one per pass kind of the 3D transforms and per particle kernel. */
enum {
  PM_T_X_FWD_REAL = 0, PM_T_X_FWD_REAL3, PM_T_X_INV_REAL, PM_T_X_NU, PM_T_X_MU,
  PM_T_Y_FWD, PM_T_Y_INV, PM_T_Z_FWD, PM_T_Z_INV, PM_T_Z_NEWTON, PM_T_Z_CURL,
  PM_T_Z_CURL_FINAL, PM_T_Z_DIV, PM_T_SORT, PM_T_DEPOSIT, PM_T_GATHER, PM_T_FILL,
  PM_T_REDUCE, PM_NUM_TIMERS
};
/* enable != 0 records an event pair around every launch from now on (host). */
pm_status pm_set_timing(pm_ctx* ctx, int enable);
/* Synchronises; adds the elapsed milliseconds and launch counts recorded since
 * the last read into total_ms[PM_NUM_TIMERS] and launches[PM_NUM_TIMERS]
 * (host arrays the caller zeroes), then forgets them. */
pm_status pm_read_timing(pm_ctx* ctx, double* total_ms, int64_t* launches);

/* Newton potential alone (the flow scheme's Newton step): phi_N = inverse FFT
 * of -4 pi G A rho_hat on the n_pad^3 box.  rho, phiN: device float
 * [n_pad^3]; they may not overlap.  Used to form the learned start's input. */
pm_status pm_newton_potential(pm_ctx* ctx, const float* rho, float* phiN);

/* External field (Sect. 5): a uniform Newtonian field (gx, gy, gz) added
 * to every later Newton solve on the context (aqual_solve, pm_step,
 * pm_newton_potential and the learned start's input), made as the paper
 * suggests by a permanent dipole sheet on the planes farthest from the
 * matter.  For each axis, the cell plane n_pad - 1 gets +rho_c and the cell
 * plane 0 gets -rho_c in every cell, with rho_c = g L / (4 pi G s^2),
 * L = n_pad s.  On the periodic box this gives the bulk the Newtonian field
 * g along that axis, up to a lattice ripple from the sharp sheets that decays
 * with the distance from them (below 1e-4 of g at 16 cells, less further in).
 * The MOND solve then acts on g_N including this field, which gives the
 * external-field effect.  The sheets' own cells carry large fields; matter
 * must stay away from them (the physical region already does).  (0, 0, 0)
 * removes the field.  PM_E_INVAL for non-finite values.  Host only, no
 * synchronisation; a captured pm_step graph keeps the value at capture. */
pm_status pm_set_external_field(pm_ctx* ctx, double gx, double gy, double gz);

/* Apparent density of Eq. apparentdensity, rho_A = -div(g)/(4 pi G) with
 * g = -grad phi, in the discretisation of the solve's projections
 * (g_M_hat = -i kt phi_hat): rho_A_hat = -|kt|^2 phi_hat / (4 pi G).  From the
 * MOND potential it gives baryonic plus phantom density, from the Newton
 * potential the baryonic density; both without their mean (a periodic
 * potential does not carry it).  phi, rho_a: device float [n_pad^3], may be
 * the same buffer. */
pm_status pm_apparent_density(pm_ctx* ctx, const float* phi, float* rho_a);

/* aqual_solve that also returns F = g_N + H of its last iteration (the field
 * whose nu gave phi) in F: device float [3][n_pad^3].  Requires a context
 * created with PM_F_RESIDUAL or tol > 0 (it keeps F); otherwise PM_E_INVAL.
 * The fixed point's H is F - g_N. */
pm_status aqual_solve_field(pm_ctx* ctx, const float* rho, const float* H0, float* phi, float* F,
                            pm_solve_info* info);

/* ---- Linearised increments (Sect. 5, items (iv) and (v)) ---------------
 * Between two steps the fields change little; the paper proposes to solve
 * for the increments with Eqs. inverse and interpolation linearised about
 * the previous fields,
 *     dg_M = nu dF + nu'(F/a0) (F . dF) / (a0 |F|) F        (about F),
 *     dF'  = mu dg_M + mu'(g_M/a0) (g_M . dg_M) / (a0 |g_M|) g_M   (about g_M),
 * the linear steps (Newton field, curl-free and divergence-free
 * projections) unchanged, and the increments stored in few digits.
 *
 * aqual_solve_increment runs the iteration of aqual_solve on increments:
 * dg_N from d_rho, dH = 0, then iters times dF = dg_N + dH, dg_M from the
 * first linearisation, its curl-free part (giving d_phi), and (except after
 * the last) dF' from the second linearisation and dH = the divergence-free
 * part of dF' - dg_N.  Both maps are zero where the field they are
 * linearised about is zero.  d_rho: device float [n_pad^3]; F, gM: device
 * float [3][n_pad^3], the previous solve's F (aqual_solve_field) and g_M
 * (pm_potential_field of its phi); d_phi: device float [n_pad^3], written;
 * d_F: device float [3][n_pad^3] or NULL, receives dF of the last
 * iteration (F + d_F and the field of phi + d_phi are the next step's F and
 * g_M).  storage: PM_STORE_FP32, or PM_STORE_FP16, which keeps every
 * intermediate spectrum of the increments in FP16, each component of each
 * pass's tile scaled by its own power of two (the Newton spectrum of d_rho
 * and the last, one-component spectrum of d_phi stay FP32).  The residual
 * r_k (PM_F_RESIDUAL or tol > 0) is ||dH_k - dH_{k-1}|| / ||dg_N||; info
 * and tol behave as in aqual_solve.  The context's kept F (warm start) is
 * overwritten when it computes residuals, so the next warm start on it
 * starts from zero. */
#define PM_STORE_FP32 0
#define PM_STORE_FP16 1
pm_status aqual_solve_increment(pm_ctx* ctx, const float* d_rho, const float* F, const float* gM,
                                int32_t storage, float* d_phi, float* d_F, pm_solve_info* info);

/* g = -i kt phi_hat on the FFT box: the field of a potential as the solve's
 * curl-free projection forms it (kt the wavevector with the Nyquist entry
 * zeroed, Sect. 2.1).  For the phi of aqual_solve it is that solve's g_M,
 * the base of the second linearisation.  phi: device float [n_pad^3];
 * g: device float [3][n_pad^3], written. */
pm_status pm_potential_field(pm_ctx* ctx, const float* phi, float* g);

/* ---- Learned starting guess --------------------------------------------
 * Sect. 2.1 lets the iteration start from any divergence-free H; the paper
 * starts from zero and notes that a good start saves iterations.  A 3-level
 * encoder-decoder of 3x3x3 convolutions (16 / 32 / 64 channels, ReLU, 2x
 * average pooling, nearest 2x upsampling with skip concatenation, a 1x1x1
 * head to 3 channels) predicts H from the Newton field.  H fills the whole
 * periodic box (about half of it lies outside the physical region), so the
 * network sees the whole box at half (or quarter) resolution, n = n_pad / f
 * voxels per axis with f = 2 (or 4), each the mean of an f^3 block of cells,
 * with periodic convolutions:
 *         g_c = block mean of g_N,  rms = sqrt(mean |g_c|^2),
 *         x = [g_c / rms, log10(|g_c| / a0 + 1e-30)],
 *         H0 = rms * net(x), each value repeated over its f^3 block;
 * aqual_solve then starts from the divergence-free part of H0.  Operands are
 * BF16 on the matrix cores with FP32 accumulation; parameters are FP32.
 * Parameter vector (pm_net_param_count floats): for each layer in the order
 * e1a (4->16), e1b (16->16), e2a (16->32), e2b (32->32), b3a (32->64),
 * b3b (64->64), d2a (96->32), d2b (32->32), d1a (48->16), d1b (16->16),
 * out (16->3, 1x1x1): weights [taps][cin][cout] (tap = (dz+1) 9 + (dy+1) 3 +
 * (dx+1)) then bias [cout].  A net's buffers belong to one stream at a time:
 * calls taking a context run on the context's stream, the others on the
 * stream given to pm_net_create. */
typedef struct pm_net pm_net;
int64_t   pm_net_param_count(void);
/* n: voxels per axis (power of two, 8..512; n_pad / 2 or n_pad / 4 of the
 * contexts it is used with); max_batch: slots for training pairs (1..64).  Parameters start
 * at zero; set them with pm_net_set_params.  Synchronises. */
pm_status pm_net_create(int32_t n, int32_t max_batch, void* stream, pm_net** out);
pm_status pm_net_destroy(pm_net* net);
/* params (host float [P]) in; also clears the optimiser state.  Synchronises. */
pm_status pm_net_set_params(pm_net* net, const float* params);
/* host float [P] out.  Synchronises. */
pm_status pm_net_get_params(pm_net* net, float* params);
/* gradients of the last pm_net_backward, host float [P].  Synchronises. */
pm_status pm_net_get_grads(pm_net* net, float* grads);
/* input channels of slot from phiN (device float [n_pad^3], the Newton
 * potential of the context's box; g_N = -D phi_N by central differences). */
pm_status pm_net_input(pm_ctx* ctx, pm_net* net, const float* phiN, int32_t slot);
/* training target of slot: block mean of (F - g_N) / rms, F as returned by
 * aqual_solve_field for the same rho, rms that of pm_net_input for the slot. */
pm_status pm_net_target(pm_ctx* ctx, pm_net* net, const float* phiN, const float* F, int32_t slot);
/* direct input / target of a slot: x device float [4][n^3], y device float
 * [3][n^3] (x fastest). */
pm_status pm_net_set_input(pm_net* net, int32_t slot, const float* x);
pm_status pm_net_set_target(pm_net* net, int32_t slot, const float* y);
/* the input channels of a slot as stored (BF16 values), device float [4][n^3]. */
pm_status pm_net_get_input(pm_net* net, int32_t slot, float* x);
/* the target of a slot, device float [3][n^3]. */
pm_status pm_net_get_target(pm_net* net, int32_t slot, float* y);
/* forward pass over slots [0, batch); outputs kept in the net. */
pm_status pm_net_run(pm_net* net, int32_t batch);
/* output of slot after pm_net_run / pm_net_backward: device float [3][n^3]. */
pm_status pm_net_output(pm_net* net, int32_t slot, float* y);
/* A tensor the last pm_net_run or pm_net_backward stored for slot, as FP32
 * channels first: out device float [C][(n >> level)^3].  which = 0..12: the
 * BF16 activations x (4 channels, level 0), a1, s1 (16, 0), p1 (16, 1),
 * a2, s2 (32, 1), p2 (32, 2), a3, b3 (64, 2), a4, d2 (32, 1), a5, d1 (16, 0),
 * in forward order (a = first convolution of a level, s = skip tensor,
 * p = pooled, b3 = bottleneck, d = decoder output); which = 13..22: the BF16
 * gradient buffers of the backward pass with their last contents: g16a,
 * g16b (16, 0), gc1 (48, 0), g32a, g32b (32, 1), gc2 (96, 1), g64a, g64b
 * (64, 2), gp1 (16, 1), gp2 (32, 2).  For per-layer checks of the kernels. */
pm_status pm_net_get_tensor(pm_net* net, int32_t which, int32_t slot, float* out);
/* rms of slot (host double out).  Synchronises. */
pm_status pm_net_get_rms(pm_net* net, int32_t slot, double* rms);
/* forward and backward over slots [0, batch) with the loss
 * mean((net(x) - y)^2) over all slots, channels and voxels; loss (host,
 * nullable) synchronises. */
pm_status pm_net_backward(pm_net* net, int32_t batch, double* loss);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the last gradients. */
pm_status pm_net_adam(pm_net* net, float lr);
pm_status pm_net_train_step(pm_net* net, int32_t batch, float lr, double* loss);
/* the learned start for the context's box: input from phiN, forward, H0
 * (device float [3][n_pad^3], overwritten).  Uses slot 0. */
pm_status pm_net_forward(pm_ctx* ctx, pm_net* net, const float* phiN, float* H0);

/* aqual_solve from the learned start in one call: the solve's own Newton
 * spectrum gives the network's features (no second Newton solve), the
 * network runs on slot 0, and its coarse output enters the Newton pass.
 * For networks of 16 to 256 voxels per axis in boxes up to 512^3 both stay
 * in Fourier space: the features' block means are the Newton spectrum's
 * aliases onto the network's grid, and the start's spectrum is the coarse
 * output's DFT times the DFT of one block (no real phi_N, no
 * full-resolution H0).  Other sizes form the features from the real
 * potential and expand the output in the forward x transform.  The result
 * of pm_newton_potential, pm_net_forward and aqual_solve with that H0: bit
 * for bit on the real-space route; on the spectral one the network's input
 * to one BF16 step where the FP32 rounding of the block means crosses a
 * BF16 boundary.  rho,
 * phi: device float [n_pad^3] (phi is written and may not be the context's
 * internal grid); info and tol as in aqual_solve.  The network's slot 0 and
 * the context's internal potential grid are overwritten. */
pm_status aqual_solve_learned(pm_ctx* ctx, pm_net* net, const float* rho, float* phi, pm_solve_info* info);

/* Last HIP error string seen by the library (host, static storage). */
const char* pm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MONDPM_H */
