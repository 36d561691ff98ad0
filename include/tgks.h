/* tgks.h -- C ABI of the MI355X (gfx950) TENO-D gas-kinetic scheme library.
 *
 * The library advances the compressible Euler or Navier-Stokes equations
 *     W_t = -div F(W),  W(0, x) = W0(x)
 * (Sec. 2.2 of Mu et al., "High-order gas-kinetic scheme with TENO class
 * reconstruction for the Euler and Navier-Stokes equations",
 * arXiv:2309.10534) on a uniform 1-D, 2-D or 3-D grid with the fifth-order
 * TENO-D reconstruction (Sec. 4.2), the gas-kinetic interface flux with the
 * kinetic-weighted equilibrium state (Sec. 2.1, Sec. 3.2) and the two-stage
 * fourth-order (S2O4) time stepping (Sec. 2.2).  Every step runs in HIP
 * kernels on the device; this header uses no torch or HIP types.
 *
 * Data layout.  A state W is FP64, structure of arrays, [nc][nz][ny][nx] with
 * x fastest, contiguous, interior cells only; nc = ndim + 2 and the
 * components are (rho, rho U, rho V, rho W, rho E) truncated to nc.
 *
 * Pointers.  Every array argument is a DEVICE pointer owned by the caller
 * unless stated otherwise; the library never frees it.  Work is enqueued on
 * the HIP stream given at creation (tgks_set_stream changes it) and the
 * calls return before it completes; a context must not be used from two
 * host threads at once.
 *
 * Errors.  A negative return value means a caller error (invalid parameter,
 * null pointer, size mismatch) or a HIP error; in the first case nothing was
 * enqueued.  Numerical failure (rho <= 0, p <= 0 or a non-finite value in a
 * reconstructed or equilibrium state at a Gauss point) is not reported
 * synchronously: it increments a device counter read by tgks_status.
 */
#ifndef TGKS_H
#define TGKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TGKS_OK 0
#define TGKS_EINVAL (-1) /* invalid argument: nothing enqueued */
#define TGKS_EHIP (-2)   /* a HIP runtime call failed */

/* boundary kinds (Sec. 5): periodic; transmissive = the non-reflecting
 * zero-gradient condition (ghost cells copy the nearest interior cell);
 * reflective = mirror image with the wall-normal momentum negated (also the
 * symmetry condition of Sec. 5.8); no-slip = the adiabatic no-slip wall of
 * Sec. 5.8, mirror image with every momentum component negated, and no mass
 * or energy flux through the wall faces; prescribed = given states (the
 * inflow, post-shock bottom and moving-shock top of the double Mach
 * reflection, Sec. 5.7; 1-D and 2-D contexts only): a ghost cell of such a
 * side, centred at coordinate s along the other axis of a 2-D grid (s = 0
 * on a 1-D grid) and r along the side's own axis (both measured from the
 * domain origin, r < 0 beyond a low side), holds at time t the state
 * bc_state[0] where s < (s0 + s_n r) + s_t t, (s0, s_n, s_t) =
 * bc_line[axis][end], and beyond that line what bc_far[axis][end] gives:
 * TGKS_BC_TRANSMISSIVE or TGKS_BC_REFLECTIVE images, or TGKS_BC_PRESCRIBED
 * for the state bc_state[1].  Stage 1 of a step from t uses time t, stage 2
 * time t + dt/2.  A ghost cell outside both axes is decided by the x side
 * first when that side is prescribed and gives a state. */
#define TGKS_SCHEME_TENO_D 0
#define TGKS_SCHEME_WENO_AO 1
#define TGKS_SCHEME_TENO5 2
#define TGKS_SCHEME_WENO_Z 3

#define TGKS_BC_PERIODIC 0
#define TGKS_BC_TRANSMISSIVE 1
#define TGKS_BC_REFLECTIVE 2
#define TGKS_BC_NOSLIP 3
#define TGKS_BC_PRESCRIBED 4

/* collision time (Sec. 5 preamble):
 * INVISCID: tau = c1 dt + c2 |p_l - p_r| / (p_l + p_r) dt
 * VISCOUS:  tau = mu / p0 + c2 |p_l - p_r| / (p_l + p_r) dt
 * ZERO:     tau = 0 (smooth inviscid accuracy tests, Sec. 5.1)
 * p_l, p_r: reconstructed pressures at the Gauss point; p0: pressure of the
 * kinetic-weighted equilibrium state; dt is the full step in both stages. */
#define TGKS_TAU_INVISCID 0
#define TGKS_TAU_VISCOUS 1
#define TGKS_TAU_ZERO 2

/* Reconstruction variables: the conservative variables component by
 * component (the paper's scheme), or the characteristic fields of the
 * Euler flux Jacobian at the mean of the two cells beside each face
 * (normal and tangential reconstruction; 1-D and 2-D grids and batches). */
#define TGKS_RECON_CONSERVATIVE 0
#define TGKS_RECON_CHARACTERISTIC 1

typedef struct tgks_params {
  int32_t ndim;      /* 1, 2 or 3 */
  int32_t n[3];      /* cells per axis, >= 3 on every used axis (1 on unused ones) */
  double dx[3];      /* cell widths, > 0 */
  int32_t bc_lo[3];  /* TGKS_BC_* at the low and high end of each axis; */
  int32_t bc_hi[3];  /* periodic must be set on both ends of an axis     */
  double gamma;      /* ratio of specific heats, > 1 (1.4 in Sec. 5) */
  double mu;         /* constant dynamic viscosity, >= 0 (0: Euler) */
  double prandtl;    /* Prandtl number, > 0; the energy flux is corrected by (1/Pr - 1) q when mu > 0 */
  int32_t tau_mode;  /* TGKS_TAU_* */
  double c1, c2;     /* collision-time constants, 0.01 and 1 in Sec. 5 */
  double ct1, ct2;   /* TENO-D cut-offs C_T1, C_T2 (1e-7, 1e-5: Eqs. 4.7, 4.12), normal direction */
  double ct1_tan, ct2_tan; /* cut-offs of the tangential reconstruction */
  double eps;        /* epsilon of Eq. 4.5 (1e-40) */
  int32_t q;         /* power of Eq. 4.5 (7) */
  int32_t recon;     /* TGKS_RECON_*; characteristic only with ndim 1 or 2 (default conservative) */
  /* prescribed sides (TGKS_BC_PRESCRIBED), ignored otherwise: */
  double bc_state[2][5];   /* states A and B, conservative, (rho, m_0 .. m_{ndim-1}, E) */
  double bc_line[3][2][3]; /* per axis and end (0 low, 1 high): (s0, s_n, s_t) */
  int32_t bc_far[3][2];    /* per axis and end: kind beyond the line */
  /* first-order fallback (not in the paper; default 0; the reverse mode
   * rejects it): 1 replaces a reconstructed Gauss-point state of one side whose
   * density or pressure, (gamma-1) (E - (0.5 sum_a m_a^2) / rho) evaluated in
   * that order, is not positive or not finite by the average of that side's
   * cell at the face, with zero slopes, before the flux is evaluated.  It is
   * not a positivity-preserving limiter: cell averages can still become
   * non-physical. */
  int32_t fallback;
  /* reconstruction scheme (default TGKS_SCHEME_TENO_D, the paper's): one of
   * the paper's comparison schemes on 1-D and 2-D grids with conservative
   * variables (no prescribed sides, no fallback; batches and the reverse mode
   * reject them):
   *   TGKS_SCHEME_WENO_AO (Sec. 3.2): linear weights d_hi, d_lo (0.85, 0.85),
   *     weights d_k (1 + (tau / (beta_k + eps_w))^2), eps_w 1e-8;
   *   TGKS_SCHEME_TENO5 (Sec. 4.1): gamma_k = (1 + tau / (beta_k + eps))^q
   *     with cut-off ct1 (set q = 6, the paper's, eps 1e-40, ct1 1e-7);
   *   TGKS_SCHEME_WENO_Z (Sec. 3.1): weights d_k (1 + tau / (beta_k + eps_w)).
   * TENO5 and WENO-Z reconstruct only the non-equilibrium interface values
   * nonlinearly; slopes follow Eq. 3.11 and the equilibrium state is
   * reconstructed separately (Eq. 3.12; in 2-D the linear quartic along the
   * face).  Stencil flags: TENO5 records its cut-offs (bit k = delta_k),
   * WENO-AO and WENO-Z record 0. */
  int32_t scheme;
  double d_hi, d_lo;
  double eps_w;
} tgks_params;

typedef struct tgks_ctx tgks_ctx;

/* Fill p with the paper's constants for an ndim-dimensional Euler problem
 * (gamma 1.4, tau inviscid, c1 0.01, c2 1, C_T 1e-7 / 1e-5, eps 1e-40, q 7,
 * transmissive boundaries); the caller sets n and dx. */
int tgks_params_default(tgks_params* p, int32_t ndim);

/* Create a context for one grid.  Allocates the device work buffers of one
 * step (about 3 states plus face fluxes); hip_stream may be NULL for the
 * default stream.  Returns TGKS_EINVAL for invalid parameters. */
int tgks_create(const tgks_params* p, void* hip_stream, tgks_ctx** out);
int tgks_destroy(tgks_ctx* ctx);
int tgks_set_stream(tgks_ctx* ctx, void* hip_stream);

/* Number of doubles of one state (nc * cells) and bytes of the flag buffer
 * of tgks_step. */
int64_t tgks_state_size(const tgks_ctx* ctx);
int64_t tgks_flag_bytes(const tgks_ctx* ctx);

/* CFL time step (Sec. 5 preamble): dt = cfl * min over cells of
 * min(dx_min / (|U| + a), dx_min^2 rho / (4 mu)), a = sqrt(gamma p / rho);
 * if t_end > 0 it is clipped to t_end - t.  Writes one double to dt_dev. */
int tgks_cfl_dt(tgks_ctx* ctx, const double* W, double cfl, double t, double t_end, double* dt_dev);

/* One S2O4 step W_out = S(W_in, dt) with dt read from the device scalar
 * dt_dev (dt <= 0 or NaN: W_out = W_in).  W_in and W_out must not overlap.
 * flags (device, tgks_flag_bytes bytes, or NULL): stage-1 stencil
 * selections, one byte per decision: bit0 = delta_{3,1} (Eq. 4.7); when it
 * is 0, bits 1..3 = delta_{0,2}, delta_{1,2}, delta_{2,2} (Eq. 4.12).
 * Layout: normal reconstruction [ndim][nc][cells], then for ndim >= 2 the
 * tangential reconstructions of each direction d in turn (Sec. 3.2 Steps
 * 1-3), faces_d indexed like a state whose axis d has n[d] + 1 entries:
 *   ndim == 2: [quantity (W, dW/dn)][side (left, right)][nc][faces_d];
 *   ndim == 3: the first sweep (along t1 = (d+1) mod 3) of the face's own
 *     line as [quantity (W, dW/dn)][side][nc][faces_d], then the second
 *     sweep (along t2 = (d+2) mod 3) as [t1 Gauss point (-, +)][quantity
 *     (W, dW/dt1, dW/dn)][side][nc][faces_d]: 16 nc planes per direction.
 * nc components in global order (rho, rho U, rho V, rho W, rho E).
 * W_star (device, one state, or NULL) receives the intermediate state W*
 * of Sec. 2.2. */
int tgks_step(tgks_ctx* ctx, const double* W_in, double* W_out, const double* dt_dev, uint8_t* flags,
              double* W_star);

/* tgks_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): one
 * S2O4 step of the grid described by p, without a context.  The step's work
 * buffers (W*, P, face fluxes, counters) are a fixed device array of
 * tgks_noalloc_capacity() doubles (64 MiB) that each GPU the library runs
 * on holds until the process ends; the call allocates nothing and calls no
 * allocating routine.  Grids needing more scratch than that
 * (tgks_noalloc_need(p) > tgks_noalloc_capacity(): 1-D beyond 698,815
 * cells, 2-D beyond 590 x 590, 3-D beyond 51^3) return TGKS_EINVAL with
 * nothing enqueued.  Work goes
 * to hip_stream (NULL: the default stream); W_in, W_out, dt_dev, flags and
 * W_star as in tgks_step (the caller's device buffers).  failures (host, or
 * NULL): if given, the call synchronises the stream and stores the number
 * of non-physical Gauss-point evaluations of the step.  Every call on one
 * GPU uses that GPU's array, which keeps the last call's contents (the
 * counters are cleared by each call): calls that overlap on one GPU, from
 * two streams or two host threads, race. */
int64_t tgks_noalloc_capacity(void);
int64_t tgks_noalloc_need(const tgks_params* p);
int tgks_step_noalloc(const tgks_params* p, void* hip_stream, const double* W_in, double* W_out,
                      const double* dt_dev, uint8_t* flags, double* W_star, int64_t* failures);

/* Advance W in place by n_steps S2O4 steps with the CFL step computed on the
 * device before every step (cfl > 0), the last step clipped so that the
 * time does not pass t_end when t_end > 0 (further steps are no-ops), or
 * with the constant step fixed_dt when cfl <= 0.  time_dev (device, 2
 * doubles, or NULL) receives (t, dt of the next step).  use_graph != 0
 * captures the n_steps loop into a HIP graph on first use and replays it. */
int tgks_run(tgks_ctx* ctx, double* W, int32_t n_steps, double cfl, double t_end, double fixed_dt,
             double* time_dev, int32_t use_graph);

/* Time of the prescribed boundary states (TGKS_BC_PRESCRIBED): tgks_step
 * advances a state of time t0, tgks_run a state of time t0 + its clock (the
 * clock starts at 0 in every call).  Default 0; does not touch the device
 * and affects later calls only. */
int tgks_set_time(tgks_ctx* ctx, double t0);

/* Tile shape of the 2-D face kernel (faces along the normal x along the
 * face, two lanes per face): 0 = 16 x 8, 1 = 16 x 16, 2 = 8 x 16; -1 selects
 * the default (0).  Other dimensions ignore it; with characteristic
 * variables, prescribed sides or the first-order fallback the 2-D shape is
 * always 2. */
int tgks_set_tile(tgks_ctx* ctx, int32_t tile);

/* Autotuner: time every tile shape over `steps` S2O4 steps of the state W
 * (device; not modified) with HIP events, select the fastest and return its
 * index in *chosen (host, may be NULL); ms_per_variant (host, 3 floats, or
 * NULL) receives the milliseconds per step of each shape (0 for shapes not
 * timed: with characteristic variables, prescribed sides or the fallback
 * only shape 2 exists).  Synchronises
 * the stream. */
int tgks_tune(tgks_ctx* ctx, const double* W, int32_t steps, int32_t* chosen, float* ms_per_variant);

/* Failure count since creation or the last tgks_reset_status (synchronises
 * the stream).  tgks_reset_status enqueues a small kernel (no memset), so
 * it may be captured into a graph. */
int tgks_status(tgks_ctx* ctx, int64_t* failures);
int tgks_reset_status(tgks_ctx* ctx);

/* Number of Gauss-point side states the first-order fallback replaced
 * (fallback = 1; both stages of every step) since the context was created
 * or tgks_reset_status last ran; synchronises the stream. */
int tgks_fallback_count(tgks_ctx* ctx, int64_t* count);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * every launch while enabled.  kind: 0 face fluxes along x, 1 along y, 2
 * along z, 3 normal reconstruction (3-D), 4 stage-1 update, 5 stage-2
 * update, 6 CFL reduction.  tgks_kernel_time synchronises and returns the
 * summed milliseconds and launch count of one kind since it was enabled. */
int tgks_timing(tgks_ctx* ctx, int32_t enable);
int tgks_kernel_time(tgks_ctx* ctx, int32_t kind, double* ms, int64_t* launches);

/* Algorithmic operation counts of the kernels for parameters p (host only,
 * no device work), from the kernels' own device math evaluated on the host
 * with a counting scalar type on smooth data: +, -, *, / and each sqrt, exp,
 * expm1, erfc count one.  out[0]: normal TENO-D reconstruction per cell,
 * direction and component; out[1], out[2]: stage-1 / stage-2 face work per
 * face beyond the normal reconstruction (tangential reconstruction, the
 * Gauss-point fluxes, the S2O4 combination); out[3], out[4]: stage-1 /
 * stage-2 update per cell; out[5]: transcendentals and out[6]: divisions per
 * stage-1 face; out[7]: CFL limit per cell.  With characteristic variables
 * the normal reconstruction is per face: out[0] is 0 and out[1], out[2]
 * include it.  nout >= 8. */
int tgks_flop_counts(const tgks_params* p, double* out, int32_t nout);

/* The roofline's two ceilings measured on the current device: FP64 FMA
 * throughput in TFLOP/s (eight independent FMA chains per thread) and
 * device-to-device copy bandwidth in GB/s (bytes read + written, 1 GiB
 * each).  Allocates and frees 2 GiB of device memory; synchronises the
 * stream (hip_stream may be NULL). */
int tgks_measure_peaks(void* hip_stream, double* fp64_tflops, double* copy_gbps);

/* Host evaluation of the device Gauss-point flux (Sec. 2.1, Eqs. 2.5-2.9,
 * kinetic weighting Eq. 2.6) for verification without a device: the same
 * code the kernels run, in double on the host.  Face frame (axis 0 normal);
 * HOST pointers: Wl, Wr [nc], dWl, dWr [ndim][nc] (derivatives along the
 * frame axes), F [2][nc] receives F(dt) and F(dt/2).  Returns 0, 1 when a
 * state is non-physical, or TGKS_EINVAL. */
int tgks_gp_flux_host(const tgks_params* p, const double* Wl, const double* Wr, const double* dWl,
                      const double* dWr, double dt, double* F);

/* The kernels' stencil selection of five values Q (host arrays), evaluated
 * on the host: the TENO-D flag (bit0 = delta_{3,1}, bits 1..3 = the small
 * stencils' cut-offs; Sec. 4.2) with the normal cut-offs and eps of p.
 * fast selects the evaluation: 0 from the weights of Eqs. 4.5-4.12 alone
 * (correctly rounded divisions); 2 as the 1-D and 2-D kernels do, from
 * approximate reciprocals where a margin makes the decision certain (on
 * the host the reciprocal is 1/x cut to 24 significant bits); 1 as the 3-D
 * kernels do, from fixed ratios of the smoothness indicators where they
 * decide, else from the weights.  The shortcuts are on only for q = 7,
 * eps >= 1e-40 and cut-offs in the ranges where they are exact; elsewhere
 * every mode evaluates the weights.
 * For verification: all three must agree for every input.  Returns the
 * flag, or TGKS_EINVAL (also for fast outside 0..2). */
int tgks_teno_flag_host(const tgks_params* p, const double* Q, int32_t fast);

/* The kernels' complementary error function, evaluated on the host: the
 * half-space moments of a Maxwellian in the flux (Sec. 2.1, the left and
 * right half-space integrals that the Heaviside split of the initial
 * distribution produces) hold erfc of the normal velocity times
 * sqrt(lambda).  A polynomial (a cut Chebyshev series) for (1 + 2|x|)
 * exp(x^2) erfc(|x|), multiplied by exp(-x^2), which the moments need
 * anyway.  For
 * verification.  Returns erfc(x) (0 or 2 at x = +-inf, NaN for NaN). */
double tgks_erfc_host(double x);

/* ------------------------------------------------------------------------
 * Reverse mode.  The derivative of one S2O4 step W_out = S(W_in) with the
 * time step dt held constant and every TENO-D stencil selection (Sec. 4.2)
 * held at the one the forward step takes on W_in; the reconstruction is then
 * linear and S is smooth.  The collision time is differentiated through the
 * pressures it depends on.  1-D and 2-D grids.
 * ------------------------------------------------------------------------ */

/* gW_in = (dW_out/dW_in)^T gW_out for the step from W_n with the step read
 * from dt_dev (device).  W_n, gW_out, gW_in: device states; gW_in must not
 * overlap gW_out.  W_star: the step's intermediate state W* as tgks_step
 * returned it for the same W_n and dt (device), or NULL to recompute it with
 * the forward kernels.  The first call allocates the context's reverse-mode
 * buffers.  TGKS_EINVAL for 3-D contexts, characteristic variables,
 * prescribed sides, the first-order fallback or invalid pointers. */
int tgks_step_adjoint(tgks_ctx* ctx, const double* W_n, const double* W_star, const double* dt_dev,
                      const double* gW_out, double* gW_in);

/* Host evaluation of the reverse of the Gauss-point flux (the same code the
 * reverse kernels run), for verification.  Face frame, HOST pointers as in
 * tgks_gp_flux_host; Fb [2][nc]: cotangents of F(dt) and F(dt/2); G receives
 * the cotangents of Wl [nc], Wr [nc], dWl [ndim][nc], dWr [ndim][nc] in this
 * order.  dt is a constant. */
int tgks_gp_flux_vjp_host(const tgks_params* p, const double* Wl, const double* Wr, const double* dWl,
                          const double* dWr, double dt, const double* Fb, double* G);

/* ------------------------------------------------------------------------
 * Batched runs: many independent 1-D or 2-D grids (uneven sizes, each with
 * its own parameters, boundary kinds, CFL time step, clock and failure
 * counter) advanced together, one launch per kernel kind and stage for the
 * whole batch.  A batched step of an instance is bit-identical to the same
 * step of that instance in its own context.
 *
 * Packed layout: the instances' states one after another, instance i at
 * doubles [offsets[i], offsets[i+1]) of W_packed, each with the layout of a
 * single state ([nc][ny][nx]).
 * ------------------------------------------------------------------------ */
typedef struct tgks_batch tgks_batch;

/* per_instance: host array of n_inst parameter sets, all with the same ndim
 * (1 or 2), the same reconstruction variables, and all Euler or all
 * Navier-Stokes with a Prandtl correction (characteristic variables or the
 * first-order fallback: one 2-D tile shape, 2).  Allocates the batch's work buffers (about three packed states plus face
 * fluxes).  TGKS_EINVAL for invalid or mixed parameters (the first-order
 * fallback must be the same for every instance; batches do not count its
 * replacements) and for prescribed sides. */
int tgks_batch_create(const tgks_params* per_instance, int32_t n_inst, void* hip_stream, tgks_batch** out);
int tgks_batch_destroy(tgks_batch* b);
int tgks_batch_set_stream(tgks_batch* b, void* hip_stream);

/* Doubles of one packed state; offsets (host, n_inst + 1 entries) of the
 * instances' states in it. */
int64_t tgks_batch_state_size(const tgks_batch* b);
int tgks_batch_offsets(const tgks_batch* b, int64_t* offsets);

/* Advance every instance in place by n_steps S2O4 steps, each with its own
 * CFL step (cfl > 0) computed on the device before every step, clipped at
 * t_end when t_end > 0.  time_dev (device, [n_inst][2] doubles, or NULL)
 * receives each instance's (t, dt of the next step).  use_graph != 0
 * captures the whole run into a HIP graph on first use and replays it. */
int tgks_batch_run(tgks_batch* b, double* W_packed, int32_t n_steps, double cfl, double t_end, double* time_dev,
                   int32_t use_graph);

/* Failure counts per instance (host array of n_inst; synchronises). */
int tgks_batch_status(tgks_batch* b, int64_t* failures);

/* Steps each instance actually took (dt > 0) in the last run (host array of
 * n_inst; synchronises): an instance stops at t_end or after a non-physical
 * state (its dt is then NaN and later steps leave it unchanged). */
int tgks_batch_steps(tgks_batch* b, int64_t* steps);
int tgks_batch_reset_status(tgks_batch* b);

/* 2-D tile shape (as tgks_set_tile) and its autotuner over the whole batch:
 * every shape is timed over `steps` batched steps of W_packed (not
 * modified); the fastest is kept.  ms_per_variant: host, 3 floats, or NULL. */
int tgks_batch_set_tile(tgks_batch* b, int32_t tile);
int tgks_batch_tune(tgks_batch* b, const double* W_packed, int32_t steps, int32_t* chosen, float* ms_per_variant);

#ifdef __cplusplus
}
#endif
#endif /* TGKS_H */
