/*
 * lbm.h -- C ABI of the MI355X library for the multiphase lattice Boltzmann
 * model with self-tuning equation of state of Huang, Wu & Adams
 * (arXiv:1809.02390): the D2Q9 step with the pairwise interaction force
 * (main Eq. 12), the moment-space collision with built-in EOS, velocity-
 * dependent collision matrix, cubic-velocity corrections and the epsilon^3
 * consistency term (main Eq. 13 = supplement Eq. 1, executed by the
 * six-step sequence of supplement Sec. IV), and streaming (supplement Eq. 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Lattice units: dx = dt = c = 1, c_s^2 = 1/3.  Periodic in x and y.
 *  - Fields are row-major with x fastest: element (y, x) of an ny-by-nx
 *    field sits at offset y*nx + x.  Distribution arrays passed as plain
 *    float arrays (f, lam) are structure-of-arrays, population i (velocity
 *    order of supplement Eq. 3: rest, +x, +y, -x, -y, +x+y, -x+y, -x-y,
 *    +x-y) at offset i*nx*ny.  The library's own buffers (A/B states,
 *    checkpoints, adjoint states) have internal layouts; size them with the
 *    *_bytes calls.
 *  - Field and buffer pointers (f, f_*, rho*, u*, lam, adj*, drho0, src,
 *    dst) are DEVICE pointers owned by the caller (any allocator; the
 *    library never frees them).  The result pointers out, sigma_out,
 *    totals, dtheta, dparams, jac and which, and the pointer arrays bufs and
 *    f_states (whose elements are device pointers), are HOST pointers.
 *  - Every call is asynchronous on the stream given to lbm_create (or
 *    lbm_set_stream), except where stated: lbm_init, lbm_moments (with
 *    totals), lbm_adjoint_theta (with dtheta) and lbm_adjoint_params
 *    synchronise that stream to return host results.
 *  - Every int-returning call returns LBM_OK (0) or a negative status;
 *    lbm_last_error() then returns a message for the calling thread.  A
 *    failed call launches nothing and leaves the state unchanged, except
 *    LBM_EHIP (a HIP runtime error), after which the state is undefined.
 *  - The library allocates only small device scratch inside the context
 *    (reduction partials, the parameter-gradient accumulator and a status
 *    word), cleared on the stream at lbm_create; lbm_destroy frees it.
 *    Every state, checkpoint and adjoint buffer belongs to the caller.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx; /* opaque, library-owned host object */

enum lbm_status {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* invalid argument or parameter                   */
  LBM_ENOCOEX = -2,    /* no two-phase coexistence (Maxwell solve failed)  */
  LBM_EHIP = -3,       /* HIP runtime error                                */
  LBM_ENONFINITE = -4, /* a non-finite total mass or momentum was found    */
  LBM_ESTATE = -5      /* call not valid in the current state              */
};

/* Storage of the post-collision populations in the A/B buffers.  The
 * 2-byte storages keep S (f_i - f_ref,i) with f_ref the rest equilibrium at
 * the reference density of the node the population streams to (that node's
 * previous density in binary16, held in the rho_ref buffer), S = 2^12 for
 * binary16 and 1 for bfloat16; arithmetic stays FP32.  The A/B buffer
 * contents are internal; lbm_set_state / lbm_get_state exchange plain FP32
 * post-streaming populations in the SoA layout above. */
enum lbm_storage {
  LBM_FP32 = 0, /* f_i stored as float                                  */
  LBM_FP16 = 1, /* scaled deviations in binary16                        */
  LBM_BF16 = 2  /* scaled deviations in bfloat16                        */
};

/* The paper's problem statement: lattice, relaxation rates, varpi, the
 * Carnahan-Starling EOS parameters (main Eq. 20), and the prescribed surface
 * tension and interface thickness (main Eq. 23). */
typedef struct lbm_params {
  int32_t nx, ny;  /* lattice size, >= 1 each, nx*ny*9 < 2^31            */
  int32_t storage; /* enum lbm_storage                                   */
  int32_t reserved;/* must be 0                                          */
  double s_p;      /* shear rate, 0 < s_p < 2; nu = (1/s_p - 1/2)/3      */
  double s_eps;    /* rate of the energy-square moment; <= 0 means s_e   */
  double varpi;    /* bulk-viscosity coefficient, 0 < varpi < 1, != 1/3  */
  double a, b;     /* CS attraction and co-volume, > 0                   */
  double r_gas;    /* gas constant R, > 0                                */
  double tr;       /* reduced temperature T/T_c, 0 < tr < 1              */
  double sigma;    /* surface tension (lattice units); <= 0 means the
                      paper's sound-speed rule, lbm_sigma_paper()        */
  double width;    /* 5%-95% interface thickness W (lattice units), > 0  */
} lbm_params;

/* Coefficients the parameter map derives (all FP64, lattice units). */
typedef struct lbm_derived {
  double rho_g, rho_l, p0;   /* Maxwell coexistence densities and pressure  */
  double c_sigma, c_w;       /* flat-interface sigma and W at K_EOS=K_INT=1 */
  double sigma, width;       /* the prescribed (or default) sigma, W        */
  double k_int, k_eos;       /* K_INT = W/C_W, K_EOS = sigma/(C_sigma K_INT) */
  double g2;                 /* G^2 = 2 K_INT^2 K_EOS a (main Eq. 21)       */
  double kp;                 /* K' = K_EOS, prefactor of the CS pressure    */
  double rt;                 /* R T = R tr T_c                              */
  double alpha2, beta2;      /* main Eq. 7 with alpha1 = -1, beta1 = 1      */
  double k, h, bs;           /* k, h, b of main Eq. 7                       */
  double s_p, s_q, s_e, s_eps; /* rates; s_q, s_e from main Eq. 16         */
  double tc;                 /* critical temperature of the CS constants    */
} lbm_derived;

/* Message for the last failed call on this thread ("" if none). */
const char* lbm_last_error(void);

/* Host-only parameter map (no GPU needed).  Validates *p and fills *out:
 * Maxwell construction (main Eq. 19), C_sigma and C_W from the flat
 * interface of the pressure tensor (main Eqs. 17-18), the sigma/W map
 * (main Eqs. 21, 23), coefficients (main Eq. 7) and rates (main Eq. 16).
 * Returns LBM_EINVAL for bad parameters, LBM_ENOCOEX if the Maxwell solve
 * fails. */
int lbm_derive(const lbm_params* p, lbm_derived* out);

/* Host-only: the sigma at which the paper's sound-speed rule (main Eq. 22)
 * gives lattice speed c = 1 for thickness `width` at `tr`. */
int lbm_sigma_paper(double width, double tr, double a, double b, double r_gas,
                    double* sigma_out);

/* Bytes of ONE distribution buffer (the caller provides two, A and B):
 * 9*P*4 for LBM_FP32 and 9*P*2 for the 2-byte storages, with P = nx*ny
 * rounded up to a multiple of 64 plus 16640 bytes' worth of elements
 * (16640/4 or 16640/2).  The layout inside is internal: the rows are
 * interleaved (the nine populations of a lattice row are nine consecutive
 * rows of the buffer, 9*nx*ny*es bytes in all).  0 on error. */
size_t lbm_state_bytes(const lbm_params* p);

/* Bytes of the reference-density buffer the 2-byte storages need (two
 * binary16 planes of nx*ny); 0 for LBM_FP32 or on error. */
size_t lbm_ref_bytes(const lbm_params* p);

/* Create a context over caller-owned device buffers f_a, f_b (each
 * lbm_state_bytes) and rho_ref (lbm_ref_bytes; may be NULL for LBM_FP32),
 * on HIP stream `stream` (a hipStream_t; NULL = default stream), on the
 * current HIP device.  Derives the coefficients and clears the context's
 * scratch on the stream.  The state is uninitialised until lbm_init,
 * lbm_set_state or lbm_load_state. */
int lbm_create(lbm_ctx** out, const lbm_params* p, void* f_a, void* f_b,
               void* rho_ref, void* stream);

/* Change the stream used by later calls.  Work already queued on the old
 * stream is ordered before anything later calls queue on the new one. */
int lbm_set_stream(lbm_ctx* ctx, void* stream);

/* Initial state f_i = (M^-1 m^eq(rho0, u0, eta(rho0)))_i at t = 0 (main
 * Eq. 3; zero velocity when ux0 / uy0 are NULL).  rho0, ux0, uy0 are device
 * float fields of nx*ny.  Synchronises the stream; LBM_EINVAL if any rho0 is
 * not finite, <= 0 or >= 4/b (the pole of the CS EOS). */
int lbm_init(lbm_ctx* ctx, const float* rho0, const float* ux0, const float* uy0);

/* Load a post-streaming state f(t) (device float, 9*nx*ny, layout above)
 * and set the step counter to 0. */
int lbm_set_state(lbm_ctx* ctx, const float* f);

/* Export the post-streaming state f(t) as device float (9*nx*ny). */
int lbm_get_state(lbm_ctx* ctx, float* f);

/* Advance n >= 0 time steps of main Eq. 13 with the force of main Eq. 12
 * (the collision by the six steps of supplement Sec. IV), alternating A
 * and B.  Each step fuses the
 * density halo, the force, the collision and the streaming.  LBM_FP32
 * (lattices up to about 3.7M nodes wide): two steps per kernel launch (the
 * state between them is never written) on tiles of 64 x 24 nodes, or of
 * 64 x 16 or 32 x 8 where the larger ones give fewer tiles than the device
 * has compute units, then one step for an odd remainder; every node is
 * updated by the same operations as in a single step, so the result is
 * bitwise that of n calls with n = 1.  The 2-byte storages take one step
 * per launch.
 * The call only launches kernels on the context's stream (no allocation,
 * copy or synchronisation), so it can be captured into a HIP graph on that
 * stream.  A graph replays the launches with the A/B buffers they were
 * recorded with, while the context switches buffers once per launch when
 * the call is made: capture n a multiple of 4, which ends on the buffer it
 * started from for every storage and launch shape, and each replay then
 * advances the state by n steps (the step counter counts the captured call
 * only). */
int lbm_step(lbm_ctx* ctx, int32_t n);

/* Macroscopic fields at the current time: rho = sum_i f_i and
 * u = (sum_i e_i f_i + F/2)/rho (main Eq. 5), written to the device float
 * fields rho, ux, uy (each may be NULL), and, if totals is not NULL, the
 * FP64 totals {sum rho, sum_x sum_i e_ix f_i, sum_x sum_i e_iy f_i} reduced
 * deterministically on the device (synchronises the stream).  Returns
 * LBM_ENONFINITE if a total is not finite. */
int lbm_moments(lbm_ctx* ctx, float* rho, float* ux, float* uy, double totals[3]);

/* lbm_moments for callers that cannot allocate or synchronise (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same fields rho, ux, uy (device, each may be NULL) from the same
 * kernel, and, if totals_dev is not NULL, the same FP64 totals written to
 * `totals_dev`, a DEVICE array of 3 doubles, with no synchronisation (so no
 * non-finite check: test the totals after the stream has finished); unlike
 * the host `totals` of the other calls, totals_dev is device memory.  The
 * call allocates nothing: the per-workgroup partial sums go to a fixed
 * 2 MiB device array of the library (each device holds one until the
 * process ends), which limits it to lattices of at most 87381 workgroups of
 * 64 x 16 nodes (about 89M nodes; LBM_EINVAL beyond, before any launch).
 * All contexts on one device share that array: calls that overlap on one
 * device race, so issue them on one stream or order them.  Nothing carries
 * over between calls (every partial is written before it is read).
 * LBM_EHIP if the runtime gave no device address for the array at
 * lbm_create. */
int lbm_moments_noalloc(lbm_ctx* ctx, float* rho, float* ux, float* uy, double* totals_dev);

/* ---- Checkpoints --------------------------------------------------------
 * A checkpoint is the library's own copy of the current state: the pull
 * buffer (lbm_state_bytes) followed, for the 2-byte storages, by the
 * reference-density plane (2*nx*ny bytes).  Its layout is internal. */

/* Bytes of one checkpoint buffer; 0 on error. */
size_t lbm_checkpoint_bytes(const lbm_params* p);

/* Copy the current state into the device buffer dst (lbm_checkpoint_bytes). */
int lbm_save_state(lbm_ctx* ctx, void* dst);

/* Make a checkpoint the current state and set the step counter to t >= 0.
 * Stepping from it repeats the run it was saved from bit for bit. */
int lbm_load_state(lbm_ctx* ctx, const void* src, int64_t t);

/* One step from the checkpoint src into the checkpoint dst (distinct device
 * buffers) with the kernel of lbm_step, so dst is bitwise what lbm_step
 * would leave; the context's own state is not touched.  This is the
 * recomputation of a checkpoint segment for the adjoint.  LBM_FP32 only. */
int lbm_step_saved(lbm_ctx* ctx, const void* src, void* dst);

/* n steps from checkpoint to checkpoint: bufs[j+1] := step(bufs[j]) for
 * j = 0 .. n-1 (a host array of n+1 device checkpoint buffers, consecutive
 * ones distinct), bitwise as lbm_step_saved.  Where bufs[j+2] is not
 * bufs[j] and lbm_step takes two steps per launch, the steps j and j+1 run
 * as one launch of its two-step kernel that also writes bufs[j+1] (all n+1
 * buffers distinct: every pair does).  One call recomputes a checkpoint
 * segment.  LBM_FP32 only. */
int lbm_step_saved_chain(lbm_ctx* ctx, void* const* bufs, int32_t n);

/* ---- Adjoint (reverse mode) of a rollout; LBM_FP32 storage only ---------
 * For a scalar loss L of the state, the adjoint of time t is
 * Lambda_i(x, t) = dL/d f_i(x, t) of the post-streaming populations.  One
 * adjoint step maps Lambda(t+1) to Lambda(t) = (d step / d f(t))^T Lambda(t+1)
 * (the transposed Jacobian of the step of main Eq. 13 with the force of main
 * Eq. 12 and streaming, supplement Eq. 2) and adds Lambda(t+1) .
 * d step / d theta to the context's FP64 accumulator of dL/d theta,
 * theta = (G'^2, K', R T).
 *
 * Adjoint states live in caller-owned device buffers of lbm_adjoint_bytes
 * (eleven FP32 fields in an internal layout: Lambda is held as nine fields
 * plus the two-component adjoint of the force-stencil gradient, which the
 * next step scatters to the neighbour densities; rows interleaved when
 * 44*nx*ny < 2^32, else eleven planes).  lbm_adjoint_seed and
 * lbm_adjoint_get convert from and to plain Lambda arrays in the SoA layout
 * of the populations.  The accumulator starts at zero when the context is
 * created and is summed and cleared by lbm_adjoint_theta.  Accumulation and
 * its sum run in a fixed order: repeated runs give identical bits. */

/* Bytes of one adjoint state buffer (11*P*4, P as for lbm_state_bytes with
 * FP32 elements); 0 for the 2-byte storages or on error. */
size_t lbm_adjoint_bytes(const lbm_params* p);

/* adj := the adjoint state of Lambda = lam (device float, 9*nx*ny). */
int lbm_adjoint_seed(lbm_ctx* ctx, const float* lam, void* adj);

/* One adjoint step: f_t is the checkpoint of the forward state at time t
 * (lbm_save_state or lbm_step_saved), adj_next the adjoint state of time
 * t+1, adj_out (a different buffer) receives that of time t.  Adds the
 * theta terms of this step to the accumulator. */
int lbm_adjoint_step(lbm_ctx* ctx, const void* f_t, const void* adj_next, void* adj_out);

/* n adjoint steps back through a segment: f_states[j] (host array of n
 * device checkpoints) is the forward state of time t0 + j; the adjoint state
 * of time t0 + n is in adj_a on entry.  The steps run from j = n-1 down to 0,
 * alternating between adj_a and adj_b; on return *which (host) is 0 if the
 * adjoint of time t0 is in adj_a, 1 if in adj_b.  Adds the theta terms of
 * every step to the accumulator. */
int lbm_adjoint_run(lbm_ctx* ctx, const void* const* f_states, int32_t n, void* adj_a, void* adj_b,
                    int32_t* which);

/* lam := Lambda of the adjoint state adj (device float, 9*nx*ny). */
int lbm_adjoint_get(lbm_ctx* ctx, const void* adj, float* lam);

/* Adjoint of the initial state f_i(x, 0) = f_i^eq(rho0(x), u0(x), eta(rho0))
 * of lbm_init: drho0(x) = sum_i Lambda_i(x, 0) d f_i^eq / d rho0 (u0 held
 * fixed; ux0 / uy0 NULL means zero) from the adjoint state adj0 of time 0;
 * adds the theta terms of eta(rho0; theta) to the accumulator.  rho0, ux0,
 * uy0 and drho0 are device float fields of nx*ny. */
int lbm_adjoint_init(lbm_ctx* ctx, const float* rho0, const float* ux0, const float* uy0, const void* adj0,
                     float* drho0);

/* If dtheta is not NULL, write the accumulated dL/d(G'^2, K', R T) there
 * (synchronises the stream); then clear the accumulator if reset != 0.
 * LBM_ENONFINITE if a component is not finite. */
int lbm_adjoint_theta(lbm_ctx* ctx, double dtheta[3], int32_t reset);

/* dL/d(sigma, W, T_r) of the accumulated adjoint: dparams[j] =
 * sum_k jac[3*k + j] dL/dtheta_k with jac = lbm_param_jacobian at the
 * context's parameters (the chain rule through theta = (G'^2, K', R T) of
 * main Eqs. 20, 21, 23).  Reads the accumulator like lbm_adjoint_theta
 * (synchronises the stream) and clears it if reset != 0; dparams (host, 3)
 * receives the three derivatives, dtheta (host, 3, may be NULL) dL/dtheta.
 * LBM_ENONFINITE if a component is not finite. */
int lbm_adjoint_params(lbm_ctx* ctx, double dparams[3], double dtheta[3], int32_t reset);

/* Host-only: jac[3*k + j] = d theta_k / d (sigma, W, T_r)_j at the point of
 * *p (main Eqs. 20, 21, 23), with sigma the value lbm_derive reports, held
 * independent of W and T_r.  The T_r column differentiates the flat-
 * interface constants numerically (fourth-order central difference). */
int lbm_param_jacobian(const lbm_params* p, double jac[9]);

/* Number of steps taken since lbm_init / lbm_set_state. */
int64_t lbm_time(const lbm_ctx* ctx);

/* Copy the derived coefficients of a context. */
int lbm_get_derived(const lbm_ctx* ctx, lbm_derived* out);

/* Destroy a context: frees its scratch on its device (waiting for its work
 * in flight); never the caller's buffers. */
void lbm_destroy(lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
