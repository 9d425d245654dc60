/*
 * mp_weno.h -- C ABI of the MI355X (gfx950) implementation of the consistent,
 * bound-preserving finite-volume WENO scheme for compressible two-/N-phase
 * flow of Huang, "Consistent and bound-preserving finite-volume WENO scheme
 * for compressible two-/N-phase flows with Phase-Field mechanism".
 *
 * The library advances the hyperbolic step of the paper's fractional-step
 * method (Sec. 2.2.1, Eq. (3)) on uniform grids:
 *   WENO5 with the relative-smoothness weights of Eq. (15) on the primitive
 *   variables, the coupled reconstruction of phase masses and volume fractions
 *   (Eq. (16)), the positivity / unity / cell-admissibility limiters
 *   (Eqs. (17)-(20)) or the consistent limiter (Eqs. (23)-(25)), the energy
 *   limiter (Eq. (21)), the HLLC or HLL flux with the consistent face velocity
 *   (Sec. 2.2.1), the source alpha_p (1 + K_p) div(u) of Eq. (1), third-order
 *   SSP Runge-Kutta (Sec. 4), the stiffened-gas / Le Metayer EOS of Eq. (26)
 *   with the pressure of Eq. (27), and the CFL time step.
 *
 * Plain C99.  No HIP or torch types appear here: device memory is passed as
 * plain pointers, the HIP stream as void*.
 *
 * Conserved-state layout (Eq. (1), n_U = 2N + d + 1, Eq. (8)):
 *   double U[n_U][n_z][n_y][n_x]  (structure of arrays, x fastest) with the
 *   component order m_1..m_N (m_p = alpha_p rho_p), (rho u)_1..(rho u)_d,
 *   rho E, alpha_1..alpha_N.  All N volume fractions are stored.
 *
 * Ownership: the caller owns every U and every output array and keeps them
 * alive until the stream has completed the call.  The library owns the
 * context and its scratch memory (RK stage buffers, reductions).  Contexts
 * are independent (no global state); one context must not be used from two
 * host threads at once.
 *
 * Errors: every entry point returns an mp_status.  On MP_ERR_HIP the HIP
 * error text is kept in the context (mp_weno_last_error).  Input states must
 * lie in the admissible set of Eq. (8) with rho > 0; without check_bounds the
 * result for inadmissible input is unspecified (but every memory access stays
 * inside the arrays described here).
 */
#ifndef MP_WENO_H
#define MP_WENO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MP_WENO_ABI_VERSION 3
#define MP_MAXP 8        /* largest N this header describes                 */
#define MP_DIAG_LEN 40   /* doubles per instance written by mp_weno_diag    */

typedef enum {
  MP_OK = 0,
  MP_ERR_ARG = -1,          /* invalid argument (message in the context)   */
  MP_ERR_HIP = -2,          /* a HIP runtime call failed                    */
  MP_ERR_OOM = -3,          /* device allocation failed                     */
  MP_ERR_INADMISSIBLE = -4, /* a state left the admissible set (Eq. (8))    */
  MP_ERR_NONFINITE = -5,    /* a state holds NaN or Inf                     */
  MP_ERR_SOLVER = -6,       /* the solve of Eq. (4) did not converge        */
  MP_ERR_UNSUPPORTED = -7   /* valid but not built (e.g. N above the build) */
} mp_status;

/* Boundary conditions per end: periodic (both ends of the direction),
 * outflow (zero-gradient ghost cells), or a symmetry plane (ghost cells are
 * the mirror images of the interior cells with the normal momentum negated:
 * no mass crosses it; the planes of the shock-vessel-bubble problem,
 * Sec. "Shock-vessel-bubble interaction").  The Phase-Field flux and
 * Eq. (4) treat outflow ends and symmetry planes alike: no face. */
enum { MP_BC_PERIODIC = 0, MP_BC_OUTFLOW = 1, MP_BC_SYMMETRY = 2 };
/* Reconstructions: WENO-C (Sec. 3.4) and WENO-CL (Sec. 3.4.1) are the
 * method; WENO_JS and WENO_W are the comparison schemes of Sec. 3.2 and
 * Sec. 3.3: plain WENO5 on the primitive variables, every variable with its
 * own weights (Eq. (12) with epsilon = 1e-6, or Eq. (15)), without the
 * coupling of Eq. (16) and without any limiter (energy_limiter is ignored
 * for them).  They exist to reproduce the consistency and temperature
 * errors of Sec. 4.1.1; they preserve neither consistency nor bounds. */
enum { MP_RECON_WENO_C = 0, MP_RECON_WENO_CL = 1, MP_RECON_WENO_JS = 2,
       MP_RECON_WENO_W = 3 };
enum { MP_FLUX_HLLC = 0, MP_FLUX_HLL = 1 };
enum { MP_MODEL_ALLAIRE = 0, MP_MODEL_KAPILA = 1 };
enum { MP_PREC_FP64 = 0, MP_PREC_MIXED = 1 };
/* Cell value of alpha_p in the source alpha_p (1 + K_p) div u of Eq. (1):
 * MP_SRC_CELL, the cell average (Eq. (3) as written, the default), or
 * MP_SRC_NORMALIZED, the average over sum_q alpha_q of the cell (equal for
 * a consistent state; then the phases' sources sum to the face-velocity
 * difference exactly as their fluxes do, so a rounding deviation of
 * sum_q alpha_q from 1 is transported but not amplified where the flow
 * expands). */
enum { MP_SRC_CELL = 0, MP_SRC_NORMALIZED = 1 };
enum { MP_WHERE_DEVICE = 0, MP_WHERE_HOST = 1 };

/* One uniform-grid problem instance (Sec. 2.1 and Eq. (26)). */
typedef struct {
  int32_t ndim;            /* 1, 2 or 3 (3: N <= 3)                         */
  int32_t n[3];            /* cells per direction, n[k] >= 1; unused = 1     */
  double dx[3];            /* uniform cell size per direction, > 0           */
  int32_t bc[3][2];        /* MP_BC_* at the low/high end of each direction  */
  int32_t nphase;          /* N, 1 <= N <= mp_weno_max_phases()              */
  double gamma[MP_MAXP];   /* gamma_p > 1 (Eq. (26))                         */
  double pinf[MP_MAXP];    /* P^inf_p (Eq. (26))                             */
  double D[MP_MAXP];       /* D_p (Eq. (26))                                 */
  double pmin[MP_MAXP];    /* (P_min)_p of the energy functional, Eq. (9)    */
  double cT[MP_MAXP];      /* C^T_p (Eq. (26)); diagnostics only, may be 0   */
  double t_end;            /* end time: the CFL step is clipped to reach it;
                              0 disables the clipping                        */
  double *U;               /* device pointer to the caller-owned state       */
} mp_weno_instance;

/* Scheme switches shared by all instances of a context. */
typedef struct {
  int32_t recon;           /* MP_RECON_WENO_C (Sec. 3.4), _WENO_CL (3.4.1),
                              or the comparators _WENO_JS, _WENO_W          */
  int32_t flux;            /* MP_FLUX_HLLC (Sec. 4.1) or MP_FLUX_HLL (4.2)   */
  int32_t model;           /* MP_MODEL_ALLAIRE (K_p = 0) or _KAPILA (Sec. 2.1)*/
  int32_t precision;       /* MP_PREC_FP64 or MP_PREC_MIXED                  */
  int32_t energy_limiter;  /* 1: apply Eq. (21) (default); 0: skip it       */
  int32_t phase_field;     /* 1: each step ends with the Phase-Field step of
                              Sec. 2.2.1 (Eqs. (4), (5), (28)); 0: off       */
  double cfl;              /* CFL number of the time step (> 0).  The bounds
                              of Eq. (8) are guaranteed for the updated
                              averages only with cfl <= 1/12 and the HLL
                              flux (Sec. 4.2: Gauss-Lobatto end weight);
                              above it (the paper runs its applications at
                              0.2) they are observed, not guaranteed, and
                              an intermediate RK stage may leave them while
                              the step's result is back inside           */
  double eta_over_dx;      /* eta / min_d dx_d of Eq. (28) (> 0; 1 in Sec. 4) */
  double cg_rtol;          /* Eq. (4) solve: stop once the true residual
                              ||res|| = ||-[div J] - K Q|| <= cg_rtol ||[div J]||
                              + 64 eps || |[div J]| + |K| |Q| || (the second
                              term: the rounding floor of res itself), or
                              once a restart no longer halves it while it is
                              <= 1e4 cg_rtol ||[div J]|| (stagnation at the
                              attainable accuracy of the FP32-preconditioned
                              flexible CG; a run whose recurrence sits within
                              1e4 cg_rtol without halving for 50 iterations
                              ends for that check); <= 0: 1e-12             */
  int32_t cg_maxit;        /* iteration limit of that solve (<= 0: 10000)    */
  int32_t check_bounds;    /* 1: mp_weno_step checks the result of each step
                              (not the intermediate RK stages; see below)  */
  int32_t use_graph;       /* 1: replay mp_weno_step as a captured HIP graph */
  int32_t alpha_source;    /* MP_SRC_CELL (0, default) or MP_SRC_NORMALIZED  */
} mp_weno_opts;

typedef struct mp_weno_ctx mp_weno_ctx;

/* MP_WENO_ABI_VERSION of the built library. */
int32_t mp_weno_abi_version(void);
/* Largest number of phases the built kernels support. */
int32_t mp_weno_max_phases(void);

/* Create a context for n_inst >= 1 instances.  inst[] and opt are copied;
 * the instances' U pointers are kept (not owned).  hip_stream is a
 * hipStream_t (NULL: the null stream; not allowed with use_graph, which
 * captures on the stream); every later call is ordered on it.
 * Allocates the scratch: two RK stage buffers and one direction accumulator
 * per instance (3 n_U doubles per cell) plus small reduction buffers; with
 * phase_field, (10 + d) N doubles per cell more (k_p, [div J_p], Q_p and the
 * two solutions before it, the CG
 * vectors r, p, K p, w and u, and the face gradients) and the FP32
 * multigrid hierarchy (6 N floats per cell of every level, 7 N in 3D:
 * about 8 N floats per cell in 2D, 12 N in 1D and 8 N in 3D).
 * Errors: MP_ERR_ARG (ndim outside 1..3, bad sizes, gamma <= 1, dx <= 0, a
 * boundary code out of range, periodic at one end of a direction only,
 * phase_field with eta_over_dx <= 0, ...), MP_ERR_UNSUPPORTED (valid but
 * beyond the build: N > mp_weno_max_phases(), or in 3D N > 3),
 * MP_ERR_OOM, MP_ERR_HIP.
 * On error *ctx is NULL. */
mp_status mp_weno_init(mp_weno_ctx **ctx, int32_t n_inst,
                       const mp_weno_instance *inst, const mp_weno_opts *opt,
                       void *hip_stream);

/* The hyperbolic semi-discrete operator L(U) of Eq. (3) (summed over the
 * directions) for every instance.  U_in: host array of n_inst device
 * pointers (NULL: use the instances' U); dUdt: host array of n_inst device
 * pointers to caller-owned outputs in the U layout.  Asynchronous on the
 * context's stream.  This is the parity entry point. */
mp_status mp_weno_rhs(mp_weno_ctx *ctx, const double *const *U_in,
                      double *const *dUdt);

/* Two-level coupling of a context's instances (block-structured refinement,
 * Sec. 3.4.2: the scheme runs unchanged on each uniform level).  Link k
 * makes instance `fine` the refinement by 2 of the W x H coarse cells
 * [lo[0], lo[0] + W) x [lo[1], lo[1] + H) of instance `coarse` (1D: W cells
 * from lo[0]).  The fine instance's grid is that block refined, 2W x 2H
 * cells, surrounded by a ring of 3 ghost cells: n = (2W + 6, 2H + 6), dx
 * half the coarse dx; its ring is overwritten by the coupling (its boundary
 * codes do not matter) and is not part of the solution.  From then on each
 * mp_weno_step / mp_weno_advance of the context, per RK stage, fills the
 * ring from the coarse stage state (each ghost cell takes its coarse
 * parent's average) and evaluates the interface fluxes of both levels;
 * after the step the coarse cells under the block take the mean of their
 * four children, the ring takes the new coarse values, and the coarse
 * cells beside the block are corrected by the difference of the fine and
 * coarse interface fluxes (RK3-weighted), with
 * the alpha source on the same face velocities: m_p, rho u and rho E are
 * conserved over the composite grid (coarse cells outside the blocks plus
 * fine cells inside) to rounding.  Linked instances share the smallest of
 * their CFL steps (an external dt must be equal for them).  Requirements:
 * same N and d (1 or 2) for every link, the block at least 3 coarse cells
 * from every coarse boundary, blocks of one coarse instance at least 6
 * coarse cells apart, an instance refining at most one block; no
 * Phase-Field step.  n_links = 0 removes the coupling.  mp_weno_rhs stays
 * per instance.  Synchronises the stream; drops captured step graphs.
 * Errors: MP_ERR_ARG (geometry), MP_ERR_UNSUPPORTED (3D, phase_field,
 * links of several (N, d)), MP_ERR_OOM. */
typedef struct {
  int32_t fine;            /* index of the refined instance                  */
  int32_t coarse;          /* index of the coarse instance                   */
  int32_t lo[3];           /* first coarse cell of the block per direction   */
} mp_weno_link;

mp_status mp_weno_amr_link(mp_weno_ctx *ctx, int32_t n_links,
                           const mp_weno_link *links);

/* Allocation-free L(U): for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The operator of mp_weno_rhs for ONE instance, without a
 * context: inst and opt as for mp_weno_init (use_graph and phase_field are
 * ignored; inst->U is not read unless U_in is NULL), U_in the device state
 * (or NULL: inst->U), dUdt a caller-owned device output in the U layout.
 * Enqueued on hip_stream (a hipStream_t; NULL: the null stream) and
 * asynchronous; calls no allocating routine, so it may be captured into a
 * graph.  Its scratch (the instance descriptor and, in 2D and 3D, the
 * direction accumulator of n_U doubles per cell) is one static device array
 * per GPU of mp_weno_rhs_noalloc_scratch_bytes() bytes (64 MiB), held until
 * the process ends: 4096 + 8 n_U cells bytes must fit (2D, N = 2: up to
 * 1.19 M cells), else MP_ERR_UNSUPPORTED.  Every call on a GPU shares that
 * array, so calls that overlap on one GPU (two streams, two host threads)
 * race; calls ordered on one stream do not.  Results equal mp_weno_rhs of a
 * context holding the same instance with its default tile shapes.
 * Errors: as mp_weno_init's argument checks; MP_ERR_HIP (launch failure or
 * no scratch address on this device). */
mp_status mp_weno_rhs_noalloc(const mp_weno_instance *inst, const mp_weno_opts *opt,
                              const double *U_in, double *dUdt, void *hip_stream);
size_t mp_weno_rhs_noalloc_scratch_bytes(void);

/* The Phase-Field fields of Sec. 2.2.1 for every instance, from the volume
 * fractions of U_in (host array of n_inst device pointers; NULL or a NULL
 * entry: the instance's U) taken as the order parameters phi_p:
 *   divj[i]: [div J_p] of Eq. (28), N fields [p][cells] (second-order
 *            Laplacian, mid-point integrals, M = eta max|u| / 2, multipliers
 *            over the present phases);
 *   grad[i]: the face gradients dQ_p/dx_d of the solution of Eq. (4), d N
 *            fields [d][p][cells], at the upper face of each cell (0 at an
 *            outflow end or a symmetry plane, across faces where
 *            phi(1 - phi) vanishes on both sides, and for a phase with
 *            [div J_p] = 0);
 *   dUdt[i]: the Phase-Field operator of Eq. (5), div F^PF, with those
 *            gradients and the WENO-C/CL face states of U_in (U layout).
 * Any of divj, grad, dUdt may be NULL (not computed); a non-NULL dUdt must
 * hold n_inst non-NULL pointers.  The solve of Eq. (4) starts from Q = 0.
 * Needs phase_field = 1 (else MP_ERR_UNSUPPORTED); synchronises the stream
 * (the solve is driven from the host); MP_ERR_SOLVER if the solve did not
 * reach cg_rtol within cg_maxit iterations (over at most 16 restarts of the
 * conjugate gradients from the current Q; the message names the residual).
 * The parity entry point of the Phase-Field step. */
mp_status mp_weno_pf_fields(mp_weno_ctx *ctx, const double *const *U_in,
                            double *const *divj, double *const *grad,
                            double *const *dUdt);

/* Autotuner: for every group of instances with the same (N, d), time the
 * tile shapes of the sweeps (x strips of 256, 128 or 64 lanes; y tiles, and
 * in 3D z tiles of the same shape, of 16 x 16, 32 x 8 or 16 x 24 lanes) and
 * the XCD-aware tile order (off / on; with the comparison schemes
 * MP_RECON_WENO_JS / WENO_W, built with the default shapes only, just the
 * order) on the current states, reps launches each (0: 8) in two interleaved rounds (the
 * faster round counts), and keep the fastest for the
 * hyperbolic sweeps of later calls.  The timing evaluates L(U) into the
 * context's stage buffer: the states, the time and the step count are not
 * touched.  Synchronises the stream; drops a captured step graph (the next
 * mp_weno_step captures again).  choice (may be NULL): host array of
 * 4 n_inst int32 that receives per instance the x strip width, the y tile
 * width and height (0 in 1D) and the tile order (0 plain, 1 XCD-aware). */
mp_status mp_weno_autotune(mp_weno_ctx *ctx, int32_t reps, int32_t *choice);

/* CFL time step per instance: dt = cfl / max_cells sum_d (|u_d| + c)/dx_d,
 * clipped so that t + dt <= t_end (t is the instance's time, advanced by
 * mp_weno_step); instances coupled by mp_weno_amr_link get the smallest of
 * their steps.  where = MP_WHERE_DEVICE: dt is a device array of n_inst
 * doubles (asynchronous); MP_WHERE_HOST: a host array (synchronises the
 * stream). */
mp_status mp_weno_dt(mp_weno_ctx *ctx, double *dt, int32_t where);

/* Advance every instance by one third-order SSP Runge-Kutta step, in place in
 * the instances' U.  An instance whose step is 0 (it reached its t_end, or
 * an external dt of 0) is skipped by the sweeps: its state stays bitwise
 * unchanged and its tiles cost nothing, so a batch retires its instances as
 * they finish.  dt_dev: device array of n_inst time steps, or NULL to
 * use the CFL step computed on the device inside the same call.  Each
 * instance's time and step counter advance on the device.  Asynchronous,
 * except with check_bounds = 1: then the call synchronises, checks the new
 * states for non-finite values (MP_ERR_NONFINITE) and for violations of the
 * bounds of Eq. (8) (MP_ERR_INADMISSIBLE); on either error every U is
 * restored to its value before the step and the time is not advanced.
 * With phase_field = 1 the hyperbolic step is followed by the Phase-Field
 * step (Sec. 2.2.1) with the same dt: [div J] and Eq. (4) on the hyperbolic
 * result (the solve starts from the previous step's Q), then SSP-RK3 of
 * Eq. (5) with the gradients frozen.  That step synchronises the stream (its
 * solve is driven from the host) and is never replayed from a graph.
 * MP_ERR_SOLVER: the solve did not converge; U then holds the hyperbolic
 * result (restored to the state before the step with check_bounds = 1) and
 * the time is not advanced. */
mp_status mp_weno_step(mp_weno_ctx *ctx, const double *dt_dev);

/* nsteps calls of mp_weno_step(ctx, NULL) (the device CFL step).  With
 * use_graph (and neither profiling, check_bounds nor the Phase-Field step,
 * which need the host between steps) runs of 16 steps are captured once as
 * one graph and replayed, so consecutive steps follow each other without a
 * graph launch between them.  Asynchronous; results identical to nsteps
 * single steps.  nsteps = 0 only captures that graph (if use_graph applies
 * and it is not captured yet) and advances nothing, so a timed run that
 * follows does not include the capture. */
mp_status mp_weno_advance(mp_weno_ctx *ctx, int32_t nsteps);

/* Diagnostics per instance, MP_DIAG_LEN doubles each (out[i*MP_DIAG_LEN+k]):
 *   k = 0 .. n_U-1 : sum over cells of U_c times the cell volume
 *   k = 20         : max over cells |sum_p alpha_p - 1|
 *   k = 21, 22, 23 : min m_p, min alpha_p, max alpha_p over cells and phases
 *   k = 24         : min over cells of psi(U) (Eq. (9))
 *   k = 25         : number of non-finite entries
 *   k = 26, 27     : instance time t and number of steps taken
 *   k = 29, 30     : Phase-Field step: CG iterations (over restarts) and
 *                    the true relative residual ||-[div J] - K Q|| /
 *                    ||[div J]|| (largest over phases) of the last solve of
 *                    Eq. (4) (0 when it is off)
 *   k = 32, 33     : the two integrals of the interface thickness N_I of
 *                    Eq. (30) for alpha_1: the volume of the cells with
 *                    0.05 <= alpha_1 <= 0.95, and the integral of
 *                    |grad alpha_1| (central differences inside, one-sided
 *                    ones at the two ends of each direction), so that
 *                    N_I = out[32] / (min_d dx_d * out[33])
 * where = MP_WHERE_HOST (synchronises) or MP_WHERE_DEVICE. */
mp_status mp_weno_diag(mp_weno_ctx *ctx, double *out, int32_t where);

/* Set the time of every instance (host array of n_inst values; synchronises
 * the stream). */
mp_status mp_weno_set_time(mp_weno_ctx *ctx, const double *t);

/* Profiling: which = 0 off; 1, 2, 3 record a HIP event pair on the context's
 * stream around the x sweeps of every RK stage made by mp_weno_step, around
 * its transverse sweeps (y, and z in 3D), or around the whole stage (graph
 * replay is bypassed while profiling).  Resets the recorded launches. */
mp_status mp_weno_profile(mp_weno_ctx *ctx, int32_t which);

/* Total elapsed milliseconds and number of the launches recorded since the
 * last reset (synchronises the stream); reset = 1 starts a new window. */
mp_status mp_weno_timing(mp_weno_ctx *ctx, int32_t reset, double *ms,
                         int64_t *launches);

/* Free the context and its scratch; never touches U.  NULL is accepted. */
mp_status mp_weno_destroy(mp_weno_ctx *ctx);

/* Static text for a status code. */
const char *mp_weno_strerror(mp_status s);
/* Text of the last error recorded in ctx ("" if none). */
const char *mp_weno_last_error(const mp_weno_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
