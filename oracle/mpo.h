/*
 * mpo.h -- the FP64 CPU oracle for the consistent, bound-preserving WENO
 * scheme ("WENO-C" / "WENO-CL") of Huang, "Consistent and bound-preserving
 * finite-volume WENO scheme for compressible two-/N-phase flows with
 * Phase-Field mechanism".
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference the GPU
 * path is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never calls it.
 * It shares no code, header, table or helper with the HIP library.
 *
 * Everything is double precision, evaluated in the paper's order with no
 * blocking, fusion or reordering (built with -ffp-contract=off).
 *
 * State layout (Sec. 2.1, Eq. (1)): U[c][z][y][x], x fastest, with the
 * component order  m_1..m_N, (rho u)_1..(rho u)_d, rho E, alpha_1..alpha_N
 * where m_p = alpha_p rho_p;  n_U = 2N + d + 1 (Eq. (8)).
 */
#ifndef MPO_H
#define MPO_H

#ifdef __cplusplus
extern "C" {
#endif

#define MPO_MAXP 8

enum { MPO_BC_PERIODIC = 0, MPO_BC_OUTFLOW = 1, MPO_BC_SYMMETRY = 2 };
/* WENO_JS and WENO_W are the comparison schemes of Sec. 3.2 and Sec. 3.3:
 * plain WENO5 on the primitive variables, every variable with its own
 * weights (Eq. (12) with epsilon = MPO_WENOJS_EPS, or Eq. (15)), no
 * coupling of Eq. (16) and none of the limiters of Sec. 3.4. */
enum { MPO_RECON_WENO_C = 0, MPO_RECON_WENO_CL = 1, MPO_RECON_WENO_JS = 2,
       MPO_RECON_WENO_W = 3 };
#define MPO_WENOJS_EPS 1e-6
/* Cell value of alpha_p in the source alpha_p (1 + K_p) div u (Eq. (1)):
 * the cell average itself (the equation as written), or the average over
 * the cell's sum of volume fractions (equal for a consistent state). */
enum { MPO_SRC_CELL = 0, MPO_SRC_NORMALIZED = 1 };
enum { MPO_FLUX_HLLC = 0, MPO_FLUX_HLL = 1 };
enum { MPO_MODEL_ALLAIRE = 0, MPO_MODEL_KAPILA = 1 };

/* status codes; the numeric values match the product library's by design */
enum {
  MPO_OK = 0, MPO_ERR_ARG = -1, MPO_ERR_INADMISSIBLE = -4,
  MPO_ERR_NONFINITE = -5, MPO_ERR_SOLVER = -6, MPO_ERR_UNSUPPORTED = -7
};

typedef struct {
  int ndim;                 /* 1, 2 (or 3)                                   */
  int n[3];                 /* cells per direction; unused directions = 1    */
  double dx[3];             /* uniform cell sizes                            */
  int bc[3][2];             /* MPO_BC_* at the low / high end per direction  */
  int nphase;               /* N in [1, MPO_MAXP]                            */
  double gamma[MPO_MAXP];   /* stiffened-gas gamma_p        (Eq. (26))       */
  double pinf[MPO_MAXP];    /* P^inf_p                      (Eq. (26))       */
  double D[MPO_MAXP];       /* D_p                          (Eq. (26))       */
  double pmin[MPO_MAXP];    /* user minimum pressure (P_min)_p (Eq. (9))     */
  double cT[MPO_MAXP];      /* C^T_p, temperature EOS, diagnostics only      */
  int recon;                /* MPO_RECON_*                                   */
  int flux;                 /* MPO_FLUX_*                                    */
  int model;                /* MPO_MODEL_*                                   */
  int energy_limiter;       /* 1: apply Eq. (21); 0: skip it (ablation)      */
  double cfl;               /* CFL number for mpo_dt                         */
  double t_end;             /* 0: no clipping                                */
  int alpha_source;         /* MPO_SRC_CELL (default) or MPO_SRC_NORMALIZED  */
} mpo_problem;

int mpo_nU(const mpo_problem *pb);
long mpo_ncells(const mpo_problem *pb);

/* ---- building blocks (exported so the tests can pin them) -------------- */

/* Fifth-order WENO on a uniform grid (Sec. 3.1, Eq. (10)): the three
 * smoothness indicators of the sub-stencils {i-2..i}, {i-1..i+1}, {i..i+2}. */
void mpo_weno5_beta(const double q[5], double beta[3]);
/* Candidate values of the three sub-stencil polynomials at x_{i+1/2} (cL) and
 * at x_{i-1/2} (cR). */
void mpo_weno5_candidates(const double q[5], double cL[3], double cR[3]);
/* Candidate increments f^(s) - fbar_i (same faces as above), computed from
 * differences of the stencil so that constant data gives exact zeros. */
void mpo_weno5_increments(const double q[5], double dL[3], double dR[3]);
/* Ideal weights d^(s) of the left-of-face (x_{i+1/2}) and right-of-face
 * (x_{i-1/2}) reconstructions. */
void mpo_weno5_ideal(double dL[3], double dR[3]);
/* Interior value f^C of a cell from its average and face values, Eq. (6)
 * inverted with the four-point Gauss-Lobatto weights (end weights 1/12). */
double mpo_gl_interior(double fbar, double fL, double fR);
/* (1 + K_p) of the alpha source of Eq. (1) at the conserved cell state U:
 * 1 for the Allaire model, rho c^2 / (rho_p c_p^2) for the Kapila model. */
double mpo_one_plus_K(const mpo_problem *pb, const double *U, int p);
/* WENO-W weights, Sec. 3.3, Eq. (15). */
void mpo_wenow_weights(const double beta[3], const double d[3], double w[3]);
/* WENO-JS weights (Eq. (12) generalised to three stencils); comparator only. */
void mpo_wenojs_weights(const double beta[3], const double d[3], double eps,
                        double w[3]);
/* Scalar WENO5-W: q[0..4] = cell averages i-2..i+2 -> qL = f^L_{i+1/2},
 * qR = f^R_{i-1/2}. */
void mpo_weno5w(const double q[5], double *qL, double *qR);

/* Pressure from the conserved state, Eq. (27); u[] receives the velocity. */
double mpo_pressure(const mpo_problem *pb, const double *U, int stride,
                    double *u);
/* Mixture sound speed, Eq. (2) with the stiffened-gas EOS; K_p per model. */
double mpo_sound_speed(const mpo_problem *pb, const double *alpha,
                       const double *m, double P);
/* Energy functional psi(U), Eq. (9), with the EOS of Eq. (26). */
double mpo_psi(const mpo_problem *pb, const double *U);
/* Temperature, Eq. (29). */
double mpo_temperature(const mpo_problem *pb, const double *U, int stride);

/* WENO-C / WENO-CL reconstruction of one cell along direction dir.
 *   Us    : five conserved states (cells i-2..i+2), each n_U contiguous
 *   UL    : out, U^L_{i+1/2}  (n_U)       VL: out, face primitives
 *   UR    : out, U^R_{i-1/2}  (n_U)       VR: out, face primitives
 * Primitive face vectors hold  m_1..m_N, u_1..u_d, P, alpha_1..alpha_N.
 * info (may be NULL) receives diagnostics: [0] = theta_i, [1] = theta_psi,
 * [2] = 1 if the closure fallback was taken. */
void mpo_reconstruct_cell(const mpo_problem *pb, const double *Us, int dir,
                          double *UL, double *UR, double *VL, double *VR,
                          double *info);

/* Numerical flux across a face normal to dir, from the left state (UL, VL)
 * and the right state (UR, VR): F (n_U entries, the alpha entries are the
 * numerical flux of alpha_p) and the face velocity uhat (Sec. 2.2.1). */
void mpo_flux(const mpo_problem *pb, int dir, const double *UL,
              const double *VL, const double *UR, const double *VR, double *F,
              double *uhat);

/* ---- whole-grid operators --------------------------------------------- */

/* Semi-discrete operator L(U) of Eq. (3) (hyperbolic step), summed over the
 * directions.  U and L are full arrays in the layout above. */
int mpo_rhs(const mpo_problem *pb, const double *U, double *L);
/* CFL time step: cfl / max_i sum_d (|u_d| + c) / dx_d, clipped so that
 * t + dt <= t_end when t_end > 0. */
double mpo_dt(const mpo_problem *pb, const double *U, double t);
/* One third-order SSP Runge-Kutta step of the hyperbolic operator, in place. */
int mpo_step(const mpo_problem *pb, double *U, double dt);
/* Diagnostics: out[0..n_U-1] = sum_cells U_c * cell volume;
 * out[n_U+0] = max |sum_p alpha_p - 1|, [n_U+1] = min_p,cells m_p,
 * [n_U+2] = min alpha_p, [n_U+3] = max alpha_p, [n_U+4] = min psi,
 * [n_U+5] = count of non-finite entries. */
int mpo_diag(const mpo_problem *pb, const double *U, double *out);

/* ---- Phase-Field step (Sec. 2.2.1, Eqs. (4)-(5); Sec. 4, Eq. (28)) ------ */

/* g'(phi) of the double well g(phi) = phi^2 (1 - phi)^2 of Eq. (28). */
double mpo_pf_gprime(double phi);

/* [div J_p] of the reduction-consistent conservative Allen-Cahn model,
 * Eq. (28), with the volume fractions of U as the order parameters phi_p:
 * second-order central Laplacian (ghost cells by the boundary rule),
 * mid-point integrals, mobility M = eta max_cells |u| / 2.
 * The multipliers B_q solve the integral system of Eq. (28); that system is
 * singular (its rows and columns sum to zero when sum_p phi_p = 1), so it is
 * solved over the present phases (integral of phi_p > 0) with B of the last
 * present phase set to 0 (reading; L^c does not depend on the choice).
 * divj: N fields, divj[p * ncells + cell].
 * info (may be NULL; 2 + MPO_MAXP entries): [0] = M, [1] = number of present
 * phases, [2 + q] = B_q. */
int mpo_pf_divj(const mpo_problem *pb, const double *U, double eta,
                double *divj, double *info);

/* Phase-Field numerical flux across a face normal to dir (reading of the
 * bound-preserving flux the paper cites): from the face primitives VL, VR
 * (m, u, P, alpha), the face gradients G_p = dQ_p/dx_dir and the face
 * coefficients kf_p of Eq. (4),
 *   F^alpha_p = min(G_p,0) c(alpha_p^L (1 - alpha_p^R))
 *             + max(G_p,0) c(alpha_p^R (1 - alpha_p^L)),  c(x) = min(x, kf_p)
 * (the donor side gives, the receiver needs room, and the flux never exceeds
 * the k_f dQ/dx that Eq. (4) delivers), F^m_p the same with m_p as the donor
 * factor (scaled by the same cap), momentum and energy carried with the
 * donor's u and (|u|^2/2, A_p P + B_p, D_p) as in F^PF of Eq. (1); then
 * S = sum_p F^alpha_p is removed in proportion to the face-average alpha_p
 * (mass in proportion to the face-average m_p, with face-average u and P), so
 * that sum_p F^alpha_p = 0 at every face. */
void mpo_pf_flux(const mpo_problem *pb, int dir, const double *VL,
                 const double *VR, const double *G, const double *kf,
                 double *F);

/* The Phase-Field operator of Eq. (5), L^PF(U) = div F^PF, with WENO-C/CL
 * face states, frozen face gradients G and frozen cell coefficients K:
 * G[(d * N + p) * ncells + cell] is dQ_p/dx_d at the upper face
 * (x_{i+1/2}) of the cell, K[p * ncells + cell] the k_p of Eq. (4) there
 * (the face coefficient is the mean of its two cells). */
int mpo_pf_rhs(const mpo_problem *pb, const double *U, const double *G,
               const double *K, double *L);
/* Third-order SSP Runge-Kutta of the Phase-Field step with G and K frozen,
 * in place (Sec. 4: the same time stepping as the hyperbolic step). */
int mpo_pf_rk3(const mpo_problem *pb, double *U, const double *G,
               const double *K, double dt);

/* threads the OpenMP loops use (1 when built without OpenMP) */
int mpo_num_threads(void);
void mpo_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
