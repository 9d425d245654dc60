/*
 * mpo.c -- FP64 CPU oracle for the WENO-C / WENO-CL hyperbolic step.
 *
 * TEST INFRASTRUCTURE ONLY (see mpo.h).  Plain loops, double precision,
 * built with -ffp-contract=off.  Each function cites the passage of the paper
 * it follows; readings of points the paper leaves open are marked "reading".
 */
#include "mpo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Gauss-Lobatto weights at the cell ends for the fifth-order scheme: the
 * quartic needs N_quad = 4, whose end weights are 1/12 (Sec. 4.2). */
static const double GL_W1 = 1.0 / 12.0;
static const double GL_WN = 1.0 / 12.0;

int mpo_nU(const mpo_problem *pb) { return 2 * pb->nphase + pb->ndim + 1; }

long mpo_ncells(const mpo_problem *pb) {
  long n = 1;
  for (int d = 0; d < pb->ndim; ++d) n *= pb->n[d];
  return n;
}

int mpo_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void mpo_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---------------------------------------------------------------------- */
/* Equation of state: Le Metayer form, Eq. (26):                           */
/*   e_p^(1)(P) = A_p P + B_p,  e_p^(2) = D_p,                             */
/*   A_p = 1/(gamma_p - 1),  B_p = gamma_p Pinf_p / (gamma_p - 1).         */
/* ---------------------------------------------------------------------- */
static double eos_A(const mpo_problem *pb, int p) {
  return 1.0 / (pb->gamma[p] - 1.0);
}
static double eos_B(const mpo_problem *pb, int p) {
  return pb->gamma[p] * pb->pinf[p] / (pb->gamma[p] - 1.0);
}

/* component offsets */
#define IM(p) (p)
#define IMOM(pb, k) ((pb)->nphase + (k))
#define IE(pb) ((pb)->nphase + (pb)->ndim)
#define IA(pb, p) ((pb)->nphase + (pb)->ndim + 1 + (p))

/* Pressure, Eq. (27): P = (rhoE - |rho u|^2/(2 rho) - sum B_p alpha_p
 *                          - sum D_p m_p) / sum A_p alpha_p.
 * Mixture density from Sec. 2.1: rho = sum_p m_p.  Velocity u = (rho u)/rho.
 * U is read with the given stride between components. */
double mpo_pressure(const mpo_problem *pb, const double *U, int stride,
                    double *u) {
  const int N = pb->nphase, d = pb->ndim;
  double rho = 0.0;
  for (int p = 0; p < N; ++p) rho = rho + U[(long)IM(p) * stride];
  double mom2 = 0.0;
  for (int k = 0; k < d; ++k) {
    double mk = U[(long)IMOM(pb, k) * stride];
    mom2 = mom2 + mk * mk;
    if (u) u[k] = (rho > 0.0) ? mk / rho : 0.0;
  }
  double ke = (rho > 0.0) ? 0.5 * mom2 / rho : 0.0;
  double sA = 0.0, sB = 0.0, sD = 0.0;
  for (int p = 0; p < N; ++p) {
    double a = U[(long)IA(pb, p) * stride];
    double m = U[(long)IM(p) * stride];
    sA = sA + eos_A(pb, p) * a;
    sB = sB + eos_B(pb, p) * a;
    sD = sD + pb->D[p] * m;
  }
  return (U[(long)IE(pb) * stride] - ke - sB - sD) / sA;
}

/* Temperature, Eq. (29), with B^T_p = Pinf_p (Eq. (26)). */
double mpo_temperature(const mpo_problem *pb, const double *U, int stride) {
  const int N = pb->nphase, d = pb->ndim;
  double rho = 0.0;
  for (int p = 0; p < N; ++p) rho = rho + U[(long)IM(p) * stride];
  double mom2 = 0.0;
  for (int k = 0; k < d; ++k) {
    double mk = U[(long)IMOM(pb, k) * stride];
    mom2 = mom2 + mk * mk;
  }
  double ke = (rho > 0.0) ? 0.5 * mom2 / rho : 0.0;
  double sC = 0.0, sB = 0.0, sD = 0.0;
  for (int p = 0; p < N; ++p) {
    double a = U[(long)IA(pb, p) * stride];
    double m = U[(long)IM(p) * stride];
    sC = sC + pb->cT[p] * m;
    sB = sB + pb->pinf[p] * a;
    sD = sD + pb->D[p] * m;
  }
  return (U[(long)IE(pb) * stride] - ke - sB - sD) / sC;
}

/* Mixture sound speed, Eq. (2).  For the EOS of Eq. (26):
 *   (de_p/dP)_rho m_p = A_p alpha_p,  rho_p c_p^2 = gamma_p (P + Pinf_p).
 * Allaire (K_p = 0): rho c^2 = sum A_p alpha_p gamma_p (P+Pinf_p) / sum A_p alpha_p.
 * Kapila (K_p = rho c^2/(rho_p c_p^2) - 1): Eq. (2) is then an identity and
 * sum_p alpha_p K_p = 0 (Sec. 2.1) fixes 1/(rho c^2) = sum alpha_p/(rho_p c_p^2).
 * Reading: a non-positive rho c^2 (strong tension) gives c = 0, never a NaN. */
double mpo_sound_speed(const mpo_problem *pb, const double *alpha,
                       const double *m, double P) {
  const int N = pb->nphase;
  double rho = 0.0;
  for (int p = 0; p < N; ++p) rho = rho + m[p];
  double rc2;
  if (pb->model == MPO_MODEL_KAPILA) {
    double s = 0.0, sa = 0.0;
    for (int p = 0; p < N; ++p) {
      if (alpha[p] == 0.0) continue;
      double k = pb->gamma[p] * (P + pb->pinf[p]);
      if (k <= 0.0) return 0.0;
      s = s + alpha[p] / k;
      sa = sa + alpha[p];
    }
    rc2 = (s > 0.0) ? sa / s : 0.0;
  } else {
    double num = 0.0, den = 0.0;
    for (int p = 0; p < N; ++p) {
      double Aa = eos_A(pb, p) * alpha[p];
      num = num + Aa * (pb->gamma[p] * (P + pb->pinf[p]));
      den = den + Aa;
    }
    rc2 = num / den;
  }
  if (!(rc2 > 0.0) || !(rho > 0.0)) return 0.0;
  return sqrt(rc2 / rho);
}

/* Energy functional, Eq. (9): psi = rhoE - |rho u|^2/(2 rho)
 *   - sum_p m_p e_p(Pmin_p, rho_p).  With Eq. (26),
 *   m_p e_p(Pmin_p, rho_p) = alpha_p (A_p Pmin_p + B_p) + m_p D_p,
 * so psi needs no phasic density (Sec. 3.4). */
double mpo_psi(const mpo_problem *pb, const double *U) {
  const int N = pb->nphase, d = pb->ndim;
  double rho = 0.0;
  for (int p = 0; p < N; ++p) rho = rho + U[IM(p)];
  double mom2 = 0.0;
  for (int k = 0; k < d; ++k) mom2 = mom2 + U[IMOM(pb, k)] * U[IMOM(pb, k)];
  double ke = (rho > 0.0) ? 0.5 * mom2 / rho : 0.0;
  double emin = 0.0;
  for (int p = 0; p < N; ++p)
    emin = emin + (U[IA(pb, p)] * (eos_A(pb, p) * pb->pmin[p] + eos_B(pb, p)) +
                   U[IM(p)] * pb->D[p]);
  return U[IE(pb)] - ke - emin;
}

/* ---------------------------------------------------------------------- */
/* Fifth-order WENO on a uniform grid (Sec. 3.1, Eq. (10); r = 2, N_s = 3). */
/* Sub-stencil s = {i-3+s, .., i-1+s}, s = 1..3 (Sec. 3.1).                 */
/* ---------------------------------------------------------------------- */
void mpo_weno5_beta(const double q[5], double beta[3]) {
  /* Jiang-Shu smoothness indicators of the three quadratics. */
  double a, b;
  a = q[0] - 2.0 * q[1] + q[2];
  b = q[0] - 4.0 * q[1] + 3.0 * q[2];
  beta[0] = 13.0 / 12.0 * a * a + 0.25 * b * b;
  a = q[1] - 2.0 * q[2] + q[3];
  b = q[1] - q[3];
  beta[1] = 13.0 / 12.0 * a * a + 0.25 * b * b;
  a = q[2] - 2.0 * q[3] + q[4];
  b = 3.0 * q[2] - 4.0 * q[3] + q[4];
  beta[2] = 13.0 / 12.0 * a * a + 0.25 * b * b;
}

void mpo_weno5_candidates(const double q[5], double cL[3], double cR[3]) {
  /* values at x_{i+1/2} of the quadratics with the given cell averages */
  cL[0] = (2.0 * q[0] - 7.0 * q[1] + 11.0 * q[2]) / 6.0;
  cL[1] = (-q[1] + 5.0 * q[2] + 2.0 * q[3]) / 6.0;
  cL[2] = (2.0 * q[2] + 5.0 * q[3] - q[4]) / 6.0;
  /* values at x_{i-1/2} */
  cR[0] = (-q[0] + 5.0 * q[1] + 2.0 * q[2]) / 6.0;
  cR[1] = (2.0 * q[1] + 5.0 * q[2] - q[3]) / 6.0;
  cR[2] = (11.0 * q[2] - 7.0 * q[3] + 2.0 * q[4]) / 6.0;
}

void mpo_weno5_ideal(double dL[3], double dR[3]) {
  dL[0] = 0.1; dL[1] = 0.6; dL[2] = 0.3;
  dR[0] = 0.3; dR[1] = 0.6; dR[2] = 0.1;
}

/* WENO-W weights, Eq. (15):
 *   w_s = d_s / (d_s + sum_{k != s} d_k (IS^(s,k))^2),
 *   IS^(s,k) = 1 if IS^(s) = IS^(k) = 0, else IS^(s)/IS^(k).
 * No epsilon (Sec. 3.3).  In IEEE arithmetic IS^(k) = 0 < IS^(s) gives an
 * infinite ratio and hence w_s = 0, the limit of the definition. */
void mpo_wenow_weights(const double beta[3], const double d[3], double w[3]) {
  for (int s = 0; s < 3; ++s) {
    double den = d[s];
    for (int k = 0; k < 3; ++k) {
      if (k == s) continue;
      double r = (beta[s] == 0.0 && beta[k] == 0.0) ? 1.0 : beta[s] / beta[k];
      den = den + d[k] * (r * r);
    }
    w[s] = d[s] / den;
  }
}

/* WENO-JS weights (Eq. (12), three stencils): comparator only. */
void mpo_wenojs_weights(const double beta[3], const double d[3], double eps,
                        double w[3]) {
  double a[3], s = 0.0;
  for (int k = 0; k < 3; ++k) {
    double t = beta[k] + eps;
    a[k] = d[k] / (t * t);
    s = s + a[k];
  }
  for (int k = 0; k < 3; ++k) w[k] = a[k] / s;
}

/* Candidate increments f^(s) - fbar_i at both faces, written with the
 * differences a = q_{i-2} - q_i, b = q_{i-1} - q_i, c = q_{i+1} - q_i,
 * e = q_{i+2} - q_i, so that a constant sub-stencil gives an exact zero. */
void mpo_weno5_increments(const double q[5], double dL[3], double dR[3]) {
  const double a = q[0] - q[2], b = q[1] - q[2], c = q[3] - q[2],
               e = q[4] - q[2];
  dL[0] = (2.0 * a - 7.0 * b) / 6.0;
  dL[1] = (2.0 * c - b) / 6.0;
  dL[2] = (5.0 * c - e) / 6.0;
  dR[0] = (5.0 * b - a) / 6.0;
  dR[1] = (2.0 * b - c) / 6.0;
  dR[2] = (2.0 * e - 7.0 * c) / 6.0;
}

/* Eq. (10) with the weights of Eq. (15).  Reading: the weighted sum is
 * evaluated as fbar + sum_s w_s (f^(s) - fbar), equal to sum_s w_s f^(s)
 * since the weights sum to one, but exact on a constant stencil.  The
 * plain sum returns fbar (1 +- ulp) there, which the consistent limiter of
 * Eq. (25) reads as a slope and answers by limiting that phase to first
 * order; the paper's limiter leaves zero-gradient fractions untouched
 * (Sec. 3.4.1). */
static void weno5w_with(const double q[5], const double wL[3],
                        const double wR[3], double *qL, double *qR) {
  double dL[3], dR[3];
  mpo_weno5_increments(q, dL, dR);
  *qL = q[2] + (wL[0] * dL[0] + wL[1] * dL[1] + wL[2] * dL[2]);
  *qR = q[2] + (wR[0] * dR[0] + wR[1] * dR[1] + wR[2] * dR[2]);
}

void mpo_weno5w(const double q[5], double *qL, double *qR) {
  double beta[3], dL[3], dR[3], wL[3], wR[3];
  mpo_weno5_beta(q, beta);
  mpo_weno5_ideal(dL, dR);
  mpo_wenow_weights(beta, dL, wL);
  mpo_wenow_weights(beta, dR, wR);
  weno5w_with(q, wL, wR, qL, qR);
}

/* ---------------------------------------------------------------------- */
/* WENO-C limiters                                                          */
/* ---------------------------------------------------------------------- */

/* Interior value from the conservation requirement, Eq. (6) inverted:
 *   f^C = (fbar - w1 f^R_{i-1/2} - wN f^L_{i+1/2}) / (1 - w1 - wN). */
static double interior_value(double fbar, double fL, double fR) {
  return (fbar - GL_W1 * fR - GL_WN * fL) / (1.0 - GL_W1 - GL_WN);
}

double mpo_gl_interior(double fbar, double fL, double fR) {
  return interior_value(fbar, fL, fR);
}

/* Positivity limiter, Eq. (18), with lower bound fmin:
 *   theta = min(1, (fbar - fmin)/(fbar - min(f^C, f^L, f^R))) in [0,1].
 * Reading: theta = 1 when the minimum is already >= fmin (this also covers
 * the 0/0 of an absent phase); the ratio is clamped to [0, 1]. */
static double theta_lower(double fbar, double fC, double fL, double fR,
                          double fmin) {
  double mu = fC;
  if (fL < mu) mu = fL;
  if (fR < mu) mu = fR;
  if (mu >= fmin) return 1.0;
  double den = fbar - mu;
  if (!(den > 0.0)) return 0.0;
  double t = (fbar - fmin) / den;
  if (t > 1.0) t = 1.0;
  if (!(t > 0.0)) t = 0.0;
  return t;
}

/* theta_p of Eq. (17): min of the mass and volume-fraction limiters. */
static double theta_phase(double mbar, double mL, double mR, double abar,
                          double aL, double aR) {
  double tm = theta_lower(mbar, interior_value(mbar, mL, mR), mL, mR, 0.0);
  double ta = theta_lower(abar, interior_value(abar, aL, aR), aL, aR, 0.0);
  return tm < ta ? tm : ta;
}

/* Consistent limiter for one face, Eqs. (23)-(25).  S[p] are the alpha
 * slopes at that face; theta[p] receives theta^(alpha_p).
 * Reading: p_hat is the lowest index among ties of max |S|; all theta = 1
 * when S_phat = 0; theta_{p != phat} = 1 when S_hat = 0 (any value then
 * satisfies sum_p theta_p S_p = 0, and 1 leaves those phases untouched). */
static void consistent_limiter(int N, const double *S, double *theta) {
  int ph = 0;
  double amax = fabs(S[0]);
  for (int p = 1; p < N; ++p)
    if (fabs(S[p]) > amax) { amax = fabs(S[p]); ph = p; }
  if (S[ph] == 0.0) {
    for (int p = 0; p < N; ++p) theta[p] = 1.0;
    return;
  }
  double sum = 0.0;
  for (int p = 0; p < N; ++p) sum = sum + S[p];
  double Shat = S[ph] - sum;
  for (int p = 0; p < N; ++p) {
    double t;
    if (p == ph) {
      t = Shat / S[ph];
    } else {
      if (Shat == 0.0) { theta[p] = 1.0; continue; }
      t = S[ph] / Shat;
    }
    if (t > 1.0) t = 1.0;
    if (!(t > 0.0)) t = 0.0;
    theta[p] = t;
  }
}

/* V -> U map (Sec. 2.2.2): rho = sum m_p, rho u = rho * u,
 * rho E = rho |u|^2 / 2 + sum_p alpha_p (A_p P + B_p) + sum_p m_p D_p
 * (the internal energy of Eq. (26) summed with the mixture rule). */
static void prim_to_cons(const mpo_problem *pb, const double *V, double *U) {
  const int N = pb->nphase, d = pb->ndim;
  const double *m = V, *u = V + N, P = V[N + d], *a = V + N + d + 1;
  double rho = 0.0;
  for (int p = 0; p < N; ++p) rho = rho + m[p];
  double u2 = 0.0;
  for (int k = 0; k < d; ++k) u2 = u2 + u[k] * u[k];
  double rhoe = 0.0;
  for (int p = 0; p < N; ++p)
    rhoe = rhoe + (a[p] * (eos_A(pb, p) * P + eos_B(pb, p)) + m[p] * pb->D[p]);
  for (int p = 0; p < N; ++p) U[IM(p)] = m[p];
  for (int k = 0; k < d; ++k) U[IMOM(pb, k)] = rho * u[k];
  U[IE(pb)] = 0.5 * rho * u2 + rhoe;
  for (int p = 0; p < N; ++p) U[IA(pb, p)] = a[p];
}

/* U -> V map: masses and volume fractions as stored, u = (rho u)/rho,
 * P from Eq. (27). */
static void cons_to_prim(const mpo_problem *pb, const double *U, double *V) {
  const int N = pb->nphase, d = pb->ndim;
  double u[3];
  double P = mpo_pressure(pb, U, 1, u);
  for (int p = 0; p < N; ++p) V[p] = U[IM(p)];
  for (int k = 0; k < d; ++k) V[N + k] = u[k];
  V[N + d] = P;
  for (int p = 0; p < N; ++p) V[N + d + 1 + p] = U[IA(pb, p)];
}

/* The WENO-C reconstruction of Sec. 3.4 (WENO-CL of Sec. 3.4.1 when
 * pb->recon == MPO_RECON_WENO_CL) for the centre cell of Us[0..4].
 * Primitive vectors: m_1..m_N, u_1..u_d, P, alpha_1..alpha_N. */
void mpo_reconstruct_cell(const mpo_problem *pb, const double *Us, int dir,
                          double *UL, double *UR, double *VL, double *VR,
                          double *info) {
  const int N = pb->nphase, d = pb->ndim, nU = mpo_nU(pb);
  const double *Ubar = Us + 2 * nU;
  double V[5][2 * MPO_MAXP + 4];
  double dL[3], dR[3];
  mpo_weno5_ideal(dL, dR);
  int fallback = 0;

  /* Primitive cell averages, Vbar = psi_{U->V}(Ubar) (Sec. 3.4). */
  for (int j = 0; j < 5; ++j) cons_to_prim(pb, Us + j * nU, V[j]);

  if (pb->recon == MPO_RECON_WENO_JS || pb->recon == MPO_RECON_WENO_W) {
    /* Comparison schemes (Sec. 3.2, Sec. 3.3): every primitive variable
     * reconstructed with its own weights, Eq. (12) (epsilon 1e-6) or
     * Eq. (15), as the weighted sum of the candidates (Eqs. (10), (13));
     * no limiter. */
    const int nV = nU;
    for (int c = 0; c < nV; ++c) {
      double q[5], beta[3], wL[3], wR[3], cL[3], cR[3];
      for (int j = 0; j < 5; ++j) q[j] = V[j][c];
      mpo_weno5_beta(q, beta);
      if (pb->recon == MPO_RECON_WENO_JS) {
        mpo_wenojs_weights(beta, dL, MPO_WENOJS_EPS, wL);
        mpo_wenojs_weights(beta, dR, MPO_WENOJS_EPS, wR);
      } else {
        mpo_wenow_weights(beta, dL, wL);
        mpo_wenow_weights(beta, dR, wR);
      }
      mpo_weno5_candidates(q, cL, cR);
      VL[c] = wL[0] * cL[0] + wL[1] * cL[1] + wL[2] * cL[2];
      VR[c] = wR[0] * cR[0] + wR[1] * cR[1] + wR[2] * cR[2];
    }
    prim_to_cons(pb, VL, UL);
    prim_to_cons(pb, VR, UR);
    if (info) { info[0] = 1.0; info[1] = 1.0; info[2] = 0.0; }
    return;
  }

  /* u and P: plain WENO-W on each primitive (Sec. 3.4, Eq. (15)). */
  for (int k = 0; k <= d; ++k) {
    double q[5];
    for (int j = 0; j < 5; ++j) q[j] = V[j][N + k];
    mpo_weno5w(q, &VL[N + k], &VR[N + k]);
  }

  /* Step 1, Eq. (16): weights from m_p, applied to m_p and alpha_p. */
  double mbar[MPO_MAXP], abar[MPO_MAXP];
  double mL[MPO_MAXP], mR[MPO_MAXP], aL[MPO_MAXP], aR[MPO_MAXP];
  for (int p = 0; p < N; ++p) {
    double qm[5], qa[5], beta[3], wL[3], wR[3];
    for (int j = 0; j < 5; ++j) {
      qm[j] = V[j][p];
      qa[j] = V[j][N + d + 1 + p];
    }
    mbar[p] = qm[2];
    abar[p] = qa[2];
    mpo_weno5_beta(qm, beta);
    mpo_wenow_weights(beta, dL, wL);
    mpo_wenow_weights(beta, dR, wR);
    weno5w_with(qm, wL, wR, &mL[p], &mR[p]);
    weno5w_with(qa, wL, wR, &aL[p], &aR[p]);
  }

  /* Step 2, Eqs. (17)-(18): positivity of m_p and alpha_p with one
   * theta_p for both (consistency). */
  for (int p = 0; p < N; ++p) {
    double th = theta_phase(mbar[p], mL[p], mR[p], abar[p], aL[p], aR[p]);
    mL[p] = mbar[p] + th * (mL[p] - mbar[p]);
    mR[p] = mbar[p] + th * (mR[p] - mbar[p]);
    aL[p] = abar[p] + th * (aL[p] - abar[p]);
    aR[p] = abar[p] + th * (aR[p] - abar[p]);
  }

  if (pb->recon == MPO_RECON_WENO_CL) {
    /* Step 3 of WENO-CL, Eqs. (23)-(25): face-wise consistent limiter on
     * the slopes S = (f^face - fbar)/(dx/2).  Reading: the R face uses the
     * same expression (the common sign cancels in every ratio). */
    const double h = 0.5 * pb->dx[dir];
    for (int side = 0; side < 2; ++side) {
      double *mf = side == 0 ? mL : mR, *af = side == 0 ? aL : aR;
      double Sa[MPO_MAXP], Sm[MPO_MAXP], th[MPO_MAXP];
      for (int p = 0; p < N; ++p) {
        Sa[p] = (af[p] - abar[p]) / h;
        Sm[p] = (mf[p] - mbar[p]) / h;
      }
      consistent_limiter(N, Sa, th);
      for (int p = 0; p < N; ++p) {
        mf[p] = mbar[p] + th[p] * Sm[p] * h;
        af[p] = abar[p] + th[p] * Sa[p] * h;
      }
    }
  } else {
    /* Step 3 of WENO-C, Eq. (19): divide by S = sum_p alpha_p at each face.
     * Reading: S <= 0 (every alpha limited to 0 at that face) falls back
     * to first order for the cell. */
    double SL = 0.0, SR = 0.0;
    for (int p = 0; p < N; ++p) { SL = SL + aL[p]; SR = SR + aR[p]; }
    if (SL > 0.0 && SR > 0.0) {
      for (int p = 0; p < N; ++p) {
        mL[p] = mL[p] / SL; aL[p] = aL[p] / SL;
        mR[p] = mR[p] / SR; aR[p] = aR[p] / SR;
      }
    } else {
      fallback = 1;
      for (int p = 0; p < N; ++p) {
        mL[p] = mR[p] = mbar[p];
        aL[p] = aR[p] = abar[p];
      }
    }
  }

  /* Step 4, Eq. (20): recompute theta_p with the updated faces, take the
   * minimum over phases and apply it to every m_p and alpha_p. */
  double thi = 1.0;
  for (int p = 0; p < N; ++p) {
    double th = theta_phase(mbar[p], mL[p], mR[p], abar[p], aL[p], aR[p]);
    if (th < thi) thi = th;
  }
  for (int p = 0; p < N; ++p) {
    mL[p] = mbar[p] + thi * (mL[p] - mbar[p]);
    mR[p] = mbar[p] + thi * (mR[p] - mbar[p]);
    aL[p] = abar[p] + thi * (aL[p] - abar[p]);
    aR[p] = abar[p] + thi * (aR[p] - abar[p]);
    /* Reading: in floating point the limited minimum lands at 0 up to an
     * ulp; clamping to the admissible box makes the bounds of Eq. (8) hold
     * exactly and changes nothing in exact arithmetic. */
    if (mL[p] < 0.0) mL[p] = 0.0;
    if (mR[p] < 0.0) mR[p] = 0.0;
    if (aL[p] < 0.0) aL[p] = 0.0;
    if (aR[p] < 0.0) aR[p] = 0.0;
    if (aL[p] > 1.0) aL[p] = 1.0;
    if (aR[p] > 1.0) aR[p] = 1.0;
  }
  for (int p = 0; p < N; ++p) {
    VL[p] = mL[p]; VR[p] = mR[p];
    VL[N + d + 1 + p] = aL[p]; VR[N + d + 1 + p] = aR[p];
  }

  /* Step 5: U^{L,R} = psi_{V->U}(V^{L,R}) (Sec. 3.4). */
  prim_to_cons(pb, VL, UL);
  prim_to_cons(pb, VR, UR);

  double thpsi = 1.0;
  if (pb->energy_limiter) {
    /* U^C by inverting Eq. (6); theta^psi from Eq. (18) applied to psi of
     * Eq. (9) at Ubar, U^L, U^R, U^C; one value for all components,
     * Eq. (21). */
    double UC[4 * MPO_MAXP + 4];
    for (int c = 0; c < nU; ++c) UC[c] = interior_value(Ubar[c], UL[c], UR[c]);
    double pbar = mpo_psi(pb, Ubar);
    thpsi = theta_lower(pbar, mpo_psi(pb, UC), mpo_psi(pb, UL),
                        mpo_psi(pb, UR), 0.0);
    if (thpsi < 1.0) {
      for (int c = 0; c < nU; ++c) {
        UL[c] = Ubar[c] + thpsi * (UL[c] - Ubar[c]);
        UR[c] = Ubar[c] + thpsi * (UR[c] - Ubar[c]);
      }
      /* Reading: the face primitives fed to the flux are those of the final
       * U^{L,R}; when theta^psi = 1 they are V^{L,R} themselves (U^{L,R}
       * is by construction their image), otherwise they are recovered from
       * U^{L,R} with Eq. (27). */
      cons_to_prim(pb, UL, VL);
      cons_to_prim(pb, UR, VR);
    }
  }
  if (info) {
    info[0] = thi;
    info[1] = thpsi;
    info[2] = fallback;
  }
}

/* ---------------------------------------------------------------------- */
/* Numerical flux (Sec. 2.2.1, Sec. 4.1 HLLC, Sec. 4.2 HLL)                 */
/* ---------------------------------------------------------------------- */

/* Physical flux of Eq. (1) along dir; the alpha entries carry u_n alpha_p
 * (the conservative part of the alpha equation, Eq. (3)). */
static void physical_flux(const mpo_problem *pb, int dir, const double *U,
                          const double *V, double *F) {
  const int N = pb->nphase, d = pb->ndim;
  const double un = V[N + dir], P = V[N + d];
  for (int p = 0; p < N; ++p) F[IM(p)] = U[IM(p)] * un;
  for (int k = 0; k < d; ++k)
    F[IMOM(pb, k)] = U[IMOM(pb, k)] * un + (k == dir ? P : 0.0);
  F[IE(pb)] = un * (U[IE(pb)] + P);
  for (int p = 0; p < N; ++p) F[IA(pb, p)] = U[IA(pb, p)] * un;
}

/* Reading of the solvers the paper cites: Davis wave speeds
 * S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R).
 * HLL: the three-branch formula applied to every component, alpha included.
 * HLLC: Toro's contact speed S* and star states, with m_p and alpha_p both
 * scaled by chi_K = (S_K - u_K)/(S_K - S*), so that the mass and volume-
 * fraction fluxes are the same linear map of their face values.
 * Face velocity (Sec. 2.2.1): uhat = numerical flux of alpha with
 * alpha^L = alpha^R = 1, i.e. (S_R u_L - S_L u_R)/(S_R - S_L) in the HLL fan
 * and chi_K S* in the HLLC star regions. */
void mpo_flux(const mpo_problem *pb, int dir, const double *UL,
              const double *VL, const double *UR, const double *VR, double *F,
              double *uhat) {
  const int N = pb->nphase, d = pb->ndim, nU = mpo_nU(pb);
  double FL[4 * MPO_MAXP + 4], FR[4 * MPO_MAXP + 4];
  double rhoL = 0.0, rhoR = 0.0;
  for (int p = 0; p < N; ++p) { rhoL = rhoL + UL[IM(p)]; rhoR = rhoR + UR[IM(p)]; }
  const double uL = VL[N + dir], uR = VR[N + dir];
  const double PL = VL[N + d], PR = VR[N + d];
  const double cL = mpo_sound_speed(pb, VL + N + d + 1, VL, PL);
  const double cR = mpo_sound_speed(pb, VR + N + d + 1, VR, PR);
  double SL = uL - cL, SR = uR + cR;
  if (uR - cR < SL) SL = uR - cR;
  if (uL + cL > SR) SR = uL + cL;
  physical_flux(pb, dir, UL, VL, FL);
  physical_flux(pb, dir, UR, VR, FR);

  if (SL >= 0.0) {
    for (int c = 0; c < nU; ++c) F[c] = FL[c];
    *uhat = uL;
    return;
  }
  if (SR <= 0.0) {
    for (int c = 0; c < nU; ++c) F[c] = FR[c];
    *uhat = uR;
    return;
  }
  if (pb->flux == MPO_FLUX_HLL) {
    const double inv = 1.0 / (SR - SL);
    for (int c = 0; c < nU; ++c)
      F[c] = (SR * FL[c] - SL * FR[c] + SL * SR * (UR[c] - UL[c])) * inv;
    *uhat = (SR * uL - SL * uR) * inv;
    return;
  }
  /* HLLC */
  const double Sstar =
      (PR - PL + rhoL * uL * (SL - uL) - rhoR * uR * (SR - uR)) /
      (rhoL * (SL - uL) - rhoR * (SR - uR));
  const int left = (Sstar >= 0.0);
  const double *UK = left ? UL : UR, *VK = left ? VL : VR, *FK = left ? FL : FR;
  const double SK = left ? SL : SR, uK = left ? uL : uR, PK = left ? PL : PR;
  const double rhoK = left ? rhoL : rhoR;
  const double chi = (SK - uK) / (SK - Sstar);
  double Us[4 * MPO_MAXP + 4];
  for (int p = 0; p < N; ++p) {
    Us[IM(p)] = chi * UK[IM(p)];
    Us[IA(pb, p)] = chi * UK[IA(pb, p)];
  }
  for (int k = 0; k < d; ++k)
    Us[IMOM(pb, k)] = chi * rhoK * (k == dir ? Sstar : VK[N + k]);
  Us[IE(pb)] =
      chi * (UK[IE(pb)] + (Sstar - uK) * (rhoK * Sstar + PK / (SK - uK)));
  for (int c = 0; c < nU; ++c) F[c] = FK[c] + SK * (Us[c] - UK[c]);
  *uhat = chi * Sstar;
}

/* ---------------------------------------------------------------------- */
/* Whole-grid operator                                                      */
/* ---------------------------------------------------------------------- */

/* Ghost cells (Sec. 4.1 periodic, Sec. 4.2 outflow).  Reading: outflow is a
 * zero-gradient copy of the nearest interior cell. */
/* Cell that stands in for index i of a line of n cells: periodic wrap,
 * outflow (zero-gradient) copy of the end cell, or, at a symmetry plane, the
 * mirror image across the end face (cell -1-i below, 2n-1-i above), clamped
 * into the line when it has fewer cells than the stencil reaches.  *flip is
 * set when the stand-in is a mirror image: its normal momentum changes sign
 * (the plane is a wall the flow does not cross). */
static long ghost_index_flip(long i, long n, int bclo, int bchi, int *flip) {
  *flip = 0;
  if (i < 0) {
    if (bclo == MPO_BC_PERIODIC) return ((i % n) + n) % n;
    if (bclo == MPO_BC_SYMMETRY) {
      long m = -1 - i;
      *flip = 1;
      return m < n ? m : n - 1;
    }
    return 0;
  }
  if (i >= n) {
    if (bchi == MPO_BC_PERIODIC) return i % n;
    if (bchi == MPO_BC_SYMMETRY) {
      long m = 2 * n - 1 - i;
      *flip = 1;
      return m >= 0 ? m : 0;
    }
    return n - 1;
  }
  return i;
}

static long ghost_index(long i, long n, int bclo, int bchi) {
  int flip;
  return ghost_index_flip(i, n, bclo, bchi, &flip);
}

static int check_problem(const mpo_problem *pb) {
  if (!pb || pb->ndim < 1 || pb->ndim > 3) return MPO_ERR_ARG;
  if (pb->nphase < 1 || pb->nphase > MPO_MAXP) return MPO_ERR_ARG;
  for (int d = 0; d < pb->ndim; ++d) {
    if (pb->n[d] < 1 || !(pb->dx[d] > 0.0)) return MPO_ERR_ARG;
    for (int e = 0; e < 2; ++e)
      if (pb->bc[d][e] < MPO_BC_PERIODIC || pb->bc[d][e] > MPO_BC_SYMMETRY) return MPO_ERR_ARG;
    /* a periodic direction is periodic at both ends */
    if ((pb->bc[d][0] == MPO_BC_PERIODIC) != (pb->bc[d][1] == MPO_BC_PERIODIC)) return MPO_ERR_ARG;
  }
  return MPO_OK;
}

/* (1 + K_p) of the source term H^HB in Eq. (1): 1 for Allaire; for Kapila
 * rho c^2 / (rho_p c_p^2) with rho_p c_p^2 = gamma_p (P + Pinf_p). */
static double one_plus_K(const mpo_problem *pb, const double *U, int p) {
  if (pb->model != MPO_MODEL_KAPILA) return 1.0;
  const int N = pb->nphase;
  double V[2 * MPO_MAXP + 4];
  cons_to_prim(pb, U, V);
  const double *m = V, *a = V + N + pb->ndim + 1, P = V[N + pb->ndim];
  double rho = 0.0;
  for (int q = 0; q < N; ++q) rho = rho + m[q];
  double c = mpo_sound_speed(pb, a, m, P);
  double k = pb->gamma[p] * (P + pb->pinf[p]);
  if (!(k > 0.0)) return 1.0;
  return rho * c * c / k;
}

double mpo_one_plus_K(const mpo_problem *pb, const double *U, int p) {
  return one_plus_K(pb, U, p);
}

/* L(U) of Eq. (3): for each direction (dimension by dimension, all from the
 * same Ubar), reconstruct cells -1..n of every line, take the flux at faces
 * -1/2..n-1/2 from (U^L of cell i, U^R of cell i+1) and add
 *   -(F_{i+1/2} - F_{i-1/2})/dx   and, for alpha_p,
 *   +alphabar_p (1 + K_p)(uhat_{i+1/2} - uhat_{i-1/2})/dx
 * (Eq. (3) with H^HB at the cell average).  With alpha_source =
 * MPO_SRC_NORMALIZED the cell value is alphabar_p / S, S = sum_q
 * alphabar_q (1 for a consistent state): the sources then sum to the u-hat
 * difference that the fluxes' alpha parts sum to, so sum_q alpha_q - 1 gets
 * no source of its own (with alphabar_p it grows as
 * (S - 1)(uhat_{i+1/2} - uhat_{i-1/2})/dx where the flow expands). */
int mpo_rhs(const mpo_problem *pb, const double *U, double *L) {
  int st = check_problem(pb);
  if (st != MPO_OK) return st;
  const int N = pb->nphase, nU = mpo_nU(pb), nd = pb->ndim;
  const long nc = mpo_ncells(pb);
  long n3[3] = {1, 1, 1};
  for (int d = 0; d < nd; ++d) n3[d] = pb->n[d];
  const long sx[3] = {1, n3[0], n3[0] * n3[1]};
  memset(L, 0, sizeof(double) * (size_t)nU * (size_t)nc);

  for (int dir = 0; dir < nd; ++dir) {
    const long n = n3[dir], s = sx[dir];
    const int o1 = (dir + 1) % 3, o2 = (dir + 2) % 3;
    const long nl = n3[o1] * n3[o2];
    const double dx = pb->dx[dir];
#pragma omp parallel
    {
      double *UL = malloc(sizeof(double) * (size_t)(n + 2) * nU);
      double *UR = malloc(sizeof(double) * (size_t)(n + 2) * nU);
      double *VL = malloc(sizeof(double) * (size_t)(n + 2) * nU);
      double *VR = malloc(sizeof(double) * (size_t)(n + 2) * nU);
      double *F = malloc(sizeof(double) * (size_t)(n + 1) * nU);
      double *uh = malloc(sizeof(double) * (size_t)(n + 1));
      double Us[5 * (4 * MPO_MAXP + 4)];
#pragma omp for schedule(static)
      for (long line = 0; line < nl; ++line) {
        const long j1 = line % n3[o1], j2 = line / n3[o1];
        const long base = j1 * sx[o1] + j2 * sx[o2];
        for (long i = -1; i <= n; ++i) {
          for (int j = 0; j < 5; ++j) {
            int flip;
            long g = ghost_index_flip(i - 2 + j, n, pb->bc[dir][0], pb->bc[dir][1], &flip);
            for (int c = 0; c < nU; ++c) Us[j * nU + c] = U[c * nc + base + g * s];
            if (flip) Us[j * nU + IMOM(pb, dir)] = -Us[j * nU + IMOM(pb, dir)];
          }
          mpo_reconstruct_cell(pb, Us, dir, UL + (i + 1) * nU, UR + (i + 1) * nU,
                               VL + (i + 1) * nU, VR + (i + 1) * nU, NULL);
        }
        for (long f = 0; f <= n; ++f) /* face between cells f-1 and f */
          mpo_flux(pb, dir, UL + f * nU, VL + f * nU, UR + (f + 1) * nU,
                   VR + (f + 1) * nU, F + f * nU, uh + f);
        for (long i = 0; i < n; ++i) {
          const long cell = base + i * s;
          for (int c = 0; c < nU; ++c)
            L[c * nc + cell] =
                L[c * nc + cell] - (F[(i + 1) * nU + c] - F[i * nU + c]) / dx;
          double Uc[4 * MPO_MAXP + 4];
          for (int c = 0; c < nU; ++c) Uc[c] = U[c * nc + cell];
          double S = 0.0;
          for (int p = 0; p < N; ++p) S = S + Uc[IA(pb, p)];
          for (int p = 0; p < N; ++p) {
            const int c = IA(pb, p);
            const double a = pb->alpha_source != MPO_SRC_NORMALIZED ? Uc[c]
                             : (S > 0.0 ? Uc[c] / S : 0.0);
            L[c * nc + cell] = L[c * nc + cell] +
                               a * one_plus_K(pb, Uc, p) * (uh[i + 1] - uh[i]) / dx;
          }
        }
      }
      free(UL); free(UR); free(VL); free(VR); free(F); free(uh);
    }
  }
  return MPO_OK;
}

/* Time step from the CFL number (Sec. 4.1.5, Sec. 4.2).  Reading: the
 * unsplit sum form max_i sum_d (|u_d| + c)/dx_d. */
double mpo_dt(const mpo_problem *pb, const double *U, double t) {
  if (check_problem(pb) != MPO_OK) return -1.0;
  const int N = pb->nphase, nU = mpo_nU(pb), nd = pb->ndim;
  const long nc = mpo_ncells(pb);
  double smax = 0.0;
#pragma omp parallel for reduction(max : smax) schedule(static)
  for (long i = 0; i < nc; ++i) {
    double Uc[4 * MPO_MAXP + 4], V[2 * MPO_MAXP + 4];
    for (int c = 0; c < nU; ++c) Uc[c] = U[c * nc + i];
    cons_to_prim(pb, Uc, V);
    double c = mpo_sound_speed(pb, V + N + nd + 1, V, V[N + nd]);
    double s = 0.0;
    for (int d = 0; d < nd; ++d) s = s + (fabs(V[N + d]) + c) / pb->dx[d];
    if (s > smax) smax = s;
  }
  double dt = pb->cfl / smax;
  if (pb->t_end > 0.0 && t + dt > pb->t_end) dt = pb->t_end - t;
  return dt;
}

/* Third-order SSP (TVD) Runge-Kutta of Shu and Osher (Sec. 4):
 *   U1 = Un + dt L(Un)
 *   U2 = 3/4 Un + 1/4 U1 + 1/4 dt L(U1)
 *   Un+1 = 1/3 Un + 2/3 U2 + 2/3 dt L(U2)                                   */
int mpo_step(const mpo_problem *pb, double *U, double dt) {
  int st = check_problem(pb);
  if (st != MPO_OK) return st;
  const long nt = (long)mpo_nU(pb) * mpo_ncells(pb);
  double *L = malloc(sizeof(double) * (size_t)nt);
  double *U1 = malloc(sizeof(double) * (size_t)nt);
  double *U2 = malloc(sizeof(double) * (size_t)nt);
  if (!L || !U1 || !U2) { free(L); free(U1); free(U2); return MPO_ERR_ARG; }
  mpo_rhs(pb, U, L);
  for (long k = 0; k < nt; ++k) U1[k] = U[k] + dt * L[k];
  mpo_rhs(pb, U1, L);
  for (long k = 0; k < nt; ++k)
    U2[k] = 0.75 * U[k] + 0.25 * U1[k] + 0.25 * (dt * L[k]);
  mpo_rhs(pb, U2, L);
  for (long k = 0; k < nt; ++k)
    U[k] = U[k] / 3.0 + 2.0 * U2[k] / 3.0 + 2.0 * (dt * L[k]) / 3.0;
  free(L); free(U1); free(U2);
  return MPO_OK;
}

/* Invariants and totals of Sec. 4.1.2 (conservation, volume-fraction sum,
 * bounds of Eq. (8)). */
int mpo_diag(const mpo_problem *pb, const double *U, double *out) {
  int st = check_problem(pb);
  if (st != MPO_OK) return st;
  const int N = pb->nphase, nU = mpo_nU(pb), nd = pb->ndim;
  const long nc = mpo_ncells(pb);
  double vol = 1.0;
  for (int d = 0; d < nd; ++d) vol *= pb->dx[d];
  for (int c = 0; c < nU; ++c) {
    double s = 0.0;
    for (long i = 0; i < nc; ++i) s = s + U[c * nc + i];
    out[c] = s * vol;
  }
  double esum = 0.0, mmin = INFINITY, amin = INFINITY, amax = -INFINITY,
         pmin = INFINITY, nonfin = 0.0;
  for (long i = 0; i < nc; ++i) {
    double Uc[4 * MPO_MAXP + 4], sa = 0.0;
    for (int c = 0; c < nU; ++c) {
      Uc[c] = U[c * nc + i];
      if (!isfinite(Uc[c])) nonfin += 1.0;
    }
    for (int p = 0; p < N; ++p) {
      double a = Uc[IA(pb, p)], m = Uc[IM(p)];
      sa = sa + a;
      if (m < mmin) mmin = m;
      if (a < amin) amin = a;
      if (a > amax) amax = a;
    }
    double e = fabs(sa - 1.0);
    if (e > esum) esum = e;
    double ps = mpo_psi(pb, Uc);
    if (ps < pmin) pmin = ps;
  }
  out[nU + 0] = esum;
  out[nU + 1] = mmin;
  out[nU + 2] = amin;
  out[nU + 3] = amax;
  out[nU + 4] = pmin;
  out[nU + 5] = nonfin;
  return MPO_OK;
}

/* ---------------------------------------------------------------------- */
/* Phase-Field step                                                         */
/* ---------------------------------------------------------------------- */

/* g(phi) = phi^2 (1 - phi)^2  =>  g'(phi) = 2 phi (1 - phi)(1 - 2 phi). */
double mpo_pf_gprime(double phi) {
  return 2.0 * phi * (1.0 - phi) * (1.0 - 2.0 * phi);
}

/* Dense Gaussian elimination with partial pivoting, n <= MPO_MAXP; returns
 * 0 if a pivot is exactly zero. */
static int small_solve(int n, double A[MPO_MAXP][MPO_MAXP], double *b) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (fabs(A[i][k]) > fabs(A[piv][k])) piv = i;
    if (A[piv][k] == 0.0) return 0;
    if (piv != k) {
      for (int j = 0; j < n; ++j) {
        double t = A[k][j]; A[k][j] = A[piv][j]; A[piv][j] = t;
      }
      double t = b[k]; b[k] = b[piv]; b[piv] = t;
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = A[i][k] / A[k][k];
      for (int j = k; j < n; ++j) A[i][j] = A[i][j] - f * A[k][j];
      b[i] = b[i] - f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int j = k + 1; j < n; ++j) s = s - A[k][j] * b[j];
    b[k] = s / A[k][k];
  }
  return 1;
}

/* W_{p,q} of Eq. (28) */
static double pf_W(const double *phi, int p, int q) {
  return p == q ? phi[p] * (1.0 - phi[q]) : -phi[p] * phi[q];
}

int mpo_pf_divj(const mpo_problem *pb, const double *U, double eta,
                double *divj, double *info) {
  int st = check_problem(pb);
  if (st != MPO_OK) return st;
  if (!(eta > 0.0)) return MPO_ERR_ARG;
  const int N = pb->nphase, nd = pb->ndim;
  const long nc = mpo_ncells(pb);
  long n3[3] = {1, 1, 1};
  for (int d = 0; d < nd; ++d) n3[d] = pb->n[d];
  const long sx[3] = {1, n3[0], n3[0] * n3[1]};
  double vol = 1.0;
  for (int d = 0; d < nd; ++d) vol *= pb->dx[d];

  /* mobility M = 0.5 eta max |u| over the cells */
  double umax = 0.0;
  for (long i = 0; i < nc; ++i) {
    double rho = 0.0, u2 = 0.0;
    for (int p = 0; p < N; ++p) rho = rho + U[IM(p) * nc + i];
    for (int k = 0; k < nd; ++k) {
      const double u = U[IMOM(pb, k) * nc + i] / rho;
      u2 = u2 + u * u;
    }
    const double s = sqrt(u2);
    if (s > umax) umax = s;
  }
  const double M = 0.5 * eta * umax;
  const double Me2 = M / (eta * eta);

  /* R_p = M/eta^2 (g'(phi_p) - phi_p sum_q g'(phi_q)) and the integrals */
  double *R = malloc(sizeof(double) * (size_t)N * (size_t)nc);
  if (!R) return MPO_ERR_ARG;
  double Wint[MPO_MAXP][MPO_MAXP], Rint[MPO_MAXP], phint[MPO_MAXP];
  for (int p = 0; p < N; ++p) {
    Rint[p] = 0.0;
    phint[p] = 0.0;
    for (int q = 0; q < N; ++q) Wint[p][q] = 0.0;
  }
  for (long i = 0; i < nc; ++i) {
    double phi[MPO_MAXP], sg = 0.0;
    for (int p = 0; p < N; ++p) phi[p] = U[IA(pb, p) * nc + i];
    for (int q = 0; q < N; ++q) sg = sg + mpo_pf_gprime(phi[q]);
    for (int p = 0; p < N; ++p) {
      const double r = Me2 * (mpo_pf_gprime(phi[p]) - phi[p] * sg);
      R[p * nc + i] = r;
      Rint[p] = Rint[p] + r * vol;
      phint[p] = phint[p] + phi[p] * vol;
      for (int q = 0; q < N; ++q) Wint[p][q] = Wint[p][q] + pf_W(phi, p, q) * vol;
    }
  }

  /* multipliers over the present phases, gauge B_last = 0 */
  int pres[MPO_MAXP], np = 0;
  for (int p = 0; p < N; ++p)
    if (phint[p] > 0.0) pres[np++] = p;
  double B[MPO_MAXP];
  for (int q = 0; q < N; ++q) B[q] = 0.0;
  if (np > 1) {
    const int n = np - 1;
    double A[MPO_MAXP][MPO_MAXP], b[MPO_MAXP];
    for (int a = 0; a < n; ++a) {
      for (int c = 0; c < n; ++c) A[a][c] = Wint[pres[a]][pres[c]];
      b[a] = Rint[pres[a]];
    }
    if (small_solve(n, A, b))
      for (int a = 0; a < n; ++a) B[pres[a]] = b[a];
  }

  /* [div J_p] = M lap(phi_p) - R_p + sum_q W_pq B_q */
  for (long i = 0; i < nc; ++i) {
    long idx[3] = {i % n3[0], (i / n3[0]) % n3[1], i / (n3[0] * n3[1])};
    double phi[MPO_MAXP];
    for (int p = 0; p < N; ++p) phi[p] = U[IA(pb, p) * nc + i];
    for (int p = 0; p < N; ++p) {
      const double *f = U + IA(pb, p) * nc;
      double lap = 0.0;
      for (int d = 0; d < nd; ++d) {
        const long base = i - idx[d] * sx[d];
        const long lo = ghost_index(idx[d] - 1, n3[d], pb->bc[d][0], pb->bc[d][1]);
        const long hi = ghost_index(idx[d] + 1, n3[d], pb->bc[d][0], pb->bc[d][1]);
        const double h2 = pb->dx[d] * pb->dx[d];
        lap = lap + (f[base + hi * sx[d]] - 2.0 * f[i] + f[base + lo * sx[d]]) / h2;
      }
      double Lc = 0.0;
      for (int q = 0; q < N; ++q) Lc = Lc + pf_W(phi, p, q) * B[q];
      divj[p * nc + i] = M * lap - R[p * nc + i] + Lc;
    }
  }
  free(R);
  if (info) {
    info[0] = M;
    info[1] = (double)np;
    for (int q = 0; q < N; ++q) info[2 + q] = B[q];
  }
  return MPO_OK;
}

void mpo_pf_flux(const mpo_problem *pb, int dir, const double *VL,
                 const double *VR, const double *G, const double *kf,
                 double *F) {
  (void)dir;
  const int N = pb->nphase, nd = pb->ndim, nU = mpo_nU(pb);
  const double *mL = VL, *uL = VL + N, PL = VL[N + nd], *aL = VL + N + nd + 1;
  const double *mR = VR, *uR = VR + N, PR = VR[N + nd], *aR = VR + N + nd + 1;
  for (int c = 0; c < nU; ++c) F[c] = 0.0;
  double keL = 0.0, keR = 0.0;
  for (int k = 0; k < nd; ++k) {
    keL = keL + uL[k] * uL[k];
    keR = keR + uR[k] * uR[k];
  }
  keL = 0.5 * keL;
  keR = 0.5 * keR;
  double S = 0.0;
  for (int p = 0; p < N; ++p) {
    const double gm = G[p] < 0.0 ? G[p] : 0.0;
    const double gp = G[p] > 0.0 ? G[p] : 0.0;
    /* donor/receiver product, capped at the face coefficient of Eq. (4) */
    const double bl = aL[p] * (1.0 - aR[p]), br = aR[p] * (1.0 - aL[p]);
    const double sl = bl > kf[p] ? kf[p] / bl : 1.0;
    const double sr = br > kf[p] ? kf[p] / br : 1.0;
    const double dl = gm * (1.0 - aR[p]) * sl;   /* left cell gives  (G < 0) */
    const double dr = gp * (1.0 - aL[p]) * sr;   /* right cell gives (G > 0) */
    const double A = eos_A(pb, p), B = eos_B(pb, p), D = pb->D[p];
    const double fa = dl * aL[p] + dr * aR[p];
    const double fm = dl * mL[p] + dr * mR[p];
    F[IA(pb, p)] = fa;
    F[IM(p)] = fm;
    for (int k = 0; k < nd; ++k)
      F[IMOM(pb, k)] = F[IMOM(pb, k)] + (dl * mL[p] * uL[k] + dr * mR[p] * uR[k]);
    F[IE(pb)] = F[IE(pb)] +
                (dl * (mL[p] * keL + aL[p] * (A * PL + B) + mL[p] * D) +
                 dr * (mR[p] * keR + aR[p] * (A * PR + B) + mR[p] * D));
    S = S + fa;
  }
  /* sum_p J_p = 0 at the face */
  double ub[3] = {0.0, 0.0, 0.0}, keb = 0.0;
  for (int k = 0; k < nd; ++k) {
    ub[k] = 0.5 * (uL[k] + uR[k]);
    keb = keb + ub[k] * ub[k];
  }
  keb = 0.5 * keb;
  const double Pb = 0.5 * (PL + PR);
  for (int p = 0; p < N; ++p) {
    const double ca = 0.5 * (aL[p] + aR[p]) * S;
    const double cm = 0.5 * (mL[p] + mR[p]) * S;
    F[IA(pb, p)] = F[IA(pb, p)] - ca;
    F[IM(p)] = F[IM(p)] - cm;
    for (int k = 0; k < nd; ++k) F[IMOM(pb, k)] = F[IMOM(pb, k)] - cm * ub[k];
    F[IE(pb)] = F[IE(pb)] - (cm * (keb + pb->D[p]) +
                             ca * (eos_A(pb, p) * Pb + eos_B(pb, p)));
  }
}

/* L^PF(U): per direction, WENO-C/CL face states of cells -1..n of every line
 * (the reconstruction of the hyperbolic step), the PF flux at faces
 * -1/2..n-1/2 with the frozen gradient of that face, and
 *   +(F_{i+1/2} - F_{i-1/2}) / dx   (Eq. (5): dU/dt = +div F^PF). */
int mpo_pf_rhs(const mpo_problem *pb, const double *U, const double *G,
               const double *K, double *L) {
  int st = check_problem(pb);
  if (st != MPO_OK) return st;
  const int N = pb->nphase, nU = mpo_nU(pb), nd = pb->ndim;
  const long nc = mpo_ncells(pb);
  long n3[3] = {1, 1, 1};
  for (int d = 0; d < nd; ++d) n3[d] = pb->n[d];
  const long sx[3] = {1, n3[0], n3[0] * n3[1]};
  memset(L, 0, sizeof(double) * (size_t)nU * (size_t)nc);

  for (int dir = 0; dir < nd; ++dir) {
    const long n = n3[dir], s = sx[dir];
    const int o1 = (dir + 1) % 3, o2 = (dir + 2) % 3;
    const long nl = n3[o1] * n3[o2];
    const double dx = pb->dx[dir];
    const int periodic = pb->bc[dir][0] == MPO_BC_PERIODIC;
#pragma omp parallel
    {
      double *UL = malloc(sizeof(double) * (size_t)(n + 2) * nU);
      double *UR = malloc(sizeof(double) * (size_t)(n + 2) * nU);
      double *VL = malloc(sizeof(double) * (size_t)(n + 2) * nU);
      double *VR = malloc(sizeof(double) * (size_t)(n + 2) * nU);
      double *F = malloc(sizeof(double) * (size_t)(n + 1) * nU);
      double Us[5 * (4 * MPO_MAXP + 4)], Gf[MPO_MAXP], kf[MPO_MAXP];
#pragma omp for schedule(static)
      for (long line = 0; line < nl; ++line) {
        const long j1 = line % n3[o1], j2 = line / n3[o1];
        const long base = j1 * sx[o1] + j2 * sx[o2];
        for (long i = -1; i <= n; ++i) {
          for (int j = 0; j < 5; ++j) {
            int flip;
            long g = ghost_index_flip(i - 2 + j, n, pb->bc[dir][0], pb->bc[dir][1], &flip);
            for (int c = 0; c < nU; ++c) Us[j * nU + c] = U[c * nc + base + g * s];
            if (flip) Us[j * nU + IMOM(pb, dir)] = -Us[j * nU + IMOM(pb, dir)];
          }
          mpo_reconstruct_cell(pb, Us, dir, UL + (i + 1) * nU, UR + (i + 1) * nU,
                               VL + (i + 1) * nU, VR + (i + 1) * nU, NULL);
        }
        for (long f = 0; f <= n; ++f) { /* face between cells f-1 and f */
          /* the upper face of cell f-1; face -1/2 is face n-1/2 when periodic
           * and carries no gradient at an outflow end */
          const long owner = f > 0 ? f - 1 : (periodic ? n - 1 : -1);
          const long other = f < n ? f : (periodic ? 0 : -1);
          for (int p = 0; p < N; ++p) {
            Gf[p] = owner >= 0 ? G[(long)(dir * N + p) * nc + base + owner * s] : 0.0;
            kf[p] = (owner >= 0 && other >= 0)
                        ? 0.5 * (K[(long)p * nc + base + owner * s] +
                                 K[(long)p * nc + base + other * s])
                        : 0.0;
          }
          mpo_pf_flux(pb, dir, VL + f * nU, VR + (f + 1) * nU, Gf, kf, F + f * nU);
        }
        for (long i = 0; i < n; ++i) {
          const long cell = base + i * s;
          for (int c = 0; c < nU; ++c)
            L[c * nc + cell] =
                L[c * nc + cell] + (F[(i + 1) * nU + c] - F[i * nU + c]) / dx;
        }
      }
      free(UL); free(UR); free(VL); free(VR); free(F);
    }
  }
  return MPO_OK;
}

int mpo_pf_rk3(const mpo_problem *pb, double *U, const double *G,
               const double *K, double dt) {
  int st = check_problem(pb);
  if (st != MPO_OK) return st;
  const long nt = (long)mpo_nU(pb) * mpo_ncells(pb);
  double *L = malloc(sizeof(double) * (size_t)nt);
  double *U1 = malloc(sizeof(double) * (size_t)nt);
  double *U2 = malloc(sizeof(double) * (size_t)nt);
  if (!L || !U1 || !U2) { free(L); free(U1); free(U2); return MPO_ERR_ARG; }
  mpo_pf_rhs(pb, U, G, K, L);
  for (long k = 0; k < nt; ++k) U1[k] = U[k] + dt * L[k];
  mpo_pf_rhs(pb, U1, G, K, L);
  for (long k = 0; k < nt; ++k)
    U2[k] = 0.75 * U[k] + 0.25 * U1[k] + 0.25 * (dt * L[k]);
  mpo_pf_rhs(pb, U2, G, K, L);
  for (long k = 0; k < nt; ++k)
    U[k] = U[k] / 3.0 + 2.0 * U2[k] / 3.0 + 2.0 * (dt * L[k]) / 3.0;
  free(L); free(U1); free(U2);
  return MPO_OK;
}
