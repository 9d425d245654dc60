/* Drives the oracle's entry points on seeded 1D, 2D and 3D states, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer: any invalid
 * access or undefined operation ends the process with a nonzero status.
 * Test infrastructure (run by tests/test_oracle_sanitize.py). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/mpo.h"

static unsigned long long rng_state = 88172645463325252ULL;
static double urand(void) { /* xorshift64 */
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 7;
  rng_state ^= rng_state << 17;
  return (double)(rng_state >> 11) / 9007199254740992.0;
}

/* a smooth admissible state with random amplitudes: N phases, u, P */
static void fill(const mpo_problem *pb, double *U) {
  const int N = pb->nphase, d = pb->ndim, nU = mpo_nU(pb);
  const long nc = mpo_ncells(pb);
  const double rho[4] = {1.0, 1000.0, 800.0, 2.0};
  double amp = 0.3 * urand(), ph = 6.28 * urand();
  for (long i = 0; i < nc; ++i) {
    double x = (double)i / (double)nc;
    double a[4], s = 0.0;
    for (int p = 0; p < N; ++p) {
      a[p] = 1.0 + (p + 1) * amp * sin(6.283185307 * (p + 1) * x + ph);
      if (a[p] < 0.0) a[p] = 0.0;
      s += a[p];
    }
    double r = 0.0, rhoe = 0.0, u[3], ke = 0.0;
    const double P = 1e5 * (1.0 + 0.5 * sin(12.0 * x));
    for (int k = 0; k < d; ++k) u[k] = 10.0 * sin(3.0 * x + k);
    for (int p = 0; p < N; ++p) {
      a[p] /= s;
      U[(long)p * nc + i] = a[p] * rho[p];
      U[(long)(N + d + 1 + p) * nc + i] = a[p];
      r += a[p] * rho[p];
      rhoe += a[p] * (P + pb->gamma[p] * pb->pinf[p]) / (pb->gamma[p] - 1.0);
    }
    for (int k = 0; k < d; ++k) {
      U[(long)(N + k) * nc + i] = r * u[k];
      ke += 0.5 * r * u[k] * u[k];
    }
    U[(long)(N + d) * nc + i] = rhoe + ke;
  }
  (void)nU;
}

static int run(int ndim, const int n[3], int N, int recon, int flux, int model) {
  mpo_problem pb;
  memset(&pb, 0, sizeof(pb));
  pb.ndim = ndim;
  for (int k = 0; k < 3; ++k) { pb.n[k] = k < ndim ? n[k] : 1; pb.dx[k] = 1.0 / pb.n[k]; }
  for (int k = 0; k < ndim; ++k) { pb.bc[k][0] = k == 0 ? 0 : 1; pb.bc[k][1] = k == 0 ? 0 : 2; }
  pb.nphase = N;
  const double g[4] = {1.4, 6.12, 4.4, 1.6}, pi[4] = {0.0, 3.43e8, 6e8, 0.0};
  for (int p = 0; p < N; ++p) {
    pb.gamma[p] = g[p];
    pb.pinf[p] = pi[p];
    pb.pmin[p] = -pi[p] + 1e-6 * (1e5 + pi[p]);
  }
  pb.recon = recon; pb.flux = flux; pb.model = model; pb.energy_limiter = 1; pb.cfl = 0.2;
  const long nt = (long)mpo_nU(&pb) * mpo_ncells(&pb);
  double *U = malloc(sizeof(double) * nt), *L = malloc(sizeof(double) * nt);
  double diag[64];
  fill(&pb, U);
  int st = mpo_rhs(&pb, U, L);
  double dt = mpo_dt(&pb, U, 0.0);
  st |= mpo_step(&pb, U, dt);
  st |= mpo_diag(&pb, U, diag);
  if (ndim <= 2) {
    const long f = (long)N * mpo_ncells(&pb);
    double *dj = malloc(sizeof(double) * f), info[2 + MPO_MAXP];
    double *G = calloc((size_t)ndim * f, sizeof(double)), *K = malloc(sizeof(double) * f);
    for (long i = 0; i < f; ++i) K[i] = 0.25;
    st |= mpo_pf_divj(&pb, U, 1.0 / n[0], dj, info);
    for (long i = 0; i < (long)ndim * f; ++i) G[i] = 1e-3 * sin((double)i);
    st |= mpo_pf_rhs(&pb, U, G, K, L);
    st |= mpo_pf_rk3(&pb, U, G, K, 1e-9);
    free(dj); free(G); free(K);
  }
  free(U); free(L);
  return st;
}

int main(void) {
  const int n1[3] = {37, 1, 1}, n2[3] = {19, 13, 1}, n3[3] = {9, 8, 7}, n0[3] = {1, 1, 1};
  int st = 0;
  for (int N = 1; N <= 4; ++N)
    for (int recon = 0; recon < 4; ++recon)
      for (int flux = 0; flux < 2; ++flux) {
        st |= run(1, n1, N, recon, flux, flux);
        st |= run(2, n2, N, recon, flux, 1 - flux);
      }
  st |= run(3, n3, 3, 0, 1, 0);
  st |= run(1, n0, 2, 0, 0, 0);
  printf("status %d\n", st);
  return st != 0;
}
