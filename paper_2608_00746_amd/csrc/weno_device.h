// weno_device.h -- per-cell device arithmetic of the WENO-C / WENO-CL scheme
// for gfx950: primitive recovery, WENO5-W weights, the coupled mass/volume-
// fraction reconstruction with its limiter chain, the energy limiter, and the
// HLLC / HLL interface flux with the consistent face velocity.
//
// Everything here works on registers; the kernels in mp_weno.hip decide where
// the five-cell stencils come from (LDS rows or a register window).
//
// Precision policy W: the type of the smoothness indicators and nonlinear
// weights (double on the FP64 path, float on the mixed path).  The combination
// of candidate values, every limiter, the EOS inversion, the V <-> U maps and
// the linear flux assembly stay in double on both paths.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpw {

constexpr int MAXP = 8;

// Per-instance constants.  A_p, B_p of Eq. (26) are formed on the host with
// the same expressions as their definition (A = 1/(gamma-1),
// B = gamma Pinf/(gamma-1)); EB_p = A_p Pmin_p + B_p enters psi (Eq. (9)).
struct Eos {
  double A[MAXP], B[MAXP], Dp[MAXP], gam[MAXP], pinf[MAXP], EB[MAXP];
};

struct Grid {
  int nx, ny, nz;          // cells per direction (1 beyond the dimension)
  int64_t nc;              // cells
  double rdx, rdy, rdz;    // 1/dx, 1/dy, 1/dz
  double hdx, hdy, hdz;    // dx/2, dy/2, dz/2 (slopes of the consistent limiter)
  int bcx0, bcx1, bcy0, bcy1, bcz0, bcz1;
  int recon, flux, model, energy;
  int asrc;                // alpha_p of the source: 0 cell average, 1 / sum alpha
};

// -------------------------------------------------------------------------
// storage types
// -------------------------------------------------------------------------
template <int N, int D>
struct Prim {             // cell-average primitives V = (m, u, P, alpha)
  double m[N], a[N], u[D], P;
};

template <int N, int D>
struct Cons {             // conserved state U = (m, rho u, rho E, alpha)
  double m[N], a[N], mom[D], E;
};

template <int N, int D>
struct Face {             // one reconstructed face state fed to the flux
  double m[N], a[N], mom[D], E;   // conserved
  double u[D], P, rho, c;         // primitives, density, sound speed
};

template <int N, int D>
struct Flux {
  double f[2 * N + D + 1];        // component order of U
  double uh;                      // face velocity
};

template <int N, int D>
__device__ __forceinline__ constexpr int nU() { return 2 * N + D + 1; }

// -------------------------------------------------------------------------
// reciprocals
// -------------------------------------------------------------------------

// Reciprocal: IEEE division in FP64; the hardware reciprocal (1 ulp) in FP32,
// where only the nonlinear weights and wave-speed coefficients use it.
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Reciprocal of a double of magnitude in [2^-1000, 2^1000] without the
// special-case scaling of the IEEE division sequence: the hardware estimate
// refined by two Newton steps (within an ulp or two of 1/x).  Used for
// quotients whose divisor is a physical quantity bounded away from zero and
// overflow (densities, sums of alpha A, wave-speed differences); a quotient
// a * rcp_normal(b) then lies within about two ulps of a / b.
__device__ __forceinline__ double rcp_normal(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp_normal(float x) { return __builtin_amdgcn_rcpf(x); }

// -------------------------------------------------------------------------
// thermodynamics
// -------------------------------------------------------------------------

// Pressure of Eq. (27) and velocity u = (rho u)/rho.  The operation order is
// fixed and contraction is off: the pressure of a stiffened-gas mixture loses
// log10(gamma Pinf / P) digits to cancellation in E - ke - sum alpha B, so
// every implementation that must agree with another to round-off has to
// round the same way there.  The quotients by rho (u and ke) share one
// reciprocal, and the last one (by sum alpha A) is a reciprocal product:
// both lie within about two ulps of the divisions and no cancellation
// follows them.
template <int N, int D>
__device__ __forceinline__ void cons_to_prim(const Cons<N, D>& U, const Eos& e,
                                             Prim<N, D>& V) {
#pragma clang fp contract(off)
  double rho = 0.0;
#pragma unroll
  for (int p = 0; p < N; ++p) rho = rho + U.m[p];
  const double ir = rho > 0.0 ? rcp_normal(rho) : 0.0;
  double mom2 = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    mom2 = mom2 + U.mom[k] * U.mom[k];
    V.u[k] = U.mom[k] * ir;
  }
  const double ke = 0.5 * mom2 * ir;
  double sA = 0.0, sB = 0.0, sD = 0.0;
#pragma unroll
  for (int p = 0; p < N; ++p) {
    sA = sA + e.A[p] * U.a[p];
    sB = sB + e.B[p] * U.a[p];
    sD = sD + e.Dp[p] * U.m[p];
    V.m[p] = U.m[p];
    V.a[p] = U.a[p];
  }
  V.P = (U.E - ke - sB - sD) * rcp_normal(sA);
}

// Mixture rho c^2 (Eq. (2) with the EOS of Eq. (26)) as a quotient
// num / den: Allaire sum A a gamma (P + Pinf) / sum A a; Kapila (Wood)
// sum a / sum a/(gamma(P+Pinf)).  num = 0 stands for a value that is not
// positive (no NaN from strong tension).
template <int N>
__device__ __forceinline__ void mix_rc2_parts(const double* a, double P, const Eos& e,
                                              int model, double& num, double& den) {
  num = 0.0;
  den = 0.0;
  if (model == 1) {
    double s = 0.0, sa = 0.0;
#pragma unroll
    for (int p = 0; p < N; ++p) {
      if (a[p] != 0.0) {
        const double k = e.gam[p] * (P + e.pinf[p]);
        if (!(k > 0.0)) return;
        s += a[p] / k;
        sa += a[p];
      }
    }
    if (s > 0.0) { num = sa; den = s; }
    return;
  }
#pragma unroll
  for (int p = 0; p < N; ++p) {
    const double Aa = e.A[p] * a[p];
    num += Aa * (e.gam[p] * (P + e.pinf[p]));
    den += Aa;
  }
  if (!(num > 0.0)) num = 0.0;
}

template <int N>
__device__ __forceinline__ double mix_rc2(const double* a, double P,
                                          const Eos& e, int model) {
  double num, den;
  mix_rc2_parts<N>(a, P, e, model, num, den);
  return num > 0.0 ? num / den : 0.0;
}

// c = sqrt(rho c^2 / rho) = sqrt(num / (den rho)) with one reciprocal; 0 when
// rho c^2 or rho is not positive.
__device__ __forceinline__ double sound_speed(double num, double den, double rho) {
  return (num > 0.0 && rho > 0.0) ? sqrt(num * rcp_normal(den * rho)) : 0.0;
}

// psi(U) of Eq. (9) with m_p e_p(Pmin_p, rho_p) = alpha_p EB_p + m_p D_p.
template <int N, int D>
__device__ __forceinline__ double psi(const double* m, const double* a,
                                      const double* mom, double E,
                                      const Eos& e) {
  double rho = 0.0, mom2 = 0.0, emin = 0.0;
#pragma unroll
  for (int p = 0; p < N; ++p) {
    rho += m[p];
    emin += a[p] * e.EB[p] + m[p] * e.Dp[p];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) mom2 += mom[k] * mom[k];
  const double ke = rho > 0.0 ? 0.5 * mom2 * rcp_normal(rho) : 0.0;
  return E - ke - emin;
}


// -------------------------------------------------------------------------
// WENO5 with the relative-smoothness weights (Sec. 3.1, 3.3)
// -------------------------------------------------------------------------

// Stencil differences relative to the centre: a = q_{i-2} - q_i,
// b = q_{i-1} - q_i, c = q_{i+1} - q_i, e = q_{i+2} - q_i.  Every quantity
// below is written with them, so constant (sub-)stencils give exact zeros.
struct Diff {
  double a, b, c, e;
};

__device__ __forceinline__ Diff diffs(double q0, double q1, double q2,
                                      double q3, double q4) {
  return Diff{q0 - q2, q1 - q2, q3 - q2, q4 - q2};
}

// Jiang-Shu indicators of the sub-stencils {i-2..i}, {i-1..i+1}, {i..i+2}.
template <typename W>
__device__ __forceinline__ void beta3(const Diff& d, W b[3]) {
  const W c13 = W(13.0 / 12.0);
  W x, y;
  x = W(d.a - 2.0 * d.b);
  y = W(d.a - 4.0 * d.b);
  b[0] = c13 * x * x + W(0.25) * y * y;
  x = W(d.b + d.c);
  y = W(d.b - d.c);
  b[1] = c13 * x * x + W(0.25) * y * y;
  x = W(d.e - 2.0 * d.c);
  y = W(d.e - 4.0 * d.c);
  b[2] = c13 * x * x + W(0.25) * y * y;
}

// Candidate increments f^(s) - fbar at x_{i+1/2} (l) and x_{i-1/2} (r).
__device__ __forceinline__ void increments(const Diff& d, double l[3],
                                           double r[3]) {
  const double s6 = 1.0 / 6.0;
  l[0] = (2.0 * d.a - 7.0 * d.b) * s6;
  l[1] = (2.0 * d.c - d.b) * s6;
  l[2] = (5.0 * d.c - d.e) * s6;
  r[0] = (5.0 * d.b - d.a) * s6;
  r[1] = (2.0 * d.b - d.c) * s6;
  r[2] = (2.0 * d.e - 7.0 * d.c) * s6;
}

// Weights of Eq. (15) for both faces.  With all indicators positive,
// w_s = d_s / (d_s + sum_{k!=s} d_k (b_s/b_k)^2) equals
// d_s prod_{k!=s} b_k^2 / sum_j d_j prod_{k!=j} b_k^2, which needs one
// division per face instead of nine; indicators are first scaled by their
// maximum so that the products cannot overflow.  Zero indicators follow the
// definition: a zero b_k with b_s > 0 gives w_s = 0, and stencils with
// b = 0 share the weight in the ratio of their d (IS^(s,k) = 1).
template <typename W>
__device__ __forceinline__ void wenow_weights(const W bin[3], W wl[3], W wr[3]) {
  W b[3] = {bin[0], bin[1], bin[2]};
  W bm = fmax(b[0], fmax(b[1], b[2]));
  if (!(bm > W(0))) {             // every stencil equally smooth
    wl[0] = W(0.1); wl[1] = W(0.6); wl[2] = W(0.3);
    wr[0] = W(0.3); wr[1] = W(0.6); wr[2] = W(0.1);
    return;
  }
  // Scale the set so that its largest member lies in [1/2, 1): an exact
  // power of two (FP64), which leaves every ratio unchanged and needs no
  // division; the hardware reciprocal of the maximum (FP32, after an exact
  // power-of-two lift of sets below 2^-100).
  constexpr bool DBL = sizeof(W) == 8;
  W s0, s1, s2;
  if constexpr (DBL) {
    int e;
    (void)frexp(bm, &e);
    s0 = ldexp(b[0], -e); s1 = ldexp(b[1], -e); s2 = ldexp(b[2], -e);
  } else {
    if (bm < W(0x1p-100)) {
      const W up = W(0x1p80);
      b[0] *= up; b[1] *= up; b[2] *= up; bm *= up;
    }
    const W r = rcp(bm);
    s0 = b[0] * r; s1 = b[1] * r; s2 = b[2] * r;
  }
  // Scaled indicators below tau join the zero set: this keeps every product
  // below (and the reciprocal of their sum) inside the normal range; the
  // face value moves by at most the spread of those candidates, which is
  // O(tau) relative to the stencil's variation.
  const W tau = DBL ? W(1e-70) : W(1e-8);
  s0 = s0 < tau ? W(0) : s0;
  s1 = s1 < tau ? W(0) : s1;
  s2 = s2 < tau ? W(0) : s2;
  s0 *= s0; s1 *= s1; s2 *= s2;
  const W p0 = s1 * s2, p1 = s0 * s2, p2 = s0 * s1;
  const W l0 = W(0.1) * p0, l1 = W(0.6) * p1, l2 = W(0.3) * p2;
  const W r0 = W(0.3) * p0, r1 = W(0.6) * p1, r2 = W(0.1) * p2;
  const W dl = l0 + l1 + l2, dr = r0 + r1 + r2;
  if (dl > W(0)) {
    // dl, dr >= 1e-281 (every nonzero scaled indicator is >= tau)
    const W il = rcp_normal(dl), ir = rcp_normal(dr);
    wl[0] = l0 * il; wl[1] = l1 * il; wl[2] = l2 * il;
    wr[0] = r0 * ir; wr[1] = r1 * ir; wr[2] = r2 * ir;
  } else {
    // at least two scaled indicators vanished: they form the zero set
    const W z0 = s0 == W(0) ? W(1) : W(0), z1 = s1 == W(0) ? W(1) : W(0),
            z2 = s2 == W(0) ? W(1) : W(0);
    const W il = W(1) / (W(0.1) * z0 + W(0.6) * z1 + W(0.3) * z2);
    const W ir = W(1) / (W(0.3) * z0 + W(0.6) * z1 + W(0.1) * z2);
    wl[0] = W(0.1) * z0 * il; wl[1] = W(0.6) * z1 * il; wl[2] = W(0.3) * z2 * il;
    wr[0] = W(0.3) * z0 * ir; wr[1] = W(0.6) * z1 * ir; wr[2] = W(0.1) * z2 * ir;
  }
}

// WENO-JS weights, Eq. (12) with three stencils and epsilon = 1e-6 (the
// comparison scheme of Sec. 3.2 only).
__device__ __forceinline__ void wenojs_weights(const double b[3], double wl[3], double wr[3]) {
  const double eps = 1e-6;
  double q[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double t = b[k] + eps;
    q[k] = 1.0 / (t * t);
  }
  const double l0 = 0.1 * q[0], l1 = 0.6 * q[1], l2 = 0.3 * q[2];
  const double r0 = 0.3 * q[0], r1 = 0.6 * q[1], r2 = 0.1 * q[2];
  const double sl = l0 + l1 + l2, sr = r0 + r1 + r2;
  wl[0] = l0 / sl; wl[1] = l1 / sl; wl[2] = l2 / sl;
  wr[0] = r0 / sr; wr[1] = r1 / sr; wr[2] = r2 / sr;
}

// Comparison schemes (Sec. 3.2, 3.3): one primitive variable reconstructed
// with its own weights, Eq. (12) (js) or Eq. (15), as the weighted candidate
// sum of Eqs. (10), (13); FP64.
__device__ __forceinline__ void plain_weno(double q0, double q1, double q2, double q3,
                                           double q4, bool js, double& fl, double& fr) {
  const Diff df = diffs(q0, q1, q2, q3, q4);
  double b[3], wl[3], wr[3];
  beta3<double>(df, b);
  if (js) wenojs_weights(b, wl, wr);
  else wenow_weights<double>(b, wl, wr);
  const double s6 = 1.0 / 6.0;
  const double cl0 = (2.0 * q0 - 7.0 * q1 + 11.0 * q2) * s6;
  const double cl1 = (-q1 + 5.0 * q2 + 2.0 * q3) * s6;
  const double cl2 = (2.0 * q2 + 5.0 * q3 - q4) * s6;
  const double cr0 = (-q0 + 5.0 * q1 + 2.0 * q2) * s6;
  const double cr1 = (2.0 * q1 + 5.0 * q2 - q3) * s6;
  const double cr2 = (11.0 * q2 - 7.0 * q3 + 2.0 * q4) * s6;
  fl = wl[0] * cl0 + wl[1] * cl1 + wl[2] * cl2;
  fr = wr[0] * cr0 + wr[1] * cr1 + wr[2] * cr2;
}

// Face values of Eq. (10): fbar + sum_s w_s (f^(s) - fbar) (equal to the
// weighted candidate sum since the weights sum to one, and exact on constant
// data).  FP64 weights and sums on the FP64 path; on the mixed path the u and
// P increments are rounded to FP32 and summed there, while m_p and alpha_p
// keep double increments and sums with the FP32 weights (Eq. (16) consistency
// needs the same arithmetic for both).
template <typename W, bool F32SUM>
__device__ __forceinline__ void combine(double q2, const double l[3],
                                        const double r[3], const W wl[3],
                                        const W wr[3], double& fl,
                                        double& fr) {
  if constexpr (F32SUM) {
    fl = q2 + double(wl[0] * float(l[0]) + wl[1] * float(l[1]) + wl[2] * float(l[2]));
    fr = q2 + double(wr[0] * float(r[0]) + wr[1] * float(r[1]) + wr[2] * float(r[2]));
  } else {
    fl = q2 + (double(wl[0]) * l[0] + double(wl[1]) * l[1] + double(wl[2]) * l[2]);
    fr = q2 + (double(wr[0]) * r[0] + double(wr[1]) * r[1] + double(wr[2]) * r[2]);
  }
}

// -------------------------------------------------------------------------
// limiters (Sec. 3.4)
// -------------------------------------------------------------------------

// f^C of Eq. (6) inverted with the four-point Gauss-Lobatto end weights 1/12.
__device__ __forceinline__ double interior(double fb, double fl, double fr) {
  return (fb - (fl + fr) * (1.0 / 12.0)) * 1.2;
}

// Eq. (18) with lower bound 0: 1 when min(f^C, f^L, f^R) >= 0, else
// fbar / (fbar - min) clamped to [0, 1].
__device__ __forceinline__ double theta_pos(double fb, double fc, double fl,
                                            double fr) {
  const double mu = fmin(fc, fmin(fl, fr));
  if (mu >= 0.0) return 1.0;
  const double den = fb - mu;
  if (!(den > 0.0)) return 0.0;
  const double t = fb / den;
  return t > 1.0 ? 1.0 : (t > 0.0 ? t : 0.0);
}

// theta_p of Eq. (17): min over the mass and volume-fraction limiters.
__device__ __forceinline__ double theta_phase(double mb, double ml, double mr,
                                              double ab, double al,
                                              double ar) {
  const double tm = theta_pos(mb, interior(mb, ml, mr), ml, mr);
  const double ta = theta_pos(ab, interior(ab, al, ar), al, ar);
  return fmin(tm, ta);
}

// Consistent limiter of Eqs. (23)-(25) at one face.  S: alpha slopes.  The
// phase with the largest |S| (lowest index on ties) takes S_hat / S_phat, the
// others S_phat / S_hat, both clamped to [0, 1]; all 1 when S_phat = 0 and
// the others 1 when S_hat = 0.
template <int N>
__device__ __forceinline__ void consistent_limiter(const double* S,
                                                   double* th) {
  int ph = 0;
  double amax = fabs(S[0]);
#pragma unroll
  for (int p = 1; p < N; ++p)
    if (fabs(S[p]) > amax) { amax = fabs(S[p]); ph = p; }
  double sph = 0.0, sum = 0.0;
#pragma unroll
  for (int p = 0; p < N; ++p) {
    sum += S[p];
    if (p == ph) sph = S[p];
  }
  if (sph == 0.0) {
#pragma unroll
    for (int p = 0; p < N; ++p) th[p] = 1.0;
    return;
  }
  const double shat = sph - sum;
  const double tp = shat / sph;
  const double to = shat == 0.0 ? 1.0 : sph / shat;
#pragma unroll
  for (int p = 0; p < N; ++p) {
    const double t = (p == ph) ? tp : to;
    th[p] = t > 1.0 ? 1.0 : (t > 0.0 ? t : 0.0);
  }
}

// -------------------------------------------------------------------------
// reconstruction of one cell along one direction
// -------------------------------------------------------------------------
// st(c, j): component c of the primitive averages of cell i-2+j (j = 0..4)
// along the direction, in the order m_1..m_N, alpha_1..alpha_N, u_1..u_D,
// P (read where it is used, from the caller's LDS rows, so that the stencil
// never sits in registers as a whole); ub: conserved average of cell i.  Outputs: fm = U^R_{i-1/2} (the cell's
// face on the minus side), fp = U^L_{i+1/2} (plus side), each with its face
// primitives, density and sound speed.  hdx = dx/2 of the direction.
// RS: the reconstructions compiled in: kReconC (WENO-C and WENO-CL, chosen
// by g.recon), kReconCmp (the comparison schemes WENO-JS and WENO-W) or
// kReconAny (all four, chosen at run time).  Keeping the comparison schemes
// out of the WENO-C kernels keeps their register use, and so their
// occupancy, what the method alone needs.
constexpr int kReconC = 0, kReconCmp = 1, kReconAny = 2;

template <int N, int D, typename W, int RS, typename S>
__device__ __forceinline__ void reconstruct(const S& st,
                                            const Cons<N, D>& ub,
                                            const Eos& e, const Grid& g,
                                            double hdx, Face<N, D>& fm,
                                            Face<N, D>& fp) {
  constexpr bool MIXED = sizeof(W) == 4;
  const bool cmp = RS == kReconCmp || (RS == kReconAny && g.recon >= 2);
  if (cmp) {
    // comparison schemes: every primitive with its own weights, no limiter
    const bool js = g.recon == 2;
#pragma unroll
    for (int p = 0; p < N; ++p) {
      plain_weno(st(p, 0), st(p, 1), st(p, 2), st(p, 3), st(p, 4), js, fp.m[p], fm.m[p]);
      plain_weno(st(N + p, 0), st(N + p, 1), st(N + p, 2), st(N + p, 3), st(N + p, 4), js,
                 fp.a[p], fm.a[p]);
    }
#pragma unroll
    for (int k = 0; k <= D; ++k) {
      const int c = 2 * N + k;
      double vl, vr;
      plain_weno(st(c, 0), st(c, 1), st(c, 2), st(c, 3), st(c, 4), js, vl, vr);
      if (k < D) { fp.u[k] = vl; fm.u[k] = vr; }
      else { fp.P = vl; fm.P = vr; }
    }
  } else {
  // u and P: WENO5-W on each primitive (Sec. 3.4)
#pragma unroll
  for (int k = 0; k <= D; ++k) {
    const int c = 2 * N + k;                 // u_k, then P
    const double q2 = st(c, 2);
    const Diff df = diffs(st(c, 0), st(c, 1), q2, st(c, 3), st(c, 4));
    W b[3], wl[3], wr[3];
    beta3<W>(df, b);
    wenow_weights<W>(b, wl, wr);
    double il[3], ir[3];
    increments(df, il, ir);
    double vl, vr;
    combine<W, MIXED>(q2, il, ir, wl, wr, vl, vr);
    if (k < D) { fp.u[k] = vl; fm.u[k] = vr; }
    else { fp.P = vl; fm.P = vr; }
  }

  // Step 1, Eq. (16): weights of m_p applied to m_p and alpha_p
  double mb[N], ab[N];
#pragma unroll
  for (int p = 0; p < N; ++p) {
    mb[p] = st(p, 2);
    ab[p] = st(N + p, 2);
    const Diff dm = diffs(st(p, 0), st(p, 1), mb[p], st(p, 3), st(p, 4));
    const Diff da = diffs(st(N + p, 0), st(N + p, 1), ab[p], st(N + p, 3), st(N + p, 4));
    W b[3], wl[3], wr[3];
    beta3<W>(dm, b);
    wenow_weights<W>(b, wl, wr);
    double il[3], ir[3];
    increments(dm, il, ir);
    combine<W, false>(mb[p], il, ir, wl, wr, fp.m[p], fm.m[p]);
    increments(da, il, ir);
    combine<W, false>(ab[p], il, ir, wl, wr, fp.a[p], fm.a[p]);
  }

  // Step 2, Eqs. (17)-(18): one theta_p for m_p and alpha_p
#pragma unroll
  for (int p = 0; p < N; ++p) {
    const double th = theta_phase(mb[p], fp.m[p], fm.m[p], ab[p], fp.a[p], fm.a[p]);
    if (th < 1.0) {
      fp.m[p] = mb[p] + th * (fp.m[p] - mb[p]);
      fm.m[p] = mb[p] + th * (fm.m[p] - mb[p]);
      fp.a[p] = ab[p] + th * (fp.a[p] - ab[p]);
      fm.a[p] = ab[p] + th * (fm.a[p] - ab[p]);
    }
  }

  if (g.recon == 1) {
    // WENO-CL, Eqs. (23)-(25), on each face
    const double rh = 1.0 / hdx;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      Face<N, D>& f = side == 0 ? fp : fm;
      double Sa[N], Sm[N], th[N];
#pragma unroll
      for (int p = 0; p < N; ++p) {
        Sa[p] = (f.a[p] - ab[p]) * rh;
        Sm[p] = (f.m[p] - mb[p]) * rh;
      }
      consistent_limiter<N>(Sa, th);
#pragma unroll
      for (int p = 0; p < N; ++p) {
        f.m[p] = mb[p] + th[p] * Sm[p] * hdx;
        f.a[p] = ab[p] + th[p] * Sa[p] * hdx;
      }
    }
  } else {
    // WENO-C, Eq. (19): divide by the face sums; S <= 0 falls back to first
    // order for the cell
    double sl = 0.0, sr = 0.0;
#pragma unroll
    for (int p = 0; p < N; ++p) { sl += fp.a[p]; sr += fm.a[p]; }
    if (sl > 0.0 && sr > 0.0) {
      const double il = rcp_normal(sl), ir = rcp_normal(sr);
#pragma unroll
      for (int p = 0; p < N; ++p) {
        fp.m[p] *= il; fp.a[p] *= il;
        fm.m[p] *= ir; fm.a[p] *= ir;
      }
    } else {
#pragma unroll
      for (int p = 0; p < N; ++p) {
        fp.m[p] = fm.m[p] = mb[p];
        fp.a[p] = fm.a[p] = ab[p];
      }
    }
  }

  // Step 4, Eq. (20): theta_i = min_p theta_p recomputed, applied to all
  double thi = 1.0;
#pragma unroll
  for (int p = 0; p < N; ++p)
    thi = fmin(thi, theta_phase(mb[p], fp.m[p], fm.m[p], ab[p], fp.a[p], fm.a[p]));
#pragma unroll
  for (int p = 0; p < N; ++p) {
    if (thi < 1.0) {
      fp.m[p] = mb[p] + thi * (fp.m[p] - mb[p]);
      fm.m[p] = mb[p] + thi * (fm.m[p] - mb[p]);
      fp.a[p] = ab[p] + thi * (fp.a[p] - ab[p]);
      fm.a[p] = ab[p] + thi * (fm.a[p] - ab[p]);
    }
    // the limited minimum lands at 0 up to rounding: clamp to the box
    fp.m[p] = fmax(fp.m[p], 0.0);
    fm.m[p] = fmax(fm.m[p], 0.0);
    fp.a[p] = fmin(fmax(fp.a[p], 0.0), 1.0);
    fm.a[p] = fmin(fmax(fm.a[p], 0.0), 1.0);
  }

  }  // WENO-C / WENO-CL

  // Step 5: U^{L,R} = psi_{V->U}(V^{L,R})
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    Face<N, D>& f = side == 0 ? fp : fm;
    double rho = 0.0, rhoe = 0.0, u2 = 0.0;
#pragma unroll
    for (int p = 0; p < N; ++p) {
      rho += f.m[p];
      rhoe += f.a[p] * (e.A[p] * f.P + e.B[p]) + f.m[p] * e.Dp[p];
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
      f.mom[k] = rho * f.u[k];
      u2 += f.u[k] * f.u[k];
    }
    f.E = 0.5 * rho * u2 + rhoe;
    f.rho = rho;
  }

  if (g.energy && !cmp) {
    // Eq. (21): one theta^psi from psi at Ubar, U^L, U^R and U^C
    double cm[N], ca[N], cmom[D];
#pragma unroll
    for (int p = 0; p < N; ++p) {
      cm[p] = interior(ub.m[p], fp.m[p], fm.m[p]);
      ca[p] = interior(ub.a[p], fp.a[p], fm.a[p]);
    }
#pragma unroll
    for (int k = 0; k < D; ++k) cmom[k] = interior(ub.mom[k], fp.mom[k], fm.mom[k]);
    const double cE = interior(ub.E, fp.E, fm.E);
    const double pb = psi<N, D>(ub.m, ub.a, ub.mom, ub.E, e);
    const double pc = psi<N, D>(cm, ca, cmom, cE, e);
    const double pl = psi<N, D>(fp.m, fp.a, fp.mom, fp.E, e);
    const double pr = psi<N, D>(fm.m, fm.a, fm.mom, fm.E, e);
    const double tps = theta_pos(pb, pc, pl, pr);
    if (tps < 1.0) {
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        Face<N, D>& f = side == 0 ? fp : fm;
        Cons<N, D> c;
#pragma unroll
        for (int p = 0; p < N; ++p) {
          c.m[p] = f.m[p] = ub.m[p] + tps * (f.m[p] - ub.m[p]);
          c.a[p] = f.a[p] = ub.a[p] + tps * (f.a[p] - ub.a[p]);
        }
#pragma unroll
        for (int k = 0; k < D; ++k) c.mom[k] = f.mom[k] = ub.mom[k] + tps * (f.mom[k] - ub.mom[k]);
        c.E = f.E = ub.E + tps * (f.E - ub.E);
        // face primitives of the limited state (Eq. (27))
        Prim<N, D> v;
        cons_to_prim<N, D>(c, e, v);
        double rho = 0.0;
#pragma unroll
        for (int p = 0; p < N; ++p) rho += f.m[p];
        f.rho = rho;
#pragma unroll
        for (int k = 0; k < D; ++k) f.u[k] = v.u[k];
        f.P = v.P;
      }
    }
  }

  // sound speeds at both faces (FP32 on the mixed path: they only set the
  // wave-speed estimates of the flux)
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    Face<N, D>& f = side == 0 ? fp : fm;
    double num, den;
    mix_rc2_parts<N>(f.a, f.P, e, g.model, num, den);
    if constexpr (MIXED) {
      const float rho = float(f.rho);
      f.c = (num > 0.0 && rho > 0.f)
                ? double(__builtin_sqrtf(float(num) * rcp(float(den) * rho))) : 0.0;
    } else {
      f.c = sound_speed(num, den, f.rho);
    }
  }
}

// -------------------------------------------------------------------------
// numerical flux (Sec. 2.2.1; HLLC Sec. 4.1, HLL Sec. 4.2)
// -------------------------------------------------------------------------
// L: state on the minus side of the face (U^L), R: plus side (U^R); dir: the
// normal direction.  Davis wave speeds; HLLC star states scale m_p and
// alpha_p by the same chi_K, so the mass and volume-fraction fluxes are the
// same linear map of their face values; uhat is the alpha flux with
// alpha = 1 on both sides.
template <int N, int D, typename W = double>
__device__ __forceinline__ void riemann(const Face<N, D>& L,
                                        const Face<N, D>& R, int dir,
                                        int kind, Flux<N, D>& F) {
  constexpr bool MIXED = sizeof(W) == 4;
  const double uL = L.u[dir], uR = R.u[dir];
  double SL, SR;
  if constexpr (MIXED) {
    const float fuL = float(uL), fuR = float(uR), fcL = float(L.c), fcR = float(R.c);
    SL = double(fminf(fuL - fcL, fuR - fcR));
    SR = double(fmaxf(fuL + fcL, fuR + fcR));
  } else {
    SL = fmin(uL - L.c, uR - R.c);
    SR = fmax(uL + L.c, uR + R.c);
  }
  constexpr int NE = N + D;

  auto phys = [&](const Face<N, D>& S, double* f) {
    const double un = S.u[dir];
#pragma unroll
    for (int p = 0; p < N; ++p) {
      f[p] = S.m[p] * un;
      f[NE + 1 + p] = S.a[p] * un;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) f[N + k] = S.mom[k] * un + (k == dir ? S.P : 0.0);
    f[NE] = un * (S.E + S.P);
  };

  if (SL >= 0.0) {
    phys(L, F.f);
    F.uh = uL;
    return;
  }
  if (SR <= 0.0) {
    phys(R, F.f);
    F.uh = uR;
    return;
  }
  if (kind == 1) {  // HLL
    double fl[nU<N, D>()], fr[nU<N, D>()];
    phys(L, fl);
    phys(R, fr);
    double cl, cr, clr;
    if constexpr (MIXED) {
      // FP32 coefficients with c_R := 1 - c_L formed in FP64 (exact for an
      // FP32 c_L in [0, 1]): c_L + c_R = 1 holds exactly at every face, so a
      // uniform velocity and pressure stay uniform
      const float fSL = float(SL), fSR = float(SR);
      const float inv = rcp(fSR - fSL);
      cl = double(fSR * inv);
      cr = 1.0 - cl;
      clr = double(fSL * fSR * inv);
    } else {
      const double inv = rcp_normal(SR - SL);
      cl = SR * inv;
      cr = -SL * inv;
      clr = SL * SR * inv;
    }
#pragma unroll
    for (int p = 0; p < N; ++p) {
      F.f[p] = cl * fl[p] + cr * fr[p] + clr * (R.m[p] - L.m[p]);
      F.f[NE + 1 + p] = cl * fl[NE + 1 + p] + cr * fr[NE + 1 + p] + clr * (R.a[p] - L.a[p]);
    }
#pragma unroll
    for (int k = 0; k < D; ++k)
      F.f[N + k] = cl * fl[N + k] + cr * fr[N + k] + clr * (R.mom[k] - L.mom[k]);
    F.f[NE] = cl * fl[NE] + cr * fr[NE] + clr * (R.E - L.E);
    F.uh = cl * uL + cr * uR;
    return;
  }
  // HLLC
  const double sL = L.rho * (SL - uL), sR = R.rho * (SR - uR);
  // star region (SL < 0 < SR): sL < 0 < sR and SK - uK, SK - Ss are nonzero
  const double Ss = (R.P - L.P + uL * sL - uR * sR) * rcp_normal(sL - sR);
  const bool left = Ss >= 0.0;
  const Face<N, D>& K = left ? L : R;
  const double SK = left ? SL : SR, uK = K.u[dir];
  const double chi = (SK - uK) * rcp_normal(SK - Ss);
  double fk[nU<N, D>()];
  phys(K, fk);
#pragma unroll
  for (int p = 0; p < N; ++p) {
    F.f[p] = fk[p] + SK * (chi * K.m[p] - K.m[p]);
    F.f[NE + 1 + p] = fk[NE + 1 + p] + SK * (chi * K.a[p] - K.a[p]);
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double ms = chi * K.rho * (k == dir ? Ss : K.u[k]);
    F.f[N + k] = fk[N + k] + SK * (ms - K.mom[k]);
  }
  const double Es = chi * (K.E + (Ss - uK) * (K.rho * Ss + K.P * rcp_normal(SK - uK)));
  F.f[NE] = fk[NE] + SK * (Es - K.E);
  F.uh = chi * Ss;
}

// -------------------------------------------------------------------------
// Phase-Field flux (Eq. (5); F^PF of Eq. (1))
// -------------------------------------------------------------------------
// Bound-preserving donor/receiver form across one face, from the face states
// L (the upper face of the lower cell) and R, and the gradients G_p = dQ_p/dx
// at the face:  the volume flux of phase p is
//   min(G_p,0) alpha_p^L (1 - alpha_p^R) + max(G_p,0) alpha_p^R (1 - alpha_p^L)
// (the giving side needs the phase, the taking side needs room); the mass
// flux uses m_p as the donor factor, momentum and energy are carried with the
// donor's u and (|u|^2/2, A_p P + B_p, D_p).  The donor/receiver product is
// capped at the face coefficient kf_p of Eq. (4), so the flux never exceeds
// the k_f |dQ/dx| that equation delivers.  The phase sum S of the volume
// fluxes is then removed in proportion to the face-average alpha_p (mass in
// proportion to the face-average m_p, with the face-average u and P), which
// makes sum_p F^alpha_p vanish at every face.
template <int N, int D>
__device__ __forceinline__ void pf_flux(const Face<N, D>& L, const Face<N, D>& R,
                                        const double* G, const double* kf, const Eos& e,
                                        Flux<N, D>& F) {
  constexpr int NE = N + D;
#pragma unroll
  for (int c = 0; c < 2 * N + D + 1; ++c) F.f[c] = 0.0;
  double keL = 0.0, keR = 0.0, keb = 0.0, ub[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    keL += L.u[k] * L.u[k];
    keR += R.u[k] * R.u[k];
    ub[k] = 0.5 * (L.u[k] + R.u[k]);
    keb += ub[k] * ub[k];
  }
  keL *= 0.5;
  keR *= 0.5;
  keb *= 0.5;
  const double Pb = 0.5 * (L.P + R.P);
  double S = 0.0;
#pragma unroll
  for (int p = 0; p < N; ++p) {
    const double bl = L.a[p] * (1.0 - R.a[p]), br = R.a[p] * (1.0 - L.a[p]);
    const double sl = bl > kf[p] ? kf[p] / bl : 1.0;
    const double sr = br > kf[p] ? kf[p] / br : 1.0;
    const double dl = fmin(G[p], 0.0) * (1.0 - R.a[p]) * sl;   // lower side gives
    const double dr = fmax(G[p], 0.0) * (1.0 - L.a[p]) * sr;   // upper side gives
    const double fa = dl * L.a[p] + dr * R.a[p];
    const double fm = dl * L.m[p] + dr * R.m[p];
    F.f[NE + 1 + p] = fa;
    F.f[p] = fm;
#pragma unroll
    for (int k = 0; k < D; ++k) F.f[N + k] += dl * L.m[p] * L.u[k] + dr * R.m[p] * R.u[k];
    F.f[NE] += dl * (L.m[p] * keL + L.a[p] * (e.A[p] * L.P + e.B[p]) + L.m[p] * e.Dp[p]) +
               dr * (R.m[p] * keR + R.a[p] * (e.A[p] * R.P + e.B[p]) + R.m[p] * e.Dp[p]);
    S += fa;
  }
#pragma unroll
  for (int p = 0; p < N; ++p) {
    const double ca = 0.5 * (L.a[p] + R.a[p]) * S;
    const double cm = 0.5 * (L.m[p] + R.m[p]) * S;
    F.f[NE + 1 + p] -= ca;
    F.f[p] -= cm;
#pragma unroll
    for (int k = 0; k < D; ++k) F.f[N + k] -= cm * ub[k];
    F.f[NE] -= cm * (keb + e.Dp[p]) + ca * (e.A[p] * Pb + e.B[p]);
  }
  F.uh = 0.0;
}

}  // namespace mpw
