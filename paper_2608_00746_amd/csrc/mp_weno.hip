// mp_weno.hip -- kernels, host runtime and C ABI of the MI355X WENO-C / WENO-CL
// hyperbolic step (declared in include/mp_weno.h).
//
// One RK stage of a 2D instance is two launches:
//   k_sweep_x : one workgroup per (row, 254-cell strip).  Each lane converts
//               one cell to primitives into an LDS row, reconstructs its cell
//               along x from the five LDS neighbours, trades its minus-side
//               face state with the left neighbour through LDS, computes the
//               flux of its plus-side face, trades fluxes, and writes the x
//               part of L(U) to a direction accumulator (1D: finishes the RK
//               stage directly).
//   k_sweep_y : the same exchange pattern on 16 x 16 tiles of lanes (one
//               cell per lane, neighbours in y through LDS, 128-byte row
//               segments); it adds the accumulator and applies the RK stage.
// Both sweeps read the same stage state (unsplit, dimension by dimension).
// The CFL step and the diagnostics are two-pass reductions with a fixed
// order (no floating-point atomics), so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mp_weno.h"
#include "weno_device.h"

namespace mpw {

constexpr int kMaxN = 5;          // phases built
constexpr int kBX = 256;          // lanes of the x sweep (254 output cells)
constexpr int kRedBlock = 256;    // reduction workgroup
constexpr int kRedMaxBlocks = 1024;
constexpr int kDiagSlots = 32;    // per-block partials of the diagnostics

struct StageArgs {
  const double* Uk;   // stage state (stencils)
  const double* Un;   // state at the start of the step (RK base)
  double* out;        // U^(k+1), or L(U) when mode == 0
  double* acc;        // x part of L (2D)
  const double* dt;   // device time step of this instance
  double a, b;        // out = a Un + b (Uk + dt L)
  int mode;           // 0: write L, 1: RK stage
};

__device__ __forceinline__ int bc_map(int i, int n, int lo, int hi) {
  if (i < 0) return lo == MP_BC_PERIODIC ? ((i % n) + n) % n : 0;
  if (i >= n) return hi == MP_BC_PERIODIC ? i % n : n - 1;
  return i;
}

template <int N, int D>
__device__ __forceinline__ void load_cons(const double* __restrict__ U,
                                          int64_t nc, int64_t idx,
                                          Cons<N, D>& c) {
#pragma unroll
  for (int p = 0; p < N; ++p) {
    c.m[p] = U[(int64_t)p * nc + idx];
    c.a[p] = U[(int64_t)(N + D + 1 + p) * nc + idx];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) c.mom[k] = U[(int64_t)(N + k) * nc + idx];
  c.E = U[(int64_t)(N + D) * nc + idx];
}

// (1 + K_p) of the source term of Eq. (1) at the cell average: 1 for the
// Allaire model, rho c^2 / (gamma_p (P + Pinf_p)) for the Kapila model.
template <int N, int D>
__device__ __forceinline__ void one_plus_k(const Cons<N, D>& ub, const Eos& e,
                                           int model, double* opk) {
  if (model != MP_MODEL_KAPILA) {
#pragma unroll
    for (int p = 0; p < N; ++p) opk[p] = 1.0;
    return;
  }
  Prim<N, D> v;
  cons_to_prim<N, D>(ub, e, v);
  const double rc2 = mix_rc2<N>(v.a, v.P, e, model);
#pragma unroll
  for (int p = 0; p < N; ++p) {
    const double k = e.gam[p] * (v.P + e.pinf[p]);
    opk[p] = k > 0.0 ? rc2 / k : 1.0;
  }
}

// RK epilogue for one cell: L in component order; writes out.
template <int N, int D>
__device__ __forceinline__ void finish_cell(const StageArgs& a, int64_t nc,
                                            int64_t idx, const Cons<N, D>& uk,
                                            const double* L) {
  constexpr int NU = 2 * N + D + 1;
  if (a.mode == 0) {
#pragma unroll
    for (int c = 0; c < NU; ++c) a.out[(int64_t)c * nc + idx] = L[c];
    return;
  }
  const double dt = *a.dt;
  double u[NU];
#pragma unroll
  for (int p = 0; p < N; ++p) { u[p] = uk.m[p]; u[N + D + 1 + p] = uk.a[p]; }
#pragma unroll
  for (int k = 0; k < D; ++k) u[N + k] = uk.mom[k];
  u[N + D] = uk.E;
  if (a.a == 0.0) {
#pragma unroll
    for (int c = 0; c < NU; ++c) a.out[(int64_t)c * nc + idx] = a.b * (u[c] + dt * L[c]);
  } else {
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      const double un = a.Un[(int64_t)c * nc + idx];
      a.out[(int64_t)c * nc + idx] = a.a * un + a.b * (u[c] + dt * L[c]);
    }
  }
}

// ---------------------------------------------------------------------------
// x sweep
// ---------------------------------------------------------------------------
template <int N, int D, typename W>
__global__ __launch_bounds__(kBX) void k_sweep_x(const Grid g, const Eos e,
                                                 const StageArgs a) {
  constexpr int NV = 2 * N + D + 1;
  constexpr int NU = NV;
  constexpr int NF = 2 * N + 2 * D + 4;
  constexpr int NFL = NU + 1;
  // the flux rows reuse the primitive rows: the stencil is in registers and
  // a barrier (after the face exchange) separates the two uses
  constexpr int NPRIM = NV * (kBX + 4), NFLX = NFL * kBX;
  __shared__ double sraw[NPRIM > NFLX ? NPRIM : NFLX];
  __shared__ double sface[NF][kBX];
  double (*sprim)[kBX + 4] = reinterpret_cast<double (*)[kBX + 4]>(sraw);
  double (*sflux)[kBX] = reinterpret_cast<double (*)[kBX]>(sraw);

  const int l = threadIdx.x;
  const int y = blockIdx.y;
  const int x0 = blockIdx.x * (kBX - 2);
  const int xi = x0 - 1 + l;
  const int64_t row = (int64_t)y * g.nx;
  const int64_t nc = g.nc;

  auto put_prim = [&](int x, int slot) {
    const int xm = bc_map(x, g.nx, g.bcx0, g.bcx1);
    Cons<N, D> c;
    load_cons<N, D>(a.Uk, nc, row + xm, c);
    Prim<N, D> v;
    cons_to_prim<N, D>(c, e, v);
#pragma unroll
    for (int p = 0; p < N; ++p) { sprim[p][slot] = v.m[p]; sprim[N + p][slot] = v.a[p]; }
#pragma unroll
    for (int k = 0; k < D; ++k) sprim[2 * N + k][slot] = v.u[k];
    sprim[2 * N + D][slot] = v.P;
  };

  const int xm = bc_map(xi, g.nx, g.bcx0, g.bcx1);
  Cons<N, D> ub;
  load_cons<N, D>(a.Uk, nc, row + xm, ub);
  {
    Prim<N, D> v;
    cons_to_prim<N, D>(ub, e, v);
#pragma unroll
    for (int p = 0; p < N; ++p) { sprim[p][l + 2] = v.m[p]; sprim[N + p][l + 2] = v.a[p]; }
#pragma unroll
    for (int k = 0; k < D; ++k) sprim[2 * N + k][l + 2] = v.u[k];
    sprim[2 * N + D][l + 2] = v.P;
  }
  if (l < 2) put_prim(x0 - 3 + l, l);
  if (l >= kBX - 2) put_prim(x0 - 1 + l + 2, l + 4);
  __syncthreads();

  Prim<N, D> s[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
#pragma unroll
    for (int p = 0; p < N; ++p) { s[j].m[p] = sprim[p][l + j]; s[j].a[p] = sprim[N + p][l + j]; }
#pragma unroll
    for (int k = 0; k < D; ++k) s[j].u[k] = sprim[2 * N + k][l + j];
    s[j].P = sprim[2 * N + D][l + j];
  }
  Face<N, D> fm, fp;
  reconstruct<N, D, W>(s, ub, e, g, g.hdx, fm, fp);

  // publish the minus-side face state for the left neighbour
#pragma unroll
  for (int p = 0; p < N; ++p) { sface[p][l] = fm.m[p]; sface[N + p][l] = fm.a[p]; }
#pragma unroll
  for (int k = 0; k < D; ++k) { sface[2 * N + k][l] = fm.mom[k]; sface[2 * N + D + k][l] = fm.u[k]; }
  sface[2 * N + 2 * D][l] = fm.E;
  sface[2 * N + 2 * D + 1][l] = fm.P;
  sface[2 * N + 2 * D + 2][l] = fm.rho;
  sface[2 * N + 2 * D + 3][l] = fm.c;
  __syncthreads();

  Flux<N, D> F;
  if (l < kBX - 1) {
    Face<N, D> R;
    const int r = l + 1;
#pragma unroll
    for (int p = 0; p < N; ++p) { R.m[p] = sface[p][r]; R.a[p] = sface[N + p][r]; }
#pragma unroll
    for (int k = 0; k < D; ++k) { R.mom[k] = sface[2 * N + k][r]; R.u[k] = sface[2 * N + D + k][r]; }
    R.E = sface[2 * N + 2 * D][r];
    R.P = sface[2 * N + 2 * D + 1][r];
    R.rho = sface[2 * N + 2 * D + 2][r];
    R.c = sface[2 * N + 2 * D + 3][r];
    riemann<N, D, W>(fp, R, 0, g.flux, F);
#pragma unroll
    for (int c = 0; c < NU; ++c) sflux[c][l] = F.f[c];
    sflux[NU][l] = F.uh;
  }
  __syncthreads();

  if (l >= 1 && l < kBX - 1 && xi < g.nx) {
    double L[NU];
    double opk[N];
    one_plus_k<N, D>(ub, e, g.model, opk);
#pragma unroll
    for (int c = 0; c < NU; ++c) L[c] = -(F.f[c] - sflux[c][l - 1]) * g.rdx;
    const double du = (F.uh - sflux[NU][l - 1]) * g.rdx;
#pragma unroll
    for (int p = 0; p < N; ++p) L[N + D + 1 + p] += ub.a[p] * opk[p] * du;
    const int64_t idx = row + xi;
    if constexpr (D == 1) {
      finish_cell<N, D>(a, nc, idx, ub, L);
    } else {
#pragma unroll
      for (int c = 0; c < NU; ++c) a.acc[(int64_t)c * nc + idx] = L[c];
    }
  }
}

// ---------------------------------------------------------------------------
// y sweep (2D) + RK epilogue
// ---------------------------------------------------------------------------
// A workgroup is a tile of kTX columns x kTY rows of lanes, one cell per lane
// (lane (tx, ty) holds cell (x0 + tx, y0 - 1 + ty)); rows y0 .. y0 + kTY - 3
// are its outputs.  Primitives of rows y0 - 3 .. y0 + kTY go to LDS (each row
// segment is kTX contiguous doubles per component, one 128-byte line), every
// lane reconstructs its cell along y from its column, and face states and
// fluxes are traded with the neighbour row through LDS, as in the x sweep.
constexpr int kTX = 16;
constexpr int kTY = 16;
constexpr int kOY = kTY - 2;      // output rows per tile

template <int N, typename W>
__global__ __launch_bounds__(kTX * kTY) void k_sweep_y(const Grid g, const Eos e,
                                                       const StageArgs a) {
  constexpr int D = 2;
  constexpr int NV = 2 * N + D + 1;
  constexpr int NU = NV;
  constexpr int NF = 2 * N + 2 * D + 4;
  constexpr int NFL = NU + 1;
  constexpr int NPRIM = NV * (kTY + 4) * kTX, NFLX = NFL * kTY * kTX;
  __shared__ double sraw[NPRIM > NFLX ? NPRIM : NFLX];
  __shared__ double sface[NF][kTY][kTX];
  double (*sprim)[kTY + 4][kTX] = reinterpret_cast<double (*)[kTY + 4][kTX]>(sraw);
  double (*sflux)[kTY][kTX] = reinterpret_cast<double (*)[kTY][kTX]>(sraw);

  const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
  const int x = blockIdx.x * kTX + tx;
  const bool colok = x < g.nx;
  const int xc = colok ? x : g.nx - 1;
  const int y0 = blockIdx.y * kOY;
  const int yi = y0 - 1 + ty;
  const int64_t nc = g.nc;

  auto put_prim = [&](int y, int slot) {
    const int ym = bc_map(y, g.ny, g.bcy0, g.bcy1);
    Cons<N, D> c;
    load_cons<N, D>(a.Uk, nc, (int64_t)ym * g.nx + xc, c);
    Prim<N, D> v;
    cons_to_prim<N, D>(c, e, v);
#pragma unroll
    for (int p = 0; p < N; ++p) { sprim[p][slot][tx] = v.m[p]; sprim[N + p][slot][tx] = v.a[p]; }
#pragma unroll
    for (int k = 0; k < D; ++k) sprim[2 * N + k][slot][tx] = v.u[k];
    sprim[2 * N + D][slot][tx] = v.P;
  };

  const int ym = bc_map(yi, g.ny, g.bcy0, g.bcy1);
  Cons<N, D> ub;
  load_cons<N, D>(a.Uk, nc, (int64_t)ym * g.nx + xc, ub);
  {
    Prim<N, D> v;
    cons_to_prim<N, D>(ub, e, v);
#pragma unroll
    for (int p = 0; p < N; ++p) { sprim[p][ty + 2][tx] = v.m[p]; sprim[N + p][ty + 2][tx] = v.a[p]; }
#pragma unroll
    for (int k = 0; k < D; ++k) sprim[2 * N + k][ty + 2][tx] = v.u[k];
    sprim[2 * N + D][ty + 2][tx] = v.P;
  }
  if (ty < 2) put_prim(y0 - 3 + ty, ty);
  if (ty >= kTY - 2) put_prim(yi + 2, ty + 4);
  __syncthreads();

  Prim<N, D> s[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
#pragma unroll
    for (int p = 0; p < N; ++p) { s[j].m[p] = sprim[p][ty + j][tx]; s[j].a[p] = sprim[N + p][ty + j][tx]; }
#pragma unroll
    for (int k = 0; k < D; ++k) s[j].u[k] = sprim[2 * N + k][ty + j][tx];
    s[j].P = sprim[2 * N + D][ty + j][tx];
  }
  Face<N, D> fm, fp;
  reconstruct<N, D, W>(s, ub, e, g, g.hdy, fm, fp);

#pragma unroll
  for (int p = 0; p < N; ++p) { sface[p][ty][tx] = fm.m[p]; sface[N + p][ty][tx] = fm.a[p]; }
#pragma unroll
  for (int k = 0; k < D; ++k) { sface[2 * N + k][ty][tx] = fm.mom[k]; sface[2 * N + D + k][ty][tx] = fm.u[k]; }
  sface[2 * N + 2 * D][ty][tx] = fm.E;
  sface[2 * N + 2 * D + 1][ty][tx] = fm.P;
  sface[2 * N + 2 * D + 2][ty][tx] = fm.rho;
  sface[2 * N + 2 * D + 3][ty][tx] = fm.c;
  __syncthreads();

  Flux<N, D> F;
  if (ty < kTY - 1) {
    Face<N, D> R;
    const int r = ty + 1;
#pragma unroll
    for (int p = 0; p < N; ++p) { R.m[p] = sface[p][r][tx]; R.a[p] = sface[N + p][r][tx]; }
#pragma unroll
    for (int k = 0; k < D; ++k) { R.mom[k] = sface[2 * N + k][r][tx]; R.u[k] = sface[2 * N + D + k][r][tx]; }
    R.E = sface[2 * N + 2 * D][r][tx];
    R.P = sface[2 * N + 2 * D + 1][r][tx];
    R.rho = sface[2 * N + 2 * D + 2][r][tx];
    R.c = sface[2 * N + 2 * D + 3][r][tx];
    riemann<N, D, W>(fp, R, 1, g.flux, F);
#pragma unroll
    for (int c = 0; c < NU; ++c) sflux[c][ty][tx] = F.f[c];
    sflux[NU][ty][tx] = F.uh;
  }
  __syncthreads();

  if (ty >= 1 && ty < kTY - 1 && colok && yi < g.ny) {
    const int64_t idx = (int64_t)yi * g.nx + x;
    double L[NU];
    double opk[N];
    one_plus_k<N, D>(ub, e, g.model, opk);
#pragma unroll
    for (int c = 0; c < NU; ++c)
      L[c] = a.acc[(int64_t)c * nc + idx] - (F.f[c] - sflux[c][ty - 1][tx]) * g.rdy;
    const double du = (F.uh - sflux[NU][ty - 1][tx]) * g.rdy;
#pragma unroll
    for (int p = 0; p < N; ++p) L[N + D + 1 + p] += ub.a[p] * opk[p] * du;
    finish_cell<N, D>(a, nc, idx, ub, L);
  }
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = -1.0;
  if (threadIdx.x == 0) {
    r = sh[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = fmax(r, sh[k]);
  }
  __syncthreads();
  return r;
}

// per-block max over cells of sum_d (|u_d| + c)/dx_d
template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_dt(const Grid g, const Eos e,
                                                  const double* __restrict__ U,
                                                  double* __restrict__ part) {
  __shared__ double sh[kRedBlock / 64];
  double smax = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.nc;
       i += (int64_t)gridDim.x * blockDim.x) {
    Cons<N, D> c;
    load_cons<N, D>(U, g.nc, i, c);
    Prim<N, D> v;
    cons_to_prim<N, D>(c, e, v);
    double rho = 0.0;
#pragma unroll
    for (int p = 0; p < N; ++p) rho += v.m[p];
    const double cs = sound_speed(mix_rc2<N>(v.a, v.P, e, g.model), rho);
    double s = (fabs(v.u[0]) + cs) * g.rdx;
    if constexpr (D > 1) s += (fabs(v.u[1]) + cs) * g.rdy;
    smax = fmax(smax, s);
  }
  const double r = block_max(smax, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// dt = cfl / max, clipped to t_end - t
__global__ __launch_bounds__(kRedBlock) void k_dt_finish(
    const double* __restrict__ part, int np, double cfl, double t_end,
    const double* __restrict__ t, double* __restrict__ dt) {
  __shared__ double sh[kRedBlock / 64];
  double m = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) m = fmax(m, part[i]);
  const double r = block_max(m, sh);
  if (threadIdx.x == 0) {
    double d = cfl / r;
    if (t_end > 0.0 && *t + d > t_end) d = t_end - *t;
    *dt = d;
  }
}

__global__ void k_advance_time(double* t, double* steps, const double* dt) {
  if (threadIdx.x == 0) {
    *t = *t + *dt;
    *steps = *steps + 1.0;
  }
}

// per-block diagnostics: slots 0..nU-1 sums, then
// [20] max|sum a - 1|, [21] min m, [22] min a, [23] max a, [24] min psi,
// [25] non-finite count, [28] max |rho E|
template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_diag(const Grid g, const Eos e,
                                                    const double* __restrict__ U,
                                                    double* __restrict__ part) {
  constexpr int NU = 2 * N + D + 1;
  __shared__ double sh[kRedBlock];
  double acc[kDiagSlots];
#pragma unroll
  for (int k = 0; k < kDiagSlots; ++k) acc[k] = 0.0;
  acc[21] = acc[22] = acc[24] = INFINITY;
  acc[23] = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.nc;
       i += (int64_t)gridDim.x * blockDim.x) {
    double u[NU];
    double nonfin = 0.0;
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      u[c] = U[(int64_t)c * g.nc + i];
      acc[c] += u[c];
      if (!isfinite(u[c])) nonfin += 1.0;
    }
    double sa = 0.0;
#pragma unroll
    for (int p = 0; p < N; ++p) {
      const double m = u[p], al = u[N + D + 1 + p];
      sa += al;
      acc[21] = fmin(acc[21], m);
      acc[22] = fmin(acc[22], al);
      acc[23] = fmax(acc[23], al);
    }
    acc[20] = fmax(acc[20], fabs(sa - 1.0));
    acc[24] = fmin(acc[24], psi<N, D>(u, u + N + D + 1, u + N, u[N + D], e));
    acc[25] += nonfin;
    acc[28] = fmax(acc[28], fabs(u[N + D]));
  }
  // fixed-order tree per slot
  for (int k = 0; k < kDiagSlots; ++k) {
    sh[threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kRedBlock / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        const double x = sh[threadIdx.x], y = sh[threadIdx.x + s];
        double r;
        if (k == 21 || k == 22 || k == 24) r = fmin(x, y);
        else if (k == 20 || k == 23 || k == 28) r = fmax(x, y);
        else r = x + y;
        sh[threadIdx.x] = r;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * kDiagSlots + k] = sh[0];
    __syncthreads();
  }
}
__global__ void k_diag_finish(const double* __restrict__ part, int np,
                              int nU, double vol, const double* t,
                              const double* steps, double* __restrict__ out) {
  const int k = threadIdx.x;
  if (k >= kDiagSlots) return;
  double r;
  if (k == 21 || k == 22 || k == 24) r = INFINITY;
  else if (k == 23) r = -INFINITY;
  else r = 0.0;
  for (int b = 0; b < np; ++b) {
    const double x = part[(int64_t)b * kDiagSlots + k];
    if (k == 21 || k == 22 || k == 24) r = fmin(r, x);
    else if (k == 20 || k == 23 || k == 28) r = fmax(r, x);
    else r = r + x;
  }
  if (k < nU) r *= vol;
  if (k == 26) r = *t;
  if (k == 27) r = *steps;
  out[k] = r;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Inst {
  mp_weno_instance in;
  Grid g;
  Eos e;
  int N, D, nU;
  int64_t nc;
  double* U1 = nullptr;
  double* U2 = nullptr;
  double* acc = nullptr;
  double* backup = nullptr;
  int nred = 1;          // reduction blocks
};

// Optional event pair recorded around one of the stage kernels (profiling).
struct Bracket {
  int which = 0;                  // 0 none, 1 x sweep, 2 y sweep, 3 whole stage
  hipEvent_t ev[2] = {nullptr, nullptr};
};

using StageFn = void (*)(const Inst&, const StageArgs&, hipStream_t, const Bracket*);
using RedFn = void (*)(const Inst&, const double*, double*, hipStream_t);

template <int N, int D, typename W>
void launch_stage(const Inst& I, const StageArgs& a, hipStream_t s, const Bracket* b) {
  const int w = b ? b->which : 0;
  dim3 gx((I.g.nx + kBX - 3) / (kBX - 2), D == 1 ? 1 : I.g.ny);
  if (w == 1 || w == 3) (void)hipEventRecord(b->ev[0], s);
  hipLaunchKernelGGL((k_sweep_x<N, D, W>), gx, dim3(kBX), 0, s, I.g, I.e, a);
  if (w == 1 || (w == 3 && D == 1)) (void)hipEventRecord(b->ev[1], s);
  if constexpr (D == 2) {
    dim3 gy((I.g.nx + kTX - 1) / kTX, (I.g.ny + kOY - 1) / kOY);
    if (w == 2) (void)hipEventRecord(b->ev[0], s);
    hipLaunchKernelGGL((k_sweep_y<N, W>), gy, dim3(kTX * kTY), 0, s, I.g, I.e, a);
    if (w == 2 || w == 3) (void)hipEventRecord(b->ev[1], s);
  }
}

template <int N, int D>
void launch_dt(const Inst& I, const double* U, double* part, hipStream_t s) {
  hipLaunchKernelGGL((k_dt<N, D>), dim3(I.nred), dim3(kRedBlock), 0, s, I.g, I.e, U, part);
}

template <int N, int D>
void launch_diag(const Inst& I, const double* U, double* part, hipStream_t s) {
  hipLaunchKernelGGL((k_diag<N, D>), dim3(I.nred), dim3(kRedBlock), 0, s, I.g, I.e, U, part);
}

struct Table {
  StageFn stage[kMaxN + 1][3][2] = {};
  RedFn dt[kMaxN + 1][3] = {};
  RedFn diag[kMaxN + 1][3] = {};
};

template <int N>
void fill(Table& t) {
  t.stage[N][1][0] = launch_stage<N, 1, double>;
  t.stage[N][1][1] = launch_stage<N, 1, float>;
  t.stage[N][2][0] = launch_stage<N, 2, double>;
  t.stage[N][2][1] = launch_stage<N, 2, float>;
  t.dt[N][1] = launch_dt<N, 1>;
  t.dt[N][2] = launch_dt<N, 2>;
  t.diag[N][1] = launch_diag<N, 1>;
  t.diag[N][2] = launch_diag<N, 2>;
}

static const Table& table() {
  static Table t = [] {
    Table x;
    fill<1>(x); fill<2>(x); fill<3>(x); fill<4>(x); fill<5>(x);
    return x;
  }();
  return t;
}

}  // namespace mpw

using namespace mpw;

struct mp_weno_ctx {
  std::vector<Inst> inst;
  mp_weno_opts opt;
  hipStream_t stream = nullptr;
  double* dt = nullptr;       // n_inst
  double* t = nullptr;        // n_inst
  double* steps = nullptr;    // n_inst
  double* part = nullptr;     // reduction partials
  double* diag = nullptr;     // n_inst * MP_DIAG_LEN
  hipGraphExec_t graph[2] = {nullptr, nullptr};   // [external dt?]
  std::string err;
  int profile = 0;                           // Bracket::which
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t ev_used = 0;

  const Bracket* next_bracket(Bracket& b) {
    if (!profile) return nullptr;
    if (ev_used == events.size()) {
      hipEvent_t e0, e1;
      if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return nullptr;
      events.emplace_back(e0, e1);
    }
    b.which = profile;
    b.ev[0] = events[ev_used].first;
    b.ev[1] = events[ev_used].second;
    ++ev_used;
    return &b;
  }
};

static mp_status fail(mp_weno_ctx* c, mp_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, call)                                                     \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      return fail((ctx), MP_ERR_HIP, std::string(#call) + ": " +              \
                                         hipGetErrorString(e_));              \
  } while (0)

static mp_status enqueue_dt(mp_weno_ctx* c) {
  const Table& T = table();
  for (size_t i = 0; i < c->inst.size(); ++i) {
    const Inst& I = c->inst[i];
    T.dt[I.N][I.D](I, I.in.U, c->part, c->stream);
    hipLaunchKernelGGL(k_dt_finish, dim3(1), dim3(kRedBlock), 0, c->stream, c->part,
                       I.nred, c->opt.cfl, I.in.t_end, c->t + i, c->dt + i);
  }
  HIPCHK(c, hipGetLastError());
  return MP_OK;
}

static mp_status enqueue_rk(mp_weno_ctx* c) {
  const Table& T = table();
  for (size_t i = 0; i < c->inst.size(); ++i) {
    const Inst& I = c->inst[i];
    StageFn f = T.stage[I.N][I.D][c->opt.precision];
    StageArgs a{};
    a.dt = c->dt + i;
    a.acc = I.acc;
    a.mode = 1;
    a.Un = I.in.U;
    // U1 = Un + dt L(Un)
    a.Uk = I.in.U; a.out = I.U1; a.a = 0.0; a.b = 1.0;
    Bracket br;
    f(I, a, c->stream, c->next_bracket(br));
    // U2 = 3/4 Un + 1/4 (U1 + dt L(U1))
    a.Uk = I.U1; a.out = I.U2; a.a = 0.75; a.b = 0.25;
    f(I, a, c->stream, c->next_bracket(br));
    // Un+1 = 1/3 Un + 2/3 (U2 + dt L(U2)), in place (pointwise in Un)
    a.Uk = I.U2; a.out = I.in.U; a.a = 1.0 / 3.0; a.b = 2.0 / 3.0;
    f(I, a, c->stream, c->next_bracket(br));
    hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(64), 0, c->stream, c->t + i,
                       c->steps + i, c->dt + i);
  }
  HIPCHK(c, hipGetLastError());
  return MP_OK;
}

static mp_status enqueue_diag(mp_weno_ctx* c) {
  const Table& T = table();
  for (size_t i = 0; i < c->inst.size(); ++i) {
    const Inst& I = c->inst[i];
    T.diag[I.N][I.D](I, I.in.U, c->part, c->stream);
    double vol = 1.0;
    for (int d = 0; d < I.D; ++d) vol *= I.in.dx[d];
    hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(64), 0, c->stream, c->part, I.nred,
                       I.nU, vol, c->t + i, c->steps + i, c->diag + i * MP_DIAG_LEN);
  }
  HIPCHK(c, hipGetLastError());
  return MP_OK;
}

extern "C" {

int32_t mp_weno_abi_version(void) { return MP_WENO_ABI_VERSION; }
int32_t mp_weno_max_phases(void) { return kMaxN; }

const char* mp_weno_strerror(mp_status s) {
  switch (s) {
    case MP_OK: return "ok";
    case MP_ERR_ARG: return "invalid argument";
    case MP_ERR_HIP: return "HIP runtime error";
    case MP_ERR_OOM: return "out of device memory";
    case MP_ERR_INADMISSIBLE: return "state left the admissible set";
    case MP_ERR_NONFINITE: return "non-finite state";
    case MP_ERR_SOLVER: return "solver did not converge";
    case MP_ERR_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

const char* mp_weno_last_error(const mp_weno_ctx* ctx) {
  return ctx ? ctx->err.c_str() : "";
}

mp_status mp_weno_destroy(mp_weno_ctx* c) {
  if (!c) return MP_OK;
  for (auto& g : c->graph)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto& e : c->events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& I : c->inst) {
    (void)hipFree(I.U1); (void)hipFree(I.U2); (void)hipFree(I.acc); (void)hipFree(I.backup);
  }
  (void)hipFree(c->dt); (void)hipFree(c->t); (void)hipFree(c->steps); (void)hipFree(c->part); (void)hipFree(c->diag);
  delete c;
  return MP_OK;
}

mp_status mp_weno_init(mp_weno_ctx** out, int32_t n_inst,
                       const mp_weno_instance* inst, const mp_weno_opts* opt,
                       void* hip_stream) {
  if (!out) return MP_ERR_ARG;
  *out = nullptr;
  if (n_inst < 1 || !inst || !opt) return MP_ERR_ARG;
  if (opt->phase_field != 0) return MP_ERR_UNSUPPORTED;
  if (opt->precision != MP_PREC_FP64 && opt->precision != MP_PREC_MIXED) return MP_ERR_ARG;
  if (opt->recon < 0 || opt->recon > 1 || opt->flux < 0 || opt->flux > 1 ||
      opt->model < 0 || opt->model > 1 || !(opt->cfl > 0.0))
    return MP_ERR_ARG;
  for (int i = 0; i < n_inst; ++i) {
    const mp_weno_instance& s = inst[i];
    if (s.ndim < 1 || s.ndim > 3 || !s.U) return MP_ERR_ARG;
    if (s.ndim > 2) return MP_ERR_UNSUPPORTED;
    if (s.nphase < 1 || s.nphase > MP_MAXP) return MP_ERR_ARG;
    if (s.nphase > kMaxN) return MP_ERR_UNSUPPORTED;
    for (int d = 0; d < s.ndim; ++d) {
      if (s.n[d] < 1 || !(s.dx[d] > 0.0)) return MP_ERR_ARG;
      for (int k = 0; k < 2; ++k)
        if (s.bc[d][k] != MP_BC_PERIODIC && s.bc[d][k] != MP_BC_OUTFLOW) return MP_ERR_ARG;
    }
    for (int p = 0; p < s.nphase; ++p)
      if (!(s.gamma[p] > 1.0) || !std::isfinite(s.pinf[p]) || !std::isfinite(s.D[p]) ||
          !std::isfinite(s.pmin[p]))
        return MP_ERR_ARG;
    const int64_t nc = (int64_t)s.n[0] * (s.ndim > 1 ? s.n[1] : 1);
    if (nc > (int64_t)1 << 31) return MP_ERR_UNSUPPORTED;
  }

  if (opt->use_graph && !hip_stream) return MP_ERR_ARG;   // no capture on the null stream
  mp_weno_ctx* c = new (std::nothrow) mp_weno_ctx();
  if (!c) return MP_ERR_OOM;
  c->opt = *opt;
  c->stream = (hipStream_t)hip_stream;
  size_t maxred = 1;
  for (int i = 0; i < n_inst; ++i) {
    Inst I;
    I.in = inst[i];
    const mp_weno_instance& s = inst[i];
    I.N = s.nphase;
    I.D = s.ndim;
    I.nU = 2 * I.N + I.D + 1;
    I.nc = (int64_t)s.n[0] * (s.ndim > 1 ? s.n[1] : 1);
    Grid& g = I.g;
    g.nx = s.n[0];
    g.ny = s.ndim > 1 ? s.n[1] : 1;
    g.nc = I.nc;
    g.rdx = 1.0 / s.dx[0];
    g.hdx = 0.5 * s.dx[0];
    g.rdy = s.ndim > 1 ? 1.0 / s.dx[1] : 0.0;
    g.hdy = s.ndim > 1 ? 0.5 * s.dx[1] : 1.0;
    g.bcx0 = s.bc[0][0]; g.bcx1 = s.bc[0][1];
    g.bcy0 = s.ndim > 1 ? s.bc[1][0] : 0;
    g.bcy1 = s.ndim > 1 ? s.bc[1][1] : 0;
    g.recon = opt->recon;
    g.flux = opt->flux;
    g.model = opt->model;
    g.energy = opt->energy_limiter ? 1 : 0;
    std::memset(&I.e, 0, sizeof(I.e));
    for (int p = 0; p < I.N; ++p) {
      const double gm = s.gamma[p], pi = s.pinf[p];
      I.e.A[p] = 1.0 / (gm - 1.0);
      I.e.B[p] = gm * pi / (gm - 1.0);
      I.e.Dp[p] = s.D[p];
      I.e.gam[p] = gm;
      I.e.pinf[p] = pi;
      I.e.EB[p] = I.e.A[p] * s.pmin[p] + I.e.B[p];
    }
    I.nred = (int)std::min<int64_t>(kRedMaxBlocks, (I.nc + kRedBlock - 1) / kRedBlock);
    maxred = std::max<size_t>(maxred, (size_t)I.nred);
    const size_t bytes = sizeof(double) * (size_t)I.nU * (size_t)I.nc;
    if (hipMalloc(&I.U1, bytes) != hipSuccess || hipMalloc(&I.U2, bytes) != hipSuccess ||
        (I.D > 1 && hipMalloc(&I.acc, bytes) != hipSuccess) ||
        (opt->check_bounds && hipMalloc(&I.backup, bytes) != hipSuccess)) {
      c->inst.push_back(I);
      mp_weno_destroy(c);
      return MP_ERR_OOM;
    }
    c->inst.push_back(I);
  }
  const size_t n = (size_t)n_inst;
  if (hipMalloc(&c->dt, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&c->t, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&c->steps, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&c->part, sizeof(double) * maxred * kDiagSlots) != hipSuccess ||
      hipMalloc(&c->diag, sizeof(double) * n * MP_DIAG_LEN) != hipSuccess) {
    mp_weno_destroy(c);
    return MP_ERR_OOM;
  }
  std::vector<double> zeros(n * MP_DIAG_LEN, 0.0);
  if (hipMemcpy(c->t, zeros.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->steps, zeros.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->dt, zeros.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess) {
    mp_weno_destroy(c);
    return MP_ERR_HIP;
  }
  *out = c;
  return MP_OK;
}

mp_status mp_weno_set_time(mp_weno_ctx* c, const double* t) {
  if (!c || !t) return MP_ERR_ARG;
  HIPCHK(c, hipMemcpyAsync(c->t, t, sizeof(double) * c->inst.size(), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MP_OK;
}

mp_status mp_weno_rhs(mp_weno_ctx* c, const double* const* U_in, double* const* dUdt) {
  if (!c || !dUdt) return fail(c, MP_ERR_ARG, "null argument");
  const Table& T = table();
  for (size_t i = 0; i < c->inst.size(); ++i) {
    const Inst& I = c->inst[i];
    if (!dUdt[i]) return fail(c, MP_ERR_ARG, "null output pointer");
    StageArgs a{};
    a.Uk = (U_in && U_in[i]) ? U_in[i] : I.in.U;
    a.out = dUdt[i];
    a.acc = I.acc;
    a.mode = 0;
    a.dt = c->dt + i;
    T.stage[I.N][I.D][c->opt.precision](I, a, c->stream, nullptr);
  }
  HIPCHK(c, hipGetLastError());
  return MP_OK;
}

mp_status mp_weno_dt(mp_weno_ctx* c, double* dt, int32_t where) {
  if (!c || !dt) return fail(c, MP_ERR_ARG, "null argument");
  mp_status s = enqueue_dt(c);
  if (s != MP_OK) return s;
  const size_t bytes = sizeof(double) * c->inst.size();
  if (where == MP_WHERE_HOST) {
    HIPCHK(c, hipMemcpyAsync(dt, c->dt, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    HIPCHK(c, hipMemcpyAsync(dt, c->dt, bytes, hipMemcpyDeviceToDevice, c->stream));
  }
  return MP_OK;
}

static mp_status enqueue_step(mp_weno_ctx* c, bool external_dt) {
  if (!external_dt) {
    mp_status s = enqueue_dt(c);
    if (s != MP_OK) return s;
  }
  return enqueue_rk(c);
}

mp_status mp_weno_step(mp_weno_ctx* c, const double* dt_dev) {
  if (!c) return MP_ERR_ARG;
  const size_t n = c->inst.size();
  if (c->opt.check_bounds) {
    for (auto& I : c->inst)
      HIPCHK(c, hipMemcpyAsync(I.backup, I.in.U, sizeof(double) * I.nU * I.nc,
                               hipMemcpyDeviceToDevice, c->stream));
  }
  std::vector<double> t_before;
  if (c->opt.check_bounds) {
    t_before.resize(2 * n);
    HIPCHK(c, hipMemcpyAsync(t_before.data(), c->t, sizeof(double) * n,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(t_before.data() + n, c->steps, sizeof(double) * n,
                             hipMemcpyDeviceToHost, c->stream));
  }
  const bool ext = dt_dev != nullptr;
  if (ext)
    HIPCHK(c, hipMemcpyAsync(c->dt, dt_dev, sizeof(double) * n, hipMemcpyDeviceToDevice,
                             c->stream));
  if (c->opt.use_graph && !c->profile) {
    hipGraphExec_t& ge = c->graph[ext ? 1 : 0];
    if (!ge) {
      hipGraph_t gph;
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      mp_status s = enqueue_step(c, ext);
      hipError_t e2 = hipStreamEndCapture(c->stream, &gph);
      if (s != MP_OK) return s;
      if (e2 != hipSuccess) return fail(c, MP_ERR_HIP, hipGetErrorString(e2));
      HIPCHK(c, hipGraphInstantiate(&ge, gph, nullptr, nullptr, 0));
      (void)hipGraphDestroy(gph);
    }
    HIPCHK(c, hipGraphLaunch(ge, c->stream));
  } else {
    mp_status s = enqueue_step(c, ext);
    if (s != MP_OK) return s;
  }
  if (c->opt.check_bounds) {
    mp_status s = enqueue_diag(c);
    if (s != MP_OK) return s;
    std::vector<double> d(n * MP_DIAG_LEN);
    HIPCHK(c, hipMemcpyAsync(d.data(), c->diag, sizeof(double) * d.size(),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    mp_status verdict = MP_OK;
    for (size_t i = 0; i < n && verdict == MP_OK; ++i) {
      const double* r = d.data() + i * MP_DIAG_LEN;
      const double tol = 1e-10;
      if (r[25] > 0.0) verdict = MP_ERR_NONFINITE;
      else if (r[21] < -tol * std::max(1.0, std::fabs(r[21])) || r[22] < -tol ||
               r[23] > 1.0 + tol || r[24] < -1e-12 * r[28])
        verdict = MP_ERR_INADMISSIBLE;
    }
    if (verdict != MP_OK) {
      for (auto& I : c->inst)
        HIPCHK(c, hipMemcpyAsync(I.in.U, I.backup, sizeof(double) * I.nU * I.nc,
                                 hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(c, hipMemcpyAsync(c->t, t_before.data(), sizeof(double) * n,
                               hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipMemcpyAsync(c->steps, t_before.data() + n, sizeof(double) * n,
                               hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      return fail(c, verdict, mp_weno_strerror(verdict));
    }
  }
  return MP_OK;
}

mp_status mp_weno_profile(mp_weno_ctx* c, int32_t which) {
  if (!c || which < 0 || which > 3) return MP_ERR_ARG;
  c->profile = which;
  c->ev_used = 0;
  return MP_OK;
}

mp_status mp_weno_timing(mp_weno_ctx* c, int32_t reset, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return MP_ERR_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double tot = 0.0;
  for (size_t i = 0; i < c->ev_used; ++i) {
    float x = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&x, c->events[i].first, c->events[i].second));
    tot += x;
  }
  *ms = tot;
  *launches = (int64_t)c->ev_used;
  if (reset) c->ev_used = 0;
  return MP_OK;
}

mp_status mp_weno_diag(mp_weno_ctx* c, double* out, int32_t where) {
  if (!c || !out) return fail(c, MP_ERR_ARG, "null argument");
  mp_status s = enqueue_diag(c);
  if (s != MP_OK) return s;
  const size_t bytes = sizeof(double) * c->inst.size() * MP_DIAG_LEN;
  if (where == MP_WHERE_HOST) {
    HIPCHK(c, hipMemcpyAsync(out, c->diag, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    HIPCHK(c, hipMemcpyAsync(out, c->diag, bytes, hipMemcpyDeviceToDevice, c->stream));
  }
  return MP_OK;
}

}  // extern "C"
