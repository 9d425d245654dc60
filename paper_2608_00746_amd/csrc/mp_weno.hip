// mp_weno.hip -- kernels, host runtime and C ABI of the MI355X WENO-C / WENO-CL
// hyperbolic step (declared in include/mp_weno.h).
//
// Instances with the same (N, d) form a group.  Each group has a device table
// of instance descriptors (grid, EOS, buffer pointers), and every kernel
// launch covers all tiles of all instances of the group: a workgroup finds its
// instance by binary search over per-instance tile offsets, so a batch of
// uneven instances is one launch per sweep.  One RK stage of a 2D group is two
// launches:
//   k_sweep_x : one workgroup per (instance, row, 254-cell strip).  Each lane
//               converts one cell to primitives into an LDS row, reconstructs
//               its cell along x from the five LDS neighbours, trades its
//               minus-side face state with the left neighbour through LDS,
//               computes the flux of its plus-side face, trades fluxes, and
//               writes the x part of L(U) to a direction accumulator (1D:
//               finishes the RK stage directly).
//   k_sweep_y : the same exchange pattern on 16 x 16 tiles of lanes (one
//               cell per lane, neighbours in y through LDS, 128-byte row
//               segments); it adds the accumulator and applies the RK stage.
// Both sweeps read the same stage state (unsplit, dimension by dimension).
// Workgroup indices can be remapped so that consecutive tiles (which share
// halo rows) run on the same XCD and its L2.  The CFL step and the
// diagnostics are per-instance reductions with a fixed order (no
// floating-point atomics), so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
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
constexpr int kDiagSlots = 32;    // per-block partials of the diagnostics

// The state pointers come from a table in device memory, so the compiler
// cannot tell their address space and would emit flat loads and stores (which
// also count against the LDS wait counter).  They always point to global
// memory; these types say so.
using gdouble = __attribute__((address_space(1))) double;
__device__ __forceinline__ const gdouble* gptr(const double* p) { return (const gdouble*)p; }
__device__ __forceinline__ gdouble* gptr(double* p) { return (gdouble*)p; }

struct StageArgs {
  const gdouble* Uk;  // stage state (stencils)
  const gdouble* Un;  // state at the start of the step (RK base)
  gdouble* out;       // U^(k+1), or L(U) when mode == 0
  gdouble* acc;       // x part of L (2D)
  const gdouble* dt;  // device time step of this instance
  double a, b;        // out = a Un + b (Uk + dt L)
  int mode;           // 0: write L, 1: RK stage
};

// One instance as the kernels see it (device memory, read with scalar loads).
struct Desc {
  Grid g;
  Eos e;
  double* U;                 // caller state U^n (updated in place)
  double* U1;                // RK stage buffers
  double* U2;
  double* acc;               // x part of L (2D)
  const double* rin;         // mp_weno_rhs input / output
  double* rout;
  double* dt;                // this instance's time step, time, step count
  double* t;
  double* steps;
  double* diag;              // MP_DIAG_LEN results
  double t_end, vol;
};

// RK stage s of Shu and Osher's third-order scheme (s = 0, 1, 2), or the
// plain operator L(U) (s = 3).
__device__ __forceinline__ StageArgs stage_args(const Desc& d, int s) {
  StageArgs a;
  a.acc = gptr(d.acc);
  a.dt = gptr(d.dt);
  a.Un = gptr(d.U);
  a.mode = 1;
  if (s == 0) { a.Uk = gptr(d.U); a.out = gptr(d.U1); a.a = 0.0; a.b = 1.0; }
  else if (s == 1) { a.Uk = gptr(d.U1); a.out = gptr(d.U2); a.a = 0.75; a.b = 0.25; }
  else if (s == 2) { a.Uk = gptr(d.U2); a.out = gptr(d.U); a.a = 1.0 / 3.0; a.b = 2.0 / 3.0; }
  else { a.Uk = gptr(d.rin); a.out = gptr(d.rout); a.a = 0.0; a.b = 0.0; a.mode = 0; }
  return a;
}

// (instance, tile within the instance) of work item `item`: one load from
// the group's tile map, none for a group of one instance
__device__ __forceinline__ int2 locate(const int2* __restrict__ map, int n, int item) {
  return n == 1 ? make_int2(0, item) : map[item];
}

// Workgroups are dispatched round-robin over the 8 XCDs; with swz set,
// logical tile j runs on XCD floor(j / (G/8)) so that neighbouring tiles
// share an L2.  A bijection of [0, G) for any G.
__device__ __forceinline__ int xcd_item(int b, int G, int swz) {
  if (!swz) return b;
  const int x = b & 7, slot = b >> 3, q = G >> 3, r = G & 7;
  return x * q + (x < r ? x : r) + slot;
}

__device__ __forceinline__ int bc_map(int i, int n, int lo, int hi) {
  if (i < 0) return lo == MP_BC_PERIODIC ? ((i % n) + n) % n : 0;
  if (i >= n) return hi == MP_BC_PERIODIC ? i % n : n - 1;
  return i;
}

template <int N, int D>
__device__ __forceinline__ void load_cons(const gdouble* __restrict__ U,
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
__global__ __launch_bounds__(kBX) void k_sweep_x(const Desc* __restrict__ descs,
                                                 const int2* __restrict__ map,
                                                 int ninst, int stage, int swz) {
  const int2 it = locate(map, ninst, xcd_item(blockIdx.x, gridDim.x, swz));
  const Desc d = descs[it.x];   // by value: loaded once, kept in registers
  const Grid& g = d.g;
  const Eos& e = d.e;
  const StageArgs a = stage_args(d, stage);
  const int ns = (g.nx + kBX - 3) / (kBX - 2);
  const int local = it.y;
  const int y = local / ns;
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
  const int x0 = (local - y * ns) * (kBX - 2);
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
__global__ __launch_bounds__(kTX * kTY) void k_sweep_y(const Desc* __restrict__ descs,
                                                       const int2* __restrict__ map,
                                                       int ninst, int stage, int swz) {
  const int2 it = locate(map, ninst, xcd_item(blockIdx.x, gridDim.x, swz));
  const Desc d = descs[it.x];
  const Grid& g = d.g;
  const Eos& e = d.e;
  const StageArgs a = stage_args(d, stage);
  const int ntx = (g.nx + kTX - 1) / kTX;
  const int local = it.y;
  const int tyb = local / ntx, txb = local - tyb * ntx;
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
  const int x = txb * kTX + tx;
  const bool colok = x < g.nx;
  const int xc = colok ? x : g.nx - 1;
  const int y0 = tyb * kOY;
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

constexpr int kRedChunk = kRedBlock * 4;    // cells per reduction workgroup

// per-workgroup max over its chunk of cells of sum_d (|u_d| + c)/dx_d
template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_dt(const Desc* __restrict__ descs,
                                                  const int2* __restrict__ map,
                                                  int ninst, double* __restrict__ part) {
  __shared__ double sh[kRedBlock / 64];
  const int2 it = locate(map, ninst, blockIdx.x);
  const Desc& d = descs[it.x];
  const Grid& g = d.g;
  const Eos& e = d.e;
  const int64_t c0 = (int64_t)it.y * kRedChunk;
  const int64_t c1 = c0 + kRedChunk < g.nc ? c0 + kRedChunk : g.nc;
  double smax = 0.0;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += kRedBlock) {
    Cons<N, D> c;
    load_cons<N, D>(gptr(d.U), g.nc, i, c);
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

// one workgroup per instance: dt = cfl / max, clipped to t_end - t
__global__ __launch_bounds__(kRedBlock) void k_dt_finish(
    const Desc* __restrict__ descs, const int* __restrict__ start,
    const double* __restrict__ part, double cfl) {
  __shared__ double sh[kRedBlock / 64];
  const Desc& d = descs[blockIdx.x];
  double m = 0.0;
  for (int i = start[blockIdx.x] + threadIdx.x; i < start[blockIdx.x + 1]; i += kRedBlock)
    m = fmax(m, part[i]);
  const double r = block_max(m, sh);
  if (threadIdx.x == 0) {
    const double t = *gptr(d.t);
    double dt = cfl / r;
    if (d.t_end > 0.0 && t + dt > d.t_end) dt = d.t_end - t;
    *gptr(d.dt) = dt;
  }
}

__global__ void k_advance_time(double* t, double* steps, const double* dt, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    t[i] = t[i] + dt[i];
    steps[i] = steps[i] + 1.0;
  }
}

// per-workgroup diagnostics: slots 0..nU-1 sums, then
// [20] max|sum a - 1|, [21] min m, [22] min a, [23] max a, [24] min psi,
// [25] non-finite count, [28] max |rho E|
template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_diag(const Desc* __restrict__ descs,
                                                    const int2* __restrict__ map,
                                                    int ninst, double* __restrict__ part) {
  constexpr int NU = 2 * N + D + 1;
  __shared__ double sh[kRedBlock];
  const int2 it = locate(map, ninst, blockIdx.x);
  const Desc& d = descs[it.x];
  const Grid& g = d.g;
  const Eos& e = d.e;
  const int64_t c0 = (int64_t)it.y * kRedChunk;
  const int64_t c1 = c0 + kRedChunk < g.nc ? c0 + kRedChunk : g.nc;
  const gdouble* U = gptr(d.U);
  double acc[kDiagSlots];
#pragma unroll
  for (int k = 0; k < kDiagSlots; ++k) acc[k] = 0.0;
  acc[21] = acc[22] = acc[24] = INFINITY;
  acc[23] = -INFINITY;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += kRedBlock) {
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

// one workgroup of kDiagSlots lanes per instance, lane k reduces slot k in
// block order
__global__ void k_diag_finish(const Desc* __restrict__ descs, const int* __restrict__ start,
                              const double* __restrict__ part) {
  const int k = threadIdx.x;
  const Desc& d = descs[blockIdx.x];
  if (k >= kDiagSlots) return;
  double r;
  if (k == 21 || k == 22 || k == 24) r = INFINITY;
  else if (k == 23) r = -INFINITY;
  else r = 0.0;
  for (int b = start[blockIdx.x]; b < start[blockIdx.x + 1]; ++b) {
    const double x = part[(int64_t)b * kDiagSlots + k];
    if (k == 21 || k == 22 || k == 24) r = fmin(r, x);
    else if (k == 20 || k == 23 || k == 28) r = fmax(r, x);
    else r = r + x;
  }
  if (k < 20) r *= d.vol;
  if (k == 26) r = *gptr(d.t);
  if (k == 27) r = *gptr(d.steps);
  gptr(d.diag)[k] = r;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Inst {
  mp_weno_instance in;
  int N, D, nU;
  int64_t nc;
  double* U1 = nullptr;
  double* U2 = nullptr;
  double* acc = nullptr;
  double* backup = nullptr;
};

// Instances of one (N, d): device descriptor table and tile offsets.
struct Group {
  int N = 0, D = 0;
  std::vector<int> ids;            // context instance indices
  std::vector<Desc> hdesc;         // host copy of the descriptors
  std::vector<int> xs, ys, rs;     // tile / reduction-chunk offsets (n + 1)
  Desc* desc = nullptr;
  int2* xmap = nullptr;            // work item -> (instance, local tile)
  int2* ymap = nullptr;
  int2* rmap = nullptr;
  int* rstart = nullptr;           // reduction-chunk offsets on the device
  size_t part_off = 0;             // this group's reduction partials
};

// Optional event pair recorded around one stage (profiling).
struct Bracket {
  int which = 0;                   // 0 none, 1 x sweep, 2 y sweep, 3 whole stage
  hipEvent_t ev[2] = {nullptr, nullptr};
};

using StageFn = void (*)(const Group&, int stage, int swz, hipStream_t);
using RedFn = void (*)(const Group&, double* part, hipStream_t);

template <int N, int D, typename W>
void launch_x(const Group& G, int stage, int swz, hipStream_t s) {
  const int n = (int)G.ids.size();
  hipLaunchKernelGGL((k_sweep_x<N, D, W>), dim3(G.xs[n]), dim3(kBX), 0, s, G.desc,
                     G.xmap, n, stage, swz);
}

template <int N, typename W>
void launch_y(const Group& G, int stage, int swz, hipStream_t s) {
  const int n = (int)G.ids.size();
  hipLaunchKernelGGL((k_sweep_y<N, W>), dim3(G.ys[n]), dim3(kTX * kTY), 0, s, G.desc,
                     G.ymap, n, stage, swz);
}

template <int N, int D>
void launch_dt(const Group& G, double* part, hipStream_t s) {
  const int n = (int)G.ids.size();
  hipLaunchKernelGGL((k_dt<N, D>), dim3(G.rs[n]), dim3(kRedBlock), 0, s, G.desc, G.rmap,
                     n, part + G.part_off);
}

template <int N, int D>
void launch_diag(const Group& G, double* part, hipStream_t s) {
  const int n = (int)G.ids.size();
  hipLaunchKernelGGL((k_diag<N, D>), dim3(G.rs[n]), dim3(kRedBlock), 0, s, G.desc, G.rmap,
                     n, part + G.part_off * kDiagSlots);
}

struct Table {
  StageFn sx[kMaxN + 1][3][2] = {};
  StageFn sy[kMaxN + 1][2] = {};
  RedFn dt[kMaxN + 1][3] = {};
  RedFn diag[kMaxN + 1][3] = {};
};

template <int N>
void fill(Table& t) {
  t.sx[N][1][0] = launch_x<N, 1, double>;
  t.sx[N][1][1] = launch_x<N, 1, float>;
  t.sx[N][2][0] = launch_x<N, 2, double>;
  t.sx[N][2][1] = launch_x<N, 2, float>;
  t.sy[N][0] = launch_y<N, double>;
  t.sy[N][1] = launch_y<N, float>;
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
  std::vector<Group> groups;
  mp_weno_opts opt;
  hipStream_t stream = nullptr;
  double* dt = nullptr;       // n_inst
  double* t = nullptr;        // n_inst
  double* steps = nullptr;    // n_inst
  double* part = nullptr;     // reduction partials (kDiagSlots per chunk)
  double* diag = nullptr;     // n_inst * MP_DIAG_LEN
  int swz = -1;               // XCD-aware tile order: 1 on, 0 off, -1 on for
                              // groups of several instances (measured: it
                              // keeps each small instance on one L2 and costs
                              // a few percent on a single grid)
  hipGraphExec_t graph[2] = {nullptr, nullptr};   // [external dt?]
  std::string err;
  int profile = 0;            // Bracket::which
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

// one RK stage (s = 0, 1, 2) or L(U) (s = 3) of every group
static mp_status enqueue_stage(mp_weno_ctx* c, int s) {
  const Table& T = table();
  const int prec = c->opt.precision;
  Bracket br;
  const Bracket* b = s < 3 ? c->next_bracket(br) : nullptr;
  const int w = b ? b->which : 0;
  if (w == 1 || w == 3) HIPCHK(c, hipEventRecord(b->ev[0], c->stream));
  auto swz = [c](const Group& G) { return c->swz < 0 ? (G.ids.size() > 1 ? 1 : 0) : c->swz; };
  for (const Group& G : c->groups) T.sx[G.N][G.D][prec](G, s, swz(G), c->stream);
  if (w == 1) HIPCHK(c, hipEventRecord(b->ev[1], c->stream));
  if (w == 2) HIPCHK(c, hipEventRecord(b->ev[0], c->stream));
  for (const Group& G : c->groups)
    if (G.D == 2) T.sy[G.N][prec](G, s, swz(G), c->stream);
  if (w == 2 || w == 3) HIPCHK(c, hipEventRecord(b->ev[1], c->stream));
  HIPCHK(c, hipGetLastError());
  return MP_OK;
}

static mp_status enqueue_dt(mp_weno_ctx* c) {
  const Table& T = table();
  for (const Group& G : c->groups) {
    T.dt[G.N][G.D](G, c->part, c->stream);
    hipLaunchKernelGGL(k_dt_finish, dim3(G.ids.size()), dim3(kRedBlock), 0, c->stream,
                       G.desc, G.rstart, c->part + G.part_off, c->opt.cfl);
  }
  HIPCHK(c, hipGetLastError());
  return MP_OK;
}

static mp_status enqueue_rk(mp_weno_ctx* c) {
  for (int s = 0; s < 3; ++s) {
    mp_status st = enqueue_stage(c, s);
    if (st != MP_OK) return st;
  }
  const int n = (int)c->inst.size();
  hipLaunchKernelGGL(k_advance_time, dim3((n + 255) / 256), dim3(256), 0, c->stream, c->t,
                     c->steps, c->dt, n);
  HIPCHK(c, hipGetLastError());
  return MP_OK;
}

static mp_status enqueue_diag(mp_weno_ctx* c) {
  const Table& T = table();
  for (const Group& G : c->groups) {
    T.diag[G.N][G.D](G, c->part, c->stream);
    hipLaunchKernelGGL(k_diag_finish, dim3(G.ids.size()), dim3(64), 0, c->stream, G.desc,
                       G.rstart, c->part + G.part_off * kDiagSlots);
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
  for (auto& G : c->groups) {
    (void)hipFree(G.desc); (void)hipFree(G.xmap); (void)hipFree(G.ymap);
    (void)hipFree(G.rmap); (void)hipFree(G.rstart);
  }
  (void)hipFree(c->dt); (void)hipFree(c->t); (void)hipFree(c->steps); (void)hipFree(c->part);
  (void)hipFree(c->diag);
  delete c;
  return MP_OK;
}

static mp_status validate(int32_t n_inst, const mp_weno_instance* inst,
                          const mp_weno_opts* opt, void* hip_stream) {
  if (n_inst < 1 || !inst || !opt) return MP_ERR_ARG;
  if (opt->phase_field != 0) return MP_ERR_UNSUPPORTED;
  if (opt->precision != MP_PREC_FP64 && opt->precision != MP_PREC_MIXED) return MP_ERR_ARG;
  if (opt->recon < 0 || opt->recon > 1 || opt->flux < 0 || opt->flux > 1 ||
      opt->model < 0 || opt->model > 1 || !(opt->cfl > 0.0))
    return MP_ERR_ARG;
  if (opt->use_graph && !hip_stream) return MP_ERR_ARG;   // no capture on the null stream
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
    if (nc > ((int64_t)1 << 31) - 1) return MP_ERR_UNSUPPORTED;
  }
  return MP_OK;
}

mp_status mp_weno_init(mp_weno_ctx** out, int32_t n_inst,
                       const mp_weno_instance* inst, const mp_weno_opts* opt,
                       void* hip_stream) {
  if (!out) return MP_ERR_ARG;
  *out = nullptr;
  const mp_status v = validate(n_inst, inst, opt, hip_stream);
  if (v != MP_OK) return v;

  mp_weno_ctx* c = new (std::nothrow) mp_weno_ctx();
  if (!c) return MP_ERR_OOM;
  c->opt = *opt;
  c->stream = (hipStream_t)hip_stream;
  const char* sw = std::getenv("MPWENO_XCD_SWIZZLE");
  if (sw) c->swz = std::atoi(sw) ? 1 : 0;
  const size_t n = (size_t)n_inst;
  if (hipMalloc(&c->dt, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&c->t, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&c->steps, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&c->diag, sizeof(double) * n * MP_DIAG_LEN) != hipSuccess) {
    mp_weno_destroy(c);
    return MP_ERR_OOM;
  }
  for (int i = 0; i < n_inst; ++i) {
    Inst I;
    I.in = inst[i];
    I.N = inst[i].nphase;
    I.D = inst[i].ndim;
    I.nU = 2 * I.N + I.D + 1;
    I.nc = (int64_t)inst[i].n[0] * (I.D > 1 ? inst[i].n[1] : 1);
    const size_t bytes = sizeof(double) * (size_t)I.nU * (size_t)I.nc;
    const bool ok = hipMalloc(&I.U1, bytes) == hipSuccess &&
                    hipMalloc(&I.U2, bytes) == hipSuccess &&
                    (I.D == 1 || hipMalloc(&I.acc, bytes) == hipSuccess) &&
                    (!opt->check_bounds || hipMalloc(&I.backup, bytes) == hipSuccess);
    c->inst.push_back(I);
    if (!ok) {
      mp_weno_destroy(c);
      return MP_ERR_OOM;
    }
  }

  // group by (N, d); larger instances first inside a group
  size_t part_total = 0;
  for (int D = 1; D <= 2; ++D)
    for (int N = 1; N <= kMaxN; ++N) {
      Group G;
      G.N = N;
      G.D = D;
      for (int i = 0; i < n_inst; ++i)
        if (c->inst[i].N == N && c->inst[i].D == D) G.ids.push_back(i);
      if (G.ids.empty()) continue;
      std::stable_sort(G.ids.begin(), G.ids.end(), [&](int a, int b) {
        return c->inst[a].nc > c->inst[b].nc;
      });
      G.xs.push_back(0); G.ys.push_back(0); G.rs.push_back(0);
      for (int id : G.ids) {
        const Inst& I = c->inst[id];
        const mp_weno_instance& s = I.in;
        Desc d;
        std::memset(&d, 0, sizeof(d));
        Grid& g = d.g;
        g.nx = s.n[0];
        g.ny = I.D > 1 ? s.n[1] : 1;
        g.nc = I.nc;
        g.rdx = 1.0 / s.dx[0];
        g.hdx = 0.5 * s.dx[0];
        g.rdy = I.D > 1 ? 1.0 / s.dx[1] : 0.0;
        g.hdy = I.D > 1 ? 0.5 * s.dx[1] : 1.0;
        g.bcx0 = s.bc[0][0]; g.bcx1 = s.bc[0][1];
        g.bcy0 = I.D > 1 ? s.bc[1][0] : 0;
        g.bcy1 = I.D > 1 ? s.bc[1][1] : 0;
        g.recon = opt->recon;
        g.flux = opt->flux;
        g.model = opt->model;
        g.energy = opt->energy_limiter ? 1 : 0;
        for (int p = 0; p < I.N; ++p) {
          const double gm = s.gamma[p], pi = s.pinf[p];
          d.e.A[p] = 1.0 / (gm - 1.0);
          d.e.B[p] = gm * pi / (gm - 1.0);
          d.e.Dp[p] = s.D[p];
          d.e.gam[p] = gm;
          d.e.pinf[p] = pi;
          d.e.EB[p] = d.e.A[p] * s.pmin[p] + d.e.B[p];
        }
        d.U = s.U;
        d.U1 = I.U1;
        d.U2 = I.U2;
        d.acc = I.acc;
        d.dt = c->dt + id;
        d.t = c->t + id;
        d.steps = c->steps + id;
        d.diag = c->diag + (size_t)id * MP_DIAG_LEN;
        d.t_end = s.t_end;
        d.vol = 1.0;
        for (int k = 0; k < I.D; ++k) d.vol *= s.dx[k];
        G.hdesc.push_back(d);
        const int64_t nstrip = (g.nx + kBX - 3) / (kBX - 2);
        const int64_t nty = I.D > 1 ? (int64_t)((g.nx + kTX - 1) / kTX) * ((g.ny + kOY - 1) / kOY) : 0;
        const int64_t nx = G.xs.back() + g.ny * nstrip;
        const int64_t ny = G.ys.back() + nty;
        const int64_t nr = G.rs.back() + (I.nc + kRedChunk - 1) / kRedChunk;
        if (std::max(nx, std::max(ny, nr)) > (int64_t)INT32_MAX) {
          mp_weno_destroy(c);
          return MP_ERR_UNSUPPORTED;     // more tiles than one launch can index
        }
        G.xs.push_back((int)nx);
        G.ys.push_back((int)ny);
        G.rs.push_back((int)nr);
      }
      G.part_off = part_total;
      part_total += (size_t)G.rs.back();
      const size_t m = G.ids.size();
      auto tile_map = [m](const std::vector<int>& st) {
        std::vector<int2> v((size_t)st[m]);
        for (size_t k = 0; k < m; ++k)
          for (int j = st[k]; j < st[k + 1]; ++j) v[(size_t)j] = make_int2((int)k, j - st[k]);
        return v;
      };
      const std::vector<int2> xm = tile_map(G.xs), ym = tile_map(G.ys), rm = tile_map(G.rs);
      bool ok = hipMalloc(&G.desc, sizeof(Desc) * m) == hipSuccess &&
                hipMalloc(&G.xmap, sizeof(int2) * std::max<size_t>(xm.size(), 1)) == hipSuccess &&
                hipMalloc(&G.ymap, sizeof(int2) * std::max<size_t>(ym.size(), 1)) == hipSuccess &&
                hipMalloc(&G.rmap, sizeof(int2) * std::max<size_t>(rm.size(), 1)) == hipSuccess &&
                hipMalloc(&G.rstart, sizeof(int) * (m + 1)) == hipSuccess;
      c->groups.push_back(G);
      if (!ok) {
        mp_weno_destroy(c);
        return MP_ERR_OOM;
      }
      Group& H = c->groups.back();
      if (hipMemcpy(H.desc, H.hdesc.data(), sizeof(Desc) * m, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(H.xmap, xm.data(), sizeof(int2) * xm.size(), hipMemcpyHostToDevice) != hipSuccess ||
          (!ym.empty() &&
           hipMemcpy(H.ymap, ym.data(), sizeof(int2) * ym.size(), hipMemcpyHostToDevice) != hipSuccess) ||
          hipMemcpy(H.rmap, rm.data(), sizeof(int2) * rm.size(), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(H.rstart, H.rs.data(), sizeof(int) * (m + 1), hipMemcpyHostToDevice) != hipSuccess) {
        mp_weno_destroy(c);
        return MP_ERR_HIP;
      }
    }
  if (hipMalloc(&c->part, sizeof(double) * std::max<size_t>(part_total, 1) * kDiagSlots) != hipSuccess) {
    mp_weno_destroy(c);
    return MP_ERR_OOM;
  }
  std::vector<double> zeros(n, 0.0);
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
  for (size_t i = 0; i < c->inst.size(); ++i)
    if (!dUdt[i]) return fail(c, MP_ERR_ARG, "null output pointer");
  // the descriptor tables carry the input/output pointers of this call
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (Group& G : c->groups) {
    for (size_t k = 0; k < G.ids.size(); ++k) {
      const int id = G.ids[k];
      G.hdesc[k].rin = (U_in && U_in[id]) ? U_in[id] : c->inst[id].in.U;
      G.hdesc[k].rout = dUdt[id];
    }
    HIPCHK(c, hipMemcpy(G.desc, G.hdesc.data(), sizeof(Desc) * G.ids.size(),
                        hipMemcpyHostToDevice));
  }
  return enqueue_stage(c, 3);
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
