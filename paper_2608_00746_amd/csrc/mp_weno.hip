// mp_weno.hip -- kernels, host runtime and C ABI of the MI355X WENO-C / WENO-CL
// hyperbolic step (declared in include/mp_weno.h).
//
// Instances with the same (N, d) form a group.  Each group has a device table
// of instance descriptors (grid, EOS, buffer pointers), and every kernel
// launch covers all tiles of all instances of the group: a workgroup finds its
// instance by binary search over per-instance tile offsets, so a batch of
// uneven instances is one launch per sweep.  One RK stage of a d-dimensional
// group is d launches:
//   k_sweep_x : one workgroup per (instance, strip of up to 254 cells of its
//               rows laid end to end, each row with its ghost cells).
//               Each lane converts one cell to primitives into an LDS row,
//               reconstructs its cell along x from the five LDS neighbours,
//               trades its minus-side face state with the left neighbour
//               through LDS, computes the flux of its plus-side face, trades
//               fluxes, and writes the x part of L(U) to a direction
//               accumulator (1D: finishes the RK stage directly).
//   k_sweep_t : the same exchange pattern along y (2D, 3D) or z (3D) on
//               16 x 16 tiles of lanes in one plane (one cell per lane,
//               neighbours along the sweep through LDS, 128-byte row
//               segments); it adds its part to the accumulator, and the last
//               direction applies the RK stage.
// Every sweep reads the same stage state (unsplit, dimension by dimension).
// Workgroup indices can be remapped so that consecutive tiles (which share
// halo rows) run on the same XCD and its L2.  The CFL step and the
// diagnostics are per-instance reductions with a fixed order (no
// floating-point atomics), so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mp_weno.h"
#include "weno_device.h"

namespace mpw {

constexpr int kMaxN = 8;          // phases built
constexpr int kMaxNT = 5;         // phases built with every tile shape (above: the defaults)
constexpr int kMaxN3 = 3;         // phases built in 3D
// Tile shapes (chosen per group by mp_weno_autotune; index 0 is the default):
// x sweep strips of kXS[v] lanes (at most kXS[v] - 2 output cells), y and z sweep
// tiles of kYX[v] x kYY[v] lanes (kYY[v] - 2 output lines; one shape for both
// in 3D).  The Phase-Field sweeps use
// the defaults.
constexpr int kXVar = 3, kYVar = 3;
constexpr int kXS[kXVar] = {256, 128, 64};
constexpr int kYX[kYVar] = {16, 32, 16};
constexpr int kYY[kYVar] = {16, 8, 24};
constexpr int kRedBlock = 256;    // reduction workgroup
constexpr int kDiagSlots = 34;    // per-block partials of the diagnostics
constexpr int kPartSlots = 88;    // partial slots per reduction chunk (stored slot-major:
                                  // slot k of chunk b at k * Desc::ps + b)
static_assert(kDiagSlots <= MP_DIAG_LEN && MP_DIAG_LEN <= 64, "diagnostic slots (finisher of 64 lanes)");
static_assert(kPartSlots >= kDiagSlots && kPartSlots >= 1 + kMaxN * kMaxN + 2 * kMaxN &&
                  kPartSlots >= 6 * kMaxN,
              "partial slots of the widest reduction (the Phase-Field integrands)");
// per-instance Phase-Field scalars (offsets into Desc::pfs): mobility,
// M / eta^2, multipliers B_q, CG iterations and relative residual at exit,
// the multigrid correction scale, and per phase ||b||^2, res.z, alpha, beta,
// done flag, iterations, mean of the preconditioned residual, true relative
// residual at the previous start, the run's best recurrence residual and the
// iteration it was reached at
constexpr int kPfsLen = 96;
constexpr int kPfFields = 10;     // Phase-Field work arrays of N fields each
// floor of k = phi (1 - phi) in Eq. (4): the equation then joins all cells,
// is solvable for every right side of zero total and stays conditioned; only
// cells with phi or 1 - phi below ~1e-6 see it
constexpr double kKFloor = 1e-6;
// the Phase-Field step's own CFL bound: |G_d| dt / dx_d <= 1/12 (the
// Gauss-Lobatto end weight); the solve's gradient is clipped there, which
// only happens in nearly pure cells where the capped flux is negligible
constexpr double kPfCfl = 1.0 / 12.0;
// Scale of the multigrid coarse-grid correction at the start of every solve:
// the piecewise-constant prolongation of an aggregation hierarchy undershoots
// the smooth error by about 2x per level, and over-correcting cuts the CG
// iterations of the Q solve 3-4x.  The cycle stays symmetric, but repeated
// over-correction down the levels can cost definiteness; a CG breakdown
// drops the scale to 1 (the plain V-cycle, positive definite) and restarts.
constexpr double kMgCorr = 1.8;
constexpr int kPfsM = 0, kPfsMe2 = 1, kPfsB = 2, kPfsIts = 10, kPfsRes = 11,
              kPfsCorr = 12, kPfsBB = 16, kPfsRZ = 24, kPfsAlpha = 32, kPfsBeta = 40,
              kPfsDone = 48, kPfsPits = 56, kPfsUbar = 64, kPfsPrev = 72,
              kPfsBest = 80, kPfsBestIt = 88;
// a run whose recurrence residual is within kPfsStallTol cg_rtol and has not
// halved for kPfsStallIts iterations has stagnated at the attainable accuracy:
// it ends, and the next start pass judges the true residual.  With the FP32
// preconditioner the attainable relative residual sits near 1e-9 on
// high-contrast states (the Sec. 4.2.1 cavity with the Kapila model stalls at
// 1.0e-9 .. 1.5e-9 over 16 restarts); the Phase-Field flux it sets moves by
// that fraction of itself
constexpr double kPfsStallTol = 1e4;
constexpr double kPfsStallIts = 50.0;

// The state pointers come from a table in device memory, so the compiler
// cannot tell their address space and would emit flat loads and stores (which
// also count against the LDS wait counter).  They always point to global
// memory; these types say so.
using gdouble = __attribute__((address_space(1))) double;
using lds_void = __attribute__((address_space(3))) void;   // LDS destination of global_load_lds
using gfloat = __attribute__((address_space(1))) float;
__device__ __forceinline__ const gdouble* gptr(const double* p) { return (const gdouble*)p; }
__device__ __forceinline__ gdouble* gptr(double* p) { return (gdouble*)p; }
__device__ __forceinline__ const gfloat* gptr(const float* p) { return (const gfloat*)p; }
__device__ __forceinline__ gfloat* gptr(float* p) { return (gfloat*)p; }

struct StageArgs {
  const gdouble* Uk;  // stage state (stencils)
  const gdouble* Un;  // state at the start of the step (RK base)
  gdouble* out;       // U^(k+1), or L(U) when mode == 0
  gdouble* acc;       // x part of L (2D)
  const gdouble* dt;  // device time step of this instance
  double a, b;        // out = a Un + b (Uk + dt L)
  int mode;           // 0: write L, 1: RK stage
};

// One level of the multigrid preconditioner of Eq. (4) for one instance
// (every array holds the N phases one after the other, [N][nc]).  Level 0 is
// the grid itself; level l + 1 aggregates 2 x 2 (3D: 2 x 2 x 2) cells of
// level l (a single cell or row at an odd end) down to one cell.  The preconditioner works in
// FP32 (half the bytes of every pass; CG, its residual and the convergence
// test stay FP64): level 0 reads the FP64 CG residual once, scaled by a power
// of two near the rms of [div J_p] (exact, and far from the FP32 range
// limits), and writes the FP64 preconditioned residual once, scaled back.
struct MgLevel {
  int nx, ny, nz;
  int64_t nc;
  float* wx;         // weight of the face to the +x neighbour (0: no face)
  float* wy;         // weight of the face to the +y neighbour
  float* wz;         // weight of the face to the +z neighbour (3D)
  float* dg;         // diagonal: sum of the cell's face weights
  float* e;          // correction
  float* t;          // Jacobi ping-pong
  float* f;          // right-hand side (level 0: the scaled CG residual)
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
  int64_t ps;                // slot stride of the reduction partials
  int64_t chunk;             // cells per reduction workgroup
  // Phase-Field step (null when it is off)
  const double* pfin;        // state whose volume fractions are phi_p
  double* pfs;               // per-instance scalars (kPfs* offsets)
  double* pf_k;              // k_p = phi_p (1 - phi_p)            [N][cells]
  double* pf_b;              // [div J_p] (right side of Eq. (4))  [N][cells]
  double* pf_q;              // Q_p                                [N][cells]
  double* pf_r;              // CG residual                        [N][cells]
  double* pf_p;              // CG direction                       [N][cells]
  double* pf_ap;             // CG s = K p                         [N][cells]
  double* pf_w;              // CG w = K u                         [N][cells]
  double* pf_u;              // preconditioned residual u = M^-1 r [N][cells]
  double* pf_qp;             // Q_p of the solve before the last   [N][cells]
  double* pf_qpp;            // and of the one before that         [N][cells]
  const struct MgLevel* mg;  // multigrid levels of the preconditioner
  int nlev;
  double* pf_g;              // dQ_p/dx_d at upper faces           [d][N][cells]
  double eta;                // interface thickness parameter
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

// Work item of a Phase-Field pass over chunks of cells: consecutive chunks
// (rows and their neighbour rows, which the stencils read) run on one XCD and
// share its L2.  Partial sums stay in the item's slot, so the order of every
// reduction is that of the items.
__device__ __forceinline__ int chunk_item() {
  return xcd_item((int)blockIdx.x, (int)gridDim.x, 1);
}

__device__ __forceinline__ int bc_map(int i, int n, int lo, int hi) {
  if (i < 0) {
    if (lo == MP_BC_PERIODIC) return ((i % n) + n) % n;
    if (lo == MP_BC_SYMMETRY) return min(-1 - i, n - 1);
    return 0;
  }
  if (i >= n) {
    if (hi == MP_BC_PERIODIC) return i % n;
    if (hi == MP_BC_SYMMETRY) return max(2 * n - 1 - i, 0);
    return n - 1;
  }
  return i;
}

// true when bc_map(i) is the mirror image across a symmetry plane: the
// stand-in cell's normal momentum then changes sign
__device__ __forceinline__ bool bc_mirror(int i, int n, int lo, int hi) {
  return (i < 0 && lo == MP_BC_SYMMETRY) || (i >= n && hi == MP_BC_SYMMETRY);
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

// RK epilogue for one cell: L in component order; writes out (U^n of the
// cell read through un(c), in stages that need it).
template <int N, int D, typename UnF>
__device__ __forceinline__ void finish_cell(const StageArgs& a, int64_t nc,
                                            int64_t idx, const Cons<N, D>& uk,
                                            const double* L, UnF un) {
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
    for (int c = 0; c < NU; ++c) a.out[(int64_t)c * nc + idx] = a.a * un(c) + a.b * (u[c] + dt * L[c]);
  }
}

// the same with U^n read from the stage arguments
template <int N, int D>
__device__ __forceinline__ void finish_cell(const StageArgs& a, int64_t nc,
                                            int64_t idx, const Cons<N, D>& uk,
                                            const double* L) {
  finish_cell<N, D>(a, nc, idx, uk, L, [&](int c) { return a.Un[(int64_t)c * nc + idx]; });
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// sum_d (|u_d| + c) / dx_d of a cell: the CFL rate of its cell average
// (contraction off: the x sweep's first stage computes it too, and the two
// must agree to the bit)
template <int N, int D>
__device__ __forceinline__ double cfl_rate(const Prim<N, D>& v, const Eos& e, const Grid& g) {
#pragma clang fp contract(off)
  double rho = 0.0;
#pragma unroll
  for (int p = 0; p < N; ++p) rho += v.m[p];
  double num, den;
  mix_rc2_parts<N>(v.a, v.P, e, g.model, num, den);
  const double cs = sound_speed(num, den, rho);
  double s = (fabs(v.u[0]) + cs) * g.rdx;
  if constexpr (D > 1) s += (fabs(v.u[1]) + cs) * g.rdy;
  if constexpr (D > 2) s += (fabs(v.u[2]) + cs) * g.rdz;
  return s;
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

// ---------------------------------------------------------------------------
// x sweep
// ---------------------------------------------------------------------------
// Waves per SIMD the sweeps are compiled for: one or two phases fit 3 (or 4)
// waves in the register file with at most a few spilled values, which hides
// FP64 latency better than 2 waves (measured +7..10 % on N = 2 in 2D); the x
// sweep of three phases in 2D on the mixed path also runs at 3 (spilling
// some values: +2 % on the batch; the transverse sweep's LDS allows only 2
// there); two phases in 3D, three and four phases otherwise would spill
// heavily at 3 and keep 2; five need the AGPRs too.
// The flux and reconstruction variants of the sweeps (template PFM):
// kRiemann: Riemann flux, WENO-C / WENO-CL; kPfFlux: the Phase-Field flux
// (any reconstruction); kRiemannCmp: Riemann flux with the comparison
// schemes (WENO-JS, WENO-W).
constexpr int kRiemann = 0, kPfFlux = 1, kRiemannCmp = 2;
template <int PFM>
constexpr int kRecon() {
  return PFM == kRiemann ? kReconC : (PFM == kRiemannCmp ? kReconCmp : kReconAny);
}

template <int N, int D, typename W, int PFM, bool XSWEEP>
constexpr int sweep_waves() {
  if (N == 3 && D == 2 && sizeof(W) == 4 && PFM == 0 && XSWEEP) return 3;
  return N == 1 ? (D == 1 ? 4 : 3) : (N == 2 ? (D == 3 ? 2 : 3) : (N <= 4 ? 2 : 1));
}

// v of lane l + 1 (SHL) or lane l - 1 (SHR) of the wave (DPP wave shift by
// one lane); the lane at the wave's end keeps its own value
template <bool SHL>
__device__ __forceinline__ double lane_shift(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
  constexpr int ctrl = SHL ? 0x130 : 0x138;      // wave_shl:1 / wave_shr:1
  const int rlo = __builtin_amdgcn_update_dpp(lo, lo, ctrl, 0xf, 0xf, false);
  const int rhi = __builtin_amdgcn_update_dpp(hi, hi, ctrl, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)rhi << 32) |
                                          (unsigned long long)(unsigned)rlo));
}

template <int N, int D>
__device__ __forceinline__ void shift_face_left(Face<N, D>& f) {
#pragma unroll
  for (int p = 0; p < N; ++p) { f.m[p] = lane_shift<true>(f.m[p]); f.a[p] = lane_shift<true>(f.a[p]); }
#pragma unroll
  for (int k = 0; k < D; ++k) { f.mom[k] = lane_shift<true>(f.mom[k]); f.u[k] = lane_shift<true>(f.u[k]); }
  f.E = lane_shift<true>(f.E);
  f.P = lane_shift<true>(f.P);
  f.rho = lane_shift<true>(f.rho);
  f.c = lane_shift<true>(f.c);
}

template <int N, int D, typename W, int PFM, int BX>
__global__ __attribute__((amdgpu_flat_work_group_size(1, BX),
                          amdgpu_waves_per_eu(sweep_waves<N, D, W, PFM, true>(), 8)))
void k_sweep_x(const Desc* __restrict__ descs,
                                                 const int2* __restrict__ map,
                                                 int ninst, int stage, int swz,
                                                 double* __restrict__ cflp) {
  const int item = xcd_item(blockIdx.x, gridDim.x, swz);
  const int2 it = locate(map, ninst, item);
  const Desc d = descs[it.x];   // by value: loaded once, kept in registers
  const Grid& g = d.g;
  const Eos& e = d.e;
  const StageArgs a = stage_args(d, stage);
  // an instance whose step is 0 (retired at its end time) is left as it is;
  // with cflp (the first stage of a step in 2D and 3D) the step is not known
  // yet: the sweep reduces the CFL rate of its output cells (of U^n) into
  // cflp[item], from which the step is taken before the transverse sweeps
  if (!cflp && a.mode == 1 && *a.dt == 0.0) return;
  constexpr int NV = 2 * N + D + 1;
  constexpr int NU = NV;
  constexpr int NF = 2 * N + 2 * D + 4;
  constexpr int NFL = NU + 1;
  // the flux rows reuse the primitive rows: the stencil is in registers and
  // a barrier (after the face exchange) separates the two uses
  // a strip of one wave trades face states and fluxes by DPP lane shifts
  // (no LDS, no barrier); wider strips through LDS
  constexpr bool kOneWave = BX == 64 && PFM != kPfFlux;
  constexpr int NPRIM = NV * (BX + 4), NFLX = kOneWave ? 0 : NFL * BX;
  __shared__ double sraw[NPRIM > NFLX ? NPRIM : NFLX];
  __shared__ double sface[kOneWave ? 1 : NF][BX];
  double (*sprim)[BX + 4] = reinterpret_cast<double (*)[BX + 4]>(sraw);
  double (*sflux)[BX] = reinterpret_cast<double (*)[BX]>(sraw);

  // The rows (ny nz of them) are laid end to end, each with its three ghost
  // cells on either side (nx + 6 cells a row), and cut into strips of BX
  // lanes that overlap by two: lane l of strip s holds cell v = s (BX - 2)
  // - 1 + l of that sequence and its neighbours along x are lanes l -+ 1.
  // Lanes 1 .. BX - 2 whose cell is a grid cell are the strip's outputs;
  // ghost cells stand in for the end conditions (every lane's reconstruction
  // of a grid or first ghost cell reads its own row only), and cells past
  // the last row are computed and dropped.  So a row shorter than a strip
  // leaves few of its lanes idle (six per row, two per strip).
  const int l = threadIdx.x;
  const int lw = g.nx + 6;
  const int64_t nc = g.nc;
  const int64_t v0 = (int64_t)it.y * (BX - 2) - 1;
  // uniform over the strip: the row of its first cell, and the base row of
  // its loads and stores (one row earlier, where the first ghost cells may
  // lie), so that every lane addresses base + a 32-bit offset
  const int64_t yb = v0 > 0 ? v0 / lw : 0;
  const int dv0 = (int)(v0 - yb * lw);                  // in [-1, lw)
  const int ylo = yb > 0 ? -1 : 0;                      // base row - yb
  const int yhi = (int)std::min<int64_t>((int64_t)g.ny * g.nz - 1 - yb, INT32_MAX / 2);
  const int64_t row = (yb + ylo) * g.nx;
  // cell k of the strip (lanes 0 .. BX - 1 are k = 0 .. BX - 1, their
  // ghost cells k = -2, -1, BX, BX + 1): its x and the offset of its row
  // from the base row; the row is clamped to the grid (x then lies outside
  // it, and the end conditions map it)
  auto cell_of = [&](int k, int& rx) -> int {
    const int dv = dv0 + k;                             // >= -3
    int r = dv >= 0 ? (int)((unsigned)dv / (unsigned)lw) : -1;
    r = r < -yb ? (int)-yb : (r > yhi ? yhi : r);
    rx = dv - r * lw - 3;
    return (r - ylo) * g.nx;
  };
  int xi;
  const int roff = cell_of(l, xi);

  auto put_prim = [&](int k, int slot) {
    int x;
    const int ro = cell_of(k, x);
    const int xm = bc_map(x, g.nx, g.bcx0, g.bcx1);
    Cons<N, D> c;
    load_cons<N, D>(a.Uk, nc, row + (unsigned)(ro + xm), c);
    if (bc_mirror(x, g.nx, g.bcx0, g.bcx1)) c.mom[0] = -c.mom[0];
    Prim<N, D> v;
    cons_to_prim<N, D>(c, e, v);
#pragma unroll
    for (int p = 0; p < N; ++p) { sprim[p][slot] = v.m[p]; sprim[N + p][slot] = v.a[p]; }
#pragma unroll
    for (int k2 = 0; k2 < D; ++k2) sprim[2 * N + k2][slot] = v.u[k2];
    sprim[2 * N + D][slot] = v.P;
  };

  const int xm = bc_map(xi, g.nx, g.bcx0, g.bcx1);
  Cons<N, D> ub;
  load_cons<N, D>(a.Uk, nc, row + (unsigned)(roff + xm), ub);
  if (bc_mirror(xi, g.nx, g.bcx0, g.bcx1)) ub.mom[0] = -ub.mom[0];
  const bool own = l >= 1 && l < BX - 1 && xi >= 0 && xi < g.nx;   // an output cell
  double rate = 0.0;
  {
    Prim<N, D> v;
    cons_to_prim<N, D>(ub, e, v);
    if (cflp && own) rate = cfl_rate<N, D>(v, e, g);
#pragma unroll
    for (int p = 0; p < N; ++p) { sprim[p][l + 2] = v.m[p]; sprim[N + p][l + 2] = v.a[p]; }
#pragma unroll
    for (int k = 0; k < D; ++k) sprim[2 * N + k][l + 2] = v.u[k];
    sprim[2 * N + D][l + 2] = v.P;
  }
  if (l < 2) put_prim(l - 2, l);
  if (l >= BX - 2) put_prim(l + 2, l + 4);
  if (cflp) {
    __shared__ double scfl[BX / 64];
    const double r = block_max(rate, scfl);
    if (l == 0) cflp[item] = r;
  }
  __syncthreads();

  Face<N, D> fm, fp;
  reconstruct<N, D, W, kRecon<PFM>()>([&](int c, int j) { return sprim[c][l + j]; }, ub, e, g,
                                      g.hdx, fm, fp);

  Flux<N, D> F;
  double Fl[NFL];            // the flux of face xi - 1/2 (one-wave strips)
  if constexpr (kOneWave) {
    Face<N, D> R = fm;
    shift_face_left<N, D>(R);            // the minus-side face of lane l + 1
    riemann<N, D, W>(fp, R, 0, g.flux, F);
#pragma unroll
    for (int c = 0; c < NU; ++c) Fl[c] = lane_shift<false>(F.f[c]);
    Fl[NU] = lane_shift<false>(F.uh);
  } else {
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

  if (l < BX - 1) {
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
    if constexpr (PFM == kPfFlux) {
      // gradient at face x_{xi+1/2}: face -1/2 is face n-1/2 when periodic
      // and carries none at an outflow end
      const int xo = xi < 0 ? (g.bcx0 == MP_BC_PERIODIC ? g.nx - 1 : -1) : (xi < g.nx ? xi : -1);
      const int xq = xo < 0 ? -1 : (xo + 1 < g.nx ? xo + 1 : (g.bcx1 == MP_BC_PERIODIC ? 0 : -1));
      double G[N], kf[N];
#pragma unroll
      for (int p = 0; p < N; ++p) {
        const bool in = xq >= 0;
        G[p] = in ? gptr(d.pf_g)[(int64_t)p * nc + row + (unsigned)(roff + xo)] : 0.0;
        kf[p] = in ? 0.5 * (gptr(d.pf_k)[(int64_t)p * nc + row + (unsigned)(roff + xo)] +
                            gptr(d.pf_k)[(int64_t)p * nc + row + (unsigned)(roff + xq)]) : 0.0;
      }
      pf_flux<N, D>(fp, R, G, kf, e, F);
    } else {
      riemann<N, D, W>(fp, R, 0, g.flux, F);
    }
#pragma unroll
    for (int c = 0; c < NU; ++c) sflux[c][l] = F.f[c];
    sflux[NU][l] = F.uh;
  }
  __syncthreads();
  }
  // the flux of face xi - 1/2, component c (NU: u-hat)
  auto fleft = [&](int c) -> double {
    if constexpr (kOneWave) return Fl[c];
    else return sflux[c][l - 1];
  };

  if (own) {
    double L[NU];
    if constexpr (PFM == kPfFlux) {
#pragma unroll
      for (int c = 0; c < NU; ++c) L[c] = (F.f[c] - fleft(c)) * g.rdx;
    } else {
      double opk[N];
      one_plus_k<N, D>(ub, e, g.model, opk);
#pragma unroll
      for (int c = 0; c < NU; ++c) L[c] = -(F.f[c] - fleft(c)) * g.rdx;
      const double du = (F.uh - fleft(NU)) * g.rdx;
      // alpha_p at the cell average, or alpha_p / sum_q alpha_q (then the
      // sources sum to du, as the fluxes' alpha parts do, and
      // sum_q alpha_q - 1 gets no source of its own)
      double isa = 1.0;
      if (g.asrc) {
        double sa = 0.0;
#pragma unroll
        for (int p = 0; p < N; ++p) sa += ub.a[p];
        isa = sa > 0.0 ? 1.0 / sa : 0.0;
      }
#pragma unroll
      for (int p = 0; p < N; ++p) L[N + D + 1 + p] += ub.a[p] * isa * opk[p] * du;
    }
    const int64_t idx = row + (unsigned)(roff + xi);
    if constexpr (D == 1) {
      finish_cell<N, D>(a, nc, idx, ub, L);
    } else {
#pragma unroll
      for (int c = 0; c < NU; ++c) a.acc[(int64_t)c * nc + idx] = L[c];
    }
  }
}

// ---------------------------------------------------------------------------
// transverse sweeps: y (2D, 3D) and z (3D), RK epilogue in the last one
// ---------------------------------------------------------------------------
// A workgroup is a tile of kTX columns x kTY lines of lanes in one plane,
// one cell per lane (lane (tx, ty) holds cell (x0 + tx, l0 - 1 + ty) of the
// sweep direction DIR); lines l0 .. l0 + kTY - 3 are its outputs.
// Primitives of lines l0 - 3 .. l0 + kTY go to LDS (each line segment is kTX
// x-contiguous doubles per component, one 128-byte line), every lane
// reconstructs its cell along DIR from its column, and face states and
// fluxes are traded with the neighbour line through LDS, as in the x sweep.
// The plane: the whole grid in 2D; a z plane for the y sweep and a y plane
// for the z sweep in 3D.  Sweeps before the last add their part of L into
// the accumulator; the last one finishes the RK stage.

template <int N, typename W, int PFM, int kTX, int kTY, int D, int DIR>
__global__ __attribute__((amdgpu_flat_work_group_size(1, kTX * kTY),
                          amdgpu_waves_per_eu(sweep_waves<N, D, W, PFM, false>(), 8)))
void k_sweep_t(const Desc* __restrict__ descs,
                                                       const int2* __restrict__ map,
                                                       int ninst, int stage, int swz) {
  static_assert(D >= 2 && DIR >= 1 && DIR < D, "sweep shape");
  constexpr bool kLast = DIR == D - 1;
  const int2 it = locate(map, ninst, xcd_item(blockIdx.x, gridDim.x, swz));
  const Desc d = descs[it.x];
  const Grid& g = d.g;
  const Eos& e = d.e;
  const StageArgs a = stage_args(d, stage);
  if (a.mode == 1 && *a.dt == 0.0) return;     // retired instance (step 0)
  constexpr int kOY = kTY - 2;      // output lines per tile
  // the sweep line: its length, stride, end conditions and spacing
  const int nl = DIR == 1 ? g.ny : g.nz;
  const int64_t ls = DIR == 1 ? (int64_t)g.nx : (int64_t)g.nx * g.ny;
  const int blo = DIR == 1 ? g.bcy0 : g.bcz0, bhi = DIR == 1 ? g.bcy1 : g.bcz1;
  const double rd = DIR == 1 ? g.rdy : g.rdz, hd = DIR == 1 ? g.hdy : g.hdz;
  const int ntx = (g.nx + kTX - 1) / kTX;
  const int per_plane = ntx * ((nl + kOY - 1) / kOY);
  const int plane = it.y / per_plane;
  const int local = it.y - plane * per_plane;
  // plane base: z plane of the y sweep (3D), y plane of the z sweep
  const int64_t pb = D == 2 ? 0 : (DIR == 1 ? (int64_t)plane * g.nx * g.ny : (int64_t)plane * g.nx);
  const int tyb = local / ntx, txb = local - tyb * ntx;
  constexpr int NV = 2 * N + D + 1;
  constexpr int NU = NV;
  constexpr int NF = 2 * N + 2 * D + 4;
  constexpr int NFL = NU + 1;
  // The primitive rows, then the minus-side face states, then the fluxes
  // share one LDS area, each phase separated from the next by a barrier;
  // the epilogue operands (the accumulator and, where the stage reads it,
  // U^n) of the output rows have an area of their own, filled while the
  // reconstruction runs.
  constexpr int NPRIM = NV * (kTY + 4) * kTX, NFACE = NF * kTY * kTX, NFLX = NFL * kTY * kTX;
  constexpr int NRAW = NPRIM > NFACE ? (NPRIM > NFLX ? NPRIM : NFLX) : (NFACE > NFLX ? NFACE : NFLX);
  __shared__ double sraw[NRAW];
  __shared__ double spre[2][NU][kOY][kTX];
  double (*sprim)[kTY + 4][kTX] = reinterpret_cast<double (*)[kTY + 4][kTX]>(sraw);
  double (*sface)[kTY][kTX] = reinterpret_cast<double (*)[kTY][kTX]>(sraw);
  double (*sflux)[kTY][kTX] = reinterpret_cast<double (*)[kTY][kTX]>(sraw);

  const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
  const int x = txb * kTX + tx;
  const bool colok = x < g.nx;
  const int xc = colok ? x : g.nx - 1;
  const int y0 = tyb * kOY;
  const int yi = y0 - 1 + ty;
  const int64_t nc = g.nc;

  auto put_prim = [&](int y, int slot) {
    const int ym = bc_map(y, nl, blo, bhi);
    Cons<N, D> c;
    load_cons<N, D>(a.Uk, nc, pb + (int64_t)ym * ls + xc, c);
    if (bc_mirror(y, nl, blo, bhi)) c.mom[DIR] = -c.mom[DIR];
    Prim<N, D> v;
    cons_to_prim<N, D>(c, e, v);
#pragma unroll
    for (int p = 0; p < N; ++p) { sprim[p][slot][tx] = v.m[p]; sprim[N + p][slot][tx] = v.a[p]; }
#pragma unroll
    for (int k = 0; k < D; ++k) sprim[2 * N + k][slot][tx] = v.u[k];
    sprim[2 * N + D][slot][tx] = v.P;
  };

  const int ym = bc_map(yi, nl, blo, bhi);
  Cons<N, D> ub;
  load_cons<N, D>(a.Uk, nc, pb + (int64_t)ym * ls + xc, ub);
  if (bc_mirror(yi, nl, blo, bhi)) ub.mom[DIR] = -ub.mom[DIR];
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

  // Epilogue operands of the tile's output rows straight into LDS
  // (global_load_lds, 4 bytes a lane, 32 doubles a wave): nothing is held in
  // registers while they are in flight, and the barrier after the
  // reconstruction waits for them.  Rows and columns beyond the grid load
  // its last row / column (in bounds; those cells are not written).
  const bool need_un = kLast && a.mode == 1 && a.a != 0.0;
  {
    constexpr int kRPL = 32 / kTX;            // rows per wave-load
    static_assert(32 % kTX == 0 && kOY % kRPL == 0, "prefetch shape");
    constexpr int kLPC = kOY / kRPL;          // wave-loads per component
    constexpr int kNW = kTX * kTY / 64;       // waves of the workgroup
    const int wave = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int dbl = ln >> 1;                  // double of this lane in a wave-load
    const int xq = min(txb * kTX + dbl % kTX, g.nx - 1);
    int64_t off[kLPC];
#pragma unroll
    for (int k = 0; k < kLPC; ++k)
      off[k] = pb + (int64_t)min(y0 + k * kRPL + dbl / kTX, nl - 1) * ls + xq;
    const int ncomp = need_un ? 2 * NU : NU;
    for (int q = wave; q < ncomp; q += kNW) {
      const int arr = q >= NU, c = q - arr * NU;
      const gdouble* arrp = arr ? a.Un : a.acc;
      const char* src = (const char*)(const double*)(arrp + (int64_t)c * nc);
#pragma unroll
      for (int k = 0; k < kLPC; ++k)
        __builtin_amdgcn_global_load_lds(src + off[k] * 8 + 4 * (ln & 1),
                                         (lds_void*)&spre[arr][c][k * kRPL][0], 4, 0, 0);
    }
  }

  Face<N, D> fm, fp;
  reconstruct<N, D, W, kRecon<PFM>()>([&](int c, int j) { return sprim[c][ty + j][tx]; }, ub, e,
                                      g, hd, fm, fp);
  __syncthreads();   // the primitive rows are read; the prefetch has landed

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
    if constexpr (PFM == kPfFlux) {
      // gradient at the upper face of line cell yi (as in the x sweep)
      const int yo = yi < 0 ? (blo == MP_BC_PERIODIC ? nl - 1 : -1) : (yi < nl ? yi : -1);
      const int yq = yo < 0 ? -1 : (yo + 1 < nl ? yo + 1 : (bhi == MP_BC_PERIODIC ? 0 : -1));
      const int64_t co = pb + (int64_t)yo * ls + xc, cq = pb + (int64_t)yq * ls + xc;
      double G[N], kf[N];
#pragma unroll
      for (int p = 0; p < N; ++p) {
        const bool in = yq >= 0;
        G[p] = in ? gptr(d.pf_g)[(int64_t)(DIR * N + p) * nc + co] : 0.0;
        kf[p] = in ? 0.5 * (gptr(d.pf_k)[(int64_t)p * nc + co] +
                            gptr(d.pf_k)[(int64_t)p * nc + cq]) : 0.0;
      }
      pf_flux<N, D>(fp, R, G, kf, e, F);
    } else {
      riemann<N, D, W>(fp, R, DIR, g.flux, F);
    }
  }
  __syncthreads();   // the face states are read
  if (ty < kTY - 1) {
#pragma unroll
    for (int c = 0; c < NU; ++c) sflux[c][ty][tx] = F.f[c];
    sflux[NU][ty][tx] = F.uh;
  }
  __syncthreads();

  if (ty >= 1 && ty < kTY - 1 && colok && yi < nl) {
    const int64_t idx = pb + (int64_t)yi * ls + x;
    double L[NU];
    if constexpr (PFM == kPfFlux) {
#pragma unroll
      for (int c = 0; c < NU; ++c)
        L[c] = spre[0][c][ty - 1][tx] + (F.f[c] - sflux[c][ty - 1][tx]) * rd;
    } else {
      double opk[N];
      one_plus_k<N, D>(ub, e, g.model, opk);
#pragma unroll
      for (int c = 0; c < NU; ++c)
        L[c] = spre[0][c][ty - 1][tx] - (F.f[c] - sflux[c][ty - 1][tx]) * rd;
      const double du = (F.uh - sflux[NU][ty - 1][tx]) * rd;
      // alpha_p at the cell average, or alpha_p / sum_q alpha_q (then the
      // sources sum to du, as the fluxes' alpha parts do, and
      // sum_q alpha_q - 1 gets no source of its own)
      double isa = 1.0;
      if (g.asrc) {
        double sa = 0.0;
#pragma unroll
        for (int p = 0; p < N; ++p) sa += ub.a[p];
        isa = sa > 0.0 ? 1.0 / sa : 0.0;
      }
#pragma unroll
      for (int p = 0; p < N; ++p) L[N + D + 1 + p] += ub.a[p] * isa * opk[p] * du;
    }
    if constexpr (kLast) {
      finish_cell<N, D>(a, nc, idx, ub, L, [&](int c) { return spre[1][c][ty - 1][tx]; });
    } else {
#pragma unroll
      for (int c = 0; c < NU; ++c) a.acc[(int64_t)c * nc + idx] = L[c];
    }
  }
}

// ---------------------------------------------------------------------------
// two-level coupling of batched instances (block-structured refinement)
// ---------------------------------------------------------------------------
// A fine instance covers a W x H block of cells of a coarse instance at
// refinement ratio 2 (Sec. 3.4.2: each level is a uniform grid the scheme
// runs on unchanged).  Its grid is the 2W x 2H refined block plus a ring of
// three ghost cells (the stencil reach), (2W + 6) x (2H + 6) cells.  Both
// levels take the same time step.  Per RK stage the ring is filled from the
// coarse stage state (each fine ghost cell takes its coarse parent's
// average: bounds, consistency m_p = rho_p alpha_p and uniform u, P carry
// over exactly), and the interface fluxes of both levels are evaluated from
// the stage states; after the step the coarse cells under the block take the
// average of their four children, the ring takes the new coarse values, and
// the coarse cells beside the block get
// the difference between the fine and coarse interface fluxes (the RK3
// weights 1/6, 1/6, 2/3 of the three stages) so that the composite grid
// conserves m_p, rho u and rho E exactly; the alpha source of those cells is
// corrected with the same face velocities so that sum_p alpha_p stays 1.
constexpr int kAmrHalo = 3;

struct AmrLink {
  double* fst[3];            // fine stage states U, U1, U2 (input of stage s)
  double* cst[3];            // coarse stage states
  Grid fg, cg;               // the two grids (scheme switches included)
  Eos e;
  int lox, loy, W, H;        // the block: coarse cells [lox, lox + W) x [loy, loy + H)
  int nface;                 // coarse faces on its boundary: 2H (+ 2W in 2D)
  double* flx;               // [nface][3][NU + 1]: coarse flux, two fine fluxes (+ u-hat)
  double* reg;               // [nface][NU]: correction of the outside coarse cell's L
  const double* dt;          // the (shared) time step
};

// coarse face f of the block's boundary: normal direction, the coarse cells
// on its minus and plus sides, which of them lies outside, and the fine
// cells on both sides of its k-th fine sub-face (k = 0, 1)
struct AmrFace {
  int dir;
  int cm[2], cp[2];          // coarse (x, y) of the minus / plus cell
  bool out_minus;            // the outside coarse cell is the minus cell
  int fm[2][2], fp[2][2];    // fine (x, y) of the minus / plus cell of sub-face k
};

__device__ __forceinline__ AmrFace amr_face(const AmrLink& L, int f) {
  AmrFace a;
  const int H = L.H, W = L.W, h = kAmrHalo;
  if (f < 2 * H) {                        // x faces: left (f < H) and right edges
    const bool left = f < H;
    const int J = L.loy + (left ? f : f - H);
    a.dir = 0;
    const int xm = left ? L.lox - 1 : L.lox + W - 1;
    a.cm[0] = xm; a.cm[1] = J; a.cp[0] = xm + 1; a.cp[1] = J;
    a.out_minus = left;
    const int fxm = left ? h - 1 : h + 2 * W - 1;
    for (int k = 0; k < 2; ++k) {
      const int fy = (L.fg.ny == 1) ? 0 : h + 2 * (J - L.loy) + k;
      a.fm[k][0] = fxm; a.fm[k][1] = fy; a.fp[k][0] = fxm + 1; a.fp[k][1] = fy;
    }
  } else {                                // y faces: bottom and top edges
    const bool bot = f < 2 * H + W;
    const int I = L.lox + (bot ? f - 2 * H : f - 2 * H - W);
    a.dir = 1;
    const int ym = bot ? L.loy - 1 : L.loy + H - 1;
    a.cm[0] = I; a.cm[1] = ym; a.cp[0] = I; a.cp[1] = ym + 1;
    a.out_minus = bot;
    const int fym = bot ? h - 1 : h + 2 * H - 1;
    for (int k = 0; k < 2; ++k) {
      const int fx = h + 2 * (I - L.lox) + k;
      a.fm[k][0] = fx; a.fm[k][1] = fym; a.fp[k][0] = fx; a.fp[k][1] = fym + 1;
    }
  }
  return a;
}

// halo cells: fine stage state <- the coarse parent's stage state
__global__ void k_amr_prolong(const AmrLink* __restrict__ links, int stage, int nU) {
  const AmrLink& L = links[blockIdx.y];
  const int fnx = L.fg.nx, fny = L.fg.ny, h = kAmrHalo;
  const int64_t fnc = L.fg.nc, cnc = L.cg.nc;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < fnc;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int fy = (int)(i / fnx), fx = (int)(i - (int64_t)fy * fnx);
    const bool inx = fx >= h && fx < fnx - h, iny = fny == 1 || (fy >= h && fy < fny - h);
    if (inx && iny) continue;
    // parent: floor((f - h) / 2) cells from the block's origin
    const int cx = L.lox + ((fx - h) >= 0 ? (fx - h) / 2 : -((h - fx + 1) / 2));
    const int cy = fny == 1 ? 0 : L.loy + ((fy - h) >= 0 ? (fy - h) / 2 : -((h - fy + 1) / 2));
    const int64_t ci = (int64_t)cy * L.cg.nx + cx;
    for (int c = 0; c < nU; ++c) L.fst[stage][c * fnc + i] = L.cst[stage][c * cnc + ci];
  }
}

// interface fluxes of stage s: item (link, face, k) with k = 0 the coarse
// face and k = 1, 2 the fine sub-faces; every flux from the two cells'
// WENO-C/CL reconstructions (5-cell stencils along the normal) and the
// Riemann solver, the functions the sweeps use
template <int N, int D, typename W>
__global__ __launch_bounds__(64) void k_amr_flux(const AmrLink* __restrict__ links,
                                                 const int2* __restrict__ items, int nitems,
                                                 int stage) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nitems) return;
  constexpr int NU = 2 * N + D + 1;
  const int2 it = items[t];
  const AmrLink& L = links[it.x];
  const int f = it.y / 3, k = it.y - 3 * (it.y / 3);
  if (D == 1 && k == 2) return;
  const AmrFace a = amr_face(L, f);
  const bool fine = k > 0;
  const Grid& g = fine ? L.fg : L.cg;
  const gdouble* U = gptr(fine ? L.fst[stage] : L.cst[stage]);
  const int mx = fine ? a.fm[k - 1][0] : a.cm[0], my = fine ? a.fm[k - 1][1] : a.cm[1];
  // the six cells along the normal: minus cell - 2 .. minus cell + 3
  Cons<N, D> cu[6];
  double V[6][2 * N + D + 1];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int x = a.dir == 0 ? mx - 2 + j : mx, y = a.dir == 1 ? my - 2 + j : my;
    load_cons<N, D>(U, g.nc, (int64_t)y * g.nx + x, cu[j]);
    Prim<N, D> v;
    cons_to_prim<N, D>(cu[j], L.e, v);
#pragma unroll
    for (int p = 0; p < N; ++p) { V[j][p] = v.m[p]; V[j][N + p] = v.a[p]; }
#pragma unroll
    for (int q = 0; q < D; ++q) V[j][2 * N + q] = v.u[q];
    V[j][2 * N + D] = v.P;
  }
  const double hd = a.dir == 0 ? g.hdx : g.hdy;
  Face<N, D> fm0, fpm, fmp, fp0;
  reconstruct<N, D, W, kReconAny>([&](int c, int j) { return V[j][c]; }, cu[2], L.e, g, hd, fm0,
                                  fpm);
  reconstruct<N, D, W, kReconAny>([&](int c, int j) { return V[j + 1][c]; }, cu[3], L.e, g, hd,
                                  fmp, fp0);
  Flux<N, D> F;
  riemann<N, D, W>(fpm, fmp, a.dir, g.flux, F);
  double* out = L.flx + ((int64_t)f * 3 + k) * (NU + 1);
#pragma unroll
  for (int c = 0; c < NU; ++c) gptr(out)[c] = F.f[c];
  gptr(out)[NU] = F.uh;
}

// the stage's correction of the outside coarse cells' L: the fine minus
// the coarse flux over the coarse width, with the alpha source on the same
// face-velocity difference; accumulated with the RK3 weight of the stage
template <int N, int D>
__global__ void k_amr_combine(const AmrLink* __restrict__ links, const int2* __restrict__ faces,
                              int nfaces, int stage) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nfaces) return;
  constexpr int NU = 2 * N + D + 1;
  const int2 it = faces[t];
  const AmrLink& L = links[it.x];
  const int f = it.y;
  const AmrFace a = amr_face(L, f);
  const gdouble* fl = gptr(L.flx) + (int64_t)f * 3 * (NU + 1);
  const double rd = a.dir == 0 ? L.cg.rdx : L.cg.rdy;
  // the outside coarse cell at the stage state
  const int ox = a.out_minus ? a.cm[0] : a.cp[0], oy = a.out_minus ? a.cm[1] : a.cp[1];
  Cons<N, D> ub;
  load_cons<N, D>(gptr(L.cst[stage]), L.cg.nc, (int64_t)oy * L.cg.nx + ox, ub);
  double opk[N];
  one_plus_k<N, D>(ub, L.e, L.cg.model, opk);
  double isa = 1.0;
  if (L.cg.asrc) {
    double sa = 0.0;
#pragma unroll
    for (int p = 0; p < N; ++p) sa += ub.a[p];
    isa = sa > 0.0 ? 1.0 / sa : 0.0;
  }
  // the face is the outside cell's upper face (block above it) or its lower one
  const double sg = a.out_minus ? -1.0 : 1.0;
  double dL[NU + 1];
#pragma unroll
  for (int c = 0; c <= NU; ++c) {
    const double ff = D == 1 ? fl[(NU + 1) + c] : 0.5 * (fl[(NU + 1) + c] + fl[2 * (NU + 1) + c]);
    dL[c] = sg * (ff - fl[c]) * rd;
  }
#pragma unroll
  for (int p = 0; p < N; ++p) dL[N + D + 1 + p] -= ub.a[p] * isa * opk[p] * dL[NU];
  const double w = stage == 2 ? 2.0 / 3.0 : 1.0 / 6.0;
  gdouble* r = gptr(L.reg) + (int64_t)f * NU;
#pragma unroll
  for (int c = 0; c < NU; ++c) r[c] = (stage == 0 ? 0.0 : r[c]) + w * dL[c];
}

// after the step: coarse cells under the block <- mean of their children;
// coarse cells beside it += dt x the accumulated correction
__global__ void k_amr_restrict(const AmrLink* __restrict__ links, int nU) {
  const AmrLink& L = links[blockIdx.y];
  const int h = kAmrHalo;
  const bool one = L.fg.ny == 1;
  const int64_t ncell = (int64_t)L.W * L.H;
  double* cU = L.cst[0];
  const double* fU = L.fst[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ncell;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int J = (int)(i / L.W), I = (int)(i - (int64_t)J * L.W);
    const int64_t ci = (int64_t)(L.loy + J) * L.cg.nx + (L.lox + I);
    const int fx = h + 2 * I;
    for (int c = 0; c < nU; ++c) {
      const double* F = fU + (int64_t)c * L.fg.nc;
      double v;
      if (one) {
        v = 0.5 * (F[fx] + F[fx + 1]);
      } else {
        const int64_t f0 = (int64_t)(h + 2 * J) * L.fg.nx + fx, f1 = f0 + L.fg.nx;
        v = 0.25 * ((F[f0] + F[f0 + 1]) + (F[f1] + F[f1 + 1]));
      }
      gptr(cU)[(int64_t)c * L.cg.nc + ci] = v;
    }
  }
}

__global__ void k_amr_reflux(const AmrLink* __restrict__ links, const int2* __restrict__ faces,
                             int nfaces, int nU) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nfaces) return;
  const int2 it = faces[t];
  const AmrLink& L = links[it.x];
  const AmrFace a = amr_face(L, it.y);
  const int ox = a.out_minus ? a.cm[0] : a.cp[0], oy = a.out_minus ? a.cm[1] : a.cp[1];
  const double dt = *gptr(L.dt);
  const double* r = L.reg + (int64_t)it.y * nU;
  for (int c = 0; c < nU; ++c) {
    gdouble* u = gptr(L.cst[0]) + (int64_t)c * L.cg.nc + (int64_t)oy * L.cg.nx + ox;
    *u = *u + dt * r[c];
  }
}

// linked instances take the smallest of their time steps
__global__ void k_amr_dt(const int* __restrict__ ids, int n, double* dt) {
  if (threadIdx.x != 0) return;
  double m = INFINITY;
  for (int k = 0; k < n; ++k) m = fmin(m, dt[ids[k]]);
  for (int k = 0; k < n; ++k) dt[ids[k]] = m;
}

// Cells per reduction workgroup: a multiple of kRedBlock chosen per instance
// (Desc::chunk) so that an instance has at most kMaxChunks chunks: small
// grids still spread over many workgroups, and the per-instance finishers
// reduce at most kMaxChunks partials per slot.
constexpr int kMaxChunks = 2048;

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
  const int64_t c0 = (int64_t)it.y * d.chunk;
  const int64_t c1 = c0 + d.chunk < g.nc ? c0 + d.chunk : g.nc;
  double smax = 0.0;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += kRedBlock) {
    Cons<N, D> c;
    load_cons<N, D>(gptr(d.U), g.nc, i, c);
    Prim<N, D> v;
    cons_to_prim<N, D>(c, e, v);
    smax = fmax(smax, cfl_rate<N, D>(v, e, g));
  }
  const double r = block_max(smax, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// one workgroup per instance: dt = cfl / max, clipped to t_end - t; with
// advance also the instance's time and step count move on (nothing in the
// RK stages reads them)
// (a workgroup of kDtBlock lanes, four independent loads in flight per lane:
// an instance's partials are one per x strip when the first x sweep of the
// step reduces them, 10^5 and more on a large 3D grid)
constexpr int kDtBlock = 1024;
__global__ __launch_bounds__(kDtBlock) void k_dt_finish(
    const Desc* __restrict__ descs, const int* __restrict__ start,
    const double* __restrict__ part, double cfl, int advance) {
  __shared__ double sh[kDtBlock / 64];
  const Desc& d = descs[blockIdx.x];
  const int b = start[blockIdx.x], n = start[blockIdx.x + 1];
  double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
  int i = b + threadIdx.x;
  for (; i + 3 * kDtBlock < n; i += 4 * kDtBlock) {
    m0 = fmax(m0, part[i]);
    m1 = fmax(m1, part[i + kDtBlock]);
    m2 = fmax(m2, part[i + 2 * kDtBlock]);
    m3 = fmax(m3, part[i + 3 * kDtBlock]);
  }
  for (; i < n; i += kDtBlock) m0 = fmax(m0, part[i]);
  const double r = block_max(fmax(fmax(m0, m1), fmax(m2, m3)), sh);
  if (threadIdx.x == 0) {
    const double t = *gptr(d.t);
    double dt = cfl / r;
    if (d.t_end > 0.0 && t + dt > d.t_end) dt = d.t_end - t;
    *gptr(d.dt) = dt;
    if (advance) {
      *gptr(d.t) = t + dt;
      // a step of 0 (the instance reached t_end) is not taken
      if (dt > 0.0) *gptr(d.steps) = *gptr(d.steps) + 1.0;
    }
  }
}

__global__ void k_advance_time(double* t, double* steps, const double* dt, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    t[i] = t[i] + dt[i];
    if (dt[i] > 0.0) steps[i] = steps[i] + 1.0;   // a step of 0 is not taken
  }
}

// per-workgroup diagnostics: slots 0..nU-1 sums, then
// [20] max|sum a - 1|, [21] min m, [22] min a, [23] max a, [24] min psi,
// [25] non-finite count, [28] max |rho E|, [32], [33] the two integrals of
// the interface thickness of Eq. (30) for alpha_1 (cells with
// 0.05 <= alpha_1 <= 0.95; |grad alpha_1| by central differences inside
// and one-sided ones at the ends of each direction)
template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_diag(const Desc* __restrict__ descs,
                                                    const int2* __restrict__ map,
                                                    int ninst, double* __restrict__ part) {
  constexpr int NU = 2 * N + D + 1;
  static_assert(NU <= 20, "the totals take the slots below 20");
  __shared__ double sh[kRedBlock];
  const int2 it = locate(map, ninst, blockIdx.x);
  const Desc& d = descs[it.x];
  const Grid& g = d.g;
  const Eos& e = d.e;
  const int64_t c0 = (int64_t)it.y * d.chunk;
  const int64_t c1 = c0 + d.chunk < g.nc ? c0 + d.chunk : g.nc;
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
    // interface thickness integrals of alpha_1
    const double a1 = u[N + D + 1];
    if (a1 >= 0.05 && a1 <= 0.95) acc[32] += 1.0;
    const gdouble* A = U + (int64_t)(N + D + 1) * g.nc;
    const int64_t plane = (int64_t)g.nx * g.ny;
    const int z = (int)(i / plane);
    const int64_t r = i - (int64_t)z * plane;
    const int y = (int)(r / g.nx), x = (int)(r - (int64_t)y * g.nx);
    double g2 = 0.0;
    auto grad = [&](int k, int n, int64_t st, double rd) {
      if (n < 2) return;
      double v;
      if (k == 0) v = (A[i + st] - A[i]) * rd;
      else if (k == n - 1) v = (A[i] - A[i - st]) * rd;
      else v = (A[i + st] - A[i - st]) * (0.5 * rd);
      g2 += v * v;
    };
    grad(x, g.nx, 1, g.rdx);
    if constexpr (D >= 2) grad(y, g.ny, g.nx, g.rdy);
    if constexpr (D >= 3) grad(z, g.nz, plane, g.rdz);
    acc[33] += sqrt(g2);
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
    if (threadIdx.x == 0) part[(int64_t)k * d.ps + blockIdx.x] = sh[0];
    __syncthreads();
  }
}

// one workgroup per instance (at least MP_DIAG_LEN lanes), lane k reduces
// slot k in block order
__global__ void k_diag_finish(const Desc* __restrict__ descs, const int* __restrict__ start,
                              const double* __restrict__ part) {
  const int k = threadIdx.x;
  const Desc& d = descs[blockIdx.x];
  if (k >= MP_DIAG_LEN) return;
  if (k >= kDiagSlots) {            // slots no reduction fills: 0
    gptr(d.diag)[k] = 0.0;
    return;
  }
  double r;
  if (k == 21 || k == 22 || k == 24) r = INFINITY;
  else if (k == 23) r = -INFINITY;
  else r = 0.0;
  for (int b = start[blockIdx.x]; b < start[blockIdx.x + 1]; ++b) {
    const double x = part[(int64_t)k * d.ps + b];
    if (k == 21 || k == 22 || k == 24) r = fmin(r, x);
    else if (k == 20 || k == 23 || k == 28) r = fmax(r, x);
    else r = r + x;
  }
  if (k < 20 || k >= 32) r *= d.vol;      // the integrals
  if (k == 26) r = *gptr(d.t);
  if (k == 27) r = *gptr(d.steps);
  if (k == 29) r = d.pfs ? gptr(d.pfs)[kPfsIts] : 0.0;
  if (k == 30) r = d.pfs ? gptr(d.pfs)[kPfsRes] : 0.0;
  gptr(d.diag)[k] = r;
}

// ---------------------------------------------------------------------------
// Phase-Field step (Sec. 2.2.1, Eqs. (4)-(5); Sec. 4, Eq. (28))
// ---------------------------------------------------------------------------
// With phi_p = alpha_p of the hyperbolic result:
//   [div J_p] = M lap(phi_p) - (M/eta^2)(g'(phi_p) - phi_p sum_q g'(phi_q))
//               + sum_q W_pq B_q,        M = eta max|u| / 2,
// where B solves the integral system of Eq. (28) over the present phases
// (B of the last present phase = 0: the system is singular and L^c does not
// depend on that choice).  Eq. (4) is solved for Q_p by Jacobi-preconditioned
// conjugate gradients on K Q = -[div J], with
//   (K Q)_i = sum over faces of k_f (Q_i - Q_j) / dx^2,  k_f = (k_i + k_j)/2,
// k = phi (1 - phi), faces across periodic ends only.  The solve starts from
// the previous step's Q and stops at ||res|| <= rtol ||div J||.  The face
// gradients are frozen and the PF flux is advanced by SSP-RK3 with the
// WENO-C face states of the sweeps.  All reductions are two-level with a
// fixed order.

__device__ __forceinline__ double gprime(double f) {
  return 2.0 * f * (1.0 - f) * (1.0 - 2.0 * f);
}

// fixed-order tree over the workgroup (256 lanes); op 0 sum, 1 max
__device__ __forceinline__ double block_reduce(double v, double* sh, int op) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kRedBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double x = sh[threadIdx.x], y = sh[threadIdx.x + s];
      sh[threadIdx.x] = op ? fmax(x, y) : x + y;
    }
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// sums of slots 0 .. K - 1 of an instance's chunk partials at once, fixed
// order: each thread adds its chunks, each wave reduces with lane exchanges,
// thread 0 adds the waves in order; the result is valid in thread 0
template <int K>
__device__ __forceinline__ void reduce_chunks_n(const double* __restrict__ part, int64_t ps,
                                                int b0, int b1, double* v, double* sh) {
  static_assert(K * (kRedBlock / 64) <= kRedBlock, "LDS of the reduction");
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (int b = b0 + (int)threadIdx.x; b < b1; b += kRedBlock)
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += part[(int64_t)k * ps + b];
#pragma unroll
  for (int k = 0; k < K; ++k)
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k * (kRedBlock / 64) + w] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double t = sh[k * (kRedBlock / 64)];
      for (int j = 1; j < kRedBlock / 64; ++j) t += sh[k * (kRedBlock / 64) + j];
      v[k] = t;
    }
}

// sum (or max) of slot k of an instance's chunk partials, fixed order
__device__ __forceinline__ double reduce_chunks(const double* __restrict__ part, int64_t ps,
                                                int b0, int b1, int k, double* sh, int op) {
  double v = 0.0;
  for (int b = b0 + (int)threadIdx.x; b < b1; b += kRedBlock) {
    const double x = part[(int64_t)k * ps + b];
    v = op ? fmax(v, x) : v + x;
  }
  return block_reduce(v, sh, op);
}

// neighbour of cell (x, y) one step along dir (+1 / -1); -1 if no face there
__device__ __forceinline__ int64_t nbr(const Grid& g, int x, int y, int z, int dir, int s) {
  const int64_t plane = (int64_t)g.nx * g.ny;
  if (dir == 0) {
    int xn = x + s;
    if (xn < 0) { if (g.bcx0 != MP_BC_PERIODIC) return -1; xn += g.nx; }
    if (xn >= g.nx) { if (g.bcx1 != MP_BC_PERIODIC) return -1; xn -= g.nx; }
    return z * plane + (int64_t)y * g.nx + xn;
  }
  if (dir == 1) {
    int yn = y + s;
    if (yn < 0) { if (g.bcy0 != MP_BC_PERIODIC) return -1; yn += g.ny; }
    if (yn >= g.ny) { if (g.bcy1 != MP_BC_PERIODIC) return -1; yn -= g.ny; }
    return z * plane + (int64_t)yn * g.nx + x;
  }
  int zn = z + s;
  if (zn < 0) { if (g.bcz0 != MP_BC_PERIODIC) return -1; zn += g.nz; }
  if (zn >= g.nz) { if (g.bcz1 != MP_BC_PERIODIC) return -1; zn -= g.nz; }
  return zn * plane + (int64_t)y * g.nx + x;
}

// coordinates of cell i (x fastest, then y, then z)
__device__ __forceinline__ void cell_xyz(const Grid& g, int64_t i, int& x, int& y, int& z) {
  const int64_t plane = (int64_t)g.nx * g.ny;
  z = (int)(i / plane);
  const int64_t r = i - z * plane;
  y = (int)(r / g.nx);
  x = (int)(r - (int64_t)y * g.nx);
}

// 1 / dx of direction dir
__device__ __forceinline__ double grid_rd(const Grid& g, int dir) {
  return dir == 0 ? g.rdx : (dir == 1 ? g.rdy : g.rdz);
}

// (K v)_i and (|K| |v|)_i for phase p at cell i
template <int D>
__device__ __forceinline__ void k_apply(const Grid& g, const gdouble* __restrict__ k,
                                        const gdouble* __restrict__ v, int64_t i, int x, int y,
                                        int z, double& Kv, double& aKv) {
  Kv = 0.0;
  aKv = 0.0;
  const double ki = k[i], vi = v[i];
#pragma unroll
  for (int dir = 0; dir < D; ++dir) {
    const double r2 = grid_rd(g, dir) * grid_rd(g, dir);
#pragma unroll
    for (int s = -1; s <= 1; s += 2) {
      const int64_t j = nbr(g, x, y, z, dir, s);
      if (j >= 0) {
        const double kf = 0.5 * (ki + k[j]) * r2;
        Kv += kf * (vi - v[j]);
        aKv += kf * (fabs(vi) + fabs(v[j]));
      }
    }
  }
}

// pass 1: k_p, max |u|, and the integrands of Eq. (28)'s multiplier system
//   slots: [0] max|u|, [1 + p N + q] W_pq, [1 + N^2 + p] (g'_p - phi_p sum g'),
//          [1 + N^2 + N + p] phi_p
template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_pf_prep(const Desc* __restrict__ descs,
                                                       const int2* __restrict__ map, int ninst,
                                                       double* __restrict__ part) {
  __shared__ double sh[kRedBlock];
  constexpr int NS = 1 + N * N + 2 * N;
  const int2 it = locate(map, ninst, chunk_item());
  const Desc& d = descs[it.x];
  const int64_t nc = d.g.nc;
  const int64_t c0 = (int64_t)it.y * d.chunk;
  const int64_t c1 = c0 + d.chunk < nc ? c0 + d.chunk : nc;
  const gdouble* U = gptr(d.pfin);
  gdouble* K = gptr(d.pf_k);
  double acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0.0;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += kRedBlock) {
    double phi[N], rho = 0.0, sg = 0.0;
#pragma unroll
    for (int p = 0; p < N; ++p) {
      phi[p] = U[(int64_t)(N + D + 1 + p) * nc + i];
      rho += U[(int64_t)p * nc + i];
      sg += gprime(phi[p]);
      K[(int64_t)p * nc + i] = fmax(phi[p] * (1.0 - phi[p]), kKFloor);
    }
    double u2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double u = U[(int64_t)(N + k) * nc + i] / rho;
      u2 += u * u;
    }
    acc[0] = fmax(acc[0], sqrt(u2));
#pragma unroll
    for (int p = 0; p < N; ++p) {
#pragma unroll
      for (int q = 0; q < N; ++q)
        acc[1 + p * N + q] += p == q ? phi[p] * (1.0 - phi[q]) : -phi[p] * phi[q];
      acc[1 + N * N + p] += gprime(phi[p]) - phi[p] * sg;
      acc[1 + N * N + N + p] += phi[p];
    }
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double r = block_reduce(acc[k], sh, k == 0 ? 1 : 0);
    if (threadIdx.x == 0) part[(int64_t)k * d.ps + chunk_item()] = r;
  }
}

// one workgroup per instance: M, and B from the reduced multiplier system
template <int N>
__global__ __launch_bounds__(kRedBlock) void k_pf_setup(const Desc* __restrict__ descs,
                                                        const int* __restrict__ start,
                                                        const double* __restrict__ part) {
  __shared__ double sh[kRedBlock];
  __shared__ double red[1 + N * N + 2 * N];
  const Desc& d = descs[blockIdx.x];
  const int b0 = start[blockIdx.x], b1 = start[blockIdx.x + 1];
  for (int k = 0; k < 1 + N * N + 2 * N; ++k) {
    const double r = reduce_chunks(part, d.ps, b0, b1, k, sh, k == 0 ? 1 : 0);
    if (threadIdx.x == 0) red[k] = r;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  gdouble* s = gptr(d.pfs);
  const double M = 0.5 * d.eta * red[0];
  const double Me2 = M / (d.eta * d.eta);
  double B[N];
  int pres[N], np = 0;
#pragma unroll
  for (int p = 0; p < N; ++p) {
    B[p] = 0.0;
    if (red[1 + N * N + N + p] > 0.0) pres[np++] = p;
  }
  if (np > 1) {
    const int n = np - 1;
    double A[N][N], b[N];
    for (int r = 0; r < n; ++r) {
      for (int c = 0; c < n; ++c) A[r][c] = red[1 + pres[r] * N + pres[c]] * d.vol;
      b[r] = Me2 * (red[1 + N * N + pres[r]] * d.vol);
    }
    bool ok = true;
    for (int k = 0; k < n && ok; ++k) {           // partial pivoting
      int pv = k;
      for (int r = k + 1; r < n; ++r)
        if (fabs(A[r][k]) > fabs(A[pv][k])) pv = r;
      if (A[pv][k] == 0.0) { ok = false; break; }
      if (pv != k) {
        for (int c = 0; c < n; ++c) { const double t = A[k][c]; A[k][c] = A[pv][c]; A[pv][c] = t; }
        const double t = b[k]; b[k] = b[pv]; b[pv] = t;
      }
      for (int r = k + 1; r < n; ++r) {
        const double f = A[r][k] / A[k][k];
        for (int c = k; c < n; ++c) A[r][c] -= f * A[k][c];
        b[r] -= f * b[k];
      }
    }
    if (ok) {
      for (int k = n - 1; k >= 0; --k) {
        double v = b[k];
        for (int c = k + 1; c < n; ++c) v -= A[k][c] * b[c];
        b[k] = v / A[k][k];
      }
      for (int r = 0; r < n; ++r) B[pres[r]] = b[r];
    }
  }
  s[kPfsM] = M;
  s[kPfsMe2] = Me2;
#pragma unroll
  for (int p = 0; p < N; ++p) s[kPfsB + p] = B[p];
  s[kPfsIts] = 0.0;
  s[kPfsRes] = 0.0;
  s[kPfsCorr] = kMgCorr;
#pragma unroll
  for (int p = 0; p < N; ++p) {
    s[kPfsPits + p] = 0.0;
    s[kPfsPrev + p] = -1.0;            // no start pass of this solve yet
  }
}

// [div J_p] at every cell; start (or restart) of the CG solve: the residual
// of the warm start r = -b - K Q; partials [p]
// ||b||^2, [N + p] ||r||^2 and [2N + p] || |b| + |K| |Q| ||^2 (the scale of
// the rounding error of r)
template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_pf_divj(const Desc* __restrict__ descs,
                                                       const int2* __restrict__ map, int ninst,
                                                       double* __restrict__ part, int cold) {
  __shared__ double sh[kRedBlock];
  const int2 it = locate(map, ninst, chunk_item());
  const Desc& d = descs[it.x];
  const Grid& g = d.g;
  const int64_t nc = g.nc;
  const int64_t c0 = (int64_t)it.y * d.chunk;
  const int64_t c1 = c0 + d.chunk < nc ? c0 + d.chunk : nc;
  const gdouble* U = gptr(d.pfin);
  const gdouble* K = gptr(d.pf_k);
  const gdouble* s = gptr(d.pfs);
  const double M = s[kPfsM], Me2 = s[kPfsMe2];
  double B[N];
#pragma unroll
  for (int p = 0; p < N; ++p) B[p] = s[kPfsB + p];
  double acc[3 * N];
#pragma unroll
  for (int k = 0; k < 3 * N; ++k) acc[k] = 0.0;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += kRedBlock) {
    int x, y, z;
    cell_xyz(g, i, x, y, z);
    double phi[N], sg = 0.0;
#pragma unroll
    for (int p = 0; p < N; ++p) {
      phi[p] = U[(int64_t)(N + D + 1 + p) * nc + i];
      sg += gprime(phi[p]);
    }
#pragma unroll
    for (int p = 0; p < N; ++p) {
      const gdouble* f = U + (int64_t)(N + D + 1 + p) * nc;
      double lap = 0.0;
#pragma unroll
      for (int dir = 0; dir < D; ++dir) {
        const int64_t lo = nbr(g, x, y, z, dir, -1), hi = nbr(g, x, y, z, dir, 1);
        const double fl = lo >= 0 ? f[lo] : phi[p];    // outflow: zero gradient
        const double fh = hi >= 0 ? f[hi] : phi[p];
        const double r2 = grid_rd(g, dir) * grid_rd(g, dir);
        lap += (fh - 2.0 * phi[p] + fl) * r2;
      }
      double Lc = 0.0;
#pragma unroll
      for (int q = 0; q < N; ++q)
        Lc += (p == q ? phi[p] * (1.0 - phi[q]) : -phi[p] * phi[q]) * B[q];
      const double b = M * lap - Me2 * (gprime(phi[p]) - phi[p] * sg) + Lc;
      const int64_t ip = (int64_t)p * nc + i;
      gptr(d.pf_b)[ip] = b;
      // K Q = -b from the previous Q (or 0)
      double Kq = 0.0, aKq = 0.0;
      if (cold)
        gptr(d.pf_q)[ip] = 0.0;
      else
        k_apply<D>(g, K + (int64_t)p * nc, gptr(d.pf_q) + (int64_t)p * nc, i, x, y, z, Kq, aKq);
      const double r = -b - Kq;
      gptr(d.pf_r)[ip] = r;
      acc[p] += b * b;
      acc[N + p] += r * r;
      const double sc = fabs(b) + aKq;
      acc[2 * N + p] += sc * sc;
    }
  }
#pragma unroll
  for (int k = 0; k < 3 * N; ++k) {
    const double r = block_reduce(acc[k], sh, 0);
    if (threadIdx.x == 0) part[(int64_t)k * d.ps + chunk_item()] = r;
  }
}

// one workgroup per instance, at the start of the solve and after every run
// of iterations: ||b||^2 and the true residual ||r|| = ||-b - K Q|| of each
// phase.  A phase with b = 0 has nothing to solve (its Q is cleared by the
// gradient pass); one with ||r|| <= rtol ||b|| + 64 eps || |b| + |K| |Q| ||
// is done (the second term is the rounding floor of r itself, which a badly
// scaled Q can lift above rtol ||b||), and so is one whose last run of
// iterations did not halve its true residual while that lies within
// 1000 rtol ||b|| (the iteration stagnates at its attainable accuracy); any
// other starts CG afresh from its Q.  The residual reported at exit is this
// true one.
template <int N>
__global__ __launch_bounds__(kRedBlock) void k_pf_cg_start(const Desc* __restrict__ descs,
                                                           const int* __restrict__ start,
                                                           const double* __restrict__ part,
                                                           double rtol) {
  __shared__ double sh[kRedBlock];
  const Desc& d = descs[blockIdx.x];
  gdouble* s = gptr(d.pfs);
  double rmax = 0.0;
  for (int p = 0; p < N; ++p) {
    const double bb = reduce_chunks(part, d.ps, start[blockIdx.x], start[blockIdx.x + 1], p, sh, 0);
    const double rr = reduce_chunks(part, d.ps, start[blockIdx.x], start[blockIdx.x + 1], N + p, sh, 0);
    const double fl = reduce_chunks(part, d.ps, start[blockIdx.x], start[blockIdx.x + 1], 2 * N + p, sh, 0);
    if (threadIdx.x == 0) {
      s[kPfsBB + p] = bb;
      const double rel = bb > 0.0 ? sqrt(rr / bb) : 0.0;
      // stagnation: a restart of this solve (iterating or breaking down at
      // once) did not halve the true residual, which is within 1000 rtol
      const double prev = s[kPfsPrev + p];
      const bool stalled = prev >= 0.0 && rel > 0.5 * prev && rel <= kPfsStallTol * rtol;
      const bool done = bb == 0.0 || sqrt(rr) <= rtol * sqrt(bb) + 64.0 * DBL_EPSILON * sqrt(fl) ||
                        stalled;
      s[kPfsPrev + p] = rel;
      rmax = fmax(rmax, rel);
      // a phase that iterated and still misses the tolerance: its recurrence
      // drifted from the true residual; restart with the plain correction
      if (!done && s[kPfsPits + p] > 0.0) s[kPfsCorr] = 1.0;
      s[kPfsDone + p] = done ? 1.0 : 0.0;
      s[kPfsPits + p] = 0.0;
    }
  }
  if (threadIdx.x == 0) s[kPfsRes] = rmax;
}

// Preconditioned conjugate gradients, z = M^-1 r the multigrid V-cycle below.
// One iteration is five passes (and the V-cycle):
//   dir:    p = (z - mean z) + beta p_prev (p = z - mean z the first time),
//           q = K p, partial [p] p.q
//   alpha:  alpha = r.z / p.q
//   axpy:   Q += alpha p, r -= alpha q
//   (V-cycle: z = M^-1 r)
//   dots:   partials [p] r.z, [N + p] r.r, [2N + p] sum z, [3N + p] sum r,
//           [4N + p] z.q, [5N + p] sum q (q = K p of this iteration)
//   beta:   done once the recurrence's ||r|| <= rtol ||b|| (then checked
//           against the true residual by the start pass); else the flexible
//           (Polak-Ribiere) beta = z'.(r - r_prev) / (r.z')_prev
//           = -alpha z'.q / (r.z')_prev with z' = z - mean z (so
//           r.z' = r.z - mean z sum r, z'.q = z.q - mean z sum q): equal to
//           r.z' / (r.z')_prev for a fixed symmetric preconditioner, and it
//           keeps the directions conjugate when the FP32 V-cycle is not
//           exactly one (plain PCG then stalls near 1e-9)
// The directions alternate between two buffers (p at neighbours is read
// while the new one is written).  K is singular (its null space: the
// constants; faces at outflow ends carry no flux) and the V-cycle's output
// carries a constant part, which K maps to zero but which would pile up in Q
// (the over-corrected cycle amplifies it level by level) until Q's rounding
// hides the solution: the directions are kept free of it.  A non-positive
// p.q or r.z (the scaled cycle lost definiteness, or round-off) stops the
// phase and drops the cycle to the plain correction for the restart.
// Phases that are done skip their work (the flag is uniform per instance).

// direction buffer of the k-th direction (k >= 1) of a phase
__device__ __forceinline__ gdouble* pf_dirbuf(const Desc& d, double k) {
  return gptr(((long long)k & 1) ? d.pf_p : d.pf_w);
}

template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_pf_cg_dir(const Desc* __restrict__ descs,
                                                         const int2* __restrict__ map, int ninst,
                                                         double* __restrict__ part) {
  __shared__ double sh[kRedBlock];
  const int2 it = locate(map, ninst, chunk_item());
  const Desc& d = descs[it.x];
  const Grid& g = d.g;
  const int64_t nc = g.nc;
  const gdouble* s = gptr(d.pfs);
  bool live[N];
  bool any = false;
#pragma unroll
  for (int p = 0; p < N; ++p) { live[p] = s[kPfsDone + p] == 0.0; any = any || live[p]; }
  if (!any) return;                       // uniform over the workgroup
  const int64_t c0 = (int64_t)it.y * d.chunk;
  const int64_t c1 = c0 + d.chunk < nc ? c0 + d.chunk : nc;
  double acc[N];
#pragma unroll
  for (int k = 0; k < N; ++k) acc[k] = 0.0;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += kRedBlock) {
    int x, y, z;
    cell_xyz(g, i, x, y, z);
#pragma unroll
    for (int p = 0; p < N; ++p) {
      if (!live[p]) continue;
      const double k = s[kPfsPits + p];
      const bool first = k == 1.0;
      const double be = s[kPfsBeta + p], zb = s[kPfsUbar + p];
      const gdouble* K = gptr(d.pf_k) + (int64_t)p * nc;
      const gdouble* Z = gptr(d.pf_u) + (int64_t)p * nc;
      const gdouble* P0 = pf_dirbuf(d, k + 1.0) + (int64_t)p * nc;
      auto dir_at = [&](int64_t j) { return first ? Z[j] - zb : (Z[j] - zb) + be * P0[j]; };
      const double pi = dir_at(i);
      double q = 0.0;
      const double ki = K[i];
#pragma unroll
      for (int dd = 0; dd < D; ++dd) {
        const double r2 = grid_rd(g, dd) * grid_rd(g, dd);
#pragma unroll
        for (int sg = -1; sg <= 1; sg += 2) {
          const int64_t j = nbr(g, x, y, z, dd, sg);
          if (j >= 0) q += 0.5 * (ki + K[j]) * r2 * (pi - dir_at(j));
        }
      }
      pf_dirbuf(d, k)[(int64_t)p * nc + i] = pi;
      gptr(d.pf_ap)[(int64_t)p * nc + i] = q;
      acc[p] += pi * q;
    }
  }
#pragma unroll
  for (int p = 0; p < N; ++p) {
    if (!live[p]) continue;
    const double r = block_reduce(acc[p], sh, 0);
    if (threadIdx.x == 0) part[(int64_t)p * d.ps + chunk_item()] = r;
  }
}

template <int N>
__global__ __launch_bounds__(kRedBlock) void k_pf_cg_alpha(const Desc* __restrict__ descs,
                                                           const int* __restrict__ start,
                                                           const double* __restrict__ part) {
  __shared__ double sh[kRedBlock];
  const Desc& d = descs[blockIdx.x];
  gdouble* s = gptr(d.pfs);
  double pq[N];
  reduce_chunks_n<N>(part, d.ps, start[blockIdx.x], start[blockIdx.x + 1], pq, sh);
  if (threadIdx.x == 0)
    for (int p = 0; p < N; ++p) {
      if (s[kPfsDone + p] != 0.0) continue;
      const double rz = s[kPfsRZ + p];
      if (!(pq[p] > 0.0) || !(rz > 0.0)) {
        s[kPfsDone + p] = 1.0;
        s[kPfsCorr] = 1.0;
      } else {
        s[kPfsAlpha + p] = rz / pq[p];
      }
    }
}

template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_pf_cg_axpy(const Desc* __restrict__ descs,
                                                          const int2* __restrict__ map, int ninst) {
  const int2 it = locate(map, ninst, chunk_item());
  const Desc& d = descs[it.x];
  const int64_t nc = d.g.nc;
  const gdouble* s = gptr(d.pfs);
  bool live[N];
  double al[N], kk[N];
  bool any = false;
#pragma unroll
  for (int p = 0; p < N; ++p) {
    live[p] = s[kPfsDone + p] == 0.0;
    al[p] = s[kPfsAlpha + p];
    kk[p] = s[kPfsPits + p];
    any = any || live[p];
  }
  if (!any) return;
  const int64_t c0 = (int64_t)it.y * d.chunk;
  const int64_t c1 = c0 + d.chunk < nc ? c0 + d.chunk : nc;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += kRedBlock) {
#pragma unroll
    for (int p = 0; p < N; ++p) {
      if (!live[p]) continue;
      const int64_t ip = (int64_t)p * nc + i;
      gptr(d.pf_q)[ip] += al[p] * pf_dirbuf(d, kk[p])[ip];
      gptr(d.pf_r)[ip] -= al[p] * gptr(d.pf_ap)[ip];
    }
  }
}

// Start of the Q solve of a step (before its first start pass), from the
// last solutions Q (the last step's), Q' and Q'' (the two before it):
// extrapolate 2: Q = 3 (Q - Q') + Q'' (quadratic in time: the solve starts
// O(dt^3) from its solution where the warm start alone is O(dt) away);
// extrapolate 1: Q = 2 Q - Q' (linear); 0: Q as it is.  Then Q'' = Q' and
// Q' = the last solution.
template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_pf_guess(const Desc* __restrict__ descs,
                                                        const int2* __restrict__ map, int ninst,
                                                        int extrapolate) {
  const int2 it = locate(map, ninst, chunk_item());
  const Desc& d = descs[it.x];
  const int64_t nc = d.g.nc;
  const int64_t c0 = (int64_t)it.y * d.chunk;
  const int64_t c1 = c0 + d.chunk < nc ? c0 + d.chunk : nc;
  gdouble* Q = gptr(d.pf_q);
  gdouble* Qp = gptr(d.pf_qp);
  gdouble* Qpp = gptr(d.pf_qpp);
  for (int64_t i = c0 + threadIdx.x; i < c1; i += kRedBlock) {
#pragma unroll
    for (int p = 0; p < N; ++p) {
      const int64_t ip = (int64_t)p * nc + i;
      const double q = Q[ip], qp = Qp[ip];
      if (extrapolate == 2) Q[ip] = 3.0 * (q - qp) + Qpp[ip];
      else if (extrapolate == 1) Q[ip] = fma(2.0, q, -qp);
      Qpp[ip] = qp;
      Qp[ip] = q;
    }
  }
}

template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_pf_cg_dots(const Desc* __restrict__ descs,
                                                          const int2* __restrict__ map, int ninst,
                                                          double* __restrict__ part) {
  __shared__ double sh[kRedBlock];
  const int2 it = locate(map, ninst, chunk_item());
  const Desc& d = descs[it.x];
  const int64_t nc = d.g.nc;
  const gdouble* s = gptr(d.pfs);
  bool live[N];
  bool any = false;
#pragma unroll
  for (int p = 0; p < N; ++p) { live[p] = s[kPfsDone + p] == 0.0; any = any || live[p]; }
  if (!any) return;
  const int64_t c0 = (int64_t)it.y * d.chunk;
  const int64_t c1 = c0 + d.chunk < nc ? c0 + d.chunk : nc;
  double acc[6 * N];
#pragma unroll
  for (int k = 0; k < 6 * N; ++k) acc[k] = 0.0;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += kRedBlock) {
#pragma unroll
    for (int p = 0; p < N; ++p) {
      if (!live[p]) continue;
      const int64_t ip = (int64_t)p * nc + i;
      const double r = gptr(d.pf_r)[ip], z = gptr(d.pf_u)[ip], q = gptr(d.pf_ap)[ip];
      acc[p] += r * z;
      acc[N + p] += r * r;
      acc[2 * N + p] += z;
      acc[3 * N + p] += r;
      acc[4 * N + p] += z * q;
      acc[5 * N + p] += q;
    }
  }
#pragma unroll
  for (int p = 0; p < N; ++p) {
    if (!live[p]) continue;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double r = block_reduce(acc[k * N + p], sh, 0);
      if (threadIdx.x == 0) part[(int64_t)(k * N + p) * d.ps + chunk_item()] = r;
    }
  }
}

template <int N>
__global__ __launch_bounds__(kRedBlock) void k_pf_cg_beta(const Desc* __restrict__ descs,
                                                          const int* __restrict__ start,
                                                          const double* __restrict__ part,
                                                          double rtol) {
  __shared__ double sh[kRedBlock];
  const Desc& d = descs[blockIdx.x];
  gdouble* s = gptr(d.pfs);
  double v[6 * N];
  reduce_chunks_n<6 * N>(part, d.ps, start[blockIdx.x], start[blockIdx.x + 1], v, sh);
  if (threadIdx.x != 0) return;
  double rmax = 0.0;
  bool stepped = false, adv = false;
  for (int p = 0; p < N; ++p) {
    if (s[kPfsDone + p] != 0.0) continue;
    const double rz0 = v[p], rr = v[N + p], zs = v[2 * N + p], rs = v[3 * N + p];
    const double zq = v[4 * N + p], qs = v[5 * N + p];
    const double zb = zs / (double)d.g.nc;
    const double rz = rz0 - zb * rs;
    stepped = true;
    {
      const double bb = s[kPfsBB + p];
      const double k = s[kPfsPits + p];
      const double rel = sqrt(rr / bb);
      rmax = fmax(rmax, rel);
      if (k == 0.0 || rel < 0.5 * s[kPfsBest + p]) {
        s[kPfsBest + p] = rel;
        s[kPfsBestIt + p] = k;
      }
      if (sqrt(rr) <= rtol * sqrt(bb)) {
        s[kPfsDone + p] = 1.0;
      } else if (rel <= kPfsStallTol * rtol && k - s[kPfsBestIt + p] >= kPfsStallIts) {
        s[kPfsDone + p] = 1.0;                 // stagnated: the start pass judges
      } else if (!(rz > 0.0)) {
        s[kPfsDone + p] = 1.0;                 // breakdown: restart
        s[kPfsCorr] = 1.0;
      } else {
        s[kPfsBeta + p] = k > 0.0 ? -s[kPfsAlpha + p] * (zq - zb * qs) / s[kPfsRZ + p] : 0.0;
        s[kPfsRZ + p] = rz;
        s[kPfsUbar + p] = zb;
        s[kPfsPits + p] = k + 1.0;
        adv = true;
      }
    }
  }
  // iterations of the solve, over its restarts
  if (stepped) {
    if (adv) s[kPfsIts] = s[kPfsIts] + 1.0;
    s[kPfsRes] = rmax;
  }
}

// ---------------------------------------------------------------------------
// Multigrid preconditioner of the Q solve: a symmetric V-cycle (damped Jacobi
// before and after the coarse correction, restriction = sum over the 2 x 2
// aggregate, prolongation = copy to it, the coarse operator the Galerkin
// product: a coarse face weight is the sum of the fine face weights between
// the two aggregates).  Symmetric; positive semidefinite as CG needs with the
// plain coarse correction (see kMgCorr for the scaled one).
// ---------------------------------------------------------------------------
constexpr int kMgMaxLev = 16;
constexpr int kMgCoarseSweeps = 8;    // sweeps on the coarsest level (even)
// damping of the Jacobi smoother: the value with the best smoothing factor
// for the model operator, 2 d / (2 d + 1): 2/3 for the 1D three-point, 4/5
// for the 2D five-point and 6/7 for the 3D seven-point Laplacian
template <int D>
constexpr double mg_omega() { return D == 1 ? 2.0 / 3.0 : (D == 2 ? 0.8 : 6.0 / 7.0); }

// arrays of a level in the LDS image of the fused cycle: the face weights of
// each direction (at least x and y), the diagonal, e, t and f
template <int D>
constexpr int mg_lds_arrays() { return D > 2 ? 7 : 6; }


// A level's arrays are read and written in global memory (AS = 1) by the
// per-level kernels, or in the LDS copy of the fused coarse cycle (AS = 3).
template <int AS>
using lfloat = __attribute__((address_space(AS))) float;
template <int AS>
__device__ __forceinline__ lfloat<AS>* lp(float* p) { return (lfloat<AS>*)p; }

// neighbour of cell (x, y, z) of a level one step along dir, with its
// coordinates; -1 if there is no face (an outflow or symmetry end, or a
// direction one aggregate wide)
__device__ __forceinline__ int lnbr_xyz(const Grid& g, const MgLevel& L, int x, int y, int z,
                                        int dir, int s, int& xn, int& yn, int& zn) {
  xn = x;
  yn = y;
  zn = z;
  if (dir == 0) {
    if (L.nx == 1) return -1;
    xn = x + s;
    if (xn < 0) { if (g.bcx0 != MP_BC_PERIODIC) return -1; xn += L.nx; }
    if (xn >= L.nx) { if (g.bcx1 != MP_BC_PERIODIC) return -1; xn -= L.nx; }
  } else if (dir == 1) {
    if (L.ny == 1) return -1;
    yn = y + s;
    if (yn < 0) { if (g.bcy0 != MP_BC_PERIODIC) return -1; yn += L.ny; }
    if (yn >= L.ny) { if (g.bcy1 != MP_BC_PERIODIC) return -1; yn -= L.ny; }
  } else {
    if (L.nz == 1) return -1;
    zn = z + s;
    if (zn < 0) { if (g.bcz0 != MP_BC_PERIODIC) return -1; zn += L.nz; }
    if (zn >= L.nz) { if (g.bcz1 != MP_BC_PERIODIC) return -1; zn -= L.nz; }
  }
  return (zn * L.ny + yn) * L.nx + xn;
}

__device__ __forceinline__ int lnbr(const Grid& g, const MgLevel& L, int x, int y, int z,
                                    int dir, int s) {
  int xn, yn, zn;
  return lnbr_xyz(g, L, x, y, z, dir, s, xn, yn, zn);
}

// coordinates of cell i of a level (levels hold < 2^31 cells)
__device__ __forceinline__ void lcell(const MgLevel& L, int i, int& x, int& y, int& z) {
  const int plane = L.nx * L.ny;
  z = i / plane;
  const int r = i - z * plane;
  y = r / L.nx;
  x = r - y * L.nx;
}

// (K v)_i of a level from its face weights; val(j, x_j, y_j, z_j) gives v
// at a cell of the level
template <int D, int AS, typename V>
__device__ __forceinline__ float lapply_v(const Grid& g, const MgLevel& L, int p, int i, int x,
                                          int y, int z, V val) {
  const float vi = val(i, x, y, z);
  float r = 0.0f;
#pragma unroll
  for (int dir = 0; dir < D; ++dir) {
    const lfloat<AS>* w = lp<AS>(dir == 0 ? L.wx : (dir == 1 ? L.wy : L.wz)) + (int64_t)p * L.nc;
    int xn, yn, zn;
    int j = lnbr_xyz(g, L, x, y, z, dir, 1, xn, yn, zn);
    if (j >= 0) r += w[i] * (vi - val(j, xn, yn, zn));
    j = lnbr_xyz(g, L, x, y, z, dir, -1, xn, yn, zn);
    if (j >= 0) r += w[j] * (vi - val(j, xn, yn, zn));
  }
  return r;
}

template <int D, int AS>
__device__ __forceinline__ float lapply(const Grid& g, const MgLevel& L, int p, const lfloat<AS>* v,
                                        int i, int x, int y, int z) {
  return lapply_v<D, AS>(g, L, p, i, x, y, z, [v](int j, int, int, int) { return (float)v[j]; });
}

// per-level work items: (instance, chunk of 256 cells of that level)
#define MG_PROLOGUE                                                         \
  const int2 it = locate(map, ninst, chunk_item());                         \
  const Desc& d = descs[it.x];                                              \
  const Grid& g = d.g;                                                      \
  const gdouble* s = gptr(d.pfs);                                           \
  bool live[N];                                                             \
  bool any = false;                                                         \
  _Pragma("unroll") for (int p = 0; p < N; ++p) {                           \
    live[p] = s[kPfsDone + p] == 0.0;                                       \
    any = any || live[p];                                                   \
  }                                                                         \
  if (!any) return;                                                         \
  const int64_t i = (int64_t)it.y * kRedBlock + threadIdx.x;

// level-0 face weights from k (frozen over the solve)
template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_mg_weights0(const Desc* __restrict__ descs,
                                                           const int2* __restrict__ map, int ninst) {
  MG_PROLOGUE
  const MgLevel L = d.mg[0];
  if (i >= L.nc) return;
  int x, y, z;
  lcell(L, (int)i, x, y, z);
#pragma unroll
  for (int p = 0; p < N; ++p) {
    const gdouble* K = gptr(d.pf_k) + (int64_t)p * L.nc;
#pragma unroll
    for (int dir = 0; dir < D; ++dir) {
      const int j = lnbr(g, L, x, y, z, dir, 1);
      const double rd = grid_rd(g, dir);
      float* w = dir == 0 ? L.wx : (dir == 1 ? L.wy : L.wz);
      gptr(w)[(int64_t)p * L.nc + i] = j >= 0 ? (float)(0.5 * (K[i] + K[j]) * rd * rd) : 0.0f;
    }
  }
}

// Galerkin face weights of level l + 1 (items over level l + 1)
template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_mg_coarsen(const Desc* __restrict__ descs,
                                                          const int2* __restrict__ map, int ninst,
                                                          int l) {
  MG_PROLOGUE
  const MgLevel F = d.mg[l], C = d.mg[l + 1];
  if (i >= C.nc) return;
  int X, Y, Z;
  lcell(C, (int)i, X, Y, Z);
  const int xr = min(2 * X + 1, F.nx - 1), yt = min(2 * Y + 1, F.ny - 1),
            zt = min(2 * Z + 1, F.nz - 1);
  const int z0 = 2 * Z, z1 = D > 2 ? zt : 0;
  auto fi = [&](int x, int y, int z) { return ((int64_t)z * F.ny + y) * F.nx + x; };
#pragma unroll
  for (int p = 0; p < N; ++p) {
    const gfloat* wx = gptr(F.wx) + (int64_t)p * F.nc;
    const gfloat* wy = gptr(F.wy) + (int64_t)p * F.nc;
    const gfloat* wz = gptr(F.wz) + (int64_t)p * F.nc;
    float cx = 0.0f, cy = 0.0f, cz = 0.0f;
    // the fine faces between this aggregate and its +x (+y, +z) neighbour
    if (C.nx > 1)
      for (int z = z0; z <= z1; ++z)
        for (int y = 2 * Y; y <= yt; ++y) cx += wx[fi(xr, y, z)];
    if constexpr (D > 1) {
      if (C.ny > 1)
        for (int z = z0; z <= z1; ++z)
          for (int x = 2 * X; x <= xr; ++x) cy += wy[fi(x, yt, z)];
    }
    if constexpr (D > 2) {
      if (C.nz > 1)
        for (int y = 2 * Y; y <= yt; ++y)
          for (int x = 2 * X; x <= xr; ++x) cz += wz[fi(x, y, zt)];
    }
    gptr(C.wx)[(int64_t)p * C.nc + i] = cx;
    if constexpr (D > 1) gptr(C.wy)[(int64_t)p * C.nc + i] = cy;
    if constexpr (D > 2) gptr(C.wz)[(int64_t)p * C.nc + i] = cz;
  }
}

// diagonal of a level from its weights
template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_mg_diag(const Desc* __restrict__ descs,
                                                       const int2* __restrict__ map, int ninst,
                                                       int l) {
  MG_PROLOGUE
  const MgLevel L = d.mg[l];
  if (i >= L.nc) return;
  int x, y, z;
  lcell(L, (int)i, x, y, z);
#pragma unroll
  for (int p = 0; p < N; ++p) {
    float dgv = 0.0f;
#pragma unroll
    for (int dir = 0; dir < D; ++dir) {
      const gfloat* w = gptr(dir == 0 ? L.wx : (dir == 1 ? L.wy : L.wz)) + (int64_t)p * L.nc;
      int j = lnbr(g, L, x, y, z, dir, 1);
      if (j >= 0) dgv += w[i];
      j = lnbr(g, L, x, y, z, dir, -1);
      if (j >= 0) dgv += w[j];
    }
    gptr(L.dg)[(int64_t)p * L.nc + i] = dgv;
  }
}

// One cell of the level passes, shared by the per-level kernels and the
// fused coarse cycle below.
// Power-of-two scale of phase p's level-0 right-hand side: near the rms of
// [div J_p] over the grid (||b||^2 of the start pass, > 0 for a live phase).
__device__ __forceinline__ int mg_scale_exp(const gdouble* s, int p, int64_t nc) {
  return ilogb(sqrt(s[kPfsBB + p]) / sqrt((double)nc));   // no underflow to 0
}

// Damped Jacobi on level L: mode 0: t = omega f / dg (from e = 0);
// mode 1: t = e + omega (f - K e) / dg; mode 2: e = t + omega (f - K t) / dg;
// mode 5: mode 1 on e' = e + corr P e(C), the coarse correction of level C
// (aggregates of 2 x 2 cells, piecewise constant) added on the fly, so the
// prolongation needs no pass of its own (e' is not kept: the next pass reads
// t); level 0 only: mode 3 is mode 0 after f = r 2^-k (the FP64 CG residual
// scaled), mode 4 is mode 2 writing u = 2^k (t + omega (f - K t) / dg) to
// the FP64 preconditioned residual instead of e (k = mg_scale_exp).
template <int D, int AS>
__device__ __forceinline__ void mg_smooth_cell(const Desc& d, const MgLevel& L, int p,
                                               int i, int mode, const MgLevel* C = nullptr,
                                               float corr = 0.0f) {
  const Grid& g = d.g;
  int x, y, z;
  lcell(L, i, x, y, z);
  const int64_t ip = (int64_t)p * L.nc + i;
  const float dgv = lp<AS>(L.dg)[ip];
  const float w = (float)mg_omega<D>();
  if (mode == 0 || mode == 3) {
    float fv;
    if (mode == 3) {
      fv = (float)ldexp(gptr(d.pf_r)[ip], -mg_scale_exp(gptr(d.pfs), p, L.nc));
      lp<AS>(L.f)[ip] = fv;
    } else {
      fv = lp<AS>(L.f)[ip];
    }
    lp<AS>(L.t)[ip] = dgv > 0.0f ? w * fv / dgv : 0.0f;
    return;
  }
  const float fv = lp<AS>(L.f)[ip];
  if (mode == 5) {
    const lfloat<AS>* e = lp<AS>(L.e) + (int64_t)p * L.nc;
    const lfloat<AS>* ec = lp<AS>(C->e) + (int64_t)p * C->nc;
    const int cnx = C->nx, cny = C->ny;
    auto ep = [=](int j, int xj, int yj, int zj) {
      return e[j] + corr * ec[((zj >> 1) * cny + (yj >> 1)) * cnx + (xj >> 1)];
    };
    const float ei = ep(i, x, y, z);
    const float kv = lapply_v<D, AS>(g, L, p, i, x, y, z, ep);
    (lp<AS>(L.t) + (int64_t)p * L.nc)[i] = dgv > 0.0f ? ei + w * (fv - kv) / dgv : ei;
    return;
  }
  const lfloat<AS>* src = lp<AS>(mode == 1 ? L.e : L.t) + (int64_t)p * L.nc;
  const float kv = lapply<D, AS>(g, L, p, src, i, x, y, z);
  const float v = dgv > 0.0f ? src[i] + w * (fv - kv) / dgv : src[i];
  if (mode == 4)
    gptr(d.pf_u)[ip] = ldexp((double)v, mg_scale_exp(gptr(d.pfs), p, L.nc));
  else
    (lp<AS>(mode == 1 ? L.t : L.e) + (int64_t)p * L.nc)[i] = v;
}

// f(C) at coarse cell i = sum over its aggregate of (f - K e) on F; smooth0:
// also C's first Jacobi pass (mode 0, pointwise): t = omega f / dg
template <int D, int AS>
__device__ __forceinline__ void mg_restrict_cell(const Grid& g, const MgLevel& F,
                                                 const MgLevel& C, int p, int i,
                                                 bool smooth0) {
  int X, Y, Z;
  lcell(C, i, X, Y, Z);
  const int xr = min(2 * X + 1, F.nx - 1), yt = min(2 * Y + 1, F.ny - 1),
            zt = D > 2 ? min(2 * Z + 1, F.nz - 1) : 0;
  const lfloat<AS>* e = lp<AS>(F.e) + (int64_t)p * F.nc;
  const lfloat<AS>* f = lp<AS>(F.f) + (int64_t)p * F.nc;
  float r = 0.0f;
  for (int z = 2 * Z; z <= zt; ++z)
    for (int y = 2 * Y; y <= yt; ++y)
      for (int x = 2 * X; x <= xr; ++x) {
        const int j = (z * F.ny + y) * F.nx + x;
        r += f[j] - lapply<D, AS>(g, F, p, e, j, x, y, z);
      }
  const int64_t ci = (int64_t)p * C.nc + i;
  lp<AS>(C.f)[ci] = r;
  if (smooth0) {
    const float dgc = lp<AS>(C.dg)[ci];
    lp<AS>(C.t)[ci] = dgc > 0.0f ? (float)mg_omega<D>() * r / dgc : 0.0f;
  }
}

template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_mg_smooth(const Desc* __restrict__ descs,
                                                         const int2* __restrict__ map, int ninst,
                                                         int l, int mode) {
  MG_PROLOGUE
  const MgLevel L = d.mg[l];
  if (i >= L.nc) return;
  MgLevel C;
  float corr = 0.0f;
  if (mode == 5) {
    C = d.mg[l + 1];
    corr = (float)s[kPfsCorr];
  }
#pragma unroll
  for (int p = 0; p < N; ++p)
    if (live[p]) mg_smooth_cell<D, 1>(d, L, p, (int)i, mode, &C, corr);
}

// f(l + 1) from level l (items over l + 1); smooth0: and t(l + 1)
template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_mg_restrict(const Desc* __restrict__ descs,
                                                           const int2* __restrict__ map, int ninst,
                                                           int l, int smooth0) {
  MG_PROLOGUE
  const MgLevel F = d.mg[l], C = d.mg[l + 1];
  if (i >= C.nc) return;
#pragma unroll
  for (int p = 0; p < N; ++p)
    if (live[p]) mg_restrict_cell<D, 1>(g, F, C, p, (int)i, smooth0 != 0);
}
#undef MG_PROLOGUE

// The V-cycle below level lf in one workgroup per instance.  Levels lf ..
// nlev - 1 are copied into LDS (face weights and diagonals, and f(lf)); every
// pass of the per-level kernels runs there, in the same order, separated by
// workgroup barriers instead of launches (the coarse levels are otherwise
// launch- and latency-bound); e(lf) goes back to global memory, where the
// first post-smoothing pass of level lf - 1 adds it (prolonged).  With
// lf = 0 the first pass reads the CG
// residual and the last one writes the preconditioned residual.  The host
// picks lf so that these levels fit the dynamic LDS of the launch (6 N floats
// per cell of each level).
constexpr int kMgFuseBlock = 1024;
constexpr int kMgFusedStatic = 4096;     // bytes kept for its static LDS

// level l's arrays in the LDS image, which holds levels lf .. l - 1 before it
template <int D>
__device__ __forceinline__ MgLevel mg_lds_level(const Desc& d, float* lds, int N, int lf, int l) {
  constexpr int A = mg_lds_arrays<D>();
  int64_t off = 0;
  for (int k = lf; k < l; ++k) off += A * (int64_t)N * d.mg[k].nc;
  MgLevel L = d.mg[l];
  const int64_t f = (int64_t)N * L.nc;
  float* b = lds + off;
  L.wx = b;
  L.wy = b + f;
  L.dg = b + 2 * f;
  L.e = b + 3 * f;
  L.t = b + 4 * f;
  L.f = b + 5 * f;
  if constexpr (D > 2) L.wz = b + 6 * f;
  return L;
}

template <int N, int D>
__global__ __launch_bounds__(kMgFuseBlock) void k_mg_fused(const Desc* __restrict__ descs,
                                                           int lf, int nlev) {
  extern __shared__ float mg_lds[];
  const Desc& d = descs[blockIdx.x];
  const Grid& g = d.g;
  const gdouble* s = gptr(d.pfs);
  bool live[N];
  bool any = false;
#pragma unroll
  for (int p = 0; p < N; ++p) {
    live[p] = s[kPfsDone + p] == 0.0;
    any = any || live[p];
  }
  if (!any) return;                       // uniform over the workgroup
  const float corr = (float)s[kPfsCorr];
  // the levels' LDS descriptors, built once (the level table is global memory,
  // which every barrier below would make the passes read again)
  __shared__ MgLevel lv[kMgMaxLev];
  static_assert(sizeof(lv) <= kMgFusedStatic, "static LDS of the fused cycle");
  if (threadIdx.x >= lf && threadIdx.x < nlev)
    lv[threadIdx.x] = mg_lds_level<D>(d, mg_lds, N, lf, threadIdx.x);
  for (int l = lf; l < nlev; ++l) {
    const MgLevel G = d.mg[l];
    const MgLevel L = mg_lds_level<D>(d, mg_lds, N, lf, l);
    const int f = N * (int)G.nc;
    for (int i = threadIdx.x; i < f; i += kMgFuseBlock) {
      lp<3>(L.wx)[i] = gptr(G.wx)[i];
      lp<3>(L.wy)[i] = gptr(G.wy)[i];
      if constexpr (D > 2) lp<3>(L.wz)[i] = gptr(G.wz)[i];
      lp<3>(L.dg)[i] = gptr(G.dg)[i];
      if (l == lf && lf > 0) lp<3>(L.f)[i] = gptr(G.f)[i];
    }
  }
  __syncthreads();
  // mode as in mg_smooth_cell; on level 0 mode 0 reads the residual (3) and
  // the last pass writes the preconditioned residual (4)
  auto smooth = [&](int l, int mode, bool last) {
    const MgLevel L = lv[l];
    const MgLevel* C = l + 1 < nlev ? &lv[l + 1] : nullptr;
    const int m = l > 0 ? mode : (mode == 0 ? 3 : (last ? 4 : mode));
    for (int i = threadIdx.x; i < (int)L.nc; i += kMgFuseBlock)
#pragma unroll
      for (int p = 0; p < N; ++p)
        if (live[p]) mg_smooth_cell<D, 3>(d, L, p, i, m, C, corr);
    __syncthreads();
  };
  const int lc = nlev - 1;
  smooth(lf, 0, false);
  for (int l = lf; l < lc; ++l) {
    smooth(l, 2, false);
    const MgLevel F = lv[l], C = lv[l + 1];
    for (int i = threadIdx.x; i < (int)C.nc; i += kMgFuseBlock)
#pragma unroll
      for (int p = 0; p < N; ++p)
        if (live[p]) mg_restrict_cell<D, 3>(g, F, C, p, i, true);   // f and t of l + 1
    __syncthreads();
  }
  smooth(lc, 2, kMgCoarseSweeps <= 2);
  for (int k = 2; k < kMgCoarseSweeps; k += 2) {
    smooth(lc, 1, false);
    smooth(lc, 2, k + 2 >= kMgCoarseSweeps);
  }
  for (int l = lc - 1; l >= lf; --l) {
    smooth(l, 5, false);                   // prolongation folded in
    smooth(l, 2, true);
  }
  if (lf > 0) {
    const MgLevel G = d.mg[lf], L = lv[lf];
    const int nc = (int)G.nc;
#pragma unroll
    for (int p = 0; p < N; ++p)
      if (live[p])
        for (int i = threadIdx.x; i < nc; i += kMgFuseBlock)
          gptr(G.e)[p * nc + i] = lp<3>(L.e)[p * nc + i];
  }
}

// allow the fused cycle's launches up to `bytes` of dynamic LDS
template <int N, int D>
hipError_t mg_fused_lds(int bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mg_fused<N, D>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// frozen face gradients dQ_p/dx_d at the upper face of every cell: none at an
// outflow end or for a phase with [div J] = 0 everywhere; clip != 0: limited
// to the Phase-Field CFL bound of the step's dt
template <int N, int D>
__global__ __launch_bounds__(kRedBlock) void k_pf_grad(const Desc* __restrict__ descs,
                                                       const int2* __restrict__ map, int ninst,
                                                       int clip) {
  const int2 it = locate(map, ninst, chunk_item());
  const Desc& d = descs[it.x];
  const Grid& g = d.g;
  const int64_t nc = g.nc;
  const gdouble* s = gptr(d.pfs);
  const int64_t c0 = (int64_t)it.y * d.chunk;
  const int64_t c1 = c0 + d.chunk < nc ? c0 + d.chunk : nc;
  const double dt = clip ? *gptr(d.dt) : 0.0;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += kRedBlock) {
    int x, y, z;
    cell_xyz(g, i, x, y, z);
#pragma unroll
    for (int p = 0; p < N; ++p) {
      const gdouble* Q = gptr(d.pf_q) + (int64_t)p * nc;
      const bool on = s[kPfsBB + p] > 0.0;
#pragma unroll
      for (int dir = 0; dir < D; ++dir) {
        const int64_t j = nbr(g, x, y, z, dir, 1);
        double G = 0.0;
        if (on && j >= 0) {
          const double rd = grid_rd(g, dir);
          G = (Q[j] - Q[i]) * rd;
          if (clip) {
            const double gm = kPfCfl / (dt * rd);
            G = fmin(fmax(G, -gm), gm);
          }
        }
        gptr(d.pf_g)[(int64_t)(dir * N + p) * nc + i] = G;
      }
    }
  }
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
  double* pf = nullptr;            // Phase-Field work arrays (one allocation)
  double* pfs = nullptr;           // Phase-Field scalars (kPfsLen)
  std::vector<MgLevel> lv;         // multigrid levels (host copy)
  MgLevel* d_mg = nullptr;         // the same on the device
  float* mgbuf = nullptr;          // arrays of the levels
};

// Instances of one (N, d): device descriptor table and tile offsets.
struct Group {
  int N = 0, D = 0;
  std::vector<int> ids;            // context instance indices
  std::vector<Desc> hdesc;         // host copy of the descriptors
  std::vector<int> xs[kXVar], ys[kYVar], zs[kYVar], rs;  // tile / chunk offsets (n + 1)
  Desc* desc = nullptr;
  int2* xmap[kXVar] = {};          // work item -> (instance, local tile)
  int2* ymap[kYVar] = {};
  int2* zmap[kYVar] = {};          // z sweep (3D): tiles of the y-sweep shapes
  int2* rmap = nullptr;
  int xv = 0, yv = 0;              // tile shapes in use (autotuned)
  int swz = -1;                    // XCD order: 0 off, 1 on, -1 on for groups
                                   // of several instances (measured: it keeps
                                   // each small instance on one L2 and costs a
                                   // few percent on a single grid)
  int* rstart = nullptr;           // reduction-chunk offsets on the device
  int* xstart[kXVar] = {};         // x-strip offsets per instance on the device
  double* cflp = nullptr;          // CFL rate per x strip (first stage of a step)
  size_t part_off = 0;             // this group's reduction partials
  int nlev = 0;                    // multigrid levels (every instance has them all)
  int mg_fuse = 0;                 // first level run by the fused coarse cycle
  size_t mg_lds = 0;               // its dynamic LDS bytes
  int2* lmap[kMgMaxLev] = {};      // work item -> (instance, 256-cell chunk) per level
  int lcount[kMgMaxLev] = {};
};

// Optional event pair recorded around one stage (profiling).
struct Bracket {
  int which = 0;                   // 0 none, 1 x sweep, 2 y sweep, 3 whole stage
  hipEvent_t ev[2] = {nullptr, nullptr};
};

// Entry g of a comma-separated list of integers ("1" or "0,2,1"); a list
// shorter than g + 1 entries gives its last one.
int env_entry(const char* s, int g) {
  for (int k = 0; k < g; ++k) {
    const char* c = std::strchr(s, ',');
    if (!c) break;
    s = c + 1;
  }
  return std::atoi(s);
}

// Strips of the x sweep over a grid: its ny nz rows of nx + 6 cells (the
// grid cells and three ghost cells on either side) laid end to end, bx - 2
// new cells a strip.
int64_t x_strips(const Grid& g, int bx) {
  return ((int64_t)g.ny * g.nz * (g.nx + 6) + bx - 3) / (bx - 2);
}

using StageFn = void (*)(const Group&, int stage, int swz, hipStream_t);
using RedFn = void (*)(const Group&, double* part, hipStream_t);
using DtFn = void (*)(const Group&, double* part, double cfl, int advance, hipStream_t);
// Phase-Field kernels: per-cell passes over reduction chunks and per-instance
// finishers (rtol is used by the finishers that test convergence)
using PfFn = void (*)(const Group&, double* part, int flag, double rtol, hipStream_t);

// stage | kStageCfl: the x sweep also reduces the CFL rates of U^n per strip
constexpr int kStageCfl = 8;

template <int N, int D, typename W, int PFM, int V>
void launch_x(const Group& G, int stage, int swz, hipStream_t s) {
  const int n = (int)G.ids.size();
  double* cflp = (stage & kStageCfl) ? G.cflp : nullptr;
  hipLaunchKernelGGL((k_sweep_x<N, D, W, PFM, kXS[V]>), dim3(G.xs[V][n]), dim3(kXS[V]), 0, s,
                     G.desc, G.xmap[V], n, stage & ~kStageCfl, swz, cflp);
}

// transverse sweep along DIR (1: y, 2: z) of a D-dimensional group
template <int N, typename W, int PFM, int V, int D, int DIR>
void launch_t(const Group& G, int stage, int swz, hipStream_t s) {
  const int n = (int)G.ids.size();
  const int tiles = DIR == 1 ? G.ys[V][n] : G.zs[V][n];
  hipLaunchKernelGGL((k_sweep_t<N, W, PFM, kYX[V], kYY[V], D, DIR>), dim3(tiles),
                     dim3(kYX[V] * kYY[V]), 0, s, G.desc, DIR == 1 ? G.ymap[V] : G.zmap[V], n,
                     stage, swz);
}

// kind: 0 prep, 1 divJ + CG start, 2 K u with the dot products, 3 axpy,
// 5 gradients
template <int N, int D, int KIND>
void launch_pf_cells(const Group& G, double* part, int flag, double, hipStream_t s) {
  const int n = (int)G.ids.size();
  double* pt = part + G.part_off;
  const dim3 grid(G.rs[n]), blk(kRedBlock);
  if constexpr (KIND == 0) hipLaunchKernelGGL((k_pf_prep<N, D>), grid, blk, 0, s, G.desc, G.rmap, n, pt);
  if constexpr (KIND == 1) hipLaunchKernelGGL((k_pf_divj<N, D>), grid, blk, 0, s, G.desc, G.rmap, n, pt, flag);
  if constexpr (KIND == 2) hipLaunchKernelGGL((k_pf_cg_dir<N, D>), grid, blk, 0, s, G.desc, G.rmap, n, pt);
  if constexpr (KIND == 3) hipLaunchKernelGGL((k_pf_cg_axpy<N, D>), grid, blk, 0, s, G.desc, G.rmap, n);
  if constexpr (KIND == 4) hipLaunchKernelGGL((k_pf_cg_dots<N, D>), grid, blk, 0, s, G.desc, G.rmap, n, pt);
  if constexpr (KIND == 5) hipLaunchKernelGGL((k_pf_grad<N, D>), grid, blk, 0, s, G.desc, G.rmap, n, flag);
  if constexpr (KIND == 6) hipLaunchKernelGGL((k_pf_guess<N, D>), grid, blk, 0, s, G.desc, G.rmap, n, flag);
}

// multigrid passes over the work items of level l (kind: 0 level-0 weights,
// 1 coarsen l -> l + 1, 2 diagonal, 3 smooth (mode), 4 restrict l -> l + 1
// (mode 1: with the first pass on l + 1), 6 the fused cycle from level l down)
using MgFn = void (*)(const Group&, int kind, int l, int mode, hipStream_t);
template <int N, int D>
void launch_mg(const Group& G, int kind, int l, int mode, hipStream_t s) {
  const int n = (int)G.ids.size();
  const dim3 blk(kRedBlock);
  switch (kind) {
    case 0: hipLaunchKernelGGL((k_mg_weights0<N, D>), dim3(G.lcount[0]), blk, 0, s, G.desc, G.lmap[0], n); break;
    case 1: hipLaunchKernelGGL((k_mg_coarsen<N, D>), dim3(G.lcount[l + 1]), blk, 0, s, G.desc, G.lmap[l + 1], n, l); break;
    case 2: hipLaunchKernelGGL((k_mg_diag<N, D>), dim3(G.lcount[l]), blk, 0, s, G.desc, G.lmap[l], n, l); break;
    case 3: hipLaunchKernelGGL((k_mg_smooth<N, D>), dim3(G.lcount[l]), blk, 0, s, G.desc, G.lmap[l], n, l, mode); break;
    case 4: hipLaunchKernelGGL((k_mg_restrict<N, D>), dim3(G.lcount[l + 1]), blk, 0, s, G.desc, G.lmap[l + 1], n, l, mode); break;
    case 6: hipLaunchKernelGGL((k_mg_fused<N, D>), dim3(n), dim3(kMgFuseBlock), G.mg_lds, s, G.desc, l, G.nlev); break;
  }
}

// kind: 0 setup (M, B), 1 CG start, 2 CG scalars
template <int N, int KIND>
void launch_pf_inst(const Group& G, double* part, int, double rtol, hipStream_t s) {
  const double* pt = part + G.part_off;
  const dim3 grid((unsigned)G.ids.size()), blk(kRedBlock);
  if constexpr (KIND == 0) hipLaunchKernelGGL((k_pf_setup<N>), grid, blk, 0, s, G.desc, G.rstart, pt);
  if constexpr (KIND == 1) hipLaunchKernelGGL((k_pf_cg_start<N>), grid, blk, 0, s, G.desc, G.rstart, pt, rtol);
  if constexpr (KIND == 2) hipLaunchKernelGGL((k_pf_cg_alpha<N>), grid, blk, 0, s, G.desc, G.rstart, pt);
  if constexpr (KIND == 3) hipLaunchKernelGGL((k_pf_cg_beta<N>), grid, blk, 0, s, G.desc, G.rstart, pt, rtol);
}

template <int N, int D>
void launch_dt(const Group& G, double* part, double cfl, int advance, hipStream_t s) {
  const int n = (int)G.ids.size();
  hipLaunchKernelGGL((k_dt<N, D>), dim3(G.rs[n]), dim3(kRedBlock), 0, s, G.desc, G.rmap,
                     n, part + G.part_off);
  hipLaunchKernelGGL(k_dt_finish, dim3(n), dim3(kDtBlock), 0, s, G.desc, G.rstart,
                     part + G.part_off, cfl, advance);
}

template <int N, int D>
void launch_diag(const Group& G, double* part, hipStream_t s) {
  const int n = (int)G.ids.size();
  hipLaunchKernelGGL((k_diag<N, D>), dim3(G.rs[n]), dim3(kRedBlock), 0, s, G.desc, G.rmap,
                     n, part + G.part_off);
}

// ---------------------------------------------------------------------------
// scratch of the allocation-free L(U) entry point
// ---------------------------------------------------------------------------
// One file-scope array per GPU (the loader places it when the library's code
// object is loaded on a device; it lives until the process ends).  Layout:
// the instance descriptor in the first kNoallocDescBytes, then the direction
// accumulator of the x sweep (n_U doubles per cell, 2D and 3D).  Host code
// never uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
constexpr size_t kNoallocDescBytes = 4096;
static_assert(sizeof(Desc) <= kNoallocDescBytes, "descriptor slot");
static __device__ __align__(256) double scratch[kNoallocScratchBytes / sizeof(double)];

// The descriptor arrives by value (a kernel argument), so no host buffer
// has to outlive the launch, and a graph captured around the call holds no
// copy node.
__global__ void k_put_desc(Desc d, Desc* dst) {
  if (threadIdx.x == 0) *dst = d;
}

// L(U) of one instance (stage 3: rin -> rout) with the default tile shapes,
// the descriptor at desc (a group of one: no tile map is read)
template <int N, int D, typename W, int PFM>
void launch_rhs_single(const Desc* desc, const Grid& g, hipStream_t s) {
  hipLaunchKernelGGL((k_sweep_x<N, D, W, PFM, kXS[0]>), dim3((unsigned)x_strips(g, kXS[0])),
                     dim3(kXS[0]), 0, s, desc, nullptr, 1, 3, 0, nullptr);
  if constexpr (D >= 2) {
    constexpr int oy = kYY[0] - 2;
    const int64_t ntx = (g.nx + kYX[0] - 1) / kYX[0];
    hipLaunchKernelGGL((k_sweep_t<N, W, PFM, kYX[0], kYY[0], D, 1>),
                       dim3((unsigned)(ntx * ((g.ny + oy - 1) / oy) * g.nz)),
                       dim3(kYX[0] * kYY[0]), 0, s, desc, nullptr, 1, 3, 0);
    if constexpr (D == 3)
      hipLaunchKernelGGL((k_sweep_t<N, W, PFM, kYX[0], kYY[0], D, 2>),
                         dim3((unsigned)(ntx * ((g.nz + oy - 1) / oy) * g.ny)),
                         dim3(kYX[0] * kYY[0]), 0, s, desc, nullptr, 1, 3, 0);
  }
}

using RhsSingleFn = void (*)(const Desc*, const Grid&, hipStream_t);

// the per-(N, d) kernels of the two-level coupling: (links, items, count,
// stage, stream)
using AmrFn = void (*)(const AmrLink*, const int2*, int, int, hipStream_t);
template <int N, int D, typename W>
void launch_amr_flux(const AmrLink* l, const int2* items, int n, int stage, hipStream_t s) {
  hipLaunchKernelGGL((k_amr_flux<N, D, W>), dim3((n + 63) / 64), dim3(64), 0, s, l, items, n,
                     stage);
}
template <int N, int D>
void launch_amr_comb(const AmrLink* l, const int2* faces, int n, int stage, hipStream_t s) {
  hipLaunchKernelGGL((k_amr_combine<N, D>), dim3((n + 63) / 64), dim3(64), 0, s, l, faces, n,
                     stage);
}

// Sweep tables: [variant][N][d][precision][shape], variant kRiemann,
// kPfFlux or kRiemannCmp (the last two with the default shapes only)
struct Table {
  StageFn sx[3][kMaxN + 1][4][2][kXVar] = {};
  RhsSingleFn rhs1[2][kMaxN + 1][4][2] = {};    // allocation-free L(U): [comparison][N][d][prec]
  AmrFn amrflux[kMaxN + 1][3][2] = {};          // interface fluxes of linked levels
  AmrFn amrcomb[kMaxN + 1][3] = {};             // their stage corrections
  StageFn sy[3][kMaxN + 1][2][kYVar] = {};      // 2D y sweep
  StageFn sy3[3][kMaxN3 + 1][2][kYVar] = {};    // 3D y sweep (adds to the accumulator)
  StageFn sz3[3][kMaxN3 + 1][2][kYVar] = {};    // 3D z sweep (finishes the stage)
  DtFn dt[kMaxN + 1][4] = {};
  RedFn diag[kMaxN + 1][4] = {};
  PfFn pfc[7][kMaxN + 1][4] = {};          // per-cell PF passes: [kind][N][d]
  PfFn pfi[4][kMaxN + 1] = {};             // per-instance PF finishers
  MgFn mg[kMaxN + 1][4] = {};
  hipError_t (*mg_lds[kMaxN + 1][4])(int) = {};
};

template <int N, int D>
void fill_pf(Table& t) {
  t.pfc[0][N][D] = launch_pf_cells<N, D, 0>;
  t.pfc[1][N][D] = launch_pf_cells<N, D, 1>;
  t.pfc[2][N][D] = launch_pf_cells<N, D, 2>;
  t.pfc[3][N][D] = launch_pf_cells<N, D, 3>;
  t.pfc[4][N][D] = launch_pf_cells<N, D, 4>;
  t.pfc[5][N][D] = launch_pf_cells<N, D, 5>;
  t.pfc[6][N][D] = launch_pf_cells<N, D, 6>;
  t.mg[N][D] = launch_mg<N, D>;
  t.mg_lds[N][D] = mg_fused_lds<N, D>;
}

// the Riemann-flux sweeps of shape V; F: kRiemann or kRiemannCmp
template <int N, int V, int F>
void fill_shapes(Table& t) {
  constexpr int C = F == kRiemannCmp;
  t.sx[F][N][1][0][V] = launch_x<N, 1, double, F, V>;
  t.sx[F][N][1][1][V] = launch_x<N, 1, float, F, V>;
  t.sx[F][N][2][0][V] = launch_x<N, 2, double, F, V>;
  t.sx[F][N][2][1][V] = launch_x<N, 2, float, F, V>;
  t.sy[F][N][0][V] = launch_t<N, double, F, V, 2, 1>;
  t.sy[F][N][1][V] = launch_t<N, float, F, V, 2, 1>;
  if constexpr (N <= kMaxN3) {
    t.sx[F][N][3][0][V] = launch_x<N, 3, double, F, V>;
    t.sx[F][N][3][1][V] = launch_x<N, 3, float, F, V>;
    t.sy3[F][N][0][V] = launch_t<N, double, F, V, 3, 1>;
    t.sy3[F][N][1][V] = launch_t<N, float, F, V, 3, 1>;
    t.sz3[F][N][0][V] = launch_t<N, double, F, V, 3, 2>;
    t.sz3[F][N][1][V] = launch_t<N, float, F, V, 3, 2>;
  }
  if constexpr (V == 0) {
    t.rhs1[C][N][1][0] = launch_rhs_single<N, 1, double, F>;
    t.rhs1[C][N][1][1] = launch_rhs_single<N, 1, float, F>;
    t.rhs1[C][N][2][0] = launch_rhs_single<N, 2, double, F>;
    t.rhs1[C][N][2][1] = launch_rhs_single<N, 2, float, F>;
    if constexpr (N <= kMaxN3) {
      t.rhs1[C][N][3][0] = launch_rhs_single<N, 3, double, F>;
      t.rhs1[C][N][3][1] = launch_rhs_single<N, 3, float, F>;
    }
  }
}

template <int N>
void fill(Table& t) {
  t.amrflux[N][1][0] = launch_amr_flux<N, 1, double>;
  t.amrflux[N][1][1] = launch_amr_flux<N, 1, float>;
  t.amrflux[N][2][0] = launch_amr_flux<N, 2, double>;
  t.amrflux[N][2][1] = launch_amr_flux<N, 2, float>;
  t.amrcomb[N][1] = launch_amr_comb<N, 1>;
  t.amrcomb[N][2] = launch_amr_comb<N, 2>;
  fill_shapes<N, 0, kRiemann>(t);
  if constexpr (N <= kMaxNT) {
    fill_shapes<N, 1, kRiemann>(t);
    fill_shapes<N, 2, kRiemann>(t);
  }
  fill_shapes<N, 0, kRiemannCmp>(t);
  // the Phase-Field sweeps: default shapes only
  t.sx[kPfFlux][N][1][0][0] = launch_x<N, 1, double, kPfFlux, 0>;
  t.sx[kPfFlux][N][1][1][0] = launch_x<N, 1, float, kPfFlux, 0>;
  t.sx[kPfFlux][N][2][0][0] = launch_x<N, 2, double, kPfFlux, 0>;
  t.sx[kPfFlux][N][2][1][0] = launch_x<N, 2, float, kPfFlux, 0>;
  t.sy[kPfFlux][N][0][0] = launch_t<N, double, kPfFlux, 0, 2, 1>;
  t.sy[kPfFlux][N][1][0] = launch_t<N, float, kPfFlux, 0, 2, 1>;
  if constexpr (N <= kMaxN3) {
    t.sx[kPfFlux][N][3][0][0] = launch_x<N, 3, double, kPfFlux, 0>;
    t.sx[kPfFlux][N][3][1][0] = launch_x<N, 3, float, kPfFlux, 0>;
    t.sy3[kPfFlux][N][0][0] = launch_t<N, double, kPfFlux, 0, 3, 1>;
    t.sy3[kPfFlux][N][1][0] = launch_t<N, float, kPfFlux, 0, 3, 1>;
    t.sz3[kPfFlux][N][0][0] = launch_t<N, double, kPfFlux, 0, 3, 2>;
    t.sz3[kPfFlux][N][1][0] = launch_t<N, float, kPfFlux, 0, 3, 2>;
    fill_pf<N, 3>(t);
  }
  fill_pf<N, 1>(t);
  fill_pf<N, 2>(t);
  t.pfi[0][N] = launch_pf_inst<N, 0>;
  t.pfi[1][N] = launch_pf_inst<N, 1>;
  t.pfi[2][N] = launch_pf_inst<N, 2>;
  t.pfi[3][N] = launch_pf_inst<N, 3>;
  t.dt[N][1] = launch_dt<N, 1>;
  t.dt[N][2] = launch_dt<N, 2>;
  t.diag[N][1] = launch_diag<N, 1>;
  t.diag[N][2] = launch_diag<N, 2>;
  if constexpr (N <= kMaxN3) {
    t.dt[N][3] = launch_dt<N, 3>;
    t.diag[N][3] = launch_diag<N, 3>;
  }
}

static const Table& table() {
  static Table t = [] {
    Table x;
    fill<1>(x); fill<2>(x); fill<3>(x); fill<4>(x); fill<5>(x); fill<6>(x); fill<7>(x);
    fill<8>(x);
    return x;
  }();
  return t;
}

}  // namespace mpw

using namespace mpw;

// Grid and EOS part of an instance descriptor (every other field zero).
// A_p, B_p of Eq. (26) and EB_p = A_p Pmin_p + B_p of Eq. (9).
static void desc_grid_eos(const mp_weno_instance& s, const mp_weno_opts& opt, Desc& d) {
  std::memset(&d, 0, sizeof(d));
  const int D = s.ndim;
  Grid& g = d.g;
  g.nx = s.n[0];
  g.ny = D > 1 ? s.n[1] : 1;
  g.nz = D > 2 ? s.n[2] : 1;
  g.nc = (int64_t)g.nx * g.ny * g.nz;
  g.rdx = 1.0 / s.dx[0];
  g.hdx = 0.5 * s.dx[0];
  g.rdy = D > 1 ? 1.0 / s.dx[1] : 0.0;
  g.hdy = D > 1 ? 0.5 * s.dx[1] : 1.0;
  g.bcx0 = s.bc[0][0]; g.bcx1 = s.bc[0][1];
  g.bcy0 = D > 1 ? s.bc[1][0] : 0;
  g.bcy1 = D > 1 ? s.bc[1][1] : 0;
  g.rdz = D > 2 ? 1.0 / s.dx[2] : 0.0;
  g.hdz = D > 2 ? 0.5 * s.dx[2] : 1.0;
  g.bcz0 = D > 2 ? s.bc[2][0] : 0;
  g.bcz1 = D > 2 ? s.bc[2][1] : 0;
  g.recon = opt.recon;
  g.flux = opt.flux;
  g.model = opt.model;
  g.energy = opt.energy_limiter ? 1 : 0;
  g.asrc = opt.alpha_source;
  for (int p = 0; p < s.nphase; ++p) {
    const double gm = s.gamma[p], pi = s.pinf[p];
    d.e.A[p] = 1.0 / (gm - 1.0);
    d.e.B[p] = gm * pi / (gm - 1.0);
    d.e.Dp[p] = s.D[p];
    d.e.gam[p] = gm;
    d.e.pinf[p] = pi;
    d.e.EB[p] = d.e.A[p] * s.pmin[p] + d.e.B[p];
  }
}

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
  double* pfs = nullptr;      // n_inst * kPfsLen Phase-Field scalars
  hipGraphExec_t graph[2] = {nullptr, nullptr};   // [external dt?]
  // kChain consecutive steps (device CFL step) captured as one graph
  static constexpr int kChain = 16;
  hipGraphExec_t chain = nullptr;
  // Phase-Field solve: one captured batch of CG iterations (replayed on
  // stream), the private stream it is captured on, pinned done flags
  hipGraphExec_t pf_graph = nullptr;
  hipStream_t cap_stream = nullptr;
  double* pf_flags = nullptr;
  // two-level coupling (mp_weno_amr_link): device link table, flux items
  // (link, 3 face + k), faces (link, face), the linked instances, one buffer
  // of interface fluxes and registers; all linked instances share (N, d)
  AmrLink* amr = nullptr;
  int2* amr_items = nullptr;
  int2* amr_faces = nullptr;
  int* amr_ids = nullptr;
  double* amr_buf = nullptr;
  int amr_nlinks = 0, amr_nitems = 0, amr_nfaces = 0, amr_nids = 0, amr_N = 0, amr_D = 0;
  int amr_maxcells = 0;       // largest fine grid (ghost-fill launch size)
  std::string err;
  int profile = 0;            // Bracket::which
  // solutions of the Q solve kept in pf_q, pf_qp, pf_qpp: 0 none, 1 the
  // last one, 2 or 3 the last two or three (the next solve starts from their
  // extrapolation)
  int pf_hist = 0;
  // the step in progress takes its CFL step in its first stage (2D and 3D
  // groups: from the rates the x sweeps reduce), with this time advance
  bool cfl_pending = false;
  int cfl_advance = 0;
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

// one RK stage (s = 0, 1, 2) or L(U) (s = 3) of every group; pf selects the
// Phase-Field flux instead of the Riemann solver
static mp_status enqueue_stage(mp_weno_ctx* c, int s, int pf = 0) {
  const Table& T = table();
  const int prec = c->opt.precision;
  Bracket br;
  const Bracket* b = (s < 3 && !pf) ? c->next_bracket(br) : nullptr;
  const int w = b ? b->which : 0;
  if (w == 1 || w == 3) HIPCHK(c, hipEventRecord(b->ev[0], c->stream));
  auto swz = [](const Group& G) {
    if (G.swz >= 0) return G.swz;
    return G.ids.size() > 1 ? 1 : 0;
  };
  // the comparison schemes and the Phase-Field flux run the default shapes
  const int cmp = c->opt.recon >= MP_RECON_WENO_JS;
  const int v = pf ? kPfFlux : (cmp ? kRiemannCmp : kRiemann);
  // the first stage of a step: 2D and 3D groups reduce the CFL rates of U^n
  // in their x sweeps, and the step (and time advance) follows from them
  // before the transverse sweeps, which are the first to use it
  const bool cfl = s == 0 && !pf && c->cfl_pending;
  for (const Group& G : c->groups)
    T.sx[v][G.N][G.D][prec][v ? 0 : G.xv](G, s | (cfl && G.D >= 2 ? kStageCfl : 0), swz(G),
                                         c->stream);
  if (cfl) {
    for (const Group& G : c->groups)
      if (G.D >= 2)
        hipLaunchKernelGGL(k_dt_finish, dim3(G.ids.size()), dim3(kDtBlock), 0, c->stream, G.desc,
                           G.xstart[v ? 0 : G.xv], G.cflp, c->opt.cfl, c->cfl_advance);
    c->cfl_pending = false;
  }
  if (w == 1) HIPCHK(c, hipEventRecord(b->ev[1], c->stream));
  if (w == 2) HIPCHK(c, hipEventRecord(b->ev[0], c->stream));
  for (const Group& G : c->groups) {
    if (G.D == 2) T.sy[v][G.N][prec][v ? 0 : G.yv](G, s, swz(G), c->stream);
    if (G.D == 3) T.sy3[v][G.N][prec][v ? 0 : G.yv](G, s, swz(G), c->stream);
  }
  for (const Group& G : c->groups)
    if (G.D == 3) T.sz3[v][G.N][prec][v ? 0 : G.yv](G, s, swz(G), c->stream);
  if (w == 2 || w == 3) HIPCHK(c, hipEventRecord(b->ev[1], c->stream));
  HIPCHK(c, hipGetLastError());
  return MP_OK;
}

// CFL step of every instance; advance: also move time and step count on
static mp_status enqueue_dt(mp_weno_ctx* c, int advance, bool only_1d = false) {
  const Table& T = table();
  for (const Group& G : c->groups)
    if (!only_1d || G.D == 1) T.dt[G.N][G.D](G, c->part, c->opt.cfl, advance, c->stream);
  HIPCHK(c, hipGetLastError());
  return MP_OK;
}

// Multigrid: level weights and diagonals for the frozen k (once per solve)
static void enqueue_mg_setup(mp_weno_ctx* c, hipStream_t st) {
  const Table& T = table();
  for (const Group& G : c->groups) {
    MgFn f = T.mg[G.N][G.D];
    f(G, 0, 0, 0, st);                               // level-0 weights
    f(G, 2, 0, 0, st);                               // and diagonal
    for (int l = 0; l + 1 < G.nlev; ++l) {
      f(G, 1, l, 0, st);                             // weights of l + 1
      f(G, 2, l + 1, 0, st);                         // diagonal of l + 1
    }
  }
}

// u = M^-1 r: one V-cycle per group (two Jacobi sweeps before and after the
// coarse correction, kMgCoarseSweeps on the coarsest level); the coarsest
// levels that fit in LDS run in one launch (k_mg_fused)
static void enqueue_vcycle(mp_weno_ctx* c, hipStream_t st) {
  const Table& T = table();
  for (const Group& G : c->groups) {
    MgFn f = T.mg[G.N][G.D];
    const int Lf = G.mg_fuse;                        // fused from here down
    if (Lf > 0) f(G, 3, 0, 3, st);                   // t = omega f / dg, f from r
    for (int l = 0; l < Lf; ++l) {
      f(G, 3, l, 2, st);                             // e = t + omega (f - K t) / dg
      f(G, 4, l, l + 1 < Lf ? 1 : 0, st);            // f(l + 1) = R (f - K e) (and its t)
    }
    f(G, 6, Lf, 0, st);                              // levels Lf .. nlev - 1
    for (int l = Lf - 1; l >= 0; --l) {
      f(G, 3, l, 5, st);                             // t = e' + omega (f - K e') / dg, e' = e + P e(l + 1)
      f(G, 3, l, l == 0 ? 4 : 2, st);                // e = t + omega (f - K t) / dg (level 0: u)
    }
  }
}

// [div J], the Q solve and the frozen gradients of every instance, from the
// volume fractions of each descriptor's pfin.  The CG loop is driven from the
// host: batches of iterations, then a look at the per-phase done flags
// (synchronises the stream).  cold: start from Q = 0 instead of the last Q.
static mp_status run_pf_solve(mp_weno_ctx* c, int cold, int clip) {
  const Table& T = table();
  const double rtol = c->opt.cg_rtol > 0.0 ? c->opt.cg_rtol : 1e-12;
  const int maxit = c->opt.cg_maxit > 0 ? c->opt.cg_maxit : 10000;
  // CG restarts after a breakdown or a recurrence that drifted from the true
  // residual (each restart recomputes the residual from Q)
  constexpr int kMaxRestarts = 16;
  for (const Group& G : c->groups) {
    T.pfc[0][G.N][G.D](G, c->part, 0, rtol, c->stream);     // k, max|u|, integrands
    T.pfi[0][G.N](G, c->part, 0, rtol, c->stream);          // M, B
  }
  HIPCHK(c, hipGetLastError());
  const size_t n = c->inst.size();
  if (!c->pf_flags)
    HIPCHK(c, hipHostMalloc((void**)&c->pf_flags, sizeof(double) * n * kPfsLen, 0));
  // z = M^-1 r, the dot products, beta and the done flags
  auto precondition = [&](hipStream_t st) {
    enqueue_vcycle(c, st);
    for (const Group& G : c->groups) {
      T.pfc[4][G.N][G.D](G, c->part, 0, rtol, st);
      T.pfi[3][G.N](G, c->part, 0, rtol, st);
    }
  };
  // kBatch iterations (direction and K p, alpha, Q and r, then the above);
  // phases that are done skip their work
  constexpr int kBatch = 4;
  auto batch = [&](int nb, hipStream_t st) {
    for (int k = 0; k < nb; ++k) {
      for (const Group& G : c->groups) {
        T.pfc[2][G.N][G.D](G, c->part, 0, rtol, st);
        T.pfi[2][G.N](G, c->part, 0, rtol, st);
        T.pfc[3][G.N][G.D](G, c->part, 0, rtol, st);
      }
      precondition(st);
    }
  };
  if (!c->pf_graph) {
    // captured once on a private stream (a context on the null stream can
    // still replay it) and launched on the context's stream
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipGraph_t gph;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    batch(kBatch, c->cap_stream);
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &gph);
    if (e1 != hipSuccess || e2 != hipSuccess)
      return fail(c, MP_ERR_HIP, "capture of the Phase-Field solve failed");
    const hipError_t e3 = hipGraphInstantiate(&c->pf_graph, gph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gph);
    if (e3 != hipSuccess) {
      c->pf_graph = nullptr;
      return fail(c, MP_ERR_HIP, hipGetErrorString(e3));
    }
  }
  // the per-phase done flags, read back (synchronises the stream)
  auto all_done = [&](bool& done) -> mp_status {
    HIPCHK(c, hipMemcpyAsync(c->pf_flags, c->pfs, sizeof(double) * n * kPfsLen,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    done = true;
    for (size_t i = 0; i < n && done; ++i)
      for (int p = 0; p < c->inst[i].N; ++p)
        if (c->pf_flags[i * kPfsLen + kPfsDone + p] == 0.0) { done = false; break; }
    return MP_OK;
  };
  // the start of a warm solve: the last three solutions extrapolated in time
  // (the last two, or the last one, while fewer are known)
  const int hist = c->pf_hist;
  if (!cold)
    for (const Group& G : c->groups)
      T.pfc[6][G.N][G.D](G, c->part, hist >= 3 ? 2 : (hist >= 2 ? 1 : 0), rtol, c->stream);
  c->pf_hist = 0;                  // until this solve has converged
  bool converged = false;
  int it = 0, restart = 0;
  for (; restart <= kMaxRestarts; ++restart) {
    // [div J], the true residual r = -b - K Q and the done flags from it
    for (const Group& G : c->groups) {
      T.pfc[1][G.N][G.D](G, c->part, cold && restart == 0, rtol, c->stream);
      T.pfi[1][G.N](G, c->part, 0, rtol, c->stream);
    }
    HIPCHK(c, hipGetLastError());
    bool done = false;
    mp_status st = all_done(done);
    if (st != MP_OK) return st;
    if (done) { converged = true; break; }
    if (it >= maxit) break;
    // the hierarchy of the phases left to solve (the multigrid passes skip
    // phases that are done, so this follows the first start pass)
    if (restart == 0) enqueue_mg_setup(c, c->stream);
    precondition(c->stream);
    HIPCHK(c, hipGetLastError());
    for (;;) {
      st = all_done(done);
      if (st != MP_OK) return st;
      if (done || it >= maxit) break;
      const int nb = std::min(kBatch, maxit - it);
      it += nb;
      if (nb == kBatch) {
        HIPCHK(c, hipGraphLaunch(c->pf_graph, c->stream));
      } else {
        batch(nb, c->stream);
        HIPCHK(c, hipGetLastError());
      }
    }
  }
  for (const Group& G : c->groups) T.pfc[5][G.N][G.D](G, c->part, clip, rtol, c->stream);
  HIPCHK(c, hipGetLastError());
  if (!converged) {
    // the largest true relative residual of the last start pass
    double rmax = 0.0;
    for (size_t i = 0; i < n; ++i) rmax = std::max(rmax, c->pf_flags[i * kPfsLen + kPfsRes]);
    char msg[160];
    std::snprintf(msg, sizeof(msg),
                  "Phase-Field CG did not reach cg_rtol: relative residual %.3e after %d "
                  "iterations and %d restarts", rmax, it, std::min(restart, kMaxRestarts));
    return fail(c, MP_ERR_SOLVER, msg);
  }
  // a cold solve starts the history; a warm one has moved the earlier
  // solutions (where there were any) to pf_qp and pf_qpp
  c->pf_hist = cold ? 1 : std::min(hist + 1, 3);
  return MP_OK;
}

// the RK stages (and the Phase-Field step); advance: move time and step
// count on at the end (when the CFL kernel did not)
// two-level coupling around stage s: ghost fill of the fine blocks from the
// coarse stage state, interface fluxes of both levels and their correction
static void enqueue_amr_stage(mp_weno_ctx* c, int s) {
  const Table& T = table();
  const int nU = 2 * c->amr_N + c->amr_D + 1;
  const int blocks = std::max(1, std::min(1024, (c->amr_maxcells + 255) / 256));
  hipLaunchKernelGGL(k_amr_prolong, dim3(blocks, c->amr_nlinks), dim3(256), 0, c->stream,
                     c->amr, s, nU);
  T.amrflux[c->amr_N][c->amr_D][c->opt.precision](c->amr, c->amr_items, c->amr_nitems, s,
                                                  c->stream);
  T.amrcomb[c->amr_N][c->amr_D](c->amr, c->amr_faces, c->amr_nfaces, s, c->stream);
}

static mp_status enqueue_rk(mp_weno_ctx* c, bool advance) {
  for (int s = 0; s < 3; ++s) {
    if (c->amr_nlinks) enqueue_amr_stage(c, s);
    mp_status st = enqueue_stage(c, s);
    if (st != MP_OK) return st;
  }
  if (c->amr_nlinks) {
    const int nU = 2 * c->amr_N + c->amr_D + 1;
    hipLaunchKernelGGL(k_amr_restrict, dim3(64, c->amr_nlinks), dim3(256), 0, c->stream, c->amr,
                       nU);
    hipLaunchKernelGGL(k_amr_reflux, dim3((c->amr_nfaces + 63) / 64), dim3(64), 0, c->stream,
                       c->amr, c->amr_faces, c->amr_nfaces, nU);
    // the rings hold the new coarse values between steps (the CFL step and
    // the diagnostics read them)
    const int blocks = std::max(1, std::min(1024, (c->amr_maxcells + 255) / 256));
    hipLaunchKernelGGL(k_amr_prolong, dim3(blocks, c->amr_nlinks), dim3(256), 0, c->stream,
                       c->amr, 0, nU);
  }
  if (c->opt.phase_field) {
    // the Phase-Field step on the hyperbolic result, same dt
    mp_status st = run_pf_solve(c, 0, 1);
    if (st != MP_OK) return st;
    for (int s = 0; s < 3; ++s) {
      st = enqueue_stage(c, s, 1);
      if (st != MP_OK) return st;
    }
  }
  if (advance) {
    const int n = (int)c->inst.size();
    hipLaunchKernelGGL(k_advance_time, dim3((n + 255) / 256), dim3(256), 0, c->stream, c->t,
                       c->steps, c->dt, n);
  }
  HIPCHK(c, hipGetLastError());
  return MP_OK;
}

static mp_status enqueue_diag(mp_weno_ctx* c) {
  const Table& T = table();
  for (const Group& G : c->groups) {
    T.diag[G.N][G.D](G, c->part, c->stream);
    hipLaunchKernelGGL(k_diag_finish, dim3(G.ids.size()), dim3(64), 0, c->stream, G.desc,
                       G.rstart, c->part + G.part_off);
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
  if (c->chain) (void)hipGraphExecDestroy(c->chain);
  if (c->pf_graph) (void)hipGraphExecDestroy(c->pf_graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->pf_flags) (void)hipHostFree(c->pf_flags);
  for (auto& e : c->events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& I : c->inst) {
    (void)hipFree(I.U1); (void)hipFree(I.U2); (void)hipFree(I.acc); (void)hipFree(I.backup);
    (void)hipFree(I.pf); (void)hipFree(I.mgbuf); (void)hipFree(I.d_mg);
  }
  for (auto& G : c->groups) {
    (void)hipFree(G.desc); (void)hipFree(G.rmap); (void)hipFree(G.rstart); (void)hipFree(G.cflp);
    for (auto* m : G.xmap) (void)hipFree(m);
    for (auto* m : G.xstart) (void)hipFree(m);
    for (auto* m : G.ymap) (void)hipFree(m);
    for (auto* m : G.zmap) (void)hipFree(m);
    for (auto* m : G.lmap) (void)hipFree(m);
  }
  (void)hipFree(c->dt); (void)hipFree(c->t); (void)hipFree(c->steps); (void)hipFree(c->part);
  (void)hipFree(c->diag); (void)hipFree(c->pfs);
  (void)hipFree(c->amr); (void)hipFree(c->amr_items); (void)hipFree(c->amr_faces);
  (void)hipFree(c->amr_ids); (void)hipFree(c->amr_buf);
  delete c;
  return MP_OK;
}

static mp_status validate(int32_t n_inst, const mp_weno_instance* inst,
                          const mp_weno_opts* opt, void* hip_stream) {
  if (n_inst < 1 || !inst || !opt) return MP_ERR_ARG;
  if (opt->phase_field != 0 && opt->phase_field != 1) return MP_ERR_ARG;
  if (opt->phase_field && !(opt->eta_over_dx > 0.0)) return MP_ERR_ARG;
  if (opt->precision != MP_PREC_FP64 && opt->precision != MP_PREC_MIXED) return MP_ERR_ARG;
  if (opt->recon < 0 || opt->recon > 3 || opt->flux < 0 || opt->flux > 1 ||
      opt->model < 0 || opt->model > 1 || !(opt->cfl > 0.0) ||
      (opt->alpha_source != MP_SRC_CELL && opt->alpha_source != MP_SRC_NORMALIZED))
    return MP_ERR_ARG;
  if (opt->use_graph && !hip_stream) return MP_ERR_ARG;   // no capture on the null stream
  for (int i = 0; i < n_inst; ++i) {
    const mp_weno_instance& s = inst[i];
    if (s.ndim < 1 || s.ndim > 3 || !s.U) return MP_ERR_ARG;
    if (s.nphase < 1 || s.nphase > MP_MAXP) return MP_ERR_ARG;
    if (s.nphase > kMaxN || (s.ndim == 3 && s.nphase > kMaxN3)) return MP_ERR_UNSUPPORTED;
    for (int d = 0; d < s.ndim; ++d) {
      if (s.n[d] < 1 || !(s.dx[d] > 0.0)) return MP_ERR_ARG;
      for (int k = 0; k < 2; ++k)
        if (s.bc[d][k] < MP_BC_PERIODIC || s.bc[d][k] > MP_BC_SYMMETRY) return MP_ERR_ARG;
      if ((s.bc[d][0] == MP_BC_PERIODIC) != (s.bc[d][1] == MP_BC_PERIODIC)) return MP_ERR_ARG;
    }
    for (int p = 0; p < s.nphase; ++p)
      if (!(s.gamma[p] > 1.0) || !std::isfinite(s.pinf[p]) || !std::isfinite(s.D[p]) ||
          !std::isfinite(s.pmin[p]))
        return MP_ERR_ARG;
    const int64_t nc = (int64_t)s.n[0] * (s.ndim > 1 ? s.n[1] : 1) * (s.ndim > 2 ? s.n[2] : 1);
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
  // initial tile shapes and tile order from the environment (indices into
  // kXS / kYX, kYY; 0 / 1 for the order), one value for every group or a
  // comma-separated list with one entry per group in group order (d, then
  // N, ascending; a short list repeats its last entry); later changed only
  // by mp_weno_autotune.  The comparison schemes are built with the default
  // shapes only.
  const char* sw = std::getenv("MPWENO_XCD_SWIZZLE");
  const char* xsh = std::getenv("MPWENO_XSHAPE");
  const char* ysh = std::getenv("MPWENO_YSHAPE");
  const bool cmp = opt->recon >= MP_RECON_WENO_JS;
  int ngroup = 0;
  const size_t n = (size_t)n_inst;
  if (hipMalloc(&c->dt, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&c->t, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&c->steps, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&c->diag, sizeof(double) * n * MP_DIAG_LEN) != hipSuccess ||
      (opt->phase_field && hipMalloc(&c->pfs, sizeof(double) * n * kPfsLen) != hipSuccess)) {
    mp_weno_destroy(c);
    return MP_ERR_OOM;
  }
  for (int i = 0; i < n_inst; ++i) {
    Inst I;
    I.in = inst[i];
    I.N = inst[i].nphase;
    I.D = inst[i].ndim;
    I.nU = 2 * I.N + I.D + 1;
    I.nc = (int64_t)inst[i].n[0] * (I.D > 1 ? inst[i].n[1] : 1) * (I.D > 2 ? inst[i].n[2] : 1);
    const size_t bytes = sizeof(double) * (size_t)I.nU * (size_t)I.nc;
    const bool ok = hipMalloc(&I.U1, bytes) == hipSuccess &&
                    hipMalloc(&I.U2, bytes) == hipSuccess &&
                    (I.D == 1 || hipMalloc(&I.acc, bytes) == hipSuccess) &&
                    (!opt->check_bounds || hipMalloc(&I.backup, bytes) == hipSuccess);
    // Phase-Field work arrays: k, b, Q, r, p, s, w, diag ([N][cells] each)
    // and the face gradients ([d][N][cells])
    const bool okpf = !opt->phase_field ||
        hipMalloc(&I.pf, sizeof(double) * (size_t)(kPfFields + I.D) * I.N * (size_t)I.nc) == hipSuccess;
    if (opt->phase_field) I.pfs = c->pfs + (size_t)i * kPfsLen;
    c->inst.push_back(I);
    if (!ok || !okpf) {
      mp_weno_destroy(c);
      return MP_ERR_OOM;
    }
  }

  // group by (N, d); larger instances first inside a group
  size_t part_total = 0;
  for (int D = 1; D <= 3; ++D)
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
      for (auto& v : G.xs) v.push_back(0);
      for (auto& v : G.ys) v.push_back(0);
      for (auto& v : G.zs) v.push_back(0);
      G.rs.push_back(0);
      if (opt->phase_field) {
        // multigrid levels: halve (rounding up) until one cell; every
        // instance of the group gets the group's largest count (extra
        // one-cell levels do nothing)
        for (int id : G.ids) {
          const Inst& I = c->inst[id];
          int nx = I.in.n[0], ny = I.D > 1 ? I.in.n[1] : 1, nz = I.D > 2 ? I.in.n[2] : 1, L = 1;
          while ((nx > 1 || ny > 1 || nz > 1) && L < kMgMaxLev) {
            nx = (nx + 1) / 2; ny = (ny + 1) / 2; nz = (nz + 1) / 2; ++L;
          }
          G.nlev = std::max(G.nlev, L);
        }
        for (int id : G.ids) {
          Inst& I = c->inst[id];
          int nx = I.in.n[0], ny = I.D > 1 ? I.in.n[1] : 1, nz = I.D > 2 ? I.in.n[2] : 1;
          size_t tot = 0;
          std::vector<std::array<int, 3>> dims;
          for (int l = 0; l < G.nlev; ++l) {
            dims.push_back({nx, ny, nz});
            tot += (size_t)nx * ny * nz * (I.D > 2 ? 7 : 6);
            nx = (nx + 1) / 2;
            ny = (ny + 1) / 2;
            nz = (nz + 1) / 2;
          }
          tot *= (size_t)I.N;
          if (hipMalloc(&I.mgbuf, sizeof(float) * tot) != hipSuccess ||
              hipMemset(I.mgbuf, 0, sizeof(float) * tot) != hipSuccess ||
              hipMalloc(&I.d_mg, sizeof(MgLevel) * G.nlev) != hipSuccess) {
            mp_weno_destroy(c);
            return MP_ERR_OOM;
          }
          float* q = I.mgbuf;
          for (int l = 0; l < G.nlev; ++l) {
            MgLevel L;
            L.nx = dims[l][0];
            L.ny = dims[l][1];
            L.nz = dims[l][2];
            L.nc = (int64_t)L.nx * L.ny * L.nz;
            const size_t f = (size_t)I.N * (size_t)L.nc;
            L.wx = q; q += f;
            L.wy = q; q += f;
            L.wz = nullptr;
            if (I.D > 2) { L.wz = q; q += f; }
            L.t = q; q += f;
            L.e = q; q += f;
            L.f = q; q += f;
            L.dg = q; q += f;
            I.lv.push_back(L);
          }
          if (hipMemcpy(I.d_mg, I.lv.data(), sizeof(MgLevel) * G.nlev,
                        hipMemcpyHostToDevice) != hipSuccess) {
            mp_weno_destroy(c);
            return MP_ERR_HIP;
          }
        }
      }
      for (int id : G.ids) {
        const Inst& I = c->inst[id];
        const mp_weno_instance& s = I.in;
        Desc d;
        desc_grid_eos(s, *opt, d);
        const Grid& g = d.g;
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
        if (opt->phase_field) {
          const size_t f = (size_t)I.N * (size_t)I.nc;
          d.pfin = s.U;
          d.pfs = I.pfs;
          d.pf_k = I.pf;
          d.pf_b = I.pf + f;
          d.pf_q = I.pf + 2 * f;
          d.pf_r = I.pf + 3 * f;
          d.pf_p = I.pf + 4 * f;
          d.pf_ap = I.pf + 5 * f;
          d.pf_w = I.pf + 6 * f;
          d.pf_u = I.pf + 7 * f;
          d.pf_qp = I.pf + 8 * f;
          d.pf_qpp = I.pf + 9 * f;
          d.pf_g = I.pf + kPfFields * f;   // after the kPfFields arrays above
          d.mg = I.d_mg;
          d.nlev = (int)I.lv.size();
          double h = s.dx[0];
          for (int k = 1; k < I.D; ++k) h = std::min(h, s.dx[k]);
          d.eta = opt->eta_over_dx * h;
        }
        d.chunk = (int64_t)kRedBlock *
                  std::max<int64_t>(1, (I.nc + (int64_t)kRedBlock * kMaxChunks - 1) /
                                           ((int64_t)kRedBlock * kMaxChunks));
        G.hdesc.push_back(d);
        int64_t top = G.rs.back() + (I.nc + d.chunk - 1) / d.chunk;
        G.rs.push_back((int)std::min<int64_t>(top, INT32_MAX));
        for (int v = 0; v < kXVar; ++v) {
          const int64_t nx = G.xs[v].back() + x_strips(g, kXS[v]);
          top = std::max(top, nx);
          G.xs[v].push_back((int)std::min<int64_t>(nx, INT32_MAX));
        }
        for (int v = 0; v < kYVar; ++v) {
          // y tiles per z plane, z tiles per y plane (the same shapes)
          const int oy = kYY[v] - 2;
          const int64_t ntx = (g.nx + kYX[v] - 1) / kYX[v];
          const int64_t nty = I.D > 1 ? ntx * ((g.ny + oy - 1) / oy) * g.nz : 0;
          const int64_t ntz = I.D > 2 ? ntx * ((g.nz + oy - 1) / oy) * g.ny : 0;
          const int64_t ny = G.ys[v].back() + nty, nz = G.zs[v].back() + ntz;
          top = std::max(top, std::max(ny, nz));
          G.ys[v].push_back((int)std::min<int64_t>(ny, INT32_MAX));
          G.zs[v].push_back((int)std::min<int64_t>(nz, INT32_MAX));
        }
        if (top >= (int64_t)INT32_MAX) {
          mp_weno_destroy(c);
          return MP_ERR_UNSUPPORTED;     // more tiles than one launch can index
        }
      }
      G.part_off = part_total;
      part_total += (size_t)G.rs.back();
      const size_t m = G.ids.size();
      std::vector<int2> lm[kMgMaxLev];
      for (int l = 0; l < G.nlev; ++l) {
        for (size_t k = 0; k < m; ++k) {
          const int64_t ncl = c->inst[G.ids[k]].lv[l].nc;
          for (int64_t ch = 0; ch * kRedBlock < ncl; ++ch) lm[l].push_back(make_int2((int)k, (int)ch));
        }
        G.lcount[l] = (int)lm[l].size();
      }
      // the fused cycle takes the coarsest levels whose LDS image (6 N floats
      // per cell, 7 N in 3D) fits the workgroup's LDS in every instance of
      // the group:
      // the device's limit when the kernel accepts it, else 64 KiB
      if (G.nlev > 0) {
        // (less kMgFusedStatic for the kernel's own LDS)
        size_t lds_budget = 65536 - kMgFusedStatic;
        int dev = 0, lmax = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lmax, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            lmax > 65536) {
          if (table().mg_lds[G.N][G.D](lmax - kMgFusedStatic) == hipSuccess)
            lds_budget = (size_t)(lmax - kMgFusedStatic);
          else
            (void)hipGetLastError();     // keep 64 KiB; clear the error
        }
        auto lds_from = [&](int l) {
          size_t mx = 0;
          for (size_t k = 0; k < m; ++k) {
            size_t b = 0;
            for (int j = l; j < G.nlev; ++j)
              b += (G.D > 2 ? 7 : 6) * sizeof(float) * (size_t)G.N *
                   (size_t)c->inst[G.ids[k]].lv[j].nc;
            mx = std::max(mx, b);
          }
          return mx;
        };
        G.mg_fuse = G.nlev - 1;
        while (G.mg_fuse > 0 && lds_from(G.mg_fuse - 1) <= lds_budget) --G.mg_fuse;
        G.mg_lds = lds_from(G.mg_fuse);
      }
      auto tile_map = [m](const std::vector<int>& st) {
        std::vector<int2> v((size_t)st[m]);
        for (size_t k = 0; k < m; ++k)
          for (int j = st[k]; j < st[k + 1]; ++j) v[(size_t)j] = make_int2((int)k, j - st[k]);
        return v;
      };
      const std::vector<int2> rm = tile_map(G.rs);
      std::vector<int2> xm[kXVar], ym[kYVar], zm[kYVar];
      bool ok = hipMalloc(&G.desc, sizeof(Desc) * m) == hipSuccess &&
                hipMalloc(&G.rmap, sizeof(int2) * std::max<size_t>(rm.size(), 1)) == hipSuccess &&
                hipMalloc(&G.rstart, sizeof(int) * (m + 1)) == hipSuccess;
      size_t most = 1;
      for (int v = 0; v < kXVar; ++v) {
        xm[v] = tile_map(G.xs[v]);
        most = std::max(most, (size_t)G.xs[v].back());
        ok = ok && hipMalloc(&G.xmap[v], sizeof(int2) * std::max<size_t>(xm[v].size(), 1)) == hipSuccess &&
             hipMalloc(&G.xstart[v], sizeof(int) * (m + 1)) == hipSuccess;
      }
      ok = ok && hipMalloc(&G.cflp, sizeof(double) * most) == hipSuccess;
      for (int v = 0; v < kYVar; ++v) {
        ym[v] = tile_map(G.ys[v]);
        ok = ok && hipMalloc(&G.ymap[v], sizeof(int2) * std::max<size_t>(ym[v].size(), 1)) == hipSuccess;
        zm[v] = tile_map(G.zs[v]);
        ok = ok && hipMalloc(&G.zmap[v], sizeof(int2) * std::max<size_t>(zm[v].size(), 1)) == hipSuccess;
      }
      if (!cmp && N <= kMaxNT) {
        G.xv = xsh ? std::min(std::max(env_entry(xsh, ngroup), 0), kXVar - 1) : 0;
        G.yv = ysh ? std::min(std::max(env_entry(ysh, ngroup), 0), kYVar - 1) : 0;
      }
      if (sw) G.swz = env_entry(sw, ngroup) ? 1 : 0;
      ++ngroup;
      c->groups.push_back(G);
      if (!ok) {
        mp_weno_destroy(c);
        return MP_ERR_OOM;
      }
      Group& H = c->groups.back();
      bool okc = hipMemcpy(H.desc, H.hdesc.data(), sizeof(Desc) * m, hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(H.rmap, rm.data(), sizeof(int2) * rm.size(), hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(H.rstart, H.rs.data(), sizeof(int) * (m + 1), hipMemcpyHostToDevice) == hipSuccess;
      for (int v = 0; v < kXVar; ++v)
        okc = okc && (xm[v].empty() ||
                      hipMemcpy(H.xmap[v], xm[v].data(), sizeof(int2) * xm[v].size(),
                                hipMemcpyHostToDevice) == hipSuccess) &&
              hipMemcpy(H.xstart[v], H.xs[v].data(), sizeof(int) * (m + 1),
                        hipMemcpyHostToDevice) == hipSuccess;
      for (int v = 0; v < kYVar; ++v)
        okc = okc && (ym[v].empty() ||
                      hipMemcpy(H.ymap[v], ym[v].data(), sizeof(int2) * ym[v].size(),
                                hipMemcpyHostToDevice) == hipSuccess) &&
              (zm[v].empty() ||
               hipMemcpy(H.zmap[v], zm[v].data(), sizeof(int2) * zm[v].size(),
                         hipMemcpyHostToDevice) == hipSuccess);
      for (int l = 0; l < H.nlev; ++l)
        okc = okc && hipMalloc(&H.lmap[l], sizeof(int2) * lm[l].size()) == hipSuccess &&
              hipMemcpy(H.lmap[l], lm[l].data(), sizeof(int2) * lm[l].size(),
                        hipMemcpyHostToDevice) == hipSuccess;
      if (!okc) {
        mp_weno_destroy(c);
        return MP_ERR_HIP;
      }
    }
  if (hipMalloc(&c->part, sizeof(double) * std::max<size_t>(part_total, 1) * kPartSlots) != hipSuccess) {
    mp_weno_destroy(c);
    return MP_ERR_OOM;
  }
  // the partials' slot stride is known once every group is built
  for (Group& G : c->groups) {
    for (Desc& d : G.hdesc) d.ps = (int64_t)part_total;
    if (hipMemcpy(G.desc, G.hdesc.data(), sizeof(Desc) * G.hdesc.size(),
                  hipMemcpyHostToDevice) != hipSuccess) {
      mp_weno_destroy(c);
      return MP_ERR_HIP;
    }
  }
  std::vector<double> zeros(n, 0.0);
  if (hipMemcpy(c->t, zeros.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->steps, zeros.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->dt, zeros.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess) {
    mp_weno_destroy(c);
    return MP_ERR_HIP;
  }
  if (opt->phase_field) {
    // Q starts at 0 (the first solve warm-starts from it); scalars cleared
    bool okz = hipMemset(c->pfs, 0, sizeof(double) * n * kPfsLen) == hipSuccess;
    for (const Inst& I : c->inst)
      okz = okz && hipMemset(I.pf, 0, sizeof(double) * (size_t)(kPfFields + I.D) * I.N * (size_t)I.nc) == hipSuccess;
    if (!okz || hipDeviceSynchronize() != hipSuccess) {
      mp_weno_destroy(c);
      return MP_ERR_HIP;
    }
  }
  if (hipDeviceSynchronize() != hipSuccess) {   // set-up copies and clears done
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

// Device address of `scratch` per device, taken once per device (with that
// device current) by the first allocation-free call on it.
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

static hipError_t noalloc_scratch(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

size_t mp_weno_rhs_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

mp_status mp_weno_rhs_noalloc(const mp_weno_instance* inst, const mp_weno_opts* opt,
                              const double* U_in, double* dUdt, void* hip_stream) {
  if (!inst || !opt || !dUdt) return MP_ERR_ARG;
  mp_weno_opts o = *opt;
  o.use_graph = 0;              // nothing is captured here; the caller may capture
  o.phase_field = 0;            // L(U) of Eq. (3) only
  const mp_status v = validate(1, inst, &o, hip_stream);
  if (v != MP_OK) return v;
  Desc d;
  desc_grid_eos(*inst, o, d);
  const int N = inst->nphase, D = inst->ndim;
  const size_t nU = (size_t)(2 * N + D + 1);
  const size_t need = kNoallocDescBytes + (D > 1 ? nU * (size_t)d.g.nc * sizeof(double) : 0);
  if (need > kNoallocScratchBytes) return MP_ERR_UNSUPPORTED;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return MP_ERR_HIP;
  void* base = nullptr;
  if (noalloc_scratch(dev, &base) != hipSuccess) return MP_ERR_HIP;
  Desc* ddesc = static_cast<Desc*>(base);
  d.U = inst->U;
  d.rin = U_in ? U_in : inst->U;
  d.rout = dUdt;
  d.acc = D > 1 ? reinterpret_cast<double*>(static_cast<char*>(base) + kNoallocDescBytes)
                : nullptr;
  d.vol = 1.0;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, st, d, ddesc);
  table().rhs1[o.recon >= MP_RECON_WENO_JS][N][D][o.precision](ddesc, d.g, st);
  return hipGetLastError() == hipSuccess ? MP_OK : MP_ERR_HIP;
}

mp_status mp_weno_amr_link(mp_weno_ctx* c, int32_t n_links, const mp_weno_link* links) {
  if (!c || n_links < 0 || (n_links > 0 && !links)) return MP_ERR_ARG;
  if (c->opt.phase_field && n_links > 0)
    return fail(c, MP_ERR_UNSUPPORTED, "coupled levels with the Phase-Field step");
  const int n = (int)c->inst.size();
  std::vector<AmrLink> L((size_t)n_links);
  std::vector<int2> items, faces;
  std::vector<int> ids;
  std::vector<char> used((size_t)n, 0), is_fine((size_t)n, 0);
  int N0 = 0, D0 = 0, maxcells = 0;
  size_t buf = 0;
  std::vector<size_t> off((size_t)n_links);
  for (int k = 0; k < n_links; ++k) {
    const mp_weno_link& a = links[k];
    if (a.fine < 0 || a.fine >= n || a.coarse < 0 || a.coarse >= n || a.fine == a.coarse)
      return fail(c, MP_ERR_ARG, "link instance index out of range");
    const Inst& F = c->inst[a.fine];
    const Inst& C = c->inst[a.coarse];
    const int D = C.D, N = C.N;
    if (F.D != D || F.N != N || D > 2)
      return fail(c, D > 2 ? MP_ERR_UNSUPPORTED : MP_ERR_ARG,
                  "linked instances need the same N and d (1 or 2)");
    if (k == 0) { N0 = N; D0 = D; }
    if (N != N0 || D != D0) return fail(c, MP_ERR_UNSUPPORTED, "links of several (N, d)");
    const int W = (F.in.n[0] - 2 * kAmrHalo) / 2, H = D > 1 ? (F.in.n[1] - 2 * kAmrHalo) / 2 : 1;
    const int lx = a.lo[0], ly = D > 1 ? a.lo[1] : 0;
    bool ok = W >= 1 && 2 * W + 2 * kAmrHalo == F.in.n[0] &&
              (D == 1 || (H >= 1 && 2 * H + 2 * kAmrHalo == F.in.n[1]));
    // the block and the coarse stencils around it stay inside the coarse grid
    ok = ok && lx >= kAmrHalo && lx + W + kAmrHalo <= C.in.n[0];
    ok = ok && (D == 1 || (ly >= kAmrHalo && ly + H + kAmrHalo <= C.in.n[1]));
    for (int d = 0; d < D && ok; ++d)
      ok = std::fabs(F.in.dx[d] * 2.0 - C.in.dx[d]) <= 1e-12 * C.in.dx[d];
    if (!ok) return fail(c, MP_ERR_ARG, "link geometry (halo 3, ratio 2, block inside the coarse grid)");
    if (is_fine[a.fine]) return fail(c, MP_ERR_ARG, "an instance refines two blocks");
    is_fine[a.fine] = 1;
    // blocks of one coarse instance: their coarse stencil regions must not meet
    for (int j = 0; j < k; ++j) {
      if (links[j].coarse != a.coarse) continue;
      const AmrLink& B = L[j];
      const int g = 2 * kAmrHalo;
      const bool apart = lx >= B.lox + B.W + g || B.lox >= lx + W + g ||
                         (D > 1 && (ly >= B.loy + B.H + g || B.loy >= ly + H + g));
      if (!apart) return fail(c, MP_ERR_ARG, "blocks of one coarse instance too close");
    }
    AmrLink& l = L[k];
    std::memset(&l, 0, sizeof(l));
    l.fst[0] = F.in.U; l.fst[1] = F.U1; l.fst[2] = F.U2;
    l.cst[0] = C.in.U; l.cst[1] = C.U1; l.cst[2] = C.U2;
    Desc df, dc;
    desc_grid_eos(F.in, c->opt, df);
    desc_grid_eos(C.in, c->opt, dc);
    l.fg = df.g; l.cg = dc.g; l.e = dc.e;
    l.lox = lx; l.loy = ly; l.W = W; l.H = H;
    l.nface = D > 1 ? 2 * H + 2 * W : 2;
    l.dt = c->dt + a.coarse;
    const int nU = 2 * N + D + 1;
    off[(size_t)k] = buf;
    buf += (size_t)l.nface * (3 * (nU + 1) + nU);
    for (int f = 0; f < l.nface; ++f) {
      faces.push_back(make_int2(k, f));
      for (int q = 0; q < 3; ++q) items.push_back(make_int2(k, 3 * f + q));
    }
    for (int id : {a.fine, a.coarse})
      if (!used[id]) { used[id] = 1; ids.push_back(id); }
    maxcells = std::max<int>(maxcells, (int)F.nc);
  }
  // drop the previous coupling and any captured step (it holds the old one)
  (void)hipFree(c->amr); (void)hipFree(c->amr_items); (void)hipFree(c->amr_faces);
  (void)hipFree(c->amr_ids); (void)hipFree(c->amr_buf);
  c->amr = nullptr; c->amr_items = nullptr; c->amr_faces = nullptr; c->amr_ids = nullptr;
  c->amr_buf = nullptr;
  c->amr_nlinks = 0;
  for (auto& g : c->graph)
    if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
  if (c->chain) { (void)hipGraphExecDestroy(c->chain); c->chain = nullptr; }
  if (n_links == 0) return MP_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (hipMalloc(&c->amr, sizeof(AmrLink) * L.size()) != hipSuccess ||
      hipMalloc(&c->amr_items, sizeof(int2) * items.size()) != hipSuccess ||
      hipMalloc(&c->amr_faces, sizeof(int2) * faces.size()) != hipSuccess ||
      hipMalloc(&c->amr_ids, sizeof(int) * ids.size()) != hipSuccess ||
      hipMalloc(&c->amr_buf, sizeof(double) * buf) != hipSuccess)
    return fail(c, MP_ERR_OOM, "coupling buffers");
  for (int k = 0; k < n_links; ++k) {
    const int nU = 2 * N0 + D0 + 1;
    L[(size_t)k].flx = c->amr_buf + off[(size_t)k];
    L[(size_t)k].reg = L[(size_t)k].flx + (size_t)L[(size_t)k].nface * 3 * (nU + 1);
  }
  HIPCHK(c, hipMemcpy(c->amr, L.data(), sizeof(AmrLink) * L.size(), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->amr_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->amr_faces, faces.data(), sizeof(int2) * faces.size(), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->amr_ids, ids.data(), sizeof(int) * ids.size(), hipMemcpyHostToDevice));
  c->amr_nlinks = n_links;
  c->amr_nitems = (int)items.size();
  c->amr_nfaces = (int)faces.size();
  c->amr_nids = (int)ids.size();
  c->amr_N = N0;
  c->amr_D = D0;
  c->amr_maxcells = maxcells;
  return MP_OK;
}

mp_status mp_weno_pf_fields(mp_weno_ctx* c, const double* const* U_in, double* const* divj,
                            double* const* grad, double* const* dUdt) {
  if (!c) return MP_ERR_ARG;
  if (!c->opt.phase_field) return fail(c, MP_ERR_UNSUPPORTED, "phase_field is off");
  if (dUdt)
    for (size_t i = 0; i < c->inst.size(); ++i)
      if (!dUdt[i]) return fail(c, MP_ERR_ARG, "null output pointer");
  // the descriptor tables carry the input/output pointers of this call
  auto set_inputs = [c, U_in, dUdt](bool call) -> mp_status {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (Group& G : c->groups) {
      for (size_t k = 0; k < G.ids.size(); ++k) {
        const int id = G.ids[k];
        const double* u = (call && U_in && U_in[id]) ? U_in[id] : c->inst[id].in.U;
        G.hdesc[k].pfin = u;
        if (call) {
          G.hdesc[k].rin = u;
          G.hdesc[k].rout = dUdt ? dUdt[id] : nullptr;
        }
      }
      HIPCHK(c, hipMemcpy(G.desc, G.hdesc.data(), sizeof(Desc) * G.ids.size(),
                          hipMemcpyHostToDevice));
    }
    return MP_OK;
  };
  mp_status st = set_inputs(true);
  if (st != MP_OK) return st;
  st = run_pf_solve(c, 1, 0);
  if (st == MP_OK) {
    for (size_t i = 0; i < c->inst.size(); ++i) {
      const Inst& I = c->inst[i];
      const size_t f = (size_t)I.N * (size_t)I.nc;
      if (divj && divj[i])
        HIPCHK(c, hipMemcpyAsync(divj[i], I.pf + f, sizeof(double) * f,
                                 hipMemcpyDeviceToDevice, c->stream));
      if (grad && grad[i])
        HIPCHK(c, hipMemcpyAsync(grad[i], I.pf + kPfFields * f, sizeof(double) * I.D * f,
                                 hipMemcpyDeviceToDevice, c->stream));
    }
    if (dUdt) st = enqueue_stage(c, 3, 1);
  }
  const mp_status st2 = set_inputs(false);
  return st != MP_OK ? st : st2;
}

mp_status mp_weno_autotune(mp_weno_ctx* c, int32_t reps, int32_t* choice) {
  if (!c || reps < 0) return fail(c, MP_ERR_ARG, "bad argument");
  if (reps == 0) reps = 8;
  const Table& T = table();
  const int prec = c->opt.precision;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // time L(U) of the current states into the stage buffer U1 (the states
  // and the step state are untouched)
  for (Group& G : c->groups) {
    for (size_t k = 0; k < G.ids.size(); ++k) {
      G.hdesc[k].rin = c->inst[G.ids[k]].in.U;
      G.hdesc[k].rout = c->inst[G.ids[k]].U1;
    }
    HIPCHK(c, hipMemcpy(G.desc, G.hdesc.data(), sizeof(Desc) * G.ids.size(),
                        hipMemcpyHostToDevice));
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(c, MP_ERR_HIP, "hipEventCreate failed");
  }
  mp_status st = MP_OK;
  // the comparison schemes are built with the default shapes only: for them
  // only the tile order is chosen
  const int cmp = c->opt.recon >= MP_RECON_WENO_JS;
  const int v = cmp ? kRiemannCmp : kRiemann;
  for (Group& G : c->groups) {
    // every candidate timed in two interleaved rounds, the faster one kept:
    // a single round is at the mercy of clock and neighbour noise (groups of
    // more than kMaxNT phases are built with the default shapes only)
    const bool fixed = cmp || G.N > kMaxNT;
    const int nxv = fixed ? 1 : kXVar;
    const int nyv = G.D >= 2 && !fixed ? kYVar : 1;
    float tmin[kXVar][kYVar][2];
    for (auto& a : tmin)
      for (auto& b : a) b[0] = b[1] = INFINITY;
    for (int round = 0; round < 2 && st == MP_OK; ++round)
      for (int xv = 0; xv < nxv && st == MP_OK; ++xv)
        for (int yv = 0; yv < nyv && st == MP_OK; ++yv)
          for (int sw = 0; sw < 2 && st == MP_OK; ++sw) {
            auto run = [&]() {
              T.sx[v][G.N][G.D][prec][xv](G, 3, sw, c->stream);
              if (G.D == 2) T.sy[v][G.N][prec][yv](G, 3, sw, c->stream);
              if (G.D == 3) {
                T.sy3[v][G.N][prec][yv](G, 3, sw, c->stream);
                T.sz3[v][G.N][prec][yv](G, 3, sw, c->stream);
              }
            };
            run();   // warm-up
            float ms = 0.0f;
            if (hipEventRecord(e0, c->stream) != hipSuccess) { st = MP_ERR_HIP; break; }
            for (int r = 0; r < reps; ++r) run();
            if (hipEventRecord(e1, c->stream) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess) {
              st = MP_ERR_HIP;
              break;
            }
            tmin[xv][yv][sw] = std::min(tmin[xv][yv][sw], ms);
          }
    // a later candidate must be faster by more than 1 %: near-ties keep the
    // earlier one, so that repeated set-ups choose alike
    float best = INFINITY;
    int bx = 0, by = 0, bs = 0;
    for (int xv = 0; xv < nxv; ++xv)
      for (int yv = 0; yv < nyv; ++yv)
        for (int sw = 0; sw < 2; ++sw)
          if (tmin[xv][yv][sw] < 0.99f * best) {
            best = tmin[xv][yv][sw];
            bx = xv;
            by = yv;
            bs = sw;
          }
    G.xv = bx;
    G.yv = by;
    G.swz = bs;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != MP_OK) return fail(c, st, "autotune launch failed");
  // a captured step holds the old launch shapes
  for (auto& g : c->graph)
    if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
  if (c->chain) { (void)hipGraphExecDestroy(c->chain); c->chain = nullptr; }
  if (choice)
    for (const Group& G : c->groups)
      for (int id : G.ids) {
        choice[4 * id + 0] = kXS[G.xv];
        choice[4 * id + 1] = G.D >= 2 ? kYX[G.yv] : 0;
        choice[4 * id + 2] = G.D >= 2 ? kYY[G.yv] : 0;
        choice[4 * id + 3] = G.swz;
      }
  return MP_OK;
}

mp_status mp_weno_dt(mp_weno_ctx* c, double* dt, int32_t where) {
  if (!c || !dt) return fail(c, MP_ERR_ARG, "null argument");
  mp_status s = enqueue_dt(c, 0);
  if (s != MP_OK) return s;
  if (c->amr_nlinks)      // linked instances share the smallest step
    hipLaunchKernelGGL(k_amr_dt, dim3(1), dim3(64), 0, c->stream, c->amr_ids, c->amr_nids, c->dt);
  const size_t bytes = sizeof(double) * c->inst.size();
  if (where == MP_WHERE_HOST) {
    HIPCHK(c, hipMemcpyAsync(dt, c->dt, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    HIPCHK(c, hipMemcpyAsync(dt, c->dt, bytes, hipMemcpyDeviceToDevice, c->stream));
  }
  return MP_OK;
}

// One step.  With the device CFL step and no Phase-Field step the CFL kernel
// moves the time on (nothing later in the step reads it); otherwise it moves
// at the end, so a failed Phase-Field solve leaves it untouched.
static mp_status enqueue_step(mp_weno_ctx* c, bool external_dt) {
  const bool early = !external_dt && !c->opt.phase_field && !c->amr_nlinks;
  c->cfl_pending = false;          // (a step that failed may have left it set)
  if (!external_dt) {
    // without coupled instances, 2D and 3D groups take the step from their
    // first x sweep (no pass of its own over U^n); 1D groups, whose x sweep
    // finishes the stage, and coupled instances (which share the smallest
    // step) take it here
    const bool fuse = !c->amr_nlinks;
    mp_status s = enqueue_dt(c, early ? 1 : 0, fuse);
    if (s != MP_OK) return s;
    c->cfl_pending = fuse;
    c->cfl_advance = early ? 1 : 0;
    if (c->amr_nlinks)
      hipLaunchKernelGGL(k_amr_dt, dim3(1), dim3(64), 0, c->stream, c->amr_ids, c->amr_nids,
                         c->dt);
  }
  return enqueue_rk(c, !early);
}

mp_status mp_weno_advance(mp_weno_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return fail(c, MP_ERR_ARG, "bad argument");
  // steps that need the host between them go one by one
  if (!c->opt.use_graph || c->profile || c->opt.phase_field || c->opt.check_bounds) {
    for (int32_t k = 0; k < nsteps; ++k) {
      const mp_status s = mp_weno_step(c, nullptr);
      if (s != MP_OK) return s;
    }
    return MP_OK;
  }
  int32_t left = nsteps;
  if (left >= mp_weno_ctx::kChain || nsteps == 0) {
    if (!c->chain) {
      hipGraph_t gph;
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      mp_status s = MP_OK;
      for (int k = 0; k < mp_weno_ctx::kChain && s == MP_OK; ++k) s = enqueue_step(c, false);
      hipError_t e2 = hipStreamEndCapture(c->stream, &gph);
      if (s != MP_OK) return s;
      if (e2 != hipSuccess) return fail(c, MP_ERR_HIP, hipGetErrorString(e2));
      HIPCHK(c, hipGraphInstantiate(&c->chain, gph, nullptr, nullptr, 0));
      (void)hipGraphDestroy(gph);
    }
    for (; left >= mp_weno_ctx::kChain; left -= mp_weno_ctx::kChain)
      HIPCHK(c, hipGraphLaunch(c->chain, c->stream));
  }
  for (; left > 0; --left) {
    const mp_status s = mp_weno_step(c, nullptr);
    if (s != MP_OK) return s;
  }
  return MP_OK;
}

mp_status mp_weno_step(mp_weno_ctx* c, const double* dt_dev) {
  if (!c) return MP_ERR_ARG;
  const size_t n = c->inst.size();
  if (c->opt.check_bounds) {
    for (auto& I : c->inst)
      HIPCHK(c, hipMemcpyAsync(I.backup, I.in.U, sizeof(double) * I.nU * I.nc,
                               hipMemcpyDeviceToDevice, c->stream));
  }
  // with check_bounds: the time and step count before the step, read back
  // now (the call synchronises anyway), so no copy into this host buffer is
  // in flight when an error returns early
  std::vector<double> t_before;
  if (c->opt.check_bounds) {
    t_before.resize(2 * n);
    HIPCHK(c, hipMemcpyAsync(t_before.data(), c->t, sizeof(double) * n,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(t_before.data() + n, c->steps, sizeof(double) * n,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  // back to the state, time and step count before the step (check_bounds)
  auto restore = [&]() -> mp_status {
    c->pf_hist = 0;                // Q belongs to the step taken back
    for (auto& I : c->inst)
      HIPCHK(c, hipMemcpyAsync(I.in.U, I.backup, sizeof(double) * I.nU * I.nc,
                               hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->t, t_before.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->steps, t_before.data() + n, sizeof(double) * n,
                        hipMemcpyHostToDevice));
    return MP_OK;
  };
  const bool ext = dt_dev != nullptr;
  if (ext)
    HIPCHK(c, hipMemcpyAsync(c->dt, dt_dev, sizeof(double) * n, hipMemcpyDeviceToDevice,
                             c->stream));
  if (c->opt.use_graph && !c->profile && !c->opt.phase_field) {
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
    if (s != MP_OK) {
      if (c->opt.check_bounds) {
        const mp_status r = restore();
        if (r != MP_OK) return r;
      }
      return s;
    }
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
      const mp_status r = restore();
      if (r != MP_OK) return r;
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
