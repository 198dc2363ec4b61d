// csph_kernels.hip -- HIP kernels of one CSPH-TVD step for gfx950.
//
// This translation unit is compiled twice, with CSPH_REAL = float and with
// CSPH_REAL = double.  The double build is compiled without floating-point
// contraction and evaluates every expression of the scheme (arXiv:1912.04855,
// Sec. 2.2) in one fixed order, so two runs, and any tiling, give the same bits.
// The float build keeps the state and most arithmetic in FP32 (fast reciprocal
// and square root) and promotes to FP64 where cancellation matters: the
// pressure + potential pair differences that carry the well-balanced property,
// the time step and the conservation totals.
//
// Per step:
//   begin  : dt from the max signal speed of U^n (FP64), CFL and viscous limits,
//            in the same launch as the ghost cells of U^n
//   stage P: predictor, Eq. (5) with Q of Eq. (7) on the lattice; the predicted
//            particle's phi* over its predicted volume, psi at r*
//   fill   : ghost cells of m*, phi*, xi* and of psi at r*
//   stage C: corrector, Eq. (6) with Q(U*, r*) of Eq. (7) in the particles'
//            reference configuration (lattice kernel gradients, the predicted
//            particles' phi* and psi at r*)
//   fill   : ghost cells of m~, E~, xi^{n+1}
//   stage E: reconstruction Eq. (8), face fluxes (swept width at the foot of the
//            face's trajectory), update Eq. (4); epilogue: signal-speed max of
//            U^{n+1}, FP64 block totals, error flags
//   end    : swap the state copies
//
// Stages P, C and E are 2.5D stencil sweeps: a workgroup owns a tile of an x-y
// plane (see Shape below) and marches along z through tz planes.  P and C are one sweep
// (stage_l_body) that keeps three planes of per-cell values (density, phi,
// velocity, potential) with a one-cell halo in LDS, so each cell's values are
// formed once per sweep instead of once per neighbour.  E keeps a register queue
// of its own column along z (U^n at k-1..k+2, the z-face flux carried to the next
// plane) and the current plane's x-y stencil (two-cell halo) in LDS.  Workgroup
// ids are remapped so that each of the 8 XCDs (separate L2s) gets a contiguous
// run of tiles, which keeps the halo reads of neighbouring tiles in one L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "csph_internal.h"

#ifndef CSPH_REAL
#error "CSPH_REAL must be float or double"
#endif

#if CSPH_IS_DOUBLE
#define CSPH_TAG k64
#else
#define CSPH_TAG k32
#endif

namespace csph {
namespace CSPH_TAG {

using Real = CSPH_REAL;
using Acc = double;
constexpr bool kF64 = std::is_same<Real, double>::value;
// The FP32 build pushes the x-face ghost cells from the stage that writes a
// field; the FP64 build fills every ghost zone in the fill kernels.
constexpr bool kPushX = !kF64;
// The FP64 build stores the predicted offset xi* = (dt/2)(u^n + u*); the FP32
// build recomputes it from rho, m^n and m* wherever it is needed, which saves
// stage P three of its eight output fields.
constexpr bool kKeepXiStar = kF64;
// Likewise for the final offset xi^{n+1}: the FP32 build forms it in stage E
// from rho, m^n, m* and m~, which saves stage C three of its seven outputs.
constexpr bool kKeepXi = kF64;

constexpr int kWave = 64;
constexpr int kXcd = 8;

// tile shape of the stencil sweeps
constexpr int TX = 32, TY = 8, NT = TX * TY;
constexpr int HX = TX + 2, HY = TY + 2, HP = HX * HY;          // one-cell halo
constexpr int EX = TX + 4, EY = TY + 4, EP = EX * EY;          // two-cell halo
constexpr int NFX = (TX + 1) * TY, NFY = TX * (TY + 1);        // x and y faces of a tile
// stage E numbers its x faces at the pitch of its two-cell-halo rows (TX + 1 of
// every EX used), so that a wave's face reads are consecutive LDS words across
// a row boundary (no bank conflicts), and its y faces start on a half-wave
constexpr int NFXP = EX * TY;

// Tile shapes of the Lagrangian sweeps: in FP32 a single grid's stages P and C
// take 64 x 4 tiles (longer rows in the loads); FP64 keeps 32 x 8 there (its
// planes of 64 x 4 tiles would hold 57 KB of LDS, two workgroups per CU), and
// the batched sweeps keep stage E's 32 x 8, which also fits members 32 cells wide.
template <int kTX>
struct Shape {
  static constexpr int TX = kTX, TY = NT / kTX;
  static constexpr int HX = TX + 2, HY = TY + 2, HP = HX * HY;
};
constexpr int kTxL = kF64 ? 32 : 64;  // single-grid stages P and C

// ------------------------------------------------------------------ indexing
__device__ __forceinline__ long long cell(const GridDev& g, int i, int j, int k) {
  return ((long long)(k + kGhost) * g.sy + (j + kGhost)) * (long long)g.sx + (i + kGhost);
}

// half neighbour set O13 in lexicographic (o_z, o_y, o_x) order; the partner of
// each offset o is -o, and every sum adds the pair's two terms first.
struct O13 {
  static constexpr int o[13][3] = {{1, 0, 0},  {-1, 1, 0}, {0, 1, 0},  {1, 1, 0},  {-1, -1, 1},
                                   {0, -1, 1}, {1, -1, 1}, {-1, 0, 1}, {0, 0, 1},  {1, 0, 1},
                                   {-1, 1, 1}, {0, 1, 1},  {1, 1, 1}};
};
constexpr int O13::o[13][3];

// Dispatch hands consecutive workgroups to the XCDs round-robin; invert that so
// XCD x owns the contiguous logical tiles [x*n/8, (x+1)*n/8).
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
  const int per = (nblocks + kXcd - 1) / kXcd;
  const int xcd = bid % kXcd, slot = bid / kXcd;
  const int t = xcd * per + slot;
  return t < nblocks ? t : -1;
}

struct Tile {
  int x0, y0, z0, z1;
};

template <int kTX = TX>
__device__ __forceinline__ int tiles_of(const GridDev& g, int tz) {
  constexpr int ty = NT / kTX;
  return ((g.nx + kTX - 1) / kTX) * ((g.ny + ty - 1) / ty) * ((g.nz + tz - 1) / tz);
}

// tile number -> tile origin; tiles are numbered x fastest, then y, then z
template <int kTX = TX>
__device__ __forceinline__ void tile_at(const GridDev& g, int tz, int id, Tile& t) {
  constexpr int ty = NT / kTX;
  const int nbx = (g.nx + kTX - 1) / kTX, nby = (g.ny + ty - 1) / ty;
  const int bx = id % nbx, r = id / nbx, by = r % nby, bz = r / nby;
  t.x0 = bx * kTX;
  t.y0 = by * ty;
  t.z0 = bz * tz;
  t.z1 = min(t.z0 + tz, g.nz);
}

// tile of this workgroup in a single-simulation launch (grid padded to 8k)
template <int kTX = TX>
__device__ __forceinline__ bool single_tile(const GridDev& g, int tz, Tile& t, int& id) {
  id = xcd_tile(blockIdx.x, gridDim.x);
  if (id < 0 || id >= tiles_of<kTX>(g, tz)) return false;
  tile_at<kTX>(g, tz, id, t);
  return true;
}

// ------------------------------------------------------------------ arithmetic
__device__ __forceinline__ Real rsqrt_(Real x) {
  if constexpr (kF64) {
    return (Real)1 / sqrt(x);  // not used by the FP64 build
  } else {
    return __builtin_amdgcn_rsqf(x);
  }
}

// square root: correctly rounded in FP64; the hardware approximation in FP32
__device__ __forceinline__ Real sqrt_fast(Real x) {
  if constexpr (kF64) {
    return sqrt(x);
  } else {
    return __builtin_amdgcn_sqrtf(x);
  }
}

// p = (gamma-1)(E - m.u/2), u = m/rho; vacuum (rho <= rho_vac): u = 0; p >= 0.
__device__ __forceinline__ void primitive(const GridDev& g, Real rho, Real mx, Real my, Real mz,
                                          Real E, Real& ux, Real& uy, Real& uz, Real& p) {
  if (rho > (Real)g.rho_vac) {
    if constexpr (kF64) {
      ux = mx / rho;
      uy = my / rho;
      uz = mz / rho;
    } else {
      const Real ir = __builtin_amdgcn_rcpf(rho);
      ux = mx * ir;
      uy = my * ir;
      uz = mz * ir;
    }
  } else {
    ux = (Real)0;
    uy = (Real)0;
    uz = (Real)0;
  }
  const Real ke = (Real)0.5 * (mx * ux + my * uy + mz * uz);
  const Real pp = (Real)g.gm1 * (E - ke);
  p = pp > (Real)0 ? pp : (Real)0;
}

// Sources and sinks (an extension, Sec. 4): half a step (hdt = dt/2) of the mass
// rate q in one cell.  q > 0 injects gas at rest with specific internal energy
// eps; q < 0 removes gas at the cell's specific values, limited at zero.
__device__ __forceinline__ void source_cell(Real q, Real eps, Real hdt, Real& r, Real& mx, Real& my,
                                            Real& mz, Real& E) {
  if (q == (Real)0) return;
  const Real d = hdt * q;
  if (q > (Real)0) {
    r = r + d;
    E = E + d * eps;
    return;
  }
  if (!(r > (Real)0)) return;
  Real rn = r + d;
  if (rn < (Real)0) rn = (Real)0;
  const Real f = rn / r;
  mx = mx * f;
  my = my * f;
  mz = mz * f;
  E = E * f;
  r = rn;
}

// velocity m / rho as primitive() forms it (0 in vacuum)
__device__ __forceinline__ void velocity(const GridDev& g, Real rho, Real mx, Real my, Real mz, Real u[3]) {
  Real p_unused;
  primitive(g, rho, mx, my, mz, (Real)0, u[0], u[1], u[2], p_unused);
}

// predicted particle offset xi* = (dt/2)(u^n + u*) of a cell, Eq. (5)
__device__ __forceinline__ void xi_star(const Real un[3], const Real us[3], Real hdt, Real xi[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) xi[d] = hdt * (un[d] + us[d]);
}

// One component of the final particle offset, Eq. (6),
// xi = xi*/2 + dt (u^n + u~)/4 with xi* = (dt/2)(u^n + u*), from a cell's rho and
// the component of m^n, m*, m~, in the operations and order that stage C uses
// (FP32 build: it is not stored there).  c = {dt/2, dt/4, h/2, 1/h}.
__device__ __forceinline__ Real xi_final(const GridDev& g, Real rho, Real mn, Real ms, Real mt,
                                         const Real c[4]) {
  Real un = (Real)0, us = (Real)0, ut = (Real)0;
  if (rho > (Real)g.rho_vac) {
    // the velocities exactly as primitive() forms them
    if constexpr (kF64) {
      un = mn / rho;
      us = ms / rho;
      ut = mt / rho;
    } else {
      const Real ir = __builtin_amdgcn_rcpf(rho);
      un = mn * ir;
      us = ms * ir;
      ut = mt * ir;
    }
  }
  const Real hdt = c[0], qdt = c[1], hx = c[2], ih = c[3];
  Real xc = hdt * (un + us);
  xc *= ih;
  return hx * xc + qdt * (un + ut);
}

__device__ __forceinline__ Real minmod(Real a, Real b) {
  if (a * b <= (Real)0) return (Real)0;
  const Real sg = a > (Real)0 ? (Real)1 : (Real)-1;
  return sg * fmin(fabs(a), fabs(b));
}

__device__ __forceinline__ Real lerp(Real a, Real b, Real t) { return a + t * (b - a); }

// trilinear psi at cell centre + (ox, oy, oz), between the cell and its
// neighbours on the side the particle moved to; P(a, b, c) reads psi at the
// cell offset (a, b, c)
template <typename At>
__device__ __forceinline__ Real psi_at(const GridDev& g, At P, Real ox, Real oy, Real oz) {
  const Real fx = ox * (Real)g.inv_h, fy = oy * (Real)g.inv_h, fz = oz * (Real)g.inv_h;
  const int di = fx >= (Real)0 ? 1 : -1;
  const int dj = fy >= (Real)0 ? 1 : -1;
  const int dk = fz >= (Real)0 ? 1 : -1;
  const Real tx = fabs(fx), ty = fabs(fy), tz = fabs(fz);
  const Real a00 = lerp(P(0, 0, 0), P(di, 0, 0), tx);
  const Real a10 = lerp(P(0, dj, 0), P(di, dj, 0), tx);
  const Real a01 = lerp(P(0, 0, dk), P(di, 0, dk), tx);
  const Real a11 = lerp(P(0, dj, dk), P(di, dj, dk), tx);
  const Real b0 = lerp(a00, a10, ty);
  const Real b1 = lerp(a01, a11, ty);
  return lerp(b0, b1, tz);
}

// Workgroup barrier that orders LDS only.  The stencil sweeps share data
// between threads through LDS alone (global inputs come from earlier launches,
// outputs are read by later ones), so their barriers need not wait for
// outstanding global loads or stores, which stay in flight across them.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A 64-bit byte offset kept as one value in a register pair: the compiler would
// otherwise split base + row + column + plane again for every field it is added to.
__device__ __forceinline__ long long opaque(long long v) {
  asm volatile("" : "+v"(v));
  return v;
}
template <typename T>
__device__ __forceinline__ T* at_bytes(T* base, long long bytes) {
  return (T*)((char*)base + bytes);
}

// Addresses within one z-plane: a scalar plane base (the field pointer plus the
// index of the plane's first padded cell) and a 32-bit byte offset in the plane.
// The offset is re-declared opaque in the block that loads or stores, so that
// the access is issued with the scalar base and the 32-bit vector offset and no
// 64-bit vector address arithmetic.  A padded plane holds fewer than 5e8 cells,
// so its byte offsets fit 32 bits in FP64 too.
__device__ __forceinline__ long long plane0(const GridDev& g, int k) {
  const long long v = (long long)(k + kGhost) * g.sy * g.sx;
  // uniform by construction; stated so that it stays in scalar registers
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ uint32_t in_plane(const GridDev& g, int i, int j) {
  return (uint32_t)((j + kGhost) * g.sx + (i + kGhost)) * (uint32_t)sizeof(Real);
}
__device__ __forceinline__ uint32_t opaque32(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}
template <typename T>
__device__ __forceinline__ T* at_plane(T* base, long long plane, uint32_t bytes) {
  return (T*)((char*)(base + plane) + (uint64_t)bytes);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ __forceinline__ Real signal_speed_r(const GridDev& g, Real r, Real mx, Real my, Real mz,
                                               Real E) {
  if (!(r > (Real)g.rho_vac)) return (Real)0;
  Real ux, uy, uz, p;
  primitive(g, r, mx, my, mz, E, ux, uy, uz, p);
  Real cs;
  if constexpr (kF64) {
    cs = sqrt((Real)g.gamma * p / r);
  } else {
    cs = sqrtf((Real)g.gamma * p * __builtin_amdgcn_rcpf(r));
  }
  return cs + fabs(ux) + fabs(uy) + fabs(uz);
}
__device__ __forceinline__ double signal_speed(const GridDev& g, Real r, Real mx, Real my, Real mz,
                                               Real E) {
  return (double)signal_speed_r(g, r, mx, my, mz, E);
}

// ==================================================================== ghost cells
__device__ __forceinline__ int map_index(int x, int n, int kind) {
  if (kind == kPeriodic) return x < 0 ? x + n : x - n;
  if (kind == kReflect) return x < 0 ? -x - 1 : 2 * n - 1 - x;
  return x < 0 ? 0 : n - 1;  // outflow (and psi at inflow faces)
}

// decode ghost cell number t into (i, j, k); false beyond the last ghost cell.
// Ghost cells are numbered in three zones: the 4 z-planes (full x-y extent),
// then the 4 y-rows of every interior z-plane (full x extent), then the 4
// x-cells of every interior row.  Counts fit in 32 bits for any grid the
// library accepts.
__device__ __forceinline__ bool ghost_cell(const GridDev& g, unsigned t, int& i, int& j, int& k) {
  const unsigned sx = (unsigned)g.sx, sxy = (unsigned)g.sx * (unsigned)g.sy;
  const unsigned zone_z = 4u * sxy;
  const unsigned zone_y = (unsigned)g.nz * 4u * sx;
  const unsigned zone_x = (unsigned)g.nz * (unsigned)g.ny * 4u;
  if (t < zone_z) {
    const unsigned kk = t / sxy, r = t - kk * sxy;
    const unsigned jj = r / sx;
    j = (int)jj - kGhost;
    i = (int)(r - jj * sx) - kGhost;
    k = kk < 2 ? (int)kk - 2 : g.nz + ((int)kk - 2);
  } else if (t < zone_z + zone_y) {
    const unsigned u = t - zone_z, row = 4u * sx;
    const unsigned kq = u / row, r = u - kq * row;
    const unsigned jj = r / sx;
    k = (int)kq;
    i = (int)(r - jj * sx) - kGhost;
    j = jj < 2 ? (int)jj - 2 : g.ny + ((int)jj - 2);
  } else if (t < zone_z + zone_y + zone_x) {
    const unsigned u = t - zone_z - zone_y, row = 4u * (unsigned)g.ny;
    const unsigned kq = u / row, r = u - kq * row;
    const unsigned jj = r >> 2, ii = r & 3u;
    k = (int)kq;
    j = (int)jj;
    i = ii < 2 ? (int)ii - 2 : g.nx + ((int)ii - 2);
  } else {
    return false;
  }
  return true;
}

// Where ghost cell (i, j, k) takes its values from.  The per-face rules are
// composed in x, y, z order, so the last axis (z) decides first: walking z, y,
// x, each out-of-range coordinate is mapped by its face's rule until an inflow
// face is met, whose Dirichlet state then gives the value (except for psi,
// which inflow faces copy like outflow).  flip holds the reflected axes met on
// the way: the normal momentum and particle offset of such an axis change sign.
struct GhostSrc {
  long long src;   // padded index of the source cell (when inflow < 0)
  int inflow;      // inflow face giving the value, or -1
  int flip;        // bit a: axis a reflected
};

__device__ __forceinline__ GhostSrc ghost_src(const GridDev& g, const BcDev& bc, int i, int j, int k,
                                              bool psi) {
  const int n[3] = {g.nx, g.ny, g.nz};
  int c[3] = {i, j, k};
  GhostSrc r{0, -1, 0};
  for (int ax = 2; ax >= 0; --ax) {
    if (c[ax] >= 0 && c[ax] < n[ax]) continue;
    const int face = 2 * ax + (c[ax] < 0 ? 0 : 1);
    const int kind = bc.kind[face];
    if (kind == kInflow && !psi) {
      r.inflow = face;
      return r;
    }
    c[ax] = map_index(c[ax], n[ax], kind);
    if (kind == kReflect) r.flip ^= 1 << ax;
  }
  r.src = cell(g, c[0], c[1], c[2]);
  return r;
}

// Dirichlet value of a field with the given role at an inflow face: the face's
// conserved state, its particle offset dt * u_in, or phi = sqrt(2 p_in) (a uniform
// inflow state is not compressed: its predicted volume is the cell's)
__device__ __forceinline__ Real inflow_value(const BcDev& bc, int face, int role, double dt) {
  if (role <= kE) return (Real)bc.cons[face][role];
  if (role == kPhi) return (Real)bc.phi[face];
  return (Real)(dt * bc.vel[face][role - kXx]);
}

// value of a field with the given role at a ghost cell
__device__ __forceinline__ Real ghost_get(const BcDev& bc, const GhostSrc& m, const Real* f, int role,
                                          double dt) {
  int axis = -1;
  if (role >= kMx && role <= kMz) axis = role - kMx;
  if (role >= kXx && role <= kXz) axis = role - kXx;
  const Real sign = (axis >= 0 && ((m.flip >> axis) & 1)) ? (Real)-1 : (Real)1;
  if (m.inflow >= 0) return sign * inflow_value(bc, m.inflow, role, dt);
  return sign * f[m.src];
}

__device__ __forceinline__ void fill_body(const FillSet<Real>& fs, const GridDev& g, const BcDev& bc,
                                          const Ctrl* ctrl, unsigned t) {
  int i, j, k;
  if (!ghost_cell(g, t, i, j, k)) return;
  const double dt = ctrl->dt;
  const long long cg = cell(g, i, j, k);
  for (int q = 0; q < fs.n; ++q) {
    const GhostSrc m = ghost_src(g, bc, i, j, k, fs.role[q] == kPsi);
    fs.f[q][cg] = ghost_get(bc, m, fs.f[q], fs.role[q], dt);
  }
}

__device__ __forceinline__ bool in_x_zone(const GridDev& g, unsigned t) {
  return t >= 4u * (unsigned)g.sx * (unsigned)g.sy + (unsigned)g.nz * 4u * (unsigned)g.sx;
}

// ghosts of the predicted particles, then psi at their predicted positions for
// the first ghost layer (the corrector reads psi* of index neighbours only)
__device__ __forceinline__ void fill_pred_body(const Fields<Real>& F, const GridDev& g, const BcDev& bc,
                                               const Ctrl* ctrl, unsigned t) {
  int i, j, k;
  if (!ghost_cell(g, t, i, j, k)) return;
  const double dt = ctrl->dt;
  const long long cg = cell(g, i, j, k);
  // the predicted state is read one cell beyond the interior only (stage C's
  // halo, stage E's one-cell halo): the second ghost layer is left unfilled
  const bool first = i >= -1 && i <= g.nx && j >= -1 && j <= g.ny && k >= -1 && k <= g.nz;
  if (!first) return;
  Real xi[3], ms[3];
  if (kPushX && in_x_zone(g, t)) {
    // stage P wrote this x ghost's predicted state; psi at its position is left
    if (i != -1 && i != g.nx) return;
    if (!g.psi) return;  // psi(r*) stays 0
#pragma unroll
    for (int q = 0; q < 3; ++q) ms[q] = F.ms[q][cg];
  } else {
    const GhostSrc m = ghost_src(g, bc, i, j, k, false);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      ms[q] = ghost_get(bc, m, F.ms[q], kMx + q, dt);
      F.ms[q][cg] = ms[q];
    }
    F.phs[cg] = ghost_get(bc, m, F.phs, kPhi, dt);
    if constexpr (kKeepXiStar) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        xi[q] = ghost_get(bc, m, F.xs[q], kXx + q, dt);
        F.xs[q][cg] = xi[q];
      }
    }
  }
  if (!g.psi) return;  // psi(r*) stays 0
  if constexpr (!kKeepXiStar) {
    // the ghost's offset from its own (already filled) rho, m^n and m*
    const int par = ctrl->par;
    const Real r = F.U[par][0][cg];
    Real un[3], us[3];
    velocity(g, r, F.U[par][1][cg], F.U[par][2][cg], F.U[par][3][cg], un);
    velocity(g, r, ms[0], ms[1], ms[2], us);
    xi_star(un, us, (Real)(0.5 * dt), xi);
  }
  {
    const Real* P = F.psic;
    auto at = [&](int a, int b, int c) { return P[cg + a + (long long)b * g.sx + (long long)c * g.sxy]; };
    F.psis[cg] = psi_at(g, at, xi[0], xi[1], xi[2]);
  }
}

// sources and sinks: the first half step on U^n (interior cells), before its
// ghosts are filled
__global__ void __launch_bounds__(256) k_source(Fields<Real> F, GridDev g, const Ctrl* __restrict__ ctrl) {
  if (!ctrl->active) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const Real hdt = (Real)(0.5 * ctrl->dt);
  Real* const* U = F.U[ctrl->par];
  for (int k = blockIdx.z; k < g.nz; k += gridDim.z) {
    const long long c = cell(g, i, j, k);
    const Real q = F.src[c];
    if (q == (Real)0) continue;
    Real r = U[0][c], mx = U[1][c], my = U[2][c], mz = U[3][c], E = U[4][c];
    source_cell(q, (Real)g.eps_src, hdt, r, mx, my, mz, E);
    U[0][c] = r;
    U[1][c] = mx;
    U[2][c] = my;
    U[3][c] = mz;
    U[4][c] = E;
  }
}

// ghosts of the post-Lagrange particles
__device__ __forceinline__ void fill_corr_body(const Fields<Real>& F, const GridDev& g, const BcDev& bc,
                                               const Ctrl* ctrl, unsigned t) {
  int i, j, k;
  if (!ghost_cell(g, t, i, j, k)) return;
  if (kPushX && in_x_zone(g, t)) return;  // written by stage C
  // read one cell beyond the interior only (stage E's one-cell halo)
  if (i < -1 || i > g.nx || j < -1 || j > g.ny || k < -1 || k > g.nz) return;
  const double dt = ctrl->dt;
  const long long cg = cell(g, i, j, k);
  const GhostSrc m = ghost_src(g, bc, i, j, k, false);
#pragma unroll
  for (int q = 0; q < 4; ++q) F.mt[q][cg] = ghost_get(bc, m, F.mt[q], kMx + q, dt);
  if constexpr (kKeepXi) {
#pragma unroll
    for (int q = 0; q < 3; ++q) F.xt[q][cg] = ghost_get(bc, m, F.xt[q], kXx + q, dt);
  }
}

__device__ __forceinline__ void fill_state_body(const Fields<Real>& F, const GridDev& g, const BcDev& bc,
                                                const Ctrl* ctrl, unsigned t) {
  int i, j, k;
  if (!ghost_cell(g, t, i, j, k)) return;
  if (kPushX && in_x_zone(g, t)) return;  // written by stage E of the previous step
  const int par = ctrl->par;
  const long long cg = cell(g, i, j, k);
  const GhostSrc m = ghost_src(g, bc, i, j, k, false);
#pragma unroll
  for (int role = 0; role < 5; ++role) F.U[par][role][cg] = ghost_get(bc, m, F.U[par][role], role, 0.0);
}

__global__ void __launch_bounds__(256) k_fill(FillSet<Real> fs, GridDev g, BcDev bc,
                                              const Ctrl* __restrict__ ctrl, int check_active) {
  if (check_active && !ctrl->active) return;
  fill_body(fs, g, bc, ctrl, blockIdx.x * blockDim.x + threadIdx.x);
}

// every ghost zone of U^n (the state copy is known on the device only)
__global__ void __launch_bounds__(256) k_fill_u(Fields<Real> F, FillSet<Real> fs, GridDev g, BcDev bc,
                                                const Ctrl* __restrict__ ctrl) {
  if (!ctrl->active) return;
  for (int v = 0; v < 5; ++v) fs.f[v] = F.U[ctrl->par][v];
  fill_body(fs, g, bc, ctrl, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(256) k_fill_pred(Fields<Real> F, GridDev g, BcDev bc,
                                                   const Ctrl* __restrict__ ctrl) {
  if (!ctrl->active) return;
  fill_pred_body(F, g, bc, ctrl, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(256) k_fill_corr(Fields<Real> F, GridDev g, BcDev bc,
                                                   const Ctrl* __restrict__ ctrl) {
  if (!ctrl->active) return;
  fill_corr_body(F, g, bc, ctrl, blockIdx.x * blockDim.x + threadIdx.x);
}


// batched ghost fills: every instance's ghost range is padded to whole blocks
// of 256, and a host-built map gives each block its (instance, first ghost)
template <int kWhich>
__global__ void __launch_bounds__(256) k_fill_batch(const Inst<Real>* __restrict__ tab,
                                                    const int2* __restrict__ map, int nblocks) {
  if ((int)blockIdx.x >= nblocks) return;
  const int2 w = map[blockIdx.x];
  const Inst<Real>& I = tab[w.x];
  if (!I.ctrl->active) return;
  const unsigned t = (unsigned)w.y + threadIdx.x;
  if (kWhich == 0) fill_state_body(I.F, I.g, I.bc, I.ctrl, t);
  else if (kWhich == 1) fill_pred_body(I.F, I.g, I.bc, I.ctrl, t);
  else fill_corr_body(I.F, I.g, I.bc, I.ctrl, t);
}

// Ghost columns of the x faces written by the stage that produces a field:
// interior cell i of an interior row calls put(gi, flip, face) for every ghost
// column gi at depth 1..D whose rule reads it (periodic wrap, outflow copy,
// reflect mirror -- flip: the x components change sign); at an inflow face the
// boundary cell writes the face's Dirichlet state (face >= 0).  Together with the
// y and z ghost zones, which the fill kernels still compute (their rows are
// contiguous, the x ghosts are not), this gives every ghost the value of the
// rules in x, y, z order.
template <int D, typename Put>
__device__ __forceinline__ void x_push(const GridDev& g, const BcDev& bc, int i, Put&& put) {
  const int n = g.nx, kl = bc.kind[0], ku = bc.kind[1];
#pragma unroll
  for (int d = 1; d <= D; ++d) {
    const int sl = kl == kPeriodic ? n - d : (kl == kReflect ? d - 1 : 0);
    if (sl == i) put(-d, kl == kReflect, kl == kInflow ? 0 : -1);
    const int su = ku == kPeriodic ? d - 1 : (ku == kReflect ? n - d : n - 1);
    if (su == i) put(n - 1 + d, ku == kReflect, ku == kInflow ? 1 : -1);
  }
}

// value of a pushed x ghost: the cell's own value v (sign-flipped for the x
// components at a reflecting face) or the inflow face's state
__device__ __forceinline__ Real x_ghost_value(const BcDev& bc, Real v, int role, bool flip, int face,
                                              double dt) {
  if (face >= 0) return inflow_value(bc, face, role, dt);
  return (flip && (role == kMx || role == kXx)) ? -v : v;
}

long long ghost_count(const GridDev& g) {
  return 4LL * g.sx * g.sy + (long long)g.nz * 4 * g.sx + (long long)g.nz * g.ny * 4;
}

// ==================================================================== time step
__device__ __forceinline__ void block_max_to(double v, unsigned long long* dst) {
  __shared__ double red[16];
  v = wave_max(v);
  const int nw = (blockDim.x * blockDim.y * blockDim.z + kWave - 1) / kWave;
  const int flat = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  if (flat % kWave == 0) red[flat / kWave] = v;
  __syncthreads();
  if (flat == 0) {
    double m = red[0];
    for (int q = 1; q < nw; ++q) m = fmax(m, red[q]);
    if (m > 0.0) atomicMax(dst, (unsigned long long)__double_as_longlong(m));
  }
}

// max signal speed of U^n (before the first step; later steps take it from the
// stage-E epilogue).  Blocks stride over the z planes, so that few blocks meet
// at the one atomic.
__global__ void __launch_bounds__(256) k_signal_max(Fields<Real> F, GridDev g, Ctrl* ctrl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int par = ctrl->par;
  double v = 0.0;
  if (i < g.nx && j < g.ny) {
    for (int k = blockIdx.z; k < g.nz; k += gridDim.z) {
      const long long c = cell(g, i, j, k);
      v = fmax(v, signal_speed(g, F.U[par][0][c], F.U[par][1][c], F.U[par][2][c], F.U[par][3][c],
                               F.U[par][4][c]));
    }
  }
  block_max_to(v, &ctrl->smax_bits[ctrl->cur]);
}

// dt = cfl h / smax, capped by dt_max (> 0) and by the time left to t_end
__device__ __forceinline__ void begin_body(Ctrl* ctrl, const GridDev& g, double dt_max, double t_end) {
  if (ctrl->status || ctrl->done) {
    ctrl->active = 0;
    return;
  }
  const double smax = __longlong_as_double((long long)ctrl->smax_bits[ctrl->cur]);
  double dt;
  const double dv = g.dt_visc;  // the viscous limit, 0 when inviscid
  if (smax > 0.0 || dv > 0.0) {
    dt = smax > 0.0 ? g.cfl_h / smax : dv;
    if (dv > 0.0 && dv < dt) dt = dv;
    if (dt_max > 0.0 && dt_max < dt) dt = dt_max;
  } else {
    if (!(dt_max > 0.0)) {
      ctrl->status |= kBadNoSignal;
      ctrl->active = 0;
      return;
    }
    dt = dt_max;
  }
  int lands = 0;
  if (isfinite(t_end) && t_end - ctrl->t <= dt) {
    dt = t_end - ctrl->t;
    lands = 1;
  }
  if (!(dt > 0.0)) {
    ctrl->done = 1;
    ctrl->active = 0;
    return;
  }
  ctrl->dt = dt;
  ctrl->t = lands ? t_end : ctrl->t + dt;
  ctrl->nsteps += 1;
  if (lands) ctrl->done = 1;
  ctrl->active = 1;
  ctrl->smax_bits[1 - ctrl->cur] = 0ULL;
}

__device__ __forceinline__ void end_body(Ctrl* ctrl) {
  if (!ctrl->active) return;
  ctrl->par = 1 - ctrl->par;
  ctrl->cur = 1 - ctrl->cur;
  ctrl->smax_valid = 1;
  ctrl->active = 0;
}

__global__ void k_begin(Ctrl* ctrl, GridDev g, double dt_max, double t_end) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  begin_body(ctrl, g, dt_max, t_end);
}

__global__ void k_end(Ctrl* ctrl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  end_body(ctrl);
}

// the step's start and the ghosts of U^n in one launch: thread 0 of block 0
// takes the step's dt (and whether it runs); every thread fills its ghost cell
// from the interior either way (the fill only restates the ghost rules, so a
// step that does not run leaves the state as it was)
__global__ void __launch_bounds__(256) k_begin_fill(Fields<Real> F, GridDev g, BcDev bc, Ctrl* ctrl,
                                                    double dt_max, double t_end) {
  if (blockIdx.x == 0 && threadIdx.x == 0) begin_body(ctrl, g, dt_max, t_end);
  fill_state_body(F, g, bc, ctrl, blockIdx.x * blockDim.x + threadIdx.x);
}

// batch members: each stops at its own step limit or end time
__global__ void k_begin_batch(const Inst<Real>* __restrict__ tab, int n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  Ctrl* c = tab[q].ctrl;
  if (c->nsteps >= c->step_limit) {
    c->done = 1;
    c->active = 0;
    return;
  }
  begin_body(c, tab[q].g, 0.0, c->t_end);
  if (c->active && c->nsteps >= c->step_limit) c->done = 1;
}

__global__ void k_end_batch(const Inst<Real>* __restrict__ tab, int n, int* __restrict__ flags) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  Ctrl* c = tab[q].ctrl;
  end_body(c);
  flags[q] = (c->done ? 1 : 0) | (c->status ? 2 : 0);
}

// ==================================================================== LDS planes
// slot of plane k in a ring of three
__device__ __forceinline__ int ring3(int k) { return ((k % 3) + 3) % 3; }
__device__ __forceinline__ int hidx(int hx, int hy) { return hy * HX + hx; }

// ==================================================================== stages P and C
// Both Lagrangian sweeps evaluate Q = -(0, A, B) of Eq. (7) with the kernel
// gradients of the particles' reference configuration: every particle starts the
// step at its cell centre, so these are the 13 lattice gradients K(-h o) (and
// their negatives), with pressure and potential in one pair-difference sum.
//   stage P, predictor (Eq. (5)), on U^n: m* = m - dt A, E* = E - dt B,
//     xi* = dt (u^n + u*)/2, psi* = psi(x + xi*), and phi* = sqrt(2 p*) of the
//     predicted particle, p* its internal energy over its predicted volume
//     V*/h^3 = 1 + dt div(u^n) (the lattice divergence);
//   stage C, corrector (Eq. (6)), on the predicted particles (rho, u* = m*/rho,
//     phi*, psi*): m~ = (m + m*)/2 - (dt/2) A*, E~ likewise, and in FP64
//     xi^{n+1} = xi*/2 + dt (u^n + u~)/4 (FP32 forms it in stage E).
// ux, uy, uz hold the velocity, or phi u in the FP32 corrector (see kPhiU)
template <class Sh>
struct PlaneL {
  static constexpr int HP = Sh::HP;
  Real rho[3][HP], phi[3][HP], ux[3][HP], uy[3][HP], uz[3][HP], psi[3][HP];
};

// kCorr: stage C (else P).  kPsi: a potential is set (g.psi); without one psi = 0
// and psi(r*) stays 0.  The plane buffers S belong to the kernel, so every form
// shares them.
// kVisc: a viscosity is set (g.nu > 0): the viscous force and its work join the sums.
// kGrav (predictor with self-gravity): psi at r* is sampled from the potential
// of the predicted density (F.psic, in memory) instead of the planes' psi.
// Sh: the tile shape.
template <bool kCorr, bool kPsi, bool kVisc, bool kGrav, class Sh>
__device__ __forceinline__ void stage_l_body(PlaneL<Sh>& S, const Fields<Real>& F, const GridDev& g,
                                             const BcDev& bc, const Ctrl* __restrict__ ctrl, const Tile& T) {
  constexpr int TX = Sh::TX, HX = Sh::HX, HP = Sh::HP;
  auto hidx = [](int hx, int hy) { return hy * HX + hx; };
  const int par = ctrl->par;
  const Real* __restrict__ R = F.U[par][0];
  const Real* __restrict__ MX = F.U[par][1];
  const Real* __restrict__ MY = F.U[par][2];
  const Real* __restrict__ MZ = F.U[par][3];
  const Real* __restrict__ EE = F.U[par][4];
  // the fields the planes are formed from: U^n and psi (P), m*, phi*, psi* (C)
  const Real* __restrict__ LX = kCorr ? F.ms[0] : MX;
  const Real* __restrict__ LY = kCorr ? F.ms[1] : MY;
  const Real* __restrict__ LZ = kCorr ? F.ms[2] : MZ;
  const Real* __restrict__ LE = kCorr ? F.phs : EE;
  const Real* __restrict__ PS = kCorr ? F.psis : F.psi;
  const double dt = ctrl->dt;
  const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
  const int i = T.x0 + tx, j = T.y0 + ty;
  const bool in = i < g.nx && j < g.ny;
  const uint32_t oc = in ? in_plane(g, i, j) : 0u;  // this column's cell in a plane
  // FP32: with K_- = -K_+ the energy sum of a pair,
  // phi_c [phi_+ (u_c + u_+) - phi_- (u_c + u_-)] . K / 2, is
  // phi_c [(phi_+ - phi_-) u_c . K + ((phi u)_+ - (phi u)_-) . K] / 2, whose first
  // part reuses the pressure difference of the momentum sum.  The corrector keeps
  // phi u in its planes instead of u (it needs no neighbour velocity otherwise).
  constexpr bool kPhiU = kCorr && !kF64 && !kVisc;

  // A plane's cells are fetched from memory into registers one iteration before
  // they are formed into the LDS ring: the loads of plane k+2 are in flight while
  // plane k is computed.  Each thread handles up to kPer halo cells of a plane.
  constexpr int kPer = (HP + NT - 1) / NT;
  struct Raw {
    Real r, x, y, z, e, p;  // rho, then m (P) or m* (C), E (P) or phi* (C), psi (P) or psi* (C)
  };
  Raw raw[kPer];
  auto cell_of = [&](int h, uint32_t& ob) {
    const int q = tid + h * NT;
    const int hx = q % HX, hy = q / HX;
    const int ii = T.x0 - 1 + hx, jj = T.y0 - 1 + hy;
    const bool ok = q < HP && ii <= g.nx && jj <= g.ny;
    ob = ok ? in_plane(g, ii, jj) : 0u;
    return ok;
  };
  auto fetch = [&](int k) {
    const long long pz = plane0(g, k);
#pragma unroll
    for (int h = 0; h < kPer; ++h) {
      uint32_t ob0;
      if (!cell_of(h, ob0)) continue;
      const uint32_t ob = opaque32(ob0);
      raw[h].r = *at_plane(R, pz, ob);
      raw[h].x = *at_plane(LX, pz, ob);
      raw[h].y = *at_plane(LY, pz, ob);
      raw[h].z = *at_plane(LZ, pz, ob);
      raw[h].e = *at_plane(LE, pz, ob);
      raw[h].p = kPsi ? *at_plane(PS, pz, ob) : (Real)0;
    }
  };
  auto put = [&](int k) {
    const int s = ring3(k);
#pragma unroll
    for (int h = 0; h < kPer; ++h) {
      uint32_t ob;
      if (!cell_of(h, ob)) continue;
      const int q = tid + h * NT;
      const Real r = raw[h].r;
      Real u[3], ph;
      if constexpr (kCorr) {
        velocity(g, r, raw[h].x, raw[h].y, raw[h].z, u);
        ph = raw[h].e;
      } else {
        Real p;
        primitive(g, r, raw[h].x, raw[h].y, raw[h].z, raw[h].e, u[0], u[1], u[2], p);
        ph = sqrt_fast((Real)2 * p);
      }
      if constexpr (kPhiU) {
#pragma unroll
        for (int d = 0; d < 3; ++d) u[d] *= ph;
      }
      S.rho[s][q] = r;
      S.phi[s][q] = ph;
      S.ux[s][q] = u[0];
      S.uy[s][q] = u[1];
      S.uz[s][q] = u[2];
      S.psi[s][q] = raw[h].p;
    }
  };

  fetch(T.z0 - 1);
  put(T.z0 - 1);
  fetch(T.z0);
  put(T.z0);
  fetch(T.z0 + 1);
  for (int k = T.z0; k < T.z1; ++k) {
    put(k + 1);
    if (k + 2 <= T.z1) fetch(k + 2);
    lds_barrier();
    if (in) {
      const int s0 = ring3(k), c0 = hidx(tx + 1, ty + 1);
      auto nb = [&](int ox, int oy, int oz) { return ring3(k + oz) * HP + hidx(tx + 1 + ox, ty + 1 + oy); };
      const Real rc = S.rho[s0][c0], fc = S.phi[s0][c0], psc = S.psi[s0][c0];
      const Real uc[3] = {S.ux[s0][c0], S.uy[s0][c0], S.uz[s0][c0]};
      const Real* phi_ = &S.phi[0][0];
      const Real* ux_ = &S.ux[0][0];
      const Real* uy_ = &S.uy[0][0];
      const Real* uz_ = &S.uz[0][0];
      const Real* psi_ = &S.psi[0][0];
      Acc a[3] = {0.0, 0.0, 0.0}, gp[3] = {0.0, 0.0, 0.0}, be = 0.0, dv = 0.0;
      Real af[3] = {0, 0, 0}, gf[3] = {0, 0, 0}, bf = 0, dvf = 0;
      Real gph[3] = {0, 0, 0};  // FP32: sum of (phi_+ - phi_-) K
      // viscous force and work (kVisc)
      Acc vm[3] = {0.0, 0.0, 0.0}, ve = 0.0;
      const Real* rho_ = &S.rho[0][0];
#pragma unroll
      for (int q = 0; q < 13; ++q) {
        const int ox = O13::o[q][0], oy = O13::o[q][1], oz = O13::o[q][2];
        const int np = nb(ox, oy, oz), nm = nb(-ox, -oy, -oz);
        const Real Kx = (Real)g.klat[q][0], Ky = (Real)g.klat[q][1], Kz = (Real)g.klat[q][2];
        if constexpr (kF64) {
          // the two terms of the pair, each as the scheme writes it, then their sum;
          // components whose offset is 0 carry an exact zero and are skipped
          Acc ta[2][3], tg[2][3], te[2], td[2];
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            const int n = side == 0 ? np : nm;
            const Real sg = side == 0 ? (Real)1 : (Real)-1;
            const Real kx = sg * Kx, ky = sg * Ky, kz = sg * Kz;
            const Acc ff = fc * phi_[n];
            const Acc dpsi = psi_[n] - psc;
            const Acc sp = ff + rc * dpsi;
            Acc ub = (uc[0] + ux_[n]) * kx;
            if (ox == 0) ub = (uc[1] + uy_[n]) * ky;
            else if (oy != 0) ub = ub + (uc[1] + uy_[n]) * ky;
            if (oz != 0) ub = ub + (uc[2] + uz_[n]) * kz;
            ub = 0.5 * ub;
            ta[side][0] = sp * kx;
            ta[side][1] = sp * ky;
            ta[side][2] = sp * kz;
            tg[side][0] = dpsi * kx;
            tg[side][1] = dpsi * ky;
            tg[side][2] = dpsi * kz;
            te[side] = ff * ub;
            if constexpr (!kCorr) {
              // K . u^n of the neighbour, for the lattice divergence
              Acc t = kx * ux_[n];
              if (ox == 0) t = ky * uy_[n];
              else if (oy != 0) t = t + ky * uy_[n];
              if (oz != 0) t = t + kz * uz_[n];
              td[side] = t;
            }
          }
          if (ox != 0) {
            a[0] = a[0] + (ta[0][0] + ta[1][0]);
            gp[0] = gp[0] + (tg[0][0] + tg[1][0]);
          }
          if (oy != 0) {
            a[1] = a[1] + (ta[0][1] + ta[1][1]);
            gp[1] = gp[1] + (tg[0][1] + tg[1][1]);
          }
          if (oz != 0) {
            a[2] = a[2] + (ta[0][2] + ta[1][2]);
            gp[2] = gp[2] + (tg[0][2] + tg[1][2]);
          }
          be = be + (te[0] + te[1]);
          if constexpr (!kCorr) dv = dv + (td[0] + td[1]);
          if constexpr (kVisc) {
            // f = nu lambda (rho_c + rho_n)/2 (u_n - u_c), work f . (u_c + u_n)/2
            Acc tv[2][3], tw[2];
#pragma unroll
            for (int side = 0; side < 2; ++side) {
              const int n = side == 0 ? np : nm;
              const Acc cv = g.nulam[q] * (0.5 * (rc + rho_[n]));
              tv[side][0] = cv * (ux_[n] - uc[0]);
              tv[side][1] = cv * (uy_[n] - uc[1]);
              tv[side][2] = cv * (uz_[n] - uc[2]);
              tw[side] = 0.5 * (tv[side][0] * (uc[0] + ux_[n]) + tv[side][1] * (uc[1] + uy_[n]) +
                                tv[side][2] * (uc[2] + uz_[n]));
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) vm[d] = vm[d] + (tv[0][d] + tv[1][d]);
            ve = ve + (tw[0] + tw[1]);
          }
        } else {
          // pair difference phi_c (phi_+ - phi_-) + rho_c (psi_+ - psi_-): the FP32
          // differences are exact for neighbours within a factor 2, the combination
          // is formed in FP64, then times the lattice K
          const Real dphi = phi_[np] - phi_[nm];
          const Real ds = psi_[np] - psi_[nm];
          const Real s = (Real)((Acc)fc * (Acc)dphi + (Acc)rc * (Acc)ds);
          if (ox != 0) {
            af[0] += s * Kx;
            gf[0] += ds * Kx;
          }
          if (oy != 0) {
            af[1] += s * Ky;
            gf[1] += ds * Ky;
          }
          if (oz != 0) {
            af[2] += s * Kz;
            gf[2] += ds * Kz;
          }
          if constexpr (kVisc) {
            const float nl = (float)g.nulam[q];
#pragma unroll
            for (int side = 0; side < 2; ++side) {
              const int n = side == 0 ? np : nm;
              const float cv = nl * (0.5f * (rc + rho_[n]));
              const float t0 = cv * (ux_[n] - uc[0]), t1 = cv * (uy_[n] - uc[1]),
                          t2 = cv * (uz_[n] - uc[2]);
              vm[0] += t0;
              vm[1] += t1;
              vm[2] += t2;
              ve += 0.5f * (t0 * (uc[0] + ux_[n]) + t1 * (uc[1] + uy_[n]) + t2 * (uc[2] + uz_[n]));
            }
          }
          // energy sum: K . ((phi u)_+ - (phi u)_-) and (phi_+ - phi_-) K (the
          // corrector's planes hold phi u; the predictor forms it here)
          const Real fp = phi_[np], fm = phi_[nm];
          auto dphiu = [&](const Real* u_) {
            if constexpr (kPhiU) return u_[np] - u_[nm];
            else return fmaf(-fm, u_[nm], fp * u_[np]);
          };
          if (ox != 0) {
            gph[0] = fmaf(dphi, Kx, gph[0]);
            bf = fmaf(Kx, dphiu(ux_), bf);
            if constexpr (!kCorr) dvf = fmaf(Kx, ux_[np] - ux_[nm], dvf);
          }
          if (oy != 0) {
            gph[1] = fmaf(dphi, Ky, gph[1]);
            bf = fmaf(Ky, dphiu(uy_), bf);
            if constexpr (!kCorr) dvf = fmaf(Ky, uy_[np] - uy_[nm], dvf);
          }
          if (oz != 0) {
            gph[2] = fmaf(dphi, Kz, gph[2]);
            bf = fmaf(Kz, dphiu(uz_), bf);
            if constexpr (!kCorr) dvf = fmaf(Kz, uz_[np] - uz_[nm], dvf);
          }
        }
      }
      const long long c = cell(g, i, j, k);
      // A and B of this cell
      Real Av[3], Bv;
      if constexpr (kF64) {
        // Q = -(0, A, B): the viscous force and its work enter with the other sign
#pragma unroll
        for (int d = 0; d < 3; ++d) Av[d] = a[d] - vm[d];
        Bv = (be + rc * (uc[0] * gp[0] + uc[1] * gp[1] + uc[2] * gp[2])) - ve;
      } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) Av[d] = af[d] - (Real)vm[d];
        // the cell's own velocity (the corrector's planes hold phi u)
        Real u0[3] = {uc[0], uc[1], uc[2]};
        if constexpr (kPhiU) velocity(g, rc, F.ms[0][c], F.ms[1][c], F.ms[2][c], u0);
        const Real ug = u0[0] * gph[0] + u0[1] * gph[1] + u0[2] * gph[2];
        Bv = (Real)0.5 * fc * (ug + bf) + rc * (u0[0] * gf[0] + u0[1] * gf[1] + u0[2] * gf[2]) -
             (Real)ve;
      }
      const Real m0[3] = {MX[c], MY[c], MZ[c]};
      if constexpr (!kCorr) {
        // ---------------------------------------------------------- predictor
        Real ms[3], Es;
        if constexpr (kF64) {
#pragma unroll
          for (int d = 0; d < 3; ++d) ms[d] = m0[d] - dt * Av[d];
          Es = EE[c] - dt * Bv;
        } else {
          const Real rdt = (Real)dt;
#pragma unroll
          for (int d = 0; d < 3; ++d) ms[d] = m0[d] - rdt * Av[d];
          Es = EE[c] - rdt * Bv;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) F.ms[d][c] = ms[d];
        F.ms[3][c] = Es;
        Real us[3], ps;
        primitive(g, rc, ms[0], ms[1], ms[2], Es, us[0], us[1], us[2], ps);
        // phi* of the predicted particle: its pressure over its predicted volume
        Real phs;
        if constexpr (kF64) {
          const Real vol = 1.0 + dt * dv;
          const Real pv = ps / vol;
          phs = sqrt(2.0 * pv);
        } else {
          const float vol = fmaf((float)dt, dvf, 1.0f);
          phs = sqrt_fast((Real)2 * (ps * __builtin_amdgcn_rcpf(vol)));
        }
        F.phs[c] = phs;
        Real xi[3];
        xi_star(uc, us, (Real)(0.5 * dt), xi);
        if constexpr (kKeepXiStar) {
#pragma unroll
          for (int d = 0; d < 3; ++d) F.xs[d][c] = xi[d];
        }
        if constexpr (kGrav) {
          const Real* Pc = F.psic;
          auto at = [&](int a_, int b_, int c_) {
            return Pc[c + a_ + (long long)b_ * g.sx + (long long)c_ * g.sxy];
          };
          F.psis[c] = psi_at(g, at, xi[0], xi[1], xi[2]);
        } else if constexpr (kPsi) {
          auto at = [&](int a_, int b_, int c_) { return psi_[nb(a_, b_, c_)]; };
          F.psis[c] = psi_at(g, at, xi[0], xi[1], xi[2]);
        }
        if (kPushX && (i < 2 || i >= g.nx - 2)) {
          // x ghosts of the predicted particles (psi at their positions is left to
          // the fill kernel: it needs loads that would stall this sweep)
          x_push<1>(g, bc, i, [&](int gi, bool flip, int face) {
            const long long cg = cell(g, gi, j, k);
            F.ms[0][cg] = x_ghost_value(bc, ms[0], kMx, flip, face, dt);
            F.ms[1][cg] = x_ghost_value(bc, ms[1], kMy, flip, face, dt);
            F.ms[2][cg] = x_ghost_value(bc, ms[2], kMz, flip, face, dt);
            F.phs[cg] = x_ghost_value(bc, phs, kPhi, flip, face, dt);
          });
        }
      } else {
        // ---------------------------------------------------------- corrector
        const Real E0 = EE[c];
        const Real msc[3] = {F.ms[0][c], F.ms[1][c], F.ms[2][c]};
        const Real Esc = F.ms[3][c];
        Real mt[3], Et;
        if constexpr (kF64) {
          const Acc hdt = 0.5 * dt;
#pragma unroll
          for (int d = 0; d < 3; ++d) mt[d] = 0.5 * (m0[d] + msc[d]) - hdt * Av[d];
          Et = 0.5 * (E0 + Esc) - hdt * Bv;
        } else {
          const Real hdt = (Real)(0.5 * dt);
#pragma unroll
          for (int d = 0; d < 3; ++d) mt[d] = (Real)0.5 * (m0[d] + msc[d]) - hdt * Av[d];
          Et = (Real)0.5 * (E0 + Esc) - hdt * Bv;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) F.mt[d][c] = mt[d];
        F.mt[3][c] = Et;
        if constexpr (kKeepXi) {
          // xi^{n+1} = xi*/2 + dt (u^n + u~)/4
          Real un[3], ut[3], pn, pt;
          primitive(g, rc, m0[0], m0[1], m0[2], E0, un[0], un[1], un[2], pn);
          primitive(g, rc, mt[0], mt[1], mt[2], Et, ut[0], ut[1], ut[2], pt);
          const Real qdt = (Real)(0.25 * dt);
#pragma unroll
          for (int d = 0; d < 3; ++d) F.xt[d][c] = (Real)0.5 * F.xs[d][c] + qdt * (un[d] + ut[d]);
        }
        if (kPushX && (i < 2 || i >= g.nx - 2)) {
          // x ghosts of the post-Lagrange particles
          x_push<1>(g, bc, i, [&](int gi, bool flip, int face) {
            const long long cg = cell(g, gi, j, k);
            F.mt[0][cg] = x_ghost_value(bc, mt[0], kMx, flip, face, dt);
            F.mt[1][cg] = x_ghost_value(bc, mt[1], kMy, flip, face, dt);
            F.mt[2][cg] = x_ghost_value(bc, mt[2], kMz, flip, face, dt);
            F.mt[3][cg] = x_ghost_value(bc, Et, kE, flip, face, dt);
          });
        }
      }
    }
    lds_barrier();
  }
}

// ==================================================================== stage E
// Rusanov damping of the face velocity jump (normal weight 1, transverse 1/2),
// acoustic speed a = max(|u_n| + c) of the two reconstructed states.
__device__ __forceinline__ void acoustic_dissipation(const GridDev& g, int axis, const Real L[5],
                                                     const Real Rr[5], Real D[5]) {
  Real uL[3], uR[3], pL, pR;
  primitive(g, L[0], L[1], L[2], L[3], L[4], uL[0], uL[1], uL[2], pL);
  primitive(g, Rr[0], Rr[1], Rr[2], Rr[3], Rr[4], uR[0], uR[1], uR[2], pR);
  Real cL, cR;
  if constexpr (kF64) {
    cL = L[0] > (Real)g.rho_vac ? sqrt((Real)g.gamma * pL / L[0]) : (Real)0;
    cR = Rr[0] > (Real)g.rho_vac ? sqrt((Real)g.gamma * pR / Rr[0]) : (Real)0;
  } else {
    cL = L[0] > (Real)g.rho_vac ? sqrtf((Real)g.gamma * pL * __builtin_amdgcn_rcpf(L[0])) : (Real)0;
    cR = Rr[0] > (Real)g.rho_vac ? sqrtf((Real)g.gamma * pR * __builtin_amdgcn_rcpf(Rr[0])) : (Real)0;
  }
  const Real a = fmax(fabs(uL[axis]) + cL, fabs(uR[axis]) + cR);
  const Real kk = (Real)-0.5 * a * fmin(L[0], Rr[0]);
  const Real kt = (Real)0.5 * kk;
  D[0] = (Real)0;
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) D[1 + cc] = (cc == axis ? kk : kt) * (uR[cc] - uL[cc]);
  D[4] = (Real)0.5 * ((uL[0] + uR[0]) * D[1] + (uL[1] + uR[1]) * D[2] + (uL[2] + uR[2]) * D[3]);
}

// TVD limiter of the slope from the forward and backward differences a, b
// (undivided): minmod, MC, van Leer or superbee (the scheme lists the limiter
// as a free option, Sec. 4).
__device__ __forceinline__ Real limit(int kind, Real a, Real b) {
  if (a * b <= (Real)0) return (Real)0;
  const Real sg = a > (Real)0 ? (Real)1 : (Real)-1;
  const Real aa = fabs(a), ab = fabs(b);
  if (kind == kLimMC) {
    const Real m = fmin((Real)2 * aa, (Real)2 * ab);
    return sg * fmin(m, (Real)0.5 * (aa + ab));
  }
  if (kind == kLimVanLeer) return (Real)2 * a * b / (a + b);
  if (kind == kLimSuperbee) return sg * fmax(fmin((Real)2 * aa, ab), fmin(aa, (Real)2 * ab));
  return sg * fmin(aa, ab);
}

// Swept content of one face: Eq. (8) shifted reconstruction, HLL with the
// advective speed = max(X,0) U^L + min(X,0) U^R, plus the damping.  X is the
// displacement of the material that reaches the face, the particle offsets
// interpolated linearly between the face's two particles and taken at the foot
// of the face's trajectory: X = (xi_L + xi_R)/2 / (1 + (xi_R - xi_L)/h).
// kGen: the limiter and flux of the grid's scheme (g.limiter, g.flux) instead of
// the default minmod + swept volume with damping.
// u4[v][0..3]: component v of U^n at cells L-1, L, L+1 (= R), R+1;
// bL, bR: post-Lagrange bases of L and R; xL, xR: particle offsets along axis.
template <bool kGen>
__device__ __forceinline__ void face_flux(const GridDev& g, int axis, const Real u4[5][4],
                                          const Real bL[5], const Real bR[5], Real xL, Real xR,
                                          Real dt, Real Fo[5]) {
  if constexpr (kGen) {
    const Real nuL = xL * (Real)g.inv_h;
    const Real nuR = xR * (Real)g.inv_h;
    const Real X = (Real)0.5 * (xL + xR) / ((Real)1 + (xR - xL) * (Real)g.inv_h);
    Real UL[5], UR[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const Real sL = limit(g.limiter, u4[v][2] - u4[v][1], u4[v][1] - u4[v][0]);
      const Real sR = limit(g.limiter, u4[v][3] - u4[v][2], u4[v][2] - u4[v][1]);
      UL[v] = bL[v] + (Real)0.5 * ((Real)1 - nuL) * sL;
      UR[v] = bR[v] - (Real)0.5 * ((Real)1 + nuR) * sR;
      if (g.flux == kFluxLF) {
        // Lax-Friedrichs with the advective speeds xi/dt (times dt)
        const Real a = fmax(fabs(xL), fabs(xR));
        Fo[v] = (Real)0.5 * (xL * UL[v] + xR * UR[v]) - (Real)0.5 * a * (UR[v] - UL[v]);
      } else {
        Fo[v] = fmax(X, (Real)0) * UL[v] + fmin(X, (Real)0) * UR[v];
      }
    }
    if (g.flux == kFluxSweptAV) {
      Real D[5];
      acoustic_dissipation(g, axis, UL, UR, D);
#pragma unroll
      for (int v = 1; v < 5; ++v) Fo[v] = Fo[v] + dt * D[v];
    }
  } else if constexpr (kF64) {
    const Real nuL = xL * (Real)g.inv_h;
    const Real nuR = xR * (Real)g.inv_h;
    const Real X = (Real)0.5 * (xL + xR) / ((Real)1 + (xR - xL) * (Real)g.inv_h);
    Real UL[5], UR[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const Real sL = minmod(u4[v][2] - u4[v][1], u4[v][1] - u4[v][0]);
      const Real sR = minmod(u4[v][3] - u4[v][2], u4[v][2] - u4[v][1]);
      UL[v] = bL[v] + (Real)0.5 * ((Real)1 - nuL) * sL;
      UR[v] = bR[v] - (Real)0.5 * ((Real)1 + nuR) * sR;
      Fo[v] = fmax(X, (Real)0) * UL[v] + fmin(X, (Real)0) * UR[v];
    }
    Real D[5];
    acoustic_dissipation(g, axis, UL, UR, D);
#pragma unroll
    for (int v = 1; v < 5; ++v) Fo[v] = Fo[v] + dt * D[v];
  } else {
    // minmod(a, b) is the median of (a, b, 0); the reconstruction weights
    // (1 -+ xi/h)/2 and the swept fractions are formed once per face
    const float ih = (float)g.inv_h, hh = 0.5f * ih;
    const float wL = fmaf(xL, -hh, 0.5f), wR = fmaf(xR, hh, 0.5f);
    const float X = (0.5f * (xL + xR)) * __builtin_amdgcn_rcpf(fmaf(xR - xL, ih, 1.0f));
    const float pL = fmaxf(X, 0.0f), pR = fminf(X, 0.0f);
    float UL[5], UR[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const float d0 = u4[v][1] - u4[v][0], d1 = u4[v][2] - u4[v][1], d2 = u4[v][3] - u4[v][2];
      UL[v] = fmaf(wL, __builtin_amdgcn_fmed3f(d1, d0, 0.0f), bL[v]);
      UR[v] = fmaf(-wR, __builtin_amdgcn_fmed3f(d2, d1, 0.0f), bR[v]);
      Fo[v] = fmaf(pL, UL[v], pR * UR[v]);
    }
    // damping of the velocity jump: vacuum sides get a zero reciprocal density,
    // which zeroes their velocity and sound speed without a branch
    const float rv = (float)g.rho_vac, gm1 = (float)g.gm1, gam = (float)g.gamma;
    const float irL = UL[0] > rv ? __builtin_amdgcn_rcpf(UL[0]) : 0.0f;
    const float irR = UR[0] > rv ? __builtin_amdgcn_rcpf(UR[0]) : 0.0f;
    float uL[3], uR[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uL[c] = UL[1 + c] * irL;
      uR[c] = UR[1 + c] * irR;
    }
    const float mL = UL[1] * uL[0] + UL[2] * uL[1] + UL[3] * uL[2];
    const float mR = UR[1] * uR[0] + UR[2] * uR[1] + UR[3] * uR[2];
    const float pLp = fmaxf(gm1 * fmaf(-0.5f, mL, UL[4]), 0.0f);
    const float pRp = fmaxf(gm1 * fmaf(-0.5f, mR, UR[4]), 0.0f);
    const float cL = __builtin_amdgcn_sqrtf(gam * pLp * irL);
    const float cR = __builtin_amdgcn_sqrtf(gam * pRp * irR);
    const float a = fmaxf(fabsf(uL[axis]) + cL, fabsf(uR[axis]) + cR);
    const float kk = -0.5f * dt * a * fminf(UL[0], UR[0]);
    float Dm[3], de = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Dm[c] = (c == axis ? kk : 0.5f * kk) * (uR[c] - uL[c]);
      de = fmaf(uL[c] + uR[c], Dm[c], de);
      Fo[1 + c] += Dm[c];
    }
    Fo[4] = fmaf(0.5f, de, Fo[4]);
  }
}

// Every x and y face of a plane is computed once and shared by its two cells
// through LDS (2.2 face evaluations per cell and plane instead of 4); the z face
// is carried in registers from one plane to the next.

struct PlaneE {
  Real u[5][EP];      // U^n of the current plane, two-cell halo
  Real b[4][HP];      // m~, E~ of the current plane, one-cell halo
  Real xx[HP], xy[HP];  // x/y offsets xi (FP64), or the m*_x, m*_y they are formed from (FP32)
  Real fx[5][NFXP];   // x-face fluxes of the tile row by row (pitch EX): face i+1/2, i = x0-1 .. x0+TX-1
  Real fy[5][NFY];    // y-face fluxes: face j+1/2, j = y0-1 .. y0+TY-1
};


__device__ __forceinline__ int eidx(int ex, int ey) { return ey * EX + ex; }

template <bool kGen>
__device__ __forceinline__ bool tile_face(const GridDev& g, const Tile& T, const PlaneE& S,
                                          int axis, int row, int col, Real dt, const Real xc[4],
                                          Real Fo[5]) {
  Real u4[5][4], bl[5], br[5];
  int hl, hr;
  if (axis == 0) {
    // face between cells (x0-1+col, y0+row) and (x0+col, y0+row)
    if (T.y0 + row >= g.ny || T.x0 - 1 + col >= g.nx) return false;
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q) u4[v][q] = S.u[v][eidx(col + q, row + 2)];
    hl = hidx(col, row + 1);
    hr = hidx(col + 1, row + 1);
  } else {
    // face between cells (x0+col, y0-1+row) and (x0+col, y0+row)
    if (T.x0 + col >= g.nx || T.y0 - 1 + row >= g.ny) return false;
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q) u4[v][q] = S.u[v][eidx(col + 2, row + q)];
    hl = hidx(col + 1, row);
    hr = hidx(col + 1, row + 1);
  }
  bl[0] = u4[0][1];
  br[0] = u4[0][2];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    bl[1 + v] = S.b[v][hl];
    br[1 + v] = S.b[v][hr];
  }
  Real xl = axis == 0 ? S.xx[hl] : S.xy[hl];
  Real xr = axis == 0 ? S.xx[hr] : S.xy[hr];
  if constexpr (!kKeepXi) {
    // the offsets of the face's two cells from rho, m^n, m* and m~
    xl = xi_final(g, u4[0][1], u4[1 + axis][1], xl, bl[1 + axis], xc);
    xr = xi_final(g, u4[0][2], u4[1 + axis][2], xr, br[1 + axis], xc);
  }
  face_flux<kGen>(g, axis, u4, bl, br, xl, xr, dt, Fo);
  return true;
}

template <bool kGen>
__device__ __forceinline__ void stage_e_body(const Fields<Real>& F, const GridDev& g, const BcDev& bc,
                                             Ctrl* ctrl,
                                             const Tile& T, double* __restrict__ slot) {
  __shared__ PlaneE S;
  __shared__ double red[6][NT / kWave];
  __shared__ int redb;
  const int par = ctrl->par;
  const Real dt = (Real)ctrl->dt;
  // dt/2, dt/4, h/2, 1/h for the offsets formed here (FP32)
  const Real xc[4] = {(Real)(0.5 * ctrl->dt), (Real)(0.25 * ctrl->dt), (Real)(0.5 * g.h), (Real)g.inv_h};
  const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
  double tot[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  Real smr = (Real)0;  // max signal speed of this thread's cells
  int bad = 0;
  if (tid == 0) redb = 0;
  {
    const int i = T.x0 + tx, j = T.y0 + ty;
    const bool in = i < g.nx && j < g.ny;
    Real* const* Un = F.U[par];
    Real* const* Uo = F.U[1 - par];
    Real* const* X = kKeepXi ? F.xt : F.ms;
    // Own column, one plane behind the plane in LDS: at iteration k the z face
    // k-1/2 and the update of cell k-1 are formed, from plane k's values in LDS
    // and these registers: U^n at k-2, k-1 (uq), the base and z offset of k-1
    // (bq, xq), the x/y face sums of k-1 (aq) and the z-face flux k-3/2 (Fz).
    Real uq[5][2], bq[5], xq, aq[5], Fz[5];
    // this column's cell in plane k of field f
    const uint32_t oc = in ? in_plane(g, i, j) : 0u;
    auto at_col = [&](Real* f, int k) { return at_plane(f, plane0(g, k), opaque32(oc)); };
    auto ld_col = [&](int k, Real out[5]) {
      const long long pz = plane0(g, k);
      const uint32_t o = opaque32(oc);
#pragma unroll
      for (int v = 0; v < 5; ++v) out[v] = *at_plane(Un[v], pz, o);
    };
    auto ld_base = [&](int k, Real out[5]) {
      const long long pz = plane0(g, k);
      const uint32_t o = opaque32(oc);
      out[0] = *at_plane(Un[0], pz, o);
#pragma unroll
      for (int v = 0; v < 4; ++v) out[1 + v] = *at_plane(F.mt[v], pz, o);
    };
    // z offset of a particle of this column: FP32 forms it from rho, m^n_z, m*_z
    // (xs) and m~_z; FP64 has it stored (xs)
    auto z_offset = [&](Real rho, Real mnz, Real xs, Real mtz) {
      if constexpr (kKeepXi) return xs;
      else return xi_final(g, rho, mnz, xs, mtz, xc);
    };
    if (in) {
      Real t[5];
      ld_col(T.z0 - 2, t);
#pragma unroll
      for (int v = 0; v < 5; ++v) uq[v][0] = t[v];
      ld_col(T.z0 - 1, t);
#pragma unroll
      for (int v = 0; v < 5; ++v) uq[v][1] = t[v];
      ld_base(T.z0 - 1, bq);
      xq = z_offset(bq[0], uq[3][1], *at_col(X[2], T.z0 - 1), bq[3]);
    }
    // The current plane in LDS: U^n with a two-cell halo, the bases and x/y
    // offsets with one.  In FP32 the next plane is copied global -> LDS by the
    // DMA path of the vector memory unit (no registers held), issued once the
    // current plane's last LDS reads are done and in flight during the z face
    // and the cell updates; the barrier that ends the iteration waits for it.
    // Each wave stages 64 consecutive plane cells, which land at consecutive LDS
    // words.
    auto plane_load = [&](int k) {
      const long long pz = plane0(g, k);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = tid + h * NT;
        // this wave's 64 consecutive plane cells start at LDS word qb (a scalar)
        const int qb = __builtin_amdgcn_readfirstlane(h * NT + (tid & ~(kWave - 1)));
        const int ex = q % EX, ey = q / EX;
        const int ii = T.x0 - 2 + ex, jj = T.y0 - 2 + ey;
        if (q < EP && ii <= g.nx + 1 && jj <= g.ny + 1) {
          const uint32_t ob = opaque32(in_plane(g, ii, jj));
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            if constexpr (kF64) {
              S.u[v][q] = *at_plane(Un[v], pz, ob);
            } else {
              __builtin_amdgcn_global_load_lds(at_plane(Un[v], pz, ob), &S.u[v][qb], 4, 0, 0);
            }
          }
        }
        const int hx = q % HX, hy = q / HX;
        const int ib = T.x0 - 1 + hx, jb = T.y0 - 1 + hy;
        if (q < HP && ib <= g.nx && jb <= g.ny) {
          const uint32_t ob = opaque32(in_plane(g, ib, jb));
          if constexpr (kF64) {
#pragma unroll
            for (int v = 0; v < 4; ++v) S.b[v][q] = *at_plane(F.mt[v], pz, ob);
            S.xx[q] = *at_plane(X[0], pz, ob);
            S.xy[q] = *at_plane(X[1], pz, ob);
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v)
              __builtin_amdgcn_global_load_lds(at_plane(F.mt[v], pz, ob), &S.b[v][qb], 4, 0, 0);
            __builtin_amdgcn_global_load_lds(at_plane(X[0], pz, ob), &S.xx[qb], 4, 0, 0);
            __builtin_amdgcn_global_load_lds(at_plane(X[1], pz, ob), &S.xy[qb], 4, 0, 0);
          }
        }
      }
    };
    // FP64 loads each plane at the top of its iteration; FP32 has it in flight
    // from the previous one
    if constexpr (!kF64) {
      plane_load(T.z0);
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the first plane has landed
    }
    // iterations z0 .. z1-1 have plane k in LDS; the last one (k = z1) only
    // closes the column with plane z1's values read from memory
    for (int k = T.z0; k <= T.z1; ++k) {
      const bool plane = k < T.z1;
      if constexpr (kF64) {
        if (plane) plane_load(k);
      }
      // own column: U^n at k+1 and the z offset's input at k, in flight during
      // the x-y faces (U^n at k+1 is also what the copy of plane k+1 reads next)
      Real un1[5], xs = (Real)0;
      if (in) {
        ld_col(k + 1, un1);
        xs = *at_col(X[2], k);
      }
      Real ak[5] = {0, 0, 0, 0, 0};
      Real uk[5], bk[5];
      if (plane) {
        // plane k complete in LDS for every wave: FP64 has just stored it; FP32's
        // copy was waited for before the barrier that ended the previous
        // iteration (the first plane's before the loop, so it needs this one)
        if (kF64 || k == T.z0) lds_barrier();
        if (in) {
          // this cell's own plane-k values (read before the faces: once the
          // faces are done, a wave may start copying the next plane over them)
          const int ce = eidx(tx + 2, ty + 2), ch = hidx(tx + 1, ty + 1);
#pragma unroll
          for (int v = 0; v < 5; ++v) uk[v] = S.u[v][ce];
          bk[0] = uk[0];
#pragma unroll
          for (int v = 0; v < 4; ++v) bk[1 + v] = S.b[v][ch];
        }
        // every x and y face of the tile once: x faces first, then y faces
#pragma unroll 1
        for (int f = tid; f < NFXP + NFY; f += NT) {
          Real Fo[5];
          if (f < NFXP) {
            const int row = f / EX, col = f % EX;
            if (col <= TX && tile_face<kGen>(g, T, S, 0, row, col, dt, xc, Fo)) {
#pragma unroll
              for (int v = 0; v < 5; ++v) S.fx[v][f] = Fo[v];
            }
          } else {
            const int fy = f - NFXP;
            if (tile_face<kGen>(g, T, S, 1, fy / TX, fy % TX, dt, xc, Fo)) {
#pragma unroll
              for (int v = 0; v < 5; ++v) S.fy[v][fy] = Fo[v];
            }
          }
        }
        lds_barrier();
        if (in) {
          // x faces i+1/2 and i-1/2 of this cell (columns tx+1 and tx of its
          // row) and y faces j+1/2, j-1/2: the last LDS reads of the iteration
          const int fxp = ty * EX + tx + 1, fxm = fxp - 1;
          const int fyp = (ty + 1) * TX + tx, fym = ty * TX + tx;
#pragma unroll
          for (int v = 0; v < 5; ++v) ak[v] = S.fx[v][fxp] - S.fx[v][fxm];
#pragma unroll
          for (int v = 0; v < 5; ++v) ak[v] = ak[v] + (S.fy[v][fyp] - S.fy[v][fym]);
        }
        // the plane buffers are free (the faces are done and read only fx, fy
        // from here): start the next plane, which lands while the z face and the
        // updates below (no LDS) are computed
        if constexpr (!kF64) {
          if (k + 1 < T.z1) plane_load(k + 1);
        }
      } else if (in) {
        ld_col(k, uk);
        ld_base(k, bk);
      }
      if (in) {
        // z face k-1/2 from U^n at k-2 .. k+1, the bases and offsets of k-1, k
        const Real xk = z_offset(bk[0], uk[3], xs, bk[3]);
        Real u4[5][4], Fp[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          u4[v][0] = uq[v][0];
          u4[v][1] = uq[v][1];
          u4[v][2] = uk[v];
          u4[v][3] = un1[v];
        }
        face_flux<kGen>(g, 2, u4, bq, bk, xq, xk, dt, Fp);
        if (k > T.z0) {
          // the update of cell k-1: x/y face sums, then the two z faces
          Real acc[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) acc[v] = aq[v] + (Fp[v] - Fz[v]);
          Real nv[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) nv[v] = bq[v] - (Real)g.inv_h * acc[v];
          if constexpr (kGen) {
            // sources and sinks: the second half step (the generic form only)
            if (F.src)
              source_cell(*at_col(F.src, k - 1), (Real)g.eps_src, (Real)(0.5 * ctrl->dt), nv[0], nv[1],
                          nv[2], nv[3], nv[4]);
          }
          const long long pz = plane0(g, k - 1);
          const uint32_t o = opaque32(oc);
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            *at_plane(Uo[v], pz, o) = nv[v];
            if (!isfinite(nv[v])) bad |= kBadNonFinite;
            tot[v] += (double)nv[v];
          }
          if (kPushX && (i < 2 || i >= g.nx - 2)) {
            // x ghosts (two deep) of the new state
            x_push<2>(g, bc, i, [&](int gi, bool flip, int face) {
              const long long cg = cell(g, gi, j, k - 1);
#pragma unroll
              for (int v = 0; v < 5; ++v) Uo[v][cg] = x_ghost_value(bc, nv[v], v, flip, face, 0.0);
            });
          }
          if ((double)nv[0] < -g.neg_tol) bad |= kBadNegDensity;
          if (!bad) smr = fmax(smr, signal_speed_r(g, nv[0], nv[1], nv[2], nv[3], nv[4]));
        }
        // advance the column by one plane
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          Fz[v] = Fp[v];
          uq[v][0] = uq[v][1];
          uq[v][1] = uk[v];
          bq[v] = bk[v];
          aq[v] = ak[v];
        }
        xq = xk;
      }
      if (plane) {
        // the next plane's LDS copy must have landed before the barrier (vmcnt(0);
        // a workgroup barrier alone does not wait for global -> LDS transfers)
        if constexpr (!kF64) __builtin_amdgcn_s_waitcnt(0x0F70);
        lds_barrier();
      }
    }
  }
  // block epilogue: FP64 totals to a per-block slot, max signal speed, flags
  const int lane = tid % kWave, w = tid / kWave;
#pragma unroll
  for (int v = 0; v < 5; ++v) tot[v] = wave_sum(tot[v]);
  double smax = wave_max((double)smr);
  lds_barrier();
  if (bad) atomicOr(&redb, bad);
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < 5; ++v) red[v][w] = tot[v];
    red[5][w] = smax;
  }
  lds_barrier();
  if (tid == 0) {
    double m = red[5][0];
    for (int q = 1; q < NT / kWave; ++q) m = fmax(m, red[5][q]);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double s = red[v][0];
      for (int q = 1; q < NT / kWave; ++q) s += red[v][q];
      slot[v] = s;
    }
    if (m > 0.0) atomicMax(&ctrl->smax_bits[1 - ctrl->cur], (unsigned long long)__double_as_longlong(m));
    if (redb) atomicOr(&ctrl->status, redb);
  }
}

// ------------------------------------------------------------------ stage launches
// one Lagrangian sweep in the form the grid needs (with or without a potential;
// kVisc fixed by the caller, so that the inviscid kernels are not given the
// viscous form's registers)
template <bool kCorr, bool kVisc, class Sh>
__device__ __forceinline__ void lattice_sweep(PlaneL<Sh>& S, const Fields<Real>& F, const GridDev& g,
                                              const BcDev& bc, const Ctrl* ctrl, const Tile& T) {
  if (g.psi) stage_l_body<kCorr, true, kVisc, false>(S, F, g, bc, ctrl, T);
  else stage_l_body<kCorr, false, kVisc, false>(S, F, g, bc, ctrl, T);
}
template <bool kCorr, class Sh>
__device__ __forceinline__ void lattice_sweep_any(PlaneL<Sh>& S, const Fields<Real>& F, const GridDev& g,
                                                  const BcDev& bc, const Ctrl* ctrl, const Tile& T) {
  if (g.nu > 0.0) lattice_sweep<kCorr, true>(S, F, g, bc, ctrl, T);
  else lattice_sweep<kCorr, false>(S, F, g, bc, ctrl, T);
}

template <bool kVisc, bool kGrav = false>
__global__ void __launch_bounds__(NT) k_stage_p(Fields<Real> F, GridDev g, BcDev bc,
                                                const Ctrl* __restrict__ ctrl, int tz) {
  if (!ctrl->active) return;
  Tile T;
  int id;
  if (!single_tile<kTxL>(g, tz, T, id)) return;
  __shared__ PlaneL<Shape<kTxL>> S;
  if constexpr (kGrav)
    stage_l_body<false, true, kVisc, true>(S, F, g, bc, ctrl, T);  // a potential is always set
  else
    lattice_sweep<false, kVisc>(S, F, g, bc, ctrl, T);
}

template <bool kVisc>
__global__ void __launch_bounds__(NT) k_stage_c(Fields<Real> F, GridDev g, BcDev bc,
                                                   const Ctrl* __restrict__ ctrl, int tz) {
  if (!ctrl->active) return;
  Tile T;
  int id;
  if (!single_tile<kTxL>(g, tz, T, id)) return;
  __shared__ PlaneL<Shape<kTxL>> S;
  lattice_sweep<true, kVisc>(S, F, g, bc, ctrl, T);
}

// Workgroups per CU the register allocation must allow: the default scheme's
// stage E fits 128 registers (four waves per SIMD); the general one keeps two.
constexpr int e_blocks(bool gen) { return gen ? 2 : 4; }

template <bool kGen>
__global__ void __launch_bounds__(NT, e_blocks(kGen)) k_stage_e(Fields<Real> F, GridDev g, BcDev bc, Ctrl* ctrl,
                                                                double* __restrict__ partials, int tz) {
  if (!ctrl->active) return;
  Tile T;
  int id;
  if (!single_tile(g, tz, T, id)) return;
  stage_e_body<kGen>(F, g, bc, ctrl, T, partials + (long long)id * 5);
}

// batched sweeps: workgroup -> (instance, tile) through a host-built map of the
// flattened tile list; the XCD inversion runs over the whole list.  kGen: the
// general form -- for stage E a member uses a non-default scheme, for stages P
// and C a member has a viscosity (each member then takes its own form)
template <int kStage, bool kGen>
__global__ void __launch_bounds__(NT, kStage == 2 ? e_blocks(kGen) : 2)
    k_stage_batch(const Inst<Real>* __restrict__ tab, const int2* __restrict__ map, int ntiles) {
  const int gid = xcd_tile(blockIdx.x, gridDim.x);
  if (gid < 0 || gid >= ntiles) return;
  const int2 w = map[gid];
  const Inst<Real>& I = tab[w.x];
  if (!I.ctrl->active) return;
  Tile T;
  tile_at(I.g, I.tz, w.y, T);
  if constexpr (kStage == 0) {
    __shared__ PlaneL<Shape<TX>> S;
    if constexpr (kGen) lattice_sweep_any<false>(S, I.F, I.g, I.bc, I.ctrl, T);
    else lattice_sweep<false, false>(S, I.F, I.g, I.bc, I.ctrl, T);
  } else if constexpr (kStage == 1) {
    __shared__ PlaneL<Shape<TX>> S;
    if constexpr (kGen) lattice_sweep_any<true>(S, I.F, I.g, I.bc, I.ctrl, T);
    else lattice_sweep<true, false>(S, I.F, I.g, I.bc, I.ctrl, T);
  } else if (!kGen || default_scheme(I.g))
    stage_e_body<false>(I.F, I.g, I.bc, I.ctrl, T, I.partials + (long long)w.y * 5);
  else
    stage_e_body<true>(I.F, I.g, I.bc, I.ctrl, T, I.partials + (long long)w.y * 5);
}

// fixed-order sum of the per-block totals
__global__ void __launch_bounds__(256) k_totals(const double* __restrict__ partials, int nblocks,
                                                double h3, double* __restrict__ out) {
  __shared__ double red[5][256];
  const int t = threadIdx.x;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = t; b < nblocks; b += blockDim.x)
    for (int v = 0; v < 5; ++v) s[v] += partials[(long long)b * 5 + v];
  for (int v = 0; v < 5; ++v) red[v][t] = s[v];
  __syncthreads();
  if (t == 0) {
    for (int v = 0; v < 5; ++v) {
      double a = 0.0;
      for (int q = 0; q < (int)blockDim.x; ++q) a += red[v][q];
      out[v] = a * h3;
    }
  }
}

// z-planes per workgroup: enough workgroups to fill 256 CUs several times over
int pick_tz(const GridDev& g) {
  const long long tiles_xy = (long long)((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY);
  int tz = 32;
  while (tz > 4 && tiles_xy * ((g.nz + tz - 1) / tz) < 2048) tz /= 2;
  return tz;
}

template <int kTX = TX>
int sweep_tiles(const GridDev& g, int tz) {
  constexpr int ty = NT / kTX;
  return ((g.nx + kTX - 1) / kTX) * ((g.ny + ty - 1) / ty) * ((g.nz + tz - 1) / tz);
}

template <int kTX = TX>
int sweep_blocks(const GridDev& g, int tz) {
  return (sweep_tiles<kTX>(g, tz) + kXcd - 1) / kXcd * kXcd;
}

dim3 cell_grid(const GridDev& g) {
  return dim3((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + 3) / 4), (unsigned)min(g.nz, 8));
}

}  // namespace CSPH_TAG

using CSPH_TAG::Real;
using namespace CSPH_TAG;

template <>
int Launch<Real>::tiles(const GridDev& g, int tz) {
  return sweep_tiles(g, tz);
}

template <>
int Launch<Real>::default_tz(const GridDev& g) {
  return pick_tz(g);
}

template <>
long long Launch<Real>::ghosts(const GridDev& g) {
  return ghost_count(g);
}

template <>
hipError_t Launch<Real>::batch_step(const Inst<Real>* tab, const int2* tile_map, const int2* fill_map,
                                    int n, int total_tiles, int fill_blocks, int* flags, bool generic,
                                    bool viscous, hipStream_t s) {
  const unsigned nb = (unsigned)((total_tiles + kXcd - 1) / kXcd * kXcd);
  const unsigned ib = (unsigned)((n + 63) / 64);
  k_begin_batch<<<ib, 64, 0, s>>>(tab, n);
  k_fill_batch<0><<<fill_blocks, 256, 0, s>>>(tab, fill_map, fill_blocks);
  if (viscous)
    k_stage_batch<0, true><<<nb, NT, 0, s>>>(tab, tile_map, total_tiles);
  else
    k_stage_batch<0, false><<<nb, NT, 0, s>>>(tab, tile_map, total_tiles);
  k_fill_batch<1><<<fill_blocks, 256, 0, s>>>(tab, fill_map, fill_blocks);
  if (viscous)
    k_stage_batch<1, true><<<nb, NT, 0, s>>>(tab, tile_map, total_tiles);
  else
    k_stage_batch<1, false><<<nb, NT, 0, s>>>(tab, tile_map, total_tiles);
  k_fill_batch<2><<<fill_blocks, 256, 0, s>>>(tab, fill_map, fill_blocks);
  if (generic)
    k_stage_batch<2, true><<<nb, NT, 0, s>>>(tab, tile_map, total_tiles);
  else
    k_stage_batch<2, false><<<nb, NT, 0, s>>>(tab, tile_map, total_tiles);
  k_end_batch<<<ib, 64, 0, s>>>(tab, n, flags);
  return hipGetLastError();
}

template <>
hipError_t Launch<Real>::fill_psi(const Fields<Real>& F, const GridDev& g, const BcDev& bc,
                                  Ctrl* ctrl, hipStream_t s) {
  FillSet<Real> fs{};
  fs.f[0] = F.psi;
  fs.role[0] = kPsi;
  fs.n = 1;
  const long long n = ghost_count(g);
  k_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(fs, g, bc, ctrl, 0);
  return hipGetLastError();
}

template <>
hipError_t Launch<Real>::fill_state(const Fields<Real>& F, const GridDev& g, const BcDev& bc, int par,
                                    Ctrl* ctrl, hipStream_t s) {
  FillSet<Real> fs{};
  for (int v = 0; v < 5; ++v) {
    fs.f[v] = F.U[par][v];
    fs.role[v] = v;
  }
  fs.n = 5;
  const long long n = ghost_count(g);
  k_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(fs, g, bc, ctrl, 0);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_fill_const(Real* __restrict__ f, Real v, long long n) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (long long)gridDim.x * blockDim.x)
    f[q] = v;
}

template <>
hipError_t Launch<Real>::fill_const(Real* f, double v, long long n, hipStream_t s) {
  const long long blocks = std::min<long long>((n + 255) / 256, 65536);
  k_fill_const<<<(unsigned)blocks, 256, 0, s>>>(f, (Real)v, n);
  return hipGetLastError();
}

template <>
hipError_t Launch<Real>::signal_max(const Fields<Real>& F, const GridDev& g, Ctrl* ctrl,
                                    hipStream_t s) {
  k_signal_max<<<cell_grid(g), dim3(64, 4), 0, s>>>(F, g, ctrl);
  return hipGetLastError();
}

template <>
hipError_t Launch<Real>::step(const Fields<Real>& F, const GridDev& g, const BcDev& bc, Ctrl* ctrl,
                              double* partials, double dt_max, double t_end, const int tz[3],
                              const Grav<Real>* gr, hipStream_t s, hipEvent_t* ev) {
  const long long ng = ghost_count(g);
  const unsigned gb = (unsigned)((ng + 255) / 256);
  // each stage has its own tile depth
  const unsigned nbp = (unsigned)sweep_blocks<kTxL>(g, tz[0]), nbc = (unsigned)sweep_blocks<kTxL>(g, tz[1]),
                 nbe = (unsigned)sweep_blocks(g, tz[2]);
  auto mark = [&](int q) {
    if (ev) (void)hipEventRecord(ev[q], s);
  };
  mark(0);
  if (!F.src) k_begin_fill<<<gb, 256, 0, s>>>(F, g, bc, ctrl, dt_max, t_end);
  if (F.src) {
    k_begin<<<1, 64, 0, s>>>(ctrl, g, dt_max, t_end);
    // sources and sinks: the first half step, then every ghost of U^n
    k_source<<<cell_grid(g), dim3(64, 4), 0, s>>>(F, g, ctrl);
    FillSet<Real> fs{};
    for (int v = 0; v < 5; ++v) {
      fs.f[v] = nullptr;
      fs.role[v] = v;
    }
    fs.n = 5;
    k_fill_u<<<gb, 256, 0, s>>>(F, fs, g, bc, ctrl);
  }
  mark(1);
  if (gr) {
    // the potentials of rho^n and of the predicted density, then their ghosts
    hipError_t e = Poisson<Real>::solve(F, g, ctrl, *gr, s);
    if (e != hipSuccess) return e;
    FillSet<Real> fs{};
    fs.f[0] = F.psi;
    fs.f[1] = gr->psih;
    fs.role[0] = fs.role[1] = kPsi;
    fs.n = 2;
    k_fill<<<gb, 256, 0, s>>>(fs, g, bc, ctrl, 1);
  }
  mark(2);
  if (gr) {
    // self-gravity: the sweep samples psi at r* from the predicted density's potential
    if (g.nu > 0.0) k_stage_p<true, true><<<nbp, NT, 0, s>>>(F, g, bc, ctrl, tz[0]);
    else k_stage_p<false, true><<<nbp, NT, 0, s>>>(F, g, bc, ctrl, tz[0]);
  } else {
    if (g.nu > 0.0) k_stage_p<true><<<nbp, NT, 0, s>>>(F, g, bc, ctrl, tz[0]);
    else k_stage_p<false><<<nbp, NT, 0, s>>>(F, g, bc, ctrl, tz[0]);
  }
  mark(3);
  mark(4);
  k_fill_pred<<<gb, 256, 0, s>>>(F, g, bc, ctrl);
  mark(5);
  if (g.nu > 0.0) k_stage_c<true><<<nbc, NT, 0, s>>>(F, g, bc, ctrl, tz[1]);
  else k_stage_c<false><<<nbc, NT, 0, s>>>(F, g, bc, ctrl, tz[1]);
  mark(6);
  k_fill_corr<<<gb, 256, 0, s>>>(F, g, bc, ctrl);
  mark(7);
  if (default_scheme(g) && !F.src)
    k_stage_e<false><<<nbe, NT, 0, s>>>(F, g, bc, ctrl, partials, tz[2]);
  else
    k_stage_e<true><<<nbe, NT, 0, s>>>(F, g, bc, ctrl, partials, tz[2]);
  mark(8);
  k_end<<<1, 64, 0, s>>>(ctrl);
  mark(9);
  return hipGetLastError();
}

template <>
hipError_t Launch<Real>::totals(const GridDev& g, const double* partials, int nblocks, double* out,
                                hipStream_t s) {
  k_totals<<<1, 256, 0, s>>>(partials, nblocks, g.h3, out);
  return hipGetLastError();
}

template struct Launch<Real>;

}  // namespace csph
