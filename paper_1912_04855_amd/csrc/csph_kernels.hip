// csph_kernels.hip -- HIP kernels of one CSPH-TVD step for gfx950.
//
// This translation unit is compiled twice, with CSPH_REAL = float and with
// CSPH_REAL = double.  The double build is compiled without floating-point
// contraction and evaluates every expression in the same order as the scheme
// is written (arXiv:1912.04855, Sec. 2.2), so it reproduces FP64 reference
// arithmetic up to the order of the final FP64 reductions.  The float build
// keeps the state and most arithmetic in FP32 and promotes to FP64 where
// cancellation matters: the pressure + potential pair sums that carry the
// well-balanced property, the time step and the conservation totals.
//
// Per step (one thread per interior cell in each stage):
//   begin  : dt from the max signal speed of U^n (FP64), CFL rule
//   fill   : ghost cells of U^n
//   stage P: predictor, Eq. (5) with Q of Eq. (7) on the lattice
//   fill   : ghost cells of m*, E*, xi*
//   stage C: corrector, Eq. (6) with Q of Eq. (7) at the displaced particles
//   fill   : ghost cells of m~, E~, xi^{n+1}
//   stage E: reconstruction Eq. (8), face fluxes, update Eq. (4); epilogue:
//            signal-speed max of U^{n+1}, FP64 block totals, error flags
//   end    : swap the state copies
#include <hip/hip_runtime.h>

#include <cmath>

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

constexpr int kWave = 64;

// ------------------------------------------------------------------ indexing
__device__ __forceinline__ long long cell(const GridDev& g, int i, int j, int k) {
  return ((long long)(k + kGhost) * g.sy + (j + kGhost)) * (long long)g.sx + (i + kGhost);
}

// half neighbour set O13 in lexicographic (o_z, o_y, o_x) order; the partner of
// each offset o is -o, and every sum adds the pair's two terms first.
__constant__ int kO13[13][3] = {{1, 0, 0},  {-1, 1, 0}, {0, 1, 0},   {1, 1, 0},  {-1, -1, 1},
                                {0, -1, 1}, {1, -1, 1}, {-1, 0, 1},  {0, 0, 1},  {1, 0, 1},
                                {-1, 1, 1}, {0, 1, 1},  {1, 1, 1}};

// ------------------------------------------------------------------ EOS
// p = (gamma-1)(E - m.u/2), u = m/rho; vacuum (rho <= rho_vac): u = 0; p >= 0.
__device__ __forceinline__ void primitive(const GridDev& g, Real rho, Real mx, Real my, Real mz,
                                          Real E, Real& ux, Real& uy, Real& uz, Real& p) {
  if (rho > (Real)g.rho_vac) {
    ux = mx / rho;
    uy = my / rho;
    uz = mz / rho;
  } else {
    ux = (Real)0;
    uy = (Real)0;
    uz = (Real)0;
  }
  const Real ke = (Real)0.5 * (mx * ux + my * uy + mz * uz);
  const Real pp = (Real)g.gm1 * (E - ke);
  p = pp > (Real)0 ? pp : (Real)0;
}

// ------------------------------------------------------------------ kernel gradient
// M4 cubic spline with support 2h: K(d) = -(kappa/h^2) (g(q)/q) d, q = |d|/h,
// g(q)/q = 3 - 9q/4 (q < 1), 3(2-q)^2/(4q) (1 <= q < 2), 0 beyond.
__device__ __forceinline__ Real g_over_q(Real q) {
  if (q < (Real)1) return (Real)3 - (Real)2.25 * q;
  if (q < (Real)2) {
    const Real t = (Real)2 - q;
    return (Real)0.75 * t * t / q;
  }
  return (Real)0;
}

__device__ __forceinline__ void kgrad(const GridDev& g, Real dx, Real dy, Real dz, Real& Kx,
                                      Real& Ky, Real& Kz) {
  const Real r2 = dx * dx + dy * dy + dz * dz;
  const Real q = sqrt(r2) * (Real)g.inv_h;
  const Real c = (Real)g.kappa_h2 * g_over_q(q);
  Kx = -(c * dx);
  Ky = -(c * dy);
  Kz = -(c * dz);
}

// ------------------------------------------------------------------ TVD slope
__device__ __forceinline__ Real minmod(Real a, Real b) {
  if (a * b <= (Real)0) return (Real)0;
  const Real sg = a > (Real)0 ? (Real)1 : (Real)-1;
  return sg * fmin(fabs(a), fabs(b));
}

// ------------------------------------------------------------------ potential at r*
__device__ __forceinline__ Real lerp(Real a, Real b, Real t) { return a + t * (b - a); }

// trilinear psi at cell centre + (ox, oy, oz), between the cell and its
// neighbours on the side the particle moved to
__device__ __forceinline__ Real psi_at(const GridDev& g, const Real* __restrict__ P, long long c,
                                       Real ox, Real oy, Real oz) {
  const Real fx = ox * (Real)g.inv_h, fy = oy * (Real)g.inv_h, fz = oz * (Real)g.inv_h;
  const long long di = fx >= (Real)0 ? 1 : -1;
  const long long dj = (fy >= (Real)0 ? 1 : -1) * (long long)g.sx;
  const long long dk = (fz >= (Real)0 ? 1 : -1) * g.sxy;
  const Real tx = fabs(fx), ty = fabs(fy), tz = fabs(fz);
  const Real a00 = lerp(P[c], P[c + di], tx);
  const Real a10 = lerp(P[c + dj], P[c + dj + di], tx);
  const Real a01 = lerp(P[c + dk], P[c + dk + di], tx);
  const Real a11 = lerp(P[c + dk + dj], P[c + dk + dj + di], tx);
  const Real b0 = lerp(a00, a10, ty);
  const Real b1 = lerp(a01, a11, ty);
  return lerp(b0, b1, tz);
}

// ------------------------------------------------------------------ reductions
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

// ==================================================================== ghost cells
__device__ __forceinline__ int map_index(int x, int n, int kind) {
  if (kind == kPeriodic) return x < 0 ? x + n : x - n;
  if (kind == kReflect) return x < 0 ? -x - 1 : 2 * n - 1 - x;
  return x < 0 ? 0 : n - 1;  // outflow (and psi at inflow faces)
}

__device__ __forceinline__ Real inflow_value(const BcDev& bc, int face, int role, double dt) {
  if (role <= kE) return (Real)bc.cons[face][role];
  return (Real)(dt * bc.vel[face][role - kXx]);
}

// Ghost cell (i,j,k): the last axis filled (z) decides first, then y, then x,
// which composes the per-face rules applied in x, y, z order.
__global__ void __launch_bounds__(256) k_fill(FillSet<Real> fs, GridDev g, BcDev bc,
                                              const Ctrl* __restrict__ ctrl, int check_active) {
  if (check_active && !ctrl->active) return;
  const long long zone_z = 4LL * g.sx * g.sy;
  const long long zone_y = (long long)g.nz * 4 * g.sx;
  const long long zone_x = (long long)g.nz * g.ny * 4;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (t < zone_z) {
    const int kk = (int)(t / ((long long)g.sx * g.sy));
    const long long r = t - (long long)kk * g.sx * g.sy;
    j = (int)(r / g.sx) - kGhost;
    i = (int)(r % g.sx) - kGhost;
    k = kk < 2 ? kk - 2 : g.nz + (kk - 2);
  } else if (t < zone_z + zone_y) {
    const long long u = t - zone_z;
    k = (int)(u / (4LL * g.sx));
    const long long r = u - (long long)k * 4 * g.sx;
    const int jj = (int)(r / g.sx);
    i = (int)(r % g.sx) - kGhost;
    j = jj < 2 ? jj - 2 : g.ny + (jj - 2);
  } else if (t < zone_z + zone_y + zone_x) {
    const long long u = t - zone_z - zone_y;
    k = (int)(u / (4LL * g.ny));
    const long long r = u - (long long)k * 4 * g.ny;
    j = (int)(r / 4);
    const int ii = (int)(r % 4);
    i = ii < 2 ? ii - 2 : g.nx + (ii - 2);
  } else {
    return;
  }
  const double dt = ctrl->dt;
  const int n[3] = {g.nx, g.ny, g.nz};
  const long long cg = cell(g, i, j, k);
  for (int q = 0; q < fs.n; ++q) {
    const int role = fs.role[q];
    Real* f = fs.f[q];
    int c[3] = {i, j, k};
    Real sign = (Real)1;
    bool done = false;
    Real val = (Real)0;
    for (int ax = 2; ax >= 0; --ax) {
      if (c[ax] >= 0 && c[ax] < n[ax]) continue;
      const int face = 2 * ax + (c[ax] < 0 ? 0 : 1);
      const int kind = bc.kind[face];
      if (kind == kInflow && role != kPsi) {
        val = sign * inflow_value(bc, face, role, dt);
        done = true;
        break;
      }
      c[ax] = map_index(c[ax], n[ax], kind);
      if (kind == kReflect && (role == kMx + ax || role == kXx + ax)) sign = -sign;
    }
    if (!done) {
      const long long cs = cell(g, c[0], c[1], c[2]);
      val = sign * f[cs];
    }
    f[cg] = val;
  }
}

// state fill reads the current copy U[par] (only known on the device)
__global__ void __launch_bounds__(256) k_fill_state(Fields<Real> F, GridDev g, BcDev bc,
                                                    const Ctrl* __restrict__ ctrl) {
  if (!ctrl->active) return;
  const long long zone_z = 4LL * g.sx * g.sy;
  const long long zone_y = (long long)g.nz * 4 * g.sx;
  const long long zone_x = (long long)g.nz * g.ny * 4;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (t < zone_z) {
    const int kk = (int)(t / ((long long)g.sx * g.sy));
    const long long r = t - (long long)kk * g.sx * g.sy;
    j = (int)(r / g.sx) - kGhost;
    i = (int)(r % g.sx) - kGhost;
    k = kk < 2 ? kk - 2 : g.nz + (kk - 2);
  } else if (t < zone_z + zone_y) {
    const long long u = t - zone_z;
    k = (int)(u / (4LL * g.sx));
    const long long r = u - (long long)k * 4 * g.sx;
    const int jj = (int)(r / g.sx);
    i = (int)(r % g.sx) - kGhost;
    j = jj < 2 ? jj - 2 : g.ny + (jj - 2);
  } else if (t < zone_z + zone_y + zone_x) {
    const long long u = t - zone_z - zone_y;
    k = (int)(u / (4LL * g.ny));
    const long long r = u - (long long)k * 4 * g.ny;
    j = (int)(r / 4);
    const int ii = (int)(r % 4);
    i = ii < 2 ? ii - 2 : g.nx + (ii - 2);
  } else {
    return;
  }
  const int par = ctrl->par;
  const int n[3] = {g.nx, g.ny, g.nz};
  const long long cg = cell(g, i, j, k);
  for (int role = 0; role < 5; ++role) {
    Real* f = F.U[par][role];
    int c[3] = {i, j, k};
    Real sign = (Real)1;
    bool done = false;
    Real val = (Real)0;
    for (int ax = 2; ax >= 0; --ax) {
      if (c[ax] >= 0 && c[ax] < n[ax]) continue;
      const int face = 2 * ax + (c[ax] < 0 ? 0 : 1);
      const int kind = bc.kind[face];
      if (kind == kInflow) {
        val = sign * (Real)bc.cons[face][role];
        done = true;
        break;
      }
      c[ax] = map_index(c[ax], n[ax], kind);
      if (kind == kReflect && role == kMx + ax) sign = -sign;
    }
    if (!done) val = sign * f[cell(g, c[0], c[1], c[2])];
    f[cg] = val;
  }
}

long long ghost_count(const GridDev& g) {
  return 4LL * g.sx * g.sy + (long long)g.nz * 4 * g.sx + (long long)g.nz * g.ny * 4;
}

// ==================================================================== time step
// signal-speed max of U[par] over interior non-vacuum cells into smax_bits[cur]
__device__ __forceinline__ double signal_speed(const GridDev& g, Real r, Real mx, Real my, Real mz,
                                               Real E) {
  if (!(r > (Real)g.rho_vac)) return 0.0;
  Real ux, uy, uz, p;
  primitive(g, r, mx, my, mz, E, ux, uy, uz, p);
  const Real cs = sqrt((Real)g.gamma * p / r);
  const Real sp = cs + fabs(ux) + fabs(uy) + fabs(uz);
  return (double)sp;
}

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

__global__ void __launch_bounds__(256) k_signal_max(Fields<Real> F, GridDev g, Ctrl* ctrl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  const int par = ctrl->par;
  double v = 0.0;
  if (i < g.nx && j < g.ny) {
    const long long c = cell(g, i, j, k);
    v = signal_speed(g, F.U[par][0][c], F.U[par][1][c], F.U[par][2][c], F.U[par][3][c],
                     F.U[par][4][c]);
  }
  block_max_to(v, &ctrl->smax_bits[ctrl->cur]);
}

// dt = cfl h / smax, capped by dt_max (> 0) and by the time left to t_end
__global__ void k_begin(Ctrl* ctrl, GridDev g, double dt_max, double t_end) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (ctrl->status || ctrl->done) {
    ctrl->active = 0;
    return;
  }
  const double smax = __longlong_as_double((long long)ctrl->smax_bits[ctrl->cur]);
  double dt;
  if (smax > 0.0) {
    dt = g.cfl_h / smax;
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

__global__ void k_end(Ctrl* ctrl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (!ctrl->active) return;
  ctrl->par = 1 - ctrl->par;
  ctrl->cur = 1 - ctrl->cur;
  ctrl->smax_valid = 1;
  ctrl->active = 0;
}

// ==================================================================== stage P
// Predictor, Eq. (5): m* = m - dt A, E* = E - dt B with Q = -(0, A, B) of Eq. (7)
// on the lattice; xi* = dt (u^n + u*)/2.
__global__ void __launch_bounds__(256) k_stage_p(Fields<Real> F, GridDev g,
                                                 const Ctrl* __restrict__ ctrl) {
  if (!ctrl->active) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const int par = ctrl->par;
  const Real* __restrict__ R = F.U[par][0];
  const Real* __restrict__ MX = F.U[par][1];
  const Real* __restrict__ MY = F.U[par][2];
  const Real* __restrict__ MZ = F.U[par][3];
  const Real* __restrict__ EE = F.U[par][4];
  const Real* __restrict__ PS = F.psi;
  const double dt = ctrl->dt;
  const long long c = cell(g, i, j, k);
  const Real rc = R[c];
  Real uc[3], pc;
  primitive(g, rc, MX[c], MY[c], MZ[c], EE[c], uc[0], uc[1], uc[2], pc);
  const Real fc = sqrt((Real)2 * pc);
  const Real psc = PS[c];
  Acc a[3] = {0.0, 0.0, 0.0}, gp[3] = {0.0, 0.0, 0.0}, be = 0.0;
#pragma unroll
  for (int q = 0; q < 13; ++q) {
    Acc ta[2][3], tg[2][3], te[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int sg = side == 0 ? 1 : -1;
      const int ox = sg * kO13[q][0], oy = sg * kO13[q][1], oz = sg * kO13[q][2];
      const long long jn = c + ox + (long long)oy * g.sx + (long long)oz * g.sxy;
      Real uj[3], pj;
      primitive(g, R[jn], MX[jn], MY[jn], MZ[jn], EE[jn], uj[0], uj[1], uj[2], pj);
      const Real fj = sqrt((Real)2 * pj);
      const Real Kx = (Real)(sg * g.klat[q][0]);
      const Real Ky = (Real)(sg * g.klat[q][1]);
      const Real Kz = (Real)(sg * g.klat[q][2]);
      const Acc ff = (Acc)fc * (Acc)fj;
      const Acc dpsi = (Acc)PS[jn] - (Acc)psc;
      const Acc sp = ff + (Acc)rc * dpsi;
      const Real ub = (Real)0.5 * ((uc[0] + uj[0]) * Kx + (uc[1] + uj[1]) * Ky + (uc[2] + uj[2]) * Kz);
      ta[side][0] = sp * (Acc)Kx;
      ta[side][1] = sp * (Acc)Ky;
      ta[side][2] = sp * (Acc)Kz;
      tg[side][0] = dpsi * (Acc)Kx;
      tg[side][1] = dpsi * (Acc)Ky;
      tg[side][2] = dpsi * (Acc)Kz;
      te[side] = ff * (Acc)ub;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      a[d] = a[d] + (ta[0][d] + ta[1][d]);
      gp[d] = gp[d] + (tg[0][d] + tg[1][d]);
    }
    be = be + (te[0] + te[1]);
  }
  const Acc B = be + (Acc)rc * ((Acc)uc[0] * gp[0] + (Acc)uc[1] * gp[1] + (Acc)uc[2] * gp[2]);
  const Real m0[3] = {MX[c], MY[c], MZ[c]};
  Real ms[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) ms[d] = (Real)((Acc)m0[d] - dt * a[d]);
  const Real Es = (Real)((Acc)EE[c] - dt * B);
  F.ms[0][c] = ms[0];
  F.ms[1][c] = ms[1];
  F.ms[2][c] = ms[2];
  F.ms[3][c] = Es;
  Real us[3], ps;
  primitive(g, rc, ms[0], ms[1], ms[2], Es, us[0], us[1], us[2], ps);
  const Real hdt = (Real)(0.5 * dt);
#pragma unroll
  for (int d = 0; d < 3; ++d) F.xs[d][c] = hdt * (uc[d] + us[d]);
}

// ==================================================================== stage C
// Corrector, Eq. (6): m~ = (m + m*)/2 - (dt/2) A*, E~ likewise, with Q(U*, r*)
// evaluated at the displaced particles r* = x + xi* (kernel gradients of the
// displaced pairs, psi interpolated at r*); xi = xi*/2 + dt (u^n + u~)/4.
__global__ void __launch_bounds__(256) k_stage_c(Fields<Real> F, GridDev g,
                                                 const Ctrl* __restrict__ ctrl) {
  if (!ctrl->active) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const int par = ctrl->par;
  const Real* __restrict__ R = F.U[par][0];
  const Real* __restrict__ MSX = F.ms[0];
  const Real* __restrict__ MSY = F.ms[1];
  const Real* __restrict__ MSZ = F.ms[2];
  const Real* __restrict__ ES = F.ms[3];
  const Real* __restrict__ XX = F.xs[0];
  const Real* __restrict__ XY = F.xs[1];
  const Real* __restrict__ XZ = F.xs[2];
  const Real* __restrict__ PS = F.psi;
  const double dt = ctrl->dt;
  const Real h = (Real)g.h;
  const long long c = cell(g, i, j, k);
  const Real rc = R[c];
  Real uc[3], pc;
  primitive(g, rc, MSX[c], MSY[c], MSZ[c], ES[c], uc[0], uc[1], uc[2], pc);
  const Real fc = sqrt((Real)2 * pc);
  const Real xc[3] = {XX[c], XY[c], XZ[c]};
  const Real psc = psi_at(g, PS, c, xc[0], xc[1], xc[2]);
  Acc a[3] = {0.0, 0.0, 0.0}, gp[3] = {0.0, 0.0, 0.0}, be = 0.0;
#pragma unroll 1
  for (int q = 0; q < 13; ++q) {
    Acc ta[2][3], tg[2][3], te[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int sg = side == 0 ? 1 : -1;
      const int ox = sg * kO13[q][0], oy = sg * kO13[q][1], oz = sg * kO13[q][2];
      const long long jn = c + ox + (long long)oy * g.sx + (long long)oz * g.sxy;
      Real uj[3], pj;
      primitive(g, R[jn], MSX[jn], MSY[jn], MSZ[jn], ES[jn], uj[0], uj[1], uj[2], pj);
      const Real fj = sqrt((Real)2 * pj);
      const Real xj[3] = {XX[jn], XY[jn], XZ[jn]};
      const Real psj = psi_at(g, PS, jn, xj[0], xj[1], xj[2]);
      const Real dx = (Real)(-ox) * h + (xc[0] - xj[0]);
      const Real dy = (Real)(-oy) * h + (xc[1] - xj[1]);
      const Real dz = (Real)(-oz) * h + (xc[2] - xj[2]);
      Real Kx, Ky, Kz;
      kgrad(g, dx, dy, dz, Kx, Ky, Kz);
      const Acc ff = (Acc)fc * (Acc)fj;
      const Acc dpsi = (Acc)psj - (Acc)psc;
      const Acc sp = ff + (Acc)rc * dpsi;
      const Real ub = (Real)0.5 * ((uc[0] + uj[0]) * Kx + (uc[1] + uj[1]) * Ky + (uc[2] + uj[2]) * Kz);
      ta[side][0] = sp * (Acc)Kx;
      ta[side][1] = sp * (Acc)Ky;
      ta[side][2] = sp * (Acc)Kz;
      tg[side][0] = dpsi * (Acc)Kx;
      tg[side][1] = dpsi * (Acc)Ky;
      tg[side][2] = dpsi * (Acc)Kz;
      te[side] = ff * (Acc)ub;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      a[d] = a[d] + (ta[0][d] + ta[1][d]);
      gp[d] = gp[d] + (tg[0][d] + tg[1][d]);
    }
    be = be + (te[0] + te[1]);
  }
  const Acc B = be + (Acc)rc * ((Acc)uc[0] * gp[0] + (Acc)uc[1] * gp[1] + (Acc)uc[2] * gp[2]);
  // U^n at the cell and its velocity
  const Real m0[3] = {F.U[par][1][c], F.U[par][2][c], F.U[par][3][c]};
  const Real E0 = F.U[par][4][c];
  Real un[3], pn;
  primitive(g, rc, m0[0], m0[1], m0[2], E0, un[0], un[1], un[2], pn);
  const Real msc[3] = {MSX[c], MSY[c], MSZ[c]};
  const Acc hdt = 0.5 * dt;
  Real mt[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) mt[d] = (Real)((Acc)((Real)0.5 * (m0[d] + msc[d])) - hdt * a[d]);
  const Real Et = (Real)((Acc)((Real)0.5 * (E0 + ES[c])) - hdt * B);
  F.mt[0][c] = mt[0];
  F.mt[1][c] = mt[1];
  F.mt[2][c] = mt[2];
  F.mt[3][c] = Et;
  Real ut[3], pt;
  primitive(g, rc, mt[0], mt[1], mt[2], Et, ut[0], ut[1], ut[2], pt);
  const Real qdt = (Real)(0.25 * dt);
#pragma unroll
  for (int d = 0; d < 3; ++d) F.xt[d][c] = (Real)0.5 * xc[d] + qdt * (un[d] + ut[d]);
}

// ==================================================================== stage E
// Rusanov damping of the face velocity jump (normal weight 1, transverse 1/2),
// acoustic speed a = max(|u_n| + c) of the two reconstructed states.
__device__ __forceinline__ void acoustic_dissipation(const GridDev& g, int axis, const Real L[5],
                                                     const Real Rr[5], Real D[5]) {
  Real uL[3], uR[3], pL, pR;
  primitive(g, L[0], L[1], L[2], L[3], L[4], uL[0], uL[1], uL[2], pL);
  primitive(g, Rr[0], Rr[1], Rr[2], Rr[3], Rr[4], uR[0], uR[1], uR[2], pR);
  const Real cL = L[0] > (Real)g.rho_vac ? sqrt((Real)g.gamma * pL / L[0]) : (Real)0;
  const Real cR = Rr[0] > (Real)g.rho_vac ? sqrt((Real)g.gamma * pR / Rr[0]) : (Real)0;
  const Real a = fmax(fabs(uL[axis]) + cL, fabs(uR[axis]) + cR);
  const Real kk = (Real)-0.5 * a * fmin(L[0], Rr[0]);
  const Real kt = (Real)0.5 * kk;
  D[0] = (Real)0;
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) D[1 + cc] = (cc == axis ? kk : kt) * (uR[cc] - uL[cc]);
  D[4] = (Real)0.5 * ((uL[0] + uR[0]) * D[1] + (uL[1] + uR[1]) * D[2] + (uL[2] + uR[2]) * D[3]);
}

// swept content of face (cL | cL + st) along axis d, all five components
__device__ __forceinline__ void face_flux(const GridDev& g, const Real* const* Un,
                                          const Real* const* Ut, const Real* __restrict__ xi,
                                          long long cL, long long st, int axis, Real dt,
                                          Real Fout[5]) {
  const long long cR = cL + st;
  const Real xL = xi[cL], xR = xi[cR];
  const Real nuL = xL * (Real)g.inv_h, nuR = xR * (Real)g.inv_h;
  Real UL[5], UR[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const Real* U = Un[v];
    const Real sL = minmod(U[cL + st] - U[cL], U[cL] - U[cL - st]);
    const Real sR = minmod(U[cR + st] - U[cR], U[cR] - U[cR - st]);
    const Real BL = Ut[v][cL], BR = Ut[v][cR];
    UL[v] = BL + (Real)0.5 * ((Real)1 - nuL) * sL;
    UR[v] = BR - (Real)0.5 * ((Real)1 + nuR) * sR;
    Fout[v] = fmax(xL, (Real)0) * UL[v] + fmin(xR, (Real)0) * UR[v];
  }
  Real D[5];
  acoustic_dissipation(g, axis, UL, UR, D);
#pragma unroll
  for (int v = 1; v < 5; ++v) Fout[v] = Fout[v] + dt * D[v];
}

__global__ void __launch_bounds__(256) k_stage_e(Fields<Real> F, GridDev g, Ctrl* ctrl,
                                                 double* __restrict__ partials) {
  if (!ctrl->active) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  const int par = ctrl->par;
  const Real dt = (Real)ctrl->dt;
  const bool in = i < g.nx && j < g.ny;
  double tot[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double smax = 0.0;
  int bad = 0;
  if (in) {
    const long long c = cell(g, i, j, k);
    const Real* Un[5] = {F.U[par][0], F.U[par][1], F.U[par][2], F.U[par][3], F.U[par][4]};
    const Real* Ut[5] = {F.U[par][0], F.mt[0], F.mt[1], F.mt[2], F.mt[3]};
    const long long stride[3] = {1, (long long)g.sx, g.sxy};
    Real acc[5] = {(Real)0, (Real)0, (Real)0, (Real)0, (Real)0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      Real Fp[5], Fm[5];
      face_flux(g, Un, Ut, F.xt[d], c, stride[d], d, dt, Fp);
      face_flux(g, Un, Ut, F.xt[d], c - stride[d], stride[d], d, dt, Fm);
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[v] = acc[v] + (Fp[v] - Fm[v]);
    }
    Real nv[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) nv[v] = Ut[v][c] - (Real)g.inv_h * acc[v];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      F.U[1 - par][v][c] = nv[v];
      if (!isfinite(nv[v])) bad |= kBadNonFinite;
      tot[v] = (double)nv[v];
    }
    if ((double)nv[0] < -g.neg_tol) bad |= kBadNegDensity;
    if (!bad) smax = signal_speed(g, nv[0], nv[1], nv[2], nv[3], nv[4]);
  }
  // block epilogue: FP64 totals to a per-block slot, max signal speed, flags
  __shared__ double red[5][16];
  __shared__ double redm[16];
  __shared__ int redb;
  const int flat = threadIdx.x + blockDim.x * threadIdx.y;
  const int nthreads = blockDim.x * blockDim.y;
  const int nw = (nthreads + kWave - 1) / kWave;
  const int lane = flat % kWave, w = flat / kWave;
  if (flat == 0) redb = 0;
#pragma unroll
  for (int v = 0; v < 5; ++v) tot[v] = wave_sum(tot[v]);
  smax = wave_max(smax);
  __syncthreads();
  if (bad) atomicOr(&redb, bad);
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < 5; ++v) red[v][w] = tot[v];
    redm[w] = smax;
  }
  __syncthreads();
  if (flat == 0) {
    const long long blk = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    double m = redm[0];
    for (int q = 1; q < nw; ++q) m = fmax(m, redm[q]);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double s = red[v][0];
      for (int q = 1; q < nw; ++q) s += red[v][q];
      partials[blk * 5 + v] = s;
    }
    if (m > 0.0) atomicMax(&ctrl->smax_bits[1 - ctrl->cur], (unsigned long long)__double_as_longlong(m));
    if (redb) atomicOr(&ctrl->status, redb);
  }
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

constexpr int kBx = 64, kBy = 4;

dim3 cell_grid(const GridDev& g) {
  return dim3((unsigned)((g.nx + kBx - 1) / kBx), (unsigned)((g.ny + kBy - 1) / kBy), (unsigned)g.nz);
}

}  // namespace CSPH_TAG

using CSPH_TAG::Real;
using namespace CSPH_TAG;

template <>
int Launch<Real>::stage_e_blocks(const GridDev& g) {
  const dim3 gr = cell_grid(g);
  return (int)(gr.x * gr.y * gr.z);
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
hipError_t Launch<Real>::fill_state(const Fields<Real>& F, const GridDev& g, const BcDev& bc,
                                    Ctrl* ctrl, hipStream_t s) {
  const long long n = ghost_count(g);
  k_fill_state<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(F, g, bc, ctrl);
  return hipGetLastError();
}

template <>
hipError_t Launch<Real>::signal_max(const Fields<Real>& F, const GridDev& g, Ctrl* ctrl,
                                    hipStream_t s) {
  k_signal_max<<<cell_grid(g), dim3(kBx, kBy), 0, s>>>(F, g, ctrl);
  return hipGetLastError();
}

template <>
hipError_t Launch<Real>::step(const Fields<Real>& F, const GridDev& g, const BcDev& bc, Ctrl* ctrl,
                              double* partials, double dt_max, double t_end, hipStream_t s) {
  const long long ng = ghost_count(g);
  const unsigned gb = (unsigned)((ng + 255) / 256);
  const dim3 gr = cell_grid(g), bl(kBx, kBy);
  k_begin<<<1, 64, 0, s>>>(ctrl, g, dt_max, t_end);
  k_fill_state<<<gb, 256, 0, s>>>(F, g, bc, ctrl);
  k_stage_p<<<gr, bl, 0, s>>>(F, g, ctrl);
  FillSet<Real> fs{};
  for (int q = 0; q < 4; ++q) {
    fs.f[q] = F.ms[q];
    fs.role[q] = kMx + q;
  }
  for (int q = 0; q < 3; ++q) {
    fs.f[4 + q] = F.xs[q];
    fs.role[4 + q] = kXx + q;
  }
  fs.n = 7;
  k_fill<<<gb, 256, 0, s>>>(fs, g, bc, ctrl, 1);
  k_stage_c<<<gr, bl, 0, s>>>(F, g, ctrl);
  for (int q = 0; q < 4; ++q) fs.f[q] = F.mt[q];
  for (int q = 0; q < 3; ++q) fs.f[4 + q] = F.xt[q];
  k_fill<<<gb, 256, 0, s>>>(fs, g, bc, ctrl, 1);
  k_stage_e<<<gr, bl, 0, s>>>(F, g, ctrl, partials);
  k_end<<<1, 64, 0, s>>>(ctrl);
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
