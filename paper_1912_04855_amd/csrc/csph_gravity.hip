// csph_gravity.hip -- the Poisson solve of the gas's self-gravity for gfx950.
//
// The self-gravity extension (arXiv:1912.04855, Sec. 4) on a periodic box: the
// gas's potential solves the 7-point discrete Poisson equation
//   L7[psi] = 4 pi G (rho - mean rho),
// which the discrete Fourier transform diagonalises with eigenvalues
//   lambda(k) = sum_d (2 cos(2 pi k_d / n_d) - 2) / h^2.
// Each step needs two potentials: that of rho^n (the predictor, Eq. (5)) and
// that of the density the continuity equation predicts for t^{n+1},
//   rho^ = rho^n - dt sum_d (m_d,i+1 - m_d,i-1) / (2h)
// (the corrector, Eq. (6), evaluates Q at the end of the step).  Both are real
// and the Green's function 4 pi G / lambda is real and even, so one complex
// transform carries both: rho^n in the real part, rho^ in the imaginary part,
// and after the multiply and the inverse transform the real part is the
// potential of rho^n and the imaginary part that of rho^.
//
// This translation unit is compiled twice (CSPH_REAL = float and double).  One
// solve is five launches over a complex work array [nz][ny][nx] (x fastest):
//   x pass, forward : forms rho^n and rho^ from U^n (constant rho_ref taken off,
//                     which the k = 0 mode discards anyway: it keeps the FP32
//                     transform of a near-uniform density well conditioned)
//   y pass, forward
//   z pass          : forward, times 4 pi G / (lambda N), inverse
//   y pass, inverse
//   x pass, inverse : psi = psi_ext + Re, psi^ = psi_ext + Im, interior cells
// Each launch owns W whole lines of one axis: it loads them into LDS (element e
// of line w at e (W + 1) + w, so the walk along lines and the walk across them
// are both free of bank conflicts), transforms them there and writes them back.
// Power-of-two lengths use in-place radix-2 FFTs: decimation in time (input in
// bit-reversed order, output natural) in the x and y passes; in the z pass
// decimation in frequency forward (natural in, bit-reversed out), the multiply
// in that order, and decimation in time back, so the z pass permutes nothing.
// Other lengths use a direct DFT (O(n^2) per line: correct for any length, meant
// for small grids).  Lines of the y and z passes are W
// neighbouring x columns, so each element row of the tile is one contiguous
// run of W complex values in memory.
//
// An isolated box (no periodic face: gas in vacuum) takes the free-space
// potential of its cells instead; the same five passes compute it as a
// convolution over the box zero-padded to power-of-two lengths m_d >= 2 n_d,
// with a tabulated Green's function in place of 4 pi G / lambda and no
// constant taken off the density.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "csph_internal.h"

#ifndef CSPH_REAL
#error "CSPH_REAL must be float or double"
#endif

#if CSPH_IS_DOUBLE
#define CSPH_GTAG g64
#else
#define CSPH_GTAG g32
#endif

namespace csph {
namespace CSPH_GTAG {

using Real = CSPH_REAL;
constexpr size_t kLdsMax = 65536;  // dynamic LDS of one workgroup
using Real2 = typename std::conditional<std::is_same<Real, double>::value, double2, float2>::type;
constexpr int NT = 256;

__device__ __forceinline__ long long cell(const GridDev& g, int i, int j, int k) {
  return ((long long)(k + kGhost) * g.sy + (j + kGhost)) * (long long)g.sx + (i + kGhost);
}

__device__ __forceinline__ int bit_reverse(int e, int log2n) {
  return (int)(__builtin_bitreverse32((unsigned)e) >> (32 - log2n));
}

// x / d and x mod d for a runtime divisor: a shift and a mask when d is a
// power of two (the tile loops' index arithmetic), else a division
struct DivMod {
  int d, sh;
  __device__ __forceinline__ void operator()(int x, int& q, int& r) const {
    if (sh >= 0) {
      q = x >> sh;
      r = x & (d - 1);
    } else {
      q = x / d;
      r = x - q * d;
    }
  }
};
__device__ __forceinline__ DivMod divmod_by(int d) {
  return DivMod{d, (d & (d - 1)) == 0 ? __builtin_ctz((unsigned)d) : -1};
}

// which pass: the axis of the lines and what the loads and stores do
enum Pass : int { kXFwd = 0, kYFwd = 1, kZ = 2, kYInv = 3, kXInv = 4 };

// The work array is [nz][my][mx] (m the transform lengths; m = n on a periodic
// box).  On an isolated box the density occupies the corner i < nx, j < ny,
// k < nz of the zero-padded box: the x passes transform only the ny nz lines
// that hold data; the y pass loads ny elements of its lines and the z pass nz,
// the rest of each line being zero; the z pass keeps only k < nz of its result,
// the y inverse only j < ny, the x inverse only i < nx.
struct Geom {
  long long base;  // y and z passes: work-array index of element 0 of line 0
  long long es;    // y and z passes: stride between the elements of a line
  int n;           // transform length
  int nin, nout;   // elements loaded (the rest zero) and stored
  int nl;          // lines of this workgroup (<= W; fewer at a ragged edge)
  int axis;
  int j, k;        // x pass: first line's (j, k); y pass: k; z pass: j
  int i0;          // y and z passes: x of line 0
};

// Workgroups go to the 8 XCDs in turn (block b to XCD b mod 8), each XCD with
// its own L2.  The y and z passes' neighbouring tiles share 128-byte lines (a
// tile row is W complex values), so give each XCD a contiguous range of tiles:
// block b takes tile (b mod 8) (nb / 8) + b / 8, the ragged last nb mod 8
// blocks keep their own index.  A permutation of [0, nb).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  constexpr int kXcd = 8;
  const int per = nb / kXcd;
  return b < per * kXcd ? (b % kXcd) * per + b / kXcd : b;
}

__device__ __forceinline__ Geom geom(const GridDev& g, const Grav<Real>& gr, int pass, int W) {
  Geom q{};
  const int b = (pass == kXFwd || pass == kXInv) ? (int)blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
  const int mx = gr.m[0], my = gr.m[1];
  if (pass == kXFwd || pass == kXInv) {
    const int lines = g.ny * g.nz;
    const int l0 = b * W;
    q.axis = 0;
    q.n = mx;
    q.nin = pass == kXFwd ? g.nx : mx;
    q.nout = pass == kXFwd ? mx : g.nx;
    q.nl = min(W, lines - l0);
    q.j = l0 % g.ny;
    q.k = l0 / g.ny;
    q.i0 = 0;
  } else {
    const int tiles_x = (mx + W - 1) / W;
    const int tx = b % tiles_x, other = b / tiles_x;
    q.i0 = tx * W;
    q.nl = min(W, mx - q.i0);
    if (pass == kZ) {
      q.axis = 2;
      q.n = gr.m[2];
      q.nin = q.nout = g.nz;
      q.j = other;
      q.base = (long long)other * mx + q.i0;
      q.es = (long long)mx * my;
    } else {
      q.axis = 1;
      q.n = my;
      q.nin = pass == kYFwd ? g.ny : my;
      q.nout = pass == kYFwd ? my : g.ny;
      q.k = other;
      q.base = (long long)other * mx * my + q.i0;
      q.es = mx;
    }
  }
  return q;
}

// the Green's function at frequency (i, j, kz): periodic box 4 pi G / (lambda
// N) (0 for the mean), isolated box G times the tabulated transform
__device__ __forceinline__ Real green_at(const Grav<Real>& gr, int i, int j, int kz) {
  if (gr.iso) {
    const int hx = gr.m[0] >> 1, hy = gr.m[1] >> 1, hz = gr.m[2] >> 1;
    const int a = i <= hx ? i : gr.m[0] - i, b = j <= hy ? j : gr.m[1] - j,
              c = kz <= hz ? kz : gr.m[2] - kz;
    return (Real)gr.fpg_n * gr.khat[((long long)c * (hy + 1) + b) * (hx + 1) + a];
  }
  if ((i | j | kz) == 0) return 0;
  const double lam = gr.lam[0][i] + gr.lam[1][j] + gr.lam[2][kz];
  return (Real)(gr.fpg_n / lam);
}

// The tile holds W lines, element e of line w at e * P + w (P = W + 1).
// tw[k] = (cos, sin) of 2 pi k / n; sg is the sign of the exponent (-1 forward,
// +1 inverse).

// radix-2 decimation in time, in place: bit-reversed input, natural output
__device__ __forceinline__ void fft_dit(Real* re, Real* im, int n, int W, const Real* __restrict__ tw,
                                        Real sg) {
  const int P = W + 1;
  for (int half = 1; half < n; half <<= 1) {
    const int tstride = n / (2 * half);
    for (int q = threadIdx.x; q < (n / 2) * W; q += NT) {
      const int w = q % W, b = q / W;
      const int pos = b & (half - 1);
      const int i1 = 2 * (b - pos) + pos, i2 = i1 + half;
      const Real cr = tw[2 * pos * tstride], ci = sg * tw[2 * pos * tstride + 1];
      const int a1 = i1 * P + w, a2 = i2 * P + w;
      const Real br = re[a2], bi = im[a2];
      const Real tr = cr * br - ci * bi, ti = cr * bi + ci * br;
      const Real ar = re[a1], ai = im[a1];
      re[a2] = ar - tr;
      im[a2] = ai - ti;
      re[a1] = ar + tr;
      im[a1] = ai + ti;
    }
    __syncthreads();
  }
}

// radix-2 decimation in frequency, in place: natural input, bit-reversed output
__device__ __forceinline__ void fft_dif(Real* re, Real* im, int n, int W, const Real* __restrict__ tw,
                                        Real sg) {
  const int P = W + 1;
  for (int half = n / 2; half >= 1; half >>= 1) {
    const int tstride = n / (2 * half);
    for (int q = threadIdx.x; q < (n / 2) * W; q += NT) {
      const int w = q % W, b = q / W;
      const int pos = b & (half - 1);
      const int i1 = 2 * (b - pos) + pos, i2 = i1 + half;
      const Real cr = tw[2 * pos * tstride], ci = sg * tw[2 * pos * tstride + 1];
      const int a1 = i1 * P + w, a2 = i2 * P + w;
      const Real ar = re[a1], ai = im[a1], br = re[a2], bi = im[a2];
      const Real dr = ar - br, di = ai - bi;
      re[a1] = ar + br;
      im[a1] = ai + bi;
      re[a2] = cr * dr - ci * di;
      im[a2] = cr * di + ci * dr;
    }
    __syncthreads();
  }
}

// direct DFT of any length, through the scratch tile (xr, xi), natural order
__device__ __forceinline__ void dft_direct(Real* re, Real* im, Real* xr, Real* xi, int n, int W,
                                           const Real* __restrict__ tw, Real sg) {
  const int P = W + 1;
  for (int q = threadIdx.x; q < n * W; q += NT) {
    const int w = q % W, k = q / W;
    Real sr = 0, si = 0;
    int idx = 0;  // (j k) mod n
    for (int j = 0; j < n; ++j) {
      const Real cr = tw[2 * idx], ci = sg * tw[2 * idx + 1];
      const Real vr = re[j * P + w], vi = im[j * P + w];
      sr += vr * cr - vi * ci;
      si += vr * ci + vi * cr;
      idx += k;
      if (idx >= n) idx -= n;
    }
    xr[k * P + w] = sr;
    xi[k * P + w] = si;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < n * W; q += NT) {
    const int w = q % W, k = q / W;
    re[k * P + w] = xr[k * P + w];
    im[k * P + w] = xi[k * P + w];
  }
  __syncthreads();
}

// ---------------------------------------------------------------- register FFT
// Power-of-two lines from kEl to NT kEl long: Stockham passes of radix R <= kEl
// (kEl, then the remainder), each thread holding kEl values of one line in
// registers: T = n / kEl threads per line, each doing kEl / R butterflies of a
// pass.  A pass reads its butterflies' inputs j + r n/R from the LDS tile,
// multiplies by exp(sg 2 pi i (j mod Ns) r / (Ns R)) (Ns: the product of the
// earlier radices), takes the R-point DFT in registers and writes the outputs
// to (j - j mod Ns) R + (j mod Ns) + r Ns: input and output in natural order,
// log_kEl(n) passes with two barriers each instead of log2(n) LDS stages.
constexpr int kEl = 8;

// cos and sin of 2 pi k / 16 (any integer k)
__host__ __device__ constexpr double cos16_0to8(int k) {
  return k == 0 ? 1.0 : k == 1 ? 0.92387953251128674 : k == 2 ? 0.70710678118654752
       : k == 3 ? 0.38268343236508977 : k == 4 ? 0.0 : k == 5 ? -0.38268343236508977
       : k == 6 ? -0.70710678118654752 : k == 7 ? -0.92387953251128674 : -1.0;
}
__host__ __device__ constexpr double cos16(int k) {
  return cos16_0to8((k & 15) <= 8 ? (k & 15) : 16 - (k & 15));
}
__host__ __device__ constexpr double sin16(int k) { return cos16(k + 12); }  // sin x = cos(x - pi/2)

__host__ __device__ constexpr int brev(int r, int bits) {
  return bits == 0 ? 0 : ((r & 1) << (bits - 1)) | brev(r >> 1, bits - 1);
}

// R-point DFT of (vr, vi) in registers, exponent sign kSg, natural order out
template <int R, int kSg>
__device__ __forceinline__ void dft_reg(Real (&vr)[R], Real (&vi)[R]) {
  constexpr int B = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
  Real ur[R], ui[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    ur[brev(r, B)] = vr[r];
    ui[brev(r, B)] = vi[r];
  }
#pragma unroll
  for (int half = 1; half < R; half *= 2) {
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const int pos = k % half, i1 = (k / half) * 2 * half + pos, i2 = i1 + half;
      const int widx = pos * (16 / (2 * half));  // W_{2 half}^pos = W_16^widx
      Real tr, ti;
      if (widx == 0) {
        tr = ur[i2];
        ti = ui[i2];
      } else if (widx == 4) {  // kSg i
        tr = (Real)(-kSg) * ui[i2];
        ti = (Real)kSg * ur[i2];
      } else {
        const Real c = (Real)cos16(widx), sn = (Real)(kSg * sin16(widx));
        tr = c * ur[i2] - sn * ui[i2];
        ti = c * ui[i2] + sn * ur[i2];
      }
      ur[i2] = ur[i1] - tr;
      ui[i2] = ui[i1] - ti;
      ur[i1] = ur[i1] + tr;
      ui[i1] = ui[i1] + ti;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    vr[r] = ur[r];
    vi[r] = ui[r];
  }
}

// one Stockham pass of radix R on the tile (line w, thread tl of the line)
template <int R, int kSg>
__device__ __forceinline__ void stockham_pass(Real* re, Real* im, int n, int P, int Ns, int w, int tl,
                                              int T, bool active, const Real* __restrict__ tw) {
  constexpr int kU = kEl / R;
  Real vr[kU][R], vi[kU][R];
  const int nR = n / R;
  if (active) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int j = tl + u * T;
      const int jm = j & (Ns - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = j + r * nR;
        vr[u][r] = re[e * P + w];
        vi[u][r] = im[e * P + w];
      }
      if (Ns > 1) {
        const int step = jm * (n / (Ns * R));
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const int k = step * r;
          const Real c = tw[2 * k], sn = (Real)kSg * tw[2 * k + 1];
          const Real xr = vr[u][r], xi = vi[u][r];
          vr[u][r] = c * xr - sn * xi;
          vi[u][r] = c * xi + sn * xr;
        }
      }
      dft_reg<R, kSg>(vr[u], vi[u]);
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int j = tl + u * T;
      const int jm = j & (Ns - 1);
      const int base = (j - jm) * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = base + r * Ns;
        re[e * P + w] = vr[u][r];
        im[e * P + w] = vi[u][r];
      }
    }
  }
  __syncthreads();
}

// the whole transform of the tile's W lines (W a power of two, W T <= NT)
template <int kSg>
__device__ __forceinline__ void stockham(Real* re, Real* im, int n, int W, const Real* __restrict__ tw) {
  const int P = W + 1;
  const int T = n / kEl;
  const int t = threadIdx.x;
  const int w = t & (W - 1), tl = t >> __builtin_ctz((unsigned)W);
  const bool active = tl < T;
  int Ns = 1;
  for (int m = n; m > 1;) {
    const int R = m > kEl ? kEl : m;
    if (R == 2) {
      stockham_pass<2, kSg>(re, im, n, P, Ns, w, tl, T, active, tw);
    } else if (R == 4) {
      if constexpr (kEl >= 4) stockham_pass<4, kSg>(re, im, n, P, Ns, w, tl, T, active, tw);
    } else if (R == 8) {
      if constexpr (kEl >= 8) stockham_pass<8, kSg>(re, im, n, P, Ns, w, tl, T, active, tw);
    } else {
      if constexpr (kEl >= 16) stockham_pass<16, kSg>(re, im, n, P, Ns, w, tl, T, active, tw);
    }
    Ns *= R;
    m /= R;
  }
}

// The same passes with the line length, the tile width and each pass's stride
// known at compile time, so that every LDS offset of a pass is a constant from
// one base: the register FFT for the lengths the grids use most.  The sequence
// of radices and the arithmetic are those of stockham(), step for step.
template <int R, int kSg, int kN, int kW, int kNs>
__device__ __forceinline__ void stockham_pass_ct(Real* re, Real* im, int w, int tl, bool active,
                                                 const Real* __restrict__ tw) {
  constexpr int kT = kN / kEl, kP = kW + 1, kU = kEl / R, kNR = kN / R;
  Real vr[kU][R], vi[kU][R];
  if (active) {
    const int b0 = tl * kP + w;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        vr[u][r] = re[b0 + (u * kT + r * kNR) * kP];
        vi[u][r] = im[b0 + (u * kT + r * kNR) * kP];
      }
      if constexpr (kNs > 1) {
        const int jm = (tl + u * kT) & (kNs - 1);
        const int step = jm * (kN / (kNs * R));
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const int k = step * r;
          const Real c = tw[2 * k], sn = (Real)kSg * tw[2 * k + 1];
          const Real xr = vr[u][r], xi = vi[u][r];
          vr[u][r] = c * xr - sn * xi;
          vi[u][r] = c * xi + sn * xr;
        }
      }
      dft_reg<R, kSg>(vr[u], vi[u]);
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int j = tl + u * kT;
      const int jm = j & (kNs - 1);
      const int sb = ((j - jm) * R + jm) * kP + w;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        re[sb + r * kNs * kP] = vr[u][r];
        im[sb + r * kNs * kP] = vi[u][r];
      }
    }
  }
  __syncthreads();
}

template <int kSg, int kN, int kW, int kNs>
__device__ __forceinline__ void stockham_ct_from(Real* re, Real* im, int w, int tl, bool active,
                                                 const Real* __restrict__ tw) {
  if constexpr (kNs < kN) {
    constexpr int kRem = kN / kNs;
    constexpr int R = kRem > kEl ? kEl : kRem;
    stockham_pass_ct<R, kSg, kN, kW, kNs>(re, im, w, tl, active, tw);
    stockham_ct_from<kSg, kN, kW, kNs * R>(re, im, w, tl, active, tw);
  }
}

template <int kSg, int kN, int kW>
__device__ __forceinline__ void stockham_ct(Real* re, Real* im, const Real* __restrict__ tw) {
  const int t = threadIdx.x;
  const int w = t & (kW - 1), tl = t / kW;
  stockham_ct_from<kSg, kN, kW, 1>(re, im, w, tl, tl < kN / kEl, tw);
}

// the register FFT of the tile: a compile-time shape where one exists (the
// widths lines() gives these lengths), else the general passes
template <int kSg>
__device__ __forceinline__ void stockham_any(Real* re, Real* im, int n, int W, const Real* __restrict__ tw) {
  if (n == 512 && W == 4) stockham_ct<kSg, 512, 4>(re, im, tw);
  else if (n == 256 && W == 8) stockham_ct<kSg, 256, 8>(re, im, tw);
  else if (n == 128 && W == 16) stockham_ct<kSg, 128, 16>(re, im, tw);
  else if (n == 1024 && W == 2) stockham_ct<kSg, 1024, 2>(re, im, tw);
  else stockham<kSg>(re, im, n, W, tw);
}

// the tile shapes with a compile-time register FFT (stockham_any); their tiles
// hold n W = NT kEl values, kEl per thread
__device__ __forceinline__ bool ct_shape(int n, int W) {
  return (n == 512 && W == 4) || (n == 256 && W == 8) || (n == 128 && W == 16) || (n == 1024 && W == 2);
}

template <int kPass>
__global__ void __launch_bounds__(NT) k_poisson(Fields<Real> F, GridDev g, const Ctrl* __restrict__ ctrl,
                                                Grav<Real> gr, int W) {
  if (!ctrl->active) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const Geom q = geom(g, gr, kPass, W);
  const int P = W + 1;
  const int n = q.n;
  const int log2n = gr.log2n[q.axis];
  Real* re = (Real*)lds_raw;
  Real* im = re + (size_t)n * P;
  Real* xr = im + (size_t)n * P;   // direct DFT only
  Real* xi = xr + (size_t)n * P;
  const Real* __restrict__ tw = gr.tw[q.axis];
  Real2* __restrict__ cw = (Real2*)gr.cw;
  const int t = threadIdx.x;
  const int tile = n * W;
  // register FFT (power-of-two lines in its range), else the LDS radix-2 FFT
  // or the direct DFT; the radix-2 x and y passes load in bit-reversed order
  const bool fast = gr.fast[q.axis] != 0;
  const DivMod dn = divmod_by(n), dW = divmod_by(W), dny = divmod_by(g.ny);
  const bool rev = log2n >= 0 && kPass != kZ && !fast;
  // x passes: work-array index of element 0 of line w of this workgroup
  auto xline = [&](int w) -> long long {
    int kq, jj;
    dny(q.j + w, kq, jj);
    return ((long long)(q.k + kq) * gr.m[1] + jj) * gr.m[0];
  };

  // ------------------------------------------------------------------- load
  if constexpr (kPass == kXFwd) {
    const int par = ctrl->par;
    const Real* __restrict__ rho = F.U[par][0];
    const Real* __restrict__ mx = F.U[par][1];
    const Real* __restrict__ my = F.U[par][2];
    const Real* __restrict__ mz = F.U[par][3];
    const double dt = ctrl->dt;
    const Real ref = (Real)gr.rho_ref;
    const Real h2 = (Real)(2.0 * g.h);
    for (int idx = t; idx < tile; idx += NT) {
      int w, e;
      dn(idx, w, e);
      Real vr = 0, vi = 0;
      if (w < q.nl && e < q.nin) {
        const int l = q.j + w;  // line index within the k plane may wrap to the next plane
        int kq, jj;
        dny(l, kq, jj);
        const int kk = q.k + kq;
        const long long c = cell(g, e, jj, kk);
        const Real r = rho[c];
        Real div = 0;
        div += (mx[c + 1] - mx[c - 1]) / h2;
        div += (my[c + g.sx] - my[c - g.sx]) / h2;
        div += (mz[c + g.sxy] - mz[c - g.sxy]) / h2;
        vr = r - ref;
        vi = (r - (Real)dt * div) - ref;
      }
      const int s = rev ? bit_reverse(e, log2n) : e;
      re[s * P + w] = vr;
      im[s * P + w] = vi;
    }
  } else if constexpr (kPass == kXInv) {
    if (fast && ct_shape(n, W)) {
      // kEl elements per thread: their loads in flight together, then to LDS
      Real2 v[kEl];
#pragma unroll
      for (int r = 0; r < kEl; ++r) {
        int w, e;
        dn(t + r * NT, w, e);
        v[r].x = 0;
        v[r].y = 0;
        if (w < q.nl) v[r] = cw[xline(w) + e];
      }
#pragma unroll
      for (int r = 0; r < kEl; ++r) {
        int w, e;
        dn(t + r * NT, w, e);
        re[e * P + w] = v[r].x;
        im[e * P + w] = v[r].y;
      }
    } else {
      for (int idx = t; idx < tile; idx += NT) {
        int w, e;
        dn(idx, w, e);
        Real2 v;
        v.x = 0;
        v.y = 0;
        if (w < q.nl) v = cw[xline(w) + e];
        const int s = rev ? bit_reverse(e, log2n) : e;
        re[s * P + w] = v.x;
        im[s * P + w] = v.y;
      }
    }
  } else {
    if (fast && ct_shape(n, W)) {
      Real2 v[kEl];
#pragma unroll
      for (int r = 0; r < kEl; ++r) {
        int e, w;
        dW(t + r * NT, e, w);
        v[r].x = 0;
        v[r].y = 0;
        if (w < q.nl && e < q.nin) v[r] = cw[q.base + w + (long long)e * q.es];
      }
#pragma unroll
      for (int r = 0; r < kEl; ++r) {
        int e, w;
        dW(t + r * NT, e, w);
        re[e * P + w] = v[r].x;
        im[e * P + w] = v[r].y;
      }
    } else {
      for (int idx = t; idx < tile; idx += NT) {
        int e, w;
        dW(idx, e, w);
        Real2 v;
        v.x = 0;
        v.y = 0;
        if (w < q.nl && e < q.nin) v = cw[q.base + w + (long long)e * q.es];
        const int s = rev ? bit_reverse(e, log2n) : e;
        re[s * P + w] = v.x;
        im[s * P + w] = v.y;
      }
    }
  }
  __syncthreads();

  // -------------------------------------------------------------- transform
  constexpr bool kFwd = kPass == kXFwd || kPass == kYFwd;
  if (fast) {
    if constexpr (kPass == kZ) {
      stockham_any<-1>(re, im, n, W, tw);
      for (int idx = t; idx < tile; idx += NT) {
        int kz, w;
        dW(idx, kz, w);
        const Real f = w < q.nl ? green_at(gr, q.i0 + w, q.j, kz) : (Real)0;
        re[kz * P + w] *= f;
        im[kz * P + w] *= f;
      }
      __syncthreads();
      stockham_any<1>(re, im, n, W, tw);
    } else {
      stockham_any<kFwd ? -1 : 1>(re, im, n, W, tw);
    }
  } else if constexpr (kPass == kZ) {
    // forward, times the Green's function 4 pi G / (lambda(k) N), inverse; slot
    // s of a power-of-two line holds frequency bitrev(s) between the two
    if (log2n >= 0)
      fft_dif(re, im, n, W, tw, (Real)-1);
    else
      dft_direct(re, im, xr, xi, n, W, tw, (Real)-1);
    for (int idx = t; idx < tile; idx += NT) {
      int s, w;
      dW(idx, s, w);
      const int kz = log2n >= 0 ? bit_reverse(s, log2n) : s;
      const Real f = w < q.nl ? green_at(gr, q.i0 + w, q.j, kz) : (Real)0;
      re[s * P + w] *= f;
      im[s * P + w] *= f;
    }
    __syncthreads();
    if (log2n >= 0)
      fft_dit(re, im, n, W, tw, (Real)1);
    else
      dft_direct(re, im, xr, xi, n, W, tw, (Real)1);
  } else {
    if (log2n >= 0)
      fft_dit(re, im, n, W, tw, kFwd ? (Real)-1 : (Real)1);
    else
      dft_direct(re, im, xr, xi, n, W, tw, kFwd ? (Real)-1 : (Real)1);
  }
  __syncthreads();

  // ------------------------------------------------------------------ store
  // element idx of the tile to memory; the compile-time FFT shapes unroll the
  // kEl elements of a thread so that their reads are issued together
  auto store = [&](int idx) {
    if constexpr (kPass == kXFwd) {
      int w, e;
      dn(idx, w, e);
      if (w < q.nl) {
        Real2 v;
        v.x = re[e * P + w];
        v.y = im[e * P + w];
        cw[xline(w) + e] = v;
      }
    } else if constexpr (kPass == kXInv) {
      int w, e;
      dn(idx, w, e);
      if (w < q.nl && e < q.nout) {
        const int l = q.j + w;
        int kq, jj;
        dny(l, kq, jj);
        const int kk = q.k + kq;
        const long long c = cell(g, e, jj, kk);
        const Real ext = gr.psi_ext[c];
        F.psi[c] = ext + re[e * P + w];
        gr.psih[c] = ext + im[e * P + w];
      }
    } else {
      int e, w;
      dW(idx, e, w);
      if (w < q.nl && e < q.nout) {
        Real2 v;
        v.x = re[e * P + w];
        v.y = im[e * P + w];
        cw[q.base + w + (long long)e * q.es] = v;
      }
    }
  };
  if (fast && ct_shape(n, W)) {
#pragma unroll
    for (int r = 0; r < kEl; ++r) store(t + r * NT);
  } else {
    for (int idx = t; idx < tile; idx += NT) store(idx);
  }
}

}  // namespace CSPH_GTAG

using CSPH_GTAG::Real;
using namespace CSPH_GTAG;

template <>
bool Poisson<Real>::fast_ok(int n, int log2n) {
  return log2n >= 0 && n >= kEl && n <= NT * kEl;
}

template <>
size_t Poisson<Real>::lds_bytes(int n, int log2n, int W) {
  const size_t tile = (size_t)n * (W + 1) * sizeof(Real);
  return (log2n >= 0 ? 2 : 4) * tile;
}

template <>
int Poisson<Real>::lines(int n, int log2n) {
  // W * n complex values per tile; W capped so a y or z tile row stays one
  // 128-byte run (16 FP32 or 8 FP64 complex values), and so the tile's LDS
  // stays within 64 KiB
  if (fast_ok(n, log2n)) {
    // one line per T = n / kEl threads, at most 64 lines
    const int w = NT * kEl / n;
    return w > 64 ? 64 : w;
  }
  constexpr int cap = std::is_same<Real, double>::value ? 2048 : 4096;
  constexpr int wmax = std::is_same<Real, double>::value ? 8 : 16;
  int w = cap / n;
  if (w > wmax) w = wmax;
  if (w < 1) w = 1;
  while (w > 1 && lds_bytes(n, log2n, w) > kLdsMax) --w;
  return w;
}

template <>
bool Poisson<Real>::length_ok(int n, int log2n) {
  if (n < 1 || (log2n < 0 && n > 1024)) return false;
  return lds_bytes(n, log2n, 1) <= kLdsMax;
}

template <>
hipError_t Poisson<Real>::solve(const Fields<Real>& F, const GridDev& g, const Ctrl* ctrl,
                                const Grav<Real>& gr, hipStream_t s) {
  int W[3];
  size_t sh[3];
  for (int a = 0; a < 3; ++a) {
    W[a] = lines(gr.m[a], gr.log2n[a]);
    sh[a] = lds_bytes(gr.m[a], gr.log2n[a], W[a]);
  }
  // x passes: the ny nz lines that hold data; y passes: mx columns of nz
  // planes; z pass: mx columns of my rows
  const unsigned bx = (unsigned)((g.ny * g.nz + W[0] - 1) / W[0]);
  const unsigned by = (unsigned)(((gr.m[0] + W[1] - 1) / W[1]) * g.nz);
  const unsigned bz = (unsigned)(((gr.m[0] + W[2] - 1) / W[2]) * gr.m[1]);
  k_poisson<kXFwd><<<bx, NT, sh[0], s>>>(F, g, ctrl, gr, W[0]);
  k_poisson<kYFwd><<<by, NT, sh[1], s>>>(F, g, ctrl, gr, W[1]);
  k_poisson<kZ><<<bz, NT, sh[2], s>>>(F, g, ctrl, gr, W[2]);
  k_poisson<kYInv><<<by, NT, sh[1], s>>>(F, g, ctrl, gr, W[1]);
  k_poisson<kXInv><<<bx, NT, sh[0], s>>>(F, g, ctrl, gr, W[0]);
  return hipGetLastError();
}

// ------------------------------------------------ isolated box: Green's function
// The free-space potential of the cells, psi_i = -G h^3 sum_j rho_j phi(r_i -
// r_j) with phi(d) = 1/|d| and phi(0) = C/h (C = 3 ln(2 + sqrt 3) - pi/2, the
// integral of 1/|x| over a unit cube), is a linear convolution over the box.
// With every transform length m_d >= 2 n_d it equals the circular convolution
// of the zero-padded density with the kernel taken at the wrapped distance
// min(t, m_d - t) along each axis (Hockney's method).  That kernel is real and
// even in every axis, so its transform is real and even too: along one axis
//   K(k) = g(0) + g(m/2) cos(pi k) + 2 sum_{0<t<m/2} g(t) cos(2 pi k t / m),
// k <= m/2, applied axis by axis to the octant of distances.  Computed once, in
// FP64, by direct sums (O(m/2) per value), then stored as Real.
namespace CSPH_GTAG {

__global__ void __launch_bounds__(256) k_green_fill(double* __restrict__ A, int hx, int hy, int hz,
                                                    double scale) {
  const long long n = (long long)(hx + 1) * (hy + 1) * (hz + 1);
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  const int a = (int)(q % (hx + 1));
  const long long r = q / (hx + 1);
  const int b = (int)(r % (hy + 1)), c = (int)(r / (hy + 1));
  const double d2 = (double)a * a + (double)b * b + (double)c * c;
  A[q] = scale * (d2 == 0.0 ? 3.0 * log(2.0 + sqrt(3.0)) - 0.5 * 3.14159265358979323846 : 1.0 / sqrt(d2));
}

// out = the cosine transform of in along axis ax, over the (hx+1)(hy+1)(hz+1)
// octant, x fastest; ct[t] = cos(2 pi t / m), m = 2 h_ax
__global__ void __launch_bounds__(256) k_green_axis(const double* __restrict__ in, double* __restrict__ out,
                                                    int hx, int hy, int hz, int ax,
                                                    const double* __restrict__ ct) {
  const long long n = (long long)(hx + 1) * (hy + 1) * (hz + 1);
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  const int a = (int)(q % (hx + 1));
  const long long r = q / (hx + 1);
  const int b = (int)(r % (hy + 1)), c = (int)(r / (hy + 1));
  const int H = ax == 0 ? hx : ax == 1 ? hy : hz;
  const int m = 2 * H;
  const int k = ax == 0 ? a : ax == 1 ? b : c;
  const long long stride = ax == 0 ? 1 : ax == 1 ? (long long)(hx + 1) : (long long)(hx + 1) * (hy + 1);
  const long long base = q - (long long)k * stride;
  double acc = in[base] + in[base + (long long)H * stride] * ct[(long long)k * H % m];
  double sum = 0.0;
  int t = k;  // (k j) mod m
  for (int j = 1; j < H; ++j, t += k) {
    if (t >= m) t -= m;
    sum += in[base + (long long)j * stride] * ct[t];
  }
  out[q] = acc + 2.0 * sum;
}

__global__ void __launch_bounds__(256) k_green_store(const double* __restrict__ in, Real* __restrict__ out,
                                                     long long n) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q < n) out[q] = (Real)in[q];
}

}  // namespace CSPH_GTAG

template <>
hipError_t Poisson<Real>::green(const Grav<Real>& gr, double h, double* tmp, const double* const ctab[3],
                                hipStream_t s) {
  const int hx = gr.m[0] / 2, hy = gr.m[1] / 2, hz = gr.m[2] / 2;
  const long long n = (long long)(hx + 1) * (hy + 1) * (hz + 1);
  const unsigned nb = (unsigned)((n + 255) / 256);
  double* A = tmp;
  double* B = tmp + n;
  // unit G: -h^3 phi = -h^2 (C or 1/sqrt(a^2+b^2+c^2)), with the inverse
  // transform's 1/(mx my mz) folded in
  const double scale = -h * h / ((double)gr.m[0] * gr.m[1] * gr.m[2]);
  k_green_fill<<<nb, 256, 0, s>>>(A, hx, hy, hz, scale);
  k_green_axis<<<nb, 256, 0, s>>>(A, B, hx, hy, hz, 0, ctab[0]);
  k_green_axis<<<nb, 256, 0, s>>>(B, A, hx, hy, hz, 1, ctab[1]);
  k_green_axis<<<nb, 256, 0, s>>>(A, B, hx, hy, hz, 2, ctab[2]);
  k_green_store<<<nb, 256, 0, s>>>(B, const_cast<Real*>(gr.khat), n);
  return hipGetLastError();
}

template struct Poisson<Real>;

}  // namespace csph
