// csph_internal.h -- structures shared by the host runtime and the HIP kernels.
//
// Data layout in HBM (one simulation): every field is a padded 3D array of
// (nx+4) x (ny+4) x (nz+4) cells (two ghost layers per face), x fastest, one
// array per field (structure of arrays), each starting on a 256-byte boundary.
// Fields: two copies of the conserved state U = (rho, mx, my, mz, E) used in
// turn as U^n and U^{n+1}; psi; the predictor output (m*, E*, xi*, psi at r*
// and phi* of the predicted particle); the corrector output (m~, E~, xi^{n+1}).  The density never changes in the
// Lagrangian stage, so rho* = rho~ = rho^n is not stored.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace csph {

constexpr int kGhost = 2;

// roles of a field for the ghost-cell rules
enum Role : int {
  kRho = 0, kMx = 1, kMy = 2, kMz = 3, kE = 4, kXx = 5, kXy = 6, kXz = 7, kPsi = 8, kPhi = 9
};
enum Bc : int { kPeriodic = 0, kOutflow = 1, kInflow = 2, kReflect = 3 };

// status bits raised on the device (sticky until set_state)
enum : int { kBadNonFinite = 1, kBadNegDensity = 2, kBadNoSignal = 4 };

struct GridDev {
  int nx, ny, nz;
  int sx, sy, sz;        // padded extents
  long long sxy;         // sx * sy
  long long ncell;       // padded cell count
  double h, inv_h, h3;
  double gamma, gm1;     // gamma, gamma - 1
  double rho_vac, neg_tol;
  double cfl_h;          // cfl * h
  double kappa_h2;       // kernel normalisation / h^2
  // 13 lattice kernel gradients K(-h o), o in the half neighbour set
  double klat[13][3];
  // Eulerian-stage scheme: TVD limiter and face flux (kLim*, kFlux*)
  int limiter, flux;
  // 1 if a potential was set; 0: psi = 0 everywhere, and psi(r*) stays 0 without
  // being loaded, interpolated or stored
  int psi;
  // viscosity: kinematic nu (0: inviscid), the explicit limit h^2/(4 nu) of dt
  // (0 when inviscid), and nu lambda_o per half-set offset, lambda_o =
  // -2 (d . K(d)) / |d|^2 at d = -h o (the lattice pair weight of the viscous force)
  double nu, dt_visc;
  double nulam[13];
  // sources and sinks: specific internal energy of the injected gas (the rates
  // are the field Fields::src)
  double eps_src;
};

enum : int { kLimMinmod = 0, kLimMC = 1, kLimVanLeer = 2, kLimSuperbee = 3 };
enum : int { kFluxSwept = 0, kFluxLF = 1, kFluxSweptAV = 2 };

// the default scheme runs the specialised stage-E kernel; others the generic one
inline __host__ __device__ bool default_scheme(const GridDev& g) {
  return g.limiter == kLimMinmod && g.flux == kFluxSweptAV;
}

struct BcDev {
  int kind[6];
  double cons[6][5];     // inflow conserved state per face
  double vel[6][3];      // inflow velocity per face (particle offset = dt * vel)
  double phi[6];         // sqrt(2 p) of the inflow state per face
};

// Per-simulation control block in device memory (FP64).
struct Ctrl {
  double t;                          // time of the current state
  double dt;                         // step being taken
  unsigned long long smax_bits[2];   // max signal speed (bits of a positive double)
  long long nsteps;
  int par;                           // which state copy holds U^n
  int cur;                           // which smax slot belongs to U^n
  int active;                        // the step being launched runs
  int done;                          // t reached the requested end time
  int status;                        // kBad* bits
  int smax_valid;                    // smax_bits[cur] describes U^n
  int pad[2];
  // batch membership: stop after this many steps in total, or at t_end
  long long step_limit;
  double t_end;
};

template <typename Real>
struct Fields {
  Real* U[2][5];
  Real* psi;
  Real* ms[4];   // m*x, m*y, m*z, E*
  Real* xs[3];   // xi*
  Real* psis;    // psi at the predicted particle positions r* = x + xi*
  Real* psic;    // the potential the corrector samples at r*: psi, or with
                 // self-gravity the potential of the density predicted for t^{n+1}
  Real* phs;     // phi* = sqrt(2 p*), p* the predicted particle's pressure at its predicted volume
  Real* mt[4];   // m~x, m~y, m~z, E~
  Real* xt[3];   // xi^{n+1}
  Real* src;     // sources and sinks: mass rate per cell (padded layout), or null
};

// one member of a batch, as the batched kernels see it (device memory)
template <typename Real>
struct Inst {
  Fields<Real> F;
  GridDev g;
  BcDev bc;
  Ctrl* ctrl;
  double* partials;
  int tz;
  int pad;
};

// up to 7 fields filled by one ghost-cell launch
template <typename Real>
struct FillSet {
  Real* f[8];
  int role[8];
  int n;
};

// Self-gravity of a periodic box: the buffers of the Poisson solve (device
// memory) and its constants.
template <typename Real>
struct Grav {
  // periodic box: transform lengths m_d = n_d.  Isolated box (no periodic
  // face): the free-space potential as a circular convolution over the box
  // zero-padded to m_d, the next power of two >= 2 n_d
  int iso;
  int m[3];              // transform length per axis
  Real* cw;              // work array [nz][my][mx] complex values (re, im), x fastest
  Real* psi_ext;         // the external potential (padded layout; interior read)
  Real* psih;            // potential of the predicted density (padded layout)
  const Real* tw[3];     // per axis: (cos, sin) of 2 pi k / m_d, k < m_d
  const double* lam[3];  // periodic: per axis (2 cos(2 pi k / n_d) - 2) / h^2
  const Real* khat;      // isolated: transform of the unit-G Green's function over
                         // (mx/2+1)(my/2+1)(mz/2+1) frequencies (it is even), / (mx my mz)
  int log2n[3];          // log2 of m_d (a power of two), else -1
  int fast[3];           // the axis uses the register FFT
  double fpg_n;          // periodic: 4 pi G / (nx ny nz); isolated: G
  double rho_ref;        // constant taken off the density before the transform
};

template <typename Real>
struct Poisson {
  // psi = psi_ext + potential of rho^n and psih = psi_ext + potential of the
  // density predicted for t^{n+1} (interior cells; ghosts are left), from U^n
  // and the step's dt; five launches on s, skipped when the step is inactive
  static hipError_t solve(const Fields<Real>& F, const GridDev& g, const Ctrl* ctrl,
                          const Grav<Real>& gr, hipStream_t s);
  static bool length_ok(int n, int log2n);  // a transform length the solve supports
  static bool fast_ok(int n, int log2n);    // a transform length of the register FFT
  static int lines(int n, int log2n);       // lines per workgroup of an axis pass
  static size_t lds_bytes(int n, int log2n, int W);
  // isolated box: fills gr.khat for transform lengths gr.m and cell size h,
  // in FP64 on s; tmp: 2 (mx/2+1)(my/2+1)(mz/2+1) doubles, ctab[d]: cos(2 pi t
  // / m_d) for t < m_d (device); the caller waits on s before freeing them
  static hipError_t green(const Grav<Real>& gr, double h, double* tmp, const double* const ctab[3],
                          hipStream_t s);
};

// launchers, instantiated for float and double by the kernel translation units
template <typename Real>
struct Launch {
  // every ghost cell of U[par] (all zones): after a new state or new boundaries
  static hipError_t fill_state(const Fields<Real>& F, const GridDev& g, const BcDev& bc, int par,
                               Ctrl* ctrl, hipStream_t s);
  static hipError_t fill_psi(const Fields<Real>& F, const GridDev& g, const BcDev& bc,
                             Ctrl* ctrl, hipStream_t s);
  static hipError_t signal_max(const Fields<Real>& F, const GridDev& g, Ctrl* ctrl,
                               hipStream_t s);
  // every element of f[0..n) set to v
  static hipError_t fill_const(Real* f, double v, long long n, hipStream_t s);
  // one full step: begin, [first half of the sources], ghosts, [self-gravity
  // potentials], stage P, ghosts, stage C, ghosts, stage E, end
  // gr (nullable): the self-gravity solve; ev (nullable): kStepEvents events
  // recorded around the launches, for kernel timing
  static constexpr int kStepEvents = 10;
  static hipError_t step(const Fields<Real>& F, const GridDev& g, const BcDev& bc, Ctrl* ctrl,
                         double* partials, double dt_max, double t_end, const int tz[3],
                         const Grav<Real>* gr, hipStream_t s, hipEvent_t* ev);
  // one step of every active member of a batch, one launch per stage
  // tile_map[t] = (member, tile of that member); fill_map[b] = (member, first
  // ghost cell of fill block b); generic: some member uses a non-default scheme
  // viscous: some member has a viscosity (the Lagrangian sweeps' viscous form)
  static hipError_t batch_step(const Inst<Real>* tab, const int2* tile_map, const int2* fill_map,
                               int n, int total_tiles, int fill_blocks, int* flags, bool generic,
                               bool viscous, hipStream_t s);
  static int tiles(const GridDev& g, int tz);
  static int default_tz(const GridDev& g);
  static long long ghosts(const GridDev& g);
  static hipError_t totals(const GridDev& g, const double* partials, int nblocks, double* out,
                           hipStream_t s);
};

}  // namespace csph
