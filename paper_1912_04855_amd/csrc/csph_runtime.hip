// csph_runtime.hip -- host runtime behind the C ABI declared in include/csph.h.
//
// One simulation = one device allocation (library-owned or caller-lent) that
// holds the padded fields, the FP64 control block and the per-block totals.
// The time loop runs on the device: the step kernels read dt, t and the state
// parity from the control block, so the host only enqueues launches and polls a
// completion flag every few steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/csph.h"
#include "csph_internal.h"

using namespace csph;

namespace {

thread_local std::string g_err;

csph_status fail(csph_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(CSPH_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// device fields: U[2][5], psi, ms[4], (xs[3]), psis, phs, mt[4], (xt[3]); the FP32
// build forms the particle offsets xs, xt where it needs them and has no storage
// for them
constexpr int kNumFields64 = 27, kNumFields32 = 21;
int num_fields(int dtype) { return dtype == CSPH_F64 ? kNumFields64 : kNumFields32; }

// tile depths (z-planes per workgroup of the stencil sweeps) the autotuner tries
constexpr int kTzMin = 2, kTzMax = 64;
constexpr int kTzCand[] = {2, 4, 8, 16, 32, 64};

// tile depths (stages P, C, E) chosen by csph_autotune, per (device, dtype,
// nx, ny, nz): later simulations of the same shape start from them
using Depths = std::array<int, 3>;
std::mutex g_tune_mu;
std::map<std::array<int, 5>, Depths> g_tune;

std::array<int, 5> tune_key(int device, const csph_grid_desc& d) {
  return {device, (int)d.dtype, d.nx, d.ny, d.nz};
}

// kernel normalisation: kappa = 1 / (2 sum_{a,b in {-1,0,1}} g(q_ab)/q_ab),
// q_ab = sqrt(1 + a^2 + b^2), g(q)/q of the M4 spline (27-point sum exact for
// linear fields)
double g_over_q(double q) {
  if (q < 1.0) return 3.0 - 2.25 * q;
  if (q < 2.0) {
    const double t = 2.0 - q;
    return 0.75 * t * t / q;
  }
  return 0.0;
}

// phi = sqrt(2 p) of a conserved state, p = (gamma - 1)(E - m.u/2) floored at 0,
// u = m/rho (0 in vacuum): the arithmetic of the kernels' FP64 primitive()
double inflow_phi(const double cons[5], double gamma, double rho_vac) {
  const double r = cons[0];
  double ux = 0.0, uy = 0.0, uz = 0.0;
  if (r > rho_vac) {
    ux = cons[1] / r;
    uy = cons[2] / r;
    uz = cons[3] / r;
  }
  const double ke = 0.5 * (cons[1] * ux + cons[2] * uy + cons[3] * uz);
  const double pp = (gamma - 1.0) * (cons[4] - ke);
  const double p = pp > 0.0 ? pp : 0.0;
  return std::sqrt(2.0 * p);
}

double kernel_kappa() {
  double sum = 0.0;
  for (int a = -1; a <= 1; ++a)
    for (int b = -1; b <= 1; ++b) sum += g_over_q(std::sqrt(1.0 + (double)(a * a) + (double)(b * b)));
  return 1.0 / (2.0 * sum);
}

const int kHalf[13][3] = {{1, 0, 0},  {-1, 1, 0}, {0, 1, 0},  {1, 1, 0},  {-1, -1, 1},
                          {0, -1, 1}, {1, -1, 1}, {-1, 0, 1}, {0, 0, 1},  {1, 0, 1},
                          {-1, 1, 1}, {0, 1, 1},  {1, 1, 1}};

bool desc_ok(const csph_grid_desc* d, std::string* why) {
  if (!d) {
    *why = "desc is NULL";
    return false;
  }
  if (d->nx < 4 || d->ny < 4 || d->nz < 4) {
    *why = "nx, ny, nz must be >= 4";
    return false;
  }
  if (!(d->h > 0.0) || !std::isfinite(d->h)) {
    *why = "h must be > 0";
    return false;
  }
  if (!(d->gamma > 1.0)) {
    *why = "gamma must be > 1";
    return false;
  }
  if (!(d->cfl > 0.0 && d->cfl <= 0.5)) {
    *why = "cfl must be in (0, 0.5]";
    return false;
  }
  if (!(d->rho_vac >= 0.0)) {
    *why = "rho_vac must be >= 0";
    return false;
  }
  if (d->dtype != CSPH_F32 && d->dtype != CSPH_F64) {
    *why = "dtype must be CSPH_F32 or CSPH_F64";
    return false;
  }
  // at most 4e9 padded cells; with nz >= 4 a padded x-y plane then holds fewer
  // than 5e8 cells, so the kernels index within a plane in 32 bits
  const double cells = (double)(d->nx + 4) * (d->ny + 4) * (d->nz + 4);
  if (cells > 4.0e9) {
    *why = "grid too large";
    return false;
  }
  return true;
}

struct Layout {
  size_t field_bytes, fields_off, ctrl_off, partials_off, totals_off, total;
  long long ncell;
  int nblocks;
};

// viscosity constants of a grid: nu lambda_o with lambda_o = -2 (d . K) / |d|^2 at
// the lattice separation d = -h o, and the explicit limit of dt (the arithmetic
// of the kernels' FP64 build, operation for operation)
void set_viscosity(GridDev& g, double nu) {
  g.nu = nu;
  g.dt_visc = nu > 0.0 ? 0.25 * g.h * g.h / nu : 0.0;
  for (int q = 0; q < 13; ++q) {
    const double dx = -kHalf[q][0] * g.h, dy = -kHalf[q][1] * g.h, dz = -kHalf[q][2] * g.h;
    const double lam = -2.0 * (dx * g.klat[q][0] + dy * g.klat[q][1] + dz * g.klat[q][2]) /
                       (dx * dx + dy * dy + dz * dz);
    g.nulam[q] = nu * lam;
  }
}

GridDev make_grid(const csph_grid_desc* d) {
  GridDev g{};
  g.nx = d->nx;
  g.ny = d->ny;
  g.nz = d->nz;
  g.sx = d->nx + 2 * kGhost;
  g.sy = d->ny + 2 * kGhost;
  g.sz = d->nz + 2 * kGhost;
  g.sxy = (long long)g.sx * g.sy;
  g.ncell = g.sxy * g.sz;
  g.h = d->h;
  g.inv_h = 1.0 / d->h;
  g.h3 = d->h * d->h * d->h;
  g.gamma = d->gamma;
  g.gm1 = d->gamma - 1.0;
  g.rho_vac = d->rho_vac;
  g.neg_tol = 0.01 * d->rho_vac;
  g.cfl_h = d->cfl * d->h;
  g.kappa_h2 = kernel_kappa() / (d->h * d->h);
  // lattice gradients K(d) = -(kappa/h^2)(g(q)/q) d at d = -h o
  for (int q = 0; q < 13; ++q) {
    const double dx = -kHalf[q][0] * d->h, dy = -kHalf[q][1] * d->h, dz = -kHalf[q][2] * d->h;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double qq = std::sqrt(r2) * g.inv_h;
    const double c = g.kappa_h2 * g_over_q(qq);
    g.klat[q][0] = -(c * dx);
    g.klat[q][1] = -(c * dy);
    g.klat[q][2] = -(c * dz);
  }
  g.limiter = kLimMinmod;
  g.flux = kFluxSweptAV;
  g.psi = 0;
  set_viscosity(g, 0.0);
  return g;
}

Layout make_layout(const csph_grid_desc* d) {
  Layout L{};
  const GridDev g = make_grid(d);
  const size_t es = d->dtype == CSPH_F64 ? 8 : 4;
  L.ncell = g.ncell;
  L.field_bytes = align_up((size_t)g.ncell * es);
  L.fields_off = 0;
  L.ctrl_off = L.fields_off + (size_t)num_fields(d->dtype) * L.field_bytes;
  // per-tile totals of stage E, sized for the shallowest tile depth a sim may use
  L.nblocks = d->dtype == CSPH_F64 ? Launch<double>::tiles(g, kTzMin) : Launch<float>::tiles(g, kTzMin);
  L.partials_off = L.ctrl_off + align_up(sizeof(Ctrl));
  L.totals_off = L.partials_off + align_up((size_t)L.nblocks * 5 * sizeof(double));
  L.total = L.totals_off + align_up(5 * sizeof(double));
  return L;
}

}  // namespace

struct csph_sim {
  csph_grid_desc desc{};
  hipStream_t stream = nullptr;
  char* buf = nullptr;
  bool owned = false;
  int device = 0;
  Layout L{};
  GridDev g{};
  BcDev bc{};
  double inflow_prim[6][5]{};
  Fields<float> f32{};
  Fields<double> f64{};
  Ctrl* ctrl = nullptr;
  double* partials = nullptr;
  double* totals_dev = nullptr;
  bool psi_dirty = true;
  bool x_stale = true;   // the x ghosts of U^n do not follow the state / boundaries
  bool need_smax = true;
  int tz[3] = {0, 0, 0};  // z-planes per workgroup of the sweeps of stages P, C, E
  int tz_last = 0;        // tile depth of the last stage E launched (its per-tile totals)
  bool in_batch = false;
  hipStream_t batch_stream = nullptr;  // stream of the batch this sim belongs to
  bool stepped = false;  // partials describe the current state
  bool in_static = false;  // lives in this device's static array (csph_create_static)
  std::vector<double> psi_host;  // interior psi, kept to refill ghosts after BC changes
  bool has_psi = false;
  // kernel timing: events of up to kProfSteps steps in flight, accumulated at syncs
  static constexpr int kProfSteps = 64;
  bool prof_on = false;
  static constexpr int kEv = Launch<float>::kStepEvents;
  std::vector<hipEvent_t> prof_ev;  // kProfSteps x kEv
  int prof_pending = 0;
  double prof_ms[6] = {0, 0, 0, 0, 0, 0};
  int64_t prof_n[6] = {0, 0, 0, 0, 0, 0};
  // self-gravity: G, and the Poisson solve's own device memory (work array,
  // external potential, potential of the predicted density, twiddle and
  // eigenvalue tables or, on an isolated box, the Green's function),
  // allocated when it is switched on; grav_iso: the box has no periodic face
  double grav = 0.0;
  bool grav_iso = false;
  char* gbuf = nullptr;
  // sources and sinks: the rate field (padded layout, own allocation) or null
  char* srcbuf = nullptr;
  Grav<float> gr32{};
  Grav<double> gr64{};

  bool is_f64() const { return desc.dtype == CSPH_F64; }
  char* field_ptr(int k) const { return buf + L.fields_off + (size_t)k * L.field_bytes; }
};

namespace {

// ------------------------------------------------------------ static array
// Device memory of csph_create_static: one array per GPU the library runs on,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in; its device address on each GPU comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address is
// handed to kernels and memory calls.  The simulation object of each slot has
// static host storage too, so creating one allocates nothing.
__device__ __align__(256) unsigned char scratch[CSPH_STATIC_BYTES];
constexpr int kMaxDevices = 64;
struct StaticSlot {
  void* dev = nullptr;   // device address of `scratch` on this GPU (set once)
  bool in_use = false;   // a simulation lives in it
  alignas(csph_sim) unsigned char host[sizeof(csph_sim)];
};
StaticSlot g_static[kMaxDevices];
std::mutex g_static_mu;

template <typename Real>
void bind_fields(csph_sim* s, Fields<Real>& F) {
  int k = 0;
  for (int p = 0; p < 2; ++p)
    for (int v = 0; v < 5; ++v) F.U[p][v] = (Real*)s->field_ptr(k++);
  F.psi = (Real*)s->field_ptr(k++);
  const bool offsets = s->is_f64();  // only the FP64 build stores xi*, xi^{n+1}
  for (int v = 0; v < 4; ++v) F.ms[v] = (Real*)s->field_ptr(k++);
  for (int v = 0; v < 3; ++v) F.xs[v] = offsets ? (Real*)s->field_ptr(k++) : nullptr;
  F.psis = (Real*)s->field_ptr(k++);
  F.psic = F.psi;
  F.src = nullptr;
  F.phs = (Real*)s->field_ptr(k++);
  for (int v = 0; v < 4; ++v) F.mt[v] = (Real*)s->field_ptr(k++);
  for (int v = 0; v < 3; ++v) F.xt[v] = offsets ? (Real*)s->field_ptr(k++) : nullptr;
}

// a batch member's device state is written on the batch's stream: reads of it
// wait for that stream first
csph_status wait_batch(const csph_sim* s) {
  if (s->in_batch && s->batch_stream) HIP_TRY(hipStreamSynchronize(s->batch_stream));
  return CSPH_OK;
}

csph_status read_ctrl(const csph_sim* s, Ctrl* out) {
  csph_status st = wait_batch(s);
  if (st) return st;
  HIP_TRY(hipMemcpyAsync(out, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return CSPH_OK;
}

csph_status write_ctrl(csph_sim* s, const Ctrl& c) {
  HIP_TRY(hipMemcpyAsync(s->ctrl, &c, sizeof(Ctrl), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return CSPH_OK;
}

csph_status status_from_bits(int bits) {
  if (bits & kBadNonFinite) return fail(CSPH_ERR_NONFINITE, "a non-finite value appeared in the state");
  if (bits & kBadNegDensity) return fail(CSPH_ERR_NEG_DENSITY, "negative density appeared in the state");
  if (bits & kBadNoSignal)
    return fail(CSPH_ERR_NO_SIGNAL, "no non-vacuum cell: the CFL step needs dt_max > 0");
  return CSPH_OK;
}

template <typename Real>
csph_status upload_field(csph_sim* s, Real* dst, const double* interior) {
  const GridDev& g = s->g;
  std::vector<Real> pad((size_t)g.ncell, (Real)0);
  size_t q = 0;
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j) {
      Real* row = pad.data() + ((size_t)(k + kGhost) * g.sy + (j + kGhost)) * g.sx + kGhost;
      for (int i = 0; i < g.nx; ++i) row[i] = (Real)interior[q++];
    }
  HIP_TRY(hipMemcpyAsync(dst, pad.data(), pad.size() * sizeof(Real), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return CSPH_OK;
}

template <typename Real>
csph_status download_field(const csph_sim* s, const Real* src, double* interior) {
  csph_status st = wait_batch(s);
  if (st) return st;
  const GridDev& g = s->g;
  std::vector<Real> pad((size_t)g.ncell);
  HIP_TRY(hipMemcpyAsync(pad.data(), src, pad.size() * sizeof(Real), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  size_t q = 0;
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j) {
      const Real* row = pad.data() + ((size_t)(k + kGhost) * g.sy + (j + kGhost)) * g.sx + kGhost;
      for (int i = 0; i < g.nx; ++i) interior[q++] = (double)row[i];
    }
  return CSPH_OK;
}

template <typename Real>
Fields<Real>& fields_of(csph_sim* s);
template <>
Fields<float>& fields_of<float>(csph_sim* s) { return s->f32; }
template <>
Fields<double>& fields_of<double>(csph_sim* s) { return s->f64; }

template <typename Real>
Grav<Real>& grav_of(csph_sim* s);
template <>
Grav<float>& grav_of<float>(csph_sim* s) { return s->gr32; }
template <>
Grav<double>& grav_of<double>(csph_sim* s) { return s->gr64; }

template <typename Real>
csph_status set_state_t(csph_sim* s, const double* cons) {
  Fields<Real>& F = fields_of<Real>(s);
  const size_t N = (size_t)s->g.nx * s->g.ny * s->g.nz;
  for (int v = 0; v < 5; ++v) {
    csph_status st = upload_field<Real>(s, F.U[0][v], cons + (size_t)v * N);
    if (st) return st;
  }
  return CSPH_OK;
}

// a box of the interior (lo: first cell, n: extent, both (x, y, z)) of one
// field from / to a host array [n_z][n_y][n_x], one 2D copy per z plane
template <typename Real>
csph_status box_upload(csph_sim* s, Real* field, const int32_t lo[3], const int32_t n[3],
                       const double* host) {
  const GridDev& g = s->g;
  const size_t plane = (size_t)n[0] * n[1];
  std::vector<Real> stage(plane * n[2]);
  for (size_t q = 0; q < stage.size(); ++q) stage[q] = (Real)host[q];
  for (int k = 0; k < n[2]; ++k) {
    Real* dst = field + ((size_t)(lo[2] + k + kGhost) * g.sy + (lo[1] + kGhost)) * g.sx + (lo[0] + kGhost);
    HIP_TRY(hipMemcpy2DAsync(dst, (size_t)g.sx * sizeof(Real), stage.data() + plane * k,
                             (size_t)n[0] * sizeof(Real), (size_t)n[0] * sizeof(Real), (size_t)n[1],
                             hipMemcpyHostToDevice, s->stream));
  }
  HIP_TRY(hipStreamSynchronize(s->stream));
  return CSPH_OK;
}

template <typename Real>
csph_status box_download(const csph_sim* s, const Real* field, const int32_t lo[3], const int32_t n[3],
                         double* host) {
  const GridDev& g = s->g;
  const size_t plane = (size_t)n[0] * n[1];
  std::vector<Real> stage(plane * n[2]);
  for (int k = 0; k < n[2]; ++k) {
    const Real* src =
        field + ((size_t)(lo[2] + k + kGhost) * g.sy + (lo[1] + kGhost)) * g.sx + (lo[0] + kGhost);
    HIP_TRY(hipMemcpy2DAsync(stage.data() + plane * k, (size_t)n[0] * sizeof(Real), src,
                             (size_t)g.sx * sizeof(Real), (size_t)n[0] * sizeof(Real), (size_t)n[1],
                             hipMemcpyDeviceToHost, s->stream));
  }
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (size_t q = 0; q < stage.size(); ++q) host[q] = (double)stage[q];
  return CSPH_OK;
}

bool box_ok(const csph_sim* s, const int32_t lo[3], const int32_t n[3]) {
  if (!lo || !n) return false;
  const int ext[3] = {s->g.nx, s->g.ny, s->g.nz};
  for (int a = 0; a < 3; ++a)
    if (lo[a] < 0 || n[a] < 1 || (long long)lo[a] + n[a] > ext[a]) return false;
  return true;
}

// conserved variables of primitive (rho, u, v, w, p) values, in place
csph_status to_conserved(double gamma, double* st, size_t count, size_t stride) {
  for (size_t q = 0; q < count; ++q) {
    const double r = st[q], ux = st[stride + q], uy = st[2 * stride + q], uz = st[3 * stride + q],
                 p = st[4 * stride + q];
    if (!(r >= 0.0)) return fail(CSPH_ERR_ARG, "density must be >= 0");
    if (!(p >= 0.0)) return fail(CSPH_ERR_ARG, "pressure must be >= 0");
    st[stride + q] = r * ux;
    st[2 * stride + q] = r * uy;
    st[3 * stride + q] = r * uz;
    st[4 * stride + q] = p / (gamma - 1.0) + 0.5 * r * (ux * ux + uy * uy + uz * uz);
  }
  return CSPH_OK;
}

template <typename Real>
csph_status prepare(csph_sim* s) {
  Fields<Real>& F = fields_of<Real>(s);
  if (s->psi_dirty) {
    HIP_TRY(Launch<Real>::fill_psi(F, s->g, s->bc, s->ctrl, s->stream));
    s->psi_dirty = false;
  }
  if (s->x_stale) {
    // the stages push the x ghosts of what they write; a state set from the host
    // (or new boundaries) needs all its ghost cells once
    Ctrl c{};
    csph_status st = read_ctrl(s, &c);
    if (st) return st;
    HIP_TRY(Launch<Real>::fill_state(F, s->g, s->bc, c.par, s->ctrl, s->stream));
    s->x_stale = false;
  }
  if (s->need_smax) {
    HIP_TRY(Launch<Real>::signal_max(F, s->g, s->ctrl, s->stream));
    s->need_smax = false;
  }
  return CSPH_OK;
}

// fold the recorded events of completed steps into the per-group totals
csph_status prof_collect(csph_sim* s) {
  if (!s->prof_on || s->prof_pending == 0) return CSPH_OK;
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (int k = 0; k < s->prof_pending; ++k) {
    hipEvent_t* e = &s->prof_ev[(size_t)k * csph_sim::kEv];
    float ms[csph_sim::kEv - 1];
    for (int q = 0; q < csph_sim::kEv - 1; ++q) HIP_TRY(hipEventElapsedTime(&ms[q], e[q], e[q + 1]));
    // e0-e1 begin + state fill, e1-e2 Poisson solve (self-gravity), e2-e3 P,
    // e3-e4 nothing, e4-e5 fill, e5-e6 C, e6-e7 fill, e7-e8 E, e8-e9 end
    s->prof_ms[0] += ms[2];
    s->prof_ms[1] += ms[5];
    s->prof_ms[2] += ms[7];
    s->prof_ms[3] += ms[0] + ms[4] + ms[6];
    s->prof_ms[4] += ms[8];
    s->prof_ms[5] += ms[1] + ms[3];
    for (int q = 0; q < 5; ++q) s->prof_n[q] += 1;
    if (s->grav > 0.0) s->prof_n[5] += 1;
  }
  s->prof_pending = 0;
  return CSPH_OK;
}

template <typename Real>
csph_status launch_steps(csph_sim* s, int n, double dt_max, double t_end) {
  csph_status st = prepare<Real>(s);
  if (st) return st;
  Fields<Real>& F = fields_of<Real>(s);
  for (int k = 0; k < n; ++k) {
    hipEvent_t* ev = nullptr;
    if (s->prof_on) {
      if (s->prof_pending == csph_sim::kProfSteps) {
        st = prof_collect(s);
        if (st) return st;
      }
      ev = &s->prof_ev[(size_t)s->prof_pending * csph_sim::kEv];
      s->prof_pending += 1;
    }
    const Grav<Real>* gr = s->grav > 0.0 ? &grav_of<Real>(s) : nullptr;
    HIP_TRY(Launch<Real>::step(F, s->g, s->bc, s->ctrl, s->partials, dt_max, t_end, s->tz, gr,
                               s->stream, ev));
  }
  s->stepped = true;
  s->tz_last = s->tz[2];
  return CSPH_OK;
}

csph_status launch(csph_sim* s, int n, double dt_max, double t_end) {
  return s->is_f64() ? launch_steps<double>(s, n, dt_max, t_end)
                  : launch_steps<float>(s, n, dt_max, t_end);
}

// self-gravity: the constant taken off the density before the transform (the
// mean density of the state, which the periodic solve discards anyway and
// mass conservation keeps; none on an isolated box, where the mean matters)
void set_rho_ref(csph_sim* s, const double* cons) {
  const size_t N = (size_t)s->g.nx * s->g.ny * s->g.nz;
  double a = 0.0;
  for (size_t q = 0; q < N; ++q) a += cons[q];
  s->gr32.rho_ref = s->gr64.rho_ref = s->grav_iso ? 0.0 : a / (double)N;
}

int log2_exact(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return (1 << l) == n ? l : -1;
}

// transform length of an axis of n cells: n on a periodic box, the next power
// of two >= 2 n on an isolated one
int grav_length(int n, bool iso) {
  if (!iso) return n;
  int m = 1;
  while (m < 2 * n) m <<= 1;
  return m;
}

// faces PERIODIC: 6 (periodic box), 0 (isolated box), else a mix
int periodic_faces(const csph_sim* s) {
  int np = 0;
  for (int f = 0; f < 6; ++f) np += s->bc.kind[f] == kPeriodic;
  return np;
}

// allocate and fill the Poisson solve's buffers and tables (once per sim); on
// failure the caller releases what was allocated (grav_release)
template <typename Real>
csph_status grav_setup(csph_sim* s) {
  Grav<Real>& gr = grav_of<Real>(s);
  const bool iso = periodic_faces(s) == 0;
  const int n[3] = {s->g.nx, s->g.ny, s->g.nz};
  int m[3];
  for (int a = 0; a < 3; ++a) m[a] = grav_length(n[a], iso);
  // work array [nz][my][mx] complex; isolated: the Green's function on
  // (mx/2+1)(my/2+1)(mz/2+1) frequencies
  const size_t octant = (size_t)(m[0] / 2 + 1) * (m[1] / 2 + 1) * (m[2] / 2 + 1);
  size_t off_tw[3], off_lam[3];
  size_t total = align_up((size_t)m[0] * m[1] * n[2] * 2 * sizeof(Real));
  const size_t off_ext = total;
  total += s->L.field_bytes;
  const size_t off_psih = total;
  total += s->L.field_bytes;
  const size_t off_khat = total;
  if (iso) total += align_up(octant * sizeof(Real));
  for (int a = 0; a < 3; ++a) {
    off_tw[a] = total;
    total += align_up((size_t)m[a] * 2 * sizeof(Real));
    off_lam[a] = total;
    total += align_up((size_t)m[a] * sizeof(double));  // isolated: cos(2 pi t / m) for the set-up
  }
  void* p = nullptr;
  if (hipMalloc(&p, total) != hipSuccess) {
    (void)hipGetLastError();
    return fail(CSPH_ERR_NOMEM, "hipMalloc of the self-gravity buffers failed");
  }
  s->gbuf = (char*)p;
  s->grav_iso = iso;
  gr.iso = iso ? 1 : 0;
  HIP_TRY(hipMemsetAsync(s->gbuf, 0, total, s->stream));
  const double kPi = 3.14159265358979323846;
  const double h2 = s->g.h * s->g.h;
  for (int a = 0; a < 3; ++a) {
    std::vector<Real> tw((size_t)m[a] * 2);
    std::vector<double> lam((size_t)m[a]);
    for (int k = 0; k < m[a]; ++k) {
      const double ang = 2.0 * kPi * k / m[a];
      tw[2 * (size_t)k] = (Real)std::cos(ang);
      tw[2 * (size_t)k + 1] = (Real)std::sin(ang);
      lam[k] = iso ? std::cos(ang) : (2.0 * std::cos(ang) - 2.0) / h2;
    }
    HIP_TRY(hipMemcpyAsync(s->gbuf + off_tw[a], tw.data(), tw.size() * sizeof(Real), hipMemcpyHostToDevice,
                           s->stream));
    HIP_TRY(hipMemcpyAsync(s->gbuf + off_lam[a], lam.data(), lam.size() * sizeof(double),
                           hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    gr.m[a] = m[a];
    gr.tw[a] = (const Real*)(s->gbuf + off_tw[a]);
    gr.lam[a] = iso ? nullptr : (const double*)(s->gbuf + off_lam[a]);
    gr.log2n[a] = log2_exact(m[a]);
    gr.fast[a] = Poisson<Real>::fast_ok(m[a], gr.log2n[a]) ? 1 : 0;
  }
  gr.cw = (Real*)s->gbuf;
  gr.psi_ext = (Real*)(s->gbuf + off_ext);
  gr.psih = (Real*)(s->gbuf + off_psih);
  gr.khat = iso ? (const Real*)(s->gbuf + off_khat) : nullptr;
  if (iso) {
    // the Green's function, through two FP64 octants of scratch
    double* tmp = nullptr;
    if (hipMalloc((void**)&tmp, 2 * octant * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(CSPH_ERR_NOMEM, "hipMalloc of the Green's function scratch failed");
    }
    const double* ctab[3];
    for (int a = 0; a < 3; ++a) ctab[a] = (const double*)(s->gbuf + off_lam[a]);
    hipError_t e = Poisson<Real>::green(gr, s->g.h, tmp, ctab, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(CSPH_ERR_DEVICE, std::string("the Green's function: ") + hipGetErrorString(e));
  }
  return CSPH_OK;
}

// the solve's device memory and tables released (after a failed set-up too)
template <typename Real>
void grav_release(csph_sim* s) {
  (void)hipStreamSynchronize(s->stream);
  if (s->gbuf) (void)hipFree(s->gbuf);
  s->gbuf = nullptr;
  s->grav_iso = false;
  grav_of<Real>(s) = Grav<Real>{};
}

template <typename Real>
csph_status grav_on(csph_sim* s, double G) {
  if (!s->gbuf) {
    csph_status st = grav_setup<Real>(s);
    if (st) {
      // a failure part-way leaves no half-built tables behind for the next call
      grav_release<Real>(s);
      return st;
    }
  }
  Grav<Real>& gr = grav_of<Real>(s);
  Fields<Real>& F = fields_of<Real>(s);
  const size_t N = (size_t)s->g.nx * s->g.ny * s->g.nz;
  gr.fpg_n = s->grav_iso ? G : 4.0 * 3.14159265358979323846 * G / (double)N;
  // the mean density of the current state
  Ctrl c{};
  csph_status st = read_ctrl(s, &c);
  if (st) return st;
  std::vector<double> rho(N);
  st = download_field<Real>(s, F.U[c.par][0], rho.data());
  if (st) return st;
  set_rho_ref(s, rho.data());
  // the external potential as set (zero if none)
  std::vector<double> ext(N, 0.0);
  if (s->has_psi) ext = s->psi_host;
  st = upload_field<Real>(s, gr.psi_ext, ext.data());
  if (st) return st;
  F.psic = gr.psih;
  s->g.psi = 1;
  s->grav = G;
  return CSPH_OK;
}

template <typename Real>
csph_status grav_off(csph_sim* s) {
  Fields<Real>& F = fields_of<Real>(s);
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->grav = 0.0;
  F.psic = F.psi;
  const size_t N = (size_t)s->g.nx * s->g.ny * s->g.nz;
  std::vector<double> ext(N, 0.0);
  if (s->has_psi) ext = s->psi_host;
  csph_status st = upload_field<Real>(s, F.psi, ext.data());
  if (st) return st;
  if (!s->has_psi) HIP_TRY(hipMemsetAsync(F.psis, 0, s->L.field_bytes, s->stream));
  s->g.psi = s->has_psi ? 1 : 0;
  s->psi_dirty = true;
  grav_release<Real>(s);
  return CSPH_OK;
}

bool periodic_pairs_ok(const csph_sim* s) {
  for (int ax = 0; ax < 3; ++ax)
    if ((s->bc.kind[2 * ax] == kPeriodic) != (s->bc.kind[2 * ax + 1] == kPeriodic)) return false;
  return true;
}

csph_status init_sim(csph_sim* s) {
  s->g = make_grid(&s->desc);
  const int tz0 = s->is_f64() ? Launch<double>::default_tz(s->g) : Launch<float>::default_tz(s->g);
  for (int q = 0; q < 3; ++q) s->tz[q] = tz0;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(s->device, s->desc));
    if (it != g_tune.end())
      for (int q = 0; q < 3; ++q) s->tz[q] = it->second[q];
  }
  s->tz_last = s->tz[2];
  for (int f = 0; f < 6; ++f) s->bc.kind[f] = kPeriodic;
  if (s->is_f64())
    bind_fields<double>(s, s->f64);
  else
    bind_fields<float>(s, s->f32);
  s->ctrl = (Ctrl*)(s->buf + s->L.ctrl_off);
  s->partials = (double*)(s->buf + s->L.partials_off);
  s->totals_dev = (double*)(s->buf + s->L.totals_off);
  // zero fields (psi = 0, state = 0) and the control block, on the device
  HIP_TRY(hipMemsetAsync(s->buf, 0, s->L.total, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return CSPH_OK;
}

}  // namespace

extern "C" {

const char* csph_last_error(void) { return g_err.c_str(); }

size_t csph_required_bytes(const csph_grid_desc* desc) {
  std::string why;
  if (!desc_ok(desc, &why)) return 0;
  return make_layout(desc).total;
}

// host_mem: storage for the simulation object (NULL: the heap)
static csph_status create_common(const csph_grid_desc* desc, void* stream, void* dev_buf,
                                 size_t bytes, csph_sim** out, void* host_mem = nullptr) {
  if (!out) return fail(CSPH_ERR_ARG, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!desc_ok(desc, &why)) return fail(CSPH_ERR_ARG, why);
  csph_sim* s = host_mem ? new (host_mem) csph_sim() : new (std::nothrow) csph_sim();
  if (!s) return fail(CSPH_ERR_NOMEM, "host allocation failed");
  auto drop = [&]() {
    if (host_mem) s->~csph_sim();
    else delete s;
  };
  s->desc = *desc;
  s->stream = (hipStream_t)stream;
  s->L = make_layout(desc);
  if (hipGetDevice(&s->device) != hipSuccess) {
    drop();
    return fail(CSPH_ERR_DEVICE, "hipGetDevice failed");
  }
  if (dev_buf) {
    if (bytes < s->L.total) {
      drop();
      return fail(CSPH_ERR_ARG, "caller buffer smaller than csph_required_bytes");
    }
    if ((uintptr_t)dev_buf % kAlign) {
      drop();
      return fail(CSPH_ERR_ARG, "caller buffer must be 256-byte aligned");
    }
    s->buf = (char*)dev_buf;
    s->owned = false;
  } else {
    void* p = nullptr;
    if (hipMalloc(&p, s->L.total) != hipSuccess) {
      (void)hipGetLastError();
      drop();
      return fail(CSPH_ERR_NOMEM, "hipMalloc failed");
    }
    s->buf = (char*)p;
    s->owned = true;
  }
  csph_status st = init_sim(s);
  if (st) {
    if (s->owned) (void)hipFree(s->buf);
    drop();
    return st;
  }
  *out = s;
  return CSPH_OK;
}

csph_status csph_create(const csph_grid_desc* desc, void* hip_stream, csph_sim** out) {
  return create_common(desc, hip_stream, nullptr, 0, out);
}

csph_status csph_create_in(const csph_grid_desc* desc, void* hip_stream, void* dev_buf,
                           size_t bytes, csph_sim** out) {
  if (!dev_buf) return fail(CSPH_ERR_ARG, "dev_buf is NULL");
  return create_common(desc, hip_stream, dev_buf, bytes, out);
}

csph_status csph_create_static(const csph_grid_desc* desc, void* hip_stream, csph_sim** out) {
  if (!out) return fail(CSPH_ERR_ARG, "out is NULL");
  *out = nullptr;
  const size_t need = csph_required_bytes(desc);
  if (need == 0) {
    std::string why;
    desc_ok(desc, &why);
    return fail(CSPH_ERR_ARG, why);
  }
  if (need > CSPH_STATIC_BYTES)
    return fail(CSPH_ERR_ARG, "grid needs " + std::to_string(need) + " device bytes; the static array holds " +
                                  std::to_string((size_t)CSPH_STATIC_BYTES));
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CSPH_ERR_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_static_mu);
  StaticSlot& slot = g_static[dev];
  if (slot.in_use)
    return fail(CSPH_ERR_STATE, "the static array of this GPU holds another simulation: destroy it first");
  if (!slot.dev) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(CSPH_ERR_DEVICE, "hipGetSymbolAddress of the static array failed");
    }
    slot.dev = p;
  }
  csph_status st = create_common(desc, hip_stream, slot.dev, CSPH_STATIC_BYTES, out, slot.host);
  if (st) return st;
  (*out)->in_static = true;
  slot.in_use = true;
  return CSPH_OK;
}

csph_status csph_destroy(csph_sim* s) {
  if (!s) return CSPH_OK;
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: remove it from the batch first");
  (void)hipStreamSynchronize(s->stream);
  for (hipEvent_t e : s->prof_ev) (void)hipEventDestroy(e);
  if (s->owned) (void)hipFree(s->buf);
  if (s->gbuf) (void)hipFree(s->gbuf);
  if (s->srcbuf) (void)hipFree(s->srcbuf);
  if (s->in_static) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    const int dev = s->device;
    s->~csph_sim();
    g_static[dev].in_use = false;
    return CSPH_OK;
  }
  delete s;
  return CSPH_OK;
}

csph_status csph_set_stream(csph_sim* s, void* hip_stream) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: remove it from the batch first");
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->stream = (hipStream_t)hip_stream;
  return CSPH_OK;
}

csph_status csph_set_state(csph_sim* s, csph_vars vars, const double* host) {
  if (!s || !host) return fail(CSPH_ERR_ARG, "sim or host array is NULL");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: remove it from the batch first");
  if (vars != CSPH_CONSERVED && vars != CSPH_PRIMITIVE) return fail(CSPH_ERR_ARG, "bad vars");
  const size_t N = (size_t)s->g.nx * s->g.ny * s->g.nz;
  std::vector<double> cons;
  const double* src = host;
  for (size_t q = 0; q < N; ++q)
    if (!(host[q] >= 0.0)) return fail(CSPH_ERR_ARG, "density must be >= 0");
  if (vars == CSPH_PRIMITIVE) {
    cons.resize(5 * N);
    const double gm1 = s->desc.gamma - 1.0;
    for (size_t q = 0; q < N; ++q) {
      const double r = host[q], ux = host[N + q], uy = host[2 * N + q], uz = host[3 * N + q],
                   p = host[4 * N + q];
      if (!(p >= 0.0)) return fail(CSPH_ERR_ARG, "pressure must be >= 0");
      cons[q] = r;
      cons[N + q] = r * ux;
      cons[2 * N + q] = r * uy;
      cons[3 * N + q] = r * uz;
      cons[4 * N + q] = p / gm1 + 0.5 * r * (ux * ux + uy * uy + uz * uz);
    }
    src = cons.data();
  }
  csph_status st = s->is_f64() ? set_state_t<double>(s, src) : set_state_t<float>(s, src);
  if (st) return st;
  if (s->grav > 0.0) set_rho_ref(s, src);
  Ctrl c{};
  Ctrl old{};
  st = read_ctrl(s, &old);
  if (st) return st;
  c.t = old.t;
  c.nsteps = old.nsteps;
  c.step_limit = old.step_limit;
  c.t_end = old.t_end;
  st = write_ctrl(s, c);
  if (st) return st;
  s->need_smax = true;
  s->x_stale = true;
  s->stepped = false;
  return CSPH_OK;
}

// the state was changed from the host: ghosts, signal speed and totals are stale
static void state_changed(csph_sim* s) {
  s->need_smax = true;
  s->x_stale = true;
  s->stepped = false;
}

csph_status csph_fill_state(csph_sim* s, csph_vars vars, const double state[5]) {
  if (!s || !state) return fail(CSPH_ERR_ARG, "sim or state is NULL");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: remove it from the batch first");
  if (vars != CSPH_CONSERVED && vars != CSPH_PRIMITIVE) return fail(CSPH_ERR_ARG, "bad vars");
  double st[5];
  for (int v = 0; v < 5; ++v) st[v] = state[v];
  if (!(st[0] >= 0.0)) return fail(CSPH_ERR_ARG, "density must be >= 0");
  if (vars == CSPH_PRIMITIVE) {
    csph_status e = to_conserved(s->desc.gamma, st, 1, 1);
    if (e) return e;
  }
  for (int v = 0; v < 5; ++v) {
    if (!std::isfinite(st[v])) return fail(CSPH_ERR_ARG, "state must be finite");
    HIP_TRY(s->is_f64() ? Launch<double>::fill_const(s->f64.U[0][v], st[v], s->g.ncell, s->stream)
                        : Launch<float>::fill_const(s->f32.U[0][v], st[v], s->g.ncell, s->stream));
  }
  HIP_TRY(hipStreamSynchronize(s->stream));
  Ctrl c{}, old{};
  csph_status e = read_ctrl(s, &old);
  if (e) return e;
  c.t = old.t;
  c.nsteps = old.nsteps;
  c.step_limit = old.step_limit;
  c.t_end = old.t_end;
  e = write_ctrl(s, c);
  if (e) return e;
  if (s->grav > 0.0 && !s->grav_iso) s->gr32.rho_ref = s->gr64.rho_ref = st[0];  // the uniform density
  state_changed(s);
  return CSPH_OK;
}

csph_status csph_set_state_box(csph_sim* s, csph_vars vars, const int32_t lo[3], const int32_t n[3],
                               const double* host) {
  if (!s || !host) return fail(CSPH_ERR_ARG, "sim or host array is NULL");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: remove it from the batch first");
  if (vars != CSPH_CONSERVED && vars != CSPH_PRIMITIVE) return fail(CSPH_ERR_ARG, "bad vars");
  if (!box_ok(s, lo, n)) return fail(CSPH_ERR_ARG, "box outside the interior");
  const size_t M = (size_t)n[0] * n[1] * n[2];
  std::vector<double> st(host, host + 5 * M);
  for (size_t q = 0; q < M; ++q)
    if (!(st[q] >= 0.0)) return fail(CSPH_ERR_ARG, "density must be >= 0");
  if (vars == CSPH_PRIMITIVE) {
    csph_status e = to_conserved(s->desc.gamma, st.data(), M, M);
    if (e) return e;
  }
  Ctrl c{};
  csph_status e = read_ctrl(s, &c);
  if (e) return e;
  for (int v = 0; v < 5; ++v) {
    e = s->is_f64() ? box_upload<double>(s, s->f64.U[c.par][v], lo, n, st.data() + (size_t)v * M)
                    : box_upload<float>(s, s->f32.U[c.par][v], lo, n, st.data() + (size_t)v * M);
    if (e) return e;
  }
  // the sticky error bits and the signal-speed maximum describe the old state
  c.status = 0;
  c.smax_valid = 0;
  c.smax_bits[c.cur] = 0ULL;
  e = write_ctrl(s, c);
  if (e) return e;
  state_changed(s);
  return CSPH_OK;
}

csph_status csph_get_state_box(const csph_sim* s, csph_vars vars, const int32_t lo[3], const int32_t n[3],
                               double* out) {
  if (!s || !out) return fail(CSPH_ERR_ARG, "sim or output is NULL");
  if (vars != CSPH_CONSERVED && vars != CSPH_PRIMITIVE) return fail(CSPH_ERR_ARG, "bad vars");
  if (!box_ok(s, lo, n)) return fail(CSPH_ERR_ARG, "box outside the interior");
  Ctrl c{};
  csph_status e = read_ctrl(s, &c);
  if (e) return e;
  const size_t M = (size_t)n[0] * n[1] * n[2];
  for (int v = 0; v < 5; ++v) {
    e = s->is_f64() ? box_download<double>(s, s->f64.U[c.par][v], lo, n, out + (size_t)v * M)
                    : box_download<float>(s, s->f32.U[c.par][v], lo, n, out + (size_t)v * M);
    if (e) return e;
  }
  if (vars == CSPH_PRIMITIVE) {
    const double gm1 = s->desc.gamma - 1.0;
    for (size_t q = 0; q < M; ++q) {
      const double r = out[q];
      double u[3] = {0.0, 0.0, 0.0};
      if (r > s->desc.rho_vac)
        for (int d = 0; d < 3; ++d) u[d] = out[(1 + d) * M + q] / r;
      const double ke = 0.5 * (out[M + q] * u[0] + out[2 * M + q] * u[1] + out[3 * M + q] * u[2]);
      const double p = gm1 * (out[4 * M + q] - ke);
      for (int d = 0; d < 3; ++d) out[(1 + d) * M + q] = u[d];
      out[4 * M + q] = p > 0.0 ? p : 0.0;
    }
  }
  return CSPH_OK;
}

csph_status csph_set_potential(csph_sim* s, const double* host_psi) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: remove it from the batch first");
  const size_t N = (size_t)s->g.nx * s->g.ny * s->g.nz;
  s->has_psi = host_psi != nullptr;
  s->psi_host.assign(N, 0.0);
  if (host_psi) std::memcpy(s->psi_host.data(), host_psi, N * sizeof(double));
  csph_status st = s->is_f64() ? upload_field<double>(s, s->f64.psi, s->psi_host.data())
                            : upload_field<float>(s, s->f32.psi, s->psi_host.data());
  if (st) return st;
  if (s->grav > 0.0) {
    // self-gravity: this is the external part; the step adds the gas's own
    st = s->is_f64() ? upload_field<double>(s, s->gr64.psi_ext, s->psi_host.data())
                     : upload_field<float>(s, s->gr32.psi_ext, s->psi_host.data());
    if (st) return st;
    s->psi_dirty = true;
    return CSPH_OK;
  }
  if (!host_psi && s->g.psi) {
    // without a potential the kernels leave psi(r*) alone: it must be 0 everywhere
    void* f = s->is_f64() ? (void*)s->f64.psis : (void*)s->f32.psis;
    HIP_TRY(hipMemsetAsync(f, 0, s->L.field_bytes, s->stream));
  }
  s->g.psi = host_psi ? 1 : 0;
  s->psi_dirty = true;
  return CSPH_OK;
}

csph_status csph_set_boundary(csph_sim* s, int32_t face, csph_bc kind, const double inflow_prim[5]) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: remove it from the batch first");
  if (face < 0 || face > 5) return fail(CSPH_ERR_ARG, "face must be 0..5");
  if (kind < CSPH_PERIODIC || kind > CSPH_REFLECT) return fail(CSPH_ERR_ARG, "bad boundary kind");
  if (s->grav > 0.0 && (kind == CSPH_PERIODIC) == s->grav_iso)
    return fail(CSPH_ERR_ARG, s->grav_iso ? "self-gravity on an isolated box: no face may become PERIODIC"
                                          : "self-gravity on a periodic box: every face stays PERIODIC");
  s->bc.kind[face] = (int)kind;
  if (kind == CSPH_INFLOW) {
    if (!inflow_prim) return fail(CSPH_ERR_ARG, "inflow state required");
    const double r = inflow_prim[0], ux = inflow_prim[1], uy = inflow_prim[2], uz = inflow_prim[3],
                 p = inflow_prim[4];
    if (!(r >= 0.0) || !(p >= 0.0)) return fail(CSPH_ERR_ARG, "inflow rho and p must be >= 0");
    for (int v = 0; v < 5; ++v) s->inflow_prim[face][v] = inflow_prim[v];
    s->bc.cons[face][0] = r;
    s->bc.cons[face][1] = r * ux;
    s->bc.cons[face][2] = r * uy;
    s->bc.cons[face][3] = r * uz;
    s->bc.cons[face][4] = p / (s->desc.gamma - 1.0) + 0.5 * r * (ux * ux + uy * uy + uz * uz);
    s->bc.vel[face][0] = ux;
    s->bc.vel[face][1] = uy;
    s->bc.vel[face][2] = uz;
    s->bc.phi[face] = inflow_phi(s->bc.cons[face], s->desc.gamma, s->desc.rho_vac);
  }
  s->psi_dirty = true;
  s->x_stale = true;
  return CSPH_OK;
}

csph_status csph_step(csph_sim* s, double dt_max, double* dt_taken) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: advance the batch");
  if (!periodic_pairs_ok(s)) return fail(CSPH_ERR_ARG, "PERIODIC must be set on both faces of an axis");
  Ctrl c{};
  // a step always runs (no end time): clear the completion flag of earlier advances
  csph_status st = read_ctrl(s, &c);
  if (st) return st;
  if (c.status) return fail(CSPH_ERR_STATE, "sticky error: call csph_set_state");
  if (c.done) {
    c.done = 0;
    st = write_ctrl(s, c);
    if (st) return st;
  }
  st = launch(s, 1, dt_max, INFINITY);
  if (st) return st;
  if (dt_taken) {
    st = read_ctrl(s, &c);
    if (st) return st;
    if (c.status) return status_from_bits(c.status);
    *dt_taken = c.dt;
  }
  return CSPH_OK;
}

csph_status csph_advance(csph_sim* s, double t_end, int64_t max_steps, int64_t* steps_taken) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: advance the batch");
  if (!periodic_pairs_ok(s)) return fail(CSPH_ERR_ARG, "PERIODIC must be set on both faces of an axis");
  if (max_steps < 0) return fail(CSPH_ERR_ARG, "max_steps must be >= 0");
  if (std::isnan(t_end)) return fail(CSPH_ERR_ARG, "t_end is NaN");
  Ctrl c{};
  csph_status st = read_ctrl(s, &c);
  if (st) return st;
  if (c.status) return fail(CSPH_ERR_STATE, "sticky error: call csph_set_state");
  const long long n0 = c.nsteps;
  if (c.done) {
    c.done = 0;
    st = write_ctrl(s, c);
    if (st) return st;
  }
  int64_t left = max_steps;
  int chunk = 4;
  while (left > 0) {
    const int n = (int)std::min<int64_t>(left, chunk);
    st = launch(s, n, 0.0, t_end);
    if (st) return st;
    left -= n;
    st = read_ctrl(s, &c);
    if (st) return st;
    if (c.status || c.done) break;
    chunk = std::min(chunk * 2, 64);
  }
  if (steps_taken) *steps_taken = c.nsteps - n0;
  if (c.status) return status_from_bits(c.status);
  return CSPH_OK;
}

csph_status csph_get_state(const csph_sim* s, csph_vars vars, double* out) {
  if (!s || !out) return fail(CSPH_ERR_ARG, "sim or output is NULL");
  if (vars != CSPH_CONSERVED && vars != CSPH_PRIMITIVE) return fail(CSPH_ERR_ARG, "bad vars");
  Ctrl c{};
  csph_status st = read_ctrl(s, &c);
  if (st) return st;
  const size_t N = (size_t)s->g.nx * s->g.ny * s->g.nz;
  for (int v = 0; v < 5; ++v) {
    st = s->is_f64() ? download_field<double>(s, s->f64.U[c.par][v], out + (size_t)v * N)
                  : download_field<float>(s, s->f32.U[c.par][v], out + (size_t)v * N);
    if (st) return st;
  }
  if (vars == CSPH_PRIMITIVE) {
    const double gm1 = s->desc.gamma - 1.0;
    for (size_t q = 0; q < N; ++q) {
      const double r = out[q];
      double u[3] = {0.0, 0.0, 0.0};
      if (r > s->desc.rho_vac)
        for (int d = 0; d < 3; ++d) u[d] = out[(1 + d) * N + q] / r;
      const double ke = 0.5 * (out[N + q] * u[0] + out[2 * N + q] * u[1] + out[3 * N + q] * u[2]);
      const double p = gm1 * (out[4 * N + q] - ke);
      for (int d = 0; d < 3; ++d) out[(1 + d) * N + q] = u[d];
      out[4 * N + q] = p > 0.0 ? p : 0.0;
    }
  }
  return CSPH_OK;
}

csph_status csph_get_time(const csph_sim* s, double* t, int64_t* nsteps) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  Ctrl c{};
  csph_status st = read_ctrl(s, &c);
  if (st) return st;
  if (t) *t = c.t;
  if (nsteps) *nsteps = c.nsteps;
  return CSPH_OK;
}

csph_status csph_set_time(csph_sim* s, double t, int64_t nsteps) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: remove it from the batch first");
  if (!std::isfinite(t) || nsteps < 0) return fail(CSPH_ERR_ARG, "bad time or step count");
  Ctrl c{};
  csph_status st = read_ctrl(s, &c);
  if (st) return st;
  c.t = t;
  c.nsteps = nsteps;
  c.done = 0;
  return write_ctrl(s, c);
}

csph_status csph_totals(const csph_sim* s, double out[5]) {
  if (!s || !out) return fail(CSPH_ERR_ARG, "sim or output is NULL");
  if (!s->stepped) {
    // no step since the state was set: sum the state on the host
    const size_t N = (size_t)s->g.nx * s->g.ny * s->g.nz;
    std::vector<double> U(5 * N);
    csph_status st = csph_get_state(s, CSPH_CONSERVED, U.data());
    if (st) return st;
    for (int v = 0; v < 5; ++v) {
      double a = 0.0;
      for (size_t q = 0; q < N; ++q) a += U[(size_t)v * N + q];
      out[v] = a * s->g.h3;
    }
    return CSPH_OK;
  }
  csph_status stw = wait_batch(s);
  if (stw) return stw;
  const int nt = s->is_f64() ? Launch<double>::tiles(s->g, s->tz_last) : Launch<float>::tiles(s->g, s->tz_last);
  HIP_TRY(s->is_f64() ? Launch<double>::totals(s->g, s->partials, nt, s->totals_dev, s->stream)
                   : Launch<float>::totals(s->g, s->partials, nt, s->totals_dev, s->stream));
  HIP_TRY(hipMemcpyAsync(out, s->totals_dev, 5 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return CSPH_OK;
}

csph_status csph_get_stage(const csph_sim* s, int32_t which, double* out) {
  if (!s || !out) return fail(CSPH_ERR_ARG, "sim or output is NULL");
  if (which < 0 || which > 16) return fail(CSPH_ERR_ARG, "which must be 0..16");
  if (which == 15)
    return s->is_f64() ? download_field<double>(s, s->f64.psi, out) : download_field<float>(s, s->f32.psi, out);
  if (which == 16) {
    if (!(s->grav > 0.0)) return fail(CSPH_ERR_ARG, "the potential of the predicted density needs self-gravity");
    return s->is_f64() ? download_field<double>(s, s->gr64.psih, out) : download_field<float>(s, s->gr32.psih, out);
  }
  if (which == 14)
    return s->is_f64() ? download_field<double>(s, s->f64.phs, out) : download_field<float>(s, s->f32.phs, out);
  if (s->is_f64()) {
    const double* src = which < 4 ? s->f64.ms[which] : which < 7 ? s->f64.xs[which - 4]
                      : which < 11 ? s->f64.mt[which - 7] : s->f64.xt[which - 11];
    return download_field<double>(s, src, out);
  }
  if ((which >= 4 && which < 7) || which >= 11)
    return fail(CSPH_ERR_ARG, "the FP32 build does not store xi* or xi^{n+1} (they are recomputed where needed)");
  const float* src = which < 4 ? s->f32.ms[which] : s->f32.mt[which - 7];
  return download_field<float>(s, src, out);
}

csph_status csph_profile_enable(csph_sim* s, int32_t on) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  if (on && s->prof_ev.empty()) {
    s->prof_ev.resize((size_t)csph_sim::kProfSteps * csph_sim::kEv);
    for (auto& e : s->prof_ev) HIP_TRY(hipEventCreate(&e));
  }
  if (!on) {
    csph_status st = prof_collect(s);
    if (st) return st;
  }
  s->prof_on = on != 0;
  for (int q = 0; q < 6; ++q) {
    s->prof_ms[q] = 0.0;
    s->prof_n[q] = 0;
  }
  s->prof_pending = 0;
  return CSPH_OK;
}

csph_status csph_profile_read(csph_sim* s, double* avg_ms, int64_t* launches, int32_t n) {
  if (!s || n < 0 || n > 6) return fail(CSPH_ERR_ARG, "bad arguments");
  csph_status st = prof_collect(s);
  if (st) return st;
  for (int q = 0; q < n; ++q) {
    const int64_t cnt = q == 3 ? 3 * s->prof_n[q] : s->prof_n[q];
    if (avg_ms) avg_ms[q] = cnt ? s->prof_ms[q] / (double)cnt : 0.0;
    if (launches) launches[q] = cnt;
  }
  return CSPH_OK;
}

csph_status csph_set_scheme(csph_sim* s, csph_limiter limiter, csph_flux flux) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  if (limiter < CSPH_LIM_MINMOD || limiter > CSPH_LIM_SUPERBEE) return fail(CSPH_ERR_ARG, "bad limiter");
  if (flux < CSPH_FLUX_SWEPT || flux > CSPH_FLUX_SWEPT_AV) return fail(CSPH_ERR_ARG, "bad flux");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: remove it first");
  s->g.limiter = (int)limiter;
  s->g.flux = (int)flux;
  return CSPH_OK;
}

csph_status csph_set_viscosity(csph_sim* s, double nu) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  if (!(nu >= 0.0) || !std::isfinite(nu)) return fail(CSPH_ERR_ARG, "nu must be finite and >= 0");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: remove it first");
  set_viscosity(s->g, nu);
  return CSPH_OK;
}

csph_status csph_set_self_gravity(csph_sim* s, double G) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  if (!(G >= 0.0) || !std::isfinite(G)) return fail(CSPH_ERR_ARG, "G must be finite and >= 0");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: remove it first");
  if (G == 0.0) {
    if (!(s->grav > 0.0)) return CSPH_OK;
    return s->is_f64() ? grav_off<double>(s) : grav_off<float>(s);
  }
  const int np = periodic_faces(s);
  if (np != 0 && np != 6)
    return fail(CSPH_ERR_ARG, "self-gravity needs PERIODIC on all six faces (a periodic box) or on none "
                              "(an isolated box)");
  if (s->in_static && !s->gbuf)
    return fail(CSPH_ERR_ARG, "self-gravity allocates its own device memory: not available to a static simulation");
  const int n[3] = {s->g.nx, s->g.ny, s->g.nz};
  for (int a = 0; a < 3; ++a) {
    const int m = grav_length(n[a], np == 0);
    const int l = log2_exact(m);
    const bool ok = s->is_f64() ? Poisson<double>::length_ok(m, l) : Poisson<float>::length_ok(m, l);
    if (!ok)
      return fail(CSPH_ERR_ARG, "self-gravity: axis length " + std::to_string(n[a]) +
                                    (np == 0 ? " unsupported on an isolated box (up to 2048 in FP32 and 1024 in FP64)"
                                             : " unsupported (a power of two up to 4096 in FP32 and 2048 in "
                                               "FP64, or any length up to 1024)"));
  }
  return s->is_f64() ? grav_on<double>(s, G) : grav_on<float>(s, G);
}

csph_status csph_set_source(csph_sim* s, const double* host_q, double eps) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: remove it first");
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (!host_q) {
    if (s->srcbuf) (void)hipFree(s->srcbuf);
    s->srcbuf = nullptr;
    s->f32.src = nullptr;
    s->f64.src = nullptr;
    s->g.eps_src = 0.0;
    return CSPH_OK;
  }
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(CSPH_ERR_ARG, "eps must be finite and >= 0");
  const size_t N = (size_t)s->g.nx * s->g.ny * s->g.nz;
  for (size_t q = 0; q < N; ++q)
    if (!std::isfinite(host_q[q])) return fail(CSPH_ERR_ARG, "source rates must be finite");
  if (!s->srcbuf) {
    if (s->in_static)
      return fail(CSPH_ERR_ARG, "sources allocate a device field: not available to a static simulation");
    void* p = nullptr;
    if (hipMalloc(&p, s->L.field_bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(CSPH_ERR_NOMEM, "hipMalloc of the source field failed");
    }
    s->srcbuf = (char*)p;
    HIP_TRY(hipMemsetAsync(s->srcbuf, 0, s->L.field_bytes, s->stream));
  }
  csph_status st = s->is_f64() ? upload_field<double>(s, (double*)s->srcbuf, host_q)
                               : upload_field<float>(s, (float*)s->srcbuf, host_q);
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (s->is_f64())
    s->f64.src = (double*)s->srcbuf;
  else
    s->f32.src = (float*)s->srcbuf;
  s->g.eps_src = eps;
  return CSPH_OK;
}

csph_status csph_get_scheme(const csph_sim* s, int32_t* limiter, int32_t* flux) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  if (limiter) *limiter = s->g.limiter;
  if (flux) *flux = s->g.flux;
  return CSPH_OK;
}

csph_status csph_set_tile_depths(csph_sim* s, const int32_t tz[3]) {
  if (!s || !tz) return fail(CSPH_ERR_ARG, "sim or tz is NULL");
  for (int q = 0; q < 3; ++q)
    if (tz[q] < kTzMin || tz[q] > kTzMax) return fail(CSPH_ERR_ARG, "tile depth must be in [2, 64]");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: remove it first");
  for (int q = 0; q < 3; ++q) s->tz[q] = tz[q];
  return CSPH_OK;
}

csph_status csph_set_tile_depth(csph_sim* s, int32_t tz) {
  const int32_t all[3] = {tz, tz, tz};
  return csph_set_tile_depths(s, all);
}

csph_status csph_get_tile_depths(const csph_sim* s, int32_t tz[3]) {
  if (!s || !tz) return fail(CSPH_ERR_ARG, "sim or tz is NULL");
  for (int q = 0; q < 3; ++q) tz[q] = s->tz[q];
  return CSPH_OK;
}

}  // extern "C"

namespace {

// event-timed wall of `fn` on `stream`, in milliseconds
template <typename Fn>
csph_status time_on(hipStream_t stream, Fn fn, double* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(CSPH_ERR_DEVICE, "hipEventCreate failed");
  }
  csph_status st = CSPH_OK;
  if (hipEventRecord(e0, stream) != hipSuccess) st = fail(CSPH_ERR_DEVICE, "hipEventRecord failed");
  if (!st) st = fn();
  if (!st && hipEventRecord(e1, stream) != hipSuccess) st = fail(CSPH_ERR_DEVICE, "hipEventRecord failed");
  if (!st && hipEventSynchronize(e1) != hipSuccess) st = fail(CSPH_ERR_DEVICE, "hipEventSynchronize failed");
  float f = 0.0f;
  if (!st && hipEventElapsedTime(&f, e0, e1) != hipSuccess) st = fail(CSPH_ERR_DEVICE, "hipEventElapsedTime failed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = f;
  return st;
}

// a library-owned copy of `s` (same description, boundaries, potential, state
// and time), for trial runs that must not disturb `s`
csph_status clone_sim(const csph_sim* s, csph_sim** out) {
  *out = nullptr;
  csph_sim* t = new (std::nothrow) csph_sim();
  if (!t) return fail(CSPH_ERR_NOMEM, "host allocation failed");
  t->desc = s->desc;
  t->stream = s->stream;
  t->L = s->L;
  t->device = s->device;
  t->g = s->g;
  t->bc = s->bc;
  std::memcpy(t->inflow_prim, s->inflow_prim, sizeof(t->inflow_prim));
  t->psi_dirty = s->psi_dirty;
  t->need_smax = s->need_smax;
  t->x_stale = s->x_stale;
  for (int q = 0; q < 3; ++q) t->tz[q] = s->tz[q];
  t->tz_last = s->tz_last;
  t->has_psi = s->has_psi;
  void* p = nullptr;
  if (hipMalloc(&p, s->L.total) != hipSuccess) {
    (void)hipGetLastError();
    delete t;
    return fail(CSPH_ERR_NOMEM, "hipMalloc of the trial copy failed");
  }
  t->buf = (char*)p;
  t->owned = true;
  if (t->is_f64())
    bind_fields<double>(t, t->f64);
  else
    bind_fields<float>(t, t->f32);
  t->ctrl = (Ctrl*)(t->buf + t->L.ctrl_off);
  t->partials = (double*)(t->buf + t->L.partials_off);
  t->totals_dev = (double*)(t->buf + t->L.totals_off);
  if (hipMemcpyAsync(t->buf, s->buf, s->L.total, hipMemcpyDeviceToDevice, s->stream) != hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess) {
    (void)hipFree(t->buf);
    delete t;
    return fail(CSPH_ERR_DEVICE, "copy of the state for the trial runs failed");
  }
  *out = t;
  return CSPH_OK;
}

// candidate depths worth trying on a grid of nz planes (deeper tiles than the
// grid add nothing)
std::vector<int> tz_candidates(int nz) {
  std::vector<int> c;
  for (int tz : kTzCand) {
    c.push_back(tz);
    if (tz >= nz) break;
  }
  return c;
}

}  // namespace

extern "C" {

csph_status csph_autotune(csph_sim* s, int32_t trial_steps, int32_t tz_out[3], double* ms_per_step) {
  if (!s) return fail(CSPH_ERR_ARG, "sim is NULL");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim is a batch member: tune the batch");
  if (trial_steps < 1 || trial_steps > 1000) return fail(CSPH_ERR_ARG, "trial_steps must be in [1, 1000]");
  if (!periodic_pairs_ok(s)) return fail(CSPH_ERR_ARG, "PERIODIC must be set on both faces of an axis");
  Ctrl c{};
  csph_status st = read_ctrl(s, &c);
  if (st) return st;
  if (c.status) return fail(CSPH_ERR_STATE, "sticky error: call csph_set_state");
  // ghosts of psi and the first dt are made once on the original, then copied
  st = s->is_f64() ? prepare<double>(s) : prepare<float>(s);
  if (st) return st;
  csph_sim* t = nullptr;
  st = clone_sim(s, &t);
  if (st) return st;
  Ctrl c0{};
  st = read_ctrl(t, &c0);
  c0.done = 0;
  // each stage's kernels are timed on their own (HIP events around every
  // launch), so one sweep over the candidate depths picks each stage's best
  int best[3] = {s->tz[0], s->tz[1], s->tz[2]};
  double best_ms[3] = {INFINITY, INFINITY, INFINITY};
  // trial_steps steps from the starting state at the current depths; with
  // `stages`, the per-stage average kernel times
  auto trial = [&](double* ms, double stages[3]) -> csph_status {
    for (int rep = 0; rep < 2; ++rep) {
      // one untimed step (first use of this launch shape), then the timed ones,
      // each from the same starting state
      if (hipMemcpyAsync(t->buf, s->buf, s->L.total, hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
        return fail(CSPH_ERR_DEVICE, "copy of the state for a trial run failed");
      csph_status e = write_ctrl(t, c0);
      if (!e && stages && rep == 1) e = csph_profile_enable(t, 1);
      if (e) return e;
      const int n = rep == 0 ? 1 : trial_steps;
      e = time_on(t->stream, [&]() { return launch(t, n, 0.0, INFINITY); }, ms);
      if (e) return e;
    }
    if (stages) {
      double avg[5];
      int64_t cnt[5];
      csph_status e = csph_profile_read(t, avg, cnt, 5);
      if (!e) e = csph_profile_enable(t, 0);
      if (e) return e;
      for (int q = 0; q < 3; ++q) stages[q] = avg[q];
    }
    return CSPH_OK;
  };
  for (int tz : tz_candidates(s->g.nz)) {
    if (st) break;
    for (int q = 0; q < 3; ++q) t->tz[q] = tz;
    double ms = 0.0, stages[3];
    st = trial(&ms, stages);
    if (st) break;
    Ctrl ct{};
    st = read_ctrl(t, &ct);
    if (st) break;
    if (ct.status) continue;  // an invalid trial (the state failed) does not count
    for (int q = 0; q < 3; ++q)
      if (stages[q] < best_ms[q]) {
        best_ms[q] = stages[q];
        best[q] = tz;
      }
  }
  // the step time at the chosen depths
  double step_ms = INFINITY;
  if (!st) {
    for (int q = 0; q < 3; ++q) t->tz[q] = best[q];
    double ms = 0.0;
    st = trial(&ms, nullptr);
    if (!st) step_ms = ms / trial_steps;
  }
  (void)hipStreamSynchronize(t->stream);
  for (hipEvent_t e : t->prof_ev) (void)hipEventDestroy(e);
  (void)hipFree(t->buf);
  delete t;
  if (st) return st;
  for (int q = 0; q < 3; ++q) s->tz[q] = best[q];
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(s->device, s->desc)] = Depths{best[0], best[1], best[2]};
  }
  if (tz_out)
    for (int q = 0; q < 3; ++q) tz_out[q] = best[q];
  if (ms_per_step) *ms_per_step = step_ms;
  return CSPH_OK;
}

// batches are implemented below

}  // extern "C"

// ====================================================================== batches
namespace {

struct Member {
  csph_sim* sim = nullptr;
  bool used = false;
};

}  // namespace

struct csph_batch {
  int dtype = CSPH_F32;
  hipStream_t stream = nullptr;
  size_t budget = 0, used_bytes = 0;
  std::vector<Member> slots;
  // device table of the members in slot order (built on change)
  void* table = nullptr;
  int2* tile_map = nullptr;   // flattened tile -> (table row, tile of that member)
  int2* fill_map = nullptr;   // ghost-fill block -> (table row, first ghost cell)
  int* flags = nullptr;
  size_t cap = 0, tile_cap = 0, fill_cap = 0;
  std::vector<int> order;  // table row -> slot
  int total_tiles = 0;
  int fill_blocks = 0;
  bool generic = false;  // a member uses a non-default scheme (generic stage-E kernel)
  bool viscous = false;  // a member has a viscosity (viscous form of the Lagrangian sweeps)
  bool dirty = true;
  // a captured k-step graph, replayed while membership does not change
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_k = 0;
  bool own_stream = false;
};

namespace {

void drop_graph(csph_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_k = 0;
}

// grow a device array to at least `need` elements (contents not kept)
template <typename T>
csph_status ensure(T** p, size_t* cap, size_t need) {
  if (need <= *cap && *p) return CSPH_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  const size_t c = std::max<size_t>(64, 2 * need);
  if (hipMalloc((void**)p, c * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    *cap = 0;
    return fail(CSPH_ERR_NOMEM, "batch table allocation failed");
  }
  *cap = c;
  return CSPH_OK;
}

template <typename Real>
csph_status build_table(csph_batch* b) {
  b->order.clear();
  for (size_t q = 0; q < b->slots.size(); ++q)
    if (b->slots[q].used) b->order.push_back((int)q);
  const size_t n = b->order.size();
  if (n > b->cap || !b->table) {
    if (b->table) (void)hipFree(b->table);
    if (b->flags) (void)hipFree(b->flags);
    b->table = nullptr;
    b->flags = nullptr;
    size_t cap = std::max<size_t>(64, 2 * n);
    if (hipMalloc(&b->table, cap * sizeof(Inst<Real>)) != hipSuccess ||
        hipMalloc((void**)&b->flags, cap * sizeof(int)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(CSPH_ERR_NOMEM, "batch table allocation failed");
    }
    b->cap = cap;
  }
  std::vector<Inst<Real>> tab(n);
  std::vector<int2> tmap, fmap;
  b->generic = false;
  b->viscous = false;
  for (size_t r = 0; r < n; ++r) {
    csph_sim* s = b->slots[b->order[r]].sim;
    Inst<Real>& I = tab[r];
    I.F = fields_of<Real>(s);
    I.g = s->g;
    I.bc = s->bc;
    I.ctrl = s->ctrl;
    I.partials = s->partials;
    // a batch sweeps every stage of a member at one depth: its stage-C depth
    I.tz = s->tz[1];
    s->tz_last = I.tz;
    if (!default_scheme(s->g)) b->generic = true;
    if (s->g.nu > 0.0) b->viscous = true;
    const int nt = Launch<Real>::tiles(s->g, I.tz);
    for (int t = 0; t < nt; ++t) tmap.push_back(make_int2((int)r, t));
    // each member's ghost cells in whole fill blocks (one member per block)
    const long long ng = Launch<Real>::ghosts(s->g);
    for (long long g0 = 0; g0 < ng; g0 += 256) fmap.push_back(make_int2((int)r, (int)g0));
  }
  b->total_tiles = (int)tmap.size();
  b->fill_blocks = (int)fmap.size();
  csph_status st = ensure(&b->tile_map, &b->tile_cap, tmap.size());
  if (!st) st = ensure(&b->fill_map, &b->fill_cap, fmap.size());
  if (st) return st;
  if (n) {
    HIP_TRY(hipMemcpyAsync(b->table, tab.data(), n * sizeof(Inst<Real>), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->tile_map, tmap.data(), tmap.size() * sizeof(int2), hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(hipMemcpyAsync(b->fill_map, fmap.data(), fmap.size() * sizeof(int2), hipMemcpyHostToDevice,
                           b->stream));
    const std::vector<int> zero(n, 0);
    HIP_TRY(hipMemcpyAsync(b->flags, zero.data(), n * sizeof(int), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
  }
  drop_graph(b);
  b->dirty = false;
  return CSPH_OK;
}

template <typename Real>
csph_status batch_launch(csph_batch* b, int k) {
  const int n = (int)b->order.size();
  if (n == 0 || k <= 0) return CSPH_OK;
  if (!b->exec || b->graph_k != k) {
    drop_graph(b);
    // capture k steps of every member; replays reuse the same table
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int q = 0; q < k && e == hipSuccess; ++q)
      e = Launch<Real>::batch_step((const Inst<Real>*)b->table, b->tile_map, b->fill_map, n,
                                   b->total_tiles, b->fill_blocks, b->flags, b->generic, b->viscous,
                                   b->stream);
    hipGraph_t gr = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &gr);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (gr) (void)hipGraphDestroy(gr);
      return fail(CSPH_ERR_DEVICE, std::string("graph capture failed: ") +
                                       hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = gr;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_k = k;
  }
  HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  return CSPH_OK;
}

}  // namespace

extern "C" {

csph_status csph_batch_create(csph_dtype dtype, void* hip_stream, size_t hbm_budget, csph_batch** out) {
  if (!out) return fail(CSPH_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (dtype != CSPH_F32 && dtype != CSPH_F64) return fail(CSPH_ERR_ARG, "bad dtype");
  csph_batch* b = new (std::nothrow) csph_batch();
  if (!b) return fail(CSPH_ERR_NOMEM, "host allocation failed");
  b->dtype = dtype;
  b->stream = (hipStream_t)hip_stream;
  if (!b->stream) {
    // a graph cannot be captured on the null stream: use a stream of our own
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return fail(CSPH_ERR_DEVICE, "hipStreamCreate failed");
    }
    b->own_stream = true;
  }
  b->budget = hbm_budget;
  *out = b;
  return CSPH_OK;
}

csph_status csph_batch_add(csph_batch* b, csph_sim* s, int64_t steps, double t_end, int32_t* slot) {
  if (!b || !s) return fail(CSPH_ERR_ARG, "batch or sim is NULL");
  if (s->desc.dtype != b->dtype) return fail(CSPH_ERR_ARG, "sim dtype differs from the batch dtype");
  if (s->in_batch) return fail(CSPH_ERR_ARG, "sim already belongs to a batch");
  if (steps < 0 || std::isnan(t_end)) return fail(CSPH_ERR_ARG, "bad steps or t_end");
  if (!periodic_pairs_ok(s)) return fail(CSPH_ERR_ARG, "PERIODIC must be set on both faces of an axis");
  if (s->grav > 0.0) return fail(CSPH_ERR_ARG, "a self-gravitating sim cannot join a batch");
  if (s->srcbuf) return fail(CSPH_ERR_ARG, "a sim with sources or sinks cannot join a batch");
  const size_t need = s->L.total;
  if (b->budget && b->used_bytes + need > b->budget) return fail(CSPH_ERR_BUDGET, "HBM budget exceeded");
  Ctrl c{};
  csph_status st = read_ctrl(s, &c);
  if (st) return st;
  if (c.status) return fail(CSPH_ERR_STATE, "sticky error: call csph_set_state");
  // ghosts of psi and the first dt of the member, on the member's own stream
  st = s->is_f64() ? prepare<double>(s) : prepare<float>(s);
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(s->stream));
  st = read_ctrl(s, &c);
  if (st) return st;
  c.done = 0;
  c.step_limit = c.nsteps + steps;
  c.t_end = t_end;
  st = write_ctrl(s, c);
  if (st) return st;
  int q = -1;
  for (size_t k = 0; k < b->slots.size(); ++k)
    if (!b->slots[k].used) {
      q = (int)k;
      break;
    }
  if (q < 0) {
    b->slots.push_back(Member{});
    q = (int)b->slots.size() - 1;
  }
  b->slots[q].sim = s;
  b->slots[q].used = true;
  s->in_batch = true;
  s->batch_stream = b->stream;
  s->stepped = true;
  b->used_bytes += need;
  b->dirty = true;
  if (slot) *slot = q;
  return CSPH_OK;
}

csph_status csph_batch_advance(csph_batch* b, int32_t k_steps, int32_t* n_done) {
  if (!b) return fail(CSPH_ERR_ARG, "batch is NULL");
  if (k_steps < 0) return fail(CSPH_ERR_ARG, "k_steps must be >= 0");
  csph_status st;
  if (b->dirty) {
    st = b->dtype == CSPH_F64 ? build_table<double>(b) : build_table<float>(b);
    if (st) return st;
  }
  st = b->dtype == CSPH_F64 ? batch_launch<double>(b, k_steps) : batch_launch<float>(b, k_steps);
  if (st) return st;
  if (n_done) {
    int32_t cnt = 0, n = 0;
    st = csph_batch_poll(b, nullptr, 0, &n);
    if (st) return st;
    cnt = n;
    *n_done = cnt;
  }
  return CSPH_OK;
}

csph_status csph_batch_poll(csph_batch* b, int32_t* done_slots, int32_t cap, int32_t* n) {
  if (!b || !n) return fail(CSPH_ERR_ARG, "batch or n is NULL");
  *n = 0;
  if (b->dirty) {
    csph_status st = b->dtype == CSPH_F64 ? build_table<double>(b) : build_table<float>(b);
    if (st) return st;
  }
  const size_t m = b->order.size();
  if (m == 0) return CSPH_OK;
  // every step's last launch writes each member's done / error flag
  std::vector<int> fl(m, 0);
  HIP_TRY(hipMemcpyAsync(fl.data(), b->flags, m * sizeof(int), hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  int32_t k = 0;
  for (size_t r = 0; r < m; ++r)
    if (fl[r]) {
      if (done_slots && k < cap) done_slots[k] = b->order[r];
      ++k;
    }
  *n = k;
  return CSPH_OK;
}

csph_status csph_batch_remove(csph_batch* b, int32_t slot) {
  if (!b || slot < 0 || slot >= (int32_t)b->slots.size() || !b->slots[slot].used)
    return fail(CSPH_ERR_ARG, "no such slot");
  HIP_TRY(hipStreamSynchronize(b->stream));
  csph_sim* s = b->slots[slot].sim;
  s->in_batch = false;
  s->batch_stream = nullptr;
  b->used_bytes -= s->L.total;
  b->slots[slot] = Member{};
  b->dirty = true;
  return CSPH_OK;
}

csph_status csph_batch_autotune(csph_batch* b, int32_t trial_steps, int32_t* tz_out,
                                double* ms_per_step) {
  if (!b) return fail(CSPH_ERR_ARG, "batch is NULL");
  if (trial_steps < 1 || trial_steps > 1000) return fail(CSPH_ERR_ARG, "trial_steps must be in [1, 1000]");
  std::vector<csph_sim*> mem;
  for (auto& m : b->slots)
    if (m.used) mem.push_back(m.sim);
  if (mem.empty()) return fail(CSPH_ERR_ARG, "batch has no members");
  HIP_TRY(hipStreamSynchronize(b->stream));
  // snapshot every member's buffer; each trial starts from it and it is
  // restored at the end, so tuning leaves the members as they were
  std::vector<void*> snap(mem.size(), nullptr);
  std::vector<Depths> tz0(mem.size());
  csph_status st = CSPH_OK;
  for (size_t q = 0; q < mem.size() && !st; ++q) {
    tz0[q] = Depths{mem[q]->tz[0], mem[q]->tz[1], mem[q]->tz[2]};
    if (hipMalloc(&snap[q], mem[q]->L.total) != hipSuccess) {
      (void)hipGetLastError();
      snap[q] = nullptr;
      st = fail(CSPH_ERR_NOMEM, "hipMalloc of a member snapshot failed");
      break;
    }
    if (hipMemcpyAsync(snap[q], mem[q]->buf, mem[q]->L.total, hipMemcpyDeviceToDevice, b->stream) != hipSuccess)
      st = fail(CSPH_ERR_DEVICE, "member snapshot copy failed");
  }
  auto restore = [&]() -> csph_status {
    for (size_t q = 0; q < mem.size(); ++q)
      if (snap[q])
        HIP_TRY(hipMemcpyAsync(mem[q]->buf, snap[q], mem[q]->L.total, hipMemcpyDeviceToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return CSPH_OK;
  };
  int nzmax = 0;
  for (csph_sim* m : mem) nzmax = std::max(nzmax, m->g.nz);
  int best = -1;
  double best_ms = INFINITY;
  for (int tz : tz_candidates(nzmax)) {
    if (st) break;
    for (csph_sim* m : mem)
      for (int q = 0; q < 3; ++q) m->tz[q] = tz;
    b->dirty = true;
    st = b->dtype == CSPH_F64 ? build_table<double>(b) : build_table<float>(b);
    if (st) break;
    double ms = 0.0;
    // the first call captures the k-step graph; the second replays it
    for (int rep = 0; rep < 2 && !st; ++rep) {
      st = restore();
      if (st) break;
      st = time_on(b->stream,
                   [&]() { return b->dtype == CSPH_F64 ? batch_launch<double>(b, trial_steps)
                                                       : batch_launch<float>(b, trial_steps); },
                   &ms);
    }
    if (st) break;
    const double per = ms / trial_steps;
    if (per < best_ms) {
      best_ms = per;
      best = tz;
    }
  }
  csph_status st2 = restore();
  for (size_t q = 0; q < mem.size(); ++q) {
    for (int r = 0; r < 3; ++r) mem[q]->tz[r] = (st || best < 0) ? tz0[q][r] : best;
    if (snap[q]) (void)hipFree(snap[q]);
  }
  b->dirty = true;
  if (st) return st;
  if (st2) return st2;
  if (tz_out) *tz_out = best;
  if (ms_per_step) *ms_per_step = best_ms;
  return CSPH_OK;
}

csph_status csph_batch_destroy(csph_batch* b) {
  if (!b) return CSPH_OK;
  (void)hipStreamSynchronize(b->stream);
  for (auto& m : b->slots)
    if (m.used) {
      m.sim->in_batch = false;
      m.sim->batch_stream = nullptr;
    }
  drop_graph(b);
  if (b->table) (void)hipFree(b->table);
  if (b->tile_map) (void)hipFree(b->tile_map);
  if (b->fill_map) (void)hipFree(b->fill_map);
  if (b->flags) (void)hipFree(b->flags);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return CSPH_OK;
}

}  // extern "C"
