/*
 * csph_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, single-threaded, FP64 CPU implementation of one CSPH-TVD time step
 * (Khrapov, Khoperskov & Khoperskov, "Lagrange-Eulerian method for numerical
 * integration of the gas dynamics equations: parallel implementation on GPUs",
 * arXiv:1912.04855).  It is the correctness authority that the HIP path is
 * compared against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product library never does.
 *
 * Arrays crossing this interface are host FP64, structure-of-arrays, x fastest:
 *   state  [5][nz][ny][nx]  (rho, rho*u, rho*v, rho*w, E)   -- conserved
 *   prim   [5][nz][ny][nx]  (rho, u, v, w, p)                -- primitive
 *   psi    [nz][ny][nx]     cell-centred external potential
 *   fields [nz][ny][nx]     one interior field
 */
#ifndef CSPH_ORACLE_H
#define CSPH_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* boundary kinds (ghost-cell rules; the paper states none) */
enum { ORC_PERIODIC = 0, ORC_OUTFLOW = 1, ORC_INFLOW = 2, ORC_REFLECT = 3 };

/* Reading of Q(U*, r*) in the corrector of Eq. (6).  The default
 * (ORC_POS_LAGRANGE) takes the 27-point kernel gradients in the particles'
 * reference configuration -- the lattice, where every particle starts the step --
 * and the state of each particle at r*: its pressure over its predicted volume
 * V* = h^3 (1 + dt div u^n) and the potential sampled at r*.  The alternatives
 * evaluate the kernel gradients at the displaced pairs r*_i - r*_j with the
 * volume left at h^3 (ORC_POS_DISPLACED), or put everything on the lattice
 * (ORC_POS_LATTICE). */
enum { ORC_POS_LAGRANGE = 0, ORC_POS_DISPLACED = 1, ORC_POS_LATTICE = 2 };
/* reconstruction base of Eq. (8): U~^{n+1} ("post") or (U^n + U~^{n+1})/2 ("mid") */
enum { ORC_BASE_POST = 0, ORC_BASE_MID = 1 };
/* TVD limiters (Sec. 2.2 allows any; Sec. 4 names the choice as an option) */
enum { ORC_LIM_MINMOD = 0, ORC_LIM_MC = 1, ORC_LIM_VANLEER = 2, ORC_LIM_SUPERBEE = 3 };
/* face flux of the advective part: HLL with the advective speeds xi/dt (= the exact
 * swept volume), the same plus the acoustic (Rusanov) velocity-jump dissipation
 * (the default), or Lax-Friedrichs with the advective speeds */
enum { ORC_FLUX_SWEPT = 0, ORC_FLUX_LF = 1, ORC_FLUX_SWEPT_AV = 2 };
/* swept width of the swept-volume fluxes: the displacement of the material that
 * reaches the face, from the offsets of the face's two particles interpolated
 * linearly to the foot of the face's trajectory (the default), or the offset of
 * the upwind particle (xi_i or xi_{i+1}) */
enum { ORC_FACE_FOOT = 0, ORC_FACE_PARTICLE = 1 };

/* status codes */
enum {
  ORC_OK = 0,
  ORC_ERR_ARG = 1,
  ORC_ERR_NOMEM = 2,
  ORC_ERR_NONFINITE = 5,
  ORC_ERR_NEG_DENSITY = 6,
  ORC_ERR_NO_SIGNAL = 7,
};

typedef struct {
  int32_t nx, ny, nz;      /* interior cells per axis, each >= 4 */
  double h;                /* the one grid spacing of all three axes */
  double origin[3];        /* coordinate of the low corner of cell (0,0,0) */
  double gamma;            /* adiabatic index, > 1 */
  double cfl;              /* Courant number C of dt = C h / max(c+|u|+|v|+|w|) */
  double rho_vac;          /* cells with rho <= rho_vac are vacuum */
  int32_t bc[6];           /* faces -x,+x,-y,+y,-z,+z */
  double inflow[6][5];     /* primitive (rho,u,v,w,p) used by ORC_INFLOW faces */
  int32_t pos_mode;        /* ORC_POS_* */
  int32_t base_mode;       /* ORC_BASE_* */
  int32_t limiter;         /* ORC_LIM_* */
  int32_t flux;            /* ORC_FLUX_* */
  int32_t face_mode;       /* ORC_FACE_* */
  double nu;               /* kinematic viscosity (0: inviscid) */
  double grav;             /* gravitational constant G of the gas's self-gravity (0: none);
                              needs all six faces periodic or none (isolated box) */
} orc_params;

typedef struct orc_sim orc_sim;

/* which stage field orc_get_field returns (values of the last completed step) */
enum {
  ORC_F_MSX = 0, ORC_F_MSY, ORC_F_MSZ, ORC_F_ES,     /* predictor m*, E*      */
  ORC_F_XSX, ORC_F_XSY, ORC_F_XSZ,                   /* predictor xi*         */
  ORC_F_MTX, ORC_F_MTY, ORC_F_MTZ, ORC_F_ET,         /* corrector m~, E~      */
  ORC_F_XTX, ORC_F_XTY, ORC_F_XTZ,                   /* corrector xi^{n+1}    */
  ORC_F_PSIS,                                        /* psi at r*             */
  ORC_F_VOL,                                         /* predicted volume / h^3 */
  ORC_F_PHIS,                                        /* phi* = sqrt(2 p*)      */
  ORC_F_PSI,                                         /* potential of the step  */
  ORC_F_PSIH,                                        /* self-gravity: potential
                                                        of the predicted density */
  ORC_F_COUNT
};

int      orc_create(const orc_params* p, orc_sim** out);
void     orc_destroy(orc_sim* s);
int      orc_set_conserved(orc_sim* s, const double* state);
int      orc_set_primitive(orc_sim* s, const double* prim);
int      orc_set_potential(orc_sim* s, const double* psi);   /* NULL: psi = 0 */
/* sources and sinks: mass rate q per cell [nz][ny][nx] (mass / volume / time; > 0
 * injects gas at rest with specific internal energy eps, < 0 removes gas at the
 * local specific values, limited at zero); NULL removes them.  Applies from the
 * next step, half before and half after the hydrodynamic step. */
int      orc_set_source(orc_sim* s, const double* q, double eps);
int      orc_get_conserved(const orc_sim* s, double* state);
int      orc_get_field(const orc_sim* s, int which, double* out);
/* one step; dt = min(CFL dt, dt_max if > 0, t_end - t if t_end is finite) */
int      orc_step(orc_sim* s, double dt_max, double t_end, double* dt_taken);
int      orc_advance(orc_sim* s, double t_end, int64_t max_steps, int64_t* steps);
void     orc_get_time(const orc_sim* s, double* t, int64_t* nsteps);
void     orc_set_time(orc_sim* s, double t, int64_t nsteps);
void     orc_totals(const orc_sim* s, double out[5]);
double   orc_cfl_dt(orc_sim* s);          /* CFL dt of the current state, no step */

/* building blocks, exposed so the tests can pin them one by one */
double   orc_kappa(void);                                       /* kernel normalisation */
void     orc_kernel_grad(double dx, double dy, double dz, double h, double out[3]);
double   orc_limiter(int kind, double a, double b);
/* lattice gradient (1/h) sum_o w_|o| (f_{i+o} - f_{i-o}) o on the interior, periodic
 * wrap of f; f and out are [nz][ny][nx] and [3][nz][ny][nx] */
int      orc_lattice_gradient(int32_t nx, int32_t ny, int32_t nz, double h,
                              const double* f, double* out);
/* self-gravity potential of a density field [nz][ny][nx] (the periodic box's
 * discrete Poisson solve, or the isolated box's free-space sum, of each step);
 * writes [nz][ny][nx] */
int      orc_self_potential(orc_sim* s, const double* rho, double* psi_out);
/* isolated box only: the self potential of rho at n cells (i, j, k) = cells[3q..3q+2],
 * each summed directly (O(N) per cell); writes out[n] */
int      orc_self_potential_at(orc_sim* s, const double* rho, const int32_t* cells, int64_t n,
                               double* out);
/* trilinear interpolation of psi (with ghosts filled by the sim's rules) at
 * cell centre + offset; writes one value per cell */
int      orc_interp_psi(orc_sim* s, const double* off /* [3][nz][ny][nx] */, double* out);
/* fill the ghost layers of one cell-shaped array (role: 0 rho,1-3 m,4 E,5-7 xi,8 psi,
 * 9 predicted volume)
 * of width nx+4 etc., given dt for inflow xi; used by the BC unit tests */
int      orc_fill_ghosts_padded(orc_sim* s, double* padded, int role, double dt);

#ifdef __cplusplus
}
#endif
#endif
