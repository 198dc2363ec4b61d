/*
 * csph_oracle.c -- TEST INFRASTRUCTURE ONLY (see csph_oracle.h).
 *
 * Plain scalar FP64, single-threaded, one array per field, one loop per step of
 * the method.  Built with -O2 -ffp-contract=off and no fast-math so that every
 * expression is evaluated exactly as written.  Nothing here is shared with the
 * HIP library: that library is checked against this file, never the reverse.
 *
 * The time step follows Sec. 2.2 of arXiv:1912.04855:
 *   Lagrangian stage  -- predictor Eq. (5), corrector Eq. (6), with the source Q
 *                        of Eq. (7) (a modified-SPH sum over the 3x3x3 index
 *                        neighbours, written with phi = sqrt(2p));
 *   Eulerian stage    -- piecewise-linear reconstruction shifted by the particle
 *                        offset (Eq. (8)), TVD-limited slopes, a Riemann-type face
 *                        flux of the advective part, and the conservative update
 *                        Eq. (4).
 * Where the paper is silent the reading used is stated at the function that
 * implements it.
 */
#include "csph_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define G 2 /* ghost layers: slopes of the first ghost layer need a second */

struct orc_sim {
  orc_params P;
  int sx, sy, sz;     /* padded extents */
  size_t n;           /* padded cell count */
  double inv_h;
  double kappa_h2;    /* kernel normalisation / h^2 */
  int has_psi;
  double inflow_cons[6][5];
  /* U^n */
  double *rho, *m[3], *E;
  double *psi;        /* cell-centred potential, ghosts filled once */
  /* primitives of the state currently being used */
  double *u[3], *p, *phi;
  /* predictor output: m*, E*, xi* ; corrector output: m~, E~, xi^{n+1} */
  double *ms[3], *Es, *xs[3];
  double *mt[3], *Et, *xt[3];
  double *psis;       /* psi at the predicted particle positions */
  double *vol;        /* predicted particle volume / h^3 (Lagrangian corrector) */
  double *psi_ext;    /* the external potential as set (self-gravity adds to it) */
  double *psih;       /* self-gravity: the potential at t^{n+1}, from the predicted density */
  double *src;        /* mass source rate per cell (mass / volume / time; < 0: sink) */
  double eps_src;     /* specific internal energy of the injected gas */
  int has_src;
  double *fre, *fim;  /* Poisson solve: one complex value per interior cell */
  /* Eulerian stage */
  double *slope[5], *flux[5], *acc[5];
  double t;
  int64_t nsteps;
  double totals[5];
};

/* ------------------------------------------------------------------------ */
/* indexing                                                                  */
/* ------------------------------------------------------------------------ */
static size_t IX(const orc_sim* s, int i, int j, int k) {
  return ((size_t)(k + G) * (size_t)s->sy + (size_t)(j + G)) * (size_t)s->sx + (size_t)(i + G);
}

/* ------------------------------------------------------------------------ */
/* smoothing kernel                                                          */
/* ------------------------------------------------------------------------ */
/* The paper leaves W open ("different smoothing kernels can be used", Sec. 4).
 * Reading: the M4 cubic spline with smoothing length h and support 2h.  With
 * q = |d|/h its radial slope is f'(q) = -g(q),
 *     g(q) = 3q - (9/4) q^2   for 0 <= q < 1,
 *     g(q) = (3/4)(2 - q)^2   for 1 <= q < 2,   0 beyond,
 * and the gradient of W(r_i - r_j) used in Eq. (7), volume factor included, is
 *     K(d) = -(kappa/h) g(q) d/|d| = -(kappa/h^2) (g(q)/q) d,   d = r_i - r_j.
 * kappa is fixed so that the 27-point lattice sum reproduces the gradient of
 * any linear field exactly: sum_{o in 3x3x3} (kappa g(|o|)/|o|) o_x^2 = 1, i.e.
 *     kappa = 1 / (2 sum_{a,b in {-1,0,1}} g(q_ab)/q_ab),  q_ab = sqrt(1+a^2+b^2). */
static double g_over_q(double q) {
  if (q < 1.0) return 3.0 - 2.25 * q;
  if (q < 2.0) {
    double t = 2.0 - q;
    return 0.75 * t * t / q;
  }
  return 0.0;
}

double orc_kappa(void) {
  double sum = 0.0;
  for (int a = -1; a <= 1; ++a)
    for (int b = -1; b <= 1; ++b) {
      double q = sqrt(1.0 + (double)(a * a) + (double)(b * b));
      sum += g_over_q(q);
    }
  return 1.0 / (2.0 * sum);
}

static void kgrad(const orc_sim* s, double dx, double dy, double dz, double K[3]) {
  double r2 = dx * dx + dy * dy + dz * dz;
  double q = sqrt(r2) * s->inv_h;
  double c = s->kappa_h2 * g_over_q(q);
  K[0] = -(c * dx);
  K[1] = -(c * dy);
  K[2] = -(c * dz);
}

void orc_kernel_grad(double dx, double dy, double dz, double h, double out[3]) {
  orc_sim tmp;
  memset(&tmp, 0, sizeof tmp);
  tmp.inv_h = 1.0 / h;
  tmp.kappa_h2 = orc_kappa() / (h * h);
  kgrad(&tmp, dx, dy, dz, out);
}

/* ------------------------------------------------------------------------ */
/* TVD limiters                                                              */
/* ------------------------------------------------------------------------ */
/* The paper asks only that the slope satisfy the TVD condition (Sec. 2.2) and
 * lists the limiter as a free option (Sec. 4).  Default reading: minmod. */
double orc_limiter(int kind, double a, double b) {
  if (a * b <= 0.0) return 0.0;
  double sg = a > 0.0 ? 1.0 : -1.0;
  double aa = fabs(a), ab = fabs(b);
  switch (kind) {
    case ORC_LIM_MC: {
      double m = fmin(2.0 * aa, 2.0 * ab);
      return sg * fmin(m, 0.5 * (aa + ab));
    }
    case ORC_LIM_VANLEER:
      return 2.0 * a * b / (a + b);
    case ORC_LIM_SUPERBEE:
      return sg * fmax(fmin(2.0 * aa, ab), fmin(aa, 2.0 * ab));
    default:
      return sg * fmin(aa, ab);
  }
}

/* ------------------------------------------------------------------------ */
/* equation of state and primitive recovery                                  */
/* ------------------------------------------------------------------------ */
/* p = (gamma-1) rho eps with E = rho(|u|^2/2 + eps) (Sec. 2.1).  Vacuum reading:
 * for rho <= rho_vac the velocity is taken as 0 and the cell is left out of the
 * CFL maximum; p is floored at 0 when primitives are formed, and E itself is
 * never changed, so the conserved totals are untouched. */
static void primitive(const orc_sim* s, double rho, double mx, double my, double mz, double E,
                      double* ux, double* uy, double* uz, double* p) {
  if (rho > s->P.rho_vac) {
    *ux = mx / rho;
    *uy = my / rho;
    *uz = mz / rho;
  } else {
    *ux = 0.0;
    *uy = 0.0;
    *uz = 0.0;
  }
  double ke = 0.5 * (mx * *ux + my * *uy + mz * *uz);
  double pp = (s->P.gamma - 1.0) * (E - ke);
  *p = pp > 0.0 ? pp : 0.0;
}

static void all_primitives(orc_sim* s, const double* rho, double* const m[3], const double* E) {
  for (size_t c = 0; c < s->n; ++c) {
    double ux, uy, uz, p;
    primitive(s, rho[c], m[0][c], m[1][c], m[2][c], E[c], &ux, &uy, &uz, &p);
    s->u[0][c] = ux;
    s->u[1][c] = uy;
    s->u[2][c] = uz;
    s->p[c] = p;
    s->phi[c] = sqrt(2.0 * p);
  }
}

/* ------------------------------------------------------------------------ */
/* boundary conditions (ghost cells)                                         */
/* ------------------------------------------------------------------------ */
/* The paper states no boundary conditions.  Reading: two ghost layers;
 * periodic = wrap; outflow = zero-gradient copy; inflow = the face's Dirichlet
 * state (particle offset dt*u_in, potential copied as for outflow); reflect =
 * mirror with the normal momentum and normal offset negated.  The axes are
 * filled in the order x, y, z, each over the full extent of the other two, so
 * edges and corners are the composition of the face rules. */
enum { R_RHO = 0, R_MX = 1, R_MY = 2, R_MZ = 3, R_E = 4, R_XX = 5, R_XY = 6, R_XZ = 7, R_PSI = 8,
       R_VOL = 9 };

static double inflow_value(const orc_sim* s, int face, int role, double dt) {
  switch (role) {
    case R_RHO: return s->inflow_cons[face][0];
    case R_MX: return s->inflow_cons[face][1];
    case R_MY: return s->inflow_cons[face][2];
    case R_MZ: return s->inflow_cons[face][3];
    case R_E: return s->inflow_cons[face][4];
    case R_XX: return dt * s->P.inflow[face][1];
    case R_XY: return dt * s->P.inflow[face][2];
    case R_XZ: return dt * s->P.inflow[face][3];
    case R_VOL: return 1.0; /* a uniform inflow state is not compressed */
    default: return 0.0;
  }
}

static int normal_component(int role, int axis) {
  return (role == R_MX + axis) || (role == R_XX + axis);
}

static void fill_ghosts(orc_sim* s, double* f, int role, double dt) {
  const int nn[3] = {s->P.nx, s->P.ny, s->P.nz};
  for (int ax = 0; ax < 3; ++ax) {
    const int n = nn[ax];
    /* other axes span their full padded range */
    int lo[3] = {-G, -G, -G}, hi[3] = {s->P.nx + G, s->P.ny + G, s->P.nz + G};
    lo[ax] = 0;
    hi[ax] = 1; /* the loop over ax is done by hand below */
    for (int side = 0; side < 2; ++side) {
      const int face = 2 * ax + side;
      const int kind = s->P.bc[face];
      for (int g = 1; g <= G; ++g) {
        const int gi = side == 0 ? -g : n - 1 + g; /* ghost index along ax */
        int src;
        double sign = 1.0;
        switch (kind) {
          case ORC_PERIODIC: src = side == 0 ? n - g : g - 1; break;
          case ORC_REFLECT:
            src = side == 0 ? g - 1 : n - g;
            if (normal_component(role, ax)) sign = -1.0;
            break;
          default: src = side == 0 ? 0 : n - 1; break; /* outflow, and psi at inflow */
        }
        const int dirichlet = (kind == ORC_INFLOW) && role != R_PSI;
        const double val = dirichlet ? inflow_value(s, face, role, dt) : 0.0;
        for (int b = lo[(ax + 2) % 3]; b < hi[(ax + 2) % 3]; ++b)
          for (int a = lo[(ax + 1) % 3]; a < hi[(ax + 1) % 3]; ++a) {
            int gcoord[3], scoord[3];
            gcoord[ax] = gi;
            scoord[ax] = src;
            gcoord[(ax + 1) % 3] = scoord[(ax + 1) % 3] = a;
            gcoord[(ax + 2) % 3] = scoord[(ax + 2) % 3] = b;
            size_t cg = IX(s, gcoord[0], gcoord[1], gcoord[2]);
            if (dirichlet) {
              f[cg] = val;
            } else {
              size_t cs = IX(s, scoord[0], scoord[1], scoord[2]);
              f[cg] = sign * f[cs];
            }
          }
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* the potential at a displaced particle                                     */
/* ------------------------------------------------------------------------ */
/* Eq. (7) needs the external force at the particle; in the corrector the
 * particles sit at r* (Eq. (6)).  Reading: psi at r* is the trilinear
 * interpolation of the cell-centred psi, taken between the cell and its
 * neighbours on the side the particle moved to.  A zero offset returns the
 * cell's own value exactly. */
static double lerp(double a, double b, double t) { return a + t * (b - a); }

static double psi_at(const orc_sim* s, const double* P, size_t c, double ox, double oy,
                     double oz) {
  const double fx = ox * s->inv_h, fy = oy * s->inv_h, fz = oz * s->inv_h;
  const long di = fx >= 0.0 ? 1 : -1;
  const long dj = (fy >= 0.0 ? 1 : -1) * (long)s->sx;
  const long dk = (fz >= 0.0 ? 1 : -1) * (long)s->sx * (long)s->sy;
  const double tx = fabs(fx), ty = fabs(fy), tz = fabs(fz);
  const long cc = (long)c;
  double a00 = lerp(P[cc], P[cc + di], tx);
  double a10 = lerp(P[cc + dj], P[cc + dj + di], tx);
  double a01 = lerp(P[cc + dk], P[cc + dk + di], tx);
  double a11 = lerp(P[cc + dk + dj], P[cc + dk + dj + di], tx);
  double b0 = lerp(a00, a10, ty);
  double b1 = lerp(a01, a11, ty);
  return lerp(b0, b1, tz);
}

/* ------------------------------------------------------------------------ */
/* the source Q of Eq. (7)                                                   */
/* ------------------------------------------------------------------------ */
/* The 26 index neighbours are visited as 13 opposite pairs (+o, -o), o in the
 * half set O13 taken in lexicographic (o_z, o_y, o_x) order, and each pair's two
 * terms are added before they join the sum.  Uniform fields then cancel exactly. */
static const int O13[13][3] = {
    {1, 0, 0},   {-1, 1, 0}, {0, 1, 0},  {1, 1, 0},  {-1, -1, 1}, {0, -1, 1}, {1, -1, 1},
    {-1, 0, 1},  {0, 0, 1},  {1, 0, 1},  {-1, 1, 1}, {0, 1, 1},   {1, 1, 1}};

/* Viscosity (Sec. 4 names viscous flows as an extension).  Reading: the SPH
 * viscous force of Morris et al. (1997) on the same 3x3x3 neighbourhood, with a
 * uniform kinematic viscosity nu.  Particle j pulls particle i towards its own
 * velocity with
 *   f_ij = nu (rho_i + rho_j)/2 lambda_ij (u_j - u_i),
 *   lambda_ij = -2 (r_ij . K(r_ij)) / |r_ij|^2   (r_ij = r_i - r_j),
 * which on the lattice is 2 w_|o| / h^2 (the operator sum_o lambda_o (f_j - f_i) is
 * the lattice Laplacian, exact for quadratics), and does the work
 * f_ij . (u_i + u_j)/2 on it.  Both are antisymmetric in i, j, so momentum and
 * total energy are conserved exactly, while the kinetic energy falls by
 * sum_pairs nu rho lambda |u_i - u_j|^2 and turns into heat.  For a uniform
 * density the force is rho nu Lap(u) and the work div(rho nu grad(|u|^2/2)). */

/* Q(U, r) at padded cell c.  The particles sit at cell centre + xi (xi == NULL:
 * on the lattice) and feel the potential psi_p (one value per particle).
 * Returns A and B with
 *   A = sum_j [phi_c phi_j + rho_c (psi_j - psi_c)] K(r_c - r_j)        (~ grad p + rho grad psi)
 *   B = sum_j phi_c phi_j (u_c + u_j)/2 . K(r_c - r_j)
 *       + rho_c u_c . sum_j (psi_j - psi_c) K(r_c - r_j)                  (~ div(p u) + rho u.grad psi)
 * so that Q = -(0, A, B).  The printed Eq. (7) carries +rho f inside -( ), which
 * with f = -grad psi (Sec. 2.1) would push gas up the potential; the signs here
 * follow the integral laws Eqs. (2)-(3): dm/dt = -grad p + rho f.
 * Pressure and potential share one difference sum, so a state with
 * phi_c (phi_j - phi_c) + rho_c (psi_j - psi_c) = 0 for every pair (for p = rho^2/2:
 * rho + psi = const) feels no force at all: the well-balanced property. */
static void hydro_force(const orc_sim* s, const double* rho, const double* phi,
                        double* const u[3], double* const xi[3], const double* psi_p, size_t c,
                        double A[3], double* B) {
  const long sx = s->sx, sxy = (long)s->sx * (long)s->sy;
  const double h = s->P.h;
  const double rc = rho[c], fc = phi[c], pc = psi_p[c];
  const double uc[3] = {u[0][c], u[1][c], u[2][c]};
  const double nu = s->P.nu;
  double a[3] = {0.0, 0.0, 0.0}, gp[3] = {0.0, 0.0, 0.0}, be = 0.0;
  double vm[3] = {0.0, 0.0, 0.0}, ve = 0.0;
  for (int q = 0; q < 13; ++q) {
    double ta[2][3], tg[2][3], te[2], tv[2][3], tw[2];
    for (int side = 0; side < 2; ++side) {
      const int sg = side == 0 ? 1 : -1;
      const int ox = sg * O13[q][0], oy = sg * O13[q][1], oz = sg * O13[q][2];
      const size_t j = (size_t)((long)c + ox + oy * sx + oz * sxy);
      double d[3] = {-ox * h, -oy * h, -oz * h};
      if (xi) {
        d[0] = d[0] + (xi[0][c] - xi[0][j]);
        d[1] = d[1] + (xi[1][c] - xi[1][j]);
        d[2] = d[2] + (xi[2][c] - xi[2][j]);
      }
      double K[3];
      kgrad(s, d[0], d[1], d[2], K);
      const double ff = fc * phi[j];
      const double dpsi = psi_p[j] - pc;
      const double sp = ff + rc * dpsi;
      const double ub = 0.5 * ((uc[0] + u[0][j]) * K[0] + (uc[1] + u[1][j]) * K[1] +
                               (uc[2] + u[2][j]) * K[2]);
      for (int k = 0; k < 3; ++k) {
        ta[side][k] = sp * K[k];
        tg[side][k] = dpsi * K[k];
      }
      te[side] = ff * ub;
      if (nu > 0.0) {
        const double lam = -2.0 * (d[0] * K[0] + d[1] * K[1] + d[2] * K[2]) /
                           (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double cv = (nu * lam) * (0.5 * (rc + rho[j]));
        for (int k = 0; k < 3; ++k) tv[side][k] = cv * (u[k][j] - uc[k]);
        tw[side] = 0.5 * (tv[side][0] * (uc[0] + u[0][j]) + tv[side][1] * (uc[1] + u[1][j]) +
                          tv[side][2] * (uc[2] + u[2][j]));
      }
    }
    for (int k = 0; k < 3; ++k) {
      a[k] = a[k] + (ta[0][k] + ta[1][k]);
      gp[k] = gp[k] + (tg[0][k] + tg[1][k]);
    }
    be = be + (te[0] + te[1]);
    if (nu > 0.0) {
      for (int k = 0; k < 3; ++k) vm[k] = vm[k] + (tv[0][k] + tv[1][k]);
      ve = ve + (tw[0] + tw[1]);
    }
  }
  /* Q = -(0, A, B): the viscous force and its work enter with the other sign */
  A[0] = a[0] - vm[0];
  A[1] = a[1] - vm[1];
  A[2] = a[2] - vm[2];
  *B = (be + rc * (uc[0] * gp[0] + uc[1] * gp[1] + uc[2] * gp[2])) - ve;
}

/* Lattice divergence of a vector field at padded cell c: the same 27-point
 * kernel gradients on the undisplaced lattice as Q, summed as 13 opposite pairs,
 *   div_c = sum_{o in O13} (K(-h o) . f_{c+o} + K(h o) . f_{c-o}).
 * A uniform field gives exactly zero. */
static double lattice_div(const orc_sim* s, double* const f[3], size_t c) {
  const long sx = s->sx, sxy = (long)s->sx * (long)s->sy;
  const double h = s->P.h;
  double dv = 0.0;
  for (int q = 0; q < 13; ++q) {
    double t[2];
    for (int side = 0; side < 2; ++side) {
      const int sg = side == 0 ? 1 : -1;
      const int ox = sg * O13[q][0], oy = sg * O13[q][1], oz = sg * O13[q][2];
      const size_t j = (size_t)((long)c + ox + oy * sx + oz * sxy);
      double K[3];
      kgrad(s, -ox * h, -oy * h, -oz * h, K);
      t[side] = K[0] * f[0][j] + K[1] * f[1][j] + K[2] * f[2][j];
    }
    dv = dv + (t[0] + t[1]);
  }
  return dv;
}

/* ------------------------------------------------------------------------ */
/* create / destroy / state                                                  */
/* ------------------------------------------------------------------------ */
static double* field(orc_sim* s) { return (double*)calloc(s->n, sizeof(double)); }

int orc_create(const orc_params* p, orc_sim** out) {
  if (!p || !out) return ORC_ERR_ARG;
  *out = NULL;
  if (p->nx < 4 || p->ny < 4 || p->nz < 4 || !(p->h > 0.0) || !(p->gamma > 1.0) ||
      !(p->cfl > 0.0) || !(p->rho_vac >= 0.0) || !(p->nu >= 0.0) || !(p->grav >= 0.0))
    return ORC_ERR_ARG;
  if (p->grav > 0.0) {
    /* a periodic box, or one with no periodic face (isolated) */
    int np = 0;
    for (int f = 0; f < 6; ++f) np += p->bc[f] == ORC_PERIODIC;
    if (np != 0 && np != 6) return ORC_ERR_ARG;
  }
  for (int ax = 0; ax < 3; ++ax) {
    int lo = p->bc[2 * ax], hi = p->bc[2 * ax + 1];
    if (lo < 0 || lo > 3 || hi < 0 || hi > 3) return ORC_ERR_ARG;
    if ((lo == ORC_PERIODIC) != (hi == ORC_PERIODIC)) return ORC_ERR_ARG;
  }
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  if (!s) return ORC_ERR_NOMEM;
  s->P = *p;
  s->sx = p->nx + 2 * G;
  s->sy = p->ny + 2 * G;
  s->sz = p->nz + 2 * G;
  s->n = (size_t)s->sx * (size_t)s->sy * (size_t)s->sz;
  s->inv_h = 1.0 / p->h;
  s->kappa_h2 = orc_kappa() / (p->h * p->h);
  for (int f = 0; f < 6; ++f) {
    const double* w = p->inflow[f];
    s->inflow_cons[f][0] = w[0];
    s->inflow_cons[f][1] = w[0] * w[1];
    s->inflow_cons[f][2] = w[0] * w[2];
    s->inflow_cons[f][3] = w[0] * w[3];
    s->inflow_cons[f][4] = w[4] / (p->gamma - 1.0) + 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
  }
  double** all[] = {&s->rho, &s->m[0], &s->m[1], &s->m[2], &s->E, &s->psi, &s->u[0], &s->u[1],
                    &s->u[2], &s->p, &s->phi, &s->ms[0], &s->ms[1], &s->ms[2], &s->Es, &s->xs[0],
                    &s->xs[1], &s->xs[2], &s->mt[0], &s->mt[1], &s->mt[2], &s->Et, &s->xt[0],
                    &s->xt[1], &s->xt[2], &s->psis, &s->vol, &s->psi_ext, &s->psih, &s->src, &s->fre, &s->fim, &s->slope[0], &s->slope[1], &s->slope[2],
                    &s->slope[3], &s->slope[4], &s->flux[0], &s->flux[1], &s->flux[2], &s->flux[3],
                    &s->flux[4], &s->acc[0], &s->acc[1], &s->acc[2], &s->acc[3], &s->acc[4]};
  for (size_t k = 0; k < sizeof all / sizeof all[0]; ++k) {
    *all[k] = field(s);
    if (!*all[k]) {
      orc_destroy(s);
      return ORC_ERR_NOMEM;
    }
  }
  *out = s;
  return ORC_OK;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  double* all[] = {s->rho, s->m[0], s->m[1], s->m[2], s->E, s->psi, s->u[0], s->u[1], s->u[2],
                   s->p, s->phi, s->ms[0], s->ms[1], s->ms[2], s->Es, s->xs[0], s->xs[1],
                   s->xs[2], s->mt[0], s->mt[1], s->mt[2], s->Et, s->xt[0], s->xt[1], s->xt[2],
                   s->psis, s->vol, s->psi_ext, s->psih, s->src, s->fre, s->fim, s->slope[0], s->slope[1], s->slope[2], s->slope[3], s->slope[4],
                   s->flux[0], s->flux[1], s->flux[2], s->flux[3], s->flux[4], s->acc[0],
                   s->acc[1], s->acc[2], s->acc[3], s->acc[4]};
  for (size_t k = 0; k < sizeof all / sizeof all[0]; ++k) free(all[k]);
  free(s);
}

static size_t ninterior(const orc_sim* s) {
  return (size_t)s->P.nx * (size_t)s->P.ny * (size_t)s->P.nz;
}

int orc_set_conserved(orc_sim* s, const double* st) {
  if (!s || !st) return ORC_ERR_ARG;
  const size_t N = ninterior(s);
  double* dst[5] = {s->rho, s->m[0], s->m[1], s->m[2], s->E};
  size_t q = 0;
  for (int k = 0; k < s->P.nz; ++k)
    for (int j = 0; j < s->P.ny; ++j)
      for (int i = 0; i < s->P.nx; ++i, ++q) {
        size_t c = IX(s, i, j, k);
        for (int v = 0; v < 5; ++v) dst[v][c] = st[(size_t)v * N + q];
      }
  return ORC_OK;
}

int orc_set_primitive(orc_sim* s, const double* w) {
  if (!s || !w) return ORC_ERR_ARG;
  const size_t N = ninterior(s);
  size_t q = 0;
  for (int k = 0; k < s->P.nz; ++k)
    for (int j = 0; j < s->P.ny; ++j)
      for (int i = 0; i < s->P.nx; ++i, ++q) {
        const double r = w[q], ux = w[N + q], uy = w[2 * N + q], uz = w[3 * N + q],
                     p = w[4 * N + q];
        if (r < 0.0 || p < 0.0) return ORC_ERR_ARG;
        size_t c = IX(s, i, j, k);
        s->rho[c] = r;
        s->m[0][c] = r * ux;
        s->m[1][c] = r * uy;
        s->m[2][c] = r * uz;
        s->E[c] = p / (s->P.gamma - 1.0) + 0.5 * r * (ux * ux + uy * uy + uz * uz);
      }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* sources and sinks                                                         */
/* ------------------------------------------------------------------------ */
/* Sec. 4 names non-stationary sources and sinks as an extension.  Reading: a
 * mass rate q per cell (mass per volume per time), which the caller may change
 * between any two steps.  A source (q > 0) injects gas at rest with specific
 * internal energy eps: rho += q dt, m unchanged, E += q dt eps (momentum is
 * conserved; the mixing of resting and moving gas heats it).  A sink (q < 0)
 * removes gas at the local specific values: rho += q dt, limited at zero, with
 * m and E scaled by the same factor, so u and E/rho are unchanged.  Both are
 * exact for a stationary cell, and applying them for a and then b is applying
 * them once for a + b.  The step applies half before and half after the
 * hydrodynamic step (Strang splitting: second order in time; the whole source
 * after the step is first order). */
static void source_cell(double q, double eps, double hdt, double* r, double* mx, double* my,
                        double* mz, double* E) {
  if (q == 0.0) return;
  const double d = hdt * q;
  if (q > 0.0) {
    *r = *r + d;
    *E = *E + d * eps;
    return;
  }
  if (!(*r > 0.0)) return;
  double rn = *r + d;
  if (rn < 0.0) rn = 0.0;
  const double f = rn / *r;
  *mx = *mx * f;
  *my = *my * f;
  *mz = *mz * f;
  *E = *E * f;
  *r = rn;
}

int orc_set_source(orc_sim* s, const double* q, double eps) {
  if (!s) return ORC_ERR_ARG;
  if (!q) {
    s->has_src = 0;
    memset(s->src, 0, s->n * sizeof(double));
    return ORC_OK;
  }
  if (!isfinite(eps) || eps < 0.0) return ORC_ERR_ARG;
  const size_t N = ninterior(s);
  for (size_t p = 0; p < N; ++p)
    if (!isfinite(q[p])) return ORC_ERR_ARG;
  size_t p = 0;
  for (int k = 0; k < s->P.nz; ++k)
    for (int j = 0; j < s->P.ny; ++j)
      for (int i = 0; i < s->P.nx; ++i, ++p) s->src[IX(s, i, j, k)] = q[p];
  s->eps_src = eps;
  s->has_src = 1;
  return ORC_OK;
}

int orc_set_potential(orc_sim* s, const double* psi) {
  if (!s) return ORC_ERR_ARG;
  memset(s->psi, 0, s->n * sizeof(double));
  s->has_psi = psi != NULL;
  if (psi) {
    size_t q = 0;
    for (int k = 0; k < s->P.nz; ++k)
      for (int j = 0; j < s->P.ny; ++j)
        for (int i = 0; i < s->P.nx; ++i, ++q) s->psi[IX(s, i, j, k)] = psi[q];
  }
  fill_ghosts(s, s->psi, R_PSI, 0.0);
  memcpy(s->psi_ext, s->psi, s->n * sizeof(double));
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* self-gravity                                                              */
/* ------------------------------------------------------------------------ */
/* Sec. 4 names the gas's self-gravity as an extension.  Reading: on a periodic
 * box the potential of the gas solves the discrete Poisson equation
 *   L7[psi] = 4 pi G (rho - mean(rho)),
 * L7 the 7-point Laplacian (f_{i+1} + f_{i-1} - 2 f_i)/h^2 summed over the axes;
 * the total potential is the external one plus this.  The predictor, Eq. (5),
 * takes the potential of rho^n.  The corrector, Eq. (6), evaluates Q at the end
 * of the step, so it takes the potential of the density predicted for t^{n+1}
 * by the continuity equation,
 *   rho^ = rho^n - dt sum_d (m_d,i+1 - m_d,i-1) / (2h),
 * which is rho^{n+1} to O(dt^2): a potential of rho^n there would make the force
 * of the corrector O(dt) wrong and the step first order in time.  The solve is
 * spectral: the discrete Fourier transform diagonalises L7 with eigenvalues
 *   lambda(k) = sum_d (2 cos(2 pi k_d / n_d) - 2) / h^2,
 * so psi_k = 4 pi G rho_k / lambda(k) for k != 0 and psi_0 = 0 (the mean density
 * has no potential on a periodic box).  The transforms are plain O(n^2) sums
 * along each axis.  A box with no periodic face (gas in vacuum) takes the
 * free-space potential of its cells instead (free_space below); a box with
 * some periodic faces and some not is refused. */

#define ORC_PI 3.14159265358979323846

/* DFT along one axis of the complex interior array (re, im), in place, with
 * the sign sg of the exponent; scratch line buffers of length n */
static void dft_axis(const orc_sim* s, double* re, double* im, int axis, double sg) {
  const int n[3] = {s->P.nx, s->P.ny, s->P.nz};
  const long st[3] = {1, n[0], (long)n[0] * n[1]};
  const int m = n[axis];
  double* lr = (double*)malloc(2 * (size_t)m * sizeof(double));
  double* li = lr + m;
  const int o1 = (axis + 1) % 3, o2 = (axis + 2) % 3;
  for (int b = 0; b < n[o2]; ++b)
    for (int a = 0; a < n[o1]; ++a) {
      const long base = (long)a * st[o1] + (long)b * st[o2];
      for (int k = 0; k < m; ++k) {
        double sr = 0.0, si = 0.0;
        for (int j = 0; j < m; ++j) {
          const double ang = sg * 2.0 * ORC_PI * (double)(((long)j * k) % m) / (double)m;
          const double c = cos(ang), sn = sin(ang);
          const double xr = re[base + j * st[axis]], xi = im[base + j * st[axis]];
          sr += xr * c - xi * sn;
          si += xr * sn + xi * c;
        }
        lr[k] = sr;
        li[k] = si;
      }
      for (int k = 0; k < m; ++k) {
        re[base + k * st[axis]] = lr[k];
        im[base + k * st[axis]] = li[k];
      }
    }
  free(lr);
}

/* psi_self of the interior density rho_in ([nz][ny][nx]) into out ([nz][ny][nx]) */
static void poisson(orc_sim* s, const double* rho_in, double* out) {
  const int nx = s->P.nx, ny = s->P.ny, nz = s->P.nz;
  const size_t N = (size_t)nx * ny * nz;
  for (size_t q = 0; q < N; ++q) {
    s->fre[q] = rho_in[q];
    s->fim[q] = 0.0;
  }
  for (int ax = 0; ax < 3; ++ax) dft_axis(s, s->fre, s->fim, ax, -1.0);
  const double h2 = s->P.h * s->P.h;
  const double fpg = 4.0 * ORC_PI * s->P.grav;
  size_t q = 0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i, ++q) {
        if (i == 0 && j == 0 && k == 0) {
          s->fre[q] = 0.0;
          s->fim[q] = 0.0;
          continue;
        }
        const double lam = (2.0 * cos(2.0 * ORC_PI * i / nx) - 2.0) / h2 +
                           (2.0 * cos(2.0 * ORC_PI * j / ny) - 2.0) / h2 +
                           (2.0 * cos(2.0 * ORC_PI * k / nz) - 2.0) / h2;
        const double f = fpg / lam / (double)N;
        s->fre[q] *= f;
        s->fim[q] *= f;
      }
  for (int ax = 2; ax >= 0; --ax) dft_axis(s, s->fre, s->fim, ax, 1.0);
  for (size_t p = 0; p < N; ++p) out[p] = s->fre[p];
}

/* Isolated boxes (no periodic face).  Reading: the gas's potential is that of
 * its mass in free space, each cell a uniform cube of side h,
 *   psi_i = -G h^3 sum_j rho_j phi(r_i - r_j),
 * phi(d) = 1/|d| between different cells (the cubes' mutual potential to
 * O((h/|d|)^2)) and phi(0) = C / h for a cell's own cube, C = 3 ln(2 + sqrt 3)
 * - pi/2 = 2.3800772..., the integral of 1/|x| over a unit cube about its
 * centre.  Written out as the direct O(N^2) sum. */
static double free_space_cell(const orc_sim* s, const double* rho_in, int i, int j, int k) {
  const int nx = s->P.nx, ny = s->P.ny, nz = s->P.nz;
  const double h = s->P.h, grav = s->P.grav;
  const double self = (3.0 * log(2.0 + sqrt(3.0)) - 0.5 * ORC_PI) / h;
  double acc = 0.0;
  size_t p = 0;
  for (int c = 0; c < nz; ++c)
    for (int b = 0; b < ny; ++b)
      for (int a = 0; a < nx; ++a, ++p) {
        const double dx = (double)(i - a) * h, dy = (double)(j - b) * h, dz = (double)(k - c) * h;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        acc += rho_in[p] * ((a == i && b == j && c == k) ? self : 1.0 / r);
      }
  return -grav * h * h * h * acc;
}

static void free_space(const orc_sim* s, const double* rho_in, double* out) {
  size_t q = 0;
  for (int k = 0; k < s->P.nz; ++k)
    for (int j = 0; j < s->P.ny; ++j)
      for (int i = 0; i < s->P.nx; ++i, ++q) out[q] = free_space_cell(s, rho_in, i, j, k);
}

static void gather(const orc_sim* s, const double* src, double* out);

static int isolated(const orc_sim* s) { return s->P.bc[0] != ORC_PERIODIC; }

/* out = psi_ext + the potential of the interior density rho_in; ghosts by the
 * potential's boundary rules */
static void self_gravity(orc_sim* s, const double* rho_in, double* out) {
  const size_t N = ninterior(s);
  double* pout = (double*)malloc(N * sizeof(double));
  if (isolated(s))
    free_space(s, rho_in, pout);
  else
    poisson(s, rho_in, pout);
  size_t q = 0;
  for (int k = 0; k < s->P.nz; ++k)
    for (int j = 0; j < s->P.ny; ++j)
      for (int i = 0; i < s->P.nx; ++i, ++q) {
        const size_t c = IX(s, i, j, k);
        out[c] = s->psi_ext[c] + pout[q];
      }
  free(pout);
  fill_ghosts(s, out, R_PSI, 0.0);
}

/* the density predicted for t^{n+1} by the continuity equation (interior) */
static void predicted_density(const orc_sim* s, double dt, double* out) {
  const long st[3] = {1, s->sx, (long)s->sx * (long)s->sy};
  size_t q = 0;
  for (int k = 0; k < s->P.nz; ++k)
    for (int j = 0; j < s->P.ny; ++j)
      for (int i = 0; i < s->P.nx; ++i, ++q) {
        const size_t c = IX(s, i, j, k);
        double div = 0.0;
        for (int d = 0; d < 3; ++d) div += (s->m[d][c + st[d]] - s->m[d][c - st[d]]) / (2.0 * s->P.h);
        out[q] = s->rho[c] - dt * div;
      }
}

int orc_self_potential_at(orc_sim* s, const double* rho, const int32_t* cells, int64_t n, double* out) {
  if (!s || !rho || !cells || !out || n < 0 || !isolated(s) || !(s->P.grav > 0.0)) return ORC_ERR_ARG;
  for (int64_t q = 0; q < n; ++q) {
    const int i = cells[3 * q], j = cells[3 * q + 1], k = cells[3 * q + 2];
    if (i < 0 || i >= s->P.nx || j < 0 || j >= s->P.ny || k < 0 || k >= s->P.nz) return ORC_ERR_ARG;
    out[q] = free_space_cell(s, rho, i, j, k);
  }
  return ORC_OK;
}

int orc_self_potential(orc_sim* s, const double* rho, double* psi_out) {
  if (!s || !rho || !psi_out) return ORC_ERR_ARG;
  if (isolated(s))
    free_space(s, rho, psi_out);
  else
    poisson(s, rho, psi_out);
  return ORC_OK;
}

static void gather(const orc_sim* s, const double* src, double* out) {
  size_t q = 0;
  for (int k = 0; k < s->P.nz; ++k)
    for (int j = 0; j < s->P.ny; ++j)
      for (int i = 0; i < s->P.nx; ++i, ++q) out[q] = src[IX(s, i, j, k)];
}

int orc_get_conserved(const orc_sim* s, double* st) {
  if (!s || !st) return ORC_ERR_ARG;
  const size_t N = ninterior(s);
  const double* src[5] = {s->rho, s->m[0], s->m[1], s->m[2], s->E};
  for (int v = 0; v < 5; ++v) gather(s, src[v], st + (size_t)v * N);
  return ORC_OK;
}

int orc_get_field(const orc_sim* s, int which, double* out) {
  if (!s || !out || which < 0 || which >= ORC_F_COUNT) return ORC_ERR_ARG;
  const double* src[ORC_F_COUNT] = {s->ms[0], s->ms[1], s->ms[2], s->Es,    s->xs[0],
                                    s->xs[1], s->xs[2], s->mt[0], s->mt[1], s->mt[2],
                                    s->Et,    s->xt[0], s->xt[1], s->xt[2], s->psis,
                                    s->vol,   s->phi,   s->psi,   s->psih};
  gather(s, src[which], out);
  return ORC_OK;
}

void orc_get_time(const orc_sim* s, double* t, int64_t* nsteps) {
  if (t) *t = s->t;
  if (nsteps) *nsteps = s->nsteps;
}

void orc_set_time(orc_sim* s, double t, int64_t nsteps) {
  s->t = t;
  s->nsteps = nsteps;
}

void orc_totals(const orc_sim* s, double out[5]) {
  for (int v = 0; v < 5; ++v) out[v] = s->totals[v];
}

/* ------------------------------------------------------------------------ */
/* the CFL time step                                                         */
/* ------------------------------------------------------------------------ */
/* The paper gives no time-step rule.  Reading: dt = C h / max over non-vacuum
 * interior cells of (c + |u| + |v| + |w|); the sum of the three speeds keeps the
 * unsplit remap's swept volume below one cell. */
static double signal_max(orc_sim* s) {
  double smax = 0.0;
  for (int k = 0; k < s->P.nz; ++k)
    for (int j = 0; j < s->P.ny; ++j)
      for (int i = 0; i < s->P.nx; ++i) {
        size_t c = IX(s, i, j, k);
        double r = s->rho[c];
        if (!(r > s->P.rho_vac)) continue;
        double ux, uy, uz, p;
        primitive(s, r, s->m[0][c], s->m[1][c], s->m[2][c], s->E[c], &ux, &uy, &uz, &p);
        double cs = sqrt(s->P.gamma * p / r);
        double sp = cs + fabs(ux) + fabs(uy) + fabs(uz);
        if (sp > smax) smax = sp;
      }
  return smax;
}

/* the explicit viscous limit of dt (Heun's method on the lattice Laplacian, whose
 * most negative eigenvalue is -4 (6 w_1 + 8 w_sqrt3) / h^2 = -5.93 / h^2, is stable
 * for nu dt <= 0.337 h^2); 0 when inviscid */
static double visc_dt(const orc_sim* s) {
  return s->P.nu > 0.0 ? 0.25 * s->P.h * s->P.h / s->P.nu : 0.0;
}

double orc_cfl_dt(orc_sim* s) {
  double smax = signal_max(s);
  double dt = smax > 0.0 ? s->P.cfl * s->P.h / smax : INFINITY;
  const double dv = visc_dt(s);
  if (dv > 0.0 && dv < dt) dt = dv;
  return dt;
}

/* ------------------------------------------------------------------------ */
/* acoustic dissipation of the face flux                                     */
/* ------------------------------------------------------------------------ */
/* Sec. 2.2 takes the face fluxes from approximate Riemann solvers (LF, HLL,
 * HLLC) that see both the left and the right state.  Their acoustic waves are
 * what damps sound in a Godunov-type scheme; the swept-volume flux alone moves
 * with the particles and damps nothing where the gas is at rest.  Reading: a
 * Rusanov (local Lax-Friedrichs) term with the acoustic speed
 * a = max(|u_L| + c_L, |u_R| + c_R) of the reconstructed face states, applied to
 * the velocity jump, with the transverse components at half weight:
 *     D_m,c = -(a/2) w_c min(rho_L, rho_R) (u_c,R - u_c,L),  w_n = 1, w_t = 1/2,
 *     D_E   = u_bar . D_m,   D_rho = 0.
 * It vanishes identically for a gas at rest and for uniform flow, so the
 * at-rest equilibrium and the uniform-flow fixed point survive, and its energy
 * flux turns the kinetic energy it removes into heat.  The normal part damps
 * sound; the transverse part damps the shear noise that the displaced-kernel
 * sums excite in a stratified gas.  As an explicit 3D diffusion each component
 * then needs (1 + 1/2 + 1/2) a dt/h <= 1, which the CFL rule meets (full weight
 * on all three would need a dt/h <= 1/3 and is unstable at C = 0.4).  The
 * smaller of the two densities keeps the momentum moved into a near-vacuum cell
 * in proportion to that cell's own mass, so the velocity update stays a bounded
 * relaxation. */
static void acoustic_dissipation(const orc_sim* s, int axis, const double L[5], const double R[5],
                                 double D[5]) {
  double uL[3], uR[3], pL, pR;
  primitive(s, L[0], L[1], L[2], L[3], L[4], &uL[0], &uL[1], &uL[2], &pL);
  primitive(s, R[0], R[1], R[2], R[3], R[4], &uR[0], &uR[1], &uR[2], &pR);
  const double cL = L[0] > s->P.rho_vac ? sqrt(s->P.gamma * pL / L[0]) : 0.0;
  const double cR = R[0] > s->P.rho_vac ? sqrt(s->P.gamma * pR / R[0]) : 0.0;
  const double a = fmax(fabs(uL[axis]) + cL, fabs(uR[axis]) + cR);
  const double k = -0.5 * a * fmin(L[0], R[0]);
  const double kt = 0.5 * k;
  D[0] = 0.0;
  for (int c = 0; c < 3; ++c) D[1 + c] = (c == axis ? k : kt) * (uR[c] - uL[c]);
  D[4] = 0.5 * ((uL[0] + uR[0]) * D[1] + (uL[1] + uR[1]) * D[2] + (uL[2] + uR[2]) * D[3]);
}

/* ------------------------------------------------------------------------ */
/* one CSPH-TVD step                                                         */
/* ------------------------------------------------------------------------ */
int orc_step(orc_sim* s, double dt_max, double t_end, double* dt_taken) {
  if (!s) return ORC_ERR_ARG;
  const int nx = s->P.nx, ny = s->P.ny, nz = s->P.nz;
  const double h = s->P.h, inv_h = s->inv_h;

  /* O1: ghosts of U^n */
  fill_ghosts(s, s->rho, R_RHO, 0.0);
  fill_ghosts(s, s->m[0], R_MX, 0.0);
  fill_ghosts(s, s->m[1], R_MY, 0.0);
  fill_ghosts(s, s->m[2], R_MZ, 0.0);
  fill_ghosts(s, s->E, R_E, 0.0);

  /* O3: time step */
  double smax = signal_max(s);
  double dt;
  const double dv = visc_dt(s);
  if (smax > 0.0 || dv > 0.0) {
    dt = smax > 0.0 ? s->P.cfl * h / smax : dv;
    if (dv > 0.0 && dv < dt) dt = dv;
    if (dt_max > 0.0 && dt_max < dt) dt = dt_max;
  } else {
    if (!(dt_max > 0.0)) return ORC_ERR_NO_SIGNAL;
    dt = dt_max;
  }
  int lands = 0;
  if (isfinite(t_end) && t_end - s->t <= dt) {
    dt = t_end - s->t;
    lands = 1;
  }
  if (!(dt > 0.0)) return ORC_ERR_ARG;

  /* sources and sinks: the first half step, then the ghosts of U^n again */
  if (s->has_src) {
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          const size_t c = IX(s, i, j, k);
          source_cell(s->src[c], s->eps_src, 0.5 * dt, &s->rho[c], &s->m[0][c], &s->m[1][c],
                      &s->m[2][c], &s->E[c]);
        }
    fill_ghosts(s, s->rho, R_RHO, 0.0);
    fill_ghosts(s, s->m[0], R_MX, 0.0);
    fill_ghosts(s, s->m[1], R_MY, 0.0);
    fill_ghosts(s, s->m[2], R_MZ, 0.0);
    fill_ghosts(s, s->E, R_E, 0.0);
  }

  /* self-gravity: the potential of rho^n, for the predictor */
  if (s->P.grav > 0.0) {
    double* rin = (double*)malloc(ninterior(s) * sizeof(double));
    gather(s, s->rho, rin);
    self_gravity(s, rin, s->psi);
    free(rin);
  }

  /* self-gravity: the potential of the density predicted for t^{n+1}, for the
   * corrector; without it the corrector samples the potential of the step */
  const double* psi_c = s->psi;
  if (s->P.grav > 0.0) {
    double* rin = (double*)malloc(ninterior(s) * sizeof(double));
    predicted_density(s, dt, rin);
    self_gravity(s, rin, s->psih);
    free(rin);
    psi_c = s->psih;
  }

  /* O2: primitives of U^n on every cell, ghosts included */
  all_primitives(s, s->rho, s->m, s->E);

  const int lagrange = s->P.pos_mode == ORC_POS_LAGRANGE;
  /* O4-O5: predictor, Eq. (5):  U* = U^n + dt Q(U^n, r^n),  r* = r^n + dt (u^n + u*)/2.
   * The particles start at the cell centres; xi* = r* - r^n. */
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t c = IX(s, i, j, k);
        double A[3], B;
        hydro_force(s, s->rho, s->phi, s->u, NULL, s->psi, c, A, &B);
        for (int d = 0; d < 3; ++d) s->ms[d][c] = s->m[d][c] - dt * A[d];
        s->Es[c] = s->E[c] - dt * B;
        double usx, usy, usz, ps;
        primitive(s, s->rho[c], s->ms[0][c], s->ms[1][c], s->ms[2][c], s->Es[c], &usx, &usy, &usz,
                  &ps);
        s->xs[0][c] = 0.5 * dt * (s->u[0][c] + usx);
        s->xs[1][c] = 0.5 * dt * (s->u[1][c] + usy);
        s->xs[2][c] = 0.5 * dt * (s->u[2][c] + usz);
        /* volume of the predicted particle relative to its cell (Lagrangian
         * corrector): V* / h^3 = 1 + dt div(u^n), to first order in dt */
        if (lagrange) s->vol[c] = 1.0 + dt * lattice_div(s, s->u, c);
      }

  /* O6: ghosts of the predicted particles (rho* = rho^n: mass is untouched) */
  fill_ghosts(s, s->ms[0], R_MX, dt);
  fill_ghosts(s, s->ms[1], R_MY, dt);
  fill_ghosts(s, s->ms[2], R_MZ, dt);
  fill_ghosts(s, s->Es, R_E, dt);
  fill_ghosts(s, s->xs[0], R_XX, dt);
  fill_ghosts(s, s->xs[1], R_XY, dt);
  fill_ghosts(s, s->xs[2], R_XZ, dt);
  if (lagrange) fill_ghosts(s, s->vol, R_VOL, dt);

  /* keep u^n for the position update before the primitives are overwritten */
  /* (slopes below use the conserved U^n, which is still intact) */
  double* un[3];
  for (int d = 0; d < 3; ++d) {
    un[d] = s->acc[d]; /* borrow: acc is not needed until the Eulerian stage */
    memcpy(un[d], s->u[d], s->n * sizeof(double));
  }

  /* O7-O8: corrector, Eq. (6):
   *   U~^{n+1} = (U^n + U*)/2 + (dt/2) Q(U*, r*),
   *   r^{n+1}  = (r^n + r*)/2 + (dt/2) (u^n + u^{n+1})/2,
   * where u^{n+1} is read as the post-Lagrange velocity m~/rho.
   * Reading (ORC_POS_LAGRANGE, the default): the corrector differentiates in the
   * particles' reference configuration.  Every particle starts the step at its
   * cell centre, so the kernel gradients of Eq. (7) are the lattice ones, and
   * the state of particle i at r* enters through its pressure and its potential:
   * the pressure is its internal energy over its predicted volume,
   * V*_i = h^3 (1 + dt div(u^n)_i) (the lattice divergence, first order in dt),
   * and psi is sampled at r*_i.  In one dimension the lattice gradient times the
   * reference volume is exactly the gradient at r* times the displaced volume,
   * so this is the Lagrangian form of Q(U*, r*); it keeps the pairwise
   * antisymmetry of the sums (hence conservation) and the exact rest state
   * (u = 0 gives V* = h^3).  Evaluating the kernel gradients at the displaced
   * separations instead (ORC_POS_DISPLACED) adds the zeroth-order consistency
   * error of SPH: the sum of the gradients of a non-uniformly displaced
   * neighbourhood is not zero, which acts as a first-order viscosity. */
  all_primitives(s, s->rho, s->ms, s->Es);
  const int displaced = s->P.pos_mode == ORC_POS_DISPLACED;
  if (lagrange) {
    /* the pressure of the predicted particle: its internal energy over its
     * predicted volume, p* = (gamma-1)(E* - m*.u* / 2) / (V* / h^3) */
    for (int k = -1; k <= nz; ++k)
      for (int j = -1; j <= ny; ++j)
        for (int i = -1; i <= nx; ++i) {
          size_t c = IX(s, i, j, k);
          s->p[c] = s->p[c] / s->vol[c];
          s->phi[c] = sqrt(2.0 * s->p[c]);
        }
  }
  for (int k = -1; k <= nz; ++k)
    for (int j = -1; j <= ny; ++j)
      for (int i = -1; i <= nx; ++i) {
        size_t c = IX(s, i, j, k);
        s->psis[c] = (displaced || lagrange)
                         ? psi_at(s, psi_c, c, s->xs[0][c], s->xs[1][c], s->xs[2][c])
                         : psi_c[c];
      }
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t c = IX(s, i, j, k);
        double A[3], B;
        hydro_force(s, s->rho, s->phi, s->u, displaced ? s->xs : NULL, s->psis, c, A, &B);
        for (int d = 0; d < 3; ++d)
          s->mt[d][c] = 0.5 * (s->m[d][c] + s->ms[d][c]) - 0.5 * dt * A[d];
        s->Et[c] = 0.5 * (s->E[c] + s->Es[c]) - 0.5 * dt * B;
        double utx, uty, utz, pt;
        primitive(s, s->rho[c], s->mt[0][c], s->mt[1][c], s->mt[2][c], s->Et[c], &utx, &uty, &utz,
                  &pt);
        s->xt[0][c] = 0.5 * s->xs[0][c] + 0.25 * dt * (un[0][c] + utx);
        s->xt[1][c] = 0.5 * s->xs[1][c] + 0.25 * dt * (un[1][c] + uty);
        s->xt[2][c] = 0.5 * s->xs[2][c] + 0.25 * dt * (un[2][c] + utz);
      }

  /* O9: ghosts of the post-Lagrange particles */
  fill_ghosts(s, s->mt[0], R_MX, dt);
  fill_ghosts(s, s->mt[1], R_MY, dt);
  fill_ghosts(s, s->mt[2], R_MZ, dt);
  fill_ghosts(s, s->Et, R_E, dt);
  fill_ghosts(s, s->xt[0], R_XX, dt);
  fill_ghosts(s, s->xt[1], R_XY, dt);
  fill_ghosts(s, s->xt[2], R_XZ, dt);

  /* O10-O12: Eulerian stage.  For every axis d and every face i+1/2 (boundary
   * faces included), Eq. (8) gives the content of each particle's slab that
   * crosses the face,
   *   U^L = B_i     + (1/2)(h - xi_i)     Theta_i,
   *   U^R = B_{i+1} - (1/2)(h + xi_{i+1}) Theta_{i+1},
   * with Theta the TVD-limited slope of U^n and B the reconstruction base.
   * The flux of the advective part (the pressure was applied in the Lagrangian
   * stage) is HLL with the advective wave speeds xi/dt, which equals the exact
   * swept volume
   *   Phi = max(xi_i, 0) U^L + min(xi_{i+1}, 0) U^R     (= dt * face flux),
   * and Eq. (4) becomes U^{n+1} = U~ - (1/h) sum_d (Phi_{i+1/2} - Phi_{i-1/2}).
   * Each face value is computed once and used by both of its cells.
   * Reading of the swept width (ORC_FACE_FOOT, the default): the face's two
   * particles are parts of one deforming medium, so the volume that crosses the
   * face during the step is the displacement of the material that reaches it,
   * the offset field interpolated linearly between the two particles and taken
   * at the foot of the face's trajectory,
   *   X = (xi_i + xi_{i+1}) / 2 / (1 + (xi_{i+1} - xi_i) / h),
   * and Phi = max(X, 0) U^L + min(X, 0) U^R.  ORC_FACE_PARTICLE sweeps the upwind
   * particle's own offset instead (max(xi_i, 0), min(xi_{i+1}, 0)), which treats
   * each particle as a rigid cube and misplaces the remap's divergence by half a
   * cell (first order on compressive flow). */
  const double* Un[5] = {s->rho, s->m[0], s->m[1], s->m[2], s->E};
  const double* Ut[5] = {s->rho, s->mt[0], s->mt[1], s->mt[2], s->Et};
  const int mid = s->P.base_mode == ORC_BASE_MID;
  const long stride[3] = {1, s->sx, (long)s->sx * (long)s->sy};
  for (int v = 0; v < 5; ++v) memset(s->acc[v], 0, s->n * sizeof(double));
  for (int d = 0; d < 3; ++d) {
    const long st = stride[d];
    const double* xi = s->xt[d];
    /* slopes on the interior and the first ghost layer along d */
    for (int k = (d == 2 ? -1 : 0); k < nz + (d == 2 ? 1 : 0); ++k)
      for (int j = (d == 1 ? -1 : 0); j < ny + (d == 1 ? 1 : 0); ++j)
        for (int i = (d == 0 ? -1 : 0); i < nx + (d == 0 ? 1 : 0); ++i) {
          size_t c = IX(s, i, j, k);
          for (int v = 0; v < 5; ++v) {
            const double* U = Un[v];
            s->slope[v][c] = orc_limiter(s->P.limiter, U[c + st] - U[c], U[c] - U[c - st]);
          }
        }
    /* face fluxes: face i+1/2 stored at cell i, i = -1 .. n-1 along d */
    for (int k = (d == 2 ? -1 : 0); k < nz; ++k)
      for (int j = (d == 1 ? -1 : 0); j < ny; ++j)
        for (int i = (d == 0 ? -1 : 0); i < nx; ++i) {
          size_t cL = IX(s, i, j, k), cR = cL + st;
          const double xL = xi[cL], xR = xi[cR];
          const double nuL = xL * inv_h, nuR = xR * inv_h;
          double fL[5], fR[5];
          for (int v = 0; v < 5; ++v) {
            double BL = Ut[v][cL], BR = Ut[v][cR];
            if (mid) {
              BL = 0.5 * (Un[v][cL] + Ut[v][cL]);
              BR = 0.5 * (Un[v][cR] + Ut[v][cR]);
            }
            const double UL = BL + 0.5 * (1.0 - nuL) * s->slope[v][cL];
            const double UR = BR - 0.5 * (1.0 + nuR) * s->slope[v][cR];
            double F;
            if (s->P.flux == ORC_FLUX_LF) {
              const double a = fmax(fabs(xL), fabs(xR));
              F = 0.5 * (xL * UL + xR * UR) - 0.5 * a * (UR - UL);
            } else if (s->P.face_mode == ORC_FACE_FOOT) {
              const double X = 0.5 * (xL + xR) / (1.0 + (xR - xL) * inv_h);
              F = fmax(X, 0.0) * UL + fmin(X, 0.0) * UR;
            } else {
              F = fmax(xL, 0.0) * UL + fmin(xR, 0.0) * UR;
            }
            s->flux[v][cL] = F;
            fL[v] = UL;
            fR[v] = UR;
          }
          if (s->P.flux == ORC_FLUX_SWEPT_AV) {
            double D[5];
            acoustic_dissipation(s, d, fL, fR, D);
            for (int v = 1; v < 5; ++v) s->flux[v][cL] = s->flux[v][cL] + dt * D[v];
          }
        }
    /* accumulate the flux differences of this axis */
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          size_t c = IX(s, i, j, k);
          for (int v = 0; v < 5; ++v)
            s->acc[v][c] = s->acc[v][c] + (s->flux[v][c] - s->flux[v][c - st]);
        }
  }
  /* Eq. (4) */
  double* Uout[5] = {s->rho, s->m[0], s->m[1], s->m[2], s->E};
  int status = ORC_OK;
  const double neg_tol = -0.01 * s->P.rho_vac;
  double tot[5] = {0, 0, 0, 0, 0};
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t c = IX(s, i, j, k);
        double nv[5];
        for (int v = 0; v < 5; ++v) nv[v] = Ut[v][c] - inv_h * s->acc[v][c];
        /* sources and sinks: the second half step */
        if (s->has_src) source_cell(s->src[c], s->eps_src, 0.5 * dt, &nv[0], &nv[1], &nv[2], &nv[3], &nv[4]);
        for (int v = 0; v < 5; ++v) {
          if (!isfinite(nv[v])) status = ORC_ERR_NONFINITE;
          tot[v] += nv[v];
        }
        if (nv[0] < neg_tol && status == ORC_OK) status = ORC_ERR_NEG_DENSITY;
        /* rho^{n+1} may be written now: every read of rho^n in this stage is done */
        for (int v = 0; v < 5; ++v) s->slope[v][c] = nv[v];
      }
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t c = IX(s, i, j, k);
        for (int v = 0; v < 5; ++v) Uout[v][c] = s->slope[v][c];
      }

  /* O13: time, totals */
  const double h3 = h * h * h;
  for (int v = 0; v < 5; ++v) s->totals[v] = tot[v] * h3;
  s->t = lands ? t_end : s->t + dt;
  s->nsteps += 1;
  if (dt_taken) *dt_taken = dt;
  return status;
}

int orc_advance(orc_sim* s, double t_end, int64_t max_steps, int64_t* steps) {
  int64_t n = 0;
  int st = ORC_OK;
  while (n < max_steps && (!isfinite(t_end) || s->t < t_end)) {
    st = orc_step(s, 0.0, t_end, NULL);
    if (st != ORC_OK) break;
    ++n;
  }
  if (steps) *steps = n;
  return st;
}

/* ------------------------------------------------------------------------ */
/* building blocks for the unit tests                                        */
/* ------------------------------------------------------------------------ */
int orc_lattice_gradient(int32_t nx, int32_t ny, int32_t nz, double h, const double* f,
                         double* out) {
  orc_params P;
  memset(&P, 0, sizeof P);
  P.nx = nx;
  P.ny = ny;
  P.nz = nz;
  P.h = h;
  P.gamma = 1.4;
  P.cfl = 0.4;
  orc_sim* s;
  int st = orc_create(&P, &s); /* all faces periodic (0) */
  if (st) return st;
  /* the gradient of f alone: phi = 1 everywhere, rho = 1, psi = f  =>  A = D[f] */
  for (size_t c = 0; c < s->n; ++c) {
    s->rho[c] = 1.0;
    s->phi[c] = 0.0;
  }
  orc_set_potential(s, f);
  const size_t N = (size_t)nx * ny * nz;
  size_t q = 0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i, ++q) {
        double A[3], B;
        hydro_force(s, s->rho, s->phi, s->u, NULL, s->psi, IX(s, i, j, k), A, &B);
        out[q] = A[0];
        out[N + q] = A[1];
        out[2 * N + q] = A[2];
      }
  orc_destroy(s);
  return ORC_OK;
}

int orc_interp_psi(orc_sim* s, const double* off, double* out) {
  if (!s || !off || !out) return ORC_ERR_ARG;
  const size_t N = ninterior(s);
  size_t q = 0;
  for (int k = 0; k < s->P.nz; ++k)
    for (int j = 0; j < s->P.ny; ++j)
      for (int i = 0; i < s->P.nx; ++i, ++q)
        out[q] = psi_at(s, s->psi, IX(s, i, j, k), off[q], off[N + q], off[2 * N + q]);
  return ORC_OK;
}

int orc_fill_ghosts_padded(orc_sim* s, double* padded, int role, double dt) {
  if (!s || !padded || role < 0 || role > 9) return ORC_ERR_ARG;
  fill_ghosts(s, padded, role, dt);
  return ORC_OK;
}
