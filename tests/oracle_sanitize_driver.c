/*
 * A host-only driver for the CPU oracle, built by the test suite with
 * AddressSanitizer and UndefinedBehaviorSanitizer.  It runs a few steps of small
 * problems that together touch every code path of the oracle: each boundary
 * kind on each face, inflow faces, vacuum cells, a potential, every limiter and
 * face flux, both corrector position modes and reconstruction bases, the error
 * returns, and the building blocks the unit tests call.  Exit status 0 and the
 * line "cases ok" mean no sanitizer report.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "csph_oracle.h"

static int fail(const char* what, int code) {
  printf("FAIL %s: %d\n", what, code);
  fflush(stdout);
  exit(1);
}

/* a seeded, non-smooth primitive state (rho, p in [0.5, 1.5], |u| <= 0.5),
 * with a vacuum slab when `vacuum` is set */
static void fill_state(double* w, int nx, int ny, int nz, unsigned seed, int vacuum) {
  const size_t N = (size_t)nx * ny * nz;
  srand(seed);
  for (size_t q = 0; q < N; ++q) {
    w[q] = 0.5 + (double)rand() / RAND_MAX;
    for (int d = 1; d < 4; ++d) w[d * N + q] = (double)rand() / RAND_MAX - 0.5;
    w[4 * N + q] = 0.5 + (double)rand() / RAND_MAX;
    if (vacuum && (q % (size_t)nx) >= (size_t)(nx / 2)) {
      for (int v = 0; v < 5; ++v) w[v * N + q] = 0.0;
    }
  }
}

static int run_case(const int bc[6], int nx, int ny, int nz, int vacuum, int psi_on, int pos,
                    int base, int lim, int flux, unsigned seed) {
  orc_params P;
  memset(&P, 0, sizeof P);
  P.nx = nx;
  P.ny = ny;
  P.nz = nz;
  P.h = 1.0 / nx;
  P.gamma = 1.4;
  P.cfl = 0.4;
  P.rho_vac = 1e-10;
  P.face_mode = (int)(seed & 1u); /* both swept widths */
  for (int f = 0; f < 6; ++f) {
    P.bc[f] = bc[f];
    P.inflow[f][0] = 1.0;
    P.inflow[f][1] = f == 0 ? 0.5 : 0.0;
    P.inflow[f][4] = 0.7;
  }
  P.pos_mode = pos;
  P.base_mode = base;
  P.limiter = lim;
  P.flux = flux;
  orc_sim* s = NULL;
  int st = orc_create(&P, &s);
  if (st) return fail("create", st);
  const size_t N = (size_t)nx * ny * nz;
  double* w = (double*)malloc(5 * N * sizeof(double));
  double* out = (double*)malloc(5 * N * sizeof(double));
  double* psi = (double*)malloc(N * sizeof(double));
  fill_state(w, nx, ny, nz, seed, vacuum);
  if ((st = orc_set_primitive(s, w))) return fail("set_primitive", st);
  for (size_t q = 0; q < N; ++q) psi[q] = 0.1 * sin(0.37 * (double)q);
  if ((st = orc_set_potential(s, psi_on ? psi : NULL))) return fail("set_potential", st);
  double dt = 0.0;
  for (int k = 0; k < 3; ++k) {
    /* the third step is shortened to land on an end time */
    double t0;
    orc_get_time(s, &t0, NULL);
    st = orc_step(s, 0.0, k == 2 ? t0 + 0.5 * dt : INFINITY, &dt);
    if (st && st != ORC_ERR_NEG_DENSITY) return fail("step", st);
  }
  int64_t n = 0;
  st = orc_advance(s, INFINITY, 2, &n);
  if (st && st != ORC_ERR_NEG_DENSITY) return fail("advance", st);
  if ((st = orc_get_conserved(s, out))) return fail("get_conserved", st);
  for (int f = 0; f < ORC_F_COUNT; ++f)
    if ((st = orc_get_field(s, f, out))) return fail("get_field", st);
  double tot[5], t;
  int64_t ns;
  orc_totals(s, tot);
  orc_get_time(s, &t, &ns);
  orc_set_time(s, t, ns);
  (void)orc_cfl_dt(s);
  if ((st = orc_interp_psi(s, out, out + 3 * N))) return fail("interp_psi", st);
  const size_t padded = (size_t)(nx + 4) * (ny + 4) * (nz + 4);
  double* pad = (double*)calloc(padded, sizeof(double));
  for (int role = 0; role <= 8; ++role)
    if ((st = orc_fill_ghosts_padded(s, pad, role, 1e-3))) return fail("fill", st);
  /* error returns: a negative density, a bad field index */
  w[0] = -1.0;
  if (orc_set_primitive(s, w) != ORC_ERR_ARG) return fail("negative density accepted", 0);
  if (orc_get_field(s, ORC_F_COUNT, out) != ORC_ERR_ARG) return fail("bad field", 0);
  free(pad);
  free(w);
  free(out);
  free(psi);
  orc_destroy(s);
  return 0;
}

int main(void) {
  int bad = 0, cases = 0;
  const int kinds[4] = {ORC_PERIODIC, ORC_OUTFLOW, ORC_INFLOW, ORC_REFLECT};
  /* every non-periodic pair on x, with the other axes cycling through rules */
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      if ((a == 0) != (b == 0)) continue;
      int bc[6] = {kinds[a], kinds[b], kinds[(a + 1) % 4], kinds[(a + 1) % 4] == 0 ? 0 : kinds[b],
                   kinds[(b + 2) % 4], kinds[(b + 2) % 4] == 0 ? 0 : kinds[a]};
      if ((bc[2] == 0) != (bc[3] == 0)) bc[3] = bc[2];
      if ((bc[4] == 0) != (bc[5] == 0)) bc[5] = bc[4];
      bad |= run_case(bc, 6, 5, 4, 0, 1, ORC_POS_LAGRANGE, ORC_BASE_POST, ORC_LIM_MINMOD,
                      ORC_FLUX_SWEPT_AV, 1u + (unsigned)(4 * a + b));
      ++cases;
    }
  const int per[6] = {0, 0, 0, 0, 0, 0};
  const int out[6] = {1, 1, 1, 1, 1, 1};
  for (int lim = 0; lim < 4; ++lim)
    for (int flux = 0; flux < 3; ++flux) {
      bad |= run_case(per, 5, 4, 6, 0, lim & 1, lim % 3, (lim >> 1) & 1, lim, flux, 77u + (unsigned)flux);
      ++cases;
    }
  bad |= run_case(out, 8, 4, 4, 1, 1, ORC_POS_LAGRANGE, ORC_BASE_POST, ORC_LIM_MINMOD,
                  ORC_FLUX_SWEPT_AV, 5u);
  ++cases;
  /* building blocks */
  double K[3];
  orc_kernel_grad(0.3, -0.2, 0.1, 1.0, K);
  (void)orc_kappa();
  for (int lim = 0; lim < 4; ++lim) (void)orc_limiter(lim, 0.3, -0.1), (void)orc_limiter(lim, 0.3, 0.1);
  {
    const int nx = 5, ny = 4, nz = 4;
    double f[80], g[240];
    for (int q = 0; q < nx * ny * nz; ++q) f[q] = cos(0.1 * q);
    if (orc_lattice_gradient(nx, ny, nz, 0.2, f, g)) bad = 1;
    ++cases;
  }
  if (bad) return 1;
  printf("%d cases ok\n", cases);
  return 0;
}
