/* Exercises every entry point of the CPU oracle on small and degenerate
 * lattices (narrower than the stencils, the minimum wall and mirror sizes),
 * for a build with the host sanitizers.  Exit status 0 when every call
 * returns the documented status; any out-of-bounds access aborts. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "olb_oracle.h"

static int failures = 0;

static void expect(const char* what, int got, int want) {
  if (got != want) {
    fprintf(stderr, "%s: got %d, want %d\n", what, got, want);
    ++failures;
  }
}

static oolb_params params(int nx, int ny, int bc_x, int bc_y) {
  oolb_params p;
  memset(&p, 0, sizeof p);
  p.nx = nx;
  p.ny = ny;
  p.ds = 1.0 / 32;
  p.dt = 5e-4;
  p.tau = 0.01;
  p.a = 9.0 / 49;
  p.b = 2.0 / 21;
  p.sigma = 1e-4;
  p.bc_x = bc_x;
  p.bc_y = bc_y;
  p.tw_lo = 0.9;
  p.tw_hi = 1.1;
  p.uw_lo = 0.0;
  p.uw_hi = 0.02;
  return p;
}

static void run(int nx, int ny, int bc_x, int bc_y) {
  oolb_params p = params(nx, ny, bc_x, bc_y);
  oolb_ctx* c = NULL;
  char what[64];
  snprintf(what, sizeof what, "init %dx%d bc %d/%d", nx, ny, bc_x, bc_y);
  expect(what, oolb_init(&p, &c), OOLB_OK);
  if (!c) return;
  size_t np = (size_t)nx * ny;
  double* n = malloc(np * sizeof(double));
  double* ux = malloc(np * sizeof(double));
  double* uy = malloc(np * sizeof(double));
  double* T = malloc(np * sizeof(double));
  double* f = malloc(25 * np * sizeof(double));
  double* L = malloc(25 * np * sizeof(double));
  double* glo = malloc(75 * (size_t)nx * sizeof(double));
  double* ghi = malloc(75 * (size_t)nx * sizeof(double));
  double* nlo = malloc((size_t)nx * sizeof(double));
  double* nhi = malloc((size_t)nx * sizeof(double));
  expect("step before fields", oolb_step(c, 1), OOLB_E_STATE);
  for (size_t i = 0; i < np; ++i) {
    n[i] = 2.0 + 0.1 * sin(0.7 * (double)i);
    ux[i] = 0.01 * cos(1.3 * (double)i);
    uy[i] = 0.01 * sin(0.4 * (double)i);
    T[i] = 1.0 + 0.05 * cos(0.9 * (double)i);
  }
  expect("set_fields", oolb_set_fields(c, n, ux, uy, T), OOLB_OK);
  expect("step", oolb_step(c, 2), OOLB_OK);
  expect("moments", oolb_moments(c, n, ux, uy, T), OOLB_OK);
  expect("get_f", oolb_get_f(c, f), OOLB_OK);
  expect("rhs", oolb_rhs(c, f, L), OOLB_OK);
  expect("set_f", oolb_set_f(c, f), OOLB_OK);
  int want = bc_y ? OOLB_OK : OOLB_E_STATE;
  expect("wall density", oolb_wall_density(c, nlo, nhi), want);
  expect("wall ghosts", oolb_wall_ghosts(c, glo, ghi), want);
  n[0] = 1.0 / p.b;    /* n >= 1/b is outside the domain */
  expect("domain", oolb_set_fields(c, n, ux, uy, T), OOLB_E_DOMAIN);
  if (strlen(oolb_last_error(c)) == 0) ++failures;
  free(n); free(ux); free(uy); free(T); free(f); free(L);
  free(glo); free(ghi); free(nlo); free(nhi);
  oolb_free(c);
}

int main(void) {
  double R[5], W[5], w[3], out[25], dx[25], dy[25], g[16], D[49];
  oolb_quadrature(R, W);
  for (int l = 0; l <= 6; ++l) (void)oolb_hermite(l, R[4]);
  for (int k = 0; k < 5; ++k) (void)oolb_g(k, 0.1, 0.8);
  oolb_feq(1.0, 0.1, -0.2, 0.9, out);
  oolb_dpf(out, dx, dy);
  double v[5] = {1, 1, 1, 2, 3};
  (void)oolb_weno_recon(v, w);
  (void)oolb_weno_recon(v, NULL);
  oolb_stencil_tables(g, D);
  double field[12];
  for (int i = 0; i < 12; ++i) field[i] = (double)(i * i);
  double o2[2];
  oolb_grad(field, 4, 3, 0.25, 0, 0, o2);
  oolb_glap(field, 4, 3, 0.25, 3, 2, o2);
  (void)oolb_pw(1.0, 1.0, 9.0 / 8, 1.0 / 3);
  /* lattices smaller than the 7x7 stencils and the WENO halo */
  run(1, 1, 0, 0);
  run(2, 5, 0, 0);
  run(7, 3, 0, 1);
  run(3, 3, 3, 1);
  run(3, 4, 3, 2);
  run(5, 3, 0, 2);
  run(9, 6, 3, 0);
  /* argument errors */
  oolb_params p = params(4, 4, 0, 0);
  oolb_ctx* c = NULL;
  expect("null", oolb_init(NULL, &c), OOLB_E_ARG);
  p.dt = 0.02;
  expect("cfl", oolb_init(&p, &c), OOLB_E_CFL);
  p = params(4, 2, 0, 1);
  expect("walls short", oolb_init(&p, &c), OOLB_E_ARG);
  p = params(2, 4, 3, 0);
  expect("mirror narrow", oolb_init(&p, &c), OOLB_E_ARG);
  p = params(4, 4, 0, 0);
  p.tau = 0.0;
  expect("tau", oolb_init(&p, &c), OOLB_E_DOMAIN);
  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("oracle: all entry points ran clean\n");
  return 0;
}
