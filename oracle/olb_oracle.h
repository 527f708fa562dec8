/*
 * olb_oracle.h -- plain FP64 CPU oracle of the D2Q25 off-lattice thermal
 * Boltzmann stage update (Busuioc, Ambrus, Biciusca, Sofonea, arXiv:1702.01690).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the GPU library; every constant here
 * is recomputed from the paper's closed forms.
 *
 * All arrays are host memory, row-major.  Macroscopic fields are [ny][nx];
 * distributions are [25][ny][nx] with population index k = 5*ky + kx, where
 * kx, ky in 0..4 index the ascending Hermite roots (p = R[kx], R[ky]).
 * Every function returns 0 on success and a negative OOLB_E_* code on error.
 */
#ifndef OLB_ORACLE_H
#define OLB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  OOLB_OK = 0,
  OOLB_E_ARG = -1,       /* bad argument (null pointer, bad size, bad kind)   */
  OOLB_E_CFL = -2,       /* p_max dt / (m ds) >= 1 (Sec. 4.1 CFL condition)   */
  OOLB_E_DOMAIN = -3,    /* n outside (0, 1/b), T <= 0, tau <= 0              */
  OOLB_E_NONFINITE = -4, /* a distribution became NaN or infinite             */
  OOLB_E_WORKSPACE = -5,
  OOLB_E_DEVICE = -6,
  OOLB_E_STATE = -7      /* call out of order (e.g. step before set_fields)   */
};

/* bc_y: OOLB_BC_DIFFUSE = diffuse walls at both ends of y;
 * OOLB_BC_SPECULAR_DIFFUSE = a specular symmetry plane at the low end (Sec.
 * 3.4.1) and a diffuse wall at the high end (the half channel of Sec. 5).
 * bc_x: periodic, or OOLB_BC_SPECULAR = specular planes at both ends of x
 * (Sec. 3.4.1 across x; with walls in y the corner ghosts are reflected
 * twice, as in the Laplace test of Sec. 6). */
enum { OOLB_BC_PERIODIC = 0, OOLB_BC_DIFFUSE = 1, OOLB_BC_SPECULAR_DIFFUSE = 2, OOLB_BC_SPECULAR = 3 };

/* Problem statement (Sec. 2 and 3): lattice nx*ny of spacing ds, RK-3 step dt,
 * BGK relaxation time tau, EOS p^w = nT/(1-bn) - a n^2, surface-tension
 * parameter sigma, per-axis boundary kind, wall temperature / tangential
 * velocity of the lower (y = -ds/2) and upper (y = (ny - 1/2) ds) walls.
 * Walls are supported perpendicular to y only; bc_x is periodic or specular.
 * precision and rho_ref exist for layout compatibility and are ignored: the
 * oracle is always FP64. */
typedef struct oolb_params {
  int32_t nx, ny;
  double ds, dt, tau;
  double a, b, sigma;
  int32_t bc_x, bc_y;
  double tw_lo, tw_hi, uw_lo, uw_hi;
  int32_t precision;
  double rho_ref;
} oolb_params;

typedef struct oolb_ctx oolb_ctx;

int oolb_init(const oolb_params* p, oolb_ctx** out);
void oolb_free(oolb_ctx* c);
/* f <- f^eq(n, u, T) at every node (equilibrium start). */
int oolb_set_fields(oolb_ctx* c, const double* n, const double* ux,
                    const double* uy, const double* T);
int oolb_set_f(oolb_ctx* c, const double* f);
int oolb_get_f(const oolb_ctx* c, double* f);
/* nsteps full RK-3 steps (Eq. rk3). */
int oolb_step(oolb_ctx* c, int32_t nsteps);
int oolb_moments(const oolb_ctx* c, double* n, double* ux, double* uy, double* T);
/* L[f] of Eq. ecast for an arbitrary f (walls: ghosts are refreshed from f). */
int oolb_rhs(oolb_ctx* c, const double* f, double* L);
/* Wall densities n_w [nx] of the most recent ghost fill (walls only). */
int oolb_wall_density(const oolb_ctx* c, double* nw_lo, double* nw_hi);
/* Ghost rows of the most recent ghost fill (walls only), [25][3][nx] per
 * wall: layer j of the lower wall is row y = -1 - j, of the upper wall row
 * y = ny + j. */
int oolb_wall_ghosts(const oolb_ctx* c, double* glo, double* ghi);
const char* oolb_last_error(const oolb_ctx* c);
void oolb_set_threads(int n);
int oolb_get_threads(void);

/* ---- individual pieces, exported so the tests can pin them one by one ---- */
/* Roots R_q of He_5 and weights W_q = Q!/He_6(R_q)^2 (Table trots). */
void oolb_quadrature(double R[5], double W[5]);
/* Probabilists' Hermite polynomial He_l(p). */
double oolb_hermite(int l, double p);
/* 1-D equilibrium factor g_k(u, T) of Eq. g_alpha, k = 0..4. */
double oolb_g(int k, double u, double T);
/* f^eq of Eq. feq at one node, out[25]. */
void oolb_feq(double n, double ux, double uy, double T, double out[25]);
/* Hermite-projected momentum derivative of Eq. derf at one node. */
void oolb_dpf(const double f[25], double dfx[25], double dfy[25]);
/* WENO-5 upwind reconstruction (Eqs. weno5_flux..weno5_sigma and Tab. weno)
 * from v = (f_{i-2}, f_{i-1}, f_i, f_{i+1}, f_{i+2}) for a positive speed;
 * returns the face value without the p/m factor, weights in w[3]. */
double oolb_weno_recon(const double v[5], double w[3]);
/* 7x7 stencils of Eqs. stencil_grad / stencil_glap applied at node (x, y) of a
 * periodic nx*ny field g (spacing ds): out = {d_x g, d_y g}. */
void oolb_grad(const double* g, int nx, int ny, double ds, int x, int y, double out[2]);
void oolb_glap(const double* g, int nx, int ny, double ds, int x, int y, double out[2]);
/* Stencil coefficient tables as the oracle uses them: gw[l][m] = w^{l,m}
 * (l, m = 0..3) and D[l+3][m+3] = coefficient of n_{i+l,j+m} in ds^3 d_x lap n. */
void oolb_stencil_tables(double gw[16], double D[49]);
/* vdW pressure p^w = nT/(1-bn) - a n^2. */
double oolb_pw(double n, double T, double a, double b);

#ifdef __cplusplus
}
#endif
#endif
