/*
 * olb_oracle.c -- plain FP64 CPU oracle of the D2Q25 off-lattice thermal
 * Boltzmann model of Busuioc, Ambrus, Biciusca, Sofonea (arXiv:1702.01690).
 *
 * TEST INFRASTRUCTURE ONLY: the GPU library never links or calls this file.
 * It follows the paper's steps in the paper's order, in plain scalar loops:
 *   Sec. 2.2  Gauss-Hermite Q=5 quadrature (Table trots) and the equilibrium
 *             of Eqs. feq / g_alpha, written as the explicit double sum.
 *   Sec. 2.3  force F of Eq. F_def and the Hermite-projected momentum
 *             derivative of Eq. derf, with the explicit l-loop.
 *   Sec. 3.1  third-order TVD Runge-Kutta of Eq. rk3 on L of Eq. ecast.
 *   Sec. 3.2  WENO-5 of Eqs. weno5_flux..weno5_sigma, no epsilon, with the
 *             vanishing-indicator table (Tab. weno).
 *   Sec. 3.3  49-point stencils of Eqs. stencil_grad and stencil_glap.
 *   Sec. 3.4  diffuse-reflection ghosts (Eqs. diffuse_flux, nw, quadratic
 *             extrapolation) and mirrored macroscopic fields.
 * Readings where the paper is silent or garbled (each is listed with its
 * justification in the project design notes):
 *   - EOS in the general form p^w = nT/(1-bn) - a n^2; the paper's reduced form
 *     is a = 9/8, b = 1/3.  m = k_B = 1.
 *   - Temperature: T = sum f |p - m u|^2 / (2 m n) (trace of Eq. sigmaq_def
 *     with p^i = nT, D = 2).
 *   - WENO for p < 0 is the mirror image of the printed p > 0 form.
 *   - Gradient-of-Laplacian coefficients c_1 and c_4 as printed are
 *     inconsistent with the 1-D reduction of Sec. 4 and with polynomial
 *     exactness; the consistent values c_1 = -17/2160 and c_4 = -59/540 are
 *     used, and the stencil is oriented so that it reduces to the printed 1-D
 *     third-derivative stencil.
 *   - Walls are perpendicular to y (the paper's rule transposed): ghost rows
 *     y = -1,-2,-3 and ny, ny+1, ny+2; wall equilibrium with normal velocity 0
 *     and tangential velocity u_w.  Ghosts, n_w and F are recomputed from the
 *     current f at every RK stage.
 * Compiled with -O2 -ffp-contract=off and no fast-math.
 */
#include "olb_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QN 5          /* quadrature order Q */
#define KV 25         /* number of velocities K = Q^2 */
#define NEXP 4        /* expansion order N of f^eq */
#define MASS 1.0      /* particle mass m, kept explicit as in the paper */

struct oolb_ctx {
  oolb_params p;
  int nx, ny;
  int have_f;
  double R[QN], W[QN];
  double *f, *f1, *f2, *L;           /* [25][ny][nx] */
  double *n, *ux, *uy, *T, *dp;       /* [ny][nx] */
  double *Fx, *Fy;                    /* [ny][nx] */
  double *glo, *ghi;                  /* wall ghosts [25][3][nx] */
  double *nwlo, *nwhi;                /* wall densities [nx] */
  char err[256];
};

/* ------------------------------------------------------------------------- */
/* Sec. 2.2: quadrature and Hermite polynomials                              */
/* ------------------------------------------------------------------------- */

double oolb_hermite(int l, double p) {
  /* He_0 = 1, He_1 = p, He_{l+1} = p He_l - l He_{l-1} (probabilists'). */
  if (l == 0) return 1.0;
  double hm = 1.0, h = p;
  for (int j = 1; j < l; ++j) {
    double hp = p * h - (double)j * hm;
    hm = h;
    h = hp;
  }
  return h;
}

void oolb_quadrature(double R[5], double W[5]) {
  /* Table trots: roots of He_5 in ascending order. */
  double s10 = sqrt(10.0);
  R[0] = -sqrt(5.0 + s10);
  R[1] = -sqrt(5.0 - s10);
  R[2] = 0.0;
  R[3] = sqrt(5.0 - s10);
  R[4] = sqrt(5.0 + s10);
  /* Weight formula of Sec. 2.2: W_q = Q! / [He_{Q+1}(R_q)]^2, Q = 5. */
  for (int q = 0; q < QN; ++q) {
    double h6 = oolb_hermite(QN + 1, R[q]);
    W[q] = 120.0 / (h6 * h6);
  }
}

static double factorial(int k) {
  double r = 1.0;
  for (int j = 2; j <= k; ++j) r *= (double)j;
  return r;
}

/* Eq. g_alpha: g_k(u, T) = w_k sum_{l=0}^{N} He_l(p_k)
 *   sum_{s=0}^{floor(l/2)} (mT - 1)^s (m u)^{l-2s} / (2^s s! (l-2s)!). */
static double g_axis(const double R[5], const double W[5], int k, double u, double T) {
  double acc = 0.0;
  for (int l = 0; l <= NEXP; ++l) {
    double inner = 0.0;
    for (int s = 0; s <= l / 2; ++s) {
      inner += pow(MASS * T - 1.0, s) * pow(MASS * u, l - 2 * s) /
               (pow(2.0, s) * factorial(s) * factorial(l - 2 * s));
    }
    acc += oolb_hermite(l, R[k]) * inner;
  }
  return W[k] * acc;
}

double oolb_g(int k, double u, double T) {
  double R[5], W[5];
  oolb_quadrature(R, W);
  return g_axis(R, W, k, u, T);
}

/* Eq. feq: f^eq_kappa = n g_{k1}(u_x, T) g_{k2}(u_y, T). */
static void feq_node(const double R[5], const double W[5], double n, double ux,
                     double uy, double T, double out[25]) {
  double gx[QN], gy[QN];
  for (int k = 0; k < QN; ++k) {
    gx[k] = g_axis(R, W, k, ux, T);
    gy[k] = g_axis(R, W, k, uy, T);
  }
  for (int ky = 0; ky < QN; ++ky)
    for (int kx = 0; kx < QN; ++kx) out[5 * ky + kx] = n * gx[kx] * gy[ky];
}

void oolb_feq(double n, double ux, double uy, double T, double out[25]) {
  double R[5], W[5];
  oolb_quadrature(R, W);
  feq_node(R, W, n, ux, uy, T, out);
}

/* Eq. derf: (d_{p_a} f)_kappa = - w_{k_a} sum_{l=0}^{N-1} (1/l!)
 *   F_{a,l;k_abar} He_{l+1}(p_{k_a}),  F_{a,l;k_abar} = sum_{k_a} f He_l(p_{k_a}). */
static void dpf_node(const double R[5], const double W[5], const double f[25],
                     double dfx[25], double dfy[25]) {
  for (int ky = 0; ky < QN; ++ky) {
    for (int kx = 0; kx < QN; ++kx) {
      /* derivative along x: sum over kx' at fixed ky */
      double sx = 0.0;
      for (int l = 0; l <= NEXP - 1; ++l) {
        double Fl = 0.0;
        for (int kk = 0; kk < QN; ++kk) Fl += f[5 * ky + kk] * oolb_hermite(l, R[kk]);
        sx += Fl * oolb_hermite(l + 1, R[kx]) / factorial(l);
      }
      dfx[5 * ky + kx] = -W[kx] * sx;
      /* derivative along y: sum over ky' at fixed kx */
      double sy = 0.0;
      for (int l = 0; l <= NEXP - 1; ++l) {
        double Fl = 0.0;
        for (int kk = 0; kk < QN; ++kk) Fl += f[5 * kk + kx] * oolb_hermite(l, R[kk]);
        sy += Fl * oolb_hermite(l + 1, R[ky]) / factorial(l);
      }
      dfy[5 * ky + kx] = -W[ky] * sy;
    }
  }
}

void oolb_dpf(const double f[25], double dfx[25], double dfy[25]) {
  double R[5], W[5];
  oolb_quadrature(R, W);
  dpf_node(R, W, f, dfx, dfy);
}

double oolb_pw(double n, double T, double a, double b) {
  /* Eq. vdw in the general van der Waals form (a = 9/8, b = 1/3 gives
   * 3nT/(3-n) - 9n^2/8). */
  return n * T / (1.0 - b * n) - a * n * n;
}

/* ------------------------------------------------------------------------- */
/* Sec. 3.2: WENO-5                                                          */
/* ------------------------------------------------------------------------- */

/* v = (f_{i-2}, f_{i-1}, f_i, f_{i+1}, f_{i+2}); reconstruction at i+1/2 for
 * a positive advection speed. */
double oolb_weno_recon(const double v[5], double w[3]) {
  const double fm2 = v[0], fm1 = v[1], f0 = v[2], fp1 = v[3], fp2 = v[4];
  /* interpolating functions (divided by p/m) */
  double c1 = (1.0 / 3.0) * fm2 - (7.0 / 6.0) * fm1 + (11.0 / 6.0) * f0;
  double c2 = -(1.0 / 6.0) * fm1 + (5.0 / 6.0) * f0 + (1.0 / 3.0) * fp1;
  double c3 = (1.0 / 3.0) * f0 + (5.0 / 6.0) * fp1 - (1.0 / 6.0) * fp2;
  /* indicators of smoothness, Eq. weno5_sigma */
  double a1 = fm2 - 2.0 * fm1 + f0, b1 = fm2 - 4.0 * fm1 + 3.0 * f0;
  double a2 = fm1 - 2.0 * f0 + fp1, b2 = fm1 - fp1;
  double a3 = f0 - 2.0 * fp1 + fp2, b3 = 3.0 * f0 - 4.0 * fp1 + fp2;
  double s1 = (13.0 / 12.0) * a1 * a1 + 0.25 * b1 * b1;
  double s2 = (13.0 / 12.0) * a2 * a2 + 0.25 * b2 * b2;
  double s3 = (13.0 / 12.0) * a3 * a3 + 0.25 * b3 * b3;
  const double d1 = 0.1, d2 = 0.6, d3 = 0.3; /* Eq. weno5_delta */
  int z1 = (s1 == 0.0), z2 = (s2 == 0.0), z3 = (s3 == 0.0);
  double w1, w2, w3;
  if (z1 && z2 && z3) {            /* Tab. weno, first row */
    w1 = 0.1; w2 = 0.6; w3 = 0.3;
  } else if (z2 && z3) {
    w1 = 0.0; w2 = 2.0 / 3.0; w3 = 1.0 / 3.0;
  } else if (z3 && z1) {
    w1 = 0.25; w2 = 0.0; w3 = 0.75;
  } else if (z1 && z2) {
    w1 = 1.0 / 7.0; w2 = 6.0 / 7.0; w3 = 0.0;
  } else if (z1) {
    w1 = 1.0; w2 = 0.0; w3 = 0.0;
  } else if (z2) {
    w1 = 0.0; w2 = 1.0; w3 = 0.0;
  } else if (z3) {
    w1 = 0.0; w2 = 0.0; w3 = 1.0;
  } else {                         /* Eq. weno5_omega, epsilon-free */
    double t1 = d1 / (s1 * s1), t2 = d2 / (s2 * s2), t3 = d3 / (s3 * s3);
    double ts = t1 + t2 + t3;
    w1 = t1 / ts; w2 = t2 / ts; w3 = t3 / ts;
  }
  if (w) { w[0] = w1; w[1] = w2; w[2] = w3; }
  return w1 * c1 + w2 * c2 + w3 * c3;
}

/* Flux through the face between nodes i and i+1 of a line g(j), j = i-2..i+3:
 * (p/m) times the upwind reconstruction; the p < 0 branch is the mirror image. */
static double face_flux(double p, double gm2, double gm1, double g0, double gp1,
                        double gp2, double gp3) {
  double v[5];
  if (p > 0.0) {
    v[0] = gm2; v[1] = gm1; v[2] = g0; v[3] = gp1; v[4] = gp2;
  } else if (p < 0.0) {
    v[0] = gp3; v[1] = gp2; v[2] = gp1; v[3] = g0; v[4] = gm1;
  } else {
    return 0.0;
  }
  return (p / MASS) * oolb_weno_recon(v, NULL);
}

/* ------------------------------------------------------------------------- */
/* Sec. 3.3: 49-point stencils                                               */
/* ------------------------------------------------------------------------- */

/* Gradient weights w^{|l|,|m|} of Eq. stencil_grad, symmetric in (l, m). */
static double grad_w(int al, int am) {
  static const double t[4][4] = {
      {0.0, 31.0 / 70.0, 0.0, -1.0 / 630.0},
      {31.0 / 70.0, 27.0 / 140.0, -3.0 / 70.0, 1.0 / 280.0},
      {0.0, -3.0 / 70.0, 3.0 / 560.0, 0.0},
      {-1.0 / 630.0, 1.0 / 280.0, 0.0, 0.0}};
  return t[al][am];
}

/* Matrix S of Eq. stencil_glap in its printed layout (rows and columns -3..3),
 * with c_1 and c_4 replaced by the consistent values (see header comment). */
static void glap_matrix(double S[7][7]) {
  const double c1 = -17.0 / 2160.0, c2 = 0.0, c3 = 0.0, c4 = -59.0 / 540.0;
  const double c5 = 0.0, c6 = 13.0 / 120.0, c7 = -7.0 / 30.0, c8 = 5.0 / 4.0;
  const double c9 = 0.0, c10 = -7.0 / 60.0, c11 = 187.0 / 240.0, c12 = -59.0 / 20.0;
  const double row[4][3] = {{c1, c5, c9}, {c2, c6, c10}, {c3, c7, c11}, {c4, c8, c12}};
  for (int r = 0; r < 7; ++r) {
    int rr = r <= 3 ? r : 6 - r;
    for (int c = 0; c < 3; ++c) {
      S[r][c] = row[rr][c];
      S[r][6 - c] = -row[rr][c];
    }
    S[r][3] = 0.0;
  }
}

/* Coefficient of n_{i+l, j+m} in ds^3 d_x (lap n): the printed column index
 * runs against l, which is the orientation that reproduces the printed 1-D
 * reduction (-1/8, 1, -13/8, 0, 13/8, -1, 1/8 for n_{i+3..i-3}). */
static double glap_D(const double S[7][7], int l, int m) { return S[3 + m][3 - l]; }

void oolb_stencil_tables(double gw[16], double D[49]) {
  double S[7][7];
  glap_matrix(S);
  for (int l = 0; l < 4; ++l)
    for (int m = 0; m < 4; ++m) gw[4 * l + m] = grad_w(l, m);
  for (int l = -3; l <= 3; ++l)
    for (int m = -3; m <= 3; ++m) D[(l + 3) * 7 + (m + 3)] = glap_D(S, l, m);
}

static int wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

void oolb_grad(const double* g, int nx, int ny, double ds, int x, int y, double out[2]) {
  double sx = 0.0, sy = 0.0;
  for (int l = -3; l <= 3; ++l)
    for (int m = -3; m <= 3; ++m) {
      double w = grad_w(abs(l), abs(m));
      double v = g[wrap(y + m, ny) * nx + wrap(x + l, nx)];
      sx += (double)l * w * v;
      sy += (double)m * w * v;
    }
  out[0] = sx / ds;
  out[1] = sy / ds;
}

void oolb_glap(const double* g, int nx, int ny, double ds, int x, int y, double out[2]) {
  double S[7][7];
  glap_matrix(S);
  double sx = 0.0, sy = 0.0;
  for (int l = -3; l <= 3; ++l)
    for (int m = -3; m <= 3; ++m) {
      double v = g[wrap(y + m, ny) * nx + wrap(x + l, nx)];
      sx += glap_D(S, l, m) * v;
      sy += glap_D(S, m, l) * v;
    }
  double h3 = ds * ds * ds;
  out[0] = sx / h3;
  out[1] = sy / h3;
}

/* ------------------------------------------------------------------------- */
/* context                                                                   */
/* ------------------------------------------------------------------------- */

static size_t plane(const oolb_ctx* c) { return (size_t)c->nx * (size_t)c->ny; }

static int fail(oolb_ctx* c, int code, const char* msg) {
  if (c) snprintf(c->err, sizeof c->err, "%s", msg);
  return code;
}

void oolb_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int oolb_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int oolb_init(const oolb_params* p, oolb_ctx** out) {
  if (!p || !out) return OOLB_E_ARG;
  *out = NULL;
  if (p->nx < 1 || p->ny < 1) return OOLB_E_ARG;
  if (p->bc_x != OOLB_BC_PERIODIC && p->bc_x != OOLB_BC_SPECULAR) return OOLB_E_ARG;
  if (p->bc_x == OOLB_BC_SPECULAR && p->nx < 3) return OOLB_E_ARG;
  if (p->bc_y != OOLB_BC_PERIODIC && p->bc_y != OOLB_BC_DIFFUSE && p->bc_y != OOLB_BC_SPECULAR_DIFFUSE)
    return OOLB_E_ARG;
  if (p->bc_y != OOLB_BC_PERIODIC && p->ny < 3) return OOLB_E_ARG;
  if (!(p->ds > 0.0) || !(p->dt > 0.0) || !isfinite(p->ds) || !isfinite(p->dt))
    return OOLB_E_ARG;
  if (!(p->sigma >= 0.0) || !(p->a >= 0.0) || !(p->b >= 0.0)) return OOLB_E_ARG;
  if (!(p->tau > 0.0)) return OOLB_E_DOMAIN;
  if (p->bc_y != OOLB_BC_PERIODIC && (!(p->tw_lo > 0.0) || !(p->tw_hi > 0.0)))
    return OOLB_E_DOMAIN;
  double R[5], W[5];
  oolb_quadrature(R, W);
  /* CFL condition of Sec. 4.1: p_max dt / (m ds) < 1. */
  if (!(R[4] * p->dt / (MASS * p->ds) < 1.0)) return OOLB_E_CFL;

  oolb_ctx* c = (oolb_ctx*)calloc(1, sizeof *c);
  if (!c) return OOLB_E_WORKSPACE;
  c->p = *p;
  c->nx = p->nx;
  c->ny = p->ny;
  memcpy(c->R, R, sizeof R);
  memcpy(c->W, W, sizeof W);
  size_t np = plane(c);
  c->f = (double*)calloc(KV * np, sizeof(double));
  c->f1 = (double*)calloc(KV * np, sizeof(double));
  c->f2 = (double*)calloc(KV * np, sizeof(double));
  c->L = (double*)calloc(KV * np, sizeof(double));
  c->n = (double*)calloc(np, sizeof(double));
  c->ux = (double*)calloc(np, sizeof(double));
  c->uy = (double*)calloc(np, sizeof(double));
  c->T = (double*)calloc(np, sizeof(double));
  c->dp = (double*)calloc(np, sizeof(double));
  c->Fx = (double*)calloc(np, sizeof(double));
  c->Fy = (double*)calloc(np, sizeof(double));
  c->glo = (double*)calloc(KV * 3 * (size_t)c->nx, sizeof(double));
  c->ghi = (double*)calloc(KV * 3 * (size_t)c->nx, sizeof(double));
  c->nwlo = (double*)calloc((size_t)c->nx, sizeof(double));
  c->nwhi = (double*)calloc((size_t)c->nx, sizeof(double));
  if (!c->f || !c->f1 || !c->f2 || !c->L || !c->n || !c->ux || !c->uy || !c->T ||
      !c->dp || !c->Fx || !c->Fy || !c->glo || !c->ghi || !c->nwlo || !c->nwhi) {
    oolb_free(c);
    return OOLB_E_WORKSPACE;
  }
  *out = c;
  return OOLB_OK;
}

void oolb_free(oolb_ctx* c) {
  if (!c) return;
  free(c->f); free(c->f1); free(c->f2); free(c->L);
  free(c->n); free(c->ux); free(c->uy); free(c->T); free(c->dp);
  free(c->Fx); free(c->Fy); free(c->glo); free(c->ghi);
  free(c->nwlo); free(c->nwhi);
  free(c);
}

const char* oolb_last_error(const oolb_ctx* c) { return c ? c->err : "null context"; }

static int check_node(const oolb_ctx* c, double n, double T) {
  if (!isfinite(n) || !isfinite(T)) return OOLB_E_DOMAIN;
  if (!(n > 0.0)) return OOLB_E_DOMAIN;
  if (c->p.b > 0.0 && !(n < 1.0 / c->p.b)) return OOLB_E_DOMAIN;
  if (!(T > 0.0)) return OOLB_E_DOMAIN;
  return OOLB_OK;
}

int oolb_set_fields(oolb_ctx* c, const double* n, const double* ux,
                    const double* uy, const double* T) {
  if (!c || !n || !ux || !uy || !T) return OOLB_E_ARG;
  size_t np = plane(c);
  for (size_t i = 0; i < np; ++i) {
    if (!isfinite(ux[i]) || !isfinite(uy[i]))
      return fail(c, OOLB_E_DOMAIN, "non-finite velocity");
    if (check_node(c, n[i], T[i]) != OOLB_OK)
      return fail(c, OOLB_E_DOMAIN, "n outside (0, 1/b) or T <= 0");
  }
  for (size_t i = 0; i < np; ++i) {
    double fe[25];
    feq_node(c->R, c->W, n[i], ux[i], uy[i], T[i], fe);
    for (int k = 0; k < KV; ++k) c->f[(size_t)k * np + i] = fe[k];
  }
  c->have_f = 1;
  return OOLB_OK;
}

int oolb_set_f(oolb_ctx* c, const double* f) {
  if (!c || !f) return OOLB_E_ARG;
  memcpy(c->f, f, KV * plane(c) * sizeof(double));
  c->have_f = 1;
  return OOLB_OK;
}

int oolb_get_f(const oolb_ctx* c, double* f) {
  if (!c || !f) return OOLB_E_ARG;
  if (!c->have_f) return OOLB_E_STATE;
  memcpy(f, c->f, KV * plane(c) * sizeof(double));
  return OOLB_OK;
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.2 moments and Sec. 3.4 boundary ghosts                             */
/* ------------------------------------------------------------------------- */

/* Moments of Sec. 2.2: n = sum f, u = sum p f / (m n),
 * T = sum f |p - m u|^2 / (2 m n)  (D = 2). */
static void moments_node(const oolb_ctx* c, const double* f, size_t i, size_t np,
                         double* n, double* ux, double* uy, double* T) {
  double s0 = 0.0, sx = 0.0, sy = 0.0;
  for (int ky = 0; ky < QN; ++ky)
    for (int kx = 0; kx < QN; ++kx) {
      double v = f[(size_t)(5 * ky + kx) * np + i];
      s0 += v;
      sx += c->R[kx] * v;
      sy += c->R[ky] * v;
    }
  double u = sx / (MASS * s0), w = sy / (MASS * s0);
  double e = 0.0;
  for (int ky = 0; ky < QN; ++ky)
    for (int kx = 0; kx < QN; ++kx) {
      double v = f[(size_t)(5 * ky + kx) * np + i];
      double qx = c->R[kx] - MASS * u, qy = c->R[ky] - MASS * w;
      e += v * (qx * qx + qy * qy);
    }
  *n = s0;
  *ux = u;
  *uy = w;
  *T = e / (2.0 * MASS * s0);
}

/* Distribution value at node (x, y) of population k: in x a periodic wrap,
 * or across a specular plane (Sec. 3.4.1) the mirror node of the population
 * with the reversed x velocity, (4 - kx, ky); then in y a periodic wrap or
 * the wall ghost rows (so that a corner ghost is reflected twice). */
static double fget(const oolb_ctx* c, const double* f, int k, int x, int y) {
  int nx = c->nx, ny = c->ny;
  if (c->p.bc_x == OOLB_BC_SPECULAR && (x < 0 || x >= nx)) {
    x = x < 0 ? -1 - x : 2 * nx - 1 - x;
    k = 5 * (k / 5) + (4 - k % 5);
  } else {
    x = wrap(x, nx);
  }
  if (c->p.bc_y == OOLB_BC_PERIODIC) {
    y = wrap(y, ny);
  } else if (y < 0) {
    return c->glo[((size_t)k * 3 + (size_t)(-1 - y)) * nx + x];
  } else if (y >= ny) {
    return c->ghi[((size_t)k * 3 + (size_t)(y - ny)) * nx + x];
  }
  return f[(size_t)k * plane(c) + (size_t)y * nx + x];
}

/* Macroscopic field at (x, y): periodic wrap, or reflection across the walls
 * and specular planes (Sec. 3.4.3: n_{1-j} = n_j, Delta p_{1-j} = Delta p_j). */
static double mget(const oolb_ctx* c, const double* g, int x, int y) {
  int nx = c->nx, ny = c->ny;
  if (c->p.bc_x == OOLB_BC_SPECULAR && (x < 0 || x >= nx))
    x = x < 0 ? -1 - x : 2 * nx - 1 - x;
  else
    x = wrap(x, nx);
  if (c->p.bc_y == OOLB_BC_PERIODIC) {
    y = wrap(y, ny);
  } else if (y < 0) {
    y = -1 - y;
  } else if (y >= ny) {
    y = 2 * ny - 1 - y;
  }
  return g[(size_t)y * nx + x];
}

/* Sec. 3.4.2, transposed to walls perpendicular to y.  For each column x:
 * populations travelling towards a wall get two ghost layers by quadratic
 * extrapolation (the third layer, never read by WENO for them, is filled with
 * the same quadratic); the WENO flux of these populations through the wall
 * face fixes n_w by Eq. nw; populations leaving the wall get three ghost
 * layers equal to n_w g_{kx}(u_w, T_w) g_{ky}(0, T_w).  p_y = 0 populations
 * carry no y-flux; their ghosts are extrapolated so that they stay finite. */
static void fill_wall_ghosts(oolb_ctx* c, const double* f) {
  const int nx = c->nx, ny = c->ny;
  const size_t np = plane(c);
  const int specular_lo = c->p.bc_y == OOLB_BC_SPECULAR_DIFFUSE;
#pragma omp parallel for schedule(static)
  for (int x = 0; x < nx; ++x) {
    for (int wall = 0; wall < 2; ++wall) {
      if (wall == 0 && specular_lo) {
        /* Sec. 3.4.1: the ghost row -1 - j of population (kx, ky) holds
         * row j of the population with the reversed y velocity, (kx, 4 - ky) */
        for (int k = 0; k < KV; ++k) {
          int kx = k % 5, ky = k / 5;
          int km = 5 * (4 - ky) + kx;
          for (int j = 0; j < 3; ++j)
            c->glo[((size_t)k * 3 + j) * nx + x] = f[(size_t)km * np + (size_t)j * nx + x];
        }
        c->nwlo[x] = 0.0;
        continue;
      }
      /* wall = 0: lower wall at y = -1/2 (towards-wall: p_y < 0);
       * wall = 1: upper wall at y = ny - 1/2 (towards-wall: p_y > 0). */
      const double Tw = wall ? c->p.tw_hi : c->p.tw_lo;
      const double uw = wall ? c->p.uw_hi : c->p.uw_lo;
      double* G = wall ? c->ghi : c->glo;
      /* interior rows nearest the wall, y0 (adjacent), y1, y2 */
      int y0 = wall ? ny - 1 : 0, y1 = wall ? ny - 2 : 1, y2 = wall ? ny - 3 : 2;
      for (int k = 0; k < KV; ++k) {
        int ky = k / 5;
        double py = c->R[ky];
        int towards = wall ? (py >= 0.0) : (py <= 0.0);
        if (!towards) continue;
        double a0 = f[(size_t)k * np + (size_t)y0 * nx + x];
        double a1 = f[(size_t)k * np + (size_t)y1 * nx + x];
        double a2 = f[(size_t)k * np + (size_t)y2 * nx + x];
        G[((size_t)k * 3 + 0) * nx + x] = 3.0 * a0 - 3.0 * a1 + a2;
        G[((size_t)k * 3 + 1) * nx + x] = 6.0 * a0 - 8.0 * a1 + 3.0 * a2;
        G[((size_t)k * 3 + 2) * nx + x] = 10.0 * a0 - 15.0 * a1 + 6.0 * a2;
      }
      /* outgoing flux through the wall face (Eq. nw numerator) */
      double out = 0.0;
      for (int k = 0; k < KV; ++k) {
        int ky = k / 5;
        double py = c->R[ky];
        if (wall == 0 && py < 0.0) {
          /* face between y = -1 and y = 0 */
          out += face_flux(py, fget(c, f, k, x, -3), fget(c, f, k, x, -2),
                           fget(c, f, k, x, -1), fget(c, f, k, x, 0),
                           fget(c, f, k, x, 1), fget(c, f, k, x, 2));
        } else if (wall == 1 && py > 0.0) {
          /* face between y = ny-1 and y = ny */
          out += face_flux(py, fget(c, f, k, x, ny - 3), fget(c, f, k, x, ny - 2),
                           fget(c, f, k, x, ny - 1), fget(c, f, k, x, ny),
                           fget(c, f, k, x, ny + 1), fget(c, f, k, x, ny + 2));
        }
      }
      /* Eq. nw denominator: sum over wall-emitted velocities of
       * g_{kx}(u_w, T_w) g_{ky}(0, T_w) p_{ky} / m */
      double den = 0.0;
      for (int ky = 0; ky < QN; ++ky) {
        double py = c->R[ky];
        int emitted = wall ? (py < 0.0) : (py > 0.0);
        if (!emitted) continue;
        for (int kx = 0; kx < QN; ++kx)
          den += g_axis(c->R, c->W, kx, uw, Tw) * g_axis(c->R, c->W, ky, 0.0, Tw) * py / MASS;
      }
      double nw = -out / den;
      if (wall) c->nwhi[x] = nw; else c->nwlo[x] = nw;
      for (int ky = 0; ky < QN; ++ky) {
        double py = c->R[ky];
        int emitted = wall ? (py < 0.0) : (py > 0.0);
        if (!emitted) continue;
        for (int kx = 0; kx < QN; ++kx) {
          int k = 5 * ky + kx;
          double v = nw * g_axis(c->R, c->W, kx, uw, Tw) * g_axis(c->R, c->W, ky, 0.0, Tw);
          for (int layer = 0; layer < 3; ++layer) G[((size_t)k * 3 + layer) * nx + x] = v;
        }
      }
    }
  }
}

int oolb_wall_ghosts(const oolb_ctx* c, double* glo, double* ghi) {
  if (!c || !glo || !ghi) return OOLB_E_ARG;
  if (c->p.bc_y == OOLB_BC_PERIODIC) return OOLB_E_STATE;
  memcpy(glo, c->glo, KV * 3 * (size_t)c->nx * sizeof(double));
  memcpy(ghi, c->ghi, KV * 3 * (size_t)c->nx * sizeof(double));
  return OOLB_OK;
}

int oolb_wall_density(const oolb_ctx* c, double* nw_lo, double* nw_hi) {
  if (!c || !nw_lo || !nw_hi) return OOLB_E_ARG;
  if (c->p.bc_y == OOLB_BC_PERIODIC) return OOLB_E_STATE;
  memcpy(nw_lo, c->nwlo, (size_t)c->nx * sizeof(double));
  memcpy(nw_hi, c->nwhi, (size_t)c->nx * sizeof(double));
  return OOLB_OK;
}

/* ------------------------------------------------------------------------- */
/* Eq. ecast: L[f] = -(p/m).grad f - F.(grad_p f) - (f - f^eq)/tau           */
/* ------------------------------------------------------------------------- */

static void rhs(oolb_ctx* c, const double* f, double* L) {
  const int nx = c->nx, ny = c->ny;
  const size_t np = plane(c);
  const oolb_params* P = &c->p;

  /* 1. ghosts of the current f (walls) */
  if (P->bc_y != OOLB_BC_PERIODIC) fill_wall_ghosts(c, f);

  /* 2. moments and Delta p = p^i - p^w at every node */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t i = (size_t)y * nx + x;
      double n, u, w, T;
      moments_node(c, f, i, np, &n, &u, &w, &T);
      c->n[i] = n; c->ux[i] = u; c->uy[i] = w; c->T[i] = T;
      c->dp[i] = n * T - oolb_pw(n, T, P->a, P->b);
    }

  /* 3. force of Eq. F_def with the 49-point stencils */
  double S[7][7];
  glap_matrix(S);
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      double gx = 0.0, gy = 0.0, lx = 0.0, ly = 0.0;
      for (int l = -3; l <= 3; ++l)
        for (int m = -3; m <= 3; ++m) {
          double w = grad_w(abs(l), abs(m));
          double dpv = mget(c, c->dp, x + l, y + m);
          double nv = mget(c, c->n, x + l, y + m);
          gx += (double)l * w * dpv;
          gy += (double)m * w * dpv;
          lx += glap_D(S, l, m) * nv;
          ly += glap_D(S, m, l) * nv;
        }
      size_t i = (size_t)y * nx + x;
      double h = P->ds, h3 = h * h * h;
      c->Fx[i] = (gx / h) / c->n[i] + P->sigma * (lx / h3);
      c->Fy[i] = (gy / h) / c->n[i] + P->sigma * (ly / h3);
    }

  /* 4. per node and population: advection, force term, BGK */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t i = (size_t)y * nx + x;
      double fl[25], dfx[25], dfy[25], fe[25];
      for (int k = 0; k < KV; ++k) fl[k] = f[(size_t)k * np + i];
      dpf_node(c->R, c->W, fl, dfx, dfy);
      feq_node(c->R, c->W, c->n[i], c->ux[i], c->uy[i], c->T[i], fe);
      for (int k = 0; k < KV; ++k) {
        double px = c->R[k % 5], py = c->R[k / 5];
        /* x faces i+1/2 and i-1/2 */
        double fxp = face_flux(px, fget(c, f, k, x - 2, y), fget(c, f, k, x - 1, y),
                               fget(c, f, k, x, y), fget(c, f, k, x + 1, y),
                               fget(c, f, k, x + 2, y), fget(c, f, k, x + 3, y));
        double fxm = face_flux(px, fget(c, f, k, x - 3, y), fget(c, f, k, x - 2, y),
                               fget(c, f, k, x - 1, y), fget(c, f, k, x, y),
                               fget(c, f, k, x + 1, y), fget(c, f, k, x + 2, y));
        double fyp = face_flux(py, fget(c, f, k, x, y - 2), fget(c, f, k, x, y - 1),
                               fget(c, f, k, x, y), fget(c, f, k, x, y + 1),
                               fget(c, f, k, x, y + 2), fget(c, f, k, x, y + 3));
        double fym = face_flux(py, fget(c, f, k, x, y - 3), fget(c, f, k, x, y - 2),
                               fget(c, f, k, x, y - 1), fget(c, f, k, x, y),
                               fget(c, f, k, x, y + 1), fget(c, f, k, x, y + 2));
        double adv = (fxp - fxm) / P->ds + (fyp - fym) / P->ds;
        double force = c->Fx[i] * dfx[k] + c->Fy[i] * dfy[k];
        double coll = -(fl[k] - fe[k]) / P->tau;
        L[(size_t)k * np + i] = -adv - force + coll;
      }
    }
}

int oolb_rhs(oolb_ctx* c, const double* f, double* L) {
  if (!c || !f || !L) return OOLB_E_ARG;
  rhs(c, f, L);
  return OOLB_OK;
}

/* Eq. rk3, third-order TVD Runge-Kutta. */
int oolb_step(oolb_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return OOLB_E_ARG;
  if (!c->have_f) return fail(c, OOLB_E_STATE, "step before set_fields/set_f");
  const size_t nt = KV * plane(c);
  const double dt = c->p.dt;
  for (int s = 0; s < nsteps; ++s) {
    rhs(c, c->f, c->L);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < nt; ++i) c->f1[i] = c->f[i] + dt * c->L[i];
    rhs(c, c->f1, c->L);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < nt; ++i)
      c->f2[i] = 0.75 * c->f[i] + 0.25 * c->f1[i] + 0.25 * dt * c->L[i];
    rhs(c, c->f2, c->L);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < nt; ++i)
      c->f[i] = (1.0 / 3.0) * c->f[i] + (2.0 / 3.0) * c->f2[i] + (2.0 / 3.0) * dt * c->L[i];
  }
  for (size_t i = 0; i < nt; ++i)
    if (!isfinite(c->f[i])) return fail(c, OOLB_E_NONFINITE, "non-finite distribution");
  return OOLB_OK;
}

int oolb_moments(const oolb_ctx* c, double* n, double* ux, double* uy, double* T) {
  if (!c || !n || !ux || !uy || !T) return OOLB_E_ARG;
  if (!c->have_f) return OOLB_E_STATE;
  size_t np = plane(c);
  for (size_t i = 0; i < np; ++i) moments_node(c, c->f, i, np, &n[i], &ux[i], &uy[i], &T[i]);
  return OOLB_OK;
}
