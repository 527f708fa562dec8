// olb_consts.hpp -- compile-time constants of the D2Q25 Gauss-Hermite model.
//
// Everything is evaluated by the compiler from closed forms, so the kernels see
// immediate operands:
//   roots and weights          Table trots (Sec. 2.2)
//   He_l(R_k)                  probabilists' Hermite polynomials
//   force matrix M             Eq. derf folded into a 5x5 matrix
//   stencil weights            Eqs. stencil_grad / stencil_glap (Sec. 3.3),
//                              gradient of the Laplacian with c1 = -17/2160 and
//                              c4 = -59/540 (the printed c1, c4 violate the
//                              1-D reduction of Sec. 4), oriented to reproduce
//                              that reduction
//   WENO ideal weights         Eq. weno5_delta
#pragma once

namespace olbc {

constexpr double csqrt_newton(double v, double x, int it) {
  return it == 0 ? x : csqrt_newton(v, 0.5 * (x + v / x), it - 1);
}
constexpr double csqrt(double v) { return v <= 0.0 ? 0.0 : csqrt_newton(v, v > 1.0 ? v : 1.0, 80); }

constexpr double S10 = csqrt(10.0);
// Table trots, ascending.
constexpr double R0 = -csqrt(5.0 + S10);
constexpr double R1 = -csqrt(5.0 - S10);
constexpr double R3 = csqrt(5.0 - S10);
constexpr double R4 = csqrt(5.0 + S10);
constexpr double Rk[5] = {R0, R1, 0.0, R3, R4};
constexpr double Wk[5] = {(7.0 - 2.0 * S10) / 60.0, (7.0 + 2.0 * S10) / 60.0, 8.0 / 15.0,
                          (7.0 + 2.0 * S10) / 60.0, (7.0 - 2.0 * S10) / 60.0};

constexpr double he(int l, double p) {
  return l == 0 ? 1.0 : (l == 1 ? p : p * he(l - 1, p) - (l - 1) * he(l - 2, p));
}
constexpr double fact(int l) { return l <= 1 ? 1.0 : l * fact(l - 1); }

// (d_p f)_k = sum_j M[k][j] f_j  with
// M[k][j] = -W_k sum_{l=0}^{N-1} He_{l+1}(R_k) He_l(R_j) / l!,  N = 4.
constexpr double Mkj(int k, int j) {
  return -Wk[k] * (he(1, Rk[k]) * he(0, Rk[j]) / fact(0) + he(2, Rk[k]) * he(1, Rk[j]) / fact(1) +
                   he(3, Rk[k]) * he(2, Rk[j]) / fact(2) + he(4, Rk[k]) * he(3, Rk[j]) / fact(3));
}

struct Tab55 {
  double v[5][5];
};
struct TabHe {
  double v[6][5];
};
constexpr Tab55 make_M() {
  Tab55 t{};
  for (int k = 0; k < 5; ++k)
    for (int j = 0; j < 5; ++j) t.v[k][j] = Mkj(k, j);
  return t;
}
constexpr TabHe make_He() {
  TabHe t{};
  for (int l = 0; l < 6; ++l)
    for (int k = 0; k < 5; ++k) t.v[l][k] = he(l, Rk[k]);
  return t;
}
constexpr Tab55 MT = make_M();   // MT.v[k][j] = M[k][j]
constexpr TabHe HE = make_He();  // HE.v[l][k] = He_l(R_k)

// 49-point gradient weights w^{|l|,|m|}.
constexpr double GW[4][4] = {{0.0, 31.0 / 70.0, 0.0, -1.0 / 630.0},
                             {31.0 / 70.0, 27.0 / 140.0, -3.0 / 70.0, 1.0 / 280.0},
                             {0.0, -3.0 / 70.0, 3.0 / 560.0, 0.0},
                             {-1.0 / 630.0, 1.0 / 280.0, 0.0, 0.0}};
// Coefficient of n_{x+l, y+m} in ds^3 d_x lap n for l = 1..3 (odd in l, even
// in m): GL[l-1][|m|].
constexpr double GL[3][4] = {{-59.0 / 20.0, 187.0 / 240.0, -7.0 / 60.0, 0.0},
                             {5.0 / 4.0, -7.0 / 30.0, 13.0 / 120.0, 0.0},
                             {-59.0 / 540.0, 0.0, 0.0, -17.0 / 2160.0}};

// WENO-5 ideal weights.
constexpr double D1 = 0.1, D2 = 0.6, D3 = 0.3;

// RK-3 (Eq. rk3) in the form f_dst = A_s f^n + B_s (f_src + dt L[f_src]).
constexpr double RK_A[3] = {0.0, 0.75, 1.0 / 3.0};
constexpr double RK_B[3] = {1.0, 0.25, 2.0 / 3.0};

}  // namespace olbc
