// Compile-time 1-D basis tables for DG degree K on the reference interval
// [-1, 1]: Lagrange basis l_j on the Gauss-Lobatto nodes, (K+1)-point Gauss
// rule, M1 = the exact 1-D mass matrix.
//   phi[q][j]  = l_j(g_q)
//   tst[i][q]  = w_q (M1^{-1} l)_i (g_q)      test contraction with M^{-1} folded in
//   dtst[i][q] = w_q (M1^{-1} l')_i (g_q)
//   lift[s][i] = (M1^{-1})_{i, 0 or K}         face lift at the lo / hi end
//   dphi[q][j] = l_j'(g_q)                      derivative interpolation
//   mass[i][j] = (M1)_ij                        exact 1-D mass matrix
// For K = 2 (nodes -1, 0, 1; points -s, 0, s with s = sqrt(3/5); weights 5/9,
// 8/9, 5/9) the dual basis M1^{-1} l is L_0 = 1.5 - 1.5x ... written out
// below in closed form, so that its exact zeros let the compiler drop terms.
#pragma once

namespace vfp {

template <int K>
struct CBasis;

template <>
struct CBasis<1> {
  static constexpr double t = 0.5773502691896258;   // 1/sqrt(3)
  static constexpr double phi[2][2] = {{0.5 * (1 + t), 0.5 * (1 - t)}, {0.5 * (1 - t), 0.5 * (1 + t)}};
  static constexpr double tst[2][2] = {{0.5 + 1.5 * t, 0.5 - 1.5 * t}, {0.5 - 1.5 * t, 0.5 + 1.5 * t}};
  static constexpr double dtst[2][2] = {{-1.5, -1.5}, {1.5, 1.5}};
  static constexpr double lift[2][2] = {{2.0, -1.0}, {-1.0, 2.0}};
  static constexpr double dphi[2][2] = {{-0.5, 0.5}, {-0.5, 0.5}};
  static constexpr double mass[2][2] = {{2.0 / 3.0, 1.0 / 3.0}, {1.0 / 3.0, 2.0 / 3.0}};
};

template <>
struct CBasis<2> {
  static constexpr double s = 0.7745966692414834;   // sqrt(3/5)
  static constexpr double phi[3][3] = {
      {0.3 + 0.5 * s, 0.4, 0.3 - 0.5 * s}, {0.0, 1.0, 0.0}, {0.3 - 0.5 * s, 0.4, 0.3 + 0.5 * s}};
  static constexpr double tst[3][3] = {{5.0 / 6.0 * (1 + s), -2.0 / 3.0, 5.0 / 6.0 * (1 - s)},
                                       {0.0, 1.0, 0.0},
                                       {5.0 / 6.0 * (1 - s), -2.0 / 3.0, 5.0 / 6.0 * (1 + s)}};
  static constexpr double dtst[3][3] = {
      {-25.0 / 6.0 * s - 5.0 / 6.0, -4.0 / 3.0, 25.0 / 6.0 * s - 5.0 / 6.0},
      {25.0 / 12.0 * s, 0.0, -25.0 / 12.0 * s},
      {-25.0 / 6.0 * s + 5.0 / 6.0, 4.0 / 3.0, 25.0 / 6.0 * s + 5.0 / 6.0}};
  static constexpr double lift[2][3] = {{4.5, -0.75, 1.5}, {1.5, -0.75, 4.5}};
  // l_0 = x(x-1)/2, l_1 = 1-x^2, l_2 = x(x+1)/2: derivatives x-1/2, -2x, x+1/2
  static constexpr double dphi[3][3] = {
      {-s - 0.5, 2.0 * s, -s + 0.5}, {-0.5, 0.0, 0.5}, {s - 0.5, -2.0 * s, s + 0.5}};
  static constexpr double mass[3][3] = {{4.0 / 15.0, 2.0 / 15.0, -1.0 / 15.0},
                                        {2.0 / 15.0, 16.0 / 15.0, 2.0 / 15.0},
                                        {-1.0 / 15.0, 2.0 / 15.0, 4.0 / 15.0}};
};

}  // namespace vfp
