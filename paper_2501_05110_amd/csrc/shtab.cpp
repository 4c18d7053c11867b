// Closed-form spherical-harmonic matrices of Sec. 2.1 (host side).
//
//  * A^x:      eq. representation-matrix-Ax
//  * Omega^x:  eq. representation-matrix-Omegax
//  * exp(pi/2 Omega^z): eq. representation-matrix-Uz with u(l',m',l,m) of
//    eq. complex-rotation (sum over every k with non-negative factorial
//    arguments)
//  * exp(pi/2 Omega^x): the transpose of eq. representation-matrix-Ux as
//    printed (the printed matrix equals exp(-pi/2 Omega^x) for the Omega^x of
//    eq. representation-matrix-Omegax; with the transpose the chain below
//    reproduces the direction operator p_z/p and the Omega^z entries of
//    eq. convergence-study-explicit-equations)
//  * A^y = e^{-pi/2 Om^z} A^x e^{pi/2 Om^z}, A^z = e^{-pi/2 Om^x} A^y e^{pi/2 Om^x},
//    and the same for Omega (eq. real-direction-op-matrices-and-rotations);
//    the rotation matrices are orthogonal, so e^{-pi/2 Om} = (e^{pi/2 Om})^T.
//  * products at L = l_max + 1 truncated to n x n (rule stated after
//    eq. real-C-matrix).
#include "shtab.hpp"

#include <cmath>
#include <stdexcept>

namespace vfp {

Mat matmul(const Mat& A, const Mat& B) {
  Mat C(A.n);
  for (int i = 0; i < A.n; ++i)
    for (int k = 0; k < A.n; ++k) {
      double aik = A(i, k);
      if (aik == 0.0) continue;
      for (int j = 0; j < A.n; ++j) C(i, j) += aik * B(k, j);
    }
  return C;
}

Mat transpose(const Mat& A) {
  Mat T(A.n);
  for (int i = 0; i < A.n; ++i)
    for (int j = 0; j < A.n; ++j) T(j, i) = A(i, j);
  return T;
}

Mat truncate(const Mat& A, int n) {
  Mat T(n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) T(i, j) = A(i, j);
  return T;
}

void jacobi_eigh(const Mat& A0, std::vector<double>& lam, Mat& V) {
  const int n = A0.n;
  Mat A = A0;
  V = Mat(n);
  for (int i = 0; i < n; ++i) V(i, i) = 1.0;
  // Rotations keep the Frobenius norm; an off-diagonal entry below 1e-18 of
  // it is set to zero (it moves no eigenvalue by more than that), and the
  // iteration ends with the first sweep that rotates nothing.  (A relative
  // test on the off-diagonal sum alone can stall at rounding level.)
  double tot = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) tot += A(i, j) * A(i, j);
  const double small = 1e-18 * std::sqrt(tot);
  for (int sweep = 0; sweep < 100; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A(p, q);
        if (std::fabs(apq) <= small) {
          A(p, q) = A(q, p) = 0.0;
          continue;
        }
        rotated = true;
        double app = A(p, p), aqq = A(q, q);
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- J^T A J, columns p, q
          double akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - s * akq;
          A(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - s * aqk;
          A(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V(k, p), vkq = V(k, q);
          V(k, p) = c * vkp - s * vkq;
          V(k, q) = s * vkp + c * vkq;
        }
      }
    if (!rotated) break;
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = A(i, i);
}

namespace {

double fact(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

Mat ax_closed(int L) {
  const int n = (L + 1) * (L + 1);
  Mat M(n);
  for (int l = 0; l <= L; ++l)
    for (int m = 0; m <= l; ++m)
      for (int s = 0; s <= (m ? 1 : 0); ++s) {
        int j = lms_index(l, m, s);
        if (l + 1 <= L)
          M(lms_index(l + 1, m, s), j) =
              std::sqrt(double((l + m + 1) * (l - m + 1)) / double((2 * l + 3) * (2 * l + 1)));
        if (l - 1 >= m)
          M(lms_index(l - 1, m, s), j) =
              std::sqrt(double((l + m) * (l - m)) / double((2 * l + 1) * (2 * l - 1)));
      }
  return M;
}

Mat omx_closed(int L) {
  const int n = (L + 1) * (L + 1);
  Mat M(n);
  for (int l = 0; l <= L; ++l)
    for (int m = 1; m <= l; ++m) {  // m = 0 rows and columns vanish
      // (Omega^x)_{(l m 0),(l m 1)} = m, (Omega^x)_{(l m 1),(l m 0)} = -m
      M(lms_index(l, m, 0), lms_index(l, m, 1)) = m;
      M(lms_index(l, m, 1), lms_index(l, m, 0)) = -m;
    }
  return M;
}

double u_coef(int lp, int mp, int l, int m) {
  if (lp != l) return 0.0;
  double tot = 0.0;
  for (int k = 0; k <= 2 * l; ++k) {
    int a0 = l - mp - k, a1 = l - m - k, a2 = mp + m + k;
    if (a0 < 0 || a1 < 0 || a2 < 0) continue;
    double num = std::sqrt(fact(l + mp) * fact(l - mp) * fact(l + m) * fact(l - m));
    tot += ((k & 1) ? -1.0 : 1.0) * num / (fact(k) * fact(a0) * fact(a1) * fact(a2));
  }
  return (((l - mp) & 1) ? -1.0 : 1.0) / std::pow(2.0, l) * tot;
}

Mat rz_closed(int L) {
  const int n = (L + 1) * (L + 1);
  Mat M(n);
  for (int l = 0; l <= L; ++l)
    for (int mp = 0; mp <= l; ++mp)
      for (int m = 0; m <= l; ++m) {
        double pm = (m & 1) ? -1.0 : 1.0;
        double up = u_coef(l, mp, l, m), um = u_coef(l, mp, l, -m);
        M(lms_index(l, mp, 0), lms_index(l, m, 0)) =
            (up + pm * um) / std::sqrt((1.0 + (mp == 0)) * (1.0 + (m == 0)));
        if (mp > 0 && m > 0) M(lms_index(l, mp, 1), lms_index(l, m, 1)) = up - pm * um;
      }
  return M;
}

Mat rx_printed(int L) {
  const int n = (L + 1) * (L + 1);
  Mat M(n);
  const double hp = 0.5 * M_PI;
  for (int l = 0; l <= L; ++l)
    for (int m = 0; m <= l; ++m) {
      double c = std::cos(hp * m), s = std::sin(hp * m);
      double d0 = (m == 0) ? 1.0 : 0.0;
      M(lms_index(l, m, 0), lms_index(l, m, 0)) = (c + d0) / (1.0 + d0);
      if (m > 0) {
        M(lms_index(l, m, 1), lms_index(l, m, 0)) = s;
        M(lms_index(l, m, 0), lms_index(l, m, 1)) = -s;
        M(lms_index(l, m, 1), lms_index(l, m, 1)) = c;
      }
    }
  return M;
}

void clean(Mat& M) {
  for (double& v : M.a)
    if (std::fabs(v) < 1e-14) v = 0.0;
}

}  // namespace

ShMatrices build_sh_matrices(int lmax) {
  if (lmax < 0 || lmax > kShAxisOnlyMaxLmax) throw std::invalid_argument("lmax");
  const int L = lmax + 1;
  const int n = (lmax + 1) * (lmax + 1);
  Mat Ax = ax_closed(L), Omx = omx_closed(L);
  if (lmax > kShFullMaxLmax) {
    // Above l_max = 7 only the x-axis matrices are built: the alternating
    // factorial sums of eq. complex-rotation lose more digits than a 1e-12
    // operator allows from l = 9 on.  A^x, Omega^x and (A^x A^x)_t carry
    // runs along x with B along x (the closure example of Sec. 4.3); the
    // other matrices stay zero and the library refuses runs that need them.
    ShMatrices S;
    S.lmax = lmax;
    S.n = n;
    S.A[0] = truncate(Ax, n);
    S.A[1] = Mat(n);
    S.A[2] = Mat(n);
    S.Om[0] = truncate(Omx, n);
    S.Om[1] = Mat(n);
    S.Om[2] = Mat(n);
    S.AXX = truncate(matmul(Ax, Ax), n);
    S.G1 = Mat(n);
    S.G2 = Mat(n);
    clean(S.AXX);
    S.C.resize(n);
    for (int l = 0; l <= lmax; ++l)
      for (int j = l * l; j < (l + 1) * (l + 1); ++j) S.C[j] = 0.5 * l * (l + 1);
    return S;
  }
  Mat Rz = rz_closed(L);
  Mat Rx = transpose(rx_printed(L));   // exp(+pi/2 Omega^x)
  Mat RzT = transpose(Rz), RxT = transpose(Rx);
  Mat Ay = matmul(matmul(RzT, Ax), Rz);
  Mat Az = matmul(matmul(RxT, Ay), Rx);
  Mat Omy = matmul(matmul(RzT, Omx), Rz);
  Mat Omz = matmul(matmul(RxT, Omy), Rx);
  for (Mat* M : {&Ay, &Az, &Omy, &Omz}) clean(*M);
  Mat AyOmz = matmul(Ay, Omz), AzOmy = matmul(Az, Omy);
  Mat G1L(AyOmz.n);
  for (size_t i = 0; i < G1L.a.size(); ++i) G1L.a[i] = AyOmz.a[i] - AzOmy.a[i];
  Mat G2L = matmul(Ax, G1L);
  Mat AXXL = matmul(Ax, Ax);
  ShMatrices S;
  S.lmax = lmax;
  S.n = n;
  S.A[0] = truncate(Ax, n);
  S.A[1] = truncate(Ay, n);
  S.A[2] = truncate(Az, n);
  S.Om[0] = truncate(Omx, n);
  S.Om[1] = truncate(Omy, n);
  S.Om[2] = truncate(Omz, n);
  S.AXX = truncate(AXXL, n);
  S.G1 = truncate(G1L, n);
  S.G2 = truncate(G2L, n);
  for (Mat* M : {&S.AXX, &S.G1, &S.G2}) clean(*M);
  S.C.resize(n);
  for (int l = 0; l <= lmax; ++l)
    for (int j = l * l; j < (l + 1) * (l + 1); ++j) S.C[j] = 0.5 * l * (l + 1);
  return S;
}

// Real spherical harmonics of App. A: Y_lms = N_lm P_l^m(cos theta)
// (cos m phi | sin m phi), eq. spherical-harmonics with the normalisation of
// eq. normalisation-spherical-harmonics and the Condon-Shortley phase inside
// P_l^m (eq. associated-legendre-polynomials).  P_l^m by the standard
// recurrences in l at fixed m, started from P_m^m = (-1)^m (2m-1)!! sin^m theta.
void real_sh_dir(int lmax, double theta, double phi, double* Y) {
  const double x = std::cos(theta), st = std::sin(theta);
  const int n = (lmax + 1) * (lmax + 1);
  for (int j = 0; j < n; ++j) Y[j] = 0.0;
  double pmm = 1.0;                                   // P_m^m
  for (int m = 0; m <= lmax; ++m) {
    if (m > 0) pmm *= -(2.0 * m - 1.0) * st;
    double plm2 = 0.0, plm1 = pmm;                    // P_{l-2}^m, P_{l-1}^m
    for (int l = m; l <= lmax; ++l) {
      double p;
      if (l == m) {
        p = pmm;
      } else if (l == m + 1) {
        p = x * (2.0 * m + 1.0) * pmm;
      } else {
        p = ((2.0 * l - 1.0) * x * plm1 - (l + m - 1.0) * plm2) / (l - m);
      }
      if (l > m) {
        plm2 = plm1;
        plm1 = p;
      }
      // N_lm^2 = (2l+1)/(2 pi (1 + delta_m0)) (l-m)!/(l+m)!
      double ratio = 1.0;
      for (int q = l - m + 1; q <= l + m; ++q) ratio /= q;
      const double nlm = std::sqrt((2.0 * l + 1.0) / (2.0 * M_PI * (m == 0 ? 2.0 : 1.0)) * ratio);
      Y[lms_index(l, m, 0)] = nlm * p * std::cos(m * phi);
      if (m > 0) Y[lms_index(l, m, 1)] = nlm * p * std::sin(m * phi);
    }
  }
}

}  // namespace vfp
