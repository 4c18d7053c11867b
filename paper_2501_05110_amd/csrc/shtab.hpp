// Spherical-harmonic system matrices from the paper's closed forms (host).
#pragma once
#include <vector>

namespace vfp {

// Dense row-major square matrix.
struct Mat {
  int n = 0;
  std::vector<double> a;
  Mat() = default;
  explicit Mat(int n_) : n(n_), a(size_t(n_) * n_, 0.0) {}
  double& operator()(int i, int j) { return a[size_t(i) * n + j]; }
  double operator()(int i, int j) const { return a[size_t(i) * n + j]; }
};

Mat matmul(const Mat& A, const Mat& B);
Mat transpose(const Mat& A);
Mat truncate(const Mat& A, int n);

inline int lms_index(int l, int m, int s) { return l * (l + 1) + (s == 1 ? m : -m); }

// Symmetric eigen-decomposition by cyclic Jacobi rotations.
// On return A = V diag(lam) V^T (columns of V are eigenvectors).
void jacobi_eigh(const Mat& A, std::vector<double>& lam, Mat& V);

struct ShMatrices {
  int lmax = 0, n = 0;
  Mat A[3];      // A^x, A^y, A^z
  Mat Om[3];     // Omega^x, Omega^y, Omega^z
  Mat AXX;       // (A^x A^x)_t
  Mat G1;        // (A^y Omega^z - A^z Omega^y)_t
  Mat G2;        // (A^x (A^y Omega^z - A^z Omega^y))_t
  std::vector<double> C;  // l(l+1)/2
};

// l_max up to which every matrix is built, and up to which the x-axis
// matrices alone are (A^x, Omega^x, (A^x A^x)_t; the others zero).
constexpr int kShFullMaxLmax = 7;
constexpr int kShAxisOnlyMaxLmax = 11;

// Builds every matrix for l_max from the closed forms: A^x and Omega^x
// directly, A^{y,z} and Omega^{y,z} through the pi/2 rotation matrices, the
// products at l_max+1 then truncated (above kShFullMaxLmax: the x-axis
// matrices only).
ShMatrices build_sh_matrices(int lmax);

// Y[lms] = Y_lms(theta, phi) for lms < (lmax+1)^2 (App. A; theta from the x
// axis, phi about it).
void real_sh_dir(int lmax, double theta, double phi, double* Y);

}  // namespace vfp
