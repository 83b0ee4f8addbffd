// Host-side reference-element construction (FP64), written independently of
// any other implementation.  Follows Sec. 3.1.4 of the paper: orthonormal
// Jacobi bases, generalised Vandermonde V, D_r = V_r V^{-1}, the
// quadrature-free mass matrix M = (V V^T)^{-1}; Sec. 3.3 fine-grid
// interpolation and mass; Sec. 3.4 modal filter on the boundary/bubble basis.
#pragma once
#include <vector>

namespace sem {

using Mat = std::vector<double>;   // dense row-major

// Orthonormal Jacobi polynomial ~P_n^(a,b)(x) and its derivative.
double jacobi_orthonormal(double x, int n, double a, double b);
double jacobi_orthonormal_deriv(double x, int n, double a, double b);
// Classical (unnormalised) Jacobi polynomial, used by the filter's bubble modes.
double jacobi_classical(double x, int n, double a, double b);

std::vector<double> gll_points(int P);          // P+1 GLL nodes on [-1, 1]
void warp_blend(int P, std::vector<double>& r, std::vector<double>& s);

// dense helpers (n x n, row-major)
Mat matmul(const Mat& A, const Mat& B, int n, int k, int m);   // (n x k)(k x m)
Mat transpose(const Mat& A, int n, int m);
bool invert(Mat& A, int n);                                      // in place, false if singular

struct Ref1D {
  int P = 0;
  std::vector<double> r;
  Mat V, Vinv, D, M;   // (P+1)^2 each
  explicit Ref1D(int P);
  Mat interp_to(const std::vector<double>& rout) const;          // rout.size() x (P+1)
};

struct RefTri {
  int P = 0, Np = 0;
  std::vector<double> r, s;
  Mat V, Vinv, Dr, Ds, M;  // Np x Np
  explicit RefTri(int P);
};

// F = V^ diag(sigma) V^{-1} on the GLL(P) nodes with the modified basis
// phi_0 = (1-r)/2, phi_1 = (1+r)/2, phi_{n+1} = (1-r)(1+r)/4 P_{n-1}^(1,1).
Mat filter_matrix(int P, int ic, double sigma_f);

}  // namespace sem
