// Host FP64 eigensolver for the 1D generalized problems K W = M W Lambda of
// Sec. 2 (one per block axis and per global axis).
#pragma once

#include <complex>
#include <string>
#include <vector>

namespace hs {

using cd = std::complex<double>;

struct AxisEig {
  int n = 0;
  std::vector<cd> lam;    // n eigenvalues of D = M^{-1} K
  std::vector<cd> W;      // n x n row-major, W[i*n + m] = component i of eigenvector m
  std::vector<cd> Winv;   // n x n row-major explicit inverse
  double kappa = 1.0;     // ||W||_1 ||W^{-1}||_1
  double eig_resid = 0;   // ||D W - W Lambda||_F / (||D||_F ||W||_F)
  double inv_resid = 0;   // max |W^{-1} W - I|
  double decouple = 0;    // max off-diagonal |W^{-1} D W| / ||D||_F
};

// D = M^{-1} K of an axis with n interior nodes and steps h[0..n].
std::vector<cd> axis_operator(int n, const cd* h);

// True if all n+1 steps are equal (the closed-form sine case).
bool axis_is_uniform(int n, const cd* h);

// Closed-form Dirichlet eigenpairs of a uniform axis: lam_m = 2(1 - cos(pi (m+1)/(n+1))) / h^2,
// W = W^{-1} = sqrt(2/(n+1)) sin(pi (i+1)(m+1)/(n+1)).
void axis_eig_uniform(int n, cd h, AxisEig& out);

// General case: complex Hessenberg QR with Wilkinson shifts to the Schur form,
// eigenvectors by back-substitution on the triangular factor, explicit LU inverse.
// Returns false (with a message) if the iteration fails or W is singular.
bool axis_eig_general(int n, const cd* h, AxisEig& out, std::string& err);

}  // namespace hs
