// Host FP64 eigensolver for the generalized 1D problems K W = M W Lambda of
// Sec. 2 (A_d W_d = M_d W_d Lambda_d with W_d = 0 on the block walls).
//
// D = M^{-1} K is a complex tridiagonal (hence upper Hessenberg) matrix.  It
// is reduced to Schur form T = Z^H D Z by the implicitly shifted complex QR
// iteration (Wilkinson shift, exceptional shifts on stagnation, deflation on
// negligible subdiagonals).  Eigenvectors of T come from back-substitution and
// W = Z Y.  Mirror-symmetric PML axes have eigenvalue pairs that agree to a
// few ulps; for such a pair the coupling T(j,k) is itself rounding-level and
// the two Schur vectors are already (to that level) a decoupled basis, so the
// back-substitution keeps them apart instead of dividing rounding noise by
// rounding noise.  W^{-1} is an explicit LU inverse (W^T M W is not diagonal
// for such pairs, so the transpose shortcut does not hold).
#include "eig.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <numeric>

namespace hs {

namespace {

inline double abs1(cd z) { return std::fabs(z.real()) + std::fabs(z.imag()); }

struct Mat {
  int n;
  std::vector<cd> a;
  explicit Mat(int n_) : n(n_), a(size_t(n_) * n_) {}
  cd& operator()(int i, int j) { return a[size_t(i) * n + j]; }
  cd operator()(int i, int j) const { return a[size_t(i) * n + j]; }
};

// Rotation G = [c s; -conj(s) c] with G [x; y] = [r; 0], c real.
inline void givens(cd x, cd y, double& c, cd& s) {
  double ay = std::abs(y);
  if (ay == 0.0) { c = 1.0; s = 0.0; return; }
  double ax = std::abs(x);
  if (ax == 0.0) { c = 0.0; s = std::conj(y) / ay; return; }
  double nrm = std::hypot(ax, ay);
  c = ax / nrm;
  s = (x / ax) * std::conj(y) / nrm;
}

bool schur(Mat& H, Mat& Z, std::string& err) {
  const int n = H.n;
  const double eps = DBL_EPSILON;
  double normH = 0;
  for (cd v : H.a) normH = std::max(normH, abs1(v));
  if (normH == 0) return true;
  int hi = n - 1;
  int iter = 0;
  long total = 0;
  const long max_total = 100L * n + 100;
  while (hi >= 0) {
    int l = hi;
    for (; l > 0; --l) {
      double s = abs1(H(l, l)) + abs1(H(l - 1, l - 1));
      if (s == 0) s = normH;
      if (abs1(H(l, l - 1)) <= eps * s) {
        H(l, l - 1) = 0.0;
        break;
      }
    }
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++total > max_total) {
      err = "QR iteration did not converge";
      return false;
    }
    ++iter;
    cd mu;
    if (iter % 10 == 0) {
      // exceptional shift to break a cycle
      mu = H(hi, hi) + cd(0.75 * abs1(H(hi, hi - 1)), 0.0);
    } else {
      cd a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
      cd half = 0.5 * (a - d);
      cd disc = std::sqrt(half * half + b * c);
      cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
      mu = (std::abs(m1 - d) <= std::abs(m2 - d)) ? m1 : m2;
    }
    cd x = H(l, l) - mu, y = H(l + 1, l);
    for (int k = l; k < hi; ++k) {
      if (k > l) {
        x = H(k, k - 1);
        y = H(k + 1, k - 1);
      }
      double c;
      cd s;
      givens(x, y, c, s);
      const int j0 = (k > l) ? k - 1 : l;
      for (int j = j0; j < n; ++j) {
        cd t1 = H(k, j), t2 = H(k + 1, j);
        H(k, j) = c * t1 + s * t2;
        H(k + 1, j) = -std::conj(s) * t1 + c * t2;
      }
      if (k > l) H(k + 1, k - 1) = 0.0;
      const int i1 = std::min(k + 2, hi);
      for (int i = 0; i <= i1; ++i) {
        cd t1 = H(i, k), t2 = H(i, k + 1);
        H(i, k) = t1 * c + t2 * std::conj(s);
        H(i, k + 1) = -t1 * s + t2 * c;
      }
      for (int i = 0; i < n; ++i) {
        cd t1 = Z(i, k), t2 = Z(i, k + 1);
        Z(i, k) = t1 * c + t2 * std::conj(s);
        Z(i, k + 1) = -t1 * s + t2 * c;
      }
    }
  }
  return true;
}

// Explicit inverse by LU with partial pivoting.  Returns false if singular.
bool lu_inverse(const std::vector<cd>& A, int n, std::vector<cd>& inv) {
  Mat LU(n);
  LU.a = A;
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(LU(k, k));
    for (int i = k + 1; i < n; ++i) {
      double v = std::abs(LU(i, k));
      if (v > best) { best = v; p = i; }
    }
    if (best == 0.0) return false;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(LU(k, j), LU(p, j));
    cd d = 1.0 / LU(k, k);
    for (int i = k + 1; i < n; ++i) {
      cd f = LU(i, k) * d;
      LU(i, k) = f;
      if (f == 0.0) continue;
      for (int j = k + 1; j < n; ++j) LU(i, j) -= f * LU(k, j);
    }
  }
  inv.assign(size_t(n) * n, 0.0);
  std::vector<cd> col(n);
  for (int c = 0; c < n; ++c) {
    std::fill(col.begin(), col.end(), cd(0.0));
    col[c] = 1.0;
    // apply the row swaps in order
    for (int k = 0; k < n; ++k)
      if (piv[k] != k) std::swap(col[k], col[piv[k]]);
    for (int i = 1; i < n; ++i) {
      cd s = col[i];
      for (int j = 0; j < i; ++j) s -= LU(i, j) * col[j];
      col[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      cd s = col[i];
      for (int j = i + 1; j < n; ++j) s -= LU(i, j) * col[j];
      col[i] = s / LU(i, i);
    }
    for (int i = 0; i < n; ++i) inv[size_t(i) * n + c] = col[i];
  }
  return true;
}

double norm1(const std::vector<cd>& A, int n) {
  double best = 0;
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += std::abs(A[size_t(i) * n + j]);
    best = std::max(best, s);
  }
  return best;
}

void fill_stats(const std::vector<cd>& D, AxisEig& e) {
  const int n = e.n;
  double nD = 0, nW = 0;
  for (cd v : D) nD += std::norm(v);
  for (cd v : e.W) nW += std::norm(v);
  nD = std::sqrt(nD);
  nW = std::sqrt(nW);
  // DW (D is tridiagonal)
  std::vector<cd> DW(size_t(n) * n);
  double res = 0;
  for (int i = 0; i < n; ++i)
    for (int m = 0; m < n; ++m) {
      cd s = D[size_t(i) * n + i] * e.W[size_t(i) * n + m];
      if (i > 0) s += D[size_t(i) * n + i - 1] * e.W[size_t(i - 1) * n + m];
      if (i + 1 < n) s += D[size_t(i) * n + i + 1] * e.W[size_t(i + 1) * n + m];
      DW[size_t(i) * n + m] = s;
      res += std::norm(s - e.W[size_t(i) * n + m] * e.lam[m]);
    }
  e.eig_resid = (nD > 0 && nW > 0) ? std::sqrt(res) / (nD * nW) : 0.0;
  double inv_res = 0, dec = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cd s = 0.0, t = 0.0;
      for (int k = 0; k < n; ++k) {
        cd w = e.Winv[size_t(i) * n + k];
        s += w * e.W[size_t(k) * n + j];
        t += w * DW[size_t(k) * n + j];
      }
      inv_res = std::max(inv_res, std::abs(s - (i == j ? cd(1.0) : cd(0.0))));
      if (i != j) dec = std::max(dec, std::abs(t));
    }
  e.inv_resid = inv_res;
  e.decouple = nD > 0 ? dec / nD : 0.0;
  e.kappa = norm1(e.W, n) * norm1(e.Winv, n);
}

}  // namespace

std::vector<cd> axis_operator(int n, const cd* h) {
  std::vector<cd> D(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) {
    cd hh = 0.5 * (h[i] + h[i + 1]);
    D[size_t(i) * n + i] = (1.0 / h[i] + 1.0 / h[i + 1]) / hh;
    if (i > 0) D[size_t(i) * n + i - 1] = -1.0 / (h[i] * hh);
    if (i + 1 < n) D[size_t(i) * n + i + 1] = -1.0 / (h[i + 1] * hh);
  }
  return D;
}

bool axis_is_uniform(int n, const cd* h) {
  for (int i = 1; i <= n; ++i)
    if (h[i] != h[0]) return false;
  return true;
}

void axis_eig_uniform(int n, cd h, AxisEig& e) {
  e.n = n;
  e.lam.resize(n);
  e.W.resize(size_t(n) * n);
  const double pi = 3.14159265358979323846;
  const double sc = std::sqrt(2.0 / (n + 1));
  for (int m = 0; m < n; ++m) e.lam[m] = 2.0 * (1.0 - std::cos(pi * (m + 1) / (n + 1))) / (h * h);
  for (int i = 0; i < n; ++i)
    for (int m = 0; m < n; ++m) {
      // reduce the angle argument exactly: (i+1)(m+1) mod 2(n+1)
      long q = (long(i + 1) * long(m + 1)) % (2L * (n + 1));
      e.W[size_t(i) * n + m] = sc * std::sin(pi * double(q) / double(n + 1));
    }
  e.Winv = e.W;  // orthonormal and symmetric
  std::vector<cd> hv(n + 1, h);
  fill_stats(axis_operator(n, hv.data()), e);
}

bool axis_eig_general(int n, const cd* h, AxisEig& e, std::string& err) {
  e.n = n;
  std::vector<cd> D = axis_operator(n, h);
  Mat H(n), Z(n);
  H.a = D;
  for (int i = 0; i < n; ++i) Z(i, i) = 1.0;
  if (!schur(H, Z, err)) return false;
  double normT = 0;
  for (cd v : H.a) normT += std::norm(v);
  normT = std::sqrt(normT);
  const double delta = 1e3 * DBL_EPSILON * normT;
  std::vector<cd> lam(n);
  for (int k = 0; k < n; ++k) lam[k] = H(k, k);
  std::vector<cd> W(size_t(n) * n, 0.0);
  std::vector<cd> y(n);
  for (int k = 0; k < n; ++k) {
    std::fill(y.begin(), y.end(), cd(0.0));
    y[k] = 1.0;
    for (int j = k - 1; j >= 0; --j) {
      cd s = 0.0;
      for (int l = j + 1; l <= k; ++l) s += H(j, l) * y[l];
      cd den = H(j, j) - lam[k];
      if (std::abs(den) < delta) {
        if (std::abs(s) <= delta) {
          y[j] = 0.0;  // clustered pair, rounding-level coupling: keep Schur vectors apart
          continue;
        }
        den = cd(delta, 0.0);
      }
      y[j] = -s / den;
      if (std::abs(y[j]) > 1e100) {
        err = "eigenvector back-substitution overflow";
        return false;
      }
    }
    double nrm = 0;
    for (int i = 0; i < n; ++i) {
      cd s = 0.0;
      for (int l = 0; l <= k; ++l) s += Z(i, l) * y[l];
      W[size_t(i) * n + k] = s;
      nrm += std::norm(s);
    }
    nrm = std::sqrt(nrm);
    for (int i = 0; i < n; ++i) W[size_t(i) * n + k] /= nrm;
  }
  // order modes by eigenvalue (real part, then imaginary)
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (lam[a].real() != lam[b].real()) return lam[a].real() < lam[b].real();
    return lam[a].imag() < lam[b].imag();
  });
  e.lam.resize(n);
  e.W.assign(size_t(n) * n, 0.0);
  for (int m = 0; m < n; ++m) {
    e.lam[m] = lam[ord[m]];
    for (int i = 0; i < n; ++i) e.W[size_t(i) * n + m] = W[size_t(i) * n + ord[m]];
  }
  if (!lu_inverse(e.W, n, e.Winv)) {
    err = "eigenvector matrix is singular";
    return false;
  }
  fill_stats(D, e);
  return true;
}

}  // namespace hs
