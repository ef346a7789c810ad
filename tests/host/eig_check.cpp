// Host check of the plan's axis eigensolver, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py: for uniform,
// graded, stretched (complex, mirror-symmetric) and tiny axes, the residuals
// of D W = W Lambda and W^{-1} W = I recomputed here from D = M^{-1} K
// (Sec. 2, the 1D generalized problems of each block axis).
#include <cmath>
#include <complex>
#include <cstdio>
#include <string>
#include <vector>

#include "eig.hpp"

using hs::cd;

static double frob(const std::vector<cd>& a) {
  double s = 0;
  for (const cd& v : a) s += std::norm(v);
  return std::sqrt(s);
}

// returns true when both residuals are within bounds
static bool check(const char* name, int n, const std::vector<cd>& h, bool uniform, double tol_eig, double tol_inv) {
  hs::AxisEig e;
  std::string err;
  if (uniform) {
    hs::axis_eig_uniform(n, h[0], e);
  } else if (!hs::axis_eig_general(n, h.data(), e, err)) {
    std::printf("%s n=%d: solver failed: %s\n", name, n, err.c_str());
    return false;
  }
  const std::vector<cd> D = hs::axis_operator(n, h.data());
  std::vector<cd> R(size_t(n) * n), I(size_t(n) * n);
  for (int i = 0; i < n; ++i)
    for (int m = 0; m < n; ++m) {
      cd dw = 0, wi = 0;
      for (int k = 0; k < n; ++k) {
        dw += D[size_t(i) * n + k] * e.W[size_t(k) * n + m];
        wi += e.Winv[size_t(i) * n + k] * e.W[size_t(k) * n + m];
      }
      R[size_t(i) * n + m] = dw - e.W[size_t(i) * n + m] * e.lam[m];
      I[size_t(i) * n + m] = wi - (i == m ? cd(1) : cd(0));
    }
  const double re = frob(R) / (frob(D) * frob(e.W));
  double ri = 0;
  for (const cd& v : I) ri = std::fmax(ri, std::abs(v));
  const bool ok = re <= tol_eig && ri <= tol_inv;
  std::printf("%-28s n=%4d  eig %.2e  inv %.2e  kappa %.2e  %s\n", name, n, re, ri, e.kappa, ok ? "ok" : "FAIL");
  return ok;
}

// the stretched axes of the workloads: a unit-step core of `core` cells and
// p cells per side whose steps grow outward as 1.2^k (1 + 0.5 i), k = 1..p
static std::vector<cd> pml_axis(int core, int p) {
  std::vector<cd> h;
  for (int k = p; k >= 1; --k) h.push_back(std::pow(1.2, k) * cd(1, 0.5));
  for (int k = 0; k < core; ++k) h.push_back(cd(1, 0));
  for (int k = 1; k <= p; ++k) h.push_back(std::pow(1.2, k) * cd(1, 0.5));
  return h;
}

int main() {
  bool ok = true;
  for (int n : {1, 2, 3, 15, 64, 255}) ok &= check("uniform closed form", n, std::vector<cd>(size_t(n) + 1, cd(0.5, 0)), true, 1e-13, 1e-12);
  for (int n : {1, 2, 3, 31, 100}) ok &= check("uniform via QR", n, std::vector<cd>(size_t(n) + 1, cd(1, 0)), false, 1e-12, 1e-10);
  for (int n : {4, 23, 97}) {
    std::vector<cd> h(size_t(n) + 1);
    unsigned s = 12345u + unsigned(n);
    for (auto& v : h) {
      s = s * 1103515245u + 12345u;
      v = cd(0.6 + 0.8 * double((s >> 8) & 0xffff) / 65535.0, 0);
    }
    ok &= check("graded real steps", n, h, false, 1e-12, 1e-10);
  }
  for (auto cp : {std::pair<int, int>{32, 8}, {128, 16}, {256, 16}, {512, 32}}) {
    const std::vector<cd> h = pml_axis(cp.first, cp.second);
    ok &= check("stretched ends (PML)", int(h.size()) - 1, h, false, 1e-12, 1e-10);
  }
  std::printf(ok ? "all ok\n" : "failures\n");
  return ok ? 0 : 1;
}
