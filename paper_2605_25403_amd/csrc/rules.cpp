// Host-built quadrature rules (rules.hpp).
#include <cmath>
#include <vector>

#include "common.hpp"
#include "rules.hpp"

namespace ipcs {

namespace {

// Jacobi polynomial P_n^(a,0)(t) and its derivative, by the three-term
// recurrence and the derivative identity
// (2n + a)(1 - t^2) P_n' = n (a - (2n + a) t) P_n + 2 n (n + a) P_{n-1}.
void jacobi(int n, double a, double t, double& p, double& dp) {
  double pm = 1.0, pc = 0.5 * (a + (a + 2.0) * t);
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    const double c = 2.0 * k * (k + a) * (2.0 * k + a - 2.0);
    const double c1 = (2.0 * k + a - 1.0) * ((2.0 * k + a) * (2.0 * k + a - 2.0) * t + a * a);
    const double c2 = 2.0 * (k + a - 1.0) * (k - 1.0) * (2.0 * k + a);
    const double pn = (c1 * pc - c2 * pm) / c;
    pm = pc;
    pc = pn;
  }
  p = pc;
  dp = (n * (a - (2.0 * n + a) * t) * pc + 2.0 * n * (n + a) * pm) /
       ((2.0 * n + a) * (1.0 - t * t));
}

// n-point Gauss-Jacobi rule on [0, 1] for the weight (1 - u)^a
void gauss_jacobi01(int n, double a, double* u, double* w) {
  int found = 0;
  const int grid = 20000;
  double tp = -1.0 + 1e-12, pp, dp;
  jacobi(n, a, tp, pp, dp);
  for (int i = 1; i <= grid && found < n; ++i) {
    const double t = -1.0 + 2.0 * i / grid - (i == grid ? 1e-12 : 0.0);
    double p;
    jacobi(n, a, t, p, dp);
    if ((p > 0) != (pp > 0)) {
      double lo = tp, hi = t;
      double x = 0.5 * (lo + hi);
      for (int it = 0; it < 200; ++it) {   // safeguarded Newton
        double fx, dfx, flo, dflo;
        jacobi(n, a, x, fx, dfx);
        jacobi(n, a, lo, flo, dflo);
        if ((fx > 0) == (flo > 0)) lo = x;
        else hi = x;
        double xn = x - fx / dfx;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (std::fabs(xn - x) < 1e-17) {
          x = xn;
          break;
        }
        x = xn;
      }
      jacobi(n, a, x, pp, dp);
      u[found] = 0.5 * (1.0 + x);
      // 2^(a+1) / ((1 - t^2) P_n'(t)^2) on [-1, 1]; / 2^(a+1) on [0, 1]
      w[found] = 1.0 / ((1.0 - x * x) * dp * dp);
      ++found;
    }
    tp = t;
    pp = p;
  }
  if (found != n) fail(IPCS_E_INVALID, "Gauss-Jacobi rule: root not found");
}

}  // namespace

void tet_rule9(double* lam, double* w) {
  constexpr int n = RuleTet9::N1;
  double u[n], wu[n], v[n], wv[n], s[n], ws[n];
  gauss_jacobi01(n, 2.0, u, wu);
  gauss_jacobi01(n, 1.0, v, wv);
  gauss_jacobi01(n, 0.0, s, ws);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        const int q = (i * n + j) * n + k;
        const double x = u[i], y = v[j] * (1.0 - u[i]), z = s[k] * (1.0 - u[i]) * (1.0 - v[j]);
        lam[4 * q + 0] = 1.0 - x - y - z;
        lam[4 * q + 1] = x;
        lam[4 * q + 2] = y;
        lam[4 * q + 3] = z;
        w[q] = wu[i] * wv[j] * ws[k];
      }
}

}  // namespace ipcs
