// Closed-form manufactured solutions of the unsteady Navier-Stokes equations
// (Section 2.1, eq. (3), density 1), evaluated on the device for Dirichlet
// data, forcing and initial states.
//   Taylor-Green 2D : u = (-cos kx sin ky, sin kx cos ky) e^{-2 nu k^2 t},
//                     p = -(cos 2kx + cos 2ky)/4 e^{-4 nu k^2 t}, f = 0.
//   John 2D         : the unsteady benchmark of Section 5.1.
//   Beltrami 3D     : Ethier & Steinman (1994), parameters a, d; f = 0.
//   Polynomial      : u = (y^2, x^2), p = x + y - 1 (2D) and
//                     u = (y^2+z^2, z^2+x^2, x^2+y^2), p = x+y+z-3/2 (3D).
//   Steady example  : Section 4.2, u = 10 x^2 (x-1)^2 y (y-1)(2y-1),
//                     v = -10 x (x-1)(2x-1) y^2 (y-1)^2, p = 10 (2x-1)(2y-1),
//                     f = -nu Lap u + (u.grad)u + grad p (steady).
// The steady example's velocity is the curl of 5 a(x) a(y) with
// a(s) = s^2 (s-1)^2: u = 5 a(x) a'(y), v = -5 a'(x) a(y).
struct SteadyPoly {
  __host__ __device__ static double a(double s) { return s * s * (s - 1.0) * (s - 1.0); }
  __host__ __device__ static double a1(double s) { return ((4.0 * s - 6.0) * s + 2.0) * s; }
  __host__ __device__ static double a2(double s) { return (12.0 * s - 12.0) * s + 2.0; }
  __host__ __device__ static double a3(double s) { return 24.0 * s - 12.0; }
};
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.hpp"
#include "ipcs.h"

namespace ipcs {

template <int D>
__host__ __device__ inline void builtin_velocity(const Builtin& bi, const double* x, double t,
                                                 double* u) {
  const double PI = 3.14159265358979323846;
  if constexpr (D == 2) {
    const double X = x[0], Y = x[1];
    switch (bi.kind) {
      case IPCS_SOL_TAYLOR_GREEN_2D: {
        const double k = bi.prm[0], e = exp(-2.0 * bi.nu * k * k * t);
        u[0] = -cos(k * X) * sin(k * Y) * e;
        u[1] = sin(k * X) * cos(k * Y) * e;
        return;
      }
      case IPCS_SOL_JOHN_2D: {
        const double S = sin(t), sx = sin(PI * X), sy = sin(PI * Y);
        u[0] = 2.0 * PI * S * sx * sx * sy * cos(PI * Y);
        u[1] = -2.0 * PI * S * sx * cos(PI * X) * sy * sy;
        return;
      }
      case IPCS_SOL_POLY_STEADY_2D:
        u[0] = Y * Y;
        u[1] = X * X;
        return;
      case IPCS_SOL_POLY_CUBIC_2D:   // stream function x^3 y + x^2 y^2
        u[0] = X * X * X + 2.0 * X * X * Y;
        u[1] = -3.0 * X * X * Y - 2.0 * X * Y * Y;
        return;
      case IPCS_SOL_STEADY_PAPER_2D:
        u[0] = 5.0 * SteadyPoly::a(X) * SteadyPoly::a1(Y);
        u[1] = -5.0 * SteadyPoly::a1(X) * SteadyPoly::a(Y);
        return;
    }
    u[0] = u[1] = 0.0;
  } else {
    const double X = x[0], Y = x[1], Z = x[2];
    switch (bi.kind) {
      case IPCS_SOL_BELTRAMI_3D: {
        const double a = bi.prm[0], d = bi.prm[1], e = exp(-bi.nu * d * d * t);
        u[0] = -a * (exp(a * X) * sin(a * Y + d * Z) + exp(a * Z) * cos(a * X + d * Y)) * e;
        u[1] = -a * (exp(a * Y) * sin(a * Z + d * X) + exp(a * X) * cos(a * Y + d * Z)) * e;
        u[2] = -a * (exp(a * Z) * sin(a * X + d * Y) + exp(a * Y) * cos(a * Z + d * X)) * e;
        return;
      }
      case IPCS_SOL_POLY_STEADY_3D:
        u[0] = Y * Y + Z * Z;
        u[1] = Z * Z + X * X;
        u[2] = X * X + Y * Y;
        return;
      case IPCS_SOL_POLY_CUBIC_3D:
        u[0] = Y * Y * Y + Z * Z;
        u[1] = Z * Z * Z + X * X;
        u[2] = X * X * X + Y * Y;
        return;
    }
    u[0] = u[1] = u[2] = 0.0;
  }
}

template <int D>
__host__ __device__ inline double builtin_pressure(const Builtin& bi, const double* x, double t) {
  if constexpr (D == 2) {
    const double X = x[0], Y = x[1];
    switch (bi.kind) {
      case IPCS_SOL_TAYLOR_GREEN_2D: {
        const double k = bi.prm[0];
        return -0.25 * (cos(2.0 * k * X) + cos(2.0 * k * Y)) * exp(-4.0 * bi.nu * k * k * t);
      }
      case IPCS_SOL_JOHN_2D: return 20.0 * sin(t) * (X * X * Y - 1.0 / 6.0);
      case IPCS_SOL_POLY_STEADY_2D: return X + Y - 1.0;
      case IPCS_SOL_POLY_CUBIC_2D: return X * X - Y * Y + X * Y - 0.25;
      case IPCS_SOL_STEADY_PAPER_2D: return 10.0 * (2.0 * X - 1.0) * (2.0 * Y - 1.0);
    }
    return 0.0;
  } else {
    const double X = x[0], Y = x[1], Z = x[2];
    switch (bi.kind) {
      case IPCS_SOL_BELTRAMI_3D: {
        const double a = bi.prm[0], d = bi.prm[1];
        const double q = exp(2 * a * X) + exp(2 * a * Y) + exp(2 * a * Z) +
                         2 * sin(a * X + d * Y) * cos(a * Z + d * X) * exp(a * (Y + Z)) +
                         2 * sin(a * Y + d * Z) * cos(a * X + d * Y) * exp(a * (Z + X)) +
                         2 * sin(a * Z + d * X) * cos(a * Y + d * Z) * exp(a * (X + Y));
        return -0.5 * a * a * q * exp(-2.0 * bi.nu * d * d * t);
      }
      case IPCS_SOL_POLY_STEADY_3D: return X + Y + Z - 1.5;
      case IPCS_SOL_POLY_CUBIC_3D: return X * Y + Y * Z + Z * X - 0.75;
    }
    return 0.0;
  }
}

// f = du/dt - nu Lap u + (u.grad)u + grad p
template <int D>
__host__ __device__ inline void builtin_force(const Builtin& bi, const double* x, double t,
                                              double* f) {
  const double PI = 3.14159265358979323846;
  const double nu = bi.nu;
  if constexpr (D == 2) {
    const double X = x[0], Y = x[1];
    if (bi.kind == IPCS_SOL_JOHN_2D) {
      const double S = sin(t), Cs = cos(t);
      const double s2x = sin(2 * PI * X), c2x = cos(2 * PI * X);
      const double s2y = sin(2 * PI * Y), c2y = cos(2 * PI * Y);
      const double sx = sin(PI * X), sy = sin(PI * Y);
      const double sx2 = sx * sx, sy2 = sy * sy;
      // u1 = pi S sin^2(pi x) sin(2 pi y), u2 = -pi S sin(2 pi x) sin^2(pi y)
      const double u1 = PI * S * sx2 * s2y, u2 = -PI * S * s2x * sy2;
      const double u1t = PI * Cs * sx2 * s2y, u2t = -PI * Cs * s2x * sy2;
      const double u1x = PI * PI * S * s2x * s2y, u1y = 2 * PI * PI * S * sx2 * c2y;
      const double u2x = -2 * PI * PI * S * c2x * sy2, u2y = -PI * PI * S * s2x * s2y;
      const double l1 = 2 * PI * PI * PI * S * s2y * (2 * c2x - 1);
      const double l2 = 2 * PI * PI * PI * S * s2x * (1 - 2 * c2y);
      f[0] = u1t - nu * l1 + u1 * u1x + u2 * u1y + 40.0 * S * X * Y;
      f[1] = u2t - nu * l2 + u1 * u2x + u2 * u2y + 20.0 * S * X * X;
      return;
    }
    if (bi.kind == IPCS_SOL_POLY_STEADY_2D) {
      f[0] = 1.0 - 2.0 * nu + 2.0 * X * X * Y;
      f[1] = 1.0 - 2.0 * nu + 2.0 * X * Y * Y;
      return;
    }
    if (bi.kind == IPCS_SOL_POLY_CUBIC_2D) {
      // (u.grad)u - nu Lap u + grad p; Lap u = (6x + 4y, -4x - 6y)
      const double u1 = X * X * X + 2.0 * X * X * Y, u2 = -3.0 * X * X * Y - 2.0 * X * Y * Y;
      const double u1x = 3.0 * X * X + 4.0 * X * Y, u1y = 2.0 * X * X;
      const double u2x = -6.0 * X * Y - 2.0 * Y * Y, u2y = -3.0 * X * X - 4.0 * X * Y;
      f[0] = u1 * u1x + u2 * u1y - nu * (6.0 * X + 4.0 * Y) + (2.0 * X + Y);
      f[1] = u1 * u2x + u2 * u2y - nu * (-4.0 * X - 6.0 * Y) + (X - 2.0 * Y);
      return;
    }
    if (bi.kind == IPCS_SOL_STEADY_PAPER_2D) {
      using S = SteadyPoly;
      const double u1 = 5.0 * S::a(X) * S::a1(Y), u2 = -5.0 * S::a1(X) * S::a(Y);
      const double u1x = 5.0 * S::a1(X) * S::a1(Y), u1y = 5.0 * S::a(X) * S::a2(Y);
      const double u2x = -5.0 * S::a2(X) * S::a(Y), u2y = -u1x;
      const double l1 = 5.0 * (S::a2(X) * S::a1(Y) + S::a(X) * S::a3(Y));
      const double l2 = -5.0 * (S::a3(X) * S::a(Y) + S::a1(X) * S::a2(Y));
      f[0] = -nu * l1 + u1 * u1x + u2 * u1y + 20.0 * (2.0 * Y - 1.0);
      f[1] = -nu * l2 + u1 * u2x + u2 * u2y + 20.0 * (2.0 * X - 1.0);
      return;
    }
    f[0] = f[1] = 0.0;
  } else {
    const double X = x[0], Y = x[1], Z = x[2];
    if (bi.kind == IPCS_SOL_POLY_STEADY_3D) {
      const double u1 = Y * Y + Z * Z, u2 = Z * Z + X * X, u3 = X * X + Y * Y;
      const double c = 1.0 - 4.0 * nu;
      f[0] = c + 2 * Y * u2 + 2 * Z * u3;
      f[1] = c + 2 * X * u1 + 2 * Z * u3;
      f[2] = c + 2 * X * u1 + 2 * Y * u2;
      return;
    }
    if (bi.kind == IPCS_SOL_POLY_CUBIC_3D) {
      // (u.grad)u - nu Lap u + grad p; Lap u = (6y + 2, 6z + 2, 6x + 2)
      const double u1 = Y * Y * Y + Z * Z, u2 = Z * Z * Z + X * X, u3 = X * X * X + Y * Y;
      f[0] = u2 * 3.0 * Y * Y + u3 * 2.0 * Z - nu * (6.0 * Y + 2.0) + (Y + Z);
      f[1] = u1 * 2.0 * X + u3 * 3.0 * Z * Z - nu * (6.0 * Z + 2.0) + (X + Z);
      f[2] = u1 * 3.0 * X * X + u2 * 2.0 * Y - nu * (6.0 * X + 2.0) + (X + Y);
      return;
    }
    f[0] = f[1] = f[2] = 0.0;
  }
}

inline bool builtin_has_force(int kind) {
  return kind == IPCS_SOL_JOHN_2D || kind == IPCS_SOL_POLY_STEADY_2D ||
         kind == IPCS_SOL_POLY_STEADY_3D || kind == IPCS_SOL_POLY_CUBIC_2D ||
         kind == IPCS_SOL_STEADY_PAPER_2D || kind == IPCS_SOL_POLY_CUBIC_3D;
}

}  // namespace ipcs
