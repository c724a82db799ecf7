"""Manufactured solutions of the unsteady Navier-Stokes equations (oracle).

The PDE is eq. (3) of Section 2.1 with density 1. Each problem supplies the
exact velocity u(x, t), pressure p(x, t) and body force
f = du/dt - nu Lap u + (u . grad) u + grad p, written out by hand and checked
against symbolic differentiation in the tests.

* TaylorGreen2D: u = (-cos kx sin ky, sin kx cos ky) e^{-2 nu k^2 t},
  p = -(cos 2kx + cos 2ky)/4 e^{-4 nu k^2 t}, f = 0.
* John2D: the unsteady benchmark of Section 5.1 (nu = rho = 1 in the paper).
* Beltrami3D: Ethier & Steinman (1994), f = 0, decay e^{-nu d^2 t}.
* PolySteady2D / PolySteady3D: quadratic divergence-free u, linear p with
  zero mean; every IPCS integrand is a polynomial of degree <= 5, so the
  interpolated exact state is a fixed point of one step.
* PolySteady2DCubic: the same for the P3-P2 pair: cubic divergence-free u
  (from a quartic stream function), quadratic zero-mean p; every integrand
  of the P3-P2 step has degree <= 8.
Points x have shape (..., d); returns have shape (..., d) or (...).
"""
import numpy as np

PI = np.pi


class TaylorGreen2D:
    dim = 2

    def __init__(self, k=PI, nu=0.01):
        self.k, self.nu = float(k), float(nu)

    def u(self, x, t):
        k = self.k
        e = np.exp(-2.0 * self.nu * k * k * t)
        X, Y = x[..., 0], x[..., 1]
        return np.stack([-np.cos(k * X) * np.sin(k * Y) * e,
                         np.sin(k * X) * np.cos(k * Y) * e], axis=-1)

    def p(self, x, t):
        k = self.k
        e = np.exp(-4.0 * self.nu * k * k * t)
        X, Y = x[..., 0], x[..., 1]
        return -0.25 * (np.cos(2 * k * X) + np.cos(2 * k * Y)) * e

    f = None


class John2D:
    """u1 = 2 pi sin t sin^2(pi x) sin(pi y) cos(pi y),
    u2 = -2 pi sin t sin(pi x) cos(pi x) sin^2(pi y), p = 20 sin t (x^2 y - 1/6)."""
    dim = 2

    def __init__(self, nu=1.0):
        self.nu = float(nu)

    def u(self, x, t):
        X, Y = x[..., 0], x[..., 1]
        S = np.sin(t)
        u1 = 2 * PI * S * np.sin(PI * X) ** 2 * np.sin(PI * Y) * np.cos(PI * Y)
        u2 = -2 * PI * S * np.sin(PI * X) * np.cos(PI * X) * np.sin(PI * Y) ** 2
        return np.stack([u1, u2], axis=-1)

    def p(self, x, t):
        X, Y = x[..., 0], x[..., 1]
        return 20.0 * np.sin(t) * (X * X * Y - 1.0 / 6.0)

    def f(self, x, t):
        X, Y = x[..., 0], x[..., 1]
        S, Cs = np.sin(t), np.cos(t)
        s2x, c2x = np.sin(2 * PI * X), np.cos(2 * PI * X)
        s2y, c2y = np.sin(2 * PI * Y), np.cos(2 * PI * Y)
        sx2 = np.sin(PI * X) ** 2
        sy2 = np.sin(PI * Y) ** 2
        u1 = PI * S * sx2 * s2y
        u2 = -PI * S * s2x * sy2
        du1dt = PI * Cs * sx2 * s2y
        du2dt = -PI * Cs * s2x * sy2
        u1x = PI ** 2 * S * s2x * s2y
        u1y = 2 * PI ** 2 * S * sx2 * c2y
        u2x = -2 * PI ** 2 * S * c2x * sy2
        u2y = -PI ** 2 * S * s2x * s2y
        lap1 = 2 * PI ** 3 * S * s2y * (2 * c2x - 1)
        lap2 = 2 * PI ** 3 * S * s2x * (1 - 2 * c2y)
        px = 40.0 * S * X * Y
        py = 20.0 * S * X * X
        f1 = du1dt - self.nu * lap1 + u1 * u1x + u2 * u1y + px
        f2 = du2dt - self.nu * lap2 + u1 * u2x + u2 * u2y + py
        return np.stack([f1, f2], axis=-1)


class Beltrami3D:
    dim = 3

    def __init__(self, a=PI / 4, d=PI / 2, nu=0.01):
        self.a, self.d, self.nu = float(a), float(d), float(nu)

    def u(self, x, t):
        a, d = self.a, self.d
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        e = np.exp(-self.nu * d * d * t)
        u1 = -a * (np.exp(a * X) * np.sin(a * Y + d * Z) + np.exp(a * Z) * np.cos(a * X + d * Y))
        u2 = -a * (np.exp(a * Y) * np.sin(a * Z + d * X) + np.exp(a * X) * np.cos(a * Y + d * Z))
        u3 = -a * (np.exp(a * Z) * np.sin(a * X + d * Y) + np.exp(a * Y) * np.cos(a * Z + d * X))
        return np.stack([u1 * e, u2 * e, u3 * e], axis=-1)

    def p(self, x, t):
        a, d = self.a, self.d
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        e = np.exp(-2.0 * self.nu * d * d * t)
        q = (np.exp(2 * a * X) + np.exp(2 * a * Y) + np.exp(2 * a * Z)
             + 2 * np.sin(a * X + d * Y) * np.cos(a * Z + d * X) * np.exp(a * (Y + Z))
             + 2 * np.sin(a * Y + d * Z) * np.cos(a * X + d * Y) * np.exp(a * (Z + X))
             + 2 * np.sin(a * Z + d * X) * np.cos(a * Y + d * Z) * np.exp(a * (X + Y)))
        return -0.5 * a * a * q * e

    f = None


class PolySteady2D:
    """u = (y^2, x^2), p = x + y - 1, f = (1 - 2nu + 2x^2 y, 1 - 2nu + 2x y^2)."""
    dim = 2

    def __init__(self, nu=0.1):
        self.nu = float(nu)

    def u(self, x, t):
        X, Y = x[..., 0], x[..., 1]
        return np.stack([Y * Y, X * X], axis=-1)

    def p(self, x, t):
        return x[..., 0] + x[..., 1] - 1.0

    def f(self, x, t):
        X, Y = x[..., 0], x[..., 1]
        c = 1.0 - 2.0 * self.nu
        return np.stack([c + 2 * X * X * Y, c + 2 * X * Y * Y], axis=-1)


class PolySteady3D:
    """u = (y^2+z^2, z^2+x^2, x^2+y^2), p = x + y + z - 3/2,
    f_1 = 1 - 4nu + 2y(z^2+x^2) + 2z(x^2+y^2) and cyclic."""
    dim = 3

    def __init__(self, nu=0.1):
        self.nu = float(nu)

    def u(self, x, t):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        return np.stack([Y * Y + Z * Z, Z * Z + X * X, X * X + Y * Y], axis=-1)

    def p(self, x, t):
        return x[..., 0] + x[..., 1] + x[..., 2] - 1.5

    def f(self, x, t):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        c = 1.0 - 4.0 * self.nu
        u1, u2, u3 = Y * Y + Z * Z, Z * Z + X * X, X * X + Y * Y
        f1 = c + 2 * Y * u2 + 2 * Z * u3
        f2 = c + 2 * X * u1 + 2 * Z * u3
        f3 = c + 2 * X * u1 + 2 * Y * u2
        return np.stack([f1, f2, f3], axis=-1)


class PolySteady3DCubic:
    """u = (y^3 + z^2, z^3 + x^2, x^3 + y^2) (each component independent of its
    own coordinate, so div u = 0), p = xy + yz + zx - 3/4 (zero mean on the
    unit cube), f = (u . grad) u - nu Lap u + grad p with
    Lap u = (6y + 2, 6z + 2, 6x + 2): every integrand of the P3-P2 step has
    degree <= 8, so the interpolated state is a fixed point."""
    dim = 3

    def __init__(self, nu=0.1):
        self.nu = float(nu)

    def u(self, x, t):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        return np.stack([Y ** 3 + Z * Z, Z ** 3 + X * X, X ** 3 + Y * Y], axis=-1)

    def p(self, x, t):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        return X * Y + Y * Z + Z * X - 0.75

    def f(self, x, t):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        u1, u2, u3 = Y ** 3 + Z * Z, Z ** 3 + X * X, X ** 3 + Y * Y
        f1 = u2 * 3 * Y * Y + u3 * 2 * Z - self.nu * (6 * Y + 2) + (Y + Z)
        f2 = u1 * 2 * X + u3 * 3 * Z * Z - self.nu * (6 * Z + 2) + (X + Z)
        f3 = u1 * 3 * X * X + u2 * 2 * Y - self.nu * (6 * X + 2) + (X + Y)
        return np.stack([f1, f2, f3], axis=-1)


class PolySteady2DCubic:
    """Stream function psi = x^3 y + x^2 y^2, u = (psi_y, -psi_x)
    = (x^3 + 2x^2 y, -3x^2 y - 2x y^2), p = x^2 - y^2 + xy - 1/4 (zero mean on
    the unit square), f = (u . grad) u - nu Lap u + grad p with
    Lap u = (6x + 4y, -4x - 6y), grad p = (2x + y, x - 2y)."""
    dim = 2

    def __init__(self, nu=0.1):
        self.nu = float(nu)

    def u(self, x, t):
        X, Y = x[..., 0], x[..., 1]
        return np.stack([X ** 3 + 2 * X * X * Y, -3 * X * X * Y - 2 * X * Y * Y], axis=-1)

    def p(self, x, t):
        X, Y = x[..., 0], x[..., 1]
        return X * X - Y * Y + X * Y - 0.25

    def f(self, x, t):
        X, Y = x[..., 0], x[..., 1]
        u1 = X ** 3 + 2 * X * X * Y
        u2 = -3 * X * X * Y - 2 * X * Y * Y
        u1x, u1y = 3 * X * X + 4 * X * Y, 2 * X * X
        u2x, u2y = -6 * X * Y - 2 * Y * Y, -3 * X * X - 4 * X * Y
        f1 = u1 * u1x + u2 * u1y - self.nu * (6 * X + 4 * Y) + (2 * X + Y)
        f2 = u1 * u2x + u2 * u2y - self.nu * (-4 * X - 6 * Y) + (X - 2 * Y)
        return np.stack([f1, f2], axis=-1)


class SteadyPaper2D:
    """The steady example of Section 4.2 on the unit square:
    u = 10 x^2 (x-1)^2 y (y-1)(2y-1), v = -10 x (x-1)(2x-1) y^2 (y-1)^2,
    p = 10 (2x-1)(2y-1), f = -nu Lap u + (u . grad) u + grad p. The fields are
    polynomials; their derivatives are taken exactly from numpy polynomial
    coefficients: with a(s) = s^2 (s-1)^2, a'(s) = 2 s (s-1)(2s-1), so
    u = 5 a(x) a'(y), v = -5 a'(x) a(y), the curl of the stream function
    5 a(x) a(y) (div u = 0)."""
    dim = 2

    def __init__(self, nu=1.0):
        from numpy.polynomial import polynomial as Pl
        self.nu = float(nu)
        a = Pl.polymul([0.0, 0.0, 1.0], Pl.polymul([-1.0, 1.0], [-1.0, 1.0]))  # s^2 (s-1)^2
        self._a = a
        self._da = Pl.polyder(a)
        self._dda = Pl.polyder(a, 2)
        self._ddda = Pl.polyder(a, 3)
        self._P = Pl

    def _ev(self, c, s):
        return self._P.polyval(s, c)

    def u(self, x, t=0.0):
        X, Y = x[..., 0], x[..., 1]
        e = self._ev
        return np.stack([5.0 * e(self._a, X) * e(self._da, Y),
                         -5.0 * e(self._da, X) * e(self._a, Y)], axis=-1)

    def p(self, x, t=0.0):
        X, Y = x[..., 0], x[..., 1]
        return 10.0 * (2 * X - 1) * (2 * Y - 1)

    def f(self, x, t=0.0):
        X, Y = x[..., 0], x[..., 1]
        e = self._ev
        a, da, dda, ddda = self._a, self._da, self._dda, self._ddda
        u1 = 5.0 * e(a, X) * e(da, Y)
        u2 = -5.0 * e(da, X) * e(a, Y)
        u1x, u1y = 5.0 * e(da, X) * e(da, Y), 5.0 * e(a, X) * e(dda, Y)
        u2x, u2y = -5.0 * e(dda, X) * e(a, Y), -5.0 * e(da, X) * e(da, Y)
        lap1 = 5.0 * (e(dda, X) * e(da, Y) + e(a, X) * e(ddda, Y))
        lap2 = -5.0 * (e(ddda, X) * e(a, Y) + e(da, X) * e(dda, Y))
        px, py = 20.0 * (2 * Y - 1), 20.0 * (2 * X - 1)
        return np.stack([-self.nu * lap1 + u1 * u1x + u2 * u1y + px,
                         -self.nu * lap2 + u1 * u2x + u2 * u2y + py], axis=-1)
