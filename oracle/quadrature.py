"""Quadrature rules on the reference simplex (oracle; test infrastructure).

The paper names numerical integration as an algorithm-level service
(Section 3.1, Algorithm Level) but does not fix a rule. Every integrand of the
IPCS step with P2-P1 elements is a polynomial of degree <= 5 (mass 4,
convection P2*(P2.grad P2) = 5, the rest <= 2), so any rule exact to degree 5
reproduces the matrices up to rounding. The oracle uses:

* triangles: the 7-point degree-5 rule of Radon (Stroud T2:5-1), whose
  points and weights have closed forms in sqrt(15);
* tetrahedra: Stroud's conical-product rule, 3 Gauss-Jacobi points per
  collapsed direction (27 points, exact to degree 5), built from
  scipy.special.roots_jacobi;
* error norms: collapsed Gauss rules with more points (degree >= 9);
* the P3-P2 pair (triangles), whose convection integrand P3 (P3 . grad P3)
  has degree 8: the collapsed (Duffy) product of two 5-point Gauss-Legendre
  rules, from numpy.polynomial.legendre.leggauss. The Jacobian factor 1 - u
  is carried by the weights, so the rule is exact to degree 8. Any rule exact
  to degree 8 gives the step's polynomial integrands up to rounding; the
  non-polynomial forcing terms depend on the rule, and this is the rule the
  kernels implement.

All rules return barycentric coordinates lam[q, 0..d] and weights that sum to
the reference-simplex measure 1/d! (area 1/2, volume 1/6).
"""
import numpy as np
from scipy.special import roots_jacobi


def triangle_deg5():
    """Radon's 7-point rule, degree 5 (barycentric points, weights sum to 1/2)."""
    s = np.sqrt(15.0)
    a = (6.0 - s) / 21.0
    b = (6.0 + s) / 21.0
    wa = (155.0 - s) / 1200.0
    wb = (155.0 + s) / 1200.0
    pts = [(1 / 3, 1 / 3, 1 / 3)]
    wts = [9.0 / 40.0]
    for c, w in ((a, wa), (b, wb)):
        for k in range(3):
            p = [c, c, c]
            p[k] = 1.0 - 2.0 * c
            pts.append(tuple(p))
            wts.append(w)
    return np.array(pts), 0.5 * np.array(wts)


def _gauss_jacobi_01(n, alpha):
    """n-point Gauss-Jacobi rule on [0,1] for weight (1-u)^alpha."""
    t, w = roots_jacobi(n, alpha, 0.0)
    u = 0.5 * (1.0 + t)
    # (1-u)^alpha = ((1-t)/2)^alpha and du = dt/2
    return u, w * 0.5 ** (alpha + 1)


def triangle_collapsed(n):
    """Collapsed (Duffy) product rule, n x n points, exact to degree 2n-1.

    x = u, y = v (1 - u), Jacobian (1 - u).
    """
    u, wu = _gauss_jacobi_01(n, 1.0)
    v, wv = _gauss_jacobi_01(n, 0.0)
    U, V = np.meshgrid(u, v, indexing="ij")
    W = np.outer(wu, wv)
    x = U.ravel()
    y = (V * (1.0 - U)).ravel()
    lam = np.stack([1.0 - x - y, x, y], axis=1)
    return lam, W.ravel()


def triangle_collapsed_gl(n):
    """Collapsed product of n-point Gauss-Legendre rules, exact to degree 2n-2.

    x = u, y = v (1 - u); the Jacobian (1 - u) multiplies the weights.
    """
    t, w = np.polynomial.legendre.leggauss(n)
    u, wu = 0.5 * (1.0 + t), 0.5 * w
    U, V = np.meshgrid(u, u, indexing="ij")
    W = np.outer(wu, wu) * (1.0 - U)
    x = U.ravel()
    y = (V * (1.0 - U)).ravel()
    lam = np.stack([1.0 - x - y, x, y], axis=1)
    return lam, W.ravel()


def tet_collapsed(n):
    """Stroud conical product on the tetrahedron, n^3 points, degree 2n-1.

    x = u, y = v (1 - u), z = w (1 - u)(1 - v), Jacobian (1-u)^2 (1-v).
    """
    u, wu = _gauss_jacobi_01(n, 2.0)
    v, wv = _gauss_jacobi_01(n, 1.0)
    s, ws = _gauss_jacobi_01(n, 0.0)
    U, V, S = np.meshgrid(u, v, s, indexing="ij")
    W = wu[:, None, None] * wv[None, :, None] * ws[None, None, :]
    x = U.ravel()
    y = (V * (1.0 - U)).ravel()
    z = (S * (1.0 - U) * (1.0 - V)).ravel()
    lam = np.stack([1.0 - x - y - z, x, y, z], axis=1)
    return lam, W.ravel()


def tet_deg5():
    """Degree-5 rule for tetrahedra used by the oracle: 27-point conical product."""
    return tet_collapsed(3)


def cell_rule(dim):
    """The degree-5 rule the oracle uses for every cell integral."""
    return triangle_deg5() if dim == 2 else tet_deg5()


def error_rule(dim):
    """High-order rule for L2 error norms (degree 9)."""
    return triangle_collapsed(5) if dim == 2 else tet_collapsed(5)
