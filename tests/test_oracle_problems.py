"""Pins of the manufactured solutions: the hand-written forcing equals the
Navier-Stokes residual du/dt - nu Lap u + (u.grad)u + grad p obtained by
symbolic differentiation, and every velocity is divergence-free."""
import numpy as np
import pytest
import sympy as sp

from oracle import problems

x, y, z, t = sp.symbols("x y z t", real=True)


def sym_fields(name, nu, k=None):
    pi = sp.pi
    if name == "tg":
        E = sp.exp(-2 * nu * k ** 2 * t)
        u = [-sp.cos(k * x) * sp.sin(k * y) * E, sp.sin(k * x) * sp.cos(k * y) * E]
        p = -sp.Rational(1, 4) * (sp.cos(2 * k * x) + sp.cos(2 * k * y)) * E ** 2
        return u, p, [x, y]
    if name == "john":
        u = [2 * pi * sp.sin(t) * sp.sin(pi * x) ** 2 * sp.sin(pi * y) * sp.cos(pi * y),
             -2 * pi * sp.sin(t) * sp.sin(pi * x) * sp.cos(pi * x) * sp.sin(pi * y) ** 2]
        p = 20 * sp.sin(t) * (x ** 2 * y - sp.Rational(1, 6))
        return u, p, [x, y]
    if name == "beltrami":
        a, d = pi / 4, pi / 2
        E = sp.exp(-nu * d ** 2 * t)
        u = [-a * (sp.exp(a * x) * sp.sin(a * y + d * z) + sp.exp(a * z) * sp.cos(a * x + d * y)) * E,
             -a * (sp.exp(a * y) * sp.sin(a * z + d * x) + sp.exp(a * x) * sp.cos(a * y + d * z)) * E,
             -a * (sp.exp(a * z) * sp.sin(a * x + d * y) + sp.exp(a * y) * sp.cos(a * z + d * x)) * E]
        p = -a ** 2 / 2 * (sp.exp(2 * a * x) + sp.exp(2 * a * y) + sp.exp(2 * a * z)
                           + 2 * sp.sin(a * x + d * y) * sp.cos(a * z + d * x) * sp.exp(a * (y + z))
                           + 2 * sp.sin(a * y + d * z) * sp.cos(a * x + d * y) * sp.exp(a * (z + x))
                           + 2 * sp.sin(a * z + d * x) * sp.cos(a * y + d * z) * sp.exp(a * (x + y))) * E ** 2
        return u, p, [x, y, z]
    if name == "poly2":
        return [y ** 2, x ** 2], x + y - 1, [x, y]
    if name == "poly2c":
        return ([x ** 3 + 2 * x ** 2 * y, -3 * x ** 2 * y - 2 * x * y ** 2],
                x ** 2 - y ** 2 + x * y - sp.Rational(1, 4), [x, y])
    if name == "steady_paper":
        return ([10 * x ** 2 * (x - 1) ** 2 * y * (y - 1) * (2 * y - 1),
                 -10 * x * (x - 1) * (2 * x - 1) * y ** 2 * (y - 1) ** 2],
                10 * (2 * x - 1) * (2 * y - 1), [x, y])
    if name == "poly3c":
        return ([y ** 3 + z ** 2, z ** 3 + x ** 2, x ** 3 + y ** 2],
                x * y + y * z + z * x - sp.Rational(3, 4), [x, y, z])
    if name == "poly3":
        return [y ** 2 + z ** 2, z ** 2 + x ** 2, x ** 2 + y ** 2], x + y + z - sp.Rational(3, 2), [x, y, z]
    raise KeyError(name)


CASES = [
    ("tg", problems.TaylorGreen2D(2 * np.pi, 0.03), dict(nu=sp.Rational(3, 100), k=2 * sp.pi)),
    ("john", problems.John2D(1.0), dict(nu=1)),
    ("john", problems.John2D(0.2), dict(nu=sp.Rational(1, 5))),
    ("beltrami", problems.Beltrami3D(nu=0.01), dict(nu=sp.Rational(1, 100))),
    ("poly2", problems.PolySteady2D(0.3), dict(nu=sp.Rational(3, 10))),
    ("poly3", problems.PolySteady3D(0.3), dict(nu=sp.Rational(3, 10))),
    ("poly2c", problems.PolySteady2DCubic(0.3), dict(nu=sp.Rational(3, 10))),
    ("poly3c", problems.PolySteady3DCubic(0.3), dict(nu=sp.Rational(3, 10))),
    ("steady_paper", problems.SteadyPaper2D(1.0), dict(nu=1)),
    ("steady_paper", problems.SteadyPaper2D(0.05), dict(nu=sp.Rational(1, 20))),
]


@pytest.mark.parametrize("name,pb,kw", CASES)
def test_forcing_is_the_navier_stokes_residual(name, pb, kw):
    u, p, X = sym_fields(name, kw["nu"], kw.get("k"))
    d = len(X)
    nu = kw["nu"]
    res = [sp.diff(u[i], t) - nu * sum(sp.diff(u[i], X[j], 2) for j in range(d))
           + sum(u[j] * sp.diff(u[i], X[j]) for j in range(d)) + sp.diff(p, X[i])
           for i in range(d)]
    div = sum(sp.diff(u[i], X[i]) for i in range(d))
    fres = sp.lambdify((*X, t), res, "numpy")
    fdiv = sp.lambdify((*X, t), div, "numpy")
    fu = sp.lambdify((*X, t), u, "numpy")
    fp = sp.lambdify((*X, t), p, "numpy")
    rng = np.random.default_rng(3)
    pts = rng.random((50, d))
    for tt in (0.0, 0.37, 1.3):
        args = [pts[:, j] for j in range(d)] + [tt]
        ref_f = np.stack([np.broadcast_to(np.asarray(v, float), (50,)) for v in fres(*args)], -1)
        got_f = np.zeros_like(ref_f) if pb.f is None else pb.f(pts, tt)
        scale = max(1.0, np.abs(ref_f).max())
        assert np.abs(got_f - ref_f).max() < 1e-12 * scale
        assert np.abs(np.asarray(fdiv(*args), float)).max() < 1e-12
        ref_u = np.stack([np.broadcast_to(np.asarray(v, float), (50,)) for v in fu(*args)], -1)
        assert np.abs(pb.u(pts, tt) - ref_u).max() < 1e-13 * max(1.0, np.abs(ref_u).max())
        ref_p = np.broadcast_to(np.asarray(fp(*args), float), (50,))
        assert np.abs(pb.p(pts, tt) - ref_p).max() < 1e-13 * max(1.0, np.abs(ref_p).max())


def test_forcing_check_catches_a_planted_sign_error():
    """A John forcing with the convection sign flipped must fail the check."""
    pb = problems.John2D(1.0)
    u, p, X = sym_fields("john", 1)
    res = [sp.diff(u[i], t) - sum(sp.diff(u[i], X[j], 2) for j in range(2))
           - sum(u[j] * sp.diff(u[i], X[j]) for j in range(2)) + sp.diff(p, X[i])
           for i in range(2)]
    f = sp.lambdify((x, y, t), res, "numpy")
    pts = np.random.default_rng(0).random((20, 2))
    ref = np.stack(f(pts[:, 0], pts[:, 1], 0.9), -1)
    assert np.abs(pb.f(pts, 0.9) - ref).max() > 1e-3
