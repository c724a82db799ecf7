"""Pins of the oracle's steady Navier-Stokes solver (Newton's method with
P2-P1, Section 2.2.1 Newton linearization; Section 4.2 example):

* the Newton matrix is the derivative of the discrete residual (central
  finite differences along random directions);
* Newton converges quadratically from the paper's start;
* the polynomial steady state u = (y^2, x^2), p = x + y - 1 (every integrand
  of degree <= 5) is reproduced exactly, in 2D and 3D;
* iterates equal those of dense direct solves of the bordered system on a
  mesh with fewer than 200 unknowns;
* the Section 4.2 example: DOF counts of the paper's table "convergence_data",
  pressure errors equal to the printed ones (nu = 1), orders u -> 3, p -> 2.
"""
import os

import numpy as np
import pytest

from oracle import errors, fem, mesh, problems, steady

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "convergence_data.txt")


def table():
    return [list(map(float, l.split())) for l in open(GOLDEN)
            if l.strip() and not l.startswith("#")]


def flat(o):
    return np.concatenate([o.U.ravel(), o.P])


def test_jacobian_is_the_derivative_of_the_residual():
    S = fem.Space(*mesh.unit_square(3, 3))
    o = steady.SteadyNewton(S, problems.SteadyPaper2D(0.2), 0.2)
    rng = np.random.default_rng(5)
    inner = ~S.bmask_u
    o.U[:, inner] += rng.standard_normal((2, int(inner.sum())))
    o.P = rng.standard_normal(S.Np)
    J = o.jacobian()
    x0 = flat(o).copy()
    for _ in range(3):
        v = np.concatenate([np.where(inner, rng.standard_normal(S.Nu), 0.0) for _ in range(2)]
                           + [rng.standard_normal(S.Np)])
        h = 1e-5
        R = []
        for sgn in (1, -1):
            x = x0 + sgn * h * v
            o.U, o.P = x[:2 * S.Nu].reshape(2, S.Nu), x[2 * S.Nu:]
            Ru, Rp = o.residual()
            R.append(np.concatenate([Ru.ravel(), Rp]))
        dR = (R[0] - R[1]) / (2 * h)
        assert np.linalg.norm(dR + J @ v) <= 1e-7 * np.linalg.norm(J @ v)


def test_newton_converges_quadratically():
    S = fem.Space(*mesh.unit_square(8, 8))
    o = steady.SteadyNewton(S, problems.SteadyPaper2D(1.0), 1.0, tol=1e-14, maxit=6)
    o.run()
    h = o.history
    assert h[-1] < 1e-13
    # e_{k+1} <= C e_k^2 once in the basin (C measured ~1e-4 here)
    for a, b in zip(h[1:], h[2:]):
        if b > 1e-15:
            assert b <= 10.0 * a * a, h


@pytest.mark.parametrize("dim", [2, 3])
def test_polynomial_steady_state_is_reproduced(dim):
    if dim == 2:
        S, pb = fem.Space(*mesh.unit_square(5, 4)), problems.PolySteady2D(0.3)
    else:
        S, pb = fem.Space(*mesh.unit_cube(2, 2, 2)), problems.PolySteady3D(0.3)
    o = steady.SteadyNewton(S, pb, 0.3)
    U, P = o.run()
    np.testing.assert_allclose(U, pb.u(S.xu, 0.0).T, atol=1e-12)
    np.testing.assert_allclose(P, pb.p(S.xp, 0.0), atol=1e-11)
    assert len(o.history) <= 5


def test_iterates_equal_dense_direct_solves():
    """n = 2: 2 * 25 + 9 = 59 unknowns; every Newton step repeated with
    numpy.linalg.solve on the dense bordered matrix."""
    S = fem.Space(*mesh.unit_square(2, 2))
    nu = 0.5
    a = steady.SteadyNewton(S, problems.SteadyPaper2D(nu), nu, maxit=4)
    b = steady.SteadyNewton(S, problems.SteadyPaper2D(nu), nu, maxit=4)
    n = 2 * S.Nu + S.Np
    for _ in range(4):
        a.step()
        Ru, Rp = b.residual()
        J = b.jacobian().toarray()
        wb = np.concatenate([np.zeros(2 * S.Nu), b.w])
        B = np.zeros((n + 1, n + 1))
        B[:n, :n], B[:n, n], B[n, :n] = J, wb, wb
        x = np.linalg.solve(B, np.concatenate([Ru.ravel(), Rp, [0.0]]))[:n]
        b.U = b.U + x[:2 * S.Nu].reshape(2, S.Nu)
        b.P = b.P + x[2 * S.Nu:]
        assert np.linalg.norm(flat(a) - flat(b)) <= 1e-12 * np.linalg.norm(flat(b))


def test_paper_example_dofs_errors_and_orders():
    """Section 4.2, table "convergence_data". u_Dofs = 2 N2 and p_Dofs = N1
    as printed. The printed pressure errors are reproduced with nu = 1 (to
    0.4% at n = 4, 0.02% from n = 16). The printed velocity errors are not:
    ours are within 20% of them (0.90, 1.04, 1.14, 1.18 times), but their
    early orders (3.19, 3.15) exceed ours (3.0), so the paper's velocity norm
    is read as a different measurement and only its order is compared."""
    rows = table()
    eu, ep = {}, {}
    for n, udofs, tu, pdofs, tp in rows[:4]:
        n = int(n)
        S = fem.Space(*mesh.unit_square(n, n))
        assert (2 * S.Nu, S.Np) == (int(udofs), int(pdofs))
        pb = problems.SteadyPaper2D(1.0)
        o = steady.SteadyNewton(S, pb, 1.0)
        U, P = o.run()
        assert o.history[-1] <= 1e-10 and len(o.history) <= 10
        eu[n] = errors.l2_velocity(S, U, lambda x, t: pb.u(x), 0.0)
        ep[n] = errors.l2_pressure(S, P, lambda x, t: pb.p(x), 0.0)
        assert abs(ep[n] / tp - 1) <= (5e-3 if n == 4 else 1e-3 if n == 8 else 2e-4), (n, ep[n], tp)
        assert abs(eu[n] / tu - 1) <= 0.2, (n, eu[n], tu)
    assert abs(np.log2(eu[16] / eu[32]) - 3.0) <= 0.1
    assert abs(np.log2(ep[16] / ep[32]) - 2.0) <= 0.05
    assert abs(np.log2(eu[8] / eu[16]) - 3.0) <= 0.15
