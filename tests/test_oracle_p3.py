"""Pins of the oracle's P3-P2 Taylor-Hood pair (the paper's higher-order
study, table "convergence_p3_p2"), on triangles and, extended to 3D, on
tetrahedra (20 P3 nodes: vertices, two per edge, one per face).

* the P3 basis is nodal at its ten nodes, sums to one, and its gradients match
  central differences;
* the local matrices (mass, stiffness, convection with a P3 velocity, and the
  P2 x P3 divergence/gradient couplings) equal the same integrals done exactly
  on a skewed triangle: every basis function is expanded into barycentric
  monomials with rational coefficients and integrated with
  int_T l0^a l1^b l2^c = 2|T| a! b! c! / (a+b+c+2)! (no quadrature involved);
* the global numbering: the P3 interpolant of a cubic field reproduces it at
  interior quadrature points of every cell (a wrong edge orientation would
  not), and the boundary mask holds exactly the nodes on the boundary;
* one step equals the same step done with dense direct solves;
* a cubic divergence-free velocity with a quadratic pressure is a fixed point
  of the step, explicit and semi-implicit (this holds for any rule of degree
  >= 4; the rule itself is pinned by the exact integrals, which a degree-5
  rule fails);
* convergence orders on Taylor-Green: velocity -> 4, pressure -> 3 on meshes
  n = 4, 8, 16, with a guard that the time error is negligible; the paper's
  P3-P2 table (stored under tests/golden with its citation) shows the same
  orders.
"""
import os
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

from oracle import errors, fem, ipcs, mesh, problems, quadrature

F = Fraction


# ---------------------------------------------------------------- exact polynomials
# a polynomial in (l0, l1, l2) is a dict {(a, b, c): Fraction}
def pmul(p, q):
    out = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = tuple(a + b for a, b in zip(ea, eb))
            out[e] = out.get(e, F(0)) + ca * cb
    return out


def padd(*ps):
    out = {}
    for p in ps:
        for e, c in p.items():
            out[e] = out.get(e, F(0)) + c
    return out


def pscale(p, s):
    return {e: c * s for e, c in p.items()}


def pdiff(p, k):
    out = {}
    for e, c in p.items():
        if e[k] > 0:
            f = list(e)
            f[k] -= 1
            out[tuple(f)] = out.get(tuple(f), F(0)) + c * e[k]
    return out


def L(k, nv=3):
    e = [0] * nv
    e[k] = 1
    return {tuple(e): F(1)}


ONE = {(0, 0, 0): F(1)}


def pint(p, area):
    """Exact integral over a triangle of the given area."""
    s = F(0)
    for (a, b, c), coef in p.items():
        s += coef * F(2 * factorial(a) * factorial(b) * factorial(c), factorial(a + b + c + 2))
    return float(s) * area


def p3_exact():
    """The P3 basis in the oracle's local order, from its definition."""
    out = []
    for i in range(3):
        out.append(pscale(pmul(L(i), pmul(padd(pscale(L(i), 3), pscale(ONE, -1)),
                                          padd(pscale(L(i), 3), pscale(ONE, -2)))), F(1, 2)))
    for a, b in fem.EDGES_2D:
        for p, q in ((a, b), (b, a)):
            out.append(pscale(pmul(pmul(L(p), L(q)), padd(pscale(L(p), 3), pscale(ONE, -1))),
                              F(9, 2)))
    out.append(pscale(pmul(L(0), pmul(L(1), L(2))), 27))
    return out


def p2_exact():
    out = [pmul(L(i), padd(pscale(L(i), 2), pscale(ONE, -1))) for i in range(3)]
    out += [pscale(pmul(L(a), L(b)), 4) for a, b in fem.EDGES_2D]
    return out


NODES3 = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1],
                   [0, 2 / 3, 1 / 3], [0, 1 / 3, 2 / 3],
                   [1 / 3, 0, 2 / 3], [2 / 3, 0, 1 / 3],
                   [2 / 3, 1 / 3, 0], [1 / 3, 2 / 3, 0],
                   [1 / 3, 1 / 3, 1 / 3]])


def test_p3_basis_is_nodal_and_a_partition_of_unity():
    phi, dphi = fem.p3_basis(NODES3)
    np.testing.assert_allclose(phi, np.eye(10), atol=1e-14)
    lam = np.random.default_rng(0).dirichlet(np.ones(3), 40)
    phi, dphi = fem.p3_basis(lam)
    np.testing.assert_allclose(phi.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(dphi.sum(axis=1), 0.0, atol=1e-13)


def test_p3_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    xy = 0.1 + 0.4 * rng.random((30, 2))
    to_lam = lambda p: np.stack([1 - p[:, 0] - p[:, 1], p[:, 0], p[:, 1]], axis=1)
    _, dphi = fem.p3_basis(to_lam(xy))
    h = 1e-6
    for a in range(2):
        e = np.zeros(2)
        e[a] = h
        fd = (fem.p3_basis(to_lam(xy + e))[0] - fem.p3_basis(to_lam(xy - e))[0]) / (2 * h)
        np.testing.assert_allclose(dphi[:, :, a], fd, atol=1e-8)


def _skewed_cell(order=3):
    X = np.array([[0.1, 0.2], [1.3, 0.4], [0.5, 1.7]])
    return fem.Space(X, np.array([[0, 1, 2]]), order=order)


def _exact_grads(S, basis):
    """Physical gradients as polynomial pairs: sum_k d phi / d l_k grad l_k."""
    G = S.Jinv[0].T @ fem.bary_grad(2).T          # (2, 3): column k = grad l_k
    out = []
    for p in basis:
        parts = [pdiff(p, k) for k in range(3)]
        out.append([padd(*[pscale(parts[k], F(G[a, k])) for k in range(3)]) for a in range(2)])
    return out


def test_p3_local_matrices_equal_exact_integrals():
    S = _skewed_cell()
    area = 0.5 * S.absdet[0]
    b3, b2 = p3_exact(), p2_exact()
    g3, g2 = _exact_grads(S, b3), _exact_grads(S, b2)
    M = np.array([[pint(pmul(p, q), area) for q in b3] for p in b3])
    K = np.array([[pint(padd(pmul(gp[0], gq[0]), pmul(gp[1], gq[1])), area) for gq in g3]
                  for gp in g3])
    np.testing.assert_allclose(fem.local_mass_u(S)[0], M, rtol=0, atol=1e-14)
    np.testing.assert_allclose(fem.local_stiff_u(S)[0], K, rtol=0, atol=1e-12)
    Mp = np.array([[pint(pmul(p, q), area) for q in b2] for p in b2])
    Kp = np.array([[pint(padd(pmul(gp[0], gq[0]), pmul(gp[1], gq[1])), area) for gq in g2]
                   for gp in g2])
    np.testing.assert_allclose(fem.local_mass_p(S)[0], Mp, rtol=0, atol=1e-14)
    np.testing.assert_allclose(fem.local_stiff_p(S)[0], Kp, rtol=0, atol=1e-12)
    # D_c (P2 rows, P3 columns) and G_c (P3 rows, P2 columns)
    for c in range(2):
        D = np.array([[pint(pmul(p, gq[c]), area) for gq in g3] for p in b2])
        Gm = np.array([[pint(pmul(p, gq[c]), area) for gq in g2] for p in b3])
        np.testing.assert_allclose(fem.local_div(S, c)[0], D, rtol=0, atol=1e-13)
        np.testing.assert_allclose(fem.local_grad(S, c)[0], Gm, rtol=0, atol=1e-13)
    # convection with a P3 velocity (degree-8 integrand): C_ij = int phi_i u_h . grad phi_j
    rng = np.random.default_rng(2)
    Uc = rng.standard_normal((2, 10))
    uh = [padd(*[pscale(b3[m], F(Uc[a, m])) for m in range(10)]) for a in range(2)]
    C = np.array([[pint(pmul(p, padd(pmul(uh[0], gq[0]), pmul(uh[1], gq[1]))), area)
                   for gq in g3] for p in b3])
    U = np.zeros((2, S.Nu))
    U[:, S.c2du[0]] = Uc
    np.testing.assert_allclose(fem.local_convection(S, U)[0], C, rtol=0, atol=1e-12)


def test_exact_integration_catches_a_planted_basis_error():
    """An edge function with the wrong node (3 l_b - 1 for the node nearer a)
    changes the mass matrix far beyond rounding."""
    S = _skewed_cell()
    area = 0.5 * S.absdet[0]
    b3 = p3_exact()
    a, b = fem.EDGES_2D[0]
    b3[3] = pscale(pmul(pmul(L(a), L(b)), padd(pscale(L(b), 3), pscale(ONE, -1))), F(9, 2))
    M = np.array([[pint(pmul(p, q), area) for q in b3] for p in b3])
    assert np.abs(fem.local_mass_u(S)[0] - M).max() > 1e-3


def test_p3_numbering_interpolates_cubics_and_marks_the_boundary():
    X, cells = mesh.unit_square(4, 3)
    S = fem.Space(X, cells, order=3)
    assert S.Nu == S.Nv + 2 * S.edges.shape[0] + S.Nc and S.Np == S.N2
    u = lambda x: x[..., 0] ** 3 - 2 * x[..., 0] * x[..., 1] ** 2 + x[..., 1] ** 3 + 0.5 * x[..., 1]
    Uh = u(S.xu)
    lam = np.random.default_rng(4).dirichlet(np.ones(3), 6)
    phi, _ = fem.p3_basis(lam)
    xq = S.map_points(lam)                                   # (Nc, nq, 2)
    np.testing.assert_allclose(np.einsum('qm,cm->cq', phi, Uh[S.c2du]), u(xq), atol=1e-13)
    on = (np.abs(S.xu[:, 0]) < 1e-12) | (np.abs(S.xu[:, 0] - 1) < 1e-12) | \
         (np.abs(S.xu[:, 1]) < 1e-12) | (np.abs(S.xu[:, 1] - 1) < 1e-12)
    np.testing.assert_array_equal(S.bmask_u, on)
    # every node is referenced, and exactly one cell owns each centroid
    assert np.unique(S.c2du).size == S.Nu


def test_p3_step_equals_dense_direct_solves():
    S = fem.Space(*mesh.unit_square(3, 3), order=3)
    pb = problems.TaylorGreen2D(np.pi, 0.05)
    dt, nu = 0.02, 0.05
    st = ipcs.IPCS(S, pb, ipcs.Params(nu=nu, dt=dt, tol_mom=1e-14, tol_p=1e-14, tol_corr=1e-14))
    U, P, t = st.U.copy(), st.P.copy(), st.t + dt
    st.step()
    d, B = 2, S.bmask_u
    g = pb.u(S.xu, t).T
    C = fem.convection(S, U)
    A = (st.M / dt + nu * st.K).tocsr()
    Us = np.zeros_like(U)
    for c in range(d):
        b = st.M @ U[c] / dt - C @ U[c] - st.G[c] @ P
        Us[c] = np.linalg.solve(fem.eliminate(A, B).toarray(), fem.lift(A, b, B, g[c]))
    r = -(1 / dt) * sum(st.D[c] @ Us[c] for c in range(d))
    n = S.Np
    Bd = np.zeros((n + 1, n + 1))
    Bd[:n, :n], Bd[:n, n], Bd[n, :n] = st.Kp.toarray(), st.w, st.w
    dP = np.linalg.solve(Bd, np.r_[r - r.mean(), 0.0])[:n]
    Un = np.zeros_like(U)
    for c in range(d):
        b = st.M @ Us[c] - dt * (st.G[c] @ dP)
        Un[c] = np.linalg.solve(fem.eliminate(st.M, B).toarray(), fem.lift(st.M, b, B, g[c]))
    assert np.linalg.norm(st.U - Un) <= 1e-11 * np.linalg.norm(Un)
    assert np.linalg.norm(st.P - (P + dP)) <= 1e-11 * np.linalg.norm(P + dP)


@pytest.mark.parametrize("semi", [False, True])
def test_p3_p2_cubic_steady_state_is_a_fixed_point(semi):
    S = fem.Space(*mesh.unit_square(4, 3), order=3)
    pb = problems.PolySteady2DCubic(0.07)
    st = ipcs.IPCS(S, pb, ipcs.Params(nu=pb.nu, dt=0.05, semi_implicit=semi,
                                      tol_mom=1e-14, tol_p=1e-14, tol_corr=1e-14))
    U0, P0 = st.U.copy(), st.P.copy()
    np.testing.assert_allclose(P0, pb.p(S.xp, 0.0), atol=1e-14)   # zero mean already
    for _ in range(2):
        st.step()
    assert np.abs(st.U - U0).max() < 1e-12
    assert np.abs(st.P - P0).max() < 1e-11


def test_exact_integrals_catch_a_too_low_rule():
    """The degree-5 rule of the P2-P1 pair is not exact for P3 mass (degree 6)
    or convection (degree 8): the exact-integral comparison rejects it. (The
    cubic fixed point does not: forcing, convection and pressure terms meet at
    the same quadrature points, and nu K needs only degree 4.)"""
    S = _skewed_cell()
    rule = fem._rule
    try:
        fem._rule = lambda space: quadrature.cell_rule(space.dim)
        M5 = fem.local_mass_u(S)[0]
        U = np.zeros((2, S.Nu))
        U[:, S.c2du[0]] = np.random.default_rng(2).standard_normal((2, 10))
        C5 = fem.local_convection(S, U)[0]
    finally:
        fem._rule = rule
    assert np.abs(M5 - fem.local_mass_u(S)[0]).max() > 1e-6
    assert np.abs(C5 - fem.local_convection(S, U)[0]).max() > 1e-6


def _tg_errors(n, dt, T=1e-4):
    pb = problems.TaylorGreen2D(np.pi, 0.01)
    S = fem.Space(*mesh.unit_square(n, n), order=3)
    st = ipcs.IPCS(S, pb, ipcs.Params(nu=0.01, dt=dt))
    st.run(int(round(T / dt)))
    return (errors.l2_velocity(S, st.U, pb.u, st.t), errors.l2_pressure(S, st.P, pb.p, st.t))


def test_p3_p2_taylor_green_convergence_orders():
    """Ten steps of dt = 1e-5 from the interpolated exact state: on these
    meshes the spatial error dominates (halving dt moves the n = 16 errors by
    < 2 %); at n = 32 an error that grows with simulated time reaches the
    spatial error's size in this short run and the observed velocity order
    falls towards 3, so the pin stops at n = 16."""
    e = {n: _tg_errors(n, 1e-5) for n in (4, 8, 16)}
    eh = _tg_errors(16, 5e-6)
    assert abs(eh[0] / e[16][0] - 1) < 0.02 and abs(eh[1] / e[16][1] - 1) < 0.02
    ou = np.log2(e[8][0] / e[16][0])
    op = np.log2(e[8][1] / e[16][1])
    assert abs(ou - 4.0) <= 0.2, ou
    assert abs(op - 3.0) <= 0.15, op
    assert np.log2(e[4][0] / e[8][0]) > 3.8 and np.log2(e[4][1] / e[8][1]) > 2.8


# ---------------------------------------------------------------- tetrahedra
ONE4 = {(0, 0, 0, 0): F(1)}


def pint_tet(p, vol):
    """Exact integral over a tetrahedron of the given volume:
    int l^alpha = 6 |T| alpha! / (|alpha| + 3)!."""
    s = F(0)
    for e, coef in p.items():
        num = 6
        for a in e:
            num *= factorial(a)
        s += coef * F(num, factorial(sum(e) + 3))
    return float(s) * vol


def p3_tet_exact():
    """The 3D P3 basis in the oracle's local order, from its definition."""
    Lt = lambda k: L(k, 4)
    out = []
    for i in range(4):
        out.append(pscale(pmul(Lt(i), pmul(padd(pscale(Lt(i), 3), pscale(ONE4, -1)),
                                           padd(pscale(Lt(i), 3), pscale(ONE4, -2)))), F(1, 2)))
    for a, b in fem.EDGES_3D:
        for p, q in ((a, b), (b, a)):
            out.append(pscale(pmul(pmul(Lt(p), Lt(q)), padd(pscale(Lt(p), 3), pscale(ONE4, -1))),
                              F(9, 2)))
    for a, b, c in fem.FACES_3D:
        out.append(pscale(pmul(Lt(a), pmul(Lt(b), Lt(c))), 27))
    return out


def p2_tet_exact():
    Lt = lambda k: L(k, 4)
    out = [pmul(Lt(i), padd(pscale(Lt(i), 2), pscale(ONE4, -1))) for i in range(4)]
    out += [pscale(pmul(Lt(a), Lt(b)), 4) for a, b in fem.EDGES_3D]
    return out


def _nodes_tet():
    lam = [np.eye(4)[i] for i in range(4)]
    for a, b in fem.EDGES_3D:
        for p, q in ((a, b), (b, a)):
            v = np.zeros(4)
            v[p], v[q] = 2 / 3, 1 / 3
            lam.append(v)
    for f in fem.FACES_3D:
        v = np.zeros(4)
        v[list(f)] = 1 / 3
        lam.append(v)
    return np.array(lam)


def test_p3_tet_basis_is_nodal_partition_of_unity_with_matching_gradients():
    phi, _ = fem.p3_basis(_nodes_tet())
    np.testing.assert_allclose(phi, np.eye(20), atol=1e-14)
    rng = np.random.default_rng(0)
    lam = rng.dirichlet(np.ones(4), 40)
    phi, dphi = fem.p3_basis(lam)
    np.testing.assert_allclose(phi.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(dphi.sum(axis=1), 0.0, atol=1e-13)
    xyz = 0.05 + 0.25 * rng.random((30, 3))
    to_lam = lambda p: np.concatenate([1 - p.sum(axis=1, keepdims=True), p], axis=1)
    _, dphi = fem.p3_basis(to_lam(xyz))
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (fem.p3_basis(to_lam(xyz + e))[0] - fem.p3_basis(to_lam(xyz - e))[0]) / (2 * h)
        np.testing.assert_allclose(dphi[:, :, a], fd, atol=1e-8)


def test_p3_tet_local_matrices_equal_exact_integrals():
    X = np.array([[0.1, 0.2, 0.0], [1.3, 0.4, 0.1], [0.5, 1.7, 0.3], [0.2, 0.4, 1.1]])
    S = fem.Space(X, np.array([[0, 1, 2, 3]]), order=3)
    vol = S.absdet[0] / 6.0
    b3, b2 = p3_tet_exact(), p2_tet_exact()

    def grads(basis):
        G = S.Jinv[0].T @ fem.bary_grad(3).T          # (3, 4): column k = grad l_k
        out = []
        for p in basis:
            parts = [pdiff(p, k) for k in range(4)]
            out.append([padd(*[pscale(parts[k], F(G[a, k])) for k in range(4)])
                        for a in range(3)])
        return out

    g3, g2 = grads(b3), grads(b2)
    dot = lambda u, v: padd(*[pmul(u[a], v[a]) for a in range(3)])
    M = np.array([[pint_tet(pmul(p, q), vol) for q in b3] for p in b3])
    K = np.array([[pint_tet(dot(gp, gq), vol) for gq in g3] for gp in g3])
    np.testing.assert_allclose(fem.local_mass_u(S)[0], M, rtol=0, atol=1e-14)
    np.testing.assert_allclose(fem.local_stiff_u(S)[0], K, rtol=0, atol=1e-12)
    Kp = np.array([[pint_tet(dot(gp, gq), vol) for gq in g2] for gp in g2])
    np.testing.assert_allclose(fem.local_stiff_p(S)[0], Kp, rtol=0, atol=1e-12)
    for c in range(3):
        D = np.array([[pint_tet(pmul(p, gq[c]), vol) for gq in g3] for p in b2])
        np.testing.assert_allclose(fem.local_div(S, c)[0], D, rtol=0, atol=1e-13)
    rng = np.random.default_rng(2)
    Uc = rng.standard_normal((3, 20))
    uh = [padd(*[pscale(b3[m], F(Uc[a, m])) for m in range(20)]) for a in range(3)]
    C = np.array([[pint_tet(pmul(p, dot(uh, gq)), vol) for gq in g3] for p in b3])
    U = np.zeros((3, S.Nu))
    U[:, S.c2du[0]] = Uc
    np.testing.assert_allclose(fem.local_convection(S, U)[0], C, rtol=0, atol=1e-12)


def test_p3_tet_numbering_interpolates_cubics_and_marks_the_boundary():
    S = fem.Space(*mesh.unit_cube(2, 2, 1), order=3)
    assert S.Nu == S.Nv + 2 * S.edges.shape[0] + S.faces.shape[0] and S.Np == S.N2
    u = lambda x: (x[..., 0] ** 3 - 2 * x[..., 0] * x[..., 1] * x[..., 2] + x[..., 2] ** 3
                   + 0.5 * x[..., 1] ** 2)
    Uh = u(S.xu)
    lam = np.random.default_rng(4).dirichlet(np.ones(4), 6)
    phi, _ = fem.p3_basis(lam)
    np.testing.assert_allclose(np.einsum('qm,cm->cq', phi, Uh[S.c2du]), u(S.map_points(lam)),
                               atol=1e-13)
    on = np.any((np.abs(S.xu) < 1e-12) | (np.abs(S.xu - 1) < 1e-12), axis=1)
    np.testing.assert_array_equal(S.bmask_u, on)
    assert np.unique(S.c2du).size == S.Nu


def test_p3_tet_step_equals_dense_direct_solves():
    """One 64-node cube (192 velocity and 27 pressure unknowns)."""
    S = fem.Space(*mesh.unit_cube(1, 1, 1), order=3)
    pb = problems.Beltrami3D(nu=0.05)
    dt, nu = 0.02, 0.05
    st = ipcs.IPCS(S, pb, ipcs.Params(nu=nu, dt=dt, tol_mom=1e-14, tol_p=1e-14, tol_corr=1e-14))
    U, P, t = st.U.copy(), st.P.copy(), st.t + dt
    st.step()
    d, B = 3, S.bmask_u
    g = pb.u(S.xu, t).T
    C = fem.convection(S, U)
    A = (st.M / dt + nu * st.K).tocsr()
    Us = np.zeros_like(U)
    for c in range(d):
        b = st.M @ U[c] / dt - C @ U[c] - st.G[c] @ P
        Us[c] = np.linalg.solve(fem.eliminate(A, B).toarray(), fem.lift(A, b, B, g[c]))
    r = -(1 / dt) * sum(st.D[c] @ Us[c] for c in range(d))
    n = S.Np
    Bd = np.zeros((n + 1, n + 1))
    Bd[:n, :n], Bd[:n, n], Bd[n, :n] = st.Kp.toarray(), st.w, st.w
    dP = np.linalg.solve(Bd, np.r_[r - r.mean(), 0.0])[:n]
    Un = np.zeros_like(U)
    for c in range(d):
        b = st.M @ Us[c] - dt * (st.G[c] @ dP)
        Un[c] = np.linalg.solve(fem.eliminate(st.M, B).toarray(), fem.lift(st.M, b, B, g[c]))
    assert np.linalg.norm(st.U - Un) <= 1e-11 * np.linalg.norm(Un)
    assert np.linalg.norm(st.P - (P + dP)) <= 1e-11 * np.linalg.norm(P + dP)


@pytest.mark.parametrize("semi", [False, True])
def test_p3_p2_tet_cubic_steady_state_is_a_fixed_point(semi):
    S = fem.Space(*mesh.unit_cube(2, 2, 2), order=3)
    pb = problems.PolySteady3DCubic(0.07)
    st = ipcs.IPCS(S, pb, ipcs.Params(nu=pb.nu, dt=0.05, semi_implicit=semi,
                                      tol_mom=1e-14, tol_p=1e-14, tol_corr=1e-14))
    U0, P0 = st.U.copy(), st.P.copy()
    np.testing.assert_allclose(P0, pb.p(S.xp, 0.0), atol=1e-14)   # zero mean already
    for _ in range(2):
        st.step()
    assert np.abs(st.U - U0).max() < 1e-12
    assert np.abs(st.P - P0).max() < 1e-11


def _beltrami_p3_errors(n, dt, T=1e-4):
    pb = problems.Beltrami3D(nu=0.01)
    S = fem.Space(*mesh.unit_cube(n, n, n), order=3)
    st = ipcs.IPCS(S, pb, ipcs.Params(nu=0.01, dt=dt))
    st.run(int(round(T / dt)))
    return (errors.l2_velocity(S, st.U, pb.u, st.t), errors.l2_pressure(S, st.P, pb.p, st.t))


@pytest.mark.slow
def test_p3_p2_tet_beltrami_convergence_orders():
    """Ten steps of dt = 1e-5 on n = 2, 4, 8 cubes (halving dt moves the
    n = 8 errors by < 3 %): velocity order 4.0 then 3.65, pressure 3.0 on the
    finest pair (measured), against the theoretical 4 and 3 of the pair."""
    e = {n: _beltrami_p3_errors(n, 1e-5) for n in (2, 4, 8)}
    eh = _beltrami_p3_errors(8, 5e-6)
    assert abs(eh[0] / e[8][0] - 1) < 0.03 and abs(eh[1] / e[8][1] - 1) < 0.03
    assert abs(np.log2(e[2][0] / e[4][0]) - 4.0) <= 0.2
    assert np.log2(e[4][0] / e[8][0]) >= 3.5
    assert abs(np.log2(e[4][1] / e[8][1]) - 3.0) <= 0.2


def test_golden_p3_p2_table_orders():
    """The paper's own P3-P2 table: its orders approach 4 and 3."""
    rows = [list(map(float, l.split())) for l in
            open(os.path.join(os.path.dirname(__file__), "golden", "convergence_p3_p2.txt"))
            if l.strip() and not l.startswith("#")]
    eu = [r[1] for r in rows]
    ep = [r[2] for r in rows]
    assert abs(np.log2(eu[-2] / eu[-1]) - 4) < 0.05
    assert abs(np.log2(ep[-2] / ep[-1]) - 3) < 0.15
