"""Pins of the oracle's spaces, local matrices and assembly.

* Local matrices: compared with exact integrals computed independently of any
  quadrature, by expanding the basis polynomials in barycentric coordinates
  with rational coefficients and integrating monomials with the closed form
  int_K lam^alpha = d! alpha! / (|alpha|+d)! |K|.
* Global invariants: sum M = |Omega|, zero row sums, integration-by-parts
  identities, G_c = -D_c^T on interior rows, DOF counts printed in the paper,
  nnz counted by brute force and by closed forms from the mesh topology.
"""
import itertools
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

from oracle import fem, mesh

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


# --------------------------------------------------------------- exact algebra
def pmul(p, q):
    out = {}
    for a, ca in p.items():
        for b, cb in q.items():
            k = tuple(x + y for x, y in zip(a, b))
            out[k] = out.get(k, 0) + ca * cb
    return out


def padd(*ps):
    out = {}
    for p in ps:
        for k, c in p.items():
            out[k] = out.get(k, 0) + c
    return out


def pscale(p, s):
    return {k: c * s for k, c in p.items()}


def pderiv(p, k):
    out = {}
    for a, c in p.items():
        if a[k] > 0:
            b = list(a)
            b[k] -= 1
            out[tuple(b)] = out.get(tuple(b), 0) + c * a[k]
    return out


def pint(p, dim):
    """Integral over the reference simplex (measure 1/d!)."""
    s = Fraction(0)
    for a, c in p.items():
        num = 1
        for x in a:
            num *= factorial(x)
        s += c * Fraction(num, factorial(sum(a) + dim))
    return s


def lam(k, dim):
    e = [0] * (dim + 1)
    e[k] = 1
    return {tuple(e): Fraction(1)}


def exact_basis(dim):
    L = [lam(k, dim) for k in range(dim + 1)]
    p1 = L
    p2 = [padd(pscale(pmul(L[i], L[i]), 2), pscale(L[i], -1)) for i in range(dim + 1)]
    edges = [(1, 2), (2, 0), (0, 1)] if dim == 2 else \
        [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    p2 += [pscale(pmul(L[a], L[b]), 4) for a, b in edges]
    return p1, p2


def grad_lambda(Xc):
    """Physical gradients of the barycentric coordinates of cell Xc (d+1, d)."""
    d = Xc.shape[1]
    J = (Xc[1:] - Xc[0]).T
    Jinv = np.linalg.inv(J)
    g = np.zeros((d + 1, d))
    g[1:] = Jinv
    g[0] = -Jinv.sum(axis=0)
    return g, abs(np.linalg.det(J))


def exact_local(Xc, U=None):
    """Exact M2, K2, M1, K1, D_c, G_c, C(U) on cell Xc (float from rationals)."""
    d = Xc.shape[1]
    p1, p2 = exact_basis(d)
    gl, det = grad_lambda(Xc)
    n2, n1 = len(p2), len(p1)
    I = lambda p: float(pint(p, d)) * det
    M2 = np.array([[I(pmul(a, b)) for b in p2] for a in p2])
    M1 = np.array([[I(pmul(a, b)) for b in p1] for a in p1])
    dp2 = [[pderiv(a, k) for k in range(d + 1)] for a in p2]
    dp1 = [[pderiv(a, k) for k in range(d + 1)] for a in p1]
    GG = gl @ gl.T

    def stiff(dp):
        n = len(dp)
        K = np.zeros((n, n))
        for i in range(n):
            for j in range(n):
                K[i, j] = sum(GG[k, l] * I(pmul(dp[i][k], dp[j][l]))
                              for k in range(d + 1) for l in range(d + 1))
        return K

    K2, K1 = stiff(dp2), stiff(dp1)
    D = np.zeros((d, n1, n2))
    G = np.zeros((d, n2, n1))
    for c in range(d):
        for k in range(n1):
            for j in range(n2):
                D[c, k, j] = sum(gl[l, c] * I(pmul(p1[k], dp2[j][l])) for l in range(d + 1))
        for i in range(n2):
            for k in range(n1):
                G[c, i, k] = sum(gl[l, c] * I(pmul(p2[i], dp1[k][l])) for l in range(d + 1))
    C = None
    if U is not None:           # U (d, n2) local nodal velocity
        C = np.zeros((n2, n2))
        for i in range(n2):
            for j in range(n2):
                s = 0.0
                for m in range(n2):
                    for l in range(d + 1):
                        s += float(U[:, m] @ gl[l]) * I(pmul(pmul(p2[i], p2[m]), dp2[j][l]))
                C[i, j] = s
    return M2, K2, M1, K1, D, G, C


# --------------------------------------------------------------- tests
def test_reference_triangle_p2_matrices_closed_form():
    """Classical P2 mass/stiffness on the reference triangle (area 1/2)."""
    Xc = np.array([[0., 0.], [1., 0.], [0., 1.]])
    S = fem.Space(Xc, np.array([[0, 1, 2]]))
    Mref = np.array([[6, -1, -1, -4, 0, 0], [-1, 6, -1, 0, -4, 0], [-1, -1, 6, 0, 0, -4],
                     [-4, 0, 0, 32, 16, 16], [0, -4, 0, 16, 32, 16], [0, 0, -4, 16, 16, 32]]
                    ) * 0.5 / 180.0
    Kref = np.array([[6, 1, 1, 0, -4, -4], [1, 3, 0, 0, 0, -4], [1, 0, 3, 0, -4, 0],
                     [0, 0, 0, 16, -8, -8], [-4, 0, -4, -8, 16, 0], [-4, -4, 0, -8, 0, 16]]
                    ) / 6.0
    np.testing.assert_allclose(fem.local_mass_p2(S)[0], Mref, atol=2e-16)
    np.testing.assert_allclose(fem.local_stiff_p2(S)[0], Kref, atol=1e-15)
    M2, K2, M1, K1, *_ = exact_local(Xc)
    np.testing.assert_allclose(M2, Mref, atol=1e-17)
    np.testing.assert_allclose(K2, Kref, atol=1e-15)
    np.testing.assert_allclose(M1, np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]]) * 0.5 / 12,
                               atol=1e-17)
    np.testing.assert_allclose(K1, 0.5 * np.array([[2, -1, -1], [-1, 1, 0], [-1, 0, 1]]),
                               atol=1e-16)


@pytest.mark.parametrize("dim", [2, 3])
def test_local_matrices_match_exact_integrals_on_a_skewed_cell(dim):
    rng = np.random.default_rng(7 + dim)
    Xc = np.eye(dim + 1, dim, -1) + 0.2 * rng.standard_normal((dim + 1, dim))
    cells = np.arange(dim + 1)[None, :]
    S = fem.Space(Xc, cells)
    U = rng.standard_normal((dim, S.N2))
    Uloc = U[:, S.c2d2[0]]
    M2, K2, M1, K1, D, G, C = exact_local(Xc, Uloc)
    sc = lambda A: np.abs(A).max()
    for got, ref in [(fem.local_mass_p2(S)[0], M2), (fem.local_stiff_p2(S)[0], K2),
                     (fem.local_mass_p1(S)[0], M1), (fem.local_stiff_p1(S)[0], K1),
                     (fem.local_convection(S, U)[0], C)]:
        assert np.abs(got - ref).max() <= 1e-13 * sc(ref)
    for c in range(dim):
        assert np.abs(fem.local_div(S, c)[0] - D[c]).max() <= 1e-13 * sc(D[c])
        assert np.abs(fem.local_grad(S, c)[0] - G[c]).max() <= 1e-13 * sc(G[c])


def test_dof_counts_match_paper_table():
    rows = [list(map(int, l.split())) for l in open(f"{GOLDEN}/convergence_data_dofs.txt")
            if l.strip() and not l.startswith("#")]
    for n, udofs, pdofs in rows:
        S = fem.Space(*mesh.unit_square(n, n))
        assert 2 * S.N2 == udofs and S.N1 == pdofs


def brute_pattern(rows_map, cols_map):
    s = set()
    for r, c in zip(rows_map, cols_map):
        for i in r:
            for j in c:
                s.add((int(i), int(j)))
    return s


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_2d_sizes_closed_forms_and_brute_force(n):
    S = fem.Space(*mesh.unit_square(n, n))
    # interior edges = 3n^2 + 2n - 4n; P2 pairs sharing a cell = 15 T - 3 E_int
    assert S.Nc == 2 * n * n and S.N1 == (n + 1) ** 2 and S.N2 == (2 * n + 1) ** 2
    M, Mp, D, G = fem.mass_p2(S), fem.mass_p1(S), fem.divergence(S, 0), fem.gradient(S, 1)
    assert M.nnz == 46 * n * n + 16 * n + 1 == len(brute_pattern(S.c2d2, S.c2d2))
    assert Mp.nnz == 7 * n * n + 6 * n + 1 == len(brute_pattern(S.c2d1, S.c2d1))
    assert D.nnz == G.nnz == 19 * n * n + 10 * n + 1 == len(brute_pattern(S.c2d1, S.c2d2))
    assert S.boundary2.sum() == 8 * n
    # CSR pattern equals the brute-force pattern exactly
    rows = np.repeat(np.arange(S.N2), np.diff(M.indptr))
    assert set(zip(rows.tolist(), M.indices.tolist())) == brute_pattern(S.c2d2, S.c2d2)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_3d_sizes_closed_forms_and_brute_force(n):
    S = fem.Space(*mesh.unit_cube(n, n, n))
    V = (n + 1) ** 3
    E = 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3
    T = 6 * n ** 3
    F = 1 - V + E + T
    assert S.Nc == T and S.N2 == (2 * n + 1) ** 3 == V + E
    M, Mp, D = fem.mass_p2(S), fem.mass_p1(S), fem.divergence(S, 2)
    # pairs sharing an edge: 3 per edge; a face but no edge: 6 per face; else 3 per tet
    assert M.nnz == S.N2 + 2 * (3 * E + 6 * F + 3 * T) == len(brute_pattern(S.c2d2, S.c2d2))
    assert Mp.nnz == V + 2 * E == len(brute_pattern(S.c2d1, S.c2d1))
    assert D.nnz == len(brute_pattern(S.c2d1, S.c2d2)) == V + 4 * E + 6 * T + 18 * n * n
    assert S.boundary2.sum() == (2 * n + 1) ** 3 - (2 * n - 1) ** 3
    assert np.all(S.detJ > 0)


@pytest.mark.parametrize("dim,n", [(2, 4), (2, 7), (3, 2)])
def test_global_invariants(dim, n):
    S = fem.Space(*(mesh.unit_square(n, n) if dim == 2 else mesh.unit_cube(n, n, n)))
    M, K, Mp, Kp = fem.mass_p2(S), fem.stiff_p2(S), fem.mass_p1(S), fem.stiff_p1(S)
    assert abs(M.sum() - 1.0) < 1e-14 and abs(Mp.sum() - 1.0) < 1e-14
    scale = lambda A: np.abs(A.data).max()
    for A in (K, Kp):
        assert np.abs(A.sum(axis=1)).max() < 1e-13 * scale(A)
        assert abs(A - A.T).max() < 1e-14 * scale(A)
    rng = np.random.default_rng(0)
    U = rng.standard_normal((dim, S.N2))
    C = fem.convection(S, U)
    assert np.abs(C.sum(axis=1)).max() < 1e-13 * scale(C)
    interior = ~S.boundary2
    # C(const u) is skew-symmetric on the interior block
    Cc = fem.convection(S, np.ones((dim, S.N2)) * np.arange(1, dim + 1)[:, None]).toarray()
    Ci = Cc[np.ix_(interior, interior)]
    assert np.abs(Ci + Ci.T).max() < 1e-13 * np.abs(Ci).max()
    # K I_h(x^2) = -2 M 1 on interior rows (x^2 is in P2)
    x2 = S.x2[:, 0] ** 2
    r = K @ x2 + 2.0 * (M @ np.ones(S.N2))
    assert np.abs(r[interior]).max() < 1e-12
    for c in range(dim):
        D, G = fem.divergence(S, c), fem.gradient(S, c)
        assert np.abs(D.sum(axis=1)).max() < 1e-13 * scale(D)
        assert np.abs(G.sum(axis=1)).max() < 1e-13 * scale(G)
        diff = (G + D.T).toarray()[interior]
        assert np.abs(diff).max() < 1e-14 * scale(G)
    # D I_h(u) = 0 for a quadratic divergence-free u
    if dim == 2:
        u = np.stack([S.x2[:, 1] ** 2 + S.x2[:, 0], S.x2[:, 0] ** 2 - S.x2[:, 1]])
    else:
        X = S.x2
        u = np.stack([X[:, 1] ** 2 + X[:, 2], X[:, 2] ** 2 + X[:, 0], X[:, 0] * X[:, 1]])
    div = sum(fem.divergence(S, c) @ u[c] for c in range(dim))
    assert np.abs(div).max() < 1e-14


def test_dirichlet_elimination_equals_reduced_system():
    S = fem.Space(*mesh.unit_square(3, 3))
    A = (fem.mass_p2(S) + 0.3 * fem.stiff_p2(S)).tocsr()
    rng = np.random.default_rng(1)
    b = rng.standard_normal(S.N2)
    g = rng.standard_normal(S.N2)
    B = S.boundary2
    I = ~B
    Ae = fem.eliminate(A, B)
    assert Ae.nnz == A.nnz
    x = np.linalg.solve(Ae.toarray(), fem.lift(A, b, B, g))
    Ad = A.toarray()
    xi = np.linalg.solve(Ad[np.ix_(I, I)], b[I] - Ad[np.ix_(I, B)] @ g[B])
    np.testing.assert_allclose(x[I], xi, rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(x[B], g[B])
    assert np.abs(Ae - Ae.T).max() <= 1e-15 * np.abs(Ae.data).max()
