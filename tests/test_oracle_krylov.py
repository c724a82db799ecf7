"""Pins of the oracle's Krylov solvers against dense direct solves
(numpy.linalg.solve) on small meshes: 2D n <= 4 (187 DOFs) and 3D n = 1."""
import numpy as np
import pytest

from oracle import fem, krylov, mesh


def spaces():
    yield fem.Space(*mesh.unit_square(4, 4))
    yield fem.Space(*mesh.unit_square(3, 2))
    yield fem.Space(*mesh.unit_cube(1, 1, 1))


@pytest.mark.parametrize("S", list(spaces()))
def test_pcg_and_bicgstab_match_dense_solve(S):
    rng = np.random.default_rng(5)
    M, K = fem.mass_p2(S), fem.stiff_p2(S)
    B = S.boundary2
    for A in (M, (M / 1e-3 + 0.05 * K).tocsr()):
        Ae = fem.eliminate(A, B)
        b = fem.lift(A, rng.standard_normal(S.N2), B, rng.standard_normal(S.N2))
        ref = np.linalg.solve(Ae.toarray(), b)
        dinv = 1.0 / Ae.diagonal()
        x0 = rng.standard_normal(S.N2)
        x0[B] = b[B]
        x1, _ = krylov.pcg(Ae, b, x0, dinv, 1e-14, 5000)
        x2, _ = krylov.bicgstab(Ae, b, x0, dinv, 1e-14, 5000)
        for x in (x1, x2):
            assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
    # a non-symmetric system for BiCGStab (momentum matrix with convection added)
    U = rng.standard_normal((S.dim, S.N2))
    A = (M / 1e-2 + 0.01 * K + fem.convection(S, U)).tocsr()
    Ae = fem.eliminate(A, B)
    b = fem.lift(A, rng.standard_normal(S.N2), B, rng.standard_normal(S.N2))
    ref = np.linalg.solve(Ae.toarray(), b)
    x, _ = krylov.bicgstab(Ae, b, np.where(B, b, 0.0), 1.0 / Ae.diagonal(), 1e-14, 5000)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("S", list(spaces()))
def test_singular_poisson_matches_bordered_system(S):
    """Kp x = r (r projected to zero sum), x normalized to zero integral mean,
    equals the solution of [[Kp, w], [w^T, 0]] [x; l] = [r; 0]."""
    rng = np.random.default_rng(9)
    Kp, Mp = fem.stiff_p1(S), fem.mass_p1(S)
    w = Mp @ np.ones(S.N1)
    r = rng.standard_normal(S.N1)
    r -= r.mean()
    x, _ = krylov.pcg(Kp, r, np.zeros(S.N1), 1.0 / Kp.diagonal(), 1e-14, 5000, project=True)
    x -= np.dot(w, x) / w.sum()
    Bd = np.zeros((S.N1 + 1, S.N1 + 1))
    Bd[:-1, :-1] = Kp.toarray()
    Bd[:-1, -1] = w
    Bd[-1, :-1] = w
    ref = np.linalg.solve(Bd, np.r_[r, 0.0])[:-1]
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_zero_rhs_and_non_convergence():
    S = fem.Space(*mesh.unit_square(4, 4))
    M = fem.eliminate(fem.mass_p2(S), S.boundary2)
    dinv = 1.0 / M.diagonal()
    x, it = krylov.pcg(M, np.zeros(S.N2), np.ones(S.N2), dinv, 1e-12, 10)
    assert it == 0 and not x.any()
    x, it = krylov.bicgstab(M, np.zeros(S.N2), np.ones(S.N2), dinv, 1e-12, 10)
    assert it == 0 and not x.any()
    b = np.random.default_rng(0).standard_normal(S.N2)
    with pytest.raises(krylov.NotConverged):
        krylov.pcg(M, b, np.zeros(S.N2), dinv, 1e-14, 1)
    with pytest.raises(krylov.NotConverged):
        krylov.bicgstab(M, b, np.zeros(S.N2), dinv, 1e-14, 1)
