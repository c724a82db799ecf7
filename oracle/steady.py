"""Steady incompressible Navier-Stokes by Newton's method, Taylor-Hood P2-P1
(oracle; test infrastructure).

Problem (Section 2.1, the steady equations): -nu Lap u + (u . grad) u +
grad p = f, div u = 0 in Omega, u = g on the boundary. Discretization: the
spaces V_h, Q_h of Section 2.2.1 (velocity P2 with Dirichlet data, pressure
P1), the same local matrices as the IPCS oracle (fem.py).

Newton's method (Section 2.2.1, the Newton linearization, with the
time-derivative term dropped for the steady problem): from (u^k, p^k) the next
iterate solves, for all v_h in V_h (vanishing on the boundary) and q_h,
    ((u^k . grad) u^{k+1}, v) + ((u^{k+1} . grad) u^k, v) - ((u^k . grad) u^k, v)
      + nu (grad u^{k+1}, grad v) - (p^{k+1}, div v) = (f, v),
    (div u^{k+1}, q) = 0.
Here it is solved for the increment (du, dp) = (u^{k+1} - u^k, p^{k+1} - p^k),
which is the same iterate: J(u^k) (dU, dP) = R(u^k, p^k) with, per velocity
component c and for velocity rows whose node is not on the boundary,
    R_c = F_c - nu K U_c - C(U) U_c - G_c P          (-(p, div v) = (grad p, v))
    R_p = - sum_c D_c U_c   (projected to zero sum: the system is singular)
    J = [[nu K + C(U) + N(U), G], [D, 0]],
    N_{ce, ij} = sum_q w |J| phi_i phi_j d_e u_c(x_q)   (the term ((du . grad) u^k, v)),
C(U) the convection matrix of fem.py, G_c = (phi_i, d_c psi_k),
D_c = (psi_k, d_c phi_j). Dirichlet: the iterates carry g on the boundary
velocity nodes from the start, so the increments vanish there (symmetric
elimination, as in fem.eliminate). The pressure is fixed by zero integral
mean: the linear systems are solved with the border w^T dP = 0, w = Mp 1, by
scipy's sparse direct solver (a library routine).

Readings (the paper is silent): u^0 is zero at interior nodes and g on the
boundary, p^0 = 0; the iteration stops when ||(dU, dP)||_2 <= tol
||(U, P)||_2 after the update (Section 4.2 runs the model with tol = 1e-10 and
at most 10 steps).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


def local_newton(space, U, c, e):
    """N_{ce}: (phi_j d_e u_c, phi_i) per cell, (Nc, nloc, nloc)."""
    lam, w = fem._rule(space)
    phi, dref = space.basis_u(lam)
    g = space.phys_grad(dref)                                   # (Nc, nq, nloc, d)
    du = np.einsum('cqm,cm->cq', g[..., e], U[c][space.c2du])   # d_e u_c at the points
    return np.einsum('q,c,cq,qi,qj->cij', w, space.absdet, du, phi, phi)


def newton_block(space, U, c, e):
    return fem.assemble(local_newton(space, U, c, e), space.c2du, space.c2du,
                        (space.Nu, space.Nu))


class SteadyNewton:
    def __init__(self, space, problem, nu, tol=1e-10, maxit=10):
        if space.order != 2:
            raise ValueError("the steady solver is built for the P2-P1 pair")
        S = space
        self.S, self.pb, self.nu, self.tol, self.maxit = S, problem, float(nu), tol, maxit
        self.K = fem.stiff_u(S)
        self.Mp = fem.mass_p(S)
        self.D = [fem.divergence(S, c) for c in range(S.dim)]
        self.G = [fem.gradient(S, c) for c in range(S.dim)]
        self.w = self.Mp @ np.ones(S.Np)
        self.F = fem.load(S, lambda x, t: problem.f(x, 0.0), 0.0) if problem.f is not None \
            else np.zeros((S.dim, S.Nu))
        g = problem.u(S.xu, 0.0).T                               # (d, Nu)
        self.U = np.where(S.bmask_u[None, :], g, 0.0)
        self.P = np.zeros(S.Np)
        self.history = []                                        # ||dx|| / ||x|| per step

    def residual(self):
        """(R_u (d, Nu) with zeros on boundary rows, R_p (Np,))."""
        S, U = self.S, self.U
        C = fem.convection(S, U)
        Ru = np.stack([self.F[c] - self.nu * (self.K @ U[c]) - C @ U[c] - self.G[c] @ self.P
                       for c in range(S.dim)])
        Ru[:, S.bmask_u] = 0.0
        Rp = -sum(self.D[c] @ U[c] for c in range(S.dim))
        # the Newton matrix is singular (constant pressure): its pressure
        # rows' right-hand side is projected to zero sum, as the Poisson
        # right-hand side of the IPCS step is
        return Ru, Rp - Rp.mean()

    def jacobian(self):
        """The Newton matrix, boundary velocity rows and columns eliminated,
        as one sparse matrix over (U_0, .., U_{d-1}, P)."""
        S, U, d = self.S, self.U, self.S.dim
        C = fem.convection(S, U)
        A = (self.nu * self.K + C).tocsr()
        blocks = [[None] * (d + 1) for _ in range(d + 1)]
        for c in range(d):
            for e in range(d):
                B = newton_block(S, U, c, e)
                blocks[c][e] = (A + B) if c == e else B
            blocks[c][d] = self.G[c]
            blocks[d][c] = self.D[c]
        J = sp.bmat(blocks, format="csr")
        mask = np.concatenate([np.tile(S.bmask_u, d), np.zeros(S.Np, dtype=bool)])
        return fem.eliminate(J, mask)

    def step(self):
        S, d = self.S, self.S.dim
        Ru, Rp = self.residual()
        J = self.jacobian()
        n = d * S.Nu + S.Np
        wb = np.concatenate([np.zeros(d * S.Nu), self.w])
        Bd = sp.bmat([[J, sp.csr_matrix(wb[:, None])], [sp.csr_matrix(wb[None, :]), None]],
                     format="csc")
        x = spla.spsolve(Bd, np.concatenate([Ru.ravel(), Rp, [0.0]]))[:n]
        dU, dP = x[:d * S.Nu].reshape(d, S.Nu), x[d * S.Nu:]
        self.U = self.U + dU
        self.P = self.P + dP
        rel = np.linalg.norm(x) / np.linalg.norm(np.concatenate([self.U.ravel(), self.P]))
        self.history.append(rel)
        return rel

    def run(self):
        for _ in range(self.maxit):
            if self.step() <= self.tol:
                break
        return self.U, self.P
