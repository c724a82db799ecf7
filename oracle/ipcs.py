"""One IPCS time step with Taylor-Hood elements, P2-P1 or P3-P2 (oracle).

The scheme is eq. (9) of Section 2.2.1 (incremental pressure correction,
Goda). With density rho and time step dt, one step n -> n+1 at
t = t0 + (n+1) dt is, in matrix form:

1. Momentum (tentative velocity u*): for each component c
      (M/dt + nu K) U*_c = M U^n_c / dt - C(U^n) U^n_c - G_c P^n + F_c(t)
   with the convection term taken explicitly as written in eq. (9)
   ((u^n . grad) u^n, v). The pressure term -(p^n, div v) of eq. (9) equals
   -(grad p^n, v) = -(G_c P^n) on rows whose test function vanishes on the
   boundary, which are the only rows that are equations (v_h in H^1_0).
   Dirichlet data g(t) is imposed by symmetric elimination.
2. Pressure increment: Kp dP = -(rho/dt) sum_c D_c U*_c.
   The printed right-hand side of the second equation carries the opposite
   sign; the sign used here is the one for which the third equation makes
   u^{n+1} discretely divergence-free (u^{n+1} = u* - dt/rho grad dP and
   div u^{n+1} = 0 give Lap dP = rho/dt div u*, whose weak form is
   (grad dP, grad q) = -(rho/dt)(div u*, q)). The system is pure Neumann:
   its right-hand side is projected to zero sum and dP is shifted to zero
   integral mean (w = Mp 1). P^{n+1} = P^n + dP.
3. Velocity correction: M U^{n+1}_c = M U*_c - (dt/rho) G_c dP with the same
   Dirichlet data on boundary rows.

Solvers: Jacobi-BiCGStab for step 1 (x0 = U^n with boundary values g),
Jacobi-PCG for steps 2 (x0 = 0) and 3 (x0 = U*).

With chorin=True the step is the non-incremental projection of Chorin and
Temam, the scheme Section 2.2.1 states before IPCS (eq. (8)): the momentum
step has no pressure term, the Poisson solve gives the new pressure itself
(Kp P^{n+1} = -(rho/dt) sum_c D_c U*_c, the same sign reading as for IPCS),
P^{n+1} is shifted to zero integral mean, and the correction uses P^{n+1}.
"""
import time

import numpy as np

from . import fem, krylov


class Params:
    def __init__(self, nu, dt, rho=1.0, t0=0.0, tol_mom=1e-12, tol_p=1e-12,
                 tol_corr=1e-12, maxit=20000, semi_implicit=False, chorin=False):
        self.nu, self.dt, self.rho, self.t0 = float(nu), float(dt), float(rho), float(t0)
        self.tol_mom, self.tol_p, self.tol_corr = tol_mom, tol_p, tol_corr
        self.maxit = maxit
        self.semi_implicit = semi_implicit
        self.chorin = chorin


class IPCS:
    def __init__(self, space, problem, params):
        self.S = space
        self.pb = problem
        self.prm = params
        S = space
        d = S.dim
        self.M = fem.mass_u(S)
        self.K = fem.stiff_u(S)
        self.Kp = fem.stiff_p(S)
        self.Mp = fem.mass_p(S)
        self.D = [fem.divergence(S, c) for c in range(d)]
        self.G = [fem.gradient(S, c) for c in range(d)]
        self.w = self.Mp @ np.ones(S.Np)
        self.bmask = S.bmask_u
        self.A = (self.M / params.dt + params.nu * self.K).tocsr()
        self.A.sort_indices()
        self.A_el = fem.eliminate(self.A, self.bmask)
        self.M_el = fem.eliminate(self.M, self.bmask)
        self.dinv_A = 1.0 / self.A_el.diagonal()
        self.dinv_M = 1.0 / self.M_el.diagonal()
        self.dinv_Kp = 1.0 / self.Kp.diagonal()
        self.t = params.t0
        self.U = problem.u(S.xu, self.t).T.copy()          # (d, Nu)
        self.P = self.normalize(problem.p(S.xp, self.t))
        self.iters = []
        # wall time (s) of each step's phases, for reporting only: the
        # momentum system (boundary data, forcing, convection matrix and
        # right-hand sides), its solves, the pressure step, the correction
        self.times = []

    def normalize(self, P):
        """Shift a pressure field to zero integral mean."""
        return P - np.dot(self.w, P) / self.w.sum()

    def set_state(self, U, P, t):
        self.U = np.array(U, dtype=np.float64).reshape(self.S.dim, self.S.Nu).copy()
        self.P = np.array(P, dtype=np.float64).copy()
        self.t = float(t)

    def dirichlet(self, t):
        """g(t) at every velocity node (only boundary entries are used)."""
        return self.pb.u(self.S.xu, t).T

    def forcing(self, t):
        if self.pb.f is None:
            return np.zeros((self.S.dim, self.S.Nu))
        return fem.load(self.S, self.pb.f, t)

    # ---- the three sub-steps, in the paper's order. Each *_system method
    # forms the linear system of its sub-step (matrix with Dirichlet rows and
    # columns eliminated, right-hand sides, initial guesses, Jacobi inverse
    # diagonal); the sub-step solves it.
    def momentum_system(self, t, g):
        S, prm = self.S, self.prm
        C = fem.convection(S, self.U)
        F = self.forcing(t)
        if prm.semi_implicit:
            A = (self.A + C).tocsr()
            A.sort_indices()
            A_el = fem.eliminate(A, self.bmask)
            dinv = 1.0 / A_el.diagonal()
        else:
            A, A_el, dinv = self.A, self.A_el, self.dinv_A
        bs, x0s = [], []
        for c in range(S.dim):
            b = self.M @ self.U[c] / prm.dt
            if not prm.chorin:
                b = b - self.G[c] @ self.P
            b = b + F[c]
            if not prm.semi_implicit:
                b = b - C @ self.U[c]
            bs.append(fem.lift(A, b, self.bmask, g[c]))
            x0s.append(np.where(self.bmask, g[c], self.U[c]))
        return A_el, bs, x0s, dinv, C

    def momentum(self, t, g):
        prm = self.prm
        A_el, bs, x0s, dinv, C = self.momentum_system(t, g)
        t0 = time.perf_counter()
        Ustar = np.zeros_like(self.U)
        its = []
        for c in range(self.S.dim):
            Ustar[c], it = krylov.bicgstab(A_el, bs[c], x0s[c], dinv, prm.tol_mom, prm.maxit)
            its.append(it)
        self._t_solve = time.perf_counter() - t0
        return Ustar, C, its

    def pressure_system(self, Ustar):
        prm = self.prm
        r = -(prm.rho / prm.dt) * sum(self.D[c] @ Ustar[c] for c in range(self.S.dim))
        return self.Kp, r - r.mean()

    def pressure(self, Ustar):
        S, prm = self.S, self.prm
        Kp, r = self.pressure_system(Ustar)
        dP, it = krylov.pcg(Kp, r, np.zeros(S.Np), self.dinv_Kp, prm.tol_p,
                            prm.maxit, project=True)
        dP = self.normalize(dP)
        return dP, it

    def correction_system(self, Ustar, dP, g):
        prm = self.prm
        bs = []
        for c in range(self.S.dim):
            b = self.M @ Ustar[c] - (prm.dt / prm.rho) * (self.G[c] @ dP)
            bs.append(fem.lift(self.M, b, self.bmask, g[c]))
        return self.M_el, bs

    def correction(self, Ustar, dP, g):
        prm = self.prm
        M_el, bs = self.correction_system(Ustar, dP, g)
        Unew = np.zeros_like(Ustar)
        its = []
        for c in range(self.S.dim):
            Unew[c], it = krylov.pcg(M_el, bs[c], Ustar[c], self.dinv_M, prm.tol_corr, prm.maxit)
            its.append(it)
        return Unew, its

    def step(self):
        c0 = time.perf_counter()
        t = self.t + self.prm.dt
        g = self.dirichlet(t)
        Ustar, _, it_m = self.momentum(t, g)
        c1 = time.perf_counter()
        dP, it_p = self.pressure(Ustar)
        c2 = time.perf_counter()
        Unew, it_c = self.correction(Ustar, dP, g)
        c3 = time.perf_counter()
        self.times.append({"asm": (c1 - c0) - self._t_solve, "momentum": self._t_solve,
                           "pressure": c2 - c1, "correction": c3 - c2})
        self.U = Unew
        self.P = dP if self.prm.chorin else self.P + dP
        self.t = t
        self.iters.append((it_m, it_p, it_c))
        return self.U, self.P

    def run(self, nsteps):
        for _ in range(nsteps):
            self.step()
        return self.U, self.P
