"""Jacobi-preconditioned CG and BiCGStab (oracle).

The solvers themselves are not given in the paper (its ComputationModel picks
library solvers, Section 3.3); the target method names Jacobi-PCG for the
pressure Poisson and velocity-correction systems and Jacobi-BiCGStab for the
momentum system. These are the textbook algorithms: preconditioned CG
(Saad, Iterative Methods for Sparse Linear Systems, 2003, Alg. 9.1) and
right-preconditioned BiCGStab (van der Vorst 1992), with z = r / diag(A).

Stopping rule shared with the HIP library: the unpreconditioned recursive
residual ||r||_2 <= tol * ||b||_2, confirmed by the true residual b - A x at
exit; if the true residual fails, the iteration restarts from the current x
(up to maxit iterations in total). b = 0 gives x = 0. A BiCGStab breakdown
(|rho| or |omega| tiny relative to the norms involved) also restarts from the
current x.
"""
import numpy as np


class NotConverged(RuntimeError):
    pass


def _norm(v):
    return float(np.sqrt(np.dot(v, v)))


def pcg(A, b, x0, dinv, tol, maxit, project=False):
    """Jacobi-PCG. If project, A is the singular pure-Neumann matrix whose
    null space is the constant vector and b is assumed already projected."""
    x = np.array(x0, dtype=np.float64, copy=True)
    bn = _norm(b)
    if bn == 0.0:
        return np.zeros_like(x), 0
    it = 0
    while True:
        r = b - A @ x
        if _norm(r) <= tol * bn:
            return x, it
        z = dinv * r
        p = z.copy()
        rho = float(np.dot(r, z))
        while it < maxit:
            q = A @ p
            alpha = rho / float(np.dot(p, q))
            x += alpha * p
            r -= alpha * q
            it += 1
            if _norm(r) <= tol * bn:
                break
            z = dinv * r
            rho_new = float(np.dot(r, z))
            p = z + (rho_new / rho) * p
            rho = rho_new
        if it >= maxit and _norm(b - A @ x) > tol * bn:
            raise NotConverged(f"pcg: {it} iterations, residual "
                               f"{_norm(b - A @ x) / bn:.3e}")


def bicgstab(A, b, x0, dinv, tol, maxit):
    """Right-preconditioned Jacobi-BiCGStab."""
    x = np.array(x0, dtype=np.float64, copy=True)
    bn = _norm(b)
    if bn == 0.0:
        return np.zeros_like(x), 0
    it = 0
    while True:
        r = b - A @ x
        if _norm(r) <= tol * bn:
            return x, it
        rhat = r.copy()
        rho = alpha = omega = 1.0
        v = np.zeros_like(x)
        p = np.zeros_like(x)
        restart = False
        while it < maxit:
            rho_new = float(np.dot(rhat, r))
            if abs(rho_new) < 1e-300:
                restart = True
                break
            beta = (rho_new / rho) * (alpha / omega)
            p = r + beta * (p - omega * v)
            phat = dinv * p
            v = A @ phat
            alpha = rho_new / float(np.dot(rhat, v))
            s = r - alpha * v
            shat = dinv * s
            t = A @ shat
            tt = float(np.dot(t, t))
            if tt == 0.0:
                x += alpha * phat
                r = s
                it += 1
                break
            omega = float(np.dot(t, s)) / tt
            x += alpha * phat + omega * shat
            r = s - omega * t
            it += 1
            rho = rho_new
            if _norm(r) <= tol * bn:
                break
            if abs(omega) < 1e-300:
                restart = True
                break
        if it >= maxit and _norm(b - A @ x) > tol * bn:
            raise NotConverged(f"bicgstab: {it} iterations, residual "
                               f"{_norm(b - A @ x) / bn:.3e}")
        if not restart and _norm(b - A @ x) <= tol * bn:
            return x, it
